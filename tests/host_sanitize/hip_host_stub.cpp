// Host-only stand-in for the part of the HIP runtime that the library's host
// driver (capi.cpp) calls, plus no-op kernel launchers.  Test infrastructure:
// it lets the planner, the input validation, the work split, the batch
// planning and every host-side size computation run under AddressSanitizer
// and UndefinedBehaviorSanitizer on a machine without a GPU.
//
// "Device" memory is host memory (calloc), copies and fills are memcpy and
// memset, streams, events and graphs are inert handles, and elapsed times are
// zero.  The kernel launchers launch nothing; the two that only fill or
// convert memory do so on the host, so that a launch sized beyond its buffer
// is reported by the sanitizer like any other out-of-bounds access.  The
// numbers a build returns are meaningless; only the host code paths are
// under test.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "../../paper_2102_02989_amd/csrc/kernels.h"

namespace {
char g_handles[4096];  // addresses handed out as stream, event and graph handles
int g_next = 0;
template <class T>
T handle() {
  g_next = (g_next + 1) % (int)sizeof(g_handles);
  return reinterpret_cast<T>(&g_handles[g_next]);
}
constexpr size_t kFree = (size_t)3 << 30, kTotal = (size_t)4 << 30;
}  // namespace

hipError_t hipMalloc(void **ptr, size_t size) {
  if (!ptr) return hipErrorInvalidValue;
  *ptr = std::calloc(size ? size : 1, 1);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *ptr) {
  std::free(ptr);
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t *free_b, size_t *total) {
  if (free_b) *free_b = kFree;
  if (total) *total = kTotal;
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
  if (n) std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int value, size_t n, hipStream_t) {
  if (n) std::memset(dst, value, n);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
  *s = handle<hipStream_t>();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = handle<hipEvent_t>();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = handle<hipEvent_t>();
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "host stub error"; }
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  *p = const_cast<void *>(symbol);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  *g = handle<hipGraph_t>();
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, hipGraphNode_t *, char *, size_t) {
  *x = handle<hipGraphExec_t>();
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

namespace rsgdf {
// fills and conversions run on the host (their sizes are checked); the rest launch nothing
hipError_t launch_zero(void *p, size_t bytes, hipStream_t) {
  if (bytes) std::memset(p, 0, bytes);
  return hipSuccess;
}
hipError_t launch_to_f32(const double *x, float *y, int64_t n, hipStream_t) {
  for (int64_t i = 0; i < n; ++i) y[i] = (float)x[i];
  return hipSuccess;
}
hipError_t launch_sr3c(int, int, const SRParams *, const SRWork *, long long *, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_sr_reduce(const SRParams &, const SRPartGroup *, int, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_fold(const FoldParams &, hipStream_t) { return hipSuccess; }
hipError_t launch_overlaps(const OvlParams &, const SmnParams &, hipStream_t) { return hipSuccess; }
hipError_t launch_auxft(const AuxFTParams &, hipStream_t) { return hipSuccess; }
hipError_t launch_lr_gemm_tiled(int, const LRGemmParams &, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_pairft_binned(const PairFTParams &, hipStream_t) { return hipSuccess; }
hipError_t launch_amax(const double *, int64_t, int, int, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_kphase(const double *, const double *, void *, bool, double *, int, int, int, int, int64_t,
                         hipStream_t) {
  return hipSuccess;
}
hipError_t launch_asplit(const double *, int64_t, int, int, int, uint16_t *, int32_t *, hipStream_t) { return hipSuccess; }
hipError_t launch_kphase_split(const double *, const double *, uint16_t *, int32_t *, double *, int, int, int, int,
                               int64_t, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_j2c_sr(int, int, const J2Params &, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_j2c_fold(const double *, const double *, const double *, double, int, int, double *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_j2c_lr_operand(const double *, int64_t, const double *, int, int, double, double, double *,
                                 hipStream_t) {
  return hipSuccess;
}
hipError_t launch_df_factor(const double *, double *, double *, int *, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_df_gemm(bool, const double *, const int32_t *, const double *, double *, int, int64_t, int,
                          hipStream_t) {
  return hipSuccess;
}
hipError_t launch_dm_contract(const double *, const double *, int, int, int, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_vj_accum(const double *, const double *, int, int, int64_t, double, double *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_features(const SRParams &, int, const int64_t *, int64_t, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_log_target(const float *, int, int64_t, float, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_mlp_step(float *, const float *, const float *, const int64_t *, int64_t, float, float *, float *,
                           float *, float *, float *, float, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_mlp_mask(const SRParams &, int, int64_t, const float *, float, uint8_t *, long long *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_mlp_predict(const float *, const float *, int64_t, int, float *, hipStream_t) { return hipSuccess; }
}  // namespace rsgdf
