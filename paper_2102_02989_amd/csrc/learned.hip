// learned.hip -- learned screening of short-range work (a project addition
// beside the rigorous bounds of the Supplementary Material, Eqs. S14-S27).
//
// Unit of screening: a candidate (aux shell P, AO shell pair, pair image n'),
// i.e. one iteration of the image loop of sr3c_kernel.  Target: log10 of the
// sum over BvK cells c1 of max |block| that the candidate adds to
// X[c1][c2][P][mu][nu], an upper bound of its effect on any output element
// (the Bloch fold combines the c1 blocks with unit-modulus phases).
//
// Network: 16 standardised features -> 64 -> 64 -> 1, ReLU, predicting that
// log10 magnitude.  Training runs here in FP32 (forward/backward kernels,
// deterministic block-partial gradient sums, Adam); inference for the keep
// mask runs on the matrix cores in FP16 (FP32 accumulation).  A candidate is
// dropped only if its features lie inside the training range and
// prediction + margin < log10(thresh); otherwise the rigorous path decides.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "learned.h"
#include "plan.h"

namespace rsgdf {

// ---- features ----------------------------------------------------------------
// 0 log10 beta_d   1 log10 p_d   2 log10 alpha_P,d   (most diffuse primitives)
// 3 R12 = |A - B - n'|          4 R_c,min: pair centre to the nearest aux image
// 5 l_a  6 l_b  7 l_P           8 log10 A (1s-model amplitude of the triplet)
// 9 log10 omega                10 log10 of the 1s estimate A e^{-beta R12^2} f(R_c,min),
//                                 f(R) = (erf(eta1 R) - erf(eta2 R))/R (Eqs. S4-S9)
// 11..15 zero
__device__ bool sr_candidate_features(const SRParams &prm, int trip, int ii, float *f) {
  const Triplet tr = prm.trip[trip];
  const Pair pr = prm.pairs[tr.pair];
  const Shell A = prm.ao[pr.sa], B = prm.ao[pr.sb], P = prm.ax[tr.aux];
  const int nk = prm.lat.nk;
  // class of image ii and its short-range count
  int cls = 0;
  while (cls < nk - 1 && prm.cls_off[pr.cls_off + cls + 1] <= ii) ++cls;
  if (ii - prm.cls_off[pr.cls_off + cls] >= prm.nsr[pr.nsr_off + cls]) return false;
  const double *nv = prm.img + 3 * (size_t)(pr.img_off + ii);
  const double Bx = B.x + nv[0], By = B.y + nv[1], Bz = B.z + nv[2];
  const double dx = A.x - Bx, dy = A.y - By, dz = A.z - Bz;
  const double r12sq = dx * dx + dy * dy + dz * dz;
  const double pd = A.a_d + B.a_d, beta = A.a_d * B.a_d / pd;
  const double Px = (A.a_d * A.x + B.a_d * Bx) / pd, Py = (A.a_d * A.y + B.a_d * By) / pd,
               Pz = (A.a_d * A.z + B.a_d * Bz) / pd;
  double X0[3] = {Px - P.x, Py - P.y, Pz - P.z};
  // nearest aux image: round the fractional coordinates, then search +-1
  const Lattice &L = prm.lat;
  int j0[3];
  for (int d = 0; d < 3; ++d)
    j0[d] = (int)floor(-(L.b[3 * d] * X0[0] + L.b[3 * d + 1] * X0[1] + L.b[3 * d + 2] * X0[2]) / (2.0 * kPi) + 0.5);
  double rc2 = 1e300;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c) {
        const int m0 = j0[0] + a, m1 = j0[1] + b, m2 = j0[2] + c;
        const double x = X0[0] + m0 * L.a[0] + m1 * L.a[3] + m2 * L.a[6];
        const double y = X0[1] + m0 * L.a[1] + m1 * L.a[4] + m2 * L.a[7];
        const double z = X0[2] + m0 * L.a[2] + m1 * L.a[5] + m2 * L.a[8];
        rc2 = fmin(rc2, x * x + y * y + z * z);
      }
  const double rc = sqrt(rc2);
  const double eta1 = sqrt(P.a_d * pd / (P.a_d + pd));
  const double eta2 = 1.0 / sqrt(1.0 / (eta1 * eta1) + 1.0 / (prm.omega * prm.omega));
  const double fr = (rc < 1e-8) ? 2.0 * (eta1 - eta2) * 0.564189583547756286948079451561
                                : (erf(eta1 * rc) - erf(eta2 * rc)) / rc;
  const double est = tr.amp * exp(-beta * r12sq) * fr;
  f[0] = (float)log10(beta);
  f[1] = (float)log10(pd);
  f[2] = (float)log10(P.a_d);
  f[3] = (float)sqrt(r12sq);
  f[4] = (float)rc;
  f[5] = (float)A.l;
  f[6] = (float)B.l;
  f[7] = (float)P.l;
  f[8] = (float)log10(fmax(tr.amp, 1e-300));
  f[9] = (float)log10(prm.omega);
  f[10] = (float)log10(fmax(est, 1e-300));
  for (int i = 11; i < kMlpF; ++i) f[i] = 0.f;
  return true;
}

__device__ __forceinline__ int find_trip(const int64_t *cand_off, int ntrip, int64_t c) {
  int lo = 0, hi = ntrip - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (cand_off[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// feat[i][16] for the candidates idx[i] (indices into the candidate list)
__global__ void features_kernel(const SRParams prm, int ntrip, const int64_t *__restrict__ idx, int64_t n,
                               float *__restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = idx[i];
  const int t = find_trip(prm.cand_off, ntrip, c);
  float f[kMlpF];
  if (!sr_candidate_features(prm, t, (int)(c - prm.cand_off[t]), f))
    for (int k = 0; k < kMlpF; ++k) f[k] = 0.f;
  for (int k = 0; k < kMlpF; ++k) feat[i * kMlpF + k] = f[k];
}

hipError_t launch_features(const SRParams &prm, int ntrip, const int64_t *idx, int64_t n, float *feat,
                           hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, stream, prm, ntrip, idx, n,
                     feat);
  return hipGetLastError();
}

// target[c] = max(log10(sum_c1 logmag[c][c1]), floor) for candidates the
// image loop reached (entries >= 0), NaN otherwise
__global__ void log_target_kernel(const float *__restrict__ logmag, int nk, int64_t ncand, float floor_,
                                  float *__restrict__ tgt) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncand) return;
  double s = 0.0;
  bool seen = false;
  for (int k = 0; k < nk; ++k) {
    const float v = logmag[c * nk + k];
    if (v >= 0.f) {
      seen = true;
      s += v;
    }
  }
  tgt[c] = seen ? fmaxf((float)log10(fmax(s, 1e-300)), floor_) : __builtin_nanf("");
}

hipError_t launch_log_target(const float *logmag, int nk, int64_t ncand, float floor_, float *tgt,
                             hipStream_t stream) {
  if (ncand <= 0) return hipSuccess;
  hipLaunchKernelGGL(log_target_kernel, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, stream, logmag, nk,
                     ncand, floor_, tgt);
  return hipGetLastError();
}

// ---- training (FP32) ---------------------------------------------------------
// One wave of 64 samples per block: per-sample forward and backward in
// registers, then the block's weight gradients summed over its samples in a
// fixed order; mlp_reduce_adam_kernel sums the block partials in block order.
// Loss: (1/B) sum_s w_s (pred_s - y_s)^2 with w_s = kappa when pred_s < y_s
// (under-prediction would drop terms that matter) and 1 otherwise.
__global__ __launch_bounds__(64) void mlp_fwd_bwd_kernel(const float *__restrict__ prm_, const float *__restrict__ X,
                                                         const float *__restrict__ y, const int64_t *__restrict__ idx,
                                                         int64_t nb, float kappa, float *__restrict__ gpart,
                                                         float *__restrict__ lpart) {
  __shared__ float sW[kMlpNParam];
  // rows padded by one word so that the 64 lanes (one sample each) hit distinct banks
  __shared__ float sx[64][kMlpF + 1];
  __shared__ float sh1[64][kMlpH + 1], sh2[64][kMlpH + 1];
  __shared__ float sd1[64][kMlpH + 1], sd2[64][kMlpH + 1];
  __shared__ float sdy[64];
  const int t = threadIdx.x;
  for (int i = t; i < kMlpNParam; i += 64) sW[i] = prm_[i];
  __syncthreads();
  const float *W1 = sW + kMlpOffW1, *b1 = sW + kMlpOffB1, *W2 = sW + kMlpOffW2, *b2 = sW + kMlpOffB2;
  const float *W3 = sW + kMlpOffW3;
  const float b3 = sW[kMlpOffB3];
  const int64_t s = (int64_t)blockIdx.x * 64 + t;
  const bool on = s < nb;
  float loss = 0.f;
  {
    const int64_t r = on ? idx[s] : 0;
    for (int k = 0; k < kMlpF; ++k)
      sx[t][k] = on ? (X[r * kMlpF + k] - sW[kMlpOffMean + k]) * sW[kMlpOffIstd + k] : 0.f;
    for (int j = 0; j < kMlpH; ++j) {
      float a = b1[j];
      for (int k = 0; k < kMlpF; ++k) a += W1[j * kMlpF + k] * sx[t][k];
      sh1[t][j] = a > 0.f ? a : 0.f;
    }
    for (int j = 0; j < kMlpH; ++j) {
      float a = b2[j];
      for (int k = 0; k < kMlpH; ++k) a += W2[j * kMlpH + k] * sh1[t][k];
      sh2[t][j] = a > 0.f ? a : 0.f;
    }
    float pred = b3;
    for (int k = 0; k < kMlpH; ++k) pred += W3[k] * sh2[t][k];
    float dy = 0.f;
    if (on) {
      const float e = pred - y[r];
      const float w = (e < 0.f) ? kappa : 1.f;
      loss = w * e * e / (float)nb;
      dy = 2.f * w * e / (float)nb;
    }
    sdy[t] = dy;
    for (int j = 0; j < kMlpH; ++j) sd2[t][j] = (sh2[t][j] > 0.f) ? dy * W3[j] : 0.f;
    for (int k = 0; k < kMlpH; ++k) {
      float a = 0.f;
      for (int j = 0; j < kMlpH; ++j) a += W2[j * kMlpH + k] * sd2[t][j];
      sd1[t][k] = (sh1[t][k] > 0.f) ? a : 0.f;
    }
  }
  __syncthreads();
  // block gradient entries, each summed over the 64 samples in order
  float *g = gpart + (size_t)blockIdx.x * kMlpNTrain;
  for (int p = t; p < kMlpNTrain; p += 64) {
    const int q = p + kMlpOffW1;  // parameter index
    float a = 0.f;
    if (q < kMlpOffB1) {
      const int j = (q - kMlpOffW1) / kMlpF, k = (q - kMlpOffW1) % kMlpF;
      for (int u = 0; u < 64; ++u) a += sd1[u][j] * sx[u][k];
    } else if (q < kMlpOffW2) {
      const int j = q - kMlpOffB1;
      for (int u = 0; u < 64; ++u) a += sd1[u][j];
    } else if (q < kMlpOffB2) {
      const int j = (q - kMlpOffW2) / kMlpH, k = (q - kMlpOffW2) % kMlpH;
      for (int u = 0; u < 64; ++u) a += sd2[u][j] * sh1[u][k];
    } else if (q < kMlpOffW3) {
      const int j = q - kMlpOffB2;
      for (int u = 0; u < 64; ++u) a += sd2[u][j];
    } else if (q < kMlpOffB3) {
      const int k = q - kMlpOffW3;
      for (int u = 0; u < 64; ++u) a += sdy[u] * sh2[u][k];
    } else {
      for (int u = 0; u < 64; ++u) a += sdy[u];
    }
    g[p] = a;
  }
  // block loss, fixed-order wave sum
  for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (t == 0) lpart[blockIdx.x] = loss;
}

// grad[p] = sum over blocks of the partials (block order); optionally one Adam step
__global__ void mlp_reduce_adam_kernel(float *__restrict__ prm_, const float *__restrict__ gpart, int nblk,
                                       float *__restrict__ grad, float *__restrict__ m, float *__restrict__ v, float lr,
                                       float b1, float b2, float eps, int step) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNTrain) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += gpart[(size_t)b * kMlpNTrain + p];
  if (grad) grad[p] = g;
  if (step > 0) {
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)step)), vh = vv / (1.f - powf(b2, (float)step));
    prm_[kMlpOffW1 + p] -= lr * mh / (sqrtf(vh) + eps);
  }
}

hipError_t launch_mlp_step(float *params, const float *X, const float *y, const int64_t *idx, int64_t nb,
                           float kappa, float *gpart, float *lpart, float *grad, float *m, float *v, float lr, int step,
                           hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  const int nblk = (int)((nb + 63) / 64);
  hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(nblk), dim3(64), 0, stream, params, X, y, idx, nb, kappa, gpart, lpart);
  hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kMlpNTrain + 255) / 256), dim3(256), 0, stream, params, gpart, nblk,
                     grad, m, v, lr, 0.9f, 0.999f, 1e-8f, step);
  return hipGetLastError();
}

// ---- inference on the matrix cores (FP16 operands, FP32 accumulation) --------
// One wave per 64 rows.  v_mfma_f32_16x16x16_f16 fragments (li = lane % 16,
// lg = lane / 16): A[li][4 lg + j], B[4 lg + j][li], D[4 lg + v][li].
typedef _Float16 mlp_h4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

struct MlpLds {
  _Float16 W1[kMlpH * kMlpF];  // [out][in]
  _Float16 W2[kMlpH * kMlpH];
  float b1[kMlpH], b2[kMlpH], W3[kMlpH], b3;
  _Float16 x[64 * kMlpF];      // standardised inputs of the wave's rows
  _Float16 h[64 * kMlpH];      // first hidden layer
  float pred[64];
};

__device__ void mlp_load_lds(const float *__restrict__ prm_, MlpLds &S) {
  for (int i = threadIdx.x; i < kMlpH * kMlpF; i += blockDim.x) S.W1[i] = (_Float16)prm_[kMlpOffW1 + i];
  for (int i = threadIdx.x; i < kMlpH * kMlpH; i += blockDim.x) S.W2[i] = (_Float16)prm_[kMlpOffW2 + i];
  for (int i = threadIdx.x; i < kMlpH; i += blockDim.x) {
    S.b1[i] = prm_[kMlpOffB1 + i];
    S.b2[i] = prm_[kMlpOffB2 + i];
    S.W3[i] = prm_[kMlpOffW3 + i];
  }
  if (threadIdx.x == 0) S.b3 = prm_[kMlpOffB3];
}

// S.x holds the 64 rows; returns the prediction of row `lane`
__device__ float mlp_wave_fp16(MlpLds &S) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  // layer 1: [64 x 16] x [16 x 64]
  for (int mt = 0; mt < 4; ++mt) {
    mlp_h4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = S.x[(mt * 16 + li) * kMlpF + 4 * lg + j];
    for (int nt = 0; nt < 4; ++nt) {
      mlp_h4 b;
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = S.W1[(nt * 16 + li) * kMlpF + 4 * lg + j];
      mlp_f4 c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = mt * 16 + 4 * lg + v, col = nt * 16 + li;
        const float hv = c[v] + S.b1[col];
        S.h[row * kMlpH + col] = (_Float16)(hv > 0.f ? hv : 0.f);
      }
    }
  }
  __syncthreads();
  // layer 2: [64 x 64] x [64 x 64], then the output layer on the fragments
  for (int mt = 0; mt < 4; ++mt) {
    float part[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nt = 0; nt < 4; ++nt) {
      mlp_f4 c = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < 4; ++kt) {
        mlp_h4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = S.h[(mt * 16 + li) * kMlpH + kt * 16 + 4 * lg + j];
          b[j] = S.W2[(nt * 16 + li) * kMlpH + kt * 16 + 4 * lg + j];
        }
        c = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
      }
      const int col = nt * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float hv = c[v] + S.b2[col];
        part[v] += S.W3[col] * (hv > 0.f ? hv : 0.f);
      }
    }
    // sum over the 16 columns held by lanes li = 0..15 of this lg
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float p = part[v];
      for (int o = 1; o < 16; o <<= 1) p += __shfl_xor(p, o, 64);
      if (li == 0) S.pred[mt * 16 + 4 * lg + v] = p + S.b3;
    }
  }
  __syncthreads();
  return S.pred[lane];
}

__device__ __forceinline__ void mlp_standardise(const float *prm_, const float *f, _Float16 *xrow, bool &inside) {
  inside = true;
  for (int k = 0; k < kMlpF; ++k) {
    const float lo = prm_[kMlpOffLo + k], hi = prm_[kMlpOffHi + k];
    if (f[k] < lo || f[k] > hi) inside = false;
    xrow[k] = (_Float16)((f[k] - prm_[kMlpOffMean + k]) * prm_[kMlpOffIstd + k]);
  }
}

// keep mask over all candidates: one wave per 64 candidates
__global__ __launch_bounds__(64) void mlp_mask_kernel(const SRParams prm, int ntrip, int64_t ncand,
                                                      const float *__restrict__ prm_, float cut, uint8_t *__restrict__ mask,
                                                      long long *__restrict__ nskip) {
  __shared__ MlpLds S;
  mlp_load_lds(prm_, S);
  const int lane = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  bool cand = false, inside = false;
  float f[kMlpF];
  for (int k = 0; k < kMlpF; ++k) f[k] = 0.f;
  if (c < ncand) {
    const int t = find_trip(prm.cand_off, ntrip, c);
    cand = sr_candidate_features(prm, t, (int)(c - prm.cand_off[t]), f);
  }
  mlp_standardise(prm_, f, &S.x[lane * kMlpF], inside);
  __syncthreads();
  const float pred = mlp_wave_fp16(S);
  const bool drop = cand && inside && (pred < cut);
  if (c < ncand) mask[c] = drop ? 0 : 1;
  long long d = drop ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
  if (lane == 0 && d) atomicAdd(reinterpret_cast<unsigned long long *>(nskip), (unsigned long long)d);
}

hipError_t launch_mlp_mask(const SRParams &prm, int ntrip, int64_t ncand, const float *params, float cut,
                           uint8_t *mask, long long *nskip, hipStream_t stream) {
  if (ncand <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_mask_kernel, dim3((unsigned)((ncand + 63) / 64)), dim3(64), 0, stream, prm, ntrip, ncand,
                     params, cut, mask, nskip);
  return hipGetLastError();
}

// predictions for raw feature rows: FP32 on the vector ALUs (mode 0) or the
// FP16 matrix-core path of the mask kernel (mode 1)
__global__ __launch_bounds__(64) void mlp_predict_kernel(const float *__restrict__ prm_, const float *__restrict__ X,
                                                         int64_t n, int mode, float *__restrict__ pred) {
  __shared__ MlpLds S;
  const int lane = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  float f[kMlpF];
  for (int k = 0; k < kMlpF; ++k) f[k] = (r < n) ? X[r * kMlpF + k] : 0.f;
  if (mode == 1) {
    mlp_load_lds(prm_, S);
    bool inside;
    mlp_standardise(prm_, f, &S.x[lane * kMlpF], inside);
    __syncthreads();
    const float p = mlp_wave_fp16(S);
    if (r < n) pred[r] = p;
    return;
  }
  float x[kMlpF], h1[kMlpH];
  for (int k = 0; k < kMlpF; ++k) x[k] = (f[k] - prm_[kMlpOffMean + k]) * prm_[kMlpOffIstd + k];
  for (int j = 0; j < kMlpH; ++j) {
    float a = prm_[kMlpOffB1 + j];
    for (int k = 0; k < kMlpF; ++k) a += prm_[kMlpOffW1 + j * kMlpF + k] * x[k];
    h1[j] = a > 0.f ? a : 0.f;
  }
  float out = prm_[kMlpOffB3];
  for (int j = 0; j < kMlpH; ++j) {
    float a = prm_[kMlpOffB2 + j];
    for (int k = 0; k < kMlpH; ++k) a += prm_[kMlpOffW2 + j * kMlpH + k] * h1[k];
    out += prm_[kMlpOffW3 + j] * (a > 0.f ? a : 0.f);
  }
  if (r < n) pred[r] = out;
}

hipError_t launch_mlp_predict(const float *params, const float *X, int64_t n, int mode, float *pred,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream, params, X, n, mode,
                     pred);
  return hipGetLastError();
}

}  // namespace rsgdf
