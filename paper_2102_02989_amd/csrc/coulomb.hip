// coulomb.hip -- contractions of the integral-direct density-fitted Coulomb
// build (a consumer of the three-center integrals that never stores them):
//   rho_Q   = sum_k sum_{lambda sigma} V^{kk}_{Q lambda sigma} D^k_{sigma lambda}
//   J^0 c   = rho                       (the fitting equation, Eq. M4, at k12 = 0)
//   J_{mu nu}(k) = (1/N_k) sum_Q V^{kk}_{Q mu nu} c_Q
// evaluated per group of aux functions on V tiles that are rebuilt for each
// pass instead of kept.  With d = (J^0)^{-1} V this is the density-fitted
// J_{mu nu}(k) = (1/N_k) sum_{k', lambda sigma} (rho^{kk}_{mu nu} | rho^{k'k'}_{lambda sigma}) D^{k'}_{sigma lambda}
// of Eq. M7 with k1 = k2 and k3 = k4.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace rsgdf {

// rho[Q] (Q in the group, written) = sum_k sum_e V[k][Q][e] D[k][nu][mu],
// e = mu nao + nu; one workgroup per Q, partial sums per thread over a fixed
// stride, then a fixed-order tree through LDS (reproducible)
__global__ __launch_bounds__(256) void dm_contract_kernel(const double *__restrict__ V, const double *__restrict__ D,
                                                          int nk, int ng, int nao, double *__restrict__ rho) {
  __shared__ double sr[256], si[256];
  const int Q = blockIdx.x, tid = threadIdx.x;
  const int64_t ne = (int64_t)nao * nao;
  double ar = 0.0, ai = 0.0;
  for (int k = 0; k < nk; ++k) {
    const double *Vk = V + 2 * (((int64_t)k * ng + Q) * ne);
    const double *Dk = D + 2 * ((int64_t)k * ne);
    for (int64_t e = tid; e < ne; e += 256) {
      const int64_t mu = e / nao, nu = e % nao;
      const double vr = Vk[2 * e], vi = Vk[2 * e + 1];
      const double dr = Dk[2 * (nu * nao + mu)], di = Dk[2 * (nu * nao + mu) + 1];
      ar += vr * dr - vi * di;
      ai += vr * di + vi * dr;
    }
  }
  sr[tid] = ar;
  si[tid] = ai;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) {
      sr[tid] += sr[tid + w];
      si[tid] += si[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    rho[2 * Q] = sr[0];
    rho[2 * Q + 1] = si[0];
  }
}

// vj[k][e] += scale sum_Q c[Q] V[k][Q][e] over the group's Q, one thread per (k, e)
__global__ __launch_bounds__(256) void vj_accum_kernel(const double *__restrict__ V, const double *__restrict__ c,
                                                       int nk, int ng, int64_t ne, double scale,
                                                       double *__restrict__ vj) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nk * ne) return;
  const int64_t k = i / ne, e = i % ne;
  double sr = 0.0, si = 0.0;
  for (int Q = 0; Q < ng; ++Q) {
    const double cr = c[2 * Q], ci = c[2 * Q + 1];
    const double vr = V[2 * ((k * ng + Q) * ne + e)], vi = V[2 * ((k * ng + Q) * ne + e) + 1];
    sr += cr * vr - ci * vi;
    si += cr * vi + ci * vr;
  }
  vj[2 * i] += scale * sr;
  vj[2 * i + 1] += scale * si;
}

hipError_t launch_dm_contract(const double *V, const double *D, int nk, int ng, int nao, double *rho,
                              hipStream_t stream) {
  if (ng == 0) return hipSuccess;
  hipLaunchKernelGGL(dm_contract_kernel, dim3((unsigned)ng), dim3(256), 0, stream, V, D, nk, ng, nao, rho);
  return hipGetLastError();
}

hipError_t launch_vj_accum(const double *V, const double *c, int nk, int ng, int64_t ne, double scale, double *vj,
                           hipStream_t stream) {
  const int64_t n = (int64_t)nk * ne;
  if (n == 0 || ng == 0) return hipSuccess;
  if ((n + 255) / 256 > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(vj_accum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, V, c, nk, ng, ne, scale,
                     vj);
  return hipGetLastError();
}

}  // namespace rsgdf
