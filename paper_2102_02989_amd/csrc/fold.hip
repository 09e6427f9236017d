// fold.hip -- Bloch fold of the BvK-binned short-range sums (Eq. M14) with the
// G = 0 correction of Eq. (M12), and the lattice-summed overlaps S_{mu nu}(k)
// of Eq. (M13c) it needs.
//
// The fold is a complex-by-real product
//     out[kp][e] = sum_{b = (c1,c2)} Phi[kp][b] X[b][e],
//     Phi[kp][(c1,c2)] = exp(-i k1.L_c1) exp(+i k2.L_c2),
// over the output elements e = (P, mu, nu) of one aux batch, tiled through LDS.
// Its epilogue subtracts pi/(Omega w^2) S_P S_{mu nu}(k) on the k1 == k2 pairs.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "plan.h"
#include "kernels.h"

namespace rsgdf {

constexpr int FOLD_TE = 64;   // elements per tile
constexpr int FOLD_TK = 16;   // k-pairs per tile
constexpr int FOLD_TB = 32;   // BvK cell pairs per LDS stage



__global__ __launch_bounds__(256) void fold_kernel(const FoldParams fp) {
  __shared__ double sX[FOLD_TB][FOLD_TE];
  __shared__ double sPr[FOLD_TK][FOLD_TB], sPi[FOLD_TK][FOLD_TB];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // ty in [0,4): 4 k-pairs each
  const int64_t e = (int64_t)blockIdx.x * FOLD_TE + tx;
  const int kp0 = blockIdx.y * FOLD_TK;
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  if (fp.X) {
    for (int b0 = 0; b0 < fp.nb; b0 += FOLD_TB) {
      for (int i = threadIdx.x; i < FOLD_TB * FOLD_TE; i += 256) {
        const int bb = i / FOLD_TE, ee = i % FOLD_TE;
        const int64_t eg = (int64_t)blockIdx.x * FOLD_TE + ee;
        sX[bb][ee] = (b0 + bb < fp.nb && eg < fp.ne) ? fp.X[(int64_t)(b0 + bb) * fp.ne + eg] : 0.0;
      }
      for (int i = threadIdx.x; i < FOLD_TK * FOLD_TB; i += 256) {
        const int kk = i / FOLD_TB, bb = i % FOLD_TB;
        const bool ok = (kp0 + kk < fp.nkp) && (b0 + bb < fp.nb);
        sPr[kk][bb] = ok ? fp.phi[2 * ((int64_t)(kp0 + kk) * fp.nb + b0 + bb)] : 0.0;
        sPi[kk][bb] = ok ? fp.phi[2 * ((int64_t)(kp0 + kk) * fp.nb + b0 + bb) + 1] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int bb = 0; bb < FOLD_TB; ++bb) {
        const double x = sX[bb][tx];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ar[j] += sPr[ty * 4 + j][bb] * x;
          ai[j] += sPi[ty * 4 + j][bb] * x;
        }
      }
      __syncthreads();
    }
  }
  if (e >= fp.ne) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kp = kp0 + ty * 4 + j;
    if (kp >= fp.nkp) continue;
    double vr = ar[j], vi = ai[j];
    const int k = fp.kdiag[kp];
    if (k >= 0 && fp.g0fac != 0.0) {
      const int64_t P = e / fp.nao2, mn = e - P * fp.nao2;
      const double s = fp.g0fac * fp.SP[P];
      vr -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn)];
      vi -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn) + 1];
    }
    const int64_t o = (int64_t)kp * fp.plane + fp.out_off + e;
    fp.out[2 * o] = vr;
    fp.out[2 * o + 1] = vi;
  }
}

hipError_t launch_fold(const FoldParams &fp, hipStream_t stream) {
  dim3 grid((unsigned)((fp.ne + FOLD_TE - 1) / FOLD_TE), (unsigned)((fp.nkp + FOLD_TK - 1) / FOLD_TK));
  hipLaunchKernelGGL(fold_kernel, grid, dim3(256), 0, stream, fp);
  return hipGetLastError();
}

// ---- lattice-summed overlaps ------------------------------------------------
// O[pair][c][a][b] = sum over images n' of BvK class c of int phi_a(r-A) phi_b(r-B-n') dr
// with the Hermite expansion: overlap = K (pi/p)^{3/2} E^x_0 E^y_0 E^z_0.


template <int LA, int LB>
__device__ void ovl_pair_class(const OvlParams &op, int ip, int c) {
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  const Pair pr = op.pairs[ip];
  const Shell sA = op.ao[pr.sa], sB = op.ao[pr.sb];
  double acc[NCA * NCB];
#pragma unroll
  for (int i = 0; i < NCA * NCB; ++i) acc[i] = 0.0;
  const int beg = op.cls_off[pr.cls_off + c], end = op.cls_off[pr.cls_off + c + 1];
  for (int ii = beg; ii < end; ++ii) {
    const double *nv = op.img + 3 * (size_t)(pr.img_off + ii);
    const double Bx = sB.x + nv[0], By = sB.y + nv[1], Bz = sB.z + nv[2];
    const double r2 = (sA.x - Bx) * (sA.x - Bx) + (sA.y - By) * (sA.y - By) + (sA.z - Bz) * (sA.z - Bz);
    for (int ka = 0; ka < sA.nprim; ++ka)
      for (int kb = 0; kb < sB.nprim; ++kb) {
        const double ga = op.ao_exp[sA.pptr + ka], gb = op.ao_exp[sB.pptr + kb];
        const double p = ga + gb, oop = 1.0 / p;
        const double arg = ga * gb * oop * r2;
        if (arg > 46.0) continue; /* e^{-46} ~ 1e-20 */
        const double K = exp(-arg) * op.ao_coef[sA.pptr + ka] * op.ao_coef[sB.pptr + kb] * kPi * oop * sqrt(kPi * oop);
        const double Px = (ga * sA.x + gb * Bx) * oop, Py = (ga * sA.y + gb * By) * oop, Pz = (ga * sA.z + gb * Bz) * oop;
        double Ex[LA + 1][LB + 1][LA + LB + 1], Ey[LA + 1][LB + 1][LA + LB + 1], Ez[LA + 1][LB + 1][LA + LB + 1];
        hermite_E<LA, LB>(Px - sA.x, Px - Bx, 0.5 * oop, Ex);
        hermite_E<LA, LB>(Py - sA.y, Py - By, 0.5 * oop, Ey);
        hermite_E<LA, LB>(Pz - sA.z, Pz - Bz, 0.5 * oop, Ez);
#pragma unroll
        for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
          for (int ib = 0; ib < NCB; ++ib)
            acc[ia * NCB + ib] += K * Ex[cart_lx(LA, ia)][cart_lx(LB, ib)][0] * Ey[cart_ly(LA, ia)][cart_ly(LB, ib)][0] *
                                  Ez[cart_lz(LA, ia)][cart_lz(LB, ib)][0];
      }
  }
  double *dst = op.O + ((size_t)ip * op.nk + c) * 36;
#pragma unroll
  for (int i = 0; i < NCA * NCB; ++i) dst[i] = acc[i];
}

__global__ void ovl_kernel(const OvlParams op) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)op.npair * op.nk) return;
  const int ip = (int)(gid / op.nk), c = (int)(gid % op.nk);
  const Pair pr = op.pairs[ip];
  const int la = op.ao[pr.sa].l, lb = op.ao[pr.sb].l;
  switch (la * 3 + lb) {
    case 0: ovl_pair_class<0, 0>(op, ip, c); break;
    case 3: ovl_pair_class<1, 0>(op, ip, c); break;
    case 4: ovl_pair_class<1, 1>(op, ip, c); break;
    case 6: ovl_pair_class<2, 0>(op, ip, c); break;
    case 7: ovl_pair_class<2, 1>(op, ip, c); break;
    case 8: ovl_pair_class<2, 2>(op, ip, c); break;
    default: break;
  }
}

// S[k][mu][nu] = sum_c exp(+i k.L_c) O[pair][c][a][b]; the transposed entry
// (nu, mu) of an off-diagonal pair is the complex conjugate.


__global__ void smn_kernel(const SmnParams sp) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)sp.npair * sp.nk * 36) return;
  const int comp = (int)(gid % 36);
  const int k = (int)((gid / 36) % sp.nk);
  const int ip = (int)(gid / (36 * (int64_t)sp.nk));
  const Pair pr = sp.pairs[ip];
  const Shell sA = sp.ao[pr.sa], sB = sp.ao[pr.sb];
  const int nca = ncart(sA.l), ncb = ncart(sB.l);
  if (comp >= nca * ncb) return;
  const int ia = comp / ncb, ib = comp % ncb;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < sp.nk; ++c) {
    const double o = sp.O[((size_t)ip * sp.nk + c) * 36 + comp];
    sr += sp.kphase[2 * (k * sp.nk + c)] * o;
    si += sp.kphase[2 * (k * sp.nk + c) + 1] * o;
  }
  const size_t base = (size_t)k * sp.nao * sp.nao;
  const int mu = sA.foff + ia, nu = sB.foff + ib;
  sp.S[2 * (base + (size_t)mu * sp.nao + nu)] = sr;
  sp.S[2 * (base + (size_t)mu * sp.nao + nu) + 1] = si;
  if (!pr.diag) {
    sp.S[2 * (base + (size_t)nu * sp.nao + mu)] = sr;
    sp.S[2 * (base + (size_t)nu * sp.nao + mu) + 1] = -si;
  }
}

hipError_t launch_overlaps(const OvlParams &op, const SmnParams &sp, hipStream_t stream) {
  int64_t n1 = (int64_t)op.npair * op.nk;
  hipLaunchKernelGGL(ovl_kernel, dim3((unsigned)((n1 + 127) / 128)), dim3(128), 0, stream, op);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t n2 = (int64_t)sp.npair * sp.nk * 36;
  hipLaunchKernelGGL(smn_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, stream, sp);
  return hipGetLastError();
}

// Zero fill with a kernel (no memset node, so the sequence can be captured
// into a graph and replayed): 16-byte stores, then the byte tail.
__global__ void zero_kernel(uint4 *__restrict__ p, size_t n16, unsigned char *__restrict__ tail, int ntail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = i; j < n16; j += stride) p[j] = make_uint4(0u, 0u, 0u, 0u);
  if (i < (size_t)ntail) tail[i] = 0;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
  if (bytes == 0 || !p) return hipSuccess;
  const size_t n16 = bytes / 16;
  const int ntail = (int)(bytes - n16 * 16);
  size_t blocks = (n16 + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<uint4 *>(p), n16,
                     reinterpret_cast<unsigned char *>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace rsgdf
