// fold.hip -- Bloch fold of the BvK-binned short-range sums (Eq. M14) with the
// G = 0 correction of Eq. (M12), and the lattice-summed overlaps S_{mu nu}(k)
// of Eq. (M13c) it needs.
//
// The phase of a BvK cell pair factorises, e^{-i k1.L_c1} e^{+i k2.L_c2}, so the
// fold is two discrete Fourier transforms over the Nk cells instead of one
// product over the Nk^2 cell pairs:
//     Y[c1][k2][e]  = sum_c2 e^{+i k2.L_c2} X[c1][c2][e]          (real input)
//     out[kp][e]    = sum_c1 e^{-i k1.L_c1} Y[c1][k2][e],  kp = (k1, k2), k1 <= k2
// over the output elements e = (P, mu, nu) of one aux batch, taken in chunks of
// E elements (Y holds Nk^2 complex values per element).  Both stages take 64
// elements x 16 transform outputs per workgroup (4 outputs per wavefront), the
// element values staged through LDS 32 cells at a time, the phases read by
// scalar loads.  Per element this is 2 Nk^3 + 4 Nk Nkp multiply-adds instead of
// 2 Nk^2 Nkp.  The second stage's epilogue subtracts pi/(Omega w^2) S_P S_{mu nu}(k)
// on the k1 == k2 pairs.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "plan.h"
#include "kernels.h"

namespace rsgdf {

constexpr int FD_TE = 64;  // elements per tile
constexpr int FD_TK = 16;  // transform outputs (k2, or k-pairs of one k2) per tile
constexpr int FD_TC = 32;  // cells per LDS stage

// stage 1: grid (element tiles of the chunk, k2 tiles, c1).  The four
// transform outputs of a wavefront are the same for its 64 lanes, so their
// phases are read with scalar loads (the wave index is made uniform), and LDS
// holds only the X tile: one LDS read per eight multiply-adds.
__global__ __launch_bounds__(256) void fold_k2_kernel(const FoldParams fp, int64_t e0, int64_t E) {
  __shared__ double sX[FD_TC][FD_TE];
  const int tx = threadIdx.x & 63;
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // 4 outputs per wave
  const int64_t e = (int64_t)blockIdx.x * FD_TE + tx;
  const int k20 = blockIdx.y * FD_TK, c1 = blockIdx.z, nk = fp.nk;
  // phase rows of the wave's outputs (a row past nk repeats a valid one; its sums are not stored)
  const double *ph[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k2 = k20 + ty * 4 + j;
    ph[j] = fp.kph + 2 * (size_t)(k2 < nk ? k2 : nk - 1) * nk;
  }
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  for (int c0 = 0; c0 < nk; c0 += FD_TC) {
    for (int i = threadIdx.x; i < FD_TC * FD_TE; i += 256) {
      const int cc = i / FD_TE, ee = i % FD_TE;
      const int64_t eg = (int64_t)blockIdx.x * FD_TE + ee;
      sX[cc][ee] = (c0 + cc < nk && eg < E) ? fp.X[(int64_t)(c1 * nk + c0 + cc) * fp.ne + e0 + eg] : 0.0;
    }
    __syncthreads();
    const int nc = nk - c0 < FD_TC ? nk - c0 : FD_TC;
#pragma unroll 4
    for (int cc = 0; cc < nc; ++cc) {
      const double x = sX[cc][tx];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ar[j] += ph[j][2 * (c0 + cc)] * x;
        ai[j] += ph[j][2 * (c0 + cc) + 1] * x;
      }
    }
    __syncthreads();
  }
  if (e >= E) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k2 = k20 + ty * 4 + j;
    if (k2 >= nk) continue;
    const int64_t o = ((int64_t)c1 * nk + k2) * E + e;
    fp.Y[2 * o] = ar[j];
    fp.Y[2 * o + 1] = ai[j];
  }
}

// stage 2: grid (element tiles of the chunk, k-pair tiles); a tile holds up to
// 16 k-pairs (k1, k2) sharing k2, so the staged Y rows serve all of them; the
// phases e^{-i k1.L_c1} of a wavefront's four k-pairs by scalar loads
__global__ __launch_bounds__(256) void fold_k1_kernel(const FoldParams fp, int64_t e0, int64_t E) {
  __shared__ double sYr[FD_TC][FD_TE], sYi[FD_TC][FD_TE];
  const int tx = threadIdx.x & 63;
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = (int64_t)blockIdx.x * FD_TE + tx;
  const int tile = blockIdx.y, nk = fp.nk;
  const int k2 = fp.tile_k2[tile];
  const double *ph[4];
  bool on[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kp = fp.tile_kp[tile * FD_TK + ty * 4 + j];
    on[j] = kp >= 0;
    ph[j] = fp.kph + 2 * (size_t)(on[j] ? fp.kp1[kp] : 0) * nk;  // an unused slot reads row 0
  }
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  if (fp.Y) {
    for (int c0 = 0; c0 < nk; c0 += FD_TC) {
      for (int i = threadIdx.x; i < FD_TC * FD_TE; i += 256) {
        const int cc = i / FD_TE, ee = i % FD_TE;
        const int64_t eg = (int64_t)blockIdx.x * FD_TE + ee;
        const bool ok = c0 + cc < nk && eg < E;
        const int64_t o = ((int64_t)(c0 + cc) * nk + k2) * E + eg;
        sYr[cc][ee] = ok ? fp.Y[2 * o] : 0.0;
        sYi[cc][ee] = ok ? fp.Y[2 * o + 1] : 0.0;
      }
      __syncthreads();
      const int nc = nk - c0 < FD_TC ? nk - c0 : FD_TC;
#pragma unroll 4
      for (int cc = 0; cc < nc; ++cc) {
        const double yr = sYr[cc][tx], yi = sYi[cc][tx];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // e^{-i k1.L_c1} = conjugate of the table entry
          const double pr = ph[j][2 * (c0 + cc)], pi = -ph[j][2 * (c0 + cc) + 1];
          ar[j] += pr * yr - pi * yi;
          ai[j] += pr * yi + pi * yr;
        }
      }
      __syncthreads();
    }
  }
  if (e >= E) return;
  const int64_t eb = e0 + e;  // element index within the aux batch
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!on[j]) continue;
    const int kp = fp.tile_kp[tile * FD_TK + ty * 4 + j];
    double vr = ar[j], vi = ai[j];
    const int k = fp.kdiag[kp];
    if (k >= 0 && fp.g0fac != 0.0) {
      const int64_t P = eb / fp.nao2, mn = eb - P * fp.nao2;
      const double s = fp.g0fac * fp.SP[P];
      vr -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn)];
      vi -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn) + 1];
    }
    const int64_t o = (int64_t)kp * fp.plane + fp.out_off + eb;
    fp.out[2 * o] = vr;
    fp.out[2 * o + 1] = vi;
  }
}

hipError_t launch_fold(const FoldParams &fp, hipStream_t stream) {
  if (fp.ne == 0 || fp.ntile == 0) return hipSuccess;
  if (fp.echunk < 1 || (fp.X && !fp.Y)) return hipErrorInvalidValue;
  for (int64_t e0 = 0; e0 < fp.ne; e0 += fp.echunk) {
    const int64_t E = fp.ne - e0 < fp.echunk ? fp.ne - e0 : fp.echunk;
    const int64_t nt = (E + FD_TE - 1) / FD_TE;
    if (nt > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (fp.X)
      hipLaunchKernelGGL(fold_k2_kernel, dim3((unsigned)nt, (unsigned)((fp.nk + FD_TK - 1) / FD_TK), (unsigned)fp.nk),
                         dim3(256), 0, stream, fp, e0, E);
    FoldParams f2 = fp;
    if (!fp.X) f2.Y = nullptr;  // no short-range part: zeros plus the G = 0 term
    hipLaunchKernelGGL(fold_k1_kernel, dim3((unsigned)nt, (unsigned)fp.ntile), dim3(256), 0, stream, f2, e0, E);
  }
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
        if (op.acut > 0.0 && ga < op.acut && gb < op.acut) continue;  // a diffuse-diffuse pair: Eq. M15
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
