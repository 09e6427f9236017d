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
// E elements (Y holds Nk^2 complex values per element).  Both stages run on
// the FP64 matrix cores, 64 elements x up to 64 transform outputs per
// workgroup, so that each reads its input about once.  Per element this is
// 2 Nk^3 + 4 Nk Nkp multiply-adds instead of 2 Nk^2 Nkp.  The second stage's epilogue subtracts pi/(Omega w^2) S_P S_{mu nu}(k)
// on the k1 == k2 pairs.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "plan.h"
#include "kernels.h"

namespace rsgdf {

typedef double fd_d4 __attribute__((ext_vector_type(4)));
typedef double fd_d2 __attribute__((ext_vector_type(2)));
constexpr int FD_TE = 64;     // elements per workgroup: 4 column blocks of 16
constexpr int FD_TKMAX = 64;  // k-pair slots per stage-2 tile at most (4 wavefronts of 16)

// Both stages are products with the phase table on the FP64 matrix cores
// (v_mfma_f64_16x16x4): a wavefront owns 16 transform outputs (rows) x 64
// elements (4 column blocks), four cells per step.  Fragments (li = lane % 16,
// lg = lane / 16): A[li][lg] = the phase of row li at cell 4 s + lg, B[lg][li]
// = the input of that cell at element li of the block, result D[lg + 4 v][li].
// The phases of a lane's row are one 16-byte load per step, the inputs are
// read straight from memory (the wavefronts of a workgroup share them in the
// caches).  Rows past the end read a valid phase row and are not stored; cells
// past nk get zero phases; elements past the chunk read the last element and
// are not stored.

// stage 1: grid (element tiles of the chunk, k2 groups of 16 W, c1), W
// wavefronts per workgroup, wavefront w taking k2 = 16 (W y + w) .. + 16:
//   Yr[k2][e] = sum_c2 cos(k2.L_c2) X[c1][c2][e],  Yi likewise with sin
__global__ __launch_bounds__(256) void fold_k2_kernel(const FoldParams fp, int64_t e0, int64_t E) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int nk = fp.nk, c1 = blockIdx.z;
  const int kb = blockIdx.y * (blockDim.x >> 6) + (threadIdx.x >> 6);  // 16-row block of k2
  if (kb * 16 >= nk) return;  // no barriers below
  const double *pha = fp.kph + 2 * (size_t)min(kb * 16 + li, nk - 1) * nk;
  const int64_t eb = (int64_t)blockIdx.x * FD_TE;
  const double *xc = fp.X + (int64_t)c1 * nk * fp.ne + e0;  // X[c1][c][e0 + e] at xc[c ne + e]
  int64_t ecol[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) ecol[cb] = min(eb + cb * 16 + li, E - 1);
  fd_d4 yc[4], ys[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) yc[cb][v] = ys[cb][v] = 0.0;
  // two register sets in turn: the operands of one step are loaded while the
  // matrix cores work on the other (a load's cell is clamped into range; the
  // products of cells past nk take zero phases)
  struct Ops {
    double ac, as, x[4];
  };
  auto load = [&](int c0, Ops &o) {
    const int c = c0 + lg, cr = min(c, nk - 1);
    const fd_d2 p = *reinterpret_cast<const fd_d2 *>(pha + 2 * cr);
    o.ac = c < nk ? p.x : 0.0;
    o.as = c < nk ? p.y : 0.0;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) o.x[cb] = xc[(int64_t)cr * fp.ne + ecol[cb]];
  };
  auto step = [&](const Ops &o) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      yc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.ac, o.x[cb], yc[cb], 0, 0, 0);
      ys[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.as, o.x[cb], ys[cb], 0, 0, 0);
    }
  };
  Ops oa, ob;
  load(0, oa);
  for (int c0 = 0; c0 < nk; c0 += 8) {
    load(c0 + 4, ob);
    step(oa);
    load(c0 + 8, oa);
    if (c0 + 4 < nk) step(ob);
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k2 = kb * 16 + lg + 4 * v;
      const int64_t e = eb + cb * 16 + li;
      if (k2 < nk && e < E) {
        const int64_t o = ((int64_t)c1 * nk + k2) * E + e;
        fp.Y[2 * o] = yc[cb][v];
        fp.Y[2 * o + 1] = ys[cb][v];
      }
    }
}

// stage 2: grid (element tiles of the chunk, k-pair tiles); a tile holds up to
// fp.tk (<= 64) k-pairs (k1, k2) sharing k2, one tile per k2 when they fit,
// wavefront w its slots 16 w .. + 16 (a wavefront whose first slot is empty has
// none and returns).  With the table entry (c, s) of k1 at c1:
//   out_re += c Yr + s Yi,  out_im += c Yi - s Yr     (e^{-i k1.L_c1} = c - i s)
// and on the k1 == k2 pairs the G = 0 term is subtracted.
__global__ __launch_bounds__(256) void fold_k1_kernel(const FoldParams fp, int64_t e0, int64_t E) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4, w = threadIdx.x >> 6;
  const int tile = blockIdx.y, nk = fp.nk, tk = fp.tk;
  const int32_t *slots = fp.tile_kp + (size_t)tile * tk;
  if (w * 16 >= tk || slots[w * 16] < 0) return;  // slots are filled in order; no barriers below
  const int k2 = fp.tile_k2[tile];
  const int sa = w * 16 + li;
  const int kpa = sa < tk ? slots[sa] : -1;
  const double *pha = fp.kph + 2 * (size_t)(kpa >= 0 ? fp.kp1[kpa] : 0) * nk;
  const int64_t eb = (int64_t)blockIdx.x * FD_TE;
  int64_t ecol[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) ecol[cb] = min(eb + cb * 16 + li, E - 1);
  fd_d4 orr[4], oi[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) orr[cb][v] = oi[cb][v] = 0.0;
  if (fp.Y) {
    // two register sets in turn, as in stage 1
    const double *yk = fp.Y + 2 * (int64_t)k2 * E;  // Y[c1][k2][e] at yk[2 (c1 nk E + e)]
    struct Ops {
      double ac, as;
      fd_d2 y[4];
    };
    auto load = [&](int c0, Ops &o) {
      const int c = c0 + lg, cr = min(c, nk - 1);
      const fd_d2 p = *reinterpret_cast<const fd_d2 *>(pha + 2 * cr);
      o.ac = c < nk ? p.x : 0.0;
      o.as = c < nk ? p.y : 0.0;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        o.y[cb] = *reinterpret_cast<const fd_d2 *>(yk + 2 * ((int64_t)cr * nk * E + ecol[cb]));
    };
    auto step = [&](const Ops &o) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        orr[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.ac, o.y[cb].x, orr[cb], 0, 0, 0);
        oi[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.ac, o.y[cb].y, oi[cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        orr[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.as, o.y[cb].y, orr[cb], 0, 0, 0);
        oi[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-o.as, o.y[cb].x, oi[cb], 0, 0, 0);
      }
    };
    Ops oa, ob;
    load(0, oa);
    for (int c0 = 0; c0 < nk; c0 += 8) {
      load(c0 + 4, ob);
      step(oa);
      load(c0 + 8, oa);
      if (c0 + 4 < nk) step(ob);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int sl = w * 16 + lg + 4 * v;
    const int kp = sl < tk ? slots[sl] : -1;
    if (kp < 0) continue;
    const int k = fp.kdiag[kp];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int64_t e = eb + cb * 16 + li;
      if (e >= E) continue;
      const int64_t ebat = e0 + e;  // element index within the aux batch
      double vr = orr[cb][v], vi = oi[cb][v];
      if (k >= 0 && fp.g0fac != 0.0) {
        const int64_t P = ebat / fp.nao2, mn = ebat - P * fp.nao2;
        const double s = fp.g0fac * fp.SP[P];
        vr -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn)];
        vi -= s * fp.Smn[2 * ((int64_t)k * fp.nao2 + mn) + 1];
      }
      const int64_t o = (int64_t)kp * fp.plane + fp.out_off + ebat;
      fp.out[2 * o] = vr;
      fp.out[2 * o + 1] = vi;
    }
  }
}

hipError_t launch_fold(const FoldParams &fp, hipStream_t stream) {
  if (fp.ne == 0 || fp.ntile == 0) return hipSuccess;
  if (fp.echunk < 1 || (fp.X && !fp.Y)) return hipErrorInvalidValue;
  if (fp.tk < 4 || fp.tk > FD_TKMAX || fp.tk % 4 != 0 || fp.nk < 1) return hipErrorInvalidValue;
  // stage 1: up to 4 wavefronts (64 k2) per workgroup; stage 2: one per 16 slots
  const int nkb = (fp.nk + 15) / 16, w1 = nkb < 4 ? nkb : 4, w2 = (fp.tk + 15) / 16;
  for (int64_t e0 = 0; e0 < fp.ne; e0 += fp.echunk) {
    const int64_t E = fp.ne - e0 < fp.echunk ? fp.ne - e0 : fp.echunk;
    const int64_t nt = (E + FD_TE - 1) / FD_TE;
    if (nt > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (fp.X)
      hipLaunchKernelGGL(fold_k2_kernel, dim3((unsigned)nt, (unsigned)((nkb + w1 - 1) / w1), (unsigned)fp.nk),
                         dim3(64 * w1), 0, stream, fp, e0, E);
    FoldParams f2 = fp;
    if (!fp.X) f2.Y = nullptr;  // no short-range part: zeros plus the G = 0 term
    hipLaunchKernelGGL(fold_k1_kernel, dim3((unsigned)nt, (unsigned)fp.ntile), dim3(64 * w2), 0, stream, f2, e0, E);
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
