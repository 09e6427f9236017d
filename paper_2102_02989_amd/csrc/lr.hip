// lr.hip -- long-range (erf-attenuated) part in reciprocal space, Eqs. (M10)
// and (M11):
//   V^LR[k1,k2][P][mu nu] = sum_{q in Q(k12)} A[P][q] rho^{k2}[q][mu nu]
//   A[P][q]               = (4 pi/Omega) exp(-|q|^2/4w^2)/|q|^2 chi~_P(-q)
//   rho^{k2}_{mu nu}(q)   = sum_n exp(+i k2.n) int phi_mu(r) phi_nu(r-n) e^{-iq.r} dr
// with q = G + k12 over one folded k12 class.  Transforms are analytic: a
// Gaussian product is expanded in Hermite Gaussians (McMurchie-Davidson E
// coefficients), whose transforms are (-i q)^t times the s-type transform.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"
#include "plan.h"
#include "kernels.h"

namespace rsgdf {

// ---- aux transforms times the kernel weight ---------------------------------


template <int LP>
__device__ void auxft_one(const AuxFTParams &ap, int iq, int s) {
  constexpr int NC = ncart(LP);
  const Shell sh = ap.ax[s];
  const double qx = ap.q[3 * iq], qy = ap.q[3 * iq + 1], qz = ap.q[3 * iq + 2];
  const double q2 = qx * qx + qy * qy + qz * qz;
  const double w = ap.wfac * exp(-q2 / (4.0 * ap.omega * ap.omega)) / q2;
  // e^{+i q.C}
  const double ph = qx * sh.x + qy * sh.y + qz * sh.z;
  const double cph = cos(ph), sph = sin(ph);
  double accr[NC], acci[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) accr[i] = acci[i] = 0.0;
  for (int k = 0; k < sh.nprim; ++k) {
    const double g = ap.ax_exp[sh.pptr + k], c = ap.ax_coef[sh.pptr + k];
    const double amp = c * kPi / g * sqrt(kPi / g) * exp(-q2 / (4.0 * g));
    double E[LP + 1][LP + 1];
    hermite_E1<LP>(0.5 / g, E);
#pragma unroll
    for (int ic = 0; ic < NC; ++ic) {
      // F_d = sum_t E[i_d][t] (i q_d)^t  (complex)
      double fr[3], fi[3];
      const double qd[3] = {qx, qy, qz};
      const int pw[3] = {cart_lx(LP, ic), cart_ly(LP, ic), cart_lz(LP, ic)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double re = 0.0, im = 0.0, pr = 1.0, pi = 0.0;  // (i q)^t
#pragma unroll
        for (int t = 0; t <= LP; ++t) {
          if (t <= pw[d]) {
            re += E[pw[d]][t] * pr;
            im += E[pw[d]][t] * pi;
          }
          const double nr = -pi * qd[d], ni = pr * qd[d];
          pr = nr;
          pi = ni;
        }
        fr[d] = re;
        fi[d] = im;
      }
      double xr = fr[0] * fr[1] - fi[0] * fi[1], xi = fr[0] * fi[1] + fi[0] * fr[1];
      const double yr = xr * fr[2] - xi * fi[2], yi = xr * fi[2] + xi * fr[2];
      accr[ic] += amp * yr;
      acci[ic] += amp * yi;
    }
  }
#pragma unroll
  for (int ic = 0; ic < NC; ++ic) {
    const double vr = accr[ic] * cph - acci[ic] * sph, vi = accr[ic] * sph + acci[ic] * cph;
    const size_t o = (size_t)(sh.foff + ic) * ap.nq + iq;
    ap.A[2 * o] = w * vr;
    ap.A[2 * o + 1] = w * vi;
  }
}

__global__ void auxft_kernel(const AuxFTParams ap) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ap.nq * ap.nshell) return;
  const int s = (int)(gid / ap.nq), iq = (int)(gid % ap.nq);
  switch (ap.ax[s].l) {
    case 0: auxft_one<0>(ap, iq, s); break;
    case 1: auxft_one<1>(ap, iq, s); break;
    case 2: auxft_one<2>(ap, iq, s); break;
    case 3: auxft_one<3>(ap, iq, s); break;
    default: break;
  }
}

hipError_t launch_auxft(const AuxFTParams &ap, hipStream_t stream) {
  const int64_t n = (int64_t)ap.nq * ap.nshell;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(auxft_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, stream, ap);
  return hipGetLastError();
}

// ---- pair transforms binned by the BvK class of the pair image ------------
// I[c][mu nu][q] = sum over images n' of class c of
//                  int phi_mu(r) phi_nu(r - n') e^{-iq.r} dr   (no Bloch phase)
// so that rho^{k2}(q) = sum_c e^{+i k2.L_c} I[c][q] for every k2 (Eq. M11 with
// the phase sum regrouped over Born-von Karman cells as in Eq. M14).
//
// Only the orientation (sa, sb) of a pair is evaluated.  Substituting
// r -> r + n' shows that the transposed block of the negated class is the
// same number times e^{+i q.n'}, and for q = G + k_cls with k_cls on the
// k-mesh that phase is e^{+i k_cls.L_c} for every image of class c:
//   I[-c][nu mu][q] = e^{+i k_cls.L_c} I[c][mu nu][q].
//
// A term (primitive pair, image) is skipped when max_P |A[P][q]| times the
// bound  |c_a c_b| (pi/p)^{3/2} e^{-q^2/4p} e^{-beta r^2} (c_q + r)^{la+lb},
// c_q = 1 + |q|/2p + sqrt((la+lb)/2p), is below eps: it can move no output
// element by more than eps.  Images of a class are sorted by r, so the loop
// ends at the first skipped image beyond the maximiser r* of the r factor.
template <int LA, int LB>
__device__ long long pairft_binned_one(const PairFTParams &pp, int ip, int c, int iq) {
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  constexpr int LT = LA + LB;
  const Pair pr = pp.pairs[ip];
  const Shell s1 = pp.ao[pr.sa];
  const Shell s2 = pp.ao[pr.sb];
  const double qx = pp.q[3 * iq], qy = pp.q[3 * iq + 1], qz = pp.q[3 * iq + 2];
  const double q2 = qx * qx + qy * qy + qz * qz;
  const double qn = sqrt(q2);
  const double am = pp.amax[iq];
  const double cut = am > 0.0 ? pp.eps / am : 1e300;
  // (-i q_d)^t = qr[d][t] + i qi[d][t]
  double qr[3][LT + 1], qi[3][LT + 1];
  {
    const double qd[3] = {qx, qy, qz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double pw = 1.0;
#pragma unroll
      for (int t = 0; t <= LT; ++t) {
        const int m = t & 3;  // (-i)^t = 1, -i, -1, i
        qr[d][t] = (m == 0) ? pw : (m == 2 ? -pw : 0.0);
        qi[d][t] = (m == 1) ? -pw : (m == 3 ? pw : 0.0);
        pw *= qd[d];
      }
    }
  }
  double accr[NCA * NCB], acci[NCA * NCB];
#pragma unroll
  for (int i = 0; i < NCA * NCB; ++i) accr[i] = acci[i] = 0.0;
  long long cnt = 0;
  const int beg = pp.cls_off[pr.cls_off + c], end = pp.cls_off[pr.cls_off + c + 1];
  for (int ka = 0; ka < s1.nprim; ++ka)
    for (int kb = 0; kb < s2.nprim; ++kb) {
      const double ga = pp.ao_exp[s1.pptr + ka], gb = pp.ao_exp[s2.pptr + kb];
      const double p = ga + gb, oop = 1.0 / p, beta = ga * gb * oop;
      const double cc = pp.ao_coef[s1.pptr + ka] * pp.ao_coef[s2.pptr + kb];
      const double pre = kPi * oop * sqrt(kPi * oop);
      const double eq = exp(-q2 * 0.25 * oop);
      const double cq = 1.0 + 0.5 * qn * oop + sqrt(0.5 * LT * oop);
      const double rstar = 0.5 * (sqrt(cq * cq + 2.0 * LT / beta) - cq);
      const double amp0 = fabs(cc) * pre * eq;
      double fmax = amp0 * exp(-beta * rstar * rstar);
#pragma unroll
      for (int t = 0; t < LT; ++t) fmax *= (cq + rstar);
      if (fmax < cut) continue;
      const double camp = cc * pre * eq;
      for (int ii = beg; ii < end; ++ii) {
        const double *nv = pp.img + 3 * (size_t)(pr.img_off + ii);
        const double Bx = s2.x + nv[0], By = s2.y + nv[1], Bz = s2.z + nv[2];
        const double Rx = Bx - s1.x, Ry = By - s1.y, Rz = Bz - s1.z;
        const double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
        const double er = exp(-beta * r2);
        const double rr = sqrt(r2);
        double bnd = amp0 * er;
#pragma unroll
        for (int t = 0; t < LT; ++t) bnd *= (cq + rr);
        if (bnd < cut) {
          if (rr > rstar) break;
          continue;
        }
        ++cnt;
        // P - A = (gb/p) R, P - B = -(ga/p) R
        const double wa = gb * oop, wb = -ga * oop;
        const double Px = s1.x + wa * Rx, Py = s1.y + wa * Ry, Pz = s1.z + wa * Rz;
        double sph, cph;
        sincos(-(qx * Px + qy * Py + qz * Pz), &sph, &cph);
        const double amp = camp * er;
        const double cr = amp * cph, ci = amp * sph;
        // F_d[i][j] = sum_t E_d[i][j][t] (-i q_d)^t
        double Fr[3][LA + 1][LB + 1], Fi[3][LA + 1][LB + 1];
        {
          double E[LA + 1][LB + 1][LT + 1];
          const double Rd[3] = {Rx, Ry, Rz};
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            hermite_E<LA, LB>(wa * Rd[d], wb * Rd[d], 0.5 * oop, E);
#pragma unroll
            for (int i = 0; i <= LA; ++i)
#pragma unroll
              for (int j = 0; j <= LB; ++j) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int t = 0; t <= i + j; ++t) {
                  if ((t & 1) == 0) re += E[i][j][t] * qr[d][t];
                  else im += E[i][j][t] * qi[d][t];
                }
                Fr[d][i][j] = re;
                Fi[d][i][j] = im;
              }
          }
        }
        // fold the amplitude and phase into the x factor
        double Gr[LA + 1][LB + 1], Gi[LA + 1][LB + 1];
#pragma unroll
        for (int i = 0; i <= LA; ++i)
#pragma unroll
          for (int j = 0; j <= LB; ++j) {
            Gr[i][j] = cr * Fr[0][i][j] - ci * Fi[0][i][j];
            Gi[i][j] = cr * Fi[0][i][j] + ci * Fr[0][i][j];
          }
#pragma unroll
        for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
          for (int ib = 0; ib < NCB; ++ib) {
            const int ax_ = cart_lx(LA, ia), ay_ = cart_ly(LA, ia), az_ = cart_lz(LA, ia);
            const int bx_ = cart_lx(LB, ib), by_ = cart_ly(LB, ib), bz_ = cart_lz(LB, ib);
            const double xr = Gr[ax_][bx_] * Fr[1][ay_][by_] - Gi[ax_][bx_] * Fi[1][ay_][by_];
            const double xi = Gr[ax_][bx_] * Fi[1][ay_][by_] + Gi[ax_][bx_] * Fr[1][ay_][by_];
            accr[ia * NCB + ib] += xr * Fr[2][az_][bz_] - xi * Fi[2][az_][bz_];
            acci[ia * NCB + ib] += xr * Fi[2][az_][bz_] + xi * Fr[2][az_][bz_];
          }
      }
    }
  const int nao = pp.nao;
  const size_t nq = pp.nq;
  double *Ic = pp.B + 2 * ((size_t)c * nao * nao * nq);
#pragma unroll
  for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NCB; ++ib) {
      const size_t o = ((size_t)(s1.foff + ia) * nao + s2.foff + ib) * nq + iq;
      Ic[2 * o] = accr[ia * NCB + ib];
      Ic[2 * o + 1] = acci[ia * NCB + ib];
    }
  if (!pr.diag) {
    const int n0 = pp.kn[0], n1 = pp.kn[1], n2 = pp.kn[2];
    const int i0 = c / (n1 * n2), i1 = (c / n2) % n1, i2 = c % n2;
    const int cneg = (((n0 - i0) % n0) * n1 + (n1 - i1) % n1) * n2 + (n2 - i2) % n2;
    // e^{+i k_cls.L_c} = e^{2 pi i sum_d j_d i_d / n_d}, reduced exactly in integers
    const int nt = n0 * n1 * n2;
    const int num = ((pp.kcls[0] * i0 % n0) * n1 * n2 + (pp.kcls[1] * i1 % n1) * n0 * n2 +
                     (pp.kcls[2] * i2 % n2) * n0 * n1) % nt;
    double sp, cp;
    sincospi(2.0 * num / nt, &sp, &cp);
    double *In = pp.B + 2 * ((size_t)cneg * nao * nao * nq);
#pragma unroll
    for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
      for (int ib = 0; ib < NCB; ++ib) {
        const size_t o = ((size_t)(s2.foff + ib) * nao + s1.foff + ia) * nq + iq;
        const double re = accr[ia * NCB + ib], im = acci[ia * NCB + ib];
        In[2 * o] = cp * re - sp * im;
        In[2 * o + 1] = cp * im + sp * re;
      }
  }
  return cnt;
}

// grid: x = (pair, class), y = 64-wide blocks of q
__global__ __launch_bounds__(64) void pairft_binned_kernel(const PairFTParams pp) {
  const int ip = (int)(blockIdx.x / pp.nk), c = (int)(blockIdx.x % pp.nk);
  const int iq = blockIdx.y * 64 + threadIdx.x;
  long long cnt = 0;
  if (iq < pp.nq) {
    const Pair pr = pp.pairs[ip];
    const int key = pp.ao[pr.sa].l * 3 + pp.ao[pr.sb].l;
    switch (key) {  // pairs are oriented with l(sa) >= l(sb)
      case 0: cnt = pairft_binned_one<0, 0>(pp, ip, c, iq); break;
      case 3: cnt = pairft_binned_one<1, 0>(pp, ip, c, iq); break;
      case 4: cnt = pairft_binned_one<1, 1>(pp, ip, c, iq); break;
      case 6: cnt = pairft_binned_one<2, 0>(pp, ip, c, iq); break;
      case 7: cnt = pairft_binned_one<2, 1>(pp, ip, c, iq); break;
      case 8: cnt = pairft_binned_one<2, 2>(pp, ip, c, iq); break;
      default: break;
    }
  }
  // wave sum of the evaluation counts, one integer atomic per wave
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (threadIdx.x == 0 && cnt) atomicAdd(reinterpret_cast<unsigned long long *>(pp.nterm), (unsigned long long)cnt);
}

hipError_t launch_pairft_binned(const PairFTParams &pp, hipStream_t stream) {
  if (pp.nq == 0 || pp.npair == 0) return hipSuccess;
  const int64_t nx = (int64_t)pp.npair * pp.nk;
  const int64_t ny = (pp.nq + 63) / 64;
  if (nx > 0x7fffffff || ny > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(pairft_binned_kernel, dim3((unsigned)nx, (unsigned)ny), dim3(64), 0, stream, pp);
  return hipGetLastError();
}

// amax[q] = max_P |A[P][q]| over the aux functions, one thread per q.
__global__ void amax_kernel(const double *__restrict__ A, int64_t lda, int naux, int nq, double *__restrict__ amax) {
  const int iq = blockIdx.x * blockDim.x + threadIdx.x;
  if (iq >= nq) return;
  double m = 0.0;
  for (int P = 0; P < naux; ++P) {
    const size_t o = (size_t)P * lda + iq;
    m = fmax(m, fabs(A[2 * o]) + fabs(A[2 * o + 1]));
  }
  amax[iq] = m;
}

hipError_t launch_amax(const double *A, int64_t lda, int naux, int nq, double *amax, hipStream_t stream) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(amax_kernel, dim3((nq + 255) / 256), dim3(256), 0, stream, A, lda, naux, nq, amax);
  return hipGetLastError();
}

// B[kpi][mn][q] = sum_c phase[kpi][c] I[c][mn][q], phase = e^{+i k2.L_c}; one
// thread per (mn, q) element.
__global__ void kphase_kernel(const double *__restrict__ I, const double *__restrict__ phase, double *__restrict__ B,
                              int nk, int nkpi, int nq, int64_t nmn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = (int64_t)nq * nmn;
  if (gid >= ne) return;
  for (int k = 0; k < nkpi; ++k) {
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nk; ++c) {
      const double ir = I[2 * ((int64_t)c * ne + gid)], ii = I[2 * ((int64_t)c * ne + gid) + 1];
      const double pr = phase[2 * (k * nk + c)], pi = phase[2 * (k * nk + c) + 1];
      sr += pr * ir - pi * ii;
      si += pr * ii + pi * ir;
    }
    B[2 * ((int64_t)k * ne + gid)] = sr;
    B[2 * ((int64_t)k * ne + gid) + 1] = si;
  }
}

hipError_t launch_kphase(const double *I, const double *phase, double *B, int nk, int nkpi, int nq, int64_t nmn,
                         hipStream_t stream) {
  const int64_t ne = (int64_t)nq * nmn;
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(kphase_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, stream, I, phase, B, nk, nkpi,
                     nq, nmn);
  return hipGetLastError();
}

// ---- G-space contraction on the matrix cores ---------------------------------
// out[kp][m][n] += sum_q A[m][q] B[kpi][n][q], complex, as real products on
// 16x16 MFMA blocks: C_re += A_re B_re - A_im B_im, C_im += A_re B_im + A_im B_re.
//   mode 0: FP64 operands, v_mfma_f64_16x16x4 (FP64 accumulation)
//   mode 1: FP32 operands (rounded from FP64), v_mfma_f32_16x16x4
//   mode 2: each FP32 operand split x = hi + lo into two BF16 numbers;
//           a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b on v_mfma_f32_16x16x16_bf16
// In modes 1 and 2 the matrix cores accumulate 16 q at a time in FP32; each
// 16-q partial is then added to FP64 registers, and the first nq_hi columns
// (the smallest |q|, whose kernel weights 1/q^2 dominate) are taken in FP64
// on the vector ALUs.
// Workgroup tile 64 x 64 (4 waves, 32 x 32 each = 2 x 2 MFMA blocks).
// Operand fragments (li = lane % 16, lg = lane / 16):
//   16x16x4 (f64, f32): A[li][lg], B[lg][li]
//   16x16x16 bf16:      A[li][4 lg + j], B[4 lg + j][li], j = 0..3 packed
// Result fragments, register v of a lane:
//   f64: D[lg + 4 v][li]       f32: D[4 lg + v][li]
typedef double lr_d4 __attribute__((ext_vector_type(4)));
typedef float lr_f4 __attribute__((ext_vector_type(4)));
typedef short lr_s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short lr_f2bf(float x) {  // round to nearest even
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float lr_bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <int MODE>
__global__ __launch_bounds__(256) void lr_gemm_mfma_kernel(const LRGemmParams gp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kpi = blockIdx.z;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const double *Bk = gp.B + 2 * (size_t)kpi * gp.nq * gp.nmn;
  const int li = lane & 15, lg = lane >> 4;

  auto loadA = [&](int m, int k, double &re, double &im) {
    if (m < gp.naux && k < gp.nq) {
      const size_t o = (size_t)m * gp.lda + k;
      re = gp.A[2 * o];
      im = gp.A[2 * o + 1];
    } else {
      re = im = 0.0;
    }
  };
  auto loadB = [&](int k, int n, double &re, double &im) {
    if (n < gp.nmn && k < gp.nq) {
      const size_t o = (size_t)n * gp.nq + k;
      re = Bk[2 * o];
      im = Bk[2 * o + 1];
    } else {
      re = im = 0.0;
    }
  };

  // FP64 results in the f32 fragment order: element v <-> row 4 lg + v
  double hre[2][2][4], him[2][2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) hre[r][c][v] = him[r][c][v] = 0.0;

  if constexpr (MODE == 0) {
    lr_d4 cre[2][2], cim[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) cre[r][c][v] = cim[r][c][v] = 0.0;
    for (int k0 = 0; k0 < gp.nq; k0 += 4) {
      const int k = k0 + lg;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) loadA(m0 + r * 16 + li, k, ar[r], ai[r]);
#pragma unroll
      for (int c = 0; c < 2; ++c) loadB(k, n0 + c * 16 + li, br[c], bi[c]);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[r], br[c], cre[r][c], 0, 0, 0);
          cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[r], bi[c], cre[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[r], bi[c], cim[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[r], br[c], cim[r][c], 0, 0, 0);
        }
    }
    // f64 fragment (row lg + 4 v) -> output
    const size_t kp = gp.kp_of[kpi];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + r * 16 + lg + 4 * v, n = n0 + c * 16 + li;
          if (m < gp.naux && n < gp.nmn) {
            const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
            gp.out[2 * o] += cre[r][c][v];
            gp.out[2 * o + 1] += cim[r][c][v];
          }
        }
    return;
  } else {
    // innermost q shell in FP64 on the vector ALUs
    const int khi = gp.nq_hi < gp.nq ? gp.nq_hi : gp.nq;
    for (int k = 0; k < khi; ++k) {
      double br[2], bi[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) loadB(k, n0 + c * 16 + li, br[c], bi[c]);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double ar, ai;
          loadA(m0 + r * 16 + 4 * lg + v, k, ar, ai);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            hre[r][c][v] += ar * br[c] - ai * bi[c];
            him[r][c][v] += ar * bi[c] + ai * br[c];
          }
        }
    }
    for (int k0 = khi; k0 < gp.nq; k0 += 16) {
      lr_f4 cre[2][2], cim[2][2];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) cre[r][c][v] = cim[r][c][v] = 0.f;
      if constexpr (MODE == 1) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int k = k0 + ks * 4 + lg;
          double ar[2], ai[2], br[2], bi[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) loadA(m0 + r * 16 + li, k, ar[r], ai[r]);
#pragma unroll
          for (int c = 0; c < 2; ++c) loadB(k, n0 + c * 16 + li, br[c], bi[c]);
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const float far = (float)ar[r], fai = (float)ai[r], fbr = (float)br[c], fbi = (float)bi[c];
              cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(far, fbr, cre[r][c], 0, 0, 0);
              cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-fai, fbi, cre[r][c], 0, 0, 0);
              cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(far, fbi, cim[r][c], 0, 0, 0);
              cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fai, fbr, cim[r][c], 0, 0, 0);
            }
        }
      } else {
        lr_s4 arh[2], arl[2], aih[2], ail[2], anh[2], anl[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            double re, im;
            loadA(m0 + r * 16 + li, k0 + 4 * lg + j, re, im);
            const float fr = (float)re, fi = (float)im;
            const unsigned short hr = lr_f2bf(fr), hi = lr_f2bf(fi);
            const unsigned short lr_ = lr_f2bf(fr - lr_bf2f(hr)), li_ = lr_f2bf(fi - lr_bf2f(hi));
            arh[r][j] = (short)hr;
            arl[r][j] = (short)lr_;
            aih[r][j] = (short)hi;
            ail[r][j] = (short)li_;
            anh[r][j] = (short)(hi ^ 0x8000u);  // -a_im
            anl[r][j] = (short)(li_ ^ 0x8000u);
          }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            double re, im;
            loadB(k0 + 4 * lg + j, n0 + c * 16 + li, re, im);
            const float fr = (float)re, fi = (float)im;
            const unsigned short hr = lr_f2bf(fr), hi = lr_f2bf(fi);
            brh[c][j] = (short)hr;
            brl[c][j] = (short)lr_f2bf(fr - lr_bf2f(hr));
            bih[c][j] = (short)hi;
            bil[c][j] = (short)lr_f2bf(fi - lr_bf2f(hi));
          }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            lr_f4 x = cre[r][c], y = cim[r][c];
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh[r], brh[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh[r], brl[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arl[r], brh[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(anh[r], bih[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(anh[r], bil[c], x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(anl[r], bih[c], x, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh[r], bih[c], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh[r], bil[c], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arl[r], bih[c], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aih[r], brh[c], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aih[r], brl[c], y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ail[r], brh[c], y, 0, 0, 0);
            cre[r][c] = x;
            cim[r][c] = y;
          }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            hre[r][c][v] += (double)cre[r][c][v];
            him[r][c][v] += (double)cim[r][c][v];
          }
    }
    const size_t kp = gp.kp_of[kpi];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + r * 16 + 4 * lg + v, n = n0 + c * 16 + li;
          if (m < gp.naux && n < gp.nmn) {
            const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
            gp.out[2 * o] += hre[r][c][v];
            gp.out[2 * o + 1] += him[r][c][v];
          }
        }
  }
}

hipError_t launch_lr_gemm_mfma(int mode, const LRGemmParams &gp, int nkpi, hipStream_t stream) {
  dim3 grid((gp.nmn + 63) / 64, (gp.naux + 63) / 64, nkpi);
  if (mode == 0) hipLaunchKernelGGL(lr_gemm_mfma_kernel<0>, grid, dim3(256), 0, stream, gp);
  else if (mode == 1) hipLaunchKernelGGL(lr_gemm_mfma_kernel<1>, grid, dim3(256), 0, stream, gp);
  else hipLaunchKernelGGL(lr_gemm_mfma_kernel<2>, grid, dim3(256), 0, stream, gp);
  return hipGetLastError();
}

}  // namespace rsgdf
