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
  const double w = ap.undamped ? ap.wfac / q2 : ap.wfac * exp(-q2 / (4.0 * ap.omega * ap.omega)) / q2;
  // e^{+i q.C}
  const double ph = qx * sh.x + qy * sh.y + qz * sh.z;
  const double cph = cos(ph), sph = sin(ph);
  double accr[NC], acci[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) accr[i] = acci[i] = 0.0;
  for (int k = 0; k < sh.nprim; ++k) {
    const double g = ap.ax_exp[sh.pptr + k], c = ap.ax_coef[sh.pptr + k];
    if ((ap.amode == 1 && g < ap.acut) || (ap.amode == 2 && g >= ap.acut)) continue;
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
// q values per lane: the image-dependent work of a term (Gaussian factor,
// bound, pair centre, E coefficients) is the same for every q, so the lanes of
// the lighter classes take several q each and do it once for all of them (s-s
// eight, p-s four, up to l_a + l_b = 3 two; the d-d accumulators leave no
// registers for more).  Measured on the 8-atom 3x3x3 workload: s-s 4 -> 8 and
// p-s 2 -> 4 took the long-range phase from 5.39 to 5.10 s; p-s 6 or
// l_a + l_b = 2 at four were slower.
__host__ __device__ constexpr int pairft_qpl(int la, int lb) {
  return la + lb == 0 ? 8 : (la + lb == 1 ? 4 : (la + lb <= 3 ? 2 : 1));
}

template <int LA, int LB>
__device__ long long pairft_binned_one(const PairFTParams &pp, int ip, int c, int iq0) {
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  constexpr int LT = LA + LB;
  constexpr int QP = pairft_qpl(LA, LB);
  const Pair pr = pp.pairs[ip];
  const Shell s1 = pp.ao[pr.sa];
  const Shell s2 = pp.ao[pr.sb];
  // lane q values iq0 + 64 s, s < QP; idle slots of the last block follow a
  // valid q and write nothing
  bool live[QP];
  double qx[QP], qy[QP], qz[QP], q2[QP];
  // The skip tests use the wave's extreme values (largest amax and |q|,
  // smallest q^2), so they bound every term of every lane and every lane takes
  // the same branch.
  double am = 0.0, q2w = 1e300, qnw = 0.0;
#pragma unroll
  for (int s = 0; s < QP; ++s) {
    const int iq = iq0 + 64 * s;
    live[s] = iq < pp.nq;
    const int iqc = live[s] ? iq : pp.nq - 1;
    qx[s] = pp.q[3 * iqc];
    qy[s] = pp.q[3 * iqc + 1];
    qz[s] = pp.q[3 * iqc + 2];
    q2[s] = qx[s] * qx[s] + qy[s] * qy[s] + qz[s] * qz[s];
    am = fmax(am, pp.amax[iqc]);
    q2w = fmin(q2w, q2[s]);
    qnw = fmax(qnw, sqrt(q2[s]));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    am = fmax(am, __shfl_xor(am, o, 64));
    q2w = fmin(q2w, __shfl_xor(q2w, o, 64));
    qnw = fmax(qnw, __shfl_xor(qnw, o, 64));
  }
  const double cut = am > 0.0 ? pp.eps / am : 1e300;
  // (-i q_d)^t = qr[s][d][t] + i qi[s][d][t]
  double qr[QP][3][LT + 1], qi[QP][3][LT + 1];
#pragma unroll
  for (int s = 0; s < QP; ++s) {
    const double qd[3] = {qx[s], qy[s], qz[s]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double pw = 1.0;
#pragma unroll
      for (int t = 0; t <= LT; ++t) {
        const int m = t & 3;  // (-i)^t = 1, -i, -1, i
        qr[s][d][t] = (m == 0) ? pw : (m == 2 ? -pw : 0.0);
        qi[s][d][t] = (m == 1) ? -pw : (m == 3 ? pw : 0.0);
        pw *= qd[d];
      }
    }
  }
  double accr[QP][NCA * NCB], acci[QP][NCA * NCB];
#pragma unroll
  for (int s = 0; s < QP; ++s)
#pragma unroll
    for (int i = 0; i < NCA * NCB; ++i) accr[s][i] = acci[s][i] = 0.0;
  long long cnt = 0;
  int nlive = 0;
#pragma unroll
  for (int s = 0; s < QP; ++s) nlive += live[s];
  const int beg = pp.cls_off[pr.cls_off + c], end = pp.cls_off[pr.cls_off + c + 1];
  for (int ka = 0; ka < s1.nprim; ++ka)
    for (int kb = 0; kb < s2.nprim; ++kb) {
      const double ga = pp.ao_exp[s1.pptr + ka], gb = pp.ao_exp[s2.pptr + kb];
      if (pp.pmode != 0) {
        const bool dd = ga < pp.acut && gb < pp.acut;
        if ((pp.pmode == 1) == dd) continue;
      }
      const double p = ga + gb, oop = 1.0 / p, beta = ga * gb * oop;
      const double cc = pp.ao_coef[s1.pptr + ka] * pp.ao_coef[s2.pptr + kb];
      const double pre = kPi * oop * sqrt(kPi * oop);
      const double cq = 1.0 + 0.5 * qnw * oop + sqrt(0.5 * LT * oop);
      const double rstar = 0.5 * (sqrt(cq * cq + 2.0 * LT / beta) - cq);
      const double amp0 = fabs(cc) * pre * exp(-q2w * 0.25 * oop);
      double fmax = amp0 * exp(-beta * rstar * rstar);
#pragma unroll
      for (int t = 0; t < LT; ++t) fmax *= (cq + rstar);
      if (fmax < cut) continue;
      double camp[QP];
#pragma unroll
      for (int s = 0; s < QP; ++s) camp[s] = cc * pre * exp(-q2[s] * 0.25 * oop);
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
        cnt += nlive;
        // P - A = (gb/p) R, P - B = -(ga/p) R
        const double wa = gb * oop, wb = -ga * oop;
        const double Px = s1.x + wa * Rx, Py = s1.y + wa * Ry, Pz = s1.z + wa * Rz;
        // F_d[i][j] = sum_t E_d[i][j][t] (-i q_d)^t, per q value of the lane
        double Fr[QP][3][LA + 1][LB + 1], Fi[QP][3][LA + 1][LB + 1];
        {
          double E[LA + 1][LB + 1][LT + 1];
          const double Rd[3] = {Rx, Ry, Rz};
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            hermite_E<LA, LB>(wa * Rd[d], wb * Rd[d], 0.5 * oop, E);
#pragma unroll
            for (int s = 0; s < QP; ++s)
#pragma unroll
              for (int i = 0; i <= LA; ++i)
#pragma unroll
                for (int j = 0; j <= LB; ++j) {
                  double re = 0.0, im = 0.0;
#pragma unroll
                  for (int t = 0; t <= i + j; ++t) {
                    if ((t & 1) == 0) re += E[i][j][t] * qr[s][d][t];
                    else im += E[i][j][t] * qi[s][d][t];
                  }
                  Fr[s][d][i][j] = re;
                  Fi[s][d][i][j] = im;
                }
          }
        }
#pragma unroll
        for (int s = 0; s < QP; ++s) {
          double sph, cph;
          sincos(-(qx[s] * Px + qy[s] * Py + qz[s] * Pz), &sph, &cph);
          const double amp = camp[s] * er;
          const double cr = amp * cph, ci = amp * sph;
          // fold the amplitude and phase into the x factor
          double Gr[LA + 1][LB + 1], Gi[LA + 1][LB + 1];
#pragma unroll
          for (int i = 0; i <= LA; ++i)
#pragma unroll
            for (int j = 0; j <= LB; ++j) {
              Gr[i][j] = cr * Fr[s][0][i][j] - ci * Fi[s][0][i][j];
              Gi[i][j] = cr * Fi[s][0][i][j] + ci * Fr[s][0][i][j];
            }
#pragma unroll
          for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NCB; ++ib) {
              const int ax_ = cart_lx(LA, ia), ay_ = cart_ly(LA, ia), az_ = cart_lz(LA, ia);
              const int bx_ = cart_lx(LB, ib), by_ = cart_ly(LB, ib), bz_ = cart_lz(LB, ib);
              const double xr = Gr[ax_][bx_] * Fr[s][1][ay_][by_] - Gi[ax_][bx_] * Fi[s][1][ay_][by_];
              const double xi = Gr[ax_][bx_] * Fi[s][1][ay_][by_] + Gi[ax_][bx_] * Fr[s][1][ay_][by_];
              accr[s][ia * NCB + ib] += xr * Fr[s][2][az_][bz_] - xi * Fi[s][2][az_][bz_];
              acci[s][ia * NCB + ib] += xr * Fi[s][2][az_][bz_] + xi * Fr[s][2][az_][bz_];
            }
        }
      }
    }
  const int nao = pp.nao;
  const size_t nq = pp.nq;
  double *Ic = pp.B + 2 * ((size_t)c * nao * nao * nq);
  double sp = 0.0, cp = 1.0;
  int cneg = 0;
  if (!pr.diag) {
    const int n0 = pp.kn[0], n1 = pp.kn[1], n2 = pp.kn[2];
    const int i0 = c / (n1 * n2), i1 = (c / n2) % n1, i2 = c % n2;
    cneg = (((n0 - i0) % n0) * n1 + (n1 - i1) % n1) * n2 + (n2 - i2) % n2;
    // e^{+i k_cls.L_c} = e^{2 pi i sum_d j_d i_d / n_d}, reduced exactly in integers
    const int nt = n0 * n1 * n2;
    const int num = ((pp.kcls[0] * i0 % n0) * n1 * n2 + (pp.kcls[1] * i1 % n1) * n0 * n2 +
                     (pp.kcls[2] * i2 % n2) * n0 * n1) % nt;
    sincospi(2.0 * num / nt, &sp, &cp);
  }
  double *In = pp.B + 2 * ((size_t)cneg * nao * nao * nq);
#pragma unroll
  for (int s = 0; s < QP; ++s) {
    if (!live[s]) continue;
    const size_t iq = (size_t)iq0 + 64 * s;
#pragma unroll
    for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
      for (int ib = 0; ib < NCB; ++ib) {
        const size_t o = ((size_t)(s1.foff + ia) * nao + s2.foff + ib) * nq + iq;
        Ic[2 * o] = accr[s][ia * NCB + ib];
        Ic[2 * o + 1] = acci[s][ia * NCB + ib];
      }
    if (!pr.diag) {
#pragma unroll
      for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
        for (int ib = 0; ib < NCB; ++ib) {
          const size_t o = ((size_t)(s2.foff + ib) * nao + s1.foff + ia) * nq + iq;
          const double re = accr[s][ia * NCB + ib], im = acci[s][ia * NCB + ib];
          In[2 * o] = cp * re - sp * im;
          In[2 * o + 1] = cp * im + sp * re;
        }
    }
  }
  return cnt;
}

// grid: x = (pair of one angular group, class), y = blocks of 64 * pairft_qpl q;
// one kernel per (l(sa), l(sb)) so that each runs at its own register count
template <int LA, int LB>
__global__ __launch_bounds__(64) void pairft_binned_kernel(const PairFTParams pp, int pbeg) {
  const int ip = pp.plist[pbeg + (int)(blockIdx.x / pp.nk)], c = (int)(blockIdx.x % pp.nk);
  const int iq0 = blockIdx.y * (64 * pairft_qpl(LA, LB)) + threadIdx.x;
  long long cnt = pairft_binned_one<LA, LB>(pp, ip, c, iq0);
  // wave sum of the evaluation counts, one integer atomic per wave
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (threadIdx.x == 0 && cnt) atomicAdd(reinterpret_cast<unsigned long long *>(pp.nterm), (unsigned long long)cnt);
}

hipError_t launch_pairft_binned(const PairFTParams &pp, hipStream_t stream) {
  if (pp.nq == 0 || pp.npair == 0) return hipSuccess;
  typedef void (*K)(const PairFTParams, int);
  const K ks[6] = {pairft_binned_kernel<2, 2>, pairft_binned_kernel<2, 1>, pairft_binned_kernel<2, 0>,
                   pairft_binned_kernel<1, 1>, pairft_binned_kernel<1, 0>, pairft_binned_kernel<0, 0>};
  static const int la_of[6] = {2, 2, 2, 1, 1, 0}, lb_of[6] = {2, 1, 0, 1, 0, 0};
  for (int g = 0; g < 6; ++g) {
    const int64_t nx = (int64_t)(pp.pgrp[g + 1] - pp.pgrp[g]) * pp.nk;
    if (nx == 0) continue;
    if (nx > 0x7fffffff) return hipErrorInvalidConfiguration;
    const int64_t qb = 64 * pairft_qpl(la_of[g], lb_of[g]);
    const int64_t ny = (pp.nq + qb - 1) / qb;
    if (ny > 65535) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(ks[g], dim3((unsigned)nx, (unsigned)ny), dim3(64), 0, stream, pp, pp.pgrp[g]);
  }
  return hipGetLastError();
}

// amax[q] = max_P (|Re A[P][q]| + |Im A[P][q]|) over the aux functions.
__global__ __launch_bounds__(1024) void amax_kernel(const double *__restrict__ A, int64_t lda, int naux, int nq,
                                                  double *__restrict__ amax) {
  // 64 columns per workgroup; wave w takes rows w, w + 16, ... (each load
  // instruction reads 64 consecutive complex values), and the 16 partial
  // maxima meet in LDS.  A maximum does not depend on the order.
  __shared__ double part[16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int iq = blockIdx.x * 64 + lane;
  double m = 0.0;
  if (iq < nq)
    for (int P = w; P < naux; P += 16) {
      const size_t o = (size_t)P * lda + iq;
      m = fmax(m, fabs(A[2 * o]) + fabs(A[2 * o + 1]));
    }
  part[w][lane] = m;
  __syncthreads();
  if (w == 0 && iq < nq) {
#pragma unroll
    for (int j = 1; j < 16; ++j) m = fmax(m, part[j][lane]);
    amax[iq] = m;
  }
}

hipError_t launch_amax(const double *A, int64_t lda, int naux, int nq, double *amax, hipStream_t stream) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(amax_kernel, dim3((nq + 63) / 64), dim3(1024), 0, stream, A, lda, naux, nq, amax);
  return hipGetLastError();
}

// B[kpi][mn][q] = sum_c phase[c][kpi] I[c][mn][q], phase = e^{+i k2.L_c}; one
// thread per (mn, q) element.  The k-pairs of the class are taken KB at a time
// with their sums in registers, KB chosen per launch so that one pass covers
// up to 28 k-pairs and the passes are even (each pass reads I once); the
// phases are uniform over the wave (scalar loads).  The cells are taken
// KPH_CB at a time, and the next group's I loads are issued before the
// current group's multiply-adds (two register sets in turn), so a wave always
// has loads in flight; the loop body has no branch (cell indices are clamped
// into range, which keeps every load in bounds, and the values of cells past
// nk are zeroed), so the compiler cannot sink a load next to its first use.  F32: B is written as FP32
// pairs (the operand format of the FP32 contraction, half the bytes), and the
// first nq_hi columns also in FP64 into Bhi[kpi][mn][nq_hi] (the columns the
// reduced-precision forms contract in FP64).
constexpr int KPH_CB = 3;

template <int KB>
__device__ __forceinline__ void kphase_sums(const double *__restrict__ I, int64_t ne, int64_t src, bool ok,
                                            const double *__restrict__ phase, int nk, int kpad, int k0,
                                            double (&sr)[KB], double (&si)[KB]) {
#pragma unroll
  for (int kk = 0; kk < KB; ++kk) sr[kk] = si[kk] = 0.0;
  if (!ok) return;
  // group g = cells [KPH_CB g, KPH_CB (g + 1)); two register sets in turn
  auto load = [&](int g, double (&xr)[KPH_CB], double (&xi)[KPH_CB]) {
#pragma unroll
    for (int j = 0; j < KPH_CB; ++j) {
      const int64_t o = 2 * ((int64_t)min(KPH_CB * g + j, nk - 1) * ne + src);
      xr[j] = I[o];
      xi[j] = I[o + 1];
    }
  };
  auto madd = [&](int g, const double (&xr)[KPH_CB], const double (&xi)[KPH_CB]) {
#pragma unroll
    for (int j = 0; j < KPH_CB; ++j) {
      const int c = KPH_CB * g + j;
      const double vr = c < nk ? xr[j] : 0.0, vi = c < nk ? xi[j] : 0.0;
      // the pass's KB phases of cell c are contiguous (zero past nkpi)
      const double *ph = phase + 2 * ((int64_t)min(c, nk - 1) * kpad + k0);
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const double pr = ph[2 * kk], pi = ph[2 * kk + 1];
        // two fused multiply-adds per real sum (the written form compiles to
        // a multiply, a fused multiply-add and an add)
        sr[kk] = fma(pr, vr, sr[kk]);
        sr[kk] = fma(-pi, vi, sr[kk]);
        si[kk] = fma(pr, vi, si[kk]);
        si[kk] = fma(pi, vr, si[kk]);
      }
    }
  };
  const int ng = (nk + KPH_CB - 1) / KPH_CB;
  double ar[KPH_CB], ai[KPH_CB], br[KPH_CB], bi[KPH_CB];
  load(0, ar, ai);
  int g = 0;
  for (; g + 1 < ng; g += 2) {
    load(g + 1, br, bi);
    madd(g, ar, ai);
    load(g + 2, ar, ai);  // past the last group: clamped, in bounds, unused
    madd(g + 1, br, bi);
  }
  if (g < ng) madd(g, ar, ai);
}

template <bool F32, int KB>
__global__ __launch_bounds__(256) void kphase_kernel(const double *__restrict__ I, const double *__restrict__ phase,
                                                     void *__restrict__ Bout, double *__restrict__ Bhi, int nq_hi,
                                                     int nk, int nkpi, int nq, int64_t nmn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = (int64_t)nq * nmn;
  if (gid >= ne) return;
  const int q = (int)(gid % nq);
  const int64_t mn = gid / nq;
  for (int k0 = 0; k0 < nkpi; k0 += KB) {
    double sr[KB], si[KB];
    kphase_sums<KB>(I, ne, gid, true, phase, nk, kphase_kpad(nkpi), k0, sr, si);
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
      if (k0 + kk < nkpi) {
        const int64_t o = (int64_t)(k0 + kk) * ne + gid;
        if constexpr (F32) {
          float *B = static_cast<float *>(Bout);
          B[2 * o] = (float)sr[kk];
          B[2 * o + 1] = (float)si[kk];
          if (Bhi && q < nq_hi) {
            const int64_t oh = ((int64_t)(k0 + kk) * nmn + mn) * nq_hi + q;
            Bhi[2 * oh] = sr[kk];
            Bhi[2 * oh + 1] = si[kk];
          }
        } else {
          double *B = static_cast<double *>(Bout);
          B[2 * o] = sr[kk];
          B[2 * o + 1] = si[kk];
        }
      }
  }
}

// calls launch(std::integral_constant<int, KB>) for KB = kb, 1 <= kb <= KBT:
// one kernel instance per pass width
template <int KBT, class F>
void kph_dispatch(int kb, F &&launch) {
  if (kb == KBT) launch(std::integral_constant<int, KBT>{});
  else if constexpr (KBT > 1) kph_dispatch<KBT - 1>(kb, launch);
}

hipError_t launch_kphase(const double *I, const double *phase, void *B, bool f32, double *Bhi, int nq_hi, int nk,
                         int nkpi, int nq, int64_t nmn, hipStream_t stream) {
  const int64_t ne = (int64_t)nq * nmn;
  if (ne == 0 || nkpi == 0) return hipSuccess;
  const dim3 grid((unsigned)((ne + 255) / 256));
  kph_dispatch<kKphKbMax>(kphase_kb(nkpi), [&](auto kbc) {
    constexpr int KB = decltype(kbc)::value;
    if (f32) hipLaunchKernelGGL((kphase_kernel<true, KB>), grid, dim3(256), 0, stream, I, phase, B, Bhi, nq_hi, nk, nkpi, nq, nmn);
    else hipLaunchKernelGGL((kphase_kernel<false, KB>), grid, dim3(256), 0, stream, I, phase, B, Bhi, nq_hi, nk, nkpi, nq, nmn);
  });
  return hipGetLastError();
}

// FP32 copy of an FP64 array (the aux operand of the reduced-precision forms)
__global__ void to_f32_kernel(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

hipError_t launch_to_f32(const double *x, float *y, int64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if ((n + 255) / 256 > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, y, n);
  return hipGetLastError();
}

// ---- G-space contraction on the matrix cores ---------------------------------
// out[kp][m][n] += sum_q A[m][q] B[kpi][n][q], complex, as real products on
// 16x16 MFMA blocks: C_re += A_re B_re - A_im B_im, C_im += A_re B_im + A_im B_re.
//   mode 0: FP64 operands, v_mfma_f64_16x16x4 (FP64 accumulation;
//           lr_gemm_f64_kernel)
//   mode 1: FP32 operands (rounded from FP64), v_mfma_f32_16x16x4
//           (lr_gemm_f32_kernel)
//   mode 2: split FP16 (lr_gemm_f16x3_kernel): each operand row scaled by a
//           power of two per 64-q group and split x = hi + lo into two FP16
//           numbers; a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b on
//           v_mfma_f32_16x16x32_f16
// In modes 1 and 2 the matrix cores accumulate in FP32 over one step (16 q)
// resp. one exponent group (64 q); each partial is then added to FP64
// registers, and the first nq_hi columns (the smallest |q|, whose kernel
// weights 1/q^2 dominate) are taken in FP64 on the vector ALUs.
// Operand fragments (li = lane % 16, lg = lane / 16):
//   16x16x4 (f64, f32): A[li][lg], B[lg][li]
//   16x16x32 f16:       A[li][8 lg + j], B[8 lg + j][li], j = 0..7 packed
// Result fragments, register v of a lane:
//   f64: D[lg + 4 v][li]       f32: D[4 lg + v][li]
typedef double lr_d4 __attribute__((ext_vector_type(4)));
typedef float lr_f4 __attribute__((ext_vector_type(4)));

// ---- FP32 contraction (mode 1) ----------------------------------------------
// Workgroup output tile 64 (aux rows) x 64 (pair columns), 4 waves; wave (wm,
// wn) = (wave / 2, wave % 2) owns rows 32 wm .. +32 and columns 32 wn .. +32
// (2 x 2 MFMA blocks).  Per step of 16 q the A and B tiles are read once,
// rounded to FP32 and staged in LDS (rows padded against bank conflicts); the
// next step's tiles are loaded into registers while the matrix cores work on
// the current one.  The FP32 block sums are promoted to FP64 registers after
// every step.  Columns q in [q_lo, nq) of the launch.
constexpr int F32_BM = 64, F32_BN = 64, F32_NT = 256, F32_BK = 16;
struct F32Tile {  // FP32 re / im planes
  float ar[F32_BM][F32_BK + 1], ai[F32_BM][F32_BK + 1], br[F32_BN][F32_BK + 1], bi[F32_BN][F32_BK + 1];
};

__global__ __launch_bounds__(F32_NT) void lr_gemm_f32_kernel(const LRGemmParams gp, int q_lo) {
  constexpr int RA = F32_BM * 4 / F32_NT, RB = F32_BN * 4 / F32_NT;  // staged rows per thread (4 threads x 4 q per row)
  __shared__ F32Tile S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int kpi = blockIdx.z;
  // Tile order: the hardware deals workgroups to the 8 XCDs in turn (workgroup
  // b to XCD b mod 8), and each XCD has its own L2.  Workgroups b, b + 8,
  // b + 16, ... are renumbered consecutively, and consecutive tile numbers
  // walk the aux rows first, so the row tiles that share one B tile (and
  // stream the same q columns of A) run together on one XCD.
  const int mt = (gp.naux + F32_BM - 1) / F32_BM, ntile = mt * ((gp.nmn + F32_BN - 1) / F32_BN);
  const int per = (ntile + 7) / 8;  // the grid holds 8 per workgroups
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntile) return;
  const int M0 = (t % mt) * F32_BM, N0 = (t / mt) * F32_BN;
  const float *Bk32 = gp.B32 + 2 * (size_t)kpi * gp.nq * gp.nmn;
  const int sr0 = tid >> 2, sq = (tid & 3) * 4;
  float ga[RA][8], gb[RB][8];  // re, im of 4 q per staged row
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + sq + j;
      const bool okk = k < gp.nq;
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int m = M0 + sr0 + r * (F32_NT / 4);
        if (okk && m < gp.naux) {
          const size_t o = (size_t)m * gp.lda + k;
          ga[r][2 * j] = gp.A32[2 * o];
          ga[r][2 * j + 1] = gp.A32[2 * o + 1];
        } else {
          ga[r][2 * j] = ga[r][2 * j + 1] = 0;
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int n = N0 + sr0 + r * (F32_NT / 4);
        if (okk && n < gp.nmn) {
          const size_t o = (size_t)n * gp.nq + k;
          gb[r][2 * j] = Bk32[2 * o];
          gb[r][2 * j + 1] = Bk32[2 * o + 1];
        } else {
          gb[r][2 * j] = gb[r][2 * j + 1] = 0;
        }
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int row = sr0 + r * (F32_NT / 4);
        S.ar[row][sq + j] = ga[r][2 * j];
        S.ai[row][sq + j] = ga[r][2 * j + 1];
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int row = sr0 + r * (F32_NT / 4);
        S.br[row][sq + j] = gb[r][2 * j];
        S.bi[row][sq + j] = gb[r][2 * j + 1];
      }
    }
  };

  lr_f4 cre[2][2], cim[2][2];
  double hre[2][2][4], him[2][2][4];  // FP64 sums (f32 fragment order)
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cre[r][c][v] = cim[r][c][v] = 0;
        hre[r][c][v] = him[r][c][v] = 0.0;
      }

  // the innermost q shell (first nq_hi columns) in FP64 on the vector ALUs,
  // rows in the f32 fragment order
  const int khi = gp.nq_hi < gp.nq ? gp.nq_hi : gp.nq;
  for (int k = q_lo; k < khi; ++k) {
    double br[2], bi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int n = N0 + wn * 32 + c * 16 + li;
      const size_t o = ((size_t)kpi * gp.nmn + n) * gp.nq_hi + k;
      br[c] = (n < gp.nmn) ? gp.Bhi[2 * o] : 0.0;
      bi[c] = (n < gp.nmn) ? gp.Bhi[2 * o + 1] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + 4 * lg + v;
        const size_t o = (size_t)m * gp.lda + k;
        const double ar = (m < gp.naux) ? gp.A[2 * o] : 0.0, ai = (m < gp.naux) ? gp.A[2 * o + 1] : 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          hre[r][c][v] += ar * br[c] - ai * bi[c];
          him[r][c][v] += ar * bi[c] + ai * br[c];
        }
      }
  }
  const int kstart = khi > q_lo ? khi : q_lo;
  gload(kstart);
  for (int k0 = kstart; k0 < gp.nq; k0 += F32_BK) {
    __syncthreads();  // previous step's fragments consumed
    sstore();
    __syncthreads();
    if (k0 + F32_BK < gp.nq) gload(k0 + F32_BK);  // in flight during the MFMAs
#pragma unroll
    for (int ks = 0; ks < F32_BK / 4; ++ks) {
      const int k = ks * 4 + lg;
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        ar[r] = S.ar[wm * 32 + r * 16 + li][k];
        ai[r] = S.ai[wm * 32 + r * 16 + li][k];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        br[c] = S.br[wn * 32 + c * 16 + li][k];
        bi[c] = S.bi[wn * 32 + c * 16 + li][k];
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[r], br[c], cre[r][c], 0, 0, 0);
          cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[r], bi[c], cre[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[r], bi[c], cim[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[r], br[c], cim[r][c], 0, 0, 0);
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
          cre[r][c][v] = 0.f;
          cim[r][c][v] = 0.f;
        }
  }
  // epilogue: f32 fragment row = 4 lg + v
  const size_t kp = gp.kp_of[kpi];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + 4 * lg + v;
        const int n = N0 + wn * 32 + c * 16 + li;
        if (m < gp.naux && n < gp.nmn) {
          const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
          gp.out[2 * o] += hre[r][c][v];
          gp.out[2 * o + 1] += him[r][c][v];
        }
      }
}

// ---- split-FP16 contraction (mode 2) ------------------------------------------
// Operand format.  The q range of a launch is cut into blocks of 32 q, and the
// blocks into exponent groups of kF16Grp = 2 blocks (64 q).  In a group every
// operand row (an aux function of A; a pair column of one k-pair's B) is
// scaled by 2^-e, e chosen so that the row's largest |re|, |im| in the group
// (over q >= q_excl: the columns contracted in FP64 do not count) lies in
// [2^14, 2^15) (e = 0 for a zero row), and each scaled value x' is split
// x' = hi + lo with hi = fp16(x'), lo = fp16(x' - hi): 22 significant bits,
// always inside the FP16 range.  Storage per (block, row): 256 bytes, the
// planes re_hi, re_lo, im_hi, im_lo of 32 halves, and the group's exponent e
// as an int; q past the end of the launch are zero (whole groups are stored).  The producers write this format
// from FP64 values (asplit_kernel from the aux transforms, kphase_split_kernel
// from the Bloch sums), so the contraction only copies 16-byte pieces.
//
// Contraction: a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (the dropped lo_a lo_b
// is 2^-22 of the product) on v_mfma_f32_16x16x32_f16, FP32 accumulation over
// one exponent group; after each group the FP32 sums are scaled back by
// 2^(e_m + e_n) (exact) and added to FP64 registers.  The first nq_hi q of the class are
// taken in FP64 on the vector ALUs as in the FP32 form.  Workgroup tile 64 x
// 64, 4 waves of 2 x 2 blocks of 16 x 16.  Fragments (li = lane % 16, lg =
// lane / 16): A[li][8 lg + j], B[8 lg + j][li], j < 8; result D[4 lg + v][li]
// (the lane layout was checked on the GPU with a probe).
typedef _Float16 lr_h8 __attribute__((ext_vector_type(8)));
constexpr int F16_BM = 64, F16_BN = 64, F16_NT = 256;
constexpr int F16_LD = kF16Blk + 8;  // LDS row stride in halves: 80 bytes, 16-byte aligned fragments
static_assert(kF16Blk == 32, "one v_mfma_f32_16x16x32_f16 per block and plane pair");

// exponent of a group row: the 64 q of a row's exponent group are the 64
// lanes of one wavefront (a 6-step butterfly)
static_assert(kF16Blk * kF16Grp == 64, "one wavefront per exponent group");
__device__ inline int f16_group_exp(double mx) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s, 64));
  return mx > 0.0 ? ilogb(mx) - 14 : 0;
}

// the scaled value is rounded to FP32 first (24 bits, of which hi + lo keep
// 22): the hardware converts FP32 to FP16 in one instruction, FP64 to FP16 only
// through a long integer sequence
__device__ inline void f16_split_store(double re, double im, int e, uint16_t *row, int l) {
  _Float16 *h = reinterpret_cast<_Float16 *>(row);
  const float xr = (float)ldexp(re, -e), xi = (float)ldexp(im, -e);
  const _Float16 hr = (_Float16)xr, hm = (_Float16)xi;
  h[l] = hr;
  h[32 + l] = (_Float16)(xr - (float)hr);
  h[64 + l] = hm;
  h[96 + l] = (_Float16)(xi - (float)hm);
}

// A[P][q] (FP64 complex, row stride lda) -> Xa[b][P][4][32], Ea[b][P]; one
// thread per (P, q) of the padded grid, 32-lane blocks along q (nb is a whole
// number of groups, so a wavefront holds the two blocks of one row's group)
__global__ __launch_bounds__(256) void asplit_kernel(const double *__restrict__ A, int64_t lda, int naux, int nq,
                                                     int q_excl, int nb, uint16_t *__restrict__ Xa,
                                                     int32_t *__restrict__ Ea) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = (int)(gid & 31);
  const int64_t t = gid >> 5;
  const int b = (int)(t % nb);
  const int64_t P = t / nb;
  const int q = b * kF16Blk + l;
  double re = 0.0, im = 0.0;
  if (P < naux && q < nq) {
    const int64_t o = P * lda + q;
    re = A[2 * o];
    im = A[2 * o + 1];
  }
  const int e = f16_group_exp(q >= q_excl ? fmax(fabs(re), fabs(im)) : 0.0);
  if (P < naux) {
    f16_split_store(re, im, e, Xa + ((int64_t)b * naux + P) * 4 * kF16Blk, l);
    if (l == 0) Ea[(int64_t)b * naux + P] = e;
  }
}

hipError_t launch_asplit(const double *A, int64_t lda, int naux, int nq, int q_excl, uint16_t *Xa, int32_t *Ea,
                         hipStream_t stream) {
  if (nq <= 0 || naux <= 0) return hipSuccess;
  const int nb = f16_nblk(nq);
  const int64_t n = (int64_t)naux * nb * kF16Blk;
  hipLaunchKernelGGL(asplit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, A, lda, naux, nq,
                     q_excl, nb, Xa, Ea);
  return hipGetLastError();
}

// kphase_kernel's Bloch sums written in the split format: Xb[kpi][b][mn][4][32],
// Eb[kpi][b][mn], and the first nq_hi columns in FP64 into Bhi[kpi][mn][nq_hi]
// (those columns do not enter the exponents).  One thread per (mn, q) of the
// padded grid, 32-lane blocks along q, a wavefront per row's exponent group.
template <int KB>
__global__ __launch_bounds__(256) void kphase_split_kernel(const double *__restrict__ I,
                                                           const double *__restrict__ phase,
                                                           uint16_t *__restrict__ Xb, int32_t *__restrict__ Eb,
                                                           double *__restrict__ Bhi, int nq_hi, int nk, int nkpi,
                                                           int nq, int nb, int64_t nmn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = (int)(gid & 31);
  const int64_t t = gid >> 5;
  const int b = (int)(t % nb);
  const int64_t mn = t / nb;
  const int q = b * kF16Blk + l;
  const bool row = mn < nmn, ok = row && q < nq;
  const int64_t ne = (int64_t)nq * nmn, src = mn * nq + q;
  const int kpad = kphase_kpad(nkpi);
  for (int k0 = 0; k0 < nkpi; k0 += KB) {
    double sr[KB], si[KB];
    kphase_sums<KB>(I, ne, src, ok, phase, nk, kpad, k0, sr, si);
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
      if (k0 + kk < nkpi) {  // uniform over the wave
        const int k = k0 + kk;
        const int e = f16_group_exp(q >= nq_hi ? fmax(fabs(sr[kk]), fabs(si[kk])) : 0.0);
        if (row) {
          const int64_t rb = ((int64_t)k * nb + b) * nmn + mn;
          f16_split_store(sr[kk], si[kk], e, Xb + rb * 4 * kF16Blk, l);
          if (l == 0) Eb[rb] = e;
        }
        if (Bhi && ok && q < nq_hi) {
          const int64_t oh = ((int64_t)k * nmn + mn) * nq_hi + q;
          Bhi[2 * oh] = sr[kk];
          Bhi[2 * oh + 1] = si[kk];
        }
      }
  }
}

hipError_t launch_kphase_split(const double *I, const double *phase, uint16_t *Xb, int32_t *Eb, double *Bhi,
                               int nq_hi, int nk, int nkpi, int nq, int64_t nmn, hipStream_t stream) {
  if (nq <= 0 || nmn <= 0 || nkpi <= 0) return hipSuccess;
  const int nb = f16_nblk(nq);
  const int64_t n = nmn * nb * kF16Blk;
  const dim3 grid((unsigned)((n + 255) / 256));
  kph_dispatch<kKphKbMax>(kphase_kb(nkpi), [&](auto kbc) {
    constexpr int KB = decltype(kbc)::value;
    hipLaunchKernelGGL((kphase_split_kernel<KB>), grid, dim3(256), 0, stream, I, phase, Xb, Eb, Bhi, nq_hi, nk, nkpi, nq,
                       nb, nmn);
  });
  return hipGetLastError();
}

// LDS stage of one block: the A and B tiles (64 rows x 256 bytes each, row r's
// 16-byte chunk c = 4 plane + part stored at chunk position c ^ (r % 16), so
// that the 16 rows a fragment read touches fall in distinct banks), then the
// 64 + 64 block exponents.  The tiles are filled by global_load_lds_dwordx4:
// one instruction writes 1 KB of LDS, lane l's 16 bytes at offset 16 l, so the
// lane that fills slot u fetches the global chunk that belongs there.
constexpr int F16_TILE = F16_BM * 4 * kF16Blk * 2;      // 16384 bytes
constexpr int F16_STAGE = 2 * F16_TILE + 2 * 64 * 4;    // + exponents
#ifndef RSGDF_F16_STAGES
#define RSGDF_F16_STAGES 2  // 2: two workgroups per CU (66 KB of LDS each); 3: one, and
                            // slower (measured on the 8-atom 3x3x3 workload, 1.90 s vs 2.65 s)
#endif
constexpr int F16_NS = RSGDF_F16_STAGES;                // stages in flight
static_assert(F16_NS == 2 || F16_NS == 3, "the waits below cover two or three stages");

// s_waitcnt with vmcnt <= n (expcnt and lgkmcnt not waited on), gfx9 encoding
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// s_waitcnt lgkmcnt(0) alone (this wave's LDS reads returned)
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }
// workgroup barrier without a memory fence; the empty asm statements keep the
// compiler from moving memory accesses across it (the waits are explicit)
__device__ __forceinline__ void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__global__ __launch_bounds__(F16_NT) void lr_gemm_f16x3_kernel(const LRGemmParams gp, int q_lo) {
  __shared__ __attribute__((aligned(16))) unsigned char S[F16_NS][F16_STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int kpi = blockIdx.z;
  // XCD-aware tile order as in lr_gemm_f32_kernel
  const int mt = (gp.naux + F16_BM - 1) / F16_BM, ntile = mt * ((gp.nmn + F16_BN - 1) / F16_BN);
  const int per = (ntile + 7) / 8;
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntile) return;
  const int M0 = (t % mt) * F16_BM, N0 = (t / mt) * F16_BN;
  const unsigned char *Xa8 = reinterpret_cast<const unsigned char *>(gp.Xa);
  const unsigned char *Xb8 =
      reinterpret_cast<const unsigned char *>(gp.Xb) + (size_t)kpi * gp.nb * gp.nmn * 4 * kF16Blk * 2;
  const int32_t *Ebk = gp.Eb + (size_t)kpi * gp.nb * gp.nmn;
  // slots u = (4 j + wave) 64 + lane, j < 4, of each tile: row u / 16, chunk
  // (u % 16) ^ (row % 16); rows past the end are clamped to the last row
  // (their results are not stored)
  int64_t ga_off[4], gb_off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int u = (4 * j + wave) * 64 + lane, r = u >> 4, c = (u & 15) ^ (r & 15);
    ga_off[j] = (int64_t)min(M0 + r, gp.naux - 1) * 256 + 16 * c;
    gb_off[j] = (int64_t)min(N0 + r, gp.nmn - 1) * 256 + 16 * c;
  }
  const int e_row = (wave == 0) ? min(M0 + lane, gp.naux - 1) : min(N0 + lane, gp.nmn - 1);
  // loads of block b into stage st: 8 per wave, 9 for waves 0 and 1 (exponents)
  auto issue = [&](int b, int st) {
    const unsigned char *xa = Xa8 + (size_t)b * gp.naux * 256, *xb = Xb8 + (size_t)b * gp.nmn * 256;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      __builtin_amdgcn_global_load_lds(xa + ga_off[j], &S[st][(4 * j + wave) * 1024], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(xb + gb_off[j], &S[st][F16_TILE + (4 * j + wave) * 1024], 16, 0, 0);
    }
    if (wave == 0) __builtin_amdgcn_global_load_lds(gp.Ea + (size_t)b * gp.naux + e_row, &S[st][2 * F16_TILE], 4, 0, 0);
    if (wave == 1)
      __builtin_amdgcn_global_load_lds(Ebk + (size_t)b * gp.nmn + e_row, &S[st][2 * F16_TILE + 256], 4, 0, 0);
  };

  lr_f4 cre[2][2], cim[2][2];
  double hre[2][2][4], him[2][2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cre[r][c][v] = cim[r][c][v] = 0.f;
        hre[r][c][v] = him[r][c][v] = 0.0;
      }
  // blocks after the FP64 columns (nq_hi is a multiple of the block; when the
  // launch is shorter than nq_hi there are none)
  const int khi = gp.nq_hi < gp.nq ? gp.nq_hi : gp.nq;
  const int b0 = (max(khi, q_lo) + kF16Blk - 1) / kF16Blk;
  // the first stages' loads in flight during the FP64 columns
#pragma unroll
  for (int i = 0; i < F16_NS - 1; ++i)
    if (b0 + i < gp.nb) issue(b0 + i, i);
  // the innermost q in FP64 on the vector ALUs (rows in the f32 fragment order)
  for (int k = q_lo; k < khi; ++k) {
    double br[2], bi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int n = N0 + wn * 32 + c * 16 + li;
      const size_t o = ((size_t)kpi * gp.nmn + n) * gp.nq_hi + k;
      br[c] = (n < gp.nmn) ? gp.Bhi[2 * o] : 0.0;
      bi[c] = (n < gp.nmn) ? gp.Bhi[2 * o + 1] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + 4 * lg + v;
        const size_t o = (size_t)m * gp.lda + k;
        const double ar = (m < gp.naux) ? gp.A[2 * o] : 0.0, ai = (m < gp.naux) ? gp.A[2 * o + 1] : 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          hre[r][c][v] += ar * br[c] - ai * bi[c];
          him[r][c][v] += ar * bi[c] + ai * br[c];
        }
      }
  }
  const int lpb = (wave < 2) ? 9 : 8;  // loads per block of this wave
  int st = 0;
  for (int b = b0; b < gp.nb; ++b) {
    // stage of block b + NS - 1 was consumed in the previous iteration (barrier below)
    const bool more = b + F16_NS - 1 < gp.nb;
    if (more) issue(b + F16_NS - 1, (st + F16_NS - 1) % F16_NS);
    // block b complete for this wave: the loads issued after it may stay outstanding
    const int after = min(F16_NS - 1, gp.nb - 1 - b);
    if (after == 2) {
      if (lpb == 9) wait_vmcnt<18>();
      else wait_vmcnt<16>();
    } else if (after == 1) {
      if (lpb == 9) wait_vmcnt<9>();
      else wait_vmcnt<8>();
    } else {
      wait_vmcnt<0>();
    }
    // every wave's part of block b in LDS (a bare barrier: a fence here would
    // also wait for the later blocks' loads)
    bare_barrier();
    const unsigned char *SA = S[st], *SB = S[st] + F16_TILE;
    const int *SE = reinterpret_cast<const int *>(S[st] + 2 * F16_TILE);
    lr_h8 a[2][4], an[2][2], bf[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int row = wm * 32 + r * 16 + li;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        a[r][pl] = *reinterpret_cast<const lr_h8 *>(SA + row * 256 + (((4 * pl + lg) ^ li) << 4));
      an[r][0] = -a[r][2];
      an[r][1] = -a[r][3];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int row = wn * 32 + c * 16 + li;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        bf[c][pl] = *reinterpret_cast<const lr_h8 *>(SB + row * 256 + (((4 * pl + lg) ^ li) << 4));
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        lr_f4 x = cre[r][c], y = cim[r][c];
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][0], bf[c][0], x, 0, 0, 0);  // re_a re_b
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][0], bf[c][1], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][1], bf[c][0], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(an[r][0], bf[c][2], x, 0, 0, 0);  // - im_a im_b
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(an[r][0], bf[c][3], x, 0, 0, 0);
        x = __builtin_amdgcn_mfma_f32_16x16x32_f16(an[r][1], bf[c][2], x, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][0], bf[c][2], y, 0, 0, 0);  // re_a im_b
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][0], bf[c][3], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][1], bf[c][2], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][2], bf[c][0], y, 0, 0, 0);  // im_a re_b
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][2], bf[c][1], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r][3], bf[c][0], y, 0, 0, 0);
        cre[r][c] = x;
        cim[r][c] = y;
      }
    // at the end of an exponent group: scale back by 2^(e_m + e_n) and promote
    // to FP64 (the blocks of a group carry the same exponents)
    const bool promote = (b % kF16Grp == kF16Grp - 1) || b + 1 == gp.nb;
    int ea[2][4], eb[2];
    if (promote) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) ea[r][v] = SE[wm * 32 + r * 16 + 4 * lg + v];
#pragma unroll
      for (int c = 0; c < 2; ++c) eb[c] = SE[64 + wn * 32 + c * 16 + li];
    }
    wait_lgkm0();    // this wave's reads of stage st returned
    bare_barrier();  // every wave's: the next iteration refills it
    if (promote) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double sc = ldexp(1.0, ea[r][v] + eb[c]);
            hre[r][c][v] = fma((double)cre[r][c][v], sc, hre[r][c][v]);
            him[r][c][v] = fma((double)cim[r][c][v], sc, him[r][c][v]);
            cre[r][c][v] = 0.f;
            cim[r][c][v] = 0.f;
          }
    }
    st = (st + 1 == F16_NS) ? 0 : st + 1;
  }
  const size_t kp = gp.kp_of[kpi];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + 4 * lg + v;
        const int n = N0 + wn * 32 + c * 16 + li;
        if (m < gp.naux && n < gp.nmn) {
          const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
          gp.out[2 * o] += hre[r][c][v];
          gp.out[2 * o + 1] += him[r][c][v];
        }
      }
}

// ---- FP64 contraction (mode 0) ------------------------------------------------
// Workgroup tile 128 x 128, 8 waves; wave (wm, wn) = (wave / 2, wave % 2) owns
// rows 32 wm .. +32 and columns 64 wn .. +64 (2 x 4 blocks of 16 x 16).  A step
// is 16 q.  Its A and B tiles (128 rows x 16 complex numbers, 32 KB each) go
// from global memory straight into LDS, one complex number (16 bytes) per lane
// and load, with two stages in flight: no registers are spent on staging, and
// the loads of step s + 1 run while the matrix cores work on step s.  Row r of
// a tile keeps its q at chunk position q ^ (r % 16), so the 16 lanes of one
// fragment read (rows li, one q) fall on 16 different groups of four banks.
// Rows past the end are clamped to the last row (their results are not
// stored) and q past the end of the launch to the last q; there the A
// fragment is replaced by zero.
constexpr int F64_BM = 128, F64_BN = 128, F64_NT = 512, F64_BK = 16;
constexpr int F64_TILE = F64_BM * F64_BK * 16;  // 32768 bytes
static_assert(F64_BM * F64_BK * 16 == 4 * F64_NT * 16, "four loads per thread and tile");
typedef double lr_d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(F64_NT) void lr_gemm_f64_kernel(const LRGemmParams gp, int q_lo) {
  __shared__ __attribute__((aligned(16))) unsigned char S[2][2 * F64_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int kpi = blockIdx.z;
  // XCD-aware tile order as in lr_gemm_f32_kernel
  const int mt = (gp.naux + F64_BM - 1) / F64_BM, ntile = mt * ((gp.nmn + F64_BN - 1) / F64_BN);
  const int per = (ntile + 7) / 8;
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntile) return;
  const int M0 = (t % mt) * F64_BM, N0 = (t / mt) * F64_BN;
  const double *Bk = gp.B + 2 * (size_t)kpi * gp.nq * gp.nmn;
  // slots u = (8 j + wave) 64 + lane, j < 4, of each tile: row u / 16, q
  // offset (u % 16) ^ (row % 16)
  const double *pa[4], *pb[4];
  int qo[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int u = (8 * j + wave) * 64 + lane, r = u >> 4;
    qo[j] = (u & 15) ^ (r & 15);
    pa[j] = gp.A + 2 * (size_t)min(M0 + r, gp.naux - 1) * gp.lda;
    pb[j] = Bk + 2 * (size_t)min(N0 + r, gp.nmn - 1) * gp.nq;
  }
  // loads of the step starting at k0 into stage st: 8 per thread
  auto issue = [&](int k0, int st) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = min(k0 + qo[j], gp.nq - 1);
      __builtin_amdgcn_global_load_lds(pa[j] + 2 * q, &S[st][(8 * j + wave) * 1024], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(pb[j] + 2 * q, &S[st][F64_TILE + (8 * j + wave) * 1024], 16, 0, 0);
    }
  };

  lr_d4 cre[2][4], cim[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) cre[r][c][v] = cim[r][c][v] = 0.0;
  // 16-row blocks of this wave inside the aux range: in the last row tile the
  // blocks past the end take no products, so a SIMD there has half the work
  const int nr = min(max((gp.naux - (M0 + wm * 32) + 15) / 16, 0), 2);
  // the products of one step (16 q) for the wave's first NR row blocks
  auto step = [&](const unsigned char *SA, const unsigned char *SB, int k0, auto nrc) {
    constexpr int NR = decltype(nrc)::value;
#pragma unroll
    for (int ks = 0; ks < F64_BK / 4; ++ks) {
      const int k = 4 * ks + lg;
      const bool kin = k0 + k < gp.nq;
      lr_d2 a[NR], b[4];
      double an[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        a[r] = *reinterpret_cast<const lr_d2 *>(SA + (wm * 32 + r * 16 + li) * 256 + ((k ^ li) << 4));
        if (!kin) a[r] = lr_d2{0.0, 0.0};
        an[r] = -a[r].y;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
        b[c] = *reinterpret_cast<const lr_d2 *>(SB + (wn * 64 + c * 16 + li) * 256 + ((k ^ li) << 4));
      // four independent rounds over the blocks, so that no product waits
      // for the one just issued into the same accumulator
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r].x, b[c].x, cre[r][c], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r].x, b[c].y, cim[r][c], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[r], b[c].y, cre[r][c], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r].y, b[c].x, cim[r][c], 0, 0, 0);
    }
  };
  const int nst = (gp.nq - q_lo + F64_BK - 1) / F64_BK;  // >= 1 (the launcher skips empty launches)
  issue(q_lo, 0);
  int st = 0;
  for (int s = 0; s < nst; ++s) {
    const int k0 = q_lo + s * F64_BK;
    // stage st ^ 1 was consumed in the previous step (barrier below)
    if (s + 1 < nst) {
      issue(k0 + F64_BK, st ^ 1);
      wait_vmcnt<8>();  // this step's loads done, the next step's in flight
    } else {
      wait_vmcnt<0>();
    }
    bare_barrier();  // every wave's part of the step in LDS
    const unsigned char *SA = S[st], *SB = S[st] + F64_TILE;
    if (nr == 2) step(SA, SB, k0, std::integral_constant<int, 2>{});
    else if (nr == 1) step(SA, SB, k0, std::integral_constant<int, 1>{});
    wait_lgkm0();    // this wave's reads of stage st returned
    bare_barrier();  // every wave's: the next step refills it
    st ^= 1;
  }
  // f64 fragment row = lg + 4 v
  const size_t kp = gp.kp_of[kpi];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + lg + 4 * v;
        const int n = N0 + wn * 64 + c * 16 + li;
        if (m < gp.naux && n < gp.nmn) {
          const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
          gp.out[2 * o] += cre[r][c][v];
          gp.out[2 * o + 1] += cim[r][c][v];
        }
      }
}

hipError_t launch_lr_gemm_tiled(int mode, const LRGemmParams &gp, int q_lo, int nkpi, hipStream_t stream) {
  if (q_lo >= gp.nq) return hipSuccess;
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  const int bm = mode == 0 ? F64_BM : mode == 1 ? F32_BM : F16_BM;
  const int bn = mode == 0 ? F64_BN : mode == 1 ? F32_BN : F16_BN;
  const int64_t ntile = (int64_t)((gp.nmn + bn - 1) / bn) * ((gp.naux + bm - 1) / bm);
  if (ntile * 8 > 0x7fffffff) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(8 * ((ntile + 7) / 8)), 1, nkpi);
  if (mode == 0) hipLaunchKernelGGL(lr_gemm_f64_kernel, grid, dim3(F64_NT), 0, stream, gp, q_lo);
  else if (mode == 1) hipLaunchKernelGGL(lr_gemm_f32_kernel, grid, dim3(F32_NT), 0, stream, gp, q_lo);
  else {
    // the split format's blocks start at q = 0 and the FP64 columns end on a block boundary
    if (q_lo != 0 || gp.nq_hi % kF16Blk != 0 || gp.nb != f16_nblk(gp.nq) || !gp.Xa || !gp.Xb ||
        !gp.Ea || !gp.Eb)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(lr_gemm_f16x3_kernel, grid, dim3(F16_NT), 0, stream, gp, q_lo);
  }
  return hipGetLastError();
}

}  // namespace rsgdf
