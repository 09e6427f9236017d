// lr.hip -- long-range (erf-attenuated) part in reciprocal space, Eqs. (M10)
// and (M11):
//   V^LR[k1,k2][P][mu nu] = sum_{q in Q(k12)} A[P][q] rho^{k2}[q][mu nu]
//   A[P][q]               = (4 pi/Omega) exp(-|q|^2/4w^2)/|q|^2 chi~_P(-q)
//   rho^{k2}_{mu nu}(q)   = sum_n exp(+i k2.n) int phi_mu(r) phi_nu(r-n) e^{-iq.r} dr
// with q = G + k12 over one folded k12 class.  Transforms are analytic: a
// Gaussian product is expanded in Hermite Gaussians (McMurchie-Davidson E
// coefficients), whose transforms are (-i q)^t times the s-type transform.
#include <hip/hip_runtime.h>

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

// ---- pair transforms ----------------------------------------------------------
// B[kpi][q][mu][nu] for the k-pairs of one class and one chunk of q vectors.
// One thread per (oriented pair, order, q, kpi); `order` 0 takes (sa, sb) with
// images +n', order 1 takes (sb, sa) with images -n'.


template <int LA, int LB>
__device__ long long pairft_one(const PairFTParams &pp, int ip, int order, int iq, int kpi) {
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  const Pair pr = pp.pairs[ip];
  const Shell s1 = pp.ao[order ? pr.sb : pr.sa];
  const Shell s2 = pp.ao[order ? pr.sa : pr.sb];
  const double sgn = order ? -1.0 : 1.0;
  const double qx = pp.q[3 * iq], qy = pp.q[3 * iq + 1], qz = pp.q[3 * iq + 2];
  const double q2 = qx * qx + qy * qy + qz * qz;
  const double kx = pp.k2[3 * kpi], ky = pp.k2[3 * kpi + 1], kz = pp.k2[3 * kpi + 2];
  double accr[NCA * NCB], acci[NCA * NCB];
#pragma unroll
  for (int i = 0; i < NCA * NCB; ++i) accr[i] = acci[i] = 0.0;
  long long cnt = 0;
  const int beg = pp.cls_off[pr.cls_off], end = pp.cls_off[pr.cls_off + pp.nk];
  for (int ii = beg; ii < end; ++ii) {
    const double *nv = pp.img + 3 * (size_t)(pr.img_off + ii);
    const double nx = sgn * nv[0], ny = sgn * nv[1], nz = sgn * nv[2];
    const double Bx = s2.x + nx, By = s2.y + ny, Bz = s2.z + nz;
    const double r2 = (s1.x - Bx) * (s1.x - Bx) + (s1.y - By) * (s1.y - By) + (s1.z - Bz) * (s1.z - Bz);
    // Bloch phase e^{+i k2.n}
    const double phk = kx * nx + ky * ny + kz * nz;
    const double ckr = cos(phk), cki = sin(phk);
    for (int ka = 0; ka < s1.nprim; ++ka)
      for (int kb = 0; kb < s2.nprim; ++kb) {
        const double ga = pp.ao_exp[s1.pptr + ka], gb = pp.ao_exp[s2.pptr + kb];
        const double p = ga + gb, oop = 1.0 / p;
        const double K = exp(-ga * gb * oop * r2) * pp.ao_coef[s1.pptr + ka] * pp.ao_coef[s2.pptr + kb] * kPi * oop *
                         sqrt(kPi * oop);
        if (fabs(K) < pp.cutoff) continue;
        ++cnt;
        const double Px = (ga * s1.x + gb * Bx) * oop, Py = (ga * s1.y + gb * By) * oop, Pz = (ga * s1.z + gb * Bz) * oop;
        double Ex[LA + 1][LB + 1][LA + LB + 1], Ey[LA + 1][LB + 1][LA + LB + 1], Ez[LA + 1][LB + 1][LA + LB + 1];
        hermite_E<LA, LB>(Px - s1.x, Px - Bx, 0.5 * oop, Ex);
        hermite_E<LA, LB>(Py - s1.y, Py - By, 0.5 * oop, Ey);
        hermite_E<LA, LB>(Pz - s1.z, Pz - Bz, 0.5 * oop, Ez);
        // K (pi/p)^{3/2} e^{-q^2/4p} e^{-i q.P} e^{+i k2.n}
        const double amp = K * exp(-q2 * 0.25 * oop);
        const double ph = -(qx * Px + qy * Py + qz * Pz);
        const double cr0 = cos(ph), ci0 = sin(ph);
        const double cr = amp * (cr0 * ckr - ci0 * cki), ci = amp * (cr0 * cki + ci0 * ckr);
        // per-dimension polynomials F_d[i][j] = sum_t E_d[i][j][t] (-i q_d)^t
        double Fr[3][LA + 1][LB + 1], Fi[3][LA + 1][LB + 1];
        const double qd[3] = {qx, qy, qz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
          for (int i = 0; i <= LA; ++i)
#pragma unroll
            for (int j = 0; j <= LB; ++j) {
              double re = 0.0, im = 0.0, pr_ = 1.0, pi_ = 0.0;
#pragma unroll
              for (int t = 0; t <= i + j; ++t) {
                const double e = (d == 0) ? Ex[i][j][t] : (d == 1 ? Ey[i][j][t] : Ez[i][j][t]);
                re += e * pr_;
                im += e * pi_;
                // multiply by (-i q_d)
                const double nr = pi_ * qd[d], ni = -pr_ * qd[d];
                pr_ = nr;
                pi_ = ni;
              }
              Fr[d][i][j] = re;
              Fi[d][i][j] = im;
            }
        }
#pragma unroll
        for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
          for (int ib = 0; ib < NCB; ++ib) {
            const int ax_ = cart_lx(LA, ia), ay_ = cart_ly(LA, ia), az_ = cart_lz(LA, ia);
            const int bx_ = cart_lx(LB, ib), by_ = cart_ly(LB, ib), bz_ = cart_lz(LB, ib);
            const double xr = Fr[0][ax_][bx_] * Fr[1][ay_][by_] - Fi[0][ax_][bx_] * Fi[1][ay_][by_];
            const double xi = Fr[0][ax_][bx_] * Fi[1][ay_][by_] + Fi[0][ax_][bx_] * Fr[1][ay_][by_];
            const double yr = xr * Fr[2][az_][bz_] - xi * Fi[2][az_][bz_];
            const double yi = xr * Fi[2][az_][bz_] + xi * Fr[2][az_][bz_];
            accr[ia * NCB + ib] += cr * yr - ci * yi;
            acci[ia * NCB + ib] += cr * yi + ci * yr;
          }
      }
  }
  const size_t base = ((size_t)kpi * pp.nq + iq) * pp.nao * pp.nao;
#pragma unroll
  for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NCB; ++ib) {
      const size_t o = base + (size_t)(s1.foff + ia) * pp.nao + s2.foff + ib;
      pp.B[2 * o] = accr[ia * NCB + ib];
      pp.B[2 * o + 1] = acci[ia * NCB + ib];
    }
  return cnt;
}

__global__ void pairft_kernel(const PairFTParams pp) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)pp.nq * pp.nkpi;
  long long cnt = 0;
  if (gid < (int64_t)pp.npair * 2 * per) {
    const int ip = (int)(gid / (2 * per));
    const int order = (int)((gid / per) % 2);
    const int rem = (int)(gid % per);
    const int iq = rem / pp.nkpi, kpi = rem % pp.nkpi;
    const Pair pr = pp.pairs[ip];
    if (!(order == 1 && pr.diag)) {
      const int la = pp.ao[pr.sa].l, lb = pp.ao[pr.sb].l;
      // order 1 swaps the shells: (lb, la)
      const int key = order ? (lb * 3 + la) : (la * 3 + lb);
      switch (key) {
        case 0: cnt = pairft_one<0, 0>(pp, ip, order, iq, kpi); break;
        case 1: cnt = pairft_one<0, 1>(pp, ip, order, iq, kpi); break;
        case 2: cnt = pairft_one<0, 2>(pp, ip, order, iq, kpi); break;
        case 3: cnt = pairft_one<1, 0>(pp, ip, order, iq, kpi); break;
        case 4: cnt = pairft_one<1, 1>(pp, ip, order, iq, kpi); break;
        case 5: cnt = pairft_one<1, 2>(pp, ip, order, iq, kpi); break;
        case 6: cnt = pairft_one<2, 0>(pp, ip, order, iq, kpi); break;
        case 7: cnt = pairft_one<2, 1>(pp, ip, order, iq, kpi); break;
        case 8: cnt = pairft_one<2, 2>(pp, ip, order, iq, kpi); break;
        default: break;
      }
    }
  }
  pp.nterm[gid] = cnt;
}

hipError_t launch_pairft(const PairFTParams &pp, int64_t nthreads_padded, hipStream_t stream) {
  if (nthreads_padded == 0) return hipSuccess;
  hipLaunchKernelGGL(pairft_kernel, dim3((unsigned)(nthreads_padded / 64)), dim3(64), 0, stream, pp);
  return hipGetLastError();
}

// ---- G-space contraction (FP64) ---------------------------------------------
// out[kp][P][mn] += sum_q A[P][q] B[kpi][q][mn], complex, one k-pair per grid z.


constexpr int LG_TM = 32, LG_TN = 64, LG_TK = 16;

__global__ __launch_bounds__(256) void lr_gemm_f64_kernel(const LRGemmParams gp) {
  __shared__ double sAr[LG_TK][LG_TM], sAi[LG_TK][LG_TM];
  __shared__ double sBr[LG_TK][LG_TN], sBi[LG_TK][LG_TN];
  const int kpi = blockIdx.z;
  const int n0 = blockIdx.x * LG_TN, m0 = blockIdx.y * LG_TM;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 4 rows x 8 = 32 rows
  const double *Bk = gp.B + 2 * (size_t)kpi * gp.nq * gp.nmn;
  double cr[8], ci[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) cr[j] = ci[j] = 0.0;
  for (int k0 = 0; k0 < gp.nq; k0 += LG_TK) {
    for (int i = threadIdx.x; i < LG_TK * LG_TM; i += 256) {
      const int kk = i / LG_TM, mm = i % LG_TM;
      const bool ok = (k0 + kk < gp.nq) && (m0 + mm < gp.naux);
      const size_t o = (size_t)(m0 + mm) * gp.lda + k0 + kk;
      sAr[kk][mm] = ok ? gp.A[2 * o] : 0.0;
      sAi[kk][mm] = ok ? gp.A[2 * o + 1] : 0.0;
    }
    for (int i = threadIdx.x; i < LG_TK * LG_TN; i += 256) {
      const int kk = i / LG_TN, nn = i % LG_TN;
      const bool ok = (k0 + kk < gp.nq) && (n0 + nn < gp.nmn);
      const size_t o = (size_t)(k0 + kk) * gp.nmn + n0 + nn;
      sBr[kk][nn] = ok ? Bk[2 * o] : 0.0;
      sBi[kk][nn] = ok ? Bk[2 * o + 1] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < LG_TK; ++kk) {
      const double br = sBr[kk][tx], bi = sBi[kk][tx];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double ar = sAr[kk][ty * 8 + j], ai = sAi[kk][ty * 8 + j];
        cr[j] += ar * br - ai * bi;
        ci[j] += ar * bi + ai * br;
      }
    }
    __syncthreads();
  }
  const int n = n0 + tx;
  if (n >= gp.nmn) return;
  const size_t kp = gp.kp_of[kpi];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = m0 + ty * 8 + j;
    if (m >= gp.naux) continue;
    const size_t o = kp * gp.plane + (size_t)m * gp.nmn + n;
    gp.out[2 * o] += cr[j];
    gp.out[2 * o + 1] += ci[j];
  }
}

hipError_t launch_lr_gemm_f64(const LRGemmParams &gp, int nkpi, hipStream_t stream) {
  dim3 grid((gp.nmn + LG_TN - 1) / LG_TN, (gp.naux + LG_TM - 1) / LG_TM, nkpi);
  hipLaunchKernelGGL(lr_gemm_f64_kernel, grid, dim3(256), 0, stream, gp);
  return hipGetLastError();
}

}  // namespace rsgdf
