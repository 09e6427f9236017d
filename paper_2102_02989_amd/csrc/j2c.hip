// j2c.hip -- the two-center metric of the density fit on gfx950 (Eq. M5):
//     J^k_PQ = sum_m e^{+i k.m} (P^0 | 1/r | Q^m),   q = 0 (G = 0 at k = 0) removed,
// range-separated like the three-center integrals (Eq. M9):
//   short range: sum_m e^{+ik.m} (P^0 | erfc(w r)/r | Q^m), binned by the
//                Born-von Karman cell of m (Eq. M14 for one lattice index) and
//                Fourier transformed over the Nk cells;
//   G = 0 term:  minus pi/(Omega w^2) S_P S_Q at k = 0 (Eq. M12's second term
//                with the pair density replaced by chi_Q);
//   long range:  (4 pi/Omega) sum_{q=G+k} e^{-q^2/4w^2}/q^2 chi~_P(-q) chi~_Q(q)
//                (Eq. M10 with the second transform chi~_Q): the matrix product
//                A A^H / w of the aux transforms A[P][q] = w(q) chi~_P(-q)
//                that the three-center long-range part already forms, on the
//                FP64 matrix cores (the contraction kernel of lr.hip).
//
// Short-range work unit: one wavefront per (P shell, Q shell, BvK cell c).
// Lanes walk the lattice vectors m of cell c (m = L_c + n (x) M over the box
// that covers the screening sphere |C_P - B_Q - m| <= r_max) and sum the
// McMurchie-Davidson Hermite integrals R_tuv of the erfc operator at
// X = C_P - (B_Q + m); a butterfly over the 64 lanes (bitwise identical on
// every lane) reduces them, and the lanes contract them with the single-centre
// Hermite coefficients of P and Q, one Cartesian element each:
//   (P|Q) = 2 pi^{5/2}/(a_P a_Q sqrt(a_P + a_Q)) sum_{tuv} E^P_{tuv}
//           sum_{t'u'v'} (-1)^{t'+u'+v'} E^Q_{t'u'v'} R_{t+t',u+u',v+v'}(rho, X),
//   rho = a_P a_Q/(a_P + a_Q).
// Every (c, P, Q) block is written by exactly one wave: no atomics, results
// reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "boys.h"
#include "device_math.h"
#include "kernels.h"
#include "plan.h"

namespace rsgdf {

template <int LP, int LQ>
__global__ __launch_bounds__(64) void j2c_sr_kernel(const J2Params jp, int p0) {
  constexpr int L = LP + LQ, NH = nherm(L), NCP = ncart(LP), NCQ = ncart(LQ), NC = NCP * NCQ;
  static_assert(NC <= 128, "two elements per lane");
  __shared__ double sR[NH];
  __shared__ double sEP[LP + 1][LP + 1], sEQ[LQ + 1][LQ + 1];
  // the order-L Boys polynomials, rows padded to 16-byte boundaries (the
  // layout gvals_sr reads)
  __shared__ __attribute__((aligned(16))) double s_boys[kBoysIntervals * (kBoysPolyDeg + 2)];
  const int lane = threadIdx.x;
  for (int i = lane; i < kBoysIntervals * (kBoysPolyDeg + 1); i += 64)
    s_boys[(i / (kBoysPolyDeg + 1)) * (kBoysPolyDeg + 2) + i % (kBoysPolyDeg + 1)] =
        jp.boys[L * kBoysIntervals * (kBoysPolyDeg + 1) + i];
  for (int i = lane; i < kBoysIntervals; i += 64) s_boys[i * (kBoysPolyDeg + 2) + kBoysPolyDeg + 1] = 0.0;
  __syncthreads();
  const J2Pair pr = jp.pairs[p0 + blockIdx.x];
  const int c = blockIdx.y;
  const Lattice &Lt = jp.lat;
  const Shell P = jp.ax[pr.P], Q = jp.ax[pr.Q];
  const int ci[3] = {c / (Lt.n[1] * Lt.n[2]), (c / Lt.n[2]) % Lt.n[1], c % Lt.n[2]};
  // box of supercell indices M: m_d = ci_d + n_d M_d with |C_P - B_Q - m| <= r_max
  const double dx = P.x - Q.x, dy = P.y - Q.y, dz = P.z - Q.z;
  int lo[3], cnt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double bx = Lt.b[3 * d], by = Lt.b[3 * d + 1], bz = Lt.b[3 * d + 2];
    const double f = (dx * bx + dy * by + dz * bz) * (0.5 / kPi);
    const double h = pr.rmax * sqrt(bx * bx + by * by + bz * bz) * (0.5 / kPi);
    lo[d] = (int)ceil((f - h - ci[d]) / Lt.n[d]);
    const int hi = (int)floor((f + h - ci[d]) / Lt.n[d]);
    cnt[d] = hi >= lo[d] ? hi - lo[d] + 1 : 0;
  }
  const int total = cnt[0] * cnt[1] * cnt[2];
  const double r2max = pr.rmax * pr.rmax;
  double acc[2] = {0.0, 0.0};
  long long nterm = 0;
  for (int iP = 0; iP < P.nprim; ++iP)
    for (int iQ = 0; iQ < Q.nprim; ++iQ) {
      const double gP = jp.ax_exp[P.pptr + iP], gQ = jp.ax_exp[Q.pptr + iQ];
      const double cP = jp.ax_coef[P.pptr + iP], cQ = jp.ax_coef[Q.pptr + iQ];
      const double s = gP + gQ, rho = gP * gQ / s;
      const double om2 = jp.omega * jp.omega, th2 = om2 / (om2 + rho), th = sqrt(th2);
      const double pref = cP * cQ * 2.0 * kPi * kPi * sqrt(kPi) / (gP * gQ * sqrt(s));
      double Rs[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) Rs[h] = 0.0;
      for (int idx = lane; idx < total; idx += 64) {
        const int i0 = idx / (cnt[1] * cnt[2]), i1 = (idx / cnt[2]) % cnt[1], i2 = idx % cnt[2];
        const int m0 = ci[0] + Lt.n[0] * (lo[0] + i0), m1 = ci[1] + Lt.n[1] * (lo[1] + i1),
                  m2 = ci[2] + Lt.n[2] * (lo[2] + i2);
        const double X = dx - (m0 * Lt.a[0] + m1 * Lt.a[3] + m2 * Lt.a[6]);
        const double Y = dy - (m0 * Lt.a[1] + m1 * Lt.a[4] + m2 * Lt.a[7]);
        const double Z = dz - (m0 * Lt.a[2] + m1 * Lt.a[5] + m2 * Lt.a[8]);
        const double r2 = X * X + Y * Y + Z * Z;
        if (r2 > r2max) continue;
        ++nterm;
        double G[L + 1], g[L + 1];
        gvals_sr<L>(rho * r2, th2, th, s_boys, G);
        double f = 1.0;
#pragma unroll
        for (int n = 0; n <= L; ++n) {
          g[n] = f * G[n];
          f *= -2.0 * rho;
        }
        hermite_R_acc<L>(X, Y, Z, g, Rs);
      }
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) Rs[h] += __shfl_xor(Rs[h], o, 64);
      if (lane == 0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) sR[h] = Rs[h];
        double EP[LP + 1][LP + 1], EQ[LQ + 1][LQ + 1];
        hermite_E1<LP>(0.5 / gP, EP);
        hermite_E1<LQ>(0.5 / gQ, EQ);
#pragma unroll
        for (int i = 0; i <= LP; ++i)
#pragma unroll
          for (int t = 0; t <= LP; ++t) sEP[i][t] = EP[i][t];
#pragma unroll
        for (int i = 0; i <= LQ; ++i)
#pragma unroll
          for (int t = 0; t <= LQ; ++t) sEQ[i][t] = EQ[i][t];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int e = lane + 64 * r;
        if (e >= NC) continue;
        const int a = e / NCQ, b = e % NCQ;
        const int px = cart_lx(LP, a), py = cart_ly(LP, a), pz = LP - px - py;
        const int qx = cart_lx(LQ, b), qy = cart_ly(LQ, b), qz = LQ - qx - qy;
        double sum = 0.0;
        for (int t = px & 1; t <= px; t += 2)
          for (int u = py & 1; u <= py; u += 2)
            for (int v = pz & 1; v <= pz; v += 2) {
              const double ep = sEP[px][t] * sEP[py][u] * sEP[pz][v];
              double inner = 0.0;
              for (int t2 = qx & 1; t2 <= qx; t2 += 2)
                for (int u2 = qy & 1; u2 <= qy; u2 += 2)
                  for (int v2 = qz & 1; v2 <= qz; v2 += 2) {
                    const double eq = sEQ[qx][t2] * sEQ[qy][u2] * sEQ[qz][v2];
                    const double sg = ((t2 + u2 + v2) & 1) ? -1.0 : 1.0;
                    inner += sg * eq * sR[hidx(t + t2, u + u2, v + v2)];
                  }
              sum += ep * inner;
            }
        acc[r] += pref * sum;
      }
      __syncthreads();
    }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = lane + 64 * r;
    if (e >= NC) continue;
    const int a = e / NCQ, b = e % NCQ;
    jp.X2[((size_t)c * jp.naux + P.foff + a) * jp.naux + Q.foff + b] = acc[r];
  }
  // evaluated (P prim, Q prim, m) terms: one integer atomic per wave
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nterm += __shfl_xor(nterm, o, 64);
  if (lane == 0 && nterm) atomicAdd(reinterpret_cast<unsigned long long *>(jp.nterm), (unsigned long long)nterm);
}

hipError_t launch_j2c_sr(int lP, int lQ, const J2Params &jp, int p0, int npair, hipStream_t stream) {
  if (npair == 0 || jp.lat.nk == 0) return hipSuccess;
  typedef void (*K)(const J2Params, int);
  static const K ks[4][4] = {
      {j2c_sr_kernel<0, 0>, j2c_sr_kernel<0, 1>, j2c_sr_kernel<0, 2>, j2c_sr_kernel<0, 3>},
      {j2c_sr_kernel<1, 0>, j2c_sr_kernel<1, 1>, j2c_sr_kernel<1, 2>, j2c_sr_kernel<1, 3>},
      {j2c_sr_kernel<2, 0>, j2c_sr_kernel<2, 1>, j2c_sr_kernel<2, 2>, j2c_sr_kernel<2, 3>},
      {j2c_sr_kernel<3, 0>, j2c_sr_kernel<3, 1>, j2c_sr_kernel<3, 2>, j2c_sr_kernel<3, 3>}};
  if (lP < 0 || lP > 3 || lQ < 0 || lQ > 3) return hipErrorInvalidValue;
  if (jp.lat.nk > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(ks[lP][lQ], dim3((unsigned)npair, (unsigned)jp.lat.nk), dim3(64), 0, stream, jp, p0);
  return hipGetLastError();
}

// J[k][e] = sum_c e^{+ik.L_c} X2[c][e] (overwrites), minus g0fac S_P S_Q at k = 0.
// One thread per element e = (P, Q) of the naux x naux plane.
__global__ __launch_bounds__(256) void j2c_fold_kernel(const double *__restrict__ X2, const double *__restrict__ kph,
                                                       const double *__restrict__ SP, double g0fac, int nk,
                                                       int32_t naux, double *__restrict__ J) {
  const int64_t n2 = (int64_t)naux * naux;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2) return;
  const double g0 = g0fac * SP[e / naux] * SP[e % naux];
  for (int k = 0; k < nk; ++k) {
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nk; ++c) {
      const double x = X2[(int64_t)c * n2 + e];
      sr += kph[2 * (k * nk + c)] * x;
      si += kph[2 * (k * nk + c) + 1] * x;
    }
    if (k == 0) sr -= g0;
    J[2 * ((int64_t)k * n2 + e)] = sr;
    J[2 * ((int64_t)k * n2 + e) + 1] = si;
  }
}

hipError_t launch_j2c_fold(const double *X2, const double *kph, const double *SP, double g0fac, int nk, int naux,
                           double *J, hipStream_t stream) {
  const int64_t n2 = (int64_t)naux * naux;
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(j2c_fold_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, stream, X2, kph, SP, g0fac,
                     nk, (int32_t)naux, J);
  return hipGetLastError();
}

// Second operand of the long-range product: B[Q][q] = conj(A[Q][q]) / w(q) =
// chi~_Q(+q) for real aux functions, w(q) = (4 pi/Omega) e^{-q^2/4w^2}/q^2,
// for the q columns [0, nq) of one class (A row stride lda, q contiguous).
__global__ __launch_bounds__(256) void j2c_lr_operand_kernel(const double *__restrict__ A, int64_t lda,
                                                             const double *__restrict__ q, int nq, int naux,
                                                             double wfac, double omega, double *__restrict__ B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)naux * nq) return;
  const int64_t P = i / nq, iq = i % nq;
  const double qx = q[3 * iq], qy = q[3 * iq + 1], qz = q[3 * iq + 2];
  const double q2 = qx * qx + qy * qy + qz * qz;
  const double w = wfac * exp(-q2 / (4.0 * omega * omega)) / q2;
  const double ar = A[2 * (P * lda + iq)], ai = A[2 * (P * lda + iq) + 1];
  B[2 * i] = ar / w;
  B[2 * i + 1] = -ai / w;
}

hipError_t launch_j2c_lr_operand(const double *A, int64_t lda, const double *q, int nq, int naux, double wfac,
                                 double omega, double *B, hipStream_t stream) {
  const int64_t n = (int64_t)naux * nq;
  if (n == 0) return hipSuccess;
  if ((n + 255) / 256 > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(j2c_lr_operand_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, A, lda, q, nq,
                     naux, wfac, omega, B);
  return hipGetLastError();
}

}  // namespace rsgdf
