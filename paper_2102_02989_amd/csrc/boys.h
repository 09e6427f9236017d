// boys.h -- FP64 Boys-function values of the erfc-attenuated Coulomb operator
// on gfx950 (shared by the three-center and two-center short-range kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace rsgdf {

// e^{-T} for T >= 0 by Cody-Waite range reduction: T = k ln 2 + r with
// k = rint(T / ln 2) and |r| <= ln(2)/2, ln 2 split into a 32-bit head (k ln2_hi
// is exact for the k that occur) and a tail; e^{-T} = 2^{-k} e^{-r}, with e^{-r}
// from its Taylor series to degree 13 (truncation below 5e-18 relative) by
// Estrin's scheme and 2^{-k} applied exactly by ldexp.  No table, so no LDS
// read in the image loop.  Zero for T >= 64 (e^{-64} < 2e-28).
__device__ __forceinline__ double exp_neg(double T) {
  const double Tc = fmin(T, 64.0);
  const double k = rint(Tc * 1.4426950408889634);  // log2(e)
  const double v = -fma(-k, 1.9082149292705877e-10, fma(-k, 0.6931471803691238, Tc));  // -r
  const double v2 = v * v, v4 = v2 * v2, v8 = v4 * v4;
  // 1/n!, n = 0..13
  const double a0 = fma(v, 1.0, 1.0);
  const double a1 = fma(v, 1.0 / 6.0, 1.0 / 2.0);
  const double a2 = fma(v, 1.0 / 120.0, 1.0 / 24.0);
  const double a3 = fma(v, 1.0 / 5040.0, 1.0 / 720.0);
  const double a4 = fma(v, 1.0 / 362880.0, 1.0 / 40320.0);
  const double a5 = fma(v, 1.0 / 39916800.0, 1.0 / 3628800.0);
  const double a6 = fma(v, 1.0 / 6227020800.0, 1.0 / 479001600.0);
  const double b0 = fma(a1, v2, a0), b1 = fma(a3, v2, a2), b2 = fma(a5, v2, a4);
  const double d0 = fma(b1, v4, b0), d1 = fma(a6, v4, b2);
  const double e = ldexp(fma(d1, v8, d0), -(int)k);
  return T < 64.0 ? e : 0.0;
}

// F_L(T) for 0 <= T < kBoysSwitch from the per-L polynomial table (Taylor
// expansion of degree kBoysPolyDeg about each unit interval's centre), then the
// downward recursion F_n = (2T F_{n+1} + e^{-T})/(2n+1), e = e^{-T} given.
// The polynomial is evaluated by Estrin's scheme (pairs, then powers u^2,
// u^4, u^8): dependency depth 5 instead of 12 for Horner's rule.  The table in
// LDS holds kBoysPolyDeg + 2 doubles per interval (the last one zero), so an
// interval starts on a 16-byte boundary and its coefficients arrive in seven
// 16-byte reads issued back to back, before the first multiply waits on them
// (boys_row; the caller issues the reads of both Boys arguments together).
static_assert(kBoysPolyDeg == 12, "Estrin evaluation below is written for degree 12");
__device__ __forceinline__ void boys_row(const double *__restrict__ tab, int i, double2 (&c)[7]) {
  const double2 *c2 = reinterpret_cast<const double2 *>(tab + i * (kBoysPolyDeg + 2));
#pragma unroll
  for (int k = 0; k < 7; ++k) c[k] = c2[k];
}
template <int L>
__device__ __forceinline__ void boys_poly(double T, int i, double e, const double2 (&c)[7], double (&F)[L + 1]) {
  const double u = T - (i + 0.5);
  const double u2 = u * u, u4 = u2 * u2, u8 = u4 * u4;
  const double a0 = fma(c[0].y, u, c[0].x), a1 = fma(c[1].y, u, c[1].x), a2 = fma(c[2].y, u, c[2].x);
  const double a3 = fma(c[3].y, u, c[3].x), a4 = fma(c[4].y, u, c[4].x), a5 = fma(c[5].y, u, c[5].x);
  const double b0 = fma(a1, u2, a0), b1 = fma(a3, u2, a2), b2 = fma(a5, u2, a4);
  const double d0 = fma(b1, u4, b0), d1 = fma(c[6].x, u4, b2);
  F[L] = fma(d1, u8, d0);
  const double t2 = 2.0 * T;
#pragma unroll
  for (int n = L - 1; n >= 0; --n) F[n] = fma(t2, F[n + 1], e) * (1.0 / (2 * n + 1));
}

// F_n(T), n = 0..L, for T >= kBoysSwitch: F_0 = sqrt(pi/T)/2 and the upward
// recursion F_{n+1} = ((2n+1) F_n - e^{-T}) / (2T), e = e^{-T} given; 1/sqrt(T)
// from one reciprocal square root, 1/T as its square.
template <int L>
__device__ __forceinline__ void boys_large_e(double T, double e, double (&F)[L + 1]) {
  const double r = rsqrt(T);
  F[0] = 0.886226925452758013649083741671 * r; /* sqrt(pi)/2 */
  const double h = 0.5 * r * r;
#pragma unroll
  for (int n = 0; n < L; ++n) F[n + 1] = ((2 * n + 1) * F[n] - e) * h;
}

// Boys values of the attenuated operator erfc(w r)/r = 1/r - erf(w r)/r: the
// erf part of a primitive triple with reduced exponent rho is the Coulomb
// part at exponent rho w^2/(rho + w^2), that is at T theta^2 with
// theta^2 = w^2/(w^2 + rho), scaled by theta^{2n+1} for order n; so
// G_n = F_n(T) - theta^{2n+1} F_n(theta^2 T), set to zero once
// theta^2 T >= kBoysSwitch (both terms share their asymptote to within e^{-theta^2 T}).
template <int L>
__device__ __forceinline__ void gvals_sr(double T, double th2, double th, const double *__restrict__ tab,
                                         double (&G)[L + 1]) {
  const double x = th2 * T;
  if (x >= kBoysSwitch) {
#pragma unroll
    for (int n = 0; n <= L; ++n) G[n] = 0.0;
    return;
  }
  double F1[L + 1], F2[L + 1];
  const int ix = (int)x;
  const int iT = T < kBoysSwitch ? (int)T : kBoysIntervals - 1;  // row read but unused for T beyond the table
  double2 cx[7], cT[7];
  boys_row(tab, ix, cx);
  boys_row(tab, iT, cT);
  const double eT = (L > 0) ? exp_neg(T) : 0.0;
  boys_poly<L>(x, ix, (L > 0) ? exp_neg(x) : 0.0, cx, F2);
  if (T < kBoysSwitch) boys_poly<L>(T, iT, eT, cT, F1);
  else boys_large_e<L>(T, eT, F1);
  double f = th;
#pragma unroll
  for (int n = 0; n <= L; ++n) {
    G[n] = F1[n] - f * F2[n];
    f *= th2;
  }
}

}  // namespace rsgdf
