// device_math.h -- gfx950 device building blocks of the three-center
// integrals: McMurchie-Davidson Hermite expansion coefficients and Hermite
// Coulomb integrals R_tuv (the Boys values are in sr3c.hip).
//
// Everything is templated on angular momenta so that all array indices are
// compile-time constants and the working sets live in VGPRs.
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace rsgdf {

// Tetrahedral index of the Hermite triple (t,u,v): shells s = t+u+v in order,
// inside a shell r = u+v ascending, then v ascending.
__host__ __device__ constexpr int hidx(int t, int u, int v) {
  return (t + u + v) * (t + u + v + 1) * (t + u + v + 2) / 6 + (u + v) * (u + v + 1) / 2 + v;
}

// Cartesian component i of angular momentum l: x power descending, then y.
__host__ __device__ constexpr int cart_lx(int l, int i) {
  int n = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      if (n == i) return lx;
      ++n;
    }
  return 0;
}
__host__ __device__ constexpr int cart_ly(int l, int i) {
  int n = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      if (n == i) return ly;
      ++n;
    }
  return 0;
}
__host__ __device__ constexpr int cart_lz(int l, int i) { return l - cart_lx(l, i) - cart_ly(l, i); }

// Hermite Coulomb integrals R_tuv (t+u+v <= L) at X = P - C from
// g[n] = (-2 rho)^n G_n: R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X R^(n+1)_{t,u,v}
// (and likewise in y, z), evaluated in place from n = L down to 0, with
// R^(0)_tuv added into Racc: levels n >= 1 are built in a scratch array of
// nherm(L-1) entries; level 0 is formed and accumulated directly, shell by
// shell from the top (it only reads level-1 values).
template <int L>
__device__ __forceinline__ void hermite_R_acc(double X, double Y, double Z, const double (&g)[L + 1],
                                              double (&Racc)[nherm(L)]) {
  if constexpr (L == 0) {
    Racc[0] += g[0];
  } else {
    double R[nherm(L - 1)];
    R[0] = g[L];
#pragma unroll
    for (int n = L - 1; n >= 1; --n) {
#pragma unroll
      for (int s = L - n; s >= 1; --s) {
#pragma unroll
        for (int t = s; t >= 0; --t) {
#pragma unroll
          for (int u = s - t; u >= 0; --u) {
            const int v = s - t - u;
            double val;
            if (t > 0) {
              val = X * R[hidx(t - 1, u, v)];
              if (t > 1) val += (t - 1) * R[hidx(t - 2, u, v)];
            } else if (u > 0) {
              val = Y * R[hidx(t, u - 1, v)];
              if (u > 1) val += (u - 1) * R[hidx(t, u - 2, v)];
            } else {
              val = Z * R[hidx(t, u, v - 1)];
              if (v > 1) val += (v - 1) * R[hidx(t, u, v - 2)];
            }
            R[hidx(t, u, v)] = val;
          }
        }
      }
      R[0] = g[n];
    }
    // level 0: R^(0)_{tuv} from level-1 entries (shells s-1, s-2)
#pragma unroll
    for (int s = L; s >= 1; --s) {
#pragma unroll
      for (int t = s; t >= 0; --t) {
#pragma unroll
        for (int u = s - t; u >= 0; --u) {
          const int v = s - t - u;
          double val;
          if (t > 0) {
            val = X * R[hidx(t - 1, u, v)];
            if (t > 1) val += (t - 1) * R[hidx(t - 2, u, v)];
          } else if (u > 0) {
            val = Y * R[hidx(t, u - 1, v)];
            if (u > 1) val += (u - 1) * R[hidx(t, u - 2, v)];
          } else {
            val = Z * R[hidx(t, u, v - 1)];
            if (v > 1) val += (v - 1) * R[hidx(t, u, v - 2)];
          }
          Racc[hidx(t, u, v)] += val;
        }
      }
    }
    Racc[0] += g[0];
  }
}


// McMurchie-Davidson expansion coefficients of a 1-D Gaussian product
// (x-A)^i (x-B)^j exp(...) = K sum_t E[i][j][t] Lambda_t:
//   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
//   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}
template <int LA, int LB>
__device__ __forceinline__ void hermite_E(double PA, double PB, double oo2p,
                                          double (&E)[LA + 1][LB + 1][LA + LB + 1]) {
#pragma unroll
  for (int i = 0; i <= LA; ++i)
#pragma unroll
    for (int j = 0; j <= LB; ++j)
#pragma unroll
      for (int t = 0; t <= LA + LB; ++t) E[i][j][t] = 0.0;
  E[0][0][0] = 1.0;
#pragma unroll
  for (int i = 0; i <= LA; ++i) {
    if (i > 0) {
#pragma unroll
      for (int t = 0; t <= i; ++t) {
        double v = 0.0;
        if (t >= 1) v += oo2p * E[i - 1][0][t - 1];
        if (t <= i - 1) v += PA * E[i - 1][0][t];
        if (t + 1 <= i - 1) v += (t + 1) * E[i - 1][0][t + 1];
        E[i][0][t] = v;
      }
    }
#pragma unroll
    for (int j = 1; j <= LB; ++j) {
#pragma unroll
      for (int t = 0; t <= i + j; ++t) {
        double v = 0.0;
        if (t >= 1) v += oo2p * E[i][j - 1][t - 1];
        if (t <= i + j - 1) v += PB * E[i][j - 1][t];
        if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        E[i][j][t] = v;
      }
    }
  }
}

// Hermite expansion of a single Cartesian Gaussian (x-C)^i exp(-g (x-C)^2):
// E^{i+1}_t = E^i_{t-1}/(2g) + (t+1) E^i_{t+1}.
template <int LP>
__device__ __forceinline__ void hermite_E1(double oo2g, double (&E)[LP + 1][LP + 1]) {
#pragma unroll
  for (int i = 0; i <= LP; ++i)
#pragma unroll
    for (int t = 0; t <= LP; ++t) E[i][t] = 0.0;
  E[0][0] = 1.0;
#pragma unroll
  for (int i = 1; i <= LP; ++i)
#pragma unroll
    for (int t = 0; t <= i; ++t) {
      double v = 0.0;
      if (t >= 1) v += oo2g * E[i - 1][t - 1];
      if (t + 1 <= i - 1) v += (t + 1) * E[i - 1][t + 1];
      E[i][t] = v;
    }
}

}  // namespace rsgdf
