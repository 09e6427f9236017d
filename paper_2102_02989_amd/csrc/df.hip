// df.hip -- the density-fitting solve of Eq. M4 on gfx950:
//     sum_Q J^{k12}_PQ d^{k1k2}_{Q mu nu} = V^{k1k2}_{P mu nu}   for every k-pair,
// with J^k Hermitian positive definite (a Coulomb metric with q = 0 removed).
// Per k of the mesh (one workgroup each, the matrices are a few MB and stay in
// L2):
//   1. Cholesky factor J = L L^H (left-looking, column by column: the rows
//      below the diagonal in parallel, each summing over the columns already
//      done; the diagonal by a fixed-order reduction through LDS);
//   2. W = L^{-1} by forward substitution, one column of W per thread.
// Then for every k-pair Y = W V and d = W^H Y (the forward and backward
// substitutions of L L^H d = V as products with the substituted inverse, which
// keeps the error of two triangular solves) as complex FP64 matrix products on
// the matrix cores (v_mfma_f64_16x16x4f64), V row-major [naux][ncol] with the
// columns (mu, nu) contiguous.  A pivot below 1e-12 of its diagonal entry of
// J^k (J numerically singular: linearly dependent aux functions) sets a flag;
// the host reports it.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace rsgdf {

constexpr int kCholThreads = 1024;

// J [nk][n][n] complex (read: lower triangle), L [nk][n][n] complex (written:
// lower triangle incl. diagonal; the strict upper triangle is zeroed), bad [nk]
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const double *__restrict__ J, double *__restrict__ L,
                                                            int n, int *__restrict__ bad) {
  __shared__ double red[kCholThreads];
  __shared__ double rowj[2 * 1024];  // L[j][0..j) of the current column, in chunks of 1024
  __shared__ double sdiag;
  const int k = blockIdx.x, tid = threadIdx.x;
  const double *Jk = J + 2 * (size_t)k * n * n;
  double *Lk = L + 2 * (size_t)k * n * n;
  for (size_t i = tid; i < (size_t)n * n; i += kCholThreads) {
    const size_t r = i / n, c = i % n;
    Lk[2 * i] = (c <= r) ? Jk[2 * i] : 0.0;
    Lk[2 * i + 1] = (c < r) ? Jk[2 * i + 1] : 0.0;
  }
  __syncthreads();
  int failed = 0;
  for (int j = 0; j < n; ++j) {
    // diagonal: J_jj - sum_{c<j} |L_jc|^2, partial sums per thread then a tree
    double s = 0.0;
    for (int c = tid; c < j; c += kCholThreads) {
      const double xr = Lk[2 * ((size_t)j * n + c)], xi = Lk[2 * ((size_t)j * n + c) + 1];
      s += xr * xr + xi * xi;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = kCholThreads / 2; w >= 1; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const double jj = Lk[2 * ((size_t)j * n + j)];
      const double dj = jj - red[0];
      if (!(dj > 1e-12 * jj)) failed = 1;
      sdiag = (dj > 0.0) ? sqrt(dj) : 1.0;
      Lk[2 * ((size_t)j * n + j)] = sdiag;
      Lk[2 * ((size_t)j * n + j) + 1] = 0.0;
    }
    __syncthreads();
    const double inv = 1.0 / sdiag;
    // rows i > j: (J_ij - sum_{c<j} L_ic conj(L_jc)) / L_jj, row j staged in LDS
    for (int i0 = j + 1; i0 < n; i0 += kCholThreads) {
      const int i = i0 + tid;
      double ar = 0.0, ai = 0.0;
      if (i < n) {
        ar = Lk[2 * ((size_t)i * n + j)];
        ai = Lk[2 * ((size_t)i * n + j) + 1];
      }
      for (int c0 = 0; c0 < j; c0 += 1024) {
        const int cn = (j - c0 < 1024) ? j - c0 : 1024;
        __syncthreads();
        for (int c = tid; c < cn; c += kCholThreads) {
          rowj[2 * c] = Lk[2 * ((size_t)j * n + c0 + c)];
          rowj[2 * c + 1] = Lk[2 * ((size_t)j * n + c0 + c) + 1];
        }
        __syncthreads();
        if (i < n) {
          const double *Li = Lk + 2 * ((size_t)i * n + c0);
          for (int c = 0; c < cn; ++c) {
            const double lr = Li[2 * c], li = Li[2 * c + 1], jr = rowj[2 * c], ji = rowj[2 * c + 1];
            // L_ic conj(L_jc)
            ar -= lr * jr + li * ji;
            ai -= li * jr - lr * ji;
          }
        }
      }
      if (i < n) {
        Lk[2 * ((size_t)i * n + j)] = ar * inv;
        Lk[2 * ((size_t)i * n + j) + 1] = ai * inv;
      }
    }
    __syncthreads();
  }
  if (tid == 0) bad[k] = failed;
}

// W = L^{-1} (lower triangular), one column of W per thread:
//   W_jj = 1/L_jj,  W_ij = -(sum_{c=j}^{i-1} L_ic W_cj) / L_ii  (i > j).
// W [nk][n][n] complex, strict upper triangle zeroed.
__global__ __launch_bounds__(256) void trinv_kernel(const double *__restrict__ L, double *__restrict__ W, int n) {
  const int k = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double *Lk = L + 2 * (size_t)k * n * n;
  double *Wk = W + 2 * (size_t)k * n * n;
  for (int i = 0; i < j; ++i) {
    Wk[2 * ((size_t)i * n + j)] = 0.0;
    Wk[2 * ((size_t)i * n + j) + 1] = 0.0;
  }
  Wk[2 * ((size_t)j * n + j)] = 1.0 / Lk[2 * ((size_t)j * n + j)];
  Wk[2 * ((size_t)j * n + j) + 1] = 0.0;
  for (int i = j + 1; i < n; ++i) {
    double sr = 0.0, si = 0.0;
    const double *Li = Lk + 2 * (size_t)i * n;
    for (int c = j; c < i; ++c) {
      const double lr = Li[2 * c], li = Li[2 * c + 1];
      const double wr = Wk[2 * ((size_t)c * n + j)], wi = Wk[2 * ((size_t)c * n + j) + 1];
      sr += lr * wr - li * wi;
      si += lr * wi + li * wr;
    }
    const double d = 1.0 / Li[2 * i];
    Wk[2 * ((size_t)i * n + j)] = -sr * d;
    Wk[2 * ((size_t)i * n + j) + 1] = -si * d;
  }
}

hipError_t launch_df_factor(const double *J, double *L, double *W, int *bad, int nk, int n, hipStream_t stream) {
  if (nk == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3((unsigned)nk), dim3(kCholThreads), 0, stream, J, L, n, bad);
  hipLaunchKernelGGL(trinv_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nk), dim3(256), 0, stream, L, W, n);
  return hipGetLastError();
}

// ---- Y = W V and d = W^H Y on the FP64 matrix cores -----------------------------
// C[t][m][n] = sum_q op(A)[cls[t]][m][q] B[t][q][n], complex, op(A) = A
// (CONJT = false) or A^H (CONJT = true, op(A)[m][q] = conj(A[q][m])); A
// [*][M][M] row-major, B and C [*][M][N] (n contiguous).  W is lower
// triangular: the q steps where op(A)'s tile is zero are skipped (q > m for W,
// q < m for W^H).  Workgroup tile 128 x 128, 8
// waves as 4 (rows of 32) x 2 (columns of 64); 16 q per step staged in LDS,
// the next step's loads in flight during the MFMAs.  Fragments (li = lane %
// 16, lg = lane / 16): A[li][lg], B[lg][li]; result D[lg + 4 v][li].
typedef double df_d4 __attribute__((ext_vector_type(4)));
constexpr int DG_BM = 128, DG_BN = 128, DG_BK = 16, DG_NT = 512;

template <bool CONJT>
__global__ __launch_bounds__(DG_NT) void df_gemm_kernel(const double *__restrict__ A, const int32_t *__restrict__ cls,
                                                        const double *__restrict__ B, double *__restrict__ C, int M,
                                                        int64_t N) {
  __shared__ double sar[DG_BM][DG_BK + 1], sai[DG_BM][DG_BK + 1];
  __shared__ double sbr[DG_BK][DG_BN + 1], sbi[DG_BK][DG_BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;
  const int t = blockIdx.z;
  const int M0 = blockIdx.y * DG_BM;
  const int64_t N0 = (int64_t)blockIdx.x * DG_BN;
  const double *At = A + 2 * (size_t)cls[t] * M * M;
  const double *Bt = B + 2 * (size_t)t * M * N;
  double *Ct = C + 2 * (size_t)t * M * N;
  // staging: A tile 128 x 16 (thread: row tid/4, 4 q), B tile 16 x 128 (thread: q tid/32, 4 columns)
  const int ar0 = tid >> 2, aq = (tid & 3) * 4;
  const int bq = tid >> 5, bc = (tid & 31) * 4;
  double ga[8], gb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = M0 + ar0, k = k0 + aq + j;
      const bool ok = m < M && k < M;
      const size_t o = CONJT ? (size_t)k * M + m : (size_t)m * M + k;
      ga[2 * j] = ok ? At[2 * o] : 0.0;
      ga[2 * j + 1] = ok ? (CONJT ? -At[2 * o + 1] : At[2 * o + 1]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + bq;
      const int64_t col = N0 + bc + j;
      const bool ok = k < M && col < N;
      gb[2 * j] = ok ? Bt[2 * ((size_t)k * N + col)] : 0.0;
      gb[2 * j + 1] = ok ? Bt[2 * ((size_t)k * N + col) + 1] : 0.0;
    }
  };
  df_d4 cre[2][4], cim[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) cre[r][c][v] = cim[r][c][v] = 0.0;
  // non-zero q range of the row tile: W (lower) has q <= m, W^H has q >= m
  const int kbeg = CONJT ? (M0 / DG_BK) * DG_BK : 0;
  const int kend = CONJT ? M : (M0 + DG_BM < M ? M0 + DG_BM : M);
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += DG_BK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sar[ar0][aq + j] = ga[2 * j];
      sai[ar0][aq + j] = ga[2 * j + 1];
      sbr[bq][bc + j] = gb[2 * j];
      sbi[bq][bc + j] = gb[2 * j + 1];
    }
    __syncthreads();
    if (k0 + DG_BK < kend) gload(k0 + DG_BK);
#pragma unroll
    for (int ks = 0; ks < DG_BK / 4; ++ks) {
      const int k = ks * 4 + lg;
      double a_r[2], a_i[2], b_r[4], b_i[4];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        a_r[r] = sar[wm * 32 + r * 16 + li][k];
        a_i[r] = sai[wm * 32 + r * 16 + li][k];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        b_r[c] = sbr[k][wn * 64 + c * 16 + li];
        b_i[c] = sbi[k][wn * 64 + c * 16 + li];
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[r], b_r[c], cre[r][c], 0, 0, 0);
          cre[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_i[r], b_i[c], cre[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[r], b_i[c], cim[r][c], 0, 0, 0);
          cim[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[r], b_r[c], cim[r][c], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = M0 + wm * 32 + r * 16 + lg + 4 * v;
        const int64_t col = N0 + wn * 64 + c * 16 + li;
        if (m < M && col < N) {
          Ct[2 * ((size_t)m * N + col)] = cre[r][c][v];
          Ct[2 * ((size_t)m * N + col) + 1] = cim[r][c][v];
        }
      }
}

hipError_t launch_df_gemm(bool conjt, const double *W, const int32_t *cls, const double *V, double *D, int naux,
                          int64_t ncol, int nkp, hipStream_t stream) {
  if (nkp == 0 || naux == 0 || ncol == 0) return hipSuccess;
  const int64_t gx = (ncol + DG_BN - 1) / DG_BN;
  if (gx > 0x7fffffff || nkp > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)gx, (unsigned)((naux + DG_BM - 1) / DG_BM), (unsigned)nkp);
  if (conjt) hipLaunchKernelGGL(df_gemm_kernel<true>, grid, dim3(DG_NT), 0, stream, W, cls, V, D, naux, ncol);
  else hipLaunchKernelGGL(df_gemm_kernel<false>, grid, dim3(DG_NT), 0, stream, W, cls, V, D, naux, ncol);
  return hipGetLastError();
}

}  // namespace rsgdf
