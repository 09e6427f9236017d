// kernels.h -- parameter blocks and host launchers of the fold, overlap and
// long-range kernels (shared by the host planner and the .hip sources).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace rsgdf {

struct FoldParams {
  const double *kph;      // complex [nk][nk]: e^{+i k.L_c}
  const double *X;        // real [nb = nk^2][ne] (may be null: no SR part)
  double *Y;              // complex [nk][nk][echunk] scratch between the two transforms
  double *out;            // complex [nkp][naux][nao][nao]
  const int32_t *kdiag;   // [nkp]: k index if k1 == k2 else -1
  const int32_t *kp1;     // [nkp]: k1 of each k-pair
  const int32_t *tile_k2; // [ntile]: k2 of the tile's k-pairs
  const int32_t *tile_kp; // [ntile][tk]: k-pair indices of the tile, -1 padded
  const double *SP;       // [naux_b] lattice-free aux integrals int chi_P
  const double *Smn;      // complex [nk][nao*nao]
  double g0fac;           // pi / (Omega w^2), 0 disables the G = 0 term
  int64_t ne;             // naux_b * nao * nao
  int64_t echunk;         // elements per pass (Y capacity)
  int64_t out_off;        // aux_f0 * nao * nao
  int64_t plane;          // naux * nao * nao
  int32_t nkp, nk, nao2, ntile;
  int32_t tk;             // k-pair slots per tile: a multiple of 4, at most 64
};

struct OvlParams {
  const Shell *ao;
  const double *ao_exp, *ao_coef;
  const Pair *pairs;
  const int32_t *cls_off;
  const double *img;
  int32_t npair, nk;
  double *O;             // [npair][nk][36]
  double acut;           // > 0: leave out primitive pairs with both exponents below acut
};

struct SmnParams {
  const Shell *ao;
  const Pair *pairs;
  const double *O;
  const double *kphase;  // complex [nk][nk]: exp(+i k.L_c)
  int32_t npair, nk, nao, pad;
  double *S;             // complex [nk][nao][nao]
};

struct AuxFTParams {
  const Shell *ax;
  const double *ax_exp, *ax_coef;
  const double *q;       // [nq][3]
  int32_t nq, nshell, naux, pad;
  double wfac;           // 4 pi / Omega
  double omega;
  double *A;             // complex [naux][nq] (row stride nq)
  double acut;           // primitive selection by exponent (amode)
  int32_t amode;         // 0 every primitive, 1 exponent >= acut, 2 exponent < acut
  int32_t undamped;      // 1: weight 4 pi/(Omega q^2) (Eq. M15), 0: times exp(-q^2/4w^2) (Eq. M10)
};

struct PairFTParams {
  const Shell *ao;
  const double *ao_exp, *ao_coef;
  const Pair *pairs;
  const int32_t *plist;   // pair indices grouped by (l(sa), l(sb)): d-d, d-p, d-s, p-p, p-s, s-s
  int32_t pgrp[7];        // plist offsets of the six groups (host-side launch split)
  const int32_t *cls_off;
  const double *img;
  const double *q;        // [nq][3] chunk, all q = G + k_cls of one class
  const double *amax;     // [nq] max_P |A[P][q]|
  int32_t npair, nq, nao, nk;
  int32_t kn[3];          // k-mesh (BvK class arithmetic)
  int32_t kcls[3];        // mesh coordinates j_d of k_cls
  double eps;             // skip terms whose weighted bound is below this
  double *B;              // complex I[Nk BvK classes][nao][nao][nq]
  long long *nterm;       // running count of transform evaluations
  double acut;            // primitive-pair selection (pmode) by exponents
  int32_t pmode;          // 0 every pair, 1 not both below acut, 2 both below acut
  int32_t pad2;
};

// leading q columns of each k12 class (the smallest |q|) that the reduced-precision
// contraction forms take in FP64
constexpr int kLrNqHi = 32;

struct LRGemmParams {
  const double *A;        // complex, row P has stride lda (complex elements); columns q0.. of the class
  int64_t lda;
  const double *B;        // complex [nkpi][nmn][nq] (mode 0)
  const float *A32;       // FP32 copy of A, same layout (modes 1, 2)
  const float *B32;       // complex FP32 [nkpi][nmn][nq] (modes 1, 2)
  const double *Bhi;      // complex FP64 [nkpi][nmn][nq_hi]: the FP64 columns of modes 1, 2
  double *out;            // complex [nkp][naux][nmn]
  const int32_t *kp_of;   // [nkpi] global k-pair index
  int64_t plane;          // naux * nmn
  int32_t naux, nq, nmn;
  int32_t nq_hi;          // leading q columns taken in FP64 by the reduced-precision forms
  // mode 2: operands split into FP16 planes in blocks of 32 q (see lr.hip)
  const uint16_t *Xa;     // [nb][naux][4][32]
  const int32_t *Ea;      // [nb][naux] block exponents of Xa
  const uint16_t *Xb;     // [nkpi][nb][nmn][4][32]
  const int32_t *Eb;      // [nkpi][nb][nmn]
  int32_t nb;             // 32-q blocks of the launch, ceil(nq / 32)
};

// two-center metric (j2c.hip): one (P shell, Q shell) pair of an angular class
struct J2Pair {
  int32_t P, Q;
  double rmax;            // short-range screening radius on |C_P - B_Q - m|
};

struct J2Params {
  const Shell *ax;
  const double *ax_exp, *ax_coef;
  const J2Pair *pairs;
  Lattice lat;
  double omega;
  const double *boys;     // Boys polynomial table [L][interval][degree + 1] (global memory)
  double *X2;             // real [nk][naux][naux] per BvK cell of m
  long long *nterm;       // evaluated (P prim, Q prim, m) terms
  int32_t naux, pad;
};

hipError_t launch_sr3c(int lP, int pc, const SRParams *prms, const SRWork *works, long long *counts, int w0,
                       int nwork, hipStream_t stream);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream);
hipError_t launch_sr_reduce(const SRParams &prm, const SRPartGroup *groups, int ngroups, int64_t nelem,
                            hipStream_t stream);
hipError_t launch_fold(const FoldParams &fp, hipStream_t stream);
hipError_t launch_overlaps(const OvlParams &op, const SmnParams &sp, hipStream_t stream);
hipError_t launch_auxft(const AuxFTParams &ap, hipStream_t stream);
hipError_t launch_lr_gemm_tiled(int mode, const LRGemmParams &gp, int q_lo, int nkpi, hipStream_t stream);
hipError_t launch_pairft_binned(const PairFTParams &pp, hipStream_t stream);
hipError_t launch_amax(const double *A, int64_t lda, int naux, int nq, double *amax, hipStream_t stream);
// k-pairs summed per pass of the k2-phase kernels for a class of nkpi k-pairs
// (passes of equal width, at most 28; a class of up to 28 takes one pass of
// exactly nkpi), and the k-pair stride of their phase table:
// phase[c][k] = e^{+i k2(k).L_c}, zero for k >= nkpi
constexpr int kKphKbMax = 28;
__host__ __device__ inline int kphase_kb(int nkpi) {
  const int npass = (nkpi + kKphKbMax - 1) / kKphKbMax;
  return (nkpi + npass - 1) / npass;
}
__host__ __device__ inline int kphase_kpad(int nkpi) {
  const int kb = kphase_kb(nkpi);
  return (nkpi + kb - 1) / kb * kb;
}
hipError_t launch_kphase(const double *I, const double *phase, void *B, bool f32, double *Bhi, int nq_hi, int nk,
                         int nkpi, int nq, int64_t nmn, hipStream_t stream);
hipError_t launch_to_f32(const double *x, float *y, int64_t n, hipStream_t stream);
// split FP16 operand formats of the mode-2 contraction (lr.hip)
constexpr int kF16Blk = 32;  // q per block (one matrix-core K step)
constexpr int kF16Grp = 2;   // blocks sharing one exponent (64 q: one wavefront of the producers)
static_assert(kLrNqHi % kF16Blk == 0, "the FP64 columns end on a split block boundary");
// blocks of the split format of nq columns: whole exponent groups (zero padded)
inline int f16_nblk(int64_t nq) {
  return (int)((nq + kF16Blk * kF16Grp - 1) / (kF16Blk * kF16Grp) * kF16Grp);
}
// byte offset of the exponents [nb][rows] behind the halves [nb][rows][4][32]
inline int64_t f16_split_eoff(int64_t rows, int64_t nb) { return (rows * nb * 4 * kF16Blk * 2 + 255) / 256 * 256; }
// bytes of the split format of rows x nq
inline int64_t f16_split_bytes(int64_t rows, int64_t nq) {
  const int64_t nb = f16_nblk(nq);
  return f16_split_eoff(rows, nb) + rows * nb * 4;
}
// q_excl: columns q < q_excl (contracted in FP64) do not enter the exponents
hipError_t launch_asplit(const double *A, int64_t lda, int naux, int nq, int q_excl, uint16_t *Xa, int32_t *Ea,
                         hipStream_t stream);
hipError_t launch_kphase_split(const double *I, const double *phase, uint16_t *Xb, int32_t *Eb, double *Bhi,
                               int nq_hi, int nk, int nkpi, int nq, int64_t nmn, hipStream_t stream);

// two-center metric (j2c.hip) and the density-fitting solve (df.hip)
hipError_t launch_j2c_sr(int lP, int lQ, const J2Params &jp, int p0, int npair, hipStream_t stream);
hipError_t launch_j2c_fold(const double *X2, const double *kph, const double *SP, double g0fac, int nk, int naux,
                           double *J, hipStream_t stream);
hipError_t launch_j2c_lr_operand(const double *A, int64_t lda, const double *q, int nq, int naux, double wfac,
                                 double omega, double *B, hipStream_t stream);
hipError_t launch_df_factor(const double *J, double *L, double *W, int *bad, int nk, int n, hipStream_t stream);
hipError_t launch_df_gemm(bool conjt, const double *W, const int32_t *cls, const double *V, double *D, int naux,
                          int64_t ncol, int nkp, hipStream_t stream);

// integral-direct density-fitted Coulomb build (coulomb.hip)
hipError_t launch_dm_contract(const double *V, const double *D, int nk, int ng, int nao, double *rho,
                              hipStream_t stream);
hipError_t launch_vj_accum(const double *V, const double *c, int nk, int ng, int64_t ne, double scale, double *vj,
                           hipStream_t stream);

// learned screening (learned.hip)
hipError_t launch_features(const SRParams &prm, int ntrip, const int64_t *idx, int64_t n, float *feat,
                           hipStream_t stream);
hipError_t launch_log_target(const float *logmag, int nk, int64_t ncand, float floor_, float *tgt,
                             hipStream_t stream);
hipError_t launch_mlp_step(float *params, const float *X, const float *y, const int64_t *idx, int64_t nb,
                           float kappa, float *gpart, float *lpart, float *grad, float *m, float *v, float lr, int step,
                           hipStream_t stream);
hipError_t launch_mlp_mask(const SRParams &prm, int ntrip, int64_t ncand, const float *params, float cut,
                           uint8_t *mask, long long *nskip, hipStream_t stream);
hipError_t launch_mlp_predict(const float *params, const float *X, int64_t n, int mode, float *pred,
                              hipStream_t stream);

}  // namespace rsgdf
