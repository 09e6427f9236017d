/*
 * rsgdf.h -- C ABI of the MI355X (gfx950) range-separated Gaussian density
 * fitting three-center integral library (librsgdf.so).
 *
 * Computes the periodic three-center Coulomb metric integrals
 *     V_{P mu nu}^{k1 k2} = (chi_P^{k12 *} | 1/r | rho_{mu nu}^{k1 k2})
 * of Eq. (M6) of Ye & Berkelbach, "Fast periodic Gaussian density fitting by
 * range separation" (arXiv 2102.02989), with the G = 0 (q = 0) component
 * removed as in Eq. (M10), by splitting 1/r into erfc(w r)/r + erf(w r)/r
 * (Eq. M9):
 *   short range : real-space double lattice sum, Eqs. (M12), (M13a), folded
 *                 to k-point pairs through Born-von Karman cells (Eq. M14),
 *                 screened with the bounds of the Supplementary Material
 *                 (Eqs. S14, S23-S27), minus the G = 0 term of Eq. (M12);
 *   long range  : reciprocal-space sum of Eq. (M10) over q = G + k12 with
 *                 exp(-|q|^2/4w^2) >= g_thresh, using analytic Fourier
 *                 transforms of the AO pair densities (Eq. M11).
 *
 * Units: bohr and hartree atomic units.  All arrays are row-major.
 *
 * Conventions
 *   - Bloch functions phi^k(r) = sum_m e^{i k.m} phi(r - m) (Eq. M1).
 *   - k-mesh: Gamma-centred k_j = sum_i (j_i / n_i) b_i, B = 2 pi A^{-T},
 *     linear index j = (j1 n2 + j2) n3 + j3.
 *   - k-pairs: only k1 <= k2, in row-major upper-triangle order
 *     (for k1 in 0..Nk-1, for k2 in k1..Nk-1).  The other half follows from
 *     V_{P nu mu}^{k2 k1} = conj(V_{P mu nu}^{k1 k2}).
 *   - Functions follow shell order; Cartesian components within a shell are
 *     x-power descending, then y-power descending (xx, xy, xz, yy, yz, zz).
 *   - Coefficients multiply bare Cartesian monomials
 *     (x-Ax)^i (y-Ay)^j (z-Az)^k exp(-a |r-A|^2); normalisation is the
 *     caller's choice.
 *   - Output: complex128, layout [nkpair][naux][nao][nao], interleaved
 *     (re, im) doubles.
 *
 * Ownership: every input is read-only and may be freed after the call
 * returns.  The output buffer is owned by the caller.  The library allocates
 * its device scratch during the call and frees it before returning.
 *
 * Errors: functions return RSGDF_OK (0) or a negative code; the message of the
 * last error on the calling thread is returned by rsgdf_last_error().
 */
#ifndef RSGDF_H
#define RSGDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSGDF_OK 0
#define RSGDF_EINVAL (-1)      /* invalid argument (shapes, l, exponents, mesh, omega, thresh, NaN) */
#define RSGDF_ESIZE (-2)       /* output capacity smaller than rsgdf_j3c_nbytes(); nothing written  */
#define RSGDF_ENOMEM (-3)      /* device scratch allocation failed                                  */
#define RSGDF_EHIP (-4)        /* HIP runtime error; output contents undefined                      */
#define RSGDF_EUNSUPPORTED (-5) /* valid request outside what this build implements                 */

/* maximum angular momenta of this build */
#define RSGDF_MAX_L_AO 2
#define RSGDF_MAX_L_AUX 3

/* long-range G-space contraction precision (Eq. M10's q sum as a complex
 * matrix product per k12 class).  In every form the transforms, the kernel
 * weight, the Bloch phases and the output are FP64; the reduced forms take
 * the 32 smallest-|q| vectors of each class in FP64 and add each 16-q FP32
 * partial (64 q in the F16X3 form) into FP64 registers. */
#define RSGDF_FP64 0   /* plain: FP64 matrix-core products                          */
#define RSGDF_FP32 1   /* operands rounded to FP32, FP32 matrix-core products        */
#define RSGDF_F16X3 2  /* operands scaled per row by 2^e, split hi + lo in FP16,
                          three FP16 products                                     */

/* short-range image screening */
#define RSGDF_SCREEN_RIGOROUS 0 /* Supplementary-Material bounds (Eqs. S14, S23-S27) */
#define RSGDF_SCREEN_LEARNED 1  /* MLP predictor with the rigorous bound as fallback  */

/* parts bit mask (for phase-by-phase checks; the default computes all) */
#define RSGDF_PART_SR 1 /* real-space erfc lattice sum, folded                     */
#define RSGDF_PART_G0 2 /* minus pi/(Omega w^2) S_P S_{mu nu}(k) on k1 == k2       */
#define RSGDF_PART_LR 4 /* reciprocal-space erf part                               */
#define RSGDF_PART_ALL 7

typedef struct {
  double lattice[9];     /* rows a1, a2, a3 (bohr); |det| > 0                       */
  int32_t natm;          /* >= 1                                                     */
  const double *coords;  /* host, [natm][3] (bohr)                                   */
} rsgdf_cell;

typedef struct {
  int32_t nshell;              /* >= 1                                                 */
  const int32_t *shell_atom;   /* host, [nshell], 0 <= atom < natm                     */
  const int32_t *shell_l;      /* host, [nshell], 0..RSGDF_MAX_L_AO / _AUX             */
  const int32_t *shell_nprim;  /* host, [nshell], 1..16                                */
  const int32_t *shell_ptr;    /* host, [nshell], offset of the shell's primitives     */
  const double *exps;          /* host, exponents > 0                                  */
  const double *coefs;         /* host, raw contraction coefficients                   */
} rsgdf_basis;

typedef struct {
  double g_thresh;       /* keep q with exp(-|q|^2/4w^2) >= g_thresh; <= 0 -> 1e-2*thresh   */
  int32_t lr_precision;  /* RSGDF_FP64 | RSGDF_FP32 | RSGDF_F16X3                           */
  int32_t screening;     /* RSGDF_SCREEN_RIGOROUS | RSGDF_SCREEN_LEARNED                    */
  int32_t parts;         /* RSGDF_PART_* mask; 0 -> RSGDF_PART_ALL                          */
  int32_t sr_slices;     /* lanes cooperating on one (k-cell pair) unit; 0 -> automatic     */
  const float *mlp_weights; /* host, RSGDF_MLP_NPARAM floats (layout below), or NULL        */
  double mlp_margin;     /* log10 margin added to the learned prediction                    */
  const float *sr_split; /* host [24] per-class work-split factors (rsgdf_autotune_sr), or NULL;
                            class g = 6 l_P + pair class of (l_a, l_b) in order ss, ps, pp, ds,
                            dp, dd                                                            */
  double alpha_cut;      /* compact/diffuse split (the paper's Fig. 1), 0 = off.  Primitives with
                            exponent < alpha_cut are diffuse; a primitive triple with a diffuse aux
                            primitive or two diffuse AO primitives is evaluated by the
                            range-separation-free reciprocal sum of Eq. M15 (weight 4 pi/(Omega q^2),
                            q^2 <= 4 alpha_cut ln(1/g_thresh) for a diffuse aux primitive, twice
                            that for a compact one with two diffuse AO primitives); the others are
                            range-separated.                                                      */
} rsgdf_options;

typedef struct rsgdf_stats {
  double t_plan_ms;      /* host planning (basis packing, screening bounds, image lists)   */
  double t_sr_ms;        /* short-range lattice-sum kernels                                 */
  double t_fold_ms;      /* Bloch fold + G = 0 correction                                   */
  double t_lr_ms;        /* aux and pair transforms + G-space contraction                   */
  double t_total_ms;     /* wall time of the call                                           */
  int64_t n_sr_terms;    /* evaluated (aux prim, AO prim a, AO prim b, image pair) tuples   */
  int64_t n_sr_shell_terms; /* kept (aux shell, AO shell pair, image pair) terms            */
  int64_t n_sr_candidates;  /* image pairs tested by the screening                          */
  int64_t n_lr_terms;    /* (primitive pair, image, q) transform evaluations                */
  int64_t n_g_total;     /* q vectors summed over the folded k12 classes                    */
  int64_t n_triplets;    /* (aux shell, AO shell pair) work items                           */
  int64_t n_aux_batches; /* aux-shell batches used to bound scratch memory                  */
  int64_t bytes_out;     /* output bytes written                                            */
  double sr_flops;       /* algorithmic FP64 operations of the SR kernels (static counts):  the
                            image loop's per-term count times the evaluated terms, plus the
                            Hermite contraction's count per (pair image, primitive triple, BvK
                            cell group) times the contractions performed                    */
  double t_lr_gemm_ms;   /* G-space contraction kernels alone                               */
  int64_t n_screen_candidates; /* (aux shell, AO pair, pair image) candidates (learned mode) */
  int64_t n_screen_skipped;    /* candidates the network dropped                            */
  double lr_gemm_flops;  /* 8 naux N_q n_AO^2 per k-pair (real operations of complex MACs)  */
} rsgdf_stats;

typedef struct {
  void *data;              /* complex128 [nkpair][naux][nao][nao]                           */
  int64_t capacity_bytes;  /* size of data in bytes                                         */
  int32_t on_device;       /* 1: data is device memory on the current HIP device;
                              0: host memory (the call stages through a device buffer)    */
  void *stream;            /* hipStream_t to run on, or NULL for the null stream           */
  int64_t nkpair, naux, nao; /* filled on success                                          */
  rsgdf_stats *stats;      /* optional, filled on success                                   */
} rsgdf_out;

/* Bytes needed for the output of rsgdf_build_j3c; < 0 on invalid input. */
int64_t rsgdf_j3c_nbytes(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                         const int32_t kmesh[3]);

/* V_{P mu nu}^{k1 k2} for all k1 <= k2 (Eq. M6 with the G = 0 term removed),
 * FP64, rigorous screening at precision thresh (Eqs. S14, S23-S27), with
 * g_thresh = 1e-2 * thresh.  Synchronous on out->stream.
 * omega > 0 (bohr^-1) is the range-separation parameter of Eq. (M9). */
int rsgdf_build_j3c(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                    const int32_t kmesh[3], double omega, double thresh, rsgdf_out *out);

/* As rsgdf_build_j3c with explicit options (NULL = defaults).  Returns
 * RSGDF_EINVAL for an unknown lr_precision and RSGDF_EUNSUPPORTED for
 * screening = RSGDF_SCREEN_LEARNED without usable mlp_weights. */
int rsgdf_build_j3c_ex(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                       const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                       rsgdf_out *out);

/* ---- density fitting: the two-center metric and the fitting solve.
 *
 * J^k_PQ = (chi_P^{k*} | 1/r | chi_Q^k) = sum_m e^{+i k.m} (P^0 | 1/r | Q^m)
 * (Eq. M5) with the q = 0 (G = 0 at k = 0) component removed, for every k of
 * the Gamma-centred mesh (index j = (j1 n2 + j2) n3 + j3), evaluated with the
 * range separation of Eq. M9 as the three-center integrals are: an erfc
 * lattice sum (screened at 1e-2 thresh, Eq. S14's bound with one AO factor
 * replaced by the aux function), minus pi/(Omega w^2) S_P S_Q at k = 0, plus
 * (4 pi/Omega) sum_{q=G+k, q!=0, exp(-q^2/4w^2) >= g_thresh} exp(-q^2/4w^2)/q^2
 * chi~_P(-q) chi~_Q(q) (Eq. M10) on the FP64 matrix cores.  J^{k12} is the
 * metric that Eq. M4 pairs with V^{k1k2} (k12 = k2 - k1 folded onto the mesh).
 * Output: complex128 [nk][naux][naux] (out->on_device as for the three-center
 * build; out->nkpair = nk and out->naux = out->nao = naux on return).  opt
 * (may be NULL): g_thresh and parts are used.  stats: t_sr_ms (short range and
 * fold), t_lr_ms, n_sr_terms (evaluated (P prim, Q prim, m) terms),
 * n_g_total, lr_gemm_flops. */
int64_t rsgdf_j2c_nbytes(const rsgdf_cell *cell, const rsgdf_basis *auxbasis, const int32_t kmesh[3]);
int rsgdf_build_j2c(const rsgdf_cell *cell, const rsgdf_basis *auxbasis, const int32_t kmesh[3], double omega,
                    double thresh, const rsgdf_options *opt, rsgdf_out *out);

/* The fitting coefficients of Eq. M4: for every k-pair (k1 <= k2, row-major)
 *     sum_Q J^{k12}_PQ d^{k1k2}_{Q,c} = V^{k1k2}_{P,c},   c = 0..ncol-1,
 * by a Cholesky factorisation J = L L^H per k, W = L^{-1} and J^{-1} = W^H W
 * (FP64 vector ALUs), then d = J^{-1} V on the FP64 matrix cores.
 *   j2c: device complex128 [nk][naux][naux] (rsgdf_build_j2c; the lower
 *        triangle of each J^k is read);
 *   j3c: device complex128 [nkpair][naux][ncol] (rsgdf_build_j3c output:
 *        ncol = nao * nao);
 *   d:   device complex128, same shape as j3c; may be j3c itself (then the
 *        result goes through a bounded device temporary).
 * Returns RSGDF_EINVAL if a J^k is not numerically positive definite (its
 * k index is named in the message; d is then untouched).  Synchronous on
 * stream (hipStream_t or NULL). */
int rsgdf_df_solve(const int32_t kmesh[3], int64_t naux, int64_t ncol, const void *j2c, const void *j3c, void *d,
                   void *stream);

/* Integral-direct density-fitted Coulomb matrix: a consumer of the
 * three-center integrals that never stores them (the paper's outlook of
 * integral-direct algorithms).  For densities D^k (device complex128
 * [nk][nao][nao], Hermitian per k):
 *   J_{mu nu}(k) = (1/Nk) sum_{k', lambda sigma} (rho^{kk}_{mu nu} | rho^{k'k'}_{lambda sigma})
 *                  D^{k'}_{sigma lambda}
 * with the ERIs of Eq. M7 (d = (J^0)^{-1} V, Eq. M4 at k12 = 0):
 *   rho_Q = sum_k sum_{lambda sigma} V^{kk}_{Q lambda sigma} D^k_{sigma lambda};  J^0 c = rho;
 *   J_{mu nu}(k) = (1/Nk) sum_Q V^{kk}_{Q mu nu} c_Q.
 * The k1 = k2 blocks of V are built per group of aux shells (aux_group
 * shells per group, 0: groups sized to 10% of free device memory, at most
 * 8 GB), contracted and dropped; the second pass rebuilds them.  vj: device
 * complex128 [nk][nao][nao] (overwritten).  opt as for rsgdf_build_j3c_ex
 * (parts must be all).  RSGDF_EINVAL if J^0 is numerically singular.
 * stats (optional): phase times and counts summed over both passes,
 * n_aux_batches = tiles built. */
int rsgdf_coulomb_direct(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                         const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                         int32_t aux_group, const void *dm, void *vj, void *stream, rsgdf_stats *stats);

/* ---- automatic choice of the range-separation parameter.  The paper picks
 * omega (and with it the number of plane waves of the long-range part) by
 * hand; here every omega screened at the same thresh and g_thresh meets the
 * same precision, so the choice is the fastest one, predicted by a cost model
 * linear in work features that the host planner computes without device work:
 *   feat[0] short-range operations (the planner's per-item cost estimate),
 *   feat[1] pair-transform candidates (q x primitive pairs x images x
 *           Cartesian components), feat[2] contraction flops, feat[3] k2-phase
 *           elements, feat[4] output elements, feat[5] short-range
 *           intermediate elements, feat[6] q vectors, feat[7] short-range
 *           primitive terms (estimate), feat[8] = 1 (fixed cost per build).
 * rsgdf_plan_features fills feat for one omega; rsgdf_choose_omega returns
 * the candidate with the smallest sum_i coef[i] feat[i] (ms), and the
 * predictions if predicted_ms (nomega doubles) is not NULL.  The coefficients
 * are fitted to measured MI355X builds (the package's cost-model file). */
#define RSGDF_NFEATURES 9
int rsgdf_plan_features(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                        const int32_t kmesh[3], double omega, double thresh, double g_thresh,
                        double feat[RSGDF_NFEATURES]);
int rsgdf_choose_omega(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                       const int32_t kmesh[3], double thresh, double g_thresh, const double *omegas, int32_t nomega,
                       const double coef[RSGDF_NFEATURES], double *best_omega, double *predicted_ms);
/* The same with the compact/diffuse split (Fig. 1, Eq. M15; options.alpha_cut):
 * rsgdf_plan_features_acut fills feat for one (omega, alpha_cut), alpha_cut = 0
 * meaning no split (then it equals rsgdf_plan_features).  With the split the
 * short-range features count only compact aux primitives and primitive pairs
 * not both diffuse, and the long-range ones add the two Eq. M15 parts on their
 * q spheres (q^2 <= 4 alpha_cut ln(1/g_thresh) for the diffuse aux primitives,
 * twice that for the diffuse-diffuse pairs).  The split changes no result
 * beyond the screening thresholds, so rsgdf_choose_params returns the grid point
 * (omegas[i], acuts[j]) with the smallest predicted time, and the predictions
 * predicted_ms[i * nacut + j] if not NULL.  RSGDF_EINVAL for null arguments,
 * empty grids, omega <= 0 or alpha_cut < 0. */
int rsgdf_plan_features_acut(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                             const int32_t kmesh[3], double omega, double alpha_cut, double thresh, double g_thresh,
                             double feat[RSGDF_NFEATURES]);
int rsgdf_choose_params(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                        const int32_t kmesh[3], double thresh, double g_thresh, const double *omegas, int32_t nomega,
                        const double *acuts, int32_t nacut, const double coef[RSGDF_NFEATURES], double *best_omega,
                        double *best_acut, double *predicted_ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * build as rsgdf_build_j3c_ex with every device scratch buffer (tables, the
 * short-range intermediate, the long-range operands, counters) carved from
 * one static device array of RSGDF_NOALLOC_SCRATCH_MB MiB that the library
 * holds per GPU until the process ends.  The call allocates no device memory
 * (no hipMalloc / hipFree / allocating library routine), creates no streams
 * or events, and runs every kernel on out->stream; aux-shell batching keeps
 * the short-range intermediate within the buffer.  out must be device memory
 * (out->on_device = 1).  Returns RSGDF_ENOMEM, with a message naming the
 * limit, when the build needs more scratch than the buffer holds (nothing is
 * written to the output then).  All calls on one GPU share its buffer: calls
 * from one process are serialised by the library; calls that overlap on one
 * GPU from separate processes, or kernels still reading the buffer, race.
 * The buffer keeps the last call's contents; every part that must start at
 * zero is cleared by a kernel at the start of each call.  Synchronous on
 * out->stream.  stats: phase times are not measured (t_total_ms is). */
#define RSGDF_NOALLOC_SCRATCH_MB 256
int rsgdf_build_j3c_noalloc(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                            const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                            rsgdf_out *out);

/* ---- learned screening (a project addition to the Supplementary-Material
 * bounds).  A candidate is one (aux shell, AO shell pair, pair image n') unit
 * of the short-range lattice sum that passed the rigorous test of Eqs.
 * S23-S27.  Its target is log10 of the sum over BvK cells c1 of max |block|
 * it adds to the short-range intermediate (an upper bound of its effect on
 * any output element), floored at log10(thresh) - 4.  Features (16 floats, raw): log10 beta_d, log10 p_d,
 * log10 alpha_P (most diffuse primitives), R12 = |A - B - n'|, R_c,min (pair
 * centre to the nearest aux image), l_a, l_b, l_P, log10 A (1s-model
 * amplitude, Eq. S4), log10 omega, log10 of the 1s estimate at R_c,min
 * (Eqs. S4-S9), then five zeros.
 *
 * Network parameters: RSGDF_MLP_NPARAM floats, in order: feature mean [16],
 * 1/std [16], W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1],
 * training-range lower bounds [16], upper bounds [16].  ReLU hidden layers. */
#define RSGDF_MLP_NFEAT 16
#define RSGDF_MLP_NPARAM 5377

/* Run the plain short-range sum with magnitude logging (no output is
 * written) and return a seeded sample (fraction sample_frac in (0, 1]) of
 * the candidates with their features and targets, host arrays feat
 * [n][16] and target [n].  *n_out is always set; RSGDF_ESIZE (nothing
 * copied) if it exceeds capacity.  stream: hipStream_t or NULL. */
int rsgdf_screen_log(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                     const int32_t kmesh[3], double omega, double thresh, double sample_frac, uint64_t seed,
                     float *feat, float *target, int64_t capacity, int64_t *n_out, void *stream);

/* Train the network on the GPU (FP32 forward/backward kernels, Adam with
 * step size lr, mini-batches of `batch`, seeded shuffles).  Loss: mean of
 * w (pred - y)^2 with w = kappa (>= 1) for under-predictions, 1 otherwise.
 * init != 0 first sets the standardisation and training range from X and
 * draws He-initialised weights from seed.  params is read and written (host,
 * RSGDF_MLP_NPARAM floats); loss_history (host, epochs floats) or NULL
 * receives the full-data loss after each epoch. */
int rsgdf_mlp_train(float *params, const float *X, const float *y, int64_t n, int32_t epochs, int32_t batch,
                    float lr, float kappa, uint64_t seed, int32_t init, float *loss_history, void *stream);

/* Loss and its gradient with respect to W1 .. b3 (5313 floats, parameter
 * order) over all n samples, from the training kernels. */
int rsgdf_mlp_grad(const float *params, const float *X, const float *y, int64_t n, float kappa, float *grad,
                   float *loss, void *stream);

/* Predictions for n raw feature rows: mode 0 FP32 vector ALUs, mode 1 the
 * FP16 matrix-core path used by the keep mask. */
int rsgdf_mlp_predict(const float *params, const float *X, int64_t n, int32_t mode, float *pred, void *stream);

/* Margin = the `quantile` quantile (1 = max) of y - prediction (mode 1) over
 * the given samples, floored at 0. */
int rsgdf_mlp_margin(const float *params, const float *X, const float *y, int64_t n, double quantile,
                     double *margin, void *stream);

/* ---- batches of cells (a project addition).  All cells share omega, thresh
 * and options; each has its own output (device memory, all on outs[0].stream).
 * The short-range work items of all cells are merged into one launch per
 * angular-momentum class; the whole device sequence is captured once into a
 * HIP graph.  create: plans, allocates and captures (ENOMEM/EUNSUPPORTED if a
 * cell would need aux-shell batching); run: replays the graph, fills each
 * out's results and stats (t_total_ms = the whole batch); destroy frees. */
typedef struct rsgdf_batch rsgdf_batch;
int rsgdf_batch_create(int32_t ncell, const rsgdf_cell *cells, const rsgdf_basis *bases, const rsgdf_basis *auxes,
                       const int32_t (*kmeshes)[3], double omega, double thresh, const rsgdf_options *opt,
                       rsgdf_out *outs, rsgdf_batch **batch);
int rsgdf_batch_run(rsgdf_batch *batch);
void rsgdf_batch_destroy(rsgdf_batch *batch);
/* create + run + destroy */
int rsgdf_build_j3c_batch(int32_t ncell, const rsgdf_cell *cells, const rsgdf_basis *bases, const rsgdf_basis *auxes,
                          const int32_t (*kmeshes)[3], double omega, double thresh, const rsgdf_options *opt,
                          rsgdf_out *outs);

/* Autotuner of the short-range work split: times every class of the given
 * cell's short-range sum at uniform split factors {1/4, 1/2, 1, 2, 4} (the
 * target work per wavefront relative to the default) and writes the fastest
 * factor per class to split[24] (and its time in ms to class_ms[24] if not
 * NULL), for rsgdf_options.sr_split. */
int rsgdf_autotune_sr(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                      const int32_t kmesh[3], double omega, double thresh, float *split, double *class_ms,
                      void *stream);

/* Device memory cache (a project addition).  The large scratch buffers of a
 * build (64 MB and more: the short-range bins, the fold intermediate, the
 * long-range q-chunk operands) are not freed when it returns but kept idle
 * for the next build on the same device, which reuses a block that holds its
 * request and wastes at most a quarter of it; idle blocks beyond 40% of the
 * device's memory are freed at once, and all idle blocks of a device when an
 * allocation there fails.  The scratch budgets count idle blocks as free
 * memory, so a build plans the same with or without them.  This call frees
 * every idle block (blocks of builds still running are not affected; do not
 * call it concurrently with a build that is returning).  Returns RSGDF_OK or
 * RSGDF_EHIP. */
int rsgdf_release_cache(void);

/* Message of the last error on this thread ("" if none). */
const char *rsgdf_last_error(void);

/* Library version string. */
const char *rsgdf_version(void);

/* Hash of the sources the library was built from (16 hex digits: SHA-256
 * over the files of csrc/ and include/, by name and content), or "unknown"
 * for a build outside the package's build script.  The Python binding
 * compares it with the sources on disk and refuses a stale library.  Static
 * string, owned by the library. */
const char *rsgdf_source_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* RSGDF_H */
