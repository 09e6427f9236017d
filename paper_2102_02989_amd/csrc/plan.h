// plan.h -- data shared between the host planner and the gfx950 kernels.
//
// Everything here is plain-old-data copied to the device once per call:
// packed shells and primitives, AO shell pairs with their lattice-image
// lists (grouped by Born-von Karman class), (aux shell, AO pair) work items
// with their screening radii, and the G-vector sets of the long-range part.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsgdf {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kMaxLAO = 2;
constexpr int kMaxLAux = 3;
constexpr int kMaxL = 2 * kMaxLAO + kMaxLAux;  // 7
constexpr int kMaxWin = 512;                   // SR screening windows of width dR
constexpr double kBoysSwitch = 36.0;           // polynomial table below, asymptotic recursion above
constexpr int kBoysIntervals = 36;             // unit intervals of T in [0, 36)
constexpr int kBoysPolyDeg = 12;               // Taylor degree about each interval centre

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Angular growth of an AO pair factor in the screening windows (Eqs.
// S23-S25): the 1s model e^{-beta R12^2} of a pair with l_a + l_b > 0 is
// multiplied by (1 + c R12)^{l_a + l_b} with c = sqrt(2 beta).  The pair
// density's polynomial prefactor (x-A)^{i}(x-B)^{j} about the product centre
// grows like (|PA| / w)^i (|PB| / w)^j in units of the primitive width w
// that the 1s-equivalent amplitude carries, and for equal exponents
// |PA| / w = |PB| / w = sqrt(2 beta) R12; the s-type model leaves it out.
__host__ __device__ inline double pair_growth_c(double beta) { return sqrt(2.0 * beta); }
__host__ __device__ constexpr int nherm(int l) { return (l + 1) * (l + 2) * (l + 3) / 6; }

// Work layout of the short-range kernels, shared with the planner's work split.
constexpr int kBlkCap = 1024;        // doubles of per-group Cartesian accumulators in LDS
constexpr int kMaxCellsPerWave = 8;  // BvK cells (lane groups) per wave
// cells per wave for which the Cartesian accumulators of a class fit in LDS
__host__ __device__ constexpr int sr_max_cells(int nblk) {
  return (kBlkCap / nblk) < 1 ? 1 : ((kBlkCap / nblk) > kMaxCellsPerWave ? kMaxCellsPerWave : kBlkCap / nblk);
}
inline int sr_cells_per_wave(int nblk) { return sr_max_cells(nblk); }
// AO pair class of (l_a, l_b), l_a >= l_b: 0 ss, 1 ps, 2 pp, 3 ds, 4 dp, 5 dd
inline int pair_class(int la, int lb) {
  static const int t[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
  return t[la][lb];
}

// Static FP64 operation count of the recursion of hermite_R_acc<L> (one multiply or add = 1).
__host__ __device__ constexpr int hermite_R_flops(int L) {
  int f = 0;
  for (int n = L - 1; n >= 0; --n)
    for (int s = L - n; s >= 1; --s)
      for (int t = s; t >= 0; --t)
        for (int u = s - t; u >= 0; --u) {
          const int v = s - t - u;
          int k = (t > 0) ? t : (u > 0 ? u : v);
          f += (k > 1) ? 3 : 1;
        }
  return f;
}

// Static per-term FP64 operation count of the image loop for class L:
// position and T (13) + attenuated Boys values (two degree-12 polynomials,
// two downward recursions, theta scaling) + (-2 rho)^n scaling (2L) +
// Hermite recursion + image accumulation (nherm(L)).  An exp counts as one.
inline int sr_term_flops(int L) {
  const int geo = 13;
  const int boys = 2 * (2 * kBoysPolyDeg + 3 * L + 1) + 3 * (L + 1);
  return geo + boys + 2 * L + hermite_R_flops(L) + nherm(L);
}

// Static FP64 operation count of the McMurchie-Davidson contraction of one
// (pair image, primitive triple, BvK cell group): the aux pass
// W[ic][tuv] = sum over the even aux Hermite orders of E^c_x E^c_y E^c_z R
// (NW = ncart(lP) nherm(la + lb) entries, (KX + 1)^3 products each, KX =
// lP / 2), then the pair pass, each Cartesian component (ncart of all three)
// summing E^ab_x E^ab_y E^ab_z W over the nherm(la + lb) Hermite orders,
// times the triple's prefactor.
inline int sr_contr_flops(int lP, int la, int lb) {
  const int lab = la + lb, kx = lP / 2 + 1;
  const int nw = ncart(lP) * nherm(lab);
  const int w = nw * (2 * kx * kx * kx + 3 * kx * kx);
  const int nblk = ncart(lP) * ncart(la) * ncart(lb);
  const int c = nblk * (2 * nherm(lab) + (lab + 1) * (lab + 2) + 2 * (lab + 1) + 1);
  return w + c;
}

// Packed shell (AO or aux).  a_d, c_d: exponent and 1s-equivalent amplitude
// of the most diffuse primitive (used by the screening bounds, which treat
// every function as 1s and a contracted shell by its most diffuse primitive).
struct Shell {
  double x, y, z;
  double a_d, c_d;
  int32_t l, nprim, pptr, foff;
};

// AO shell pair, oriented so that l(sa) >= l(sb).  Images n' of shell sb are
// listed in img[img_off + cls_off[c] .. img_off + cls_off[c+1]) for each BvK
// class c of n', sorted by |A - B - n'| within a class.  nsr[c] is the count
// of leading images of class c inside the short-range R12 radius.
struct Pair {
  int32_t sa, sb, diag, pad;
  int32_t img_off;   // offset into the image-vector array
  int32_t cls_off;   // offset into the per-class offset array (Nk + 1 entries)
  int32_t nsr_off;   // offset into the per-class short-range count array (Nk entries)
  int32_t pad2;
  double beta_d;     // a_d(sa) a_d(sb) / (a_d(sa) + a_d(sb))
  double R12min;     // Eq. S25 crossing radius
  double R12sr;      // largest R12 any window of any aux shell can keep
};

// (aux shell, AO pair) short-range work item.
struct Triplet {
  int32_t aux, pair, nwin, pad;
  double rc_cut;     // Eq. S14 bound on R_c
  double amp;        // 1s-model amplitude A of Eq. S4 (primitive amplitudes summed)
};

// One wavefront's share of a work item of cell `cell`: BvK cells c1 in
// [cb0, cb0 + ncb) and pair images with list index = slice (mod nslice).  part >= 0: the wave
// writes its sums to a private partial block [ncb][Nk][nblk] at that offset
// (summed into X afterwards in a fixed order); part < 0: it adds into X.
struct SRWork {
  int32_t trip;
  int16_t cb0, ncb;
  int16_t slice, nslice;
  int32_t cell;      // index into the per-cell parameter table of the launch
  int64_t part;
};

// Partial blocks of one (work item, cell range) split over nslice waves.
struct SRPartGroup {
  int32_t trip, cb0, ncb, nslice;
  int64_t part;       // first slice's block (doubles)
  int64_t elem_off;   // prefix sum of ncb * Nk * nblk over groups
};

// Lattice and k-mesh constants.
struct Lattice {
  double a[9];       // rows a1, a2, a3
  double b[9];       // rows b1, b2, b3, a_i . b_j = 2 pi delta_ij
  double vol;
  int32_t n[3];      // k-mesh
  int32_t nk;
  int32_t pad;
};

struct SRParams {
  const Shell *ao;
  const Shell *ax;
  const double *ao_exp, *ao_coef;
  const double *ax_exp, *ax_coef;
  const double *ao_c1s, *ax_c1s;  // 1s-equivalent amplitudes per primitive (screening)
  const Pair *pairs;
  const int32_t *cls_off;   // per pair: Nk+1 offsets
  const int32_t *nsr;       // per pair: Nk counts
  const double *img;        // image vectors, 3 doubles each
  const Triplet *trip;
  double *part;             // partial blocks of split work items
  Lattice lat;
  double omega, eps, dR;
  double ncell_nf, ncell_r0;  // N_cell model of Eq. S19
  const double *boys;       // [L = 0..kMaxL][kBoysIntervals][kBoysPolyDeg + 1]
  double acut;              // > 0: compact/diffuse split (primitive triples with a diffuse aux
                            // primitive or two diffuse AO primitives are left to Eq. M15)
  double *X;                // [Nk][Nk][naux_b][nao][nao]
  int32_t aux_f0, naux_b, nao, pad;
  // learned screening: candidate (triplet, pair image ii) has index cand_off[trip] + ii
  const int64_t *cand_off;  // [ntrip] (null when neither mask nor logmag is used)
  const uint8_t *mask;      // keep flag per candidate, or null (rigorous screening only)
  float *logmag;            // magnitude log: [candidate][Nk] max |block| per BvK cell c1, or null
};

}  // namespace rsgdf
