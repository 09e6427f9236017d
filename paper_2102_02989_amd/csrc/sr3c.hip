// sr3c.hip -- short-range (erfc-attenuated) three-center lattice sums on gfx950.
//
// Work item: (aux shell P, AO shell pair); a wavefront takes a range of BvK
// cells c1 and an interleaved share of the pair images (SRWork).
// The term (P^0 | erfc(w r)/r | mu^m nu^{m+n'}) of Eq. (M12)/(M13a) is
// rewritten by translation as (P^{-m} | mu^0 nu^{n'}): for a pair image n' the
// AO pair density is fixed and the aux function moves over lattice vectors m.
// Terms are grouped by Born-von Karman cells (Eq. M14): c1 = c(m) and
// c2 = c(m + n').
//
// Lane layout: the 64 lanes form groups of gs lanes, group g owning BvK cell
// c1 = g.  For each pair image n' (taken in the pair list order, which is
// sorted by the BvK class of n', so the target (c1, c2) changes only with the
// class) the wave
//   1. enumerates the lattice vectors m of each cell inside the screening
//      radius and keeps those passing the per-term window test of the
//      Supplementary Material (R_c <= R_c^cut of Eq. S14 and R12 <= R12^cut(R_c)
//      of Eqs. S23-S25, most diffuse primitives as 1s functions); survivors are
//      compacted into per-group LDS lists with ballots (deterministic order);
//   2. for every primitive pair (and aux primitive) sums the Hermite Coulomb
//      integrals R_tuv of the erfc operator over the group's list (the only
//      m-dependent factor of the McMurchie-Davidson expression), reduces them
//      over the group's lanes in lane order (transposed through LDS), and
//      contracts them with the aux (E^c) and pair (E^ab) Hermite coefficients;
//   3. adds the Cartesian block into an LDS accumulator per group, flushed to
//      X[c1][c2][P][mu][nu] (or to the wave's partial block when the images
//      of the item are split over several waves) when the class of n' changes.
// Every X element (and every partial element) is owned by one wave and one
// group, so results are deterministic without atomics; split items are summed
// by sr_reduce_kernel in slice order.
#include <hip/hip_runtime.h>

#include "boys.h"
#include "device_math.h"
#include "kernels.h"
#include "plan.h"

namespace rsgdf {

constexpr int kCandCap = 1536;    // lattice-vector candidates held in LDS per wave
constexpr int kSRWinCap = 256;    // screening windows held in LDS
constexpr int kTripCap = 40;         // primitive triples whose constants are held in LDS
constexpr int kTripC = 9;            // constants per primitive triple

// Constants of a primitive triple (AO a, AO b, aux c) that do not depend on
// the pair image: t[0] 1/p, t[1] g_b/p (P = A + t[1] (B - A)), t[2] g_a g_b/p
// (K_ab = e^{-t[2] R12^2}), t[3] rho, t[4] theta^2, t[5] theta, t[6] the
// signed contraction prefactor c_c c_a c_b 2 pi^{5/2}/(p g_c sqrt(p + g_c)),
// t[7] the 1s screening estimate per unit K_ab and lattice vector
// (Eqs. S4-S9 with the erfc attenuation), t[8] 1/(2 g_c).
template <int LP>
__device__ __forceinline__ void triple_consts(double ga, double gb, double gc, double ca, double cb, double cc,
                                              double ca1, double cb1, double cc1, double omega, double acut,
                                              double *t) {
  const double p = ga + gb, oop = 1.0 / p;
  const double rpc = 1.0 / (p + gc);
  const double rho = p * gc * rpc;
  const double om2 = omega * omega;
  const double th2 = om2 / (om2 + rho);
  const double e1 = sqrt(rho);
  const double e2 = 1.0 / sqrt(1.0 / rho + 1.0 / om2);
  t[0] = oop;
  t[1] = gb * oop;
  t[2] = ga * gb * oop;
  t[3] = rho;
  t[4] = th2;
  t[5] = sqrt(th2);
  t[6] = ((LP & 1) ? -1.0 : 1.0) * cc * ca * cb * 2.0 * kPi * kPi * sqrt(kPi) * sqrt(rpc) / (p * gc);
  t[7] = kPi * kPi * kPi * cc1 * ca1 * cb1 / (gc * p * sqrt(gc * p)) * 2.0 * (e1 - e2) *
         0.564189583547756286948079451561;
  t[8] = 0.5 / gc;
  // compact/diffuse split: a diffuse aux primitive or two diffuse AO
  // primitives put the triple into the Eq. M15 part; a zero screening estimate
  // makes the image loop's primitive screen skip it
  if (acut > 0.0 && (gc < acut || (ga < acut && gb < acut))) {
    t[6] = 0.0;
    t[7] = 0.0;
  }
}


// (t,u,v) of Hermite index h (inverse of hidx)
__device__ __forceinline__ void herm_decode(int h, int &t, int &u, int &v) {
  int s = 0;
  while (nherm(s) <= h) ++s;
  const int rem = h - (s > 0 ? nherm(s - 1) : 0);
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= rem) ++r;
  v = rem - r * (r + 1) / 2;
  u = r - v;
  t = s - r;
}

// Cartesian powers of component i of angular momentum l
__device__ __forceinline__ void cart_decode(int l, int i, int &x, int &y, int &z) {
  int n = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      if (n == i) {
        x = lx;
        y = ly;
        z = l - lx - ly;
        return;
      }
      ++n;
    }
  x = y = z = 0;
}

__device__ __forceinline__ int pack3(int a, int b, int c) {
  return ((a + 512) & 1023) | (((b + 512) & 1023) << 10) | (((c + 512) & 1023) << 20);
}
__device__ __forceinline__ void unpack3(int v, int &a, int &b, int &c) {
  a = (v & 1023) - 512;
  b = ((v >> 10) & 1023) - 512;
  c = ((v >> 20) & 1023) - 512;
}

// waves per SIMD the class's register need allows (the image loop keeps the
// nherm(L) running sums and an nherm(L-1) recursion scratch live).  L = 4
// runs two waves with some spilling (its LDS allows six workgroups per CU):
// 2% faster on the 8-atom 2x2x2 workload than one wave.
__host__ __device__ constexpr int sr_waves(int L) { return L >= 5 ? 1 : 2; }

template <int LP, int LA, int LB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sr_waves(LP + LA + LB))))
void sr3c_kernel(const SRParams *__restrict__ prms, const SRWork *__restrict__ works, long long *__restrict__ counts,
                 const int w0) {
  constexpr int NCP = ncart(LP), NCA = ncart(LA), NCB = ncart(LB);
  constexpr int NBLK = NCP * NCA * NCB;
  constexpr int LAB = LA + LB, L = LAB + LP;
  constexpr int NH = nherm(L);
  constexpr int NHAB = nherm(LAB);
  constexpr int EA = (LA + 1) * (LB + 1) * (LAB + 1);
  constexpr int BLK = NBLK * sr_max_cells(NBLK);
  __shared__ float s_nf[kSRWinCap];
  __shared__ __attribute__((aligned(16))) double s_boys[kBoysIntervals * (kBoysPolyDeg + 2)];
  __shared__ int s_cand[kCandCap];
  __shared__ double s_blk[BLK];
  // contraction of all lane groups at once: W[g][ic][h] from the group sums
  // R[g][h'] through a table of Hermite indices (NH marks an invalid aux
  // order and reads the zero slot), then the components from W
  constexpr int CH = 7;                    // Hermite entries per step of the group reduction (an odd
                                           // row stride: the 64 lanes' rows start in distinct LDS banks)
  constexpr int KX = LP / 2;               // aux Hermite orders tau = (c & 1) + 2k, k <= KX
  constexpr int NK = (KX + 1) * (KX + 1) * (KX + 1);
  constexpr int NW = NCP * NHAB;           // W entries per group
  constexpr int MG = sr_max_cells(NBLK);   // groups per wave
  // The reduction scratch (lane x entry) and the W table of the contraction
  // share one buffer: within a primitive triple the reduction ends with a
  // barrier before W is written, and the comps pass ends with one before the
  // next triple's reduction writes its scratch.  (The classes with L >= 6
  // stay under 40 KB of LDS this way: four one-wave workgroups per CU.)
  constexpr int NTW = (64 * CH > MG * NW) ? 64 * CH : MG * NW;
  __shared__ double s_TW[NTW];
  double *const s_T = s_TW;
  double *const s_W = s_TW;
  __shared__ double s_R[MG * (NH + 1)];    // group sums (tetrahedral order) + a zero slot
  __shared__ int s_wtab[NW];               // W entry (ic, h): cx | cy << 2 | cz << 4
  __shared__ short s_widx[NW * NK];        // Hermite index of h + (tau nu phi), or NH
  __shared__ int s_ctab[NBLK];             // component: ic | (ax,bx) << 8 | (ay,by) << 16 | (az,bz) << 24
  __shared__ double s_E[3 * EA];
  __shared__ double s_EP[(LP + 1) * (LP + 1)];
  __shared__ double s_tc[kTripCap * kTripC];

  const int lane = threadIdx.x;
  const SRWork wk = works[w0 + blockIdx.x];
  const SRParams &prm = prms[wk.cell];
  const int S = wk.nslice;
  const int slice = wk.slice;
  const Triplet tr = prm.trip[wk.trip];
  const Shell shP = prm.ax[tr.aux];
  const Pair pr = prm.pairs[tr.pair];
  const Shell shA = prm.ao[pr.sa];
  const Shell shB = prm.ao[pr.sb];
  const Lattice &lat = prm.lat;
  const int nk = lat.nk;
  const double omega = prm.omega, eps = prm.eps, dR = prm.dR;
  const double fourpi_vol = 4.0 * kPi / lat.vol;

  // ---- per-item tables in LDS: Boys polynomials of order L, screening windows
  for (int i = lane; i < kBoysIntervals * (kBoysPolyDeg + 1); i += 64)
    s_boys[(i / (kBoysPolyDeg + 1)) * (kBoysPolyDeg + 2) + i % (kBoysPolyDeg + 1)] = prm.boys[L * kBoysIntervals * (kBoysPolyDeg + 1) + i];
  for (int i = lane; i < kBoysIntervals; i += 64) s_boys[i * (kBoysPolyDeg + 2) + kBoysPolyDeg + 1] = 0.0;
  const int nta = shA.nprim, ntb = shB.nprim, ntcp = shP.nprim;
  const int ntrip_p = nta * ntb * ntcp;
  const bool tc_lds = ntrip_p <= kTripCap;
  if (tc_lds)
    for (int t = lane; t < ntrip_p; t += 64) {
      const int kc = t % ntcp, kab = t / ntcp, kb = kab % ntb, ka = kab / ntb;
      triple_consts<LP>(prm.ao_exp[shA.pptr + ka], prm.ao_exp[shB.pptr + kb], prm.ax_exp[shP.pptr + kc],
                        prm.ao_coef[shA.pptr + ka], prm.ao_coef[shB.pptr + kb], prm.ax_coef[shP.pptr + kc],
                        prm.ao_c1s[shA.pptr + ka], prm.ao_c1s[shB.pptr + kb], prm.ax_c1s[shP.pptr + kc], prm.omega, prm.acut,
                        s_tc + t * kTripC);
    }
  const double pd = shA.a_d + shB.a_d;
  const double beta = shA.a_d * shB.a_d / pd;
  const double eta1 = sqrt(shP.a_d * pd / (shP.a_d + pd));
  const double eta2 = 1.0 / sqrt(1.0 / (eta1 * eta1) + 1.0 / (omega * omega));
  const int W = tr.nwin;
  const double rc_cut = tr.rc_cut;
  {
    const double pref = tr.amp * fourpi_vol / (2.0 * beta);
    for (int w = lane; w < W; w += 64) {
      const double R = w * dR;
      const double N = (R > prm.ncell_r0) ? fourpi_vol * 2.0 * (R + dR) * (R + dR) * dR : prm.ncell_nf;
      const double f = (R < 1e-12) ? 2.0 * (eta1 - eta2) * 0.564189583547756286948079451561 /* 1/sqrt(pi) */
                                   : (erf(eta1 * R) - erf(eta2 * R)) / R;
      s_nf[w] = (float)(pref * N * f);
    }
  }
  for (int i = lane; i < BLK; i += 64) s_blk[i] = 0.0;
  for (int i = lane; i < MG * (NH + 1); i += 64) s_R[i] = 0.0;
  for (int idx = lane; idx < NW; idx += 64) {
    const int ic = idx / NHAB, h = idx % NHAB;
    int t, u, v, cx, cy, cz;
    herm_decode(h, t, u, v);
    cart_decode(LP, ic, cx, cy, cz);
    s_wtab[idx] = cx | (cy << 2) | (cz << 4);
    for (int k = 0; k < NK; ++k) {
      const int kx = k / ((KX + 1) * (KX + 1)), ky = (k / (KX + 1)) % (KX + 1), kz = k % (KX + 1);
      const int tx = (cx & 1) + 2 * kx, ty = (cy & 1) + 2 * ky, tz = (cz & 1) + 2 * kz;
      s_widx[idx * NK + k] = (tx <= cx && ty <= cy && tz <= cz) ? (short)hidx(t + tx, u + ty, v + tz) : (short)NH;
    }
  }
  for (int comp = lane; comp < NBLK; comp += 64) {
    const int ic = comp / (NCA * NCB), ia = (comp / NCB) % NCA, ib = comp % NCB;
    int ax_, ay_, az_, bx_, by_, bz_;
    cart_decode(LA, ia, ax_, ay_, az_);
    cart_decode(LB, ib, bx_, by_, bz_);
    s_ctab[comp] = ic | ((ax_ * (LB + 1) + bx_) << 8) | ((ay_ * (LB + 1) + by_) << 16) | ((az_ * (LB + 1) + bz_) << 24);
  }
  __syncthreads();
  const bool logging = prm.logmag != nullptr;
  const int64_t cbase = (prm.mask || logging) ? prm.cand_off[wk.trip] : 0;
  const double xstar = 1.0 / sqrt(2.0 * beta);
  const double gmax = xstar * exp(-0.5);
  const double wgrow = pair_growth_c(beta);
  const double inv_dR = 1.0 / dR;

  const double Ax = shA.x, Ay = shA.y, Az = shA.z;
  const double Cx = shP.x, Cy = shP.y, Cz = shP.z;
  const double *a = lat.a;
  const double *b = lat.b;
  const double inv2pi = 1.0 / (2.0 * kPi);
  double bn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) bn[d] = sqrt(b[3 * d] * b[3 * d] + b[3 * d + 1] * b[3 * d + 1] + b[3 * d + 2] * b[3 * d + 2]);

  // group layout: ncb groups of gs = floor(64 / ncb) lanes (any count, so that
  // 5, 6 or 7 cells per wave keep 60-63 lanes busy), group gl owns BvK cell cb0 + gl
  const int ncbw = wk.ncb;
  const int gs = 64 / ncbw;
  const int lig = lane % gs;
  const int gl = lane / gs;
  const unsigned long long gmask_lo = (gs == 64) ? ~0ull : ((1ull << gs) - 1ull);
  const bool blk_in_lds = NBLK * ncbw <= BLK;
  double *const part = (wk.part >= 0) ? prm.part + wk.part : nullptr;

  const size_t xplane = (size_t)prm.naux_b * prm.nao * prm.nao;
  const int pf0 = shP.foff - prm.aux_f0;
  long long n_terms = 0, n_contr = 0, n_shell = 0;

  const int nimg_all = prm.cls_off[pr.cls_off + nk];

  {
    const int c1 = wk.cb0 + gl;  // this group's BvK cell
    const int ngrp = ncbw;
    const bool grp_on = gl < ngrp;
    int i1[3] = {0, 0, 0};
    if (grp_on) {
      i1[0] = c1 / (lat.n[1] * lat.n[2]);
      i1[1] = (c1 / lat.n[2]) % lat.n[1];
      i1[2] = c1 % lat.n[2];
    }
    const int capb = kCandCap / ngrp;
    int cur_cls = -1;  // class of the n' whose sums sit in the LDS accumulator

    // flush the LDS accumulator of class cls into X
    auto flush = [&](int cls) {
      if (!blk_in_lds || cls < 0) return;
      if (grp_on) {
        // c2 = c1 + cls (component-wise mod n)
        const int dc0 = cls / (lat.n[1] * lat.n[2]), dc1 = (cls / lat.n[2]) % lat.n[1], dc2 = cls % lat.n[2];
        const int c2 = (((i1[0] + dc0) % lat.n[0]) * lat.n[1] + (i1[1] + dc1) % lat.n[1]) * lat.n[2] +
                       (i1[2] + dc2) % lat.n[2];
        double *X12 = prm.X + (size_t)(c1 * nk + c2) * xplane;
        double *X21 = prm.X + (size_t)(c2 * nk + c1) * xplane;
        double *pb = part ? part + ((size_t)gl * nk + c2) * NBLK : nullptr;
        for (int comp = lig; comp < NBLK; comp += gs) {
          const double v = s_blk[gl * NBLK + comp];
          s_blk[gl * NBLK + comp] = 0.0;
          if (v == 0.0) continue;
          if (pb) {
            pb[comp] += v;
            continue;
          }
          const int ic = comp / (NCA * NCB), ia = (comp / NCB) % NCA, ib = comp % NCB;
          const size_t rowP = (size_t)(pf0 + ic) * prm.nao;
          double *x12 = X12 + (rowP + shA.foff + ia) * prm.nao + shB.foff + ib;
          double *x21 = X21 + (rowP + shB.foff + ib) * prm.nao + shA.foff + ia;
          // Outside logging runs each element is flushed once: the class's
          // images are contiguous in the list, the item's cell range is its
          // own, and the transposed block lies in the other shell's rows.  X
          // starts at zero, so a store replaces the read-modify-write.
          if (logging) {
            *x12 += v;
            if (!pr.diag) *x21 += v;
          } else {
            *x12 = v;
            if (!pr.diag) *x21 = v;
          }
        }
      }
    };

    int cls = 0;
    for (int ii = slice; ii < nimg_all; ii += S) {
      // class of this image (the list is grouped by class)
      while (prm.cls_off[pr.cls_off + cls + 1] <= ii) ++cls;
      if (ii - prm.cls_off[pr.cls_off + cls] >= prm.nsr[pr.nsr_off + cls]) continue;  // beyond the SR radius
      if (prm.mask && !prm.mask[cbase + ii]) continue;  // dropped by the learned screen
      const double *nv = prm.img + 3 * (size_t)(pr.img_off + ii);
      const double Bx = shB.x + nv[0], By = shB.y + nv[1], Bz = shB.z + nv[2];
      const double ABx = Ax - Bx, ABy = Ay - By, ABz = Az - Bz;
      const double r12sq = ABx * ABx + ABy * ABy + ABz * ABz;
      const double R12 = sqrt(r12sq);
      // window test of Eqs. S23-S24: keep R_c window w iff R12 <= R12cut(w)
      double thr;
      if (R12 <= pr.R12min) thr = 0.0;
      else {
        double gx = (R12 <= xstar) ? gmax : R12 * exp(-beta * r12sq);
        if constexpr (LA + LB > 0) {  // angular growth of the pair factor
          const double gr = fma(wgrow, R12, 1.0);
          double gp = gr;
#pragma unroll
          for (int i = 1; i < LA + LB; ++i) gp *= gr;
          gx *= gp;
        }
        thr = eps / gx;
      }
      int wmax = -1;
      for (int w = 0; w < W; ++w)
        if (s_nf[w] >= thr) wmax = w;
      if (wmax < 0) continue;
      if (cls != cur_cls) {
        flush(cur_cls);
        cur_cls = cls;
      }
      const double rmax = fmin((wmax + 1) * dR, rc_cut);
      const double rmax2 = rmax * rmax;
      // diffuse pair centre relative to the aux centre
      const double Pdx = (shA.a_d * Ax + shB.a_d * Bx) / pd, Pdy = (shA.a_d * Ay + shB.a_d * By) / pd,
                   Pdz = (shA.a_d * Az + shB.a_d * Bz) / pd;
      const double X0x = Pdx - Cx, X0y = Pdy - Cy, X0z = Pdz - Cz;
      // box of lattice coordinates M_d = i1_d + n_d j_d around -X0
      int lo0, lo1, lo2, dim0, dim1, dim2;
      {
        const double f0 = -(b[0] * X0x + b[1] * X0y + b[2] * X0z) * inv2pi;
        const double f1 = -(b[3] * X0x + b[4] * X0y + b[5] * X0z) * inv2pi;
        const double f2 = -(b[6] * X0x + b[7] * X0y + b[8] * X0z) * inv2pi;
        const double sp0 = rmax * bn[0] * inv2pi, sp1 = rmax * bn[1] * inv2pi, sp2 = rmax * bn[2] * inv2pi;
        lo0 = (int)ceil((f0 - sp0 - i1[0]) / lat.n[0]);
        lo1 = (int)ceil((f1 - sp1 - i1[1]) / lat.n[1]);
        lo2 = (int)ceil((f2 - sp2 - i1[2]) / lat.n[2]);
        dim0 = max(0, (int)floor((f0 + sp0 - i1[0]) / lat.n[0]) - lo0 + 1);
        dim1 = max(0, (int)floor((f1 + sp1 - i1[1]) / lat.n[1]) - lo1 + 1);
        dim2 = max(0, (int)floor((f2 + sp2 - i1[2]) / lat.n[2]) - lo2 + 1);
      }
      const int nbox = grp_on ? dim0 * dim1 * dim2 : 0;
      // chunks of gs candidates; the wave loops to the largest group box
      int nchunk = (nbox + gs - 1) / gs;
      for (int off = 32; off >= 1; off >>= 1) nchunk = max(nchunk, __shfl_xor(nchunk, off, 64));

      int pass = 0;
      for (;;) {
        // ---- enumerate and compact (this pass keeps candidates [pass*capb, (pass+1)*capb))
        const int base = pass * capb;
        int cnt = 0;
        for (int ch = 0; ch < nchunk; ++ch) {
          const int q = ch * gs + lig;
          bool valid = false;
          int M0 = 0, M1 = 0, M2 = 0;
          if (q < nbox) {
            const int j2 = q % dim2, j1 = (q / dim2) % dim1, j0 = q / (dim1 * dim2);
            M0 = i1[0] + lat.n[0] * (lo0 + j0);
            M1 = i1[1] + lat.n[1] * (lo1 + j1);
            M2 = i1[2] + lat.n[2] * (lo2 + j2);
            const double mx = X0x + M0 * a[0] + M1 * a[3] + M2 * a[6];
            const double my = X0y + M0 * a[1] + M1 * a[4] + M2 * a[7];
            const double mz = X0z + M0 * a[2] + M1 * a[5] + M2 * a[8];
            const double rc2 = mx * mx + my * my + mz * mz;
            if (rc2 <= rmax2) {
              const double rc = sqrt(rc2);
              const int w = (int)(rc * inv_dR);
              valid = (rc <= rc_cut) && (w < W) && (s_nf[w] >= thr);
            }
          }
          const unsigned long long bal = __ballot(valid);
          const unsigned long long gb = (bal >> (gl * gs)) & gmask_lo;
          const int pos = cnt + __popcll(gb & ((1ull << lig) - 1ull));
          if (valid && pos >= base && pos < base + capb) s_cand[gl * capb + pos - base] = pack3(M0, M1, M2);
          cnt += __popcll(gb);
        }
        const int total = cnt;
        const int navail = min(max(total - base, 0), capb);
        if (pass == 0 && lig == 0 && grp_on) n_shell += total;
        // groups (bit gl * gs) holding lattice vectors in this pass; empty ones
        // contribute nothing and skip their contraction
        const unsigned long long gnz = __ballot(grp_on && lig == 0 && navail > 0);
        __syncthreads();

        // ---- primitive triples: image-summed Hermite integrals, then contraction
        const double nm = 4.18879020478639098 * rmax2 * rmax / lat.vol + 1.0;
        for (int tt = 0; tt < (gnz ? ntrip_p : 0); ++tt) {
          double tcl[kTripC];
          if (tc_lds) {
#pragma unroll
            for (int q = 0; q < kTripC; ++q) tcl[q] = s_tc[tt * kTripC + q];
          } else {
            const int kc = tt % ntcp, kab = tt / ntcp, kb = kab % ntb, ka = kab / ntb;
            triple_consts<LP>(prm.ao_exp[shA.pptr + ka], prm.ao_exp[shB.pptr + kb], prm.ax_exp[shP.pptr + kc],
                              prm.ao_coef[shA.pptr + ka], prm.ao_coef[shB.pptr + kb], prm.ax_coef[shP.pptr + kc],
                              prm.ao_c1s[shA.pptr + ka], prm.ao_c1s[shB.pptr + kb], prm.ax_c1s[shP.pptr + kc],
                              omega, prm.acut, tcl);
          }
          const double oop = tcl[0];
          const double Kab = exp(-tcl[2] * r12sq);
          // primitive screen: image-summed 1s estimate for this n' far below
          // the target precision
          if (tcl[7] * Kab * nm < 1e-4 * eps) continue;
          const double Px = Ax + tcl[1] * (Bx - Ax), Py = Ay + tcl[1] * (By - Ay), Pz = Az + tcl[1] * (Bz - Az);
          // offset of this primitive pair's centre from the aux centre at m = 0
          const double dPx = Px - Pdx + X0x, dPy = Py - Pdy + X0y, dPz = Pz - Pdz + X0z;
          {
              const double rho = tcl[3];
              const double th2 = tcl[4];
              const double th = tcl[5];
              const double m2rho = -2.0 * rho;
              double Rb[NH];
#pragma unroll
              for (int i = 0; i < NH; ++i) Rb[i] = 0.0;
              for (int e = lig; e < navail; e += gs) {
                int M0, M1, M2;
                unpack3(s_cand[gl * capb + e], M0, M1, M2);
                const double X = dPx + M0 * a[0] + M1 * a[3] + M2 * a[6];
                const double Y = dPy + M0 * a[1] + M1 * a[4] + M2 * a[7];
                const double Z = dPz + M0 * a[2] + M1 * a[5] + M2 * a[8];
                const double T = rho * (X * X + Y * Y + Z * Z);
                double g[L + 1];
                gvals_sr<L>(T, th2, th, s_boys, g);
                double f = 1.0;
#pragma unroll
                for (int n = 1; n <= L; ++n) {
                  f *= m2rho;
                  g[n] *= f;
                }
                hermite_R_acc<L>(X, Y, Z, g, Rb);
                ++n_terms;
              }
              // group reduction, transposed through LDS in chunks of CH entries:
              // each entry of a group is summed by one lane over the group's gs
              // lanes in lane order (deterministic), into s_R[group][h]
#pragma unroll
              for (int c0 = 0; c0 < NH; c0 += CH) {
#pragma unroll
                for (int j = 0; j < CH; ++j)
                  if (c0 + j < NH) s_T[lane * CH + j] = Rb[c0 + j];
                __syncthreads();
                if (grp_on) {
                  for (int j = lig; j < CH && c0 + j < NH; j += gs) {
                    // reads issued eight at a time (gs >= 8); the sum keeps lane order
                    const double *col = s_T + gl * gs * CH + j;
                    double acc = 0.0;
                    int r = 0;
                    for (; r + 8 <= gs; r += 8) {
                      double v[8];
#pragma unroll
                      for (int q = 0; q < 8; ++q) v[q] = col[(r + q) * CH];
#pragma unroll
                      for (int q = 0; q < 8; ++q) acc += v[q];
                    }
                    for (; r < gs; ++r) acc += col[r * CH];
                    s_R[gl * (NH + 1) + c0 + j] = acc;
                  }
                }
                __syncthreads();
              }
              // ---- contraction with the Hermite expansion coefficients: one
              // group at a time, its sums in the LDS cube, output components
              // spread over the 64 lanes; every loop bound is compile-time
              if (lane < 3) {
                double E1[LA + 1][LB + 1][LAB + 1];
                const double PAd = (lane == 0) ? Px - Ax : (lane == 1 ? Py - Ay : Pz - Az);
                const double PBd = (lane == 0) ? Px - Bx : (lane == 1 ? Py - By : Pz - Bz);
                hermite_E<LA, LB>(PAd, PBd, 0.5 * oop, E1);
#pragma unroll
                for (int i = 0; i <= LA; ++i)
#pragma unroll
                  for (int j = 0; j <= LB; ++j)
#pragma unroll
                    for (int t = 0; t <= LAB; ++t) s_E[lane * EA + (i * (LB + 1) + j) * (LAB + 1) + t] = E1[i][j][t];
              } else if (lane == 3) {
                double E2[LP + 1][LP + 1];
                hermite_E1<LP>(tcl[8], E2);
#pragma unroll
                for (int i = 0; i <= LP; ++i)
#pragma unroll
                  for (int t = 0; t <= LP; ++t) s_EP[i * (LP + 1) + t] = E2[i][t];
              }
              const double coef = tcl[6] * Kab;
              __syncthreads();  // E coefficients and group sums visible to every lane
              // W[g][ic][h] = sum_{tau nu phi} E^c_{cx,tau} E^c_{cy,nu} E^c_{cz,phi} R[g][h + (tau nu phi)]
              if constexpr (L >= 5) {
              // L >= 5 (one wave per SIMD, registers to spare in the AGPRs): a lane
              // holds one entry's aux factors and Hermite indices and runs over the
              // groups of its lane set (64 / NW sets when NW < 64); the lighter
              // classes spill if they hold them, so their lanes take (group, entry)
              // pairs in turn
              constexpr int RW = NW >= 64 ? 1 : 64 / NW;
              for (int cb = lane; cb < NW * RW; cb += 64) {
                const int idx = cb % NW, gset = cb / NW;
                const int w = s_wtab[idx];
                const int cx = w & 3, cy = (w >> 2) & 3, cz = (w >> 4) & 3;
                double ex[KX + 1], ey[KX + 1], ez[KX + 1];
#pragma unroll
                for (int k = 0; k <= KX; ++k) {
                  const int tx = (cx & 1) + 2 * k, ty = (cy & 1) + 2 * k, tz = (cz & 1) + 2 * k;
                  ex[k] = (tx <= cx) ? s_EP[cx * (LP + 1) + min(tx, LP)] : 0.0;
                  ey[k] = (ty <= cy) ? s_EP[cy * (LP + 1) + min(ty, LP)] : 0.0;
                  ez[k] = (tz <= cz) ? s_EP[cz * (LP + 1) + min(tz, LP)] : 0.0;
                }
                const short *wip = s_widx + idx * NK;
                int wi[NK];
#pragma unroll
                for (int k = 0; k < NK; ++k) wi[k] = wip[k];
                for (int g = gset; g < ngrp; g += RW) {
                  if (!((gnz >> (g * gs)) & 1ull)) continue;
                  const double *rg = s_R + g * (NH + 1);
                  // every group sum this entry needs, read before the first multiply
                  double rv[NK];
#pragma unroll
                  for (int k = 0; k < NK; ++k) rv[k] = rg[wi[k]];
                  double sw = 0.0;
#pragma unroll
                  for (int kx = 0; kx <= KX; ++kx)
#pragma unroll
                    for (int ky = 0; ky <= KX; ++ky) {
                      double sz = 0.0;
#pragma unroll
                      for (int kz = 0; kz <= KX; ++kz) sz += ez[kz] * rv[(kx * (KX + 1) + ky) * (KX + 1) + kz];
                      sw += ex[kx] * ey[ky] * sz;
                    }
                  s_W[g * NW + idx] = sw;
                }
              }
              } else {
              for (int e = lane; e < ngrp * NW; e += 64) {
                const int g = e / NW, idx = e - g * NW;
                if (!((gnz >> (g * gs)) & 1ull)) continue;
                const int w = s_wtab[idx];
                const int cx = w & 3, cy = (w >> 2) & 3, cz = (w >> 4) & 3;
                double ex[KX + 1], ey[KX + 1], ez[KX + 1];
#pragma unroll
                for (int k = 0; k <= KX; ++k) {
                  const int tx = (cx & 1) + 2 * k, ty = (cy & 1) + 2 * k, tz = (cz & 1) + 2 * k;
                  ex[k] = (tx <= cx) ? s_EP[cx * (LP + 1) + min(tx, LP)] : 0.0;
                  ey[k] = (ty <= cy) ? s_EP[cy * (LP + 1) + min(ty, LP)] : 0.0;
                  ez[k] = (tz <= cz) ? s_EP[cz * (LP + 1) + min(tz, LP)] : 0.0;
                }
                const double *rg = s_R + g * (NH + 1);
                const short *wi = s_widx + idx * NK;
                // every group sum this entry needs, read before the first multiply
                double rv[NK];
#pragma unroll
                for (int k = 0; k < NK; ++k) rv[k] = rg[wi[k]];
                double sw = 0.0;
#pragma unroll
                for (int kx = 0; kx <= KX; ++kx)
#pragma unroll
                  for (int ky = 0; ky <= KX; ++ky) {
                    double sz = 0.0;
#pragma unroll
                    for (int kz = 0; kz <= KX; ++kz) sz += ez[kz] * rv[(kx * (KX + 1) + ky) * (KX + 1) + kz];
                    sw += ex[kx] * ey[ky] * sz;
                  }
                s_W[g * NW + idx] = sw;
              }
              }
              __syncthreads();
              // component (ic, ia, ib) of group g = sum_{tuv} E^x_t E^y_u E^z_v W[g][ic][tuv]
              if constexpr (L >= 5) {
              // L >= 5: a lane holds one component's E rows in registers and runs
              // over the groups of its lane set (64 / NBLK sets share the groups when
              // NBLK < 64), so the rows are read once per component, not per group
              constexpr int RS = NBLK >= 64 ? 1 : 64 / NBLK;
              for (int cb = lane; cb < NBLK * RS; cb += 64) {
                const int comp = cb % NBLK, gset = cb / NBLK;
                const int c = s_ctab[comp];
                const int ic = c & 0xff;
                double ex[LAB + 1], ey[LAB + 1], ez[LAB + 1];
#pragma unroll
                for (int t = 0; t <= LAB; ++t) {
                  ex[t] = s_E[0 * EA + ((c >> 8) & 0xff) * (LAB + 1) + t];
                  ey[t] = s_E[1 * EA + ((c >> 16) & 0xff) * (LAB + 1) + t];
                  ez[t] = s_E[2 * EA + ((c >> 24) & 0xff) * (LAB + 1) + t];
                }
                for (int g = gset; g < ngrp; g += RS) {
                if (!((gnz >> (g * gs)) & 1ull)) continue;
                const double *wr = s_W + g * NW + ic * NHAB;
                double so = 0.0;
#pragma unroll
                for (int t = 0; t <= LAB; ++t) {
                  double st = 0.0;
#pragma unroll
                  for (int u = 0; u <= LAB - t; ++u) {
                    double su = 0.0;
#pragma unroll
                    for (int v = 0; v <= LAB - t - u; ++v) su += ez[v] * wr[hidx(t, u, v)];
                    st += ey[u] * su;
                  }
                  so += ex[t] * st;
                }
                const double val = coef * so;
                if (blk_in_lds) {
                  s_blk[g * NBLK + comp] += val;
                } else {
                  const int cg = wk.cb0 + g;
                  const int ig0 = cg / (lat.n[1] * lat.n[2]), ig1 = (cg / lat.n[2]) % lat.n[1], ig2 = cg % lat.n[2];
                  const int dc0 = cls / (lat.n[1] * lat.n[2]), dc1 = (cls / lat.n[2]) % lat.n[1], dc2 = cls % lat.n[2];
                  const int c2 = (((ig0 + dc0) % lat.n[0]) * lat.n[1] + (ig1 + dc1) % lat.n[1]) * lat.n[2] +
                                 (ig2 + dc2) % lat.n[2];
                  if (part) {
                    part[((size_t)g * nk + c2) * NBLK + comp] += val;
                  } else {
                    const int ia = (comp / NCB) % NCA, ib = comp % NCB;
                    const size_t rowP = (size_t)(pf0 + ic) * prm.nao;
                    prm.X[(size_t)(cg * nk + c2) * xplane + (rowP + shA.foff + ia) * prm.nao + shB.foff + ib] += val;
                    if (!pr.diag)
                      prm.X[(size_t)(c2 * nk + cg) * xplane + (rowP + shB.foff + ib) * prm.nao + shA.foff + ia] += val;
                  }
                }
                }
              }
              } else {
              for (int e = lane; e < ngrp * NBLK; e += 64) {
                const int g = e / NBLK, comp = e - g * NBLK;
                if (!((gnz >> (g * gs)) & 1ull)) continue;
                const int c = s_ctab[comp];
                const int ic = c & 0xff;
                const double *ex = s_E + 0 * EA + ((c >> 8) & 0xff) * (LAB + 1);
                const double *ey = s_E + 1 * EA + ((c >> 16) & 0xff) * (LAB + 1);
                const double *ez = s_E + 2 * EA + ((c >> 24) & 0xff) * (LAB + 1);
                const double *wr = s_W + g * NW + ic * NHAB;
                double so = 0.0;
#pragma unroll
                for (int t = 0; t <= LAB; ++t) {
                  double st = 0.0;
#pragma unroll
                  for (int u = 0; u <= LAB - t; ++u) {
                    double su = 0.0;
#pragma unroll
                    for (int v = 0; v <= LAB - t - u; ++v) su += ez[v] * wr[hidx(t, u, v)];
                    st += ey[u] * su;
                  }
                  so += ex[t] * st;
                }
                const double val = coef * so;
                if (blk_in_lds) {
                  s_blk[g * NBLK + comp] += val;
                } else {
                  const int cg = wk.cb0 + g;
                  const int ig0 = cg / (lat.n[1] * lat.n[2]), ig1 = (cg / lat.n[2]) % lat.n[1], ig2 = cg % lat.n[2];
                  const int dc0 = cls / (lat.n[1] * lat.n[2]), dc1 = (cls / lat.n[2]) % lat.n[1], dc2 = cls % lat.n[2];
                  const int c2 = (((ig0 + dc0) % lat.n[0]) * lat.n[1] + (ig1 + dc1) % lat.n[1]) * lat.n[2] +
                                 (ig2 + dc2) % lat.n[2];
                  if (part) {
                    part[((size_t)g * nk + c2) * NBLK + comp] += val;
                  } else {
                    const int ia = (comp / NCB) % NCA, ib = comp % NCB;
                    const size_t rowP = (size_t)(pf0 + ic) * prm.nao;
                    prm.X[(size_t)(cg * nk + c2) * xplane + (rowP + shA.foff + ia) * prm.nao + shB.foff + ib] += val;
                    if (!pr.diag)
                      prm.X[(size_t)(c2 * nk + cg) * xplane + (rowP + shB.foff + ib) * prm.nao + shA.foff + ia] += val;
                  }
                }
              }
              }
              __syncthreads();
              if (lane == 0) n_contr += __popcll(gnz);  // (image, triple, cell group) contractions
          }
        }
        // more candidates than one pass holds?
        int more = (total > base + capb) ? 1 : 0;
        for (int off = 32; off >= 1; off >>= 1) more = max(more, __shfl_xor(more, off, 64));
        __syncthreads();
        if (!more) break;
        ++pass;
      }
      if (logging && blk_in_lds) {
        // magnitude log: the accumulator holds only this pair image's block (it is
        // flushed after every image in logging runs); max |block| per BvK cell c1,
        // each (ii, c1) owned by one wave
        if (grp_on && lig == 0) {
          double mx = 0.0;
          for (int comp = 0; comp < NBLK; ++comp) mx = fmax(mx, fabs(s_blk[gl * NBLK + comp]));
          prm.logmag[(cbase + ii) * nk + c1] = (float)mx;
        }
        flush(cur_cls);
        __syncthreads();
      }
    }
    flush(cur_cls);
    __syncthreads();
  }

  // ---- work counters (deterministic integer reduction), one slot per item
  for (int off = 32; off >= 1; off >>= 1) {
    n_terms += __shfl_xor(n_terms, off, 64);
    n_contr += __shfl_xor(n_contr, off, 64);
    n_shell += __shfl_xor(n_shell, off, 64);
  }
  if (lane == 0) {
    long long *dst = counts + 4 * ((size_t)w0 + blockIdx.x);
    dst[0] = n_terms;
    dst[1] = n_contr;
    dst[2] = n_shell;
    dst[3] = 0;
  }
}


// Sum the partial blocks of split work items (slice order) into X, direct and
// transposed entries.  One thread per element of a (work item, cell range).
__global__ void sr_reduce_kernel(const SRParams prm, const SRPartGroup *__restrict__ groups, int ngroups,
                                 int64_t nelem) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nelem) return;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (groups[mid].elem_off <= gid) lo = mid;
    else hi = mid - 1;
  }
  const SRPartGroup g = groups[lo];
  const int64_t e = gid - g.elem_off;
  const Triplet tr = prm.trip[g.trip];
  const Pair pr = prm.pairs[tr.pair];
  const Shell shP = prm.ax[tr.aux], shA = prm.ao[pr.sa], shB = prm.ao[pr.sb];
  const int nca = ncart(shA.l), ncb = ncart(shB.l), nblk = ncart(shP.l) * nca * ncb;
  const int nk = prm.lat.nk;
  const int64_t blk = (int64_t)g.ncb * nk * nblk;
  double v = 0.0;
  for (int s = 0; s < g.nslice; ++s) v += prm.part[g.part + s * blk + e];
  const int comp = (int)(e % nblk);
  const int c2 = (int)((e / nblk) % nk);
  const int c1 = g.cb0 + (int)(e / ((int64_t)nblk * nk));
  const int ic = comp / (nca * ncb), ia = (comp / ncb) % nca, ib = comp % ncb;
  const size_t xplane = (size_t)prm.naux_b * prm.nao * prm.nao;
  const size_t rowP = (size_t)(shP.foff - prm.aux_f0 + ic) * prm.nao;
  prm.X[(size_t)(c1 * nk + c2) * xplane + (rowP + shA.foff + ia) * prm.nao + shB.foff + ib] += v;
  if (!pr.diag) prm.X[(size_t)(c2 * nk + c1) * xplane + (rowP + shB.foff + ib) * prm.nao + shA.foff + ia] += v;
}

hipError_t launch_sr_reduce(const SRParams &prm, const SRPartGroup *groups, int ngroups, int64_t nelem,
                            hipStream_t stream) {
  if (ngroups <= 0 || nelem <= 0) return hipSuccess;
  hipLaunchKernelGGL(sr_reduce_kernel, dim3((unsigned)((nelem + 255) / 256)), dim3(256), 0, stream, prm, groups,
                     ngroups, nelem);
  return hipGetLastError();
}

typedef void (*sr_kernel_t)(const SRParams *, const SRWork *, long long *, const int);

#define RSGDF_SR_ENTRY(LP, LA, LB) &sr3c_kernel<LP, LA, LB>
static const sr_kernel_t kSRTable[4][6] = {
    {RSGDF_SR_ENTRY(0, 0, 0), RSGDF_SR_ENTRY(0, 1, 0), RSGDF_SR_ENTRY(0, 1, 1), RSGDF_SR_ENTRY(0, 2, 0),
     RSGDF_SR_ENTRY(0, 2, 1), RSGDF_SR_ENTRY(0, 2, 2)},
    {RSGDF_SR_ENTRY(1, 0, 0), RSGDF_SR_ENTRY(1, 1, 0), RSGDF_SR_ENTRY(1, 1, 1), RSGDF_SR_ENTRY(1, 2, 0),
     RSGDF_SR_ENTRY(1, 2, 1), RSGDF_SR_ENTRY(1, 2, 2)},
    {RSGDF_SR_ENTRY(2, 0, 0), RSGDF_SR_ENTRY(2, 1, 0), RSGDF_SR_ENTRY(2, 1, 1), RSGDF_SR_ENTRY(2, 2, 0),
     RSGDF_SR_ENTRY(2, 2, 1), RSGDF_SR_ENTRY(2, 2, 2)},
    {RSGDF_SR_ENTRY(3, 0, 0), RSGDF_SR_ENTRY(3, 1, 0), RSGDF_SR_ENTRY(3, 1, 1), RSGDF_SR_ENTRY(3, 2, 0),
     RSGDF_SR_ENTRY(3, 2, 1), RSGDF_SR_ENTRY(3, 2, 2)},
};

// pair class index of (la, lb) with la >= lb
hipError_t launch_sr3c(int lP, int pc, const SRParams *prms, const SRWork *works, long long *counts, int w0,
                       int nwork, hipStream_t stream) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(kSRTable[lP][pc], dim3((unsigned)nwork), dim3(64), 0, stream, prms, works, counts, w0);
  return hipGetLastError();
}

}  // namespace rsgdf
