/*
 * oracle.c -- plain, slow, FP64 CPU reference for the range-separated
 * three-center Coulomb integrals of periodic Gaussian density fitting
 * (Ye & Berkelbach, "Fast periodic Gaussian density fitting by range
 * separation", arXiv 2102.02989).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU path and uses different
 * algorithms on purpose:
 *   - SR integrals by the Obara-Saika vertical recurrence on the bra centre
 *     and the aux centre, then the horizontal recurrence (the GPU path uses
 *     McMurchie-Davidson Hermite sums);
 *   - Boys function by its power series plus downward recursion (small T)
 *     and the erf closed form plus upward recursion (large T);
 *   - Fourier transforms by binomial expansion about the Gaussian-product
 *     centre and Hermite polynomials (the GPU path uses Hermite E
 *     coefficients);
 *   - a direct double DFT for the Bloch fold;
 *   - its own, deliberately loose, image-truncation rule.
 *
 * What is computed (paper, Eqs. M6, M9-M14):
 *   j3c[k1,k2][P][mu][nu] = SR - G0 + LR, with
 *   SR = sum_{m,n} e^{-i k1.m} e^{+i k2.n} (P^0 | erfc(w r)/r | mu^m nu^n)   (Eq. M12, M13a)
 *   G0 = delta_{k1k2} pi/(Omega w^2) S_P S_munu(k1)                          (Eq. M12 2nd term, M13b-c)
 *   LR = (4 pi/Omega) sum_{q=G+k12, q!=0, exp(-q^2/4w^2)>=gthr}
 *          exp(-q^2/4w^2)/q^2 chi~_P(-q) rho^_munu^{k2}(q)                   (Eq. M10, M11)
 * with chi~(q) = int chi(r) e^{-iq.r} dr over all space and
 * rho^^{k2}(q) = sum_n e^{+i k2.n} int phi_mu(r) phi_nu(r-n) e^{-iq.r} dr.
 * The sum j3c equals the G=0-removed full-Coulomb integral (Eq. M15 with a
 * 1/Omega normalisation) and is independent of w.
 *
 * Phase convention: Bloch functions phi^k = sum_m e^{ik.m} phi(r-m)
 * (Eq. M1), so the pair-image phase in rho^ is e^{+i k2.n}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

enum { ORC_COUL = 0, ORC_ERF = 1, ORC_ERFC = 2 };
enum { ORC_PART_SR = 1, ORC_PART_G0 = 2, ORC_PART_LR = 4, ORC_PART_M15 = 8 };

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian components of angular momentum l: x power descending, then y. */
static void cart_powers(int l, int pw[][3]) {
  int n = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      pw[n][0] = lx; pw[n][1] = ly; pw[n][2] = l - lx - ly; ++n;
    }
}

/* ------------------------------------------------------------------ Boys */
/* F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt for m = 0..mmax.
 * T <= 40: power series F_mmax(T) = e^{-T} sum_k (2T)^k / prod_{j=0..k}(2mmax+2j+1),
 *          then the exact downward recursion F_m = (2T F_{m+1} + e^{-T})/(2m+1).
 * T  > 40: F_0 = sqrt(pi/T) erf(sqrt T)/2 and the upward recursion
 *          F_{m+1} = ((2m+1) F_m - e^{-T})/(2T), stable when T > m. */
void orc_boys_array(int mmax, double T, double *F) {
  if (T <= 40.0) {
    double term = 1.0 / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 2000; ++k) {
      term *= 2.0 * T / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    double e = exp(-T);
    F[mmax] = e * sum;
    for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) / (2 * m + 1);
  } else {
    double e = exp(-T);
    F[0] = 0.5 * sqrt(ORC_PI / T) * erf(sqrt(T));
    for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0 * T);
  }
}

double orc_boys(int m, double T) {
  double F[64];
  if (m < 0 || m > 60) return NAN;
  orc_boys_array(m, T, F);
  return F[m];
}

/* Operator-dependent auxiliary values G_m (m = 0..mmax) at T = rho |P-C|^2:
 *   Coulomb 1/r         : F_m(T)
 *   erf(w r)/r          : theta^{2m+1} F_m(theta^2 T),  theta^2 = w^2/(w^2+rho)
 *   erfc(w r)/r         : F_m(T) - theta^{2m+1} F_m(theta^2 T)
 * (attenuated-operator Boys values; the erf case is the Gaussian-charge
 *  convolution of the kernel, cf. Eq. M9 and the s-type closed form Eq. S3-S9).
 * All three obey dG_m/dT = -G_{m+1}, which is all the Obara-Saika
 * recurrences below need. */
void orc_gvals(int kind, int mmax, double T, double theta2, double *G) {
  double Fc[64], Fe[64];
  if (kind != ORC_ERF) orc_boys_array(mmax, T, Fc);
  if (kind != ORC_COUL) orc_boys_array(mmax, theta2 * T, Fe);
  for (int m = 0; m <= mmax; ++m) {
    double e = 0.0;
    if (kind != ORC_COUL) e = pow(theta2, m + 0.5) * Fe[m];
    if (kind == ORC_COUL) G[m] = Fc[m];
    else if (kind == ORC_ERF) G[m] = e;
    else G[m] = Fc[m] - e;
  }
}

/* ------------------------------------------- isolated primitive 3-centre */
/* (c | w | a b) for unnormalised Cartesian primitives
 *   c(r) = (x-Cx)^i (y-Cy)^j (z-Cz)^k exp(-gc |r-C|^2)   (aux, lc)
 *   a(r) ~ exp(-ga |r-A|^2) (la),  b(r) ~ exp(-gb |r-B|^2) (lb)
 * Obara-Saika: build [e0|c]^(m) for |e| <= la+lb, |c| <= lc by the vertical
 * recurrences on A and on C, then transfer to (a b| with the horizontal
 * recurrence (a, b+1_i| = (a+1_i, b| + (A_i - B_i)(a b|.
 * out[(ic*nca + ia)*ncb + ib]. */
#define LE_MAX 8
#define LC_MAX 4
typedef struct {
  int Le, Lc, Lt;
  double *V; /* dims (Le+1)^3 x (Lc+1)^3 x (Lt+1) */
} vrr_tab;

static size_t vidx(const vrr_tab *t, const int *e, const int *c, int m) {
  int d1 = t->Le + 1, d2 = t->Lc + 1, d3 = t->Lt + 1;
  return ((((((size_t)e[0] * d1 + e[1]) * d1 + e[2]) * d2 + c[0]) * d2 + c[1]) * d2 + c[2]) * d3 + m;
}

static double hrr(const vrr_tab *t, const double *AB, int a0, int a1, int a2, int b0, int b1, int b2,
                  const int *c) {
  if (b0 == 0 && b1 == 0 && b2 == 0) {
    int e[3] = {a0, a1, a2};
    return t->V[vidx(t, e, c, 0)];
  }
  if (b0 > 0) return hrr(t, AB, a0 + 1, a1, a2, b0 - 1, b1, b2, c) + AB[0] * hrr(t, AB, a0, a1, a2, b0 - 1, b1, b2, c);
  if (b1 > 0) return hrr(t, AB, a0, a1 + 1, a2, b0, b1 - 1, b2, c) + AB[1] * hrr(t, AB, a0, a1, a2, b0, b1 - 1, b2, c);
  return hrr(t, AB, a0, a1, a2 + 1, b0, b1, b2 - 1, c) + AB[2] * hrr(t, AB, a0, a1, a2, b0, b1, b2 - 1, c);
}

int orc_prim3c(int kind, double omega, int lc, double gc, const double *C, int la, double ga,
               const double *A, int lb, double gb, const double *B, double *out) {
  if (la < 0 || lb < 0 || lc < 0 || la + lb > LE_MAX || lc > LC_MAX) return -1;
  const int Le = la + lb, Lc = lc, Lt = Le + Lc;
  const double p = ga + gb, rho = p * gc / (p + gc);
  double P[3], W[3], PA[3], WP[3], WC[3], AB[3], ab2 = 0.0, pc2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    P[i] = (ga * A[i] + gb * B[i]) / p;
    W[i] = (p * P[i] + gc * C[i]) / (p + gc);
    PA[i] = P[i] - A[i];
    WP[i] = W[i] - P[i];
    WC[i] = W[i] - C[i];
    AB[i] = A[i] - B[i];
    ab2 += AB[i] * AB[i];
    pc2 += (P[i] - C[i]) * (P[i] - C[i]);
  }
  const double K = exp(-ga * gb / p * ab2);
  const double pref = 2.0 * pow(ORC_PI, 2.5) / (p * gc * sqrt(p + gc)) * K;
  const double theta2 = (kind == ORC_COUL) ? 1.0 : omega * omega / (omega * omega + rho);
  double G[LE_MAX + LC_MAX + 2];
  orc_gvals(kind, Lt, rho * pc2, theta2, G);

  vrr_tab t;
  t.Le = Le; t.Lc = Lc; t.Lt = Lt;
  size_t n = (size_t)(Le + 1) * (Le + 1) * (Le + 1) * (Lc + 1) * (Lc + 1) * (Lc + 1) * (Lt + 1);
  static __thread double *vbuf = NULL;
  static __thread size_t vcap = 0;
  if (n > vcap) {
    free(vbuf);
    vbuf = (double *)malloc(n * sizeof(double));
    vcap = vbuf ? n : 0;
    if (!vbuf) return -2;
  }
  t.V = vbuf; /* every entry read below is written earlier in the fill order */

  int e[3], c[3];
  for (int sc = 0; sc <= Lc; ++sc)
    for (c[0] = sc; c[0] >= 0; --c[0])
      for (c[1] = sc - c[0]; c[1] >= 0; --c[1]) {
        c[2] = sc - c[0] - c[1];
        for (int se = 0; se <= Le; ++se)
          for (e[0] = se; e[0] >= 0; --e[0])
            for (e[1] = se - e[0]; e[1] >= 0; --e[1]) {
              e[2] = se - e[0] - e[1];
              for (int m = 0; m <= Lt - se - sc; ++m) {
                double v;
                if (sc == 0 && se == 0) {
                  v = pref * G[m];
                } else if (sc == 0) {
                  /* [e|0]^(m) from e' = e - 1_i (vertical recurrence on A) */
                  int i = (e[0] > 0) ? 0 : (e[1] > 0 ? 1 : 2);
                  int e1[3] = {e[0], e[1], e[2]};
                  e1[i] -= 1;
                  int z[3] = {0, 0, 0};
                  v = PA[i] * t.V[vidx(&t, e1, z, m)] + WP[i] * t.V[vidx(&t, e1, z, m + 1)];
                  if (e1[i] > 0) {
                    int e2[3] = {e1[0], e1[1], e1[2]};
                    e2[i] -= 1;
                    v += e1[i] / (2.0 * p) * (t.V[vidx(&t, e2, z, m)] - rho / p * t.V[vidx(&t, e2, z, m + 1)]);
                  }
                } else {
                  /* [e|c]^(m) from c' = c - 1_i (vertical recurrence on C) */
                  int i = (c[0] > 0) ? 0 : (c[1] > 0 ? 1 : 2);
                  int c1[3] = {c[0], c[1], c[2]};
                  c1[i] -= 1;
                  v = WC[i] * t.V[vidx(&t, e, c1, m + 1)];
                  if (c1[i] > 0) {
                    int c2[3] = {c1[0], c1[1], c1[2]};
                    c2[i] -= 1;
                    v += c1[i] / (2.0 * gc) * (t.V[vidx(&t, e, c2, m)] - rho / gc * t.V[vidx(&t, e, c2, m + 1)]);
                  }
                  if (e[i] > 0) {
                    int e1[3] = {e[0], e[1], e[2]};
                    e1[i] -= 1;
                    v += e[i] / (2.0 * (p + gc)) * t.V[vidx(&t, e1, c1, m + 1)];
                  }
                }
                t.V[vidx(&t, e, c, m)] = v;
              }
            }
      }

  int pa[64][3], pb[64][3], pcw[64][3];
  cart_powers(la, pa);
  cart_powers(lb, pb);
  cart_powers(lc, pcw);
  const int nca = ncart(la), ncb = ncart(lb), ncc = ncart(lc);
  for (int ic = 0; ic < ncc; ++ic)
    for (int ia = 0; ia < nca; ++ia)
      for (int ib = 0; ib < ncb; ++ib)
        out[((size_t)ic * nca + ia) * ncb + ib] =
            hrr(&t, AB, pa[ia][0], pa[ia][1], pa[ia][2], pb[ib][0], pb[ib][1], pb[ib][2], pcw[ic]);
  return 0;
}

/* ----------------------------------------------- 1-D Gaussian utilities */
static double dfact(int n) { /* n!! with (-1)!! = 1 */
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}
static double binom(int n, int k) {
  double r = 1.0;
  for (int j = 1; j <= k; ++j) r = r * (n - k + j) / j;
  return r;
}

/* int y^s exp(-p y^2) dy over the real line */
static double gauss_moment(int s, double p) {
  if (s & 1) return 0.0;
  return dfact(s - 1) / pow(2.0 * p, s / 2) * sqrt(ORC_PI / p);
}

/* physicists' Hermite polynomial H_n(x) */
static double hermite_h(int n, double x) {
  double h0 = 1.0, h1 = 2.0 * x;
  if (n == 0) return h0;
  for (int k = 1; k < n; ++k) {
    double h2 = 2.0 * x * h1 - 2.0 * k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

/* int y^s exp(-p y^2) exp(-i q y) dy = sqrt(pi/p) (-i/(2 sqrt p))^s H_s(q/(2 sqrt p)) exp(-q^2/4p)
 * returned as (re, im). */
static void gauss_ft1(int s, double p, double q, double *re, double *im) {
  double sp = sqrt(p);
  double mag = sqrt(ORC_PI / p) * pow(1.0 / (2.0 * sp), s) * hermite_h(s, q / (2.0 * sp)) * exp(-q * q / (4.0 * p));
  /* (-i)^s */
  switch (s & 3) {
    case 0: *re = mag; *im = 0.0; break;
    case 1: *re = 0.0; *im = -mag; break;
    case 2: *re = -mag; *im = 0.0; break;
    default: *re = 0.0; *im = mag; break;
  }
}

/* 1-D product expansion about the product centre:
 * (x-A)^a (x-B)^b = sum_s c_s (x-P)^s,  c_s = sum_{i+j=s} C(a,i) C(b,j) (P-A)^{a-i} (P-B)^{b-j} */
static void product_poly(int a, int b, double PA, double PB, double *cs /* a+b+1 */) {
  for (int s = 0; s <= a + b; ++s) cs[s] = 0.0;
  for (int i = 0; i <= a; ++i)
    for (int j = 0; j <= b; ++j)
      cs[i + j] += binom(a, i) * binom(b, j) * pow(PA, a - i) * pow(PB, b - j);
}

/* overlap of two unnormalised Cartesian primitives over all space */
static double prim_overlap(const int *pa, double ga, const double *A, const int *pb, double gb, const double *B) {
  double p = ga + gb, r = 1.0;
  for (int d = 0; d < 3; ++d) {
    double P = (ga * A[d] + gb * B[d]) / p;
    double cs[16];
    product_poly(pa[d], pb[d], P - A[d], P - B[d], cs);
    double s1 = 0.0;
    for (int s = 0; s <= pa[d] + pb[d]; ++s) s1 += cs[s] * gauss_moment(s, p);
    r *= exp(-ga * gb / p * (A[d] - B[d]) * (A[d] - B[d])) * s1;
  }
  return r;
}

/* Fourier transform over all space of a product of two unnormalised
 * Cartesian primitives: int a(r) b(r) e^{-i q.r} dr  -> (re, im). */
static void prim_pair_ft(const int *pa, double ga, const double *A, const int *pb, double gb, const double *B,
                         const double *q, double *re, double *im) {
  double p = ga + gb;
  double cr = 1.0, ci = 0.0;
  for (int d = 0; d < 3; ++d) {
    double P = (ga * A[d] + gb * B[d]) / p;
    double cs[16];
    product_poly(pa[d], pb[d], P - A[d], P - B[d], cs);
    double sr = 0.0, si = 0.0;
    for (int s = 0; s <= pa[d] + pb[d]; ++s) {
      double fr, fi;
      gauss_ft1(s, p, q[d], &fr, &fi);
      sr += cs[s] * fr;
      si += cs[s] * fi;
    }
    double K = exp(-ga * gb / p * (A[d] - B[d]) * (A[d] - B[d]));
    /* shift to centre P: factor e^{-i q P} */
    double ph = -q[d] * P;
    double tr = K * (sr * cos(ph) - si * sin(ph));
    double ti = K * (sr * sin(ph) + si * cos(ph));
    double nr = cr * tr - ci * ti, ni = cr * ti + ci * tr;
    cr = nr;
    ci = ni;
  }
  *re = cr;
  *im = ci;
}

/* All Cartesian components of a primitive pair transform at once:
 * out[2*(ia*ncb+ib)+{0,1}] = int a(r) b(r) e^{-iq.r} dr.  The 3-D transform
 * factorises into 1-D ones; each 1-D factor is tabulated for every power
 * pair (i <= la, j <= lb) and the components are products of them. */
static void prim_pair_ft_block(int la, double ga, const double *A, int lb, double gb, const double *B,
                               const double *q, double *out) {
  double p = ga + gb;
  double tr[3][8][8], ti[3][8][8];
  for (int d = 0; d < 3; ++d) {
    double P = (ga * A[d] + gb * B[d]) / p;
    double K = exp(-ga * gb / p * (A[d] - B[d]) * (A[d] - B[d]));
    double fr[16], fi[16];
    for (int s = 0; s <= la + lb; ++s) gauss_ft1(s, p, q[d], &fr[s], &fi[s]);
    double cph = cos(-q[d] * P), sph = sin(-q[d] * P);
    for (int i = 0; i <= la; ++i)
      for (int j = 0; j <= lb; ++j) {
        double cs[16];
        product_poly(i, j, P - A[d], P - B[d], cs);
        double sr = 0.0, si = 0.0;
        for (int s = 0; s <= i + j; ++s) {
          sr += cs[s] * fr[s];
          si += cs[s] * fi[s];
        }
        tr[d][i][j] = K * (sr * cph - si * sph);
        ti[d][i][j] = K * (sr * sph + si * cph);
      }
  }
  int pa[64][3], pb[64][3];
  cart_powers(la, pa);
  cart_powers(lb, pb);
  for (int ia = 0; ia < ncart(la); ++ia)
    for (int ib = 0; ib < ncart(lb); ++ib) {
      double cr = 1.0, ci = 0.0;
      for (int d = 0; d < 3; ++d) {
        double xr = tr[d][pa[ia][d]][pb[ib][d]], xi = ti[d][pa[ia][d]][pb[ib][d]];
        double nr = cr * xr - ci * xi, ni = cr * xi + ci * xr;
        cr = nr;
        ci = ni;
      }
      out[2 * (ia * ncart(lb) + ib)] = cr;
      out[2 * (ia * ncart(lb) + ib) + 1] = ci;
    }
}

/* exported wrappers used by the pins */
int orc_prim_ft(int l, int comp, double g, const double *C, const double *q, double *reim) {
  int pw[64][3];
  if (l < 0 || l > 6 || comp < 0 || comp >= ncart(l)) return -1;
  cart_powers(l, pw);
  /* (x-C)^i e^{-g (x-C)^2}: shift y = x - C gives e^{-i q C} times the 1-D transform */
  double cr = 1.0, ci = 0.0;
  for (int d = 0; d < 3; ++d) {
    double fr, fi;
    gauss_ft1(pw[comp][d], g, q[d], &fr, &fi);
    double ph = -q[d] * C[d];
    double tr = fr * cos(ph) - fi * sin(ph), ti = fr * sin(ph) + fi * cos(ph);
    double nr = cr * tr - ci * ti, ni = cr * ti + ci * tr;
    cr = nr;
    ci = ni;
  }
  reim[0] = cr;
  reim[1] = ci;
  return 0;
}

int orc_pair_ft(int la, int ca, double ga, const double *A, int lb, int cb, double gb, const double *B,
                const double *q, double *reim) {
  int pa[64][3], pb[64][3];
  if (la < 0 || lb < 0 || la > 6 || lb > 6) return -1;
  cart_powers(la, pa);
  cart_powers(lb, pb);
  prim_pair_ft(pa[ca], ga, A, pb[cb], gb, B, q, &reim[0], &reim[1]);
  return 0;
}

double orc_overlap(int la, int ca, double ga, const double *A, int lb, int cb, double gb, const double *B) {
  int pa[64][3], pb[64][3];
  cart_powers(la, pa);
  cart_powers(lb, pb);
  return prim_overlap(pa[ca], ga, A, pb[cb], gb, B);
}

/* --------------------------------------------------------- periodic part */
typedef struct {
  int nshell;
  const int32_t *atom, *l, *nprim, *ptr;
  const double *exps, *coefs;
} orc_basis;

typedef struct {
  double a[3][3]; /* rows: lattice vectors (bohr) */
  double b[3][3]; /* rows: reciprocal vectors, a_i . b_j = 2 pi delta_ij */
  double vol;
} orc_lat;

static int make_lattice(const double *lat, orc_lat *L) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) L->a[i][j] = lat[3 * i + j];
  double (*a)[3] = L->a;
  double c0[3] = {a[1][1] * a[2][2] - a[1][2] * a[2][1], a[1][2] * a[2][0] - a[1][0] * a[2][2],
                  a[1][0] * a[2][1] - a[1][1] * a[2][0]};
  double det = a[0][0] * c0[0] + a[0][1] * c0[1] + a[0][2] * c0[2];
  if (!(fabs(det) > 1e-10)) return -1;
  L->vol = fabs(det);
  /* b_i = 2 pi (a_j x a_k)/det */
  double c1[3] = {a[2][1] * a[0][2] - a[2][2] * a[0][1], a[2][2] * a[0][0] - a[2][0] * a[0][2],
                  a[2][0] * a[0][1] - a[2][1] * a[0][0]};
  double c2[3] = {a[0][1] * a[1][2] - a[0][2] * a[1][1], a[0][2] * a[1][0] - a[0][0] * a[1][2],
                  a[0][0] * a[1][1] - a[0][1] * a[1][0]};
  for (int j = 0; j < 3; ++j) {
    L->b[0][j] = 2.0 * ORC_PI * c0[j] / det;
    L->b[1][j] = 2.0 * ORC_PI * c1[j] / det;
    L->b[2][j] = 2.0 * ORC_PI * c2[j] / det;
  }
  return 0;
}

static void lat_vec(const orc_lat *L, int n0, int n1, int n2, double *v) {
  for (int j = 0; j < 3; ++j) v[j] = n0 * L->a[0][j] + n1 * L->a[1][j] + n2 * L->a[2][j];
}

/* integer search half-width along a_i covering a sphere of radius R */
static int box_halfwidth(const orc_lat *L, int i, double R) {
  double bn = sqrt(L->b[i][0] * L->b[i][0] + L->b[i][1] * L->b[i][1] + L->b[i][2] * L->b[i][2]);
  return (int)ceil(R * bn / (2.0 * ORC_PI)) + 1;
}

/* 1s-type model of a primitive pair and aux primitive used by the oracle's
 * truncation rule: f(R) = [erf(eta1 R) - erf(eta2 R)]/R (Eq. S7), R -> 0 limit. */
static double f_sr(double R, double eta1, double eta2) {
  if (R < 1e-8) return 2.0 * (eta1 - eta2) / sqrt(ORC_PI);
  return (erf(eta1 * R) - erf(eta2 * R)) / R;
}

/* Function offsets of a basis (Cartesian). */
static int basis_offsets(const orc_basis *bs, int *off) {
  int n = 0;
  for (int s = 0; s < bs->nshell; ++s) {
    off[s] = n;
    n += ncart(bs->l[s]);
  }
  return n;
}

static void bvk_of(const int *mm, const int *kmesh, int *cidx) {
  int r[3];
  for (int d = 0; d < 3; ++d) {
    r[d] = mm[d] % kmesh[d];
    if (r[d] < 0) r[d] += kmesh[d];
  }
  *cidx = (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2];
}

/*
 * orc_j3c: the periodic three-center integrals.
 *   lattice[9], natm, coords[natm*3], basis/aux (shell arrays), kmesh[3],
 *   omega, cut   : per-term truncation cutoff of the oracle's own rule,
 *   g_thr        : keep q with exp(-q^2/4w^2) >= g_thr,
 *   parts        : bitmask ORC_PART_SR | ORC_PART_G0 | ORC_PART_LR, or
 *                  ORC_PART_M15 alone (the range-separation-free q sum),
 *   all_pairs    : 0 -> k-pairs k1<=k2 (row-major upper triangle),
 *                  1 -> all Nk^2 ordered pairs (k1 major),
 *   naux_sel, aux_sel : aux shells to compute (others left zero),
 *   npair_sel, pair_sel[2*npair_sel] : AO shell pairs (mu, nu) to compute
 *                  (npair_sel < 0 means all),
 *   nkp_sel, kp_sel[nkp_sel] : k-pair indices to compute (nkp_sel < 0 means all),
 *   out          : complex128 [nkpair][naux][nao][nao], interleaved re/im,
 *                  zero-filled by the caller,
 *   counts[2]    : SR primitive-triplet image terms, LR pair-FT evaluations.
 */
int orc_j3c(const double *lattice, int natm, const double *coords, int nbs, const int32_t *bs_atom,
            const int32_t *bs_l, const int32_t *bs_nprim, const int32_t *bs_ptr, const double *bs_exps,
            const double *bs_coefs, int nax, const int32_t *ax_atom, const int32_t *ax_l,
            const int32_t *ax_nprim, const int32_t *ax_ptr, const double *ax_exps, const double *ax_coefs,
            const int32_t *kmesh, double omega, double cut, double g_thr, int parts, int all_pairs,
            int naux_sel, const int32_t *aux_sel, int npair_sel, const int32_t *pair_sel, int nkp_sel,
            const int32_t *kp_sel, double *out, int64_t *counts) {
  orc_lat L;
  if (make_lattice(lattice, &L)) return -1;
  if (!(omega > 0.0) || !(cut > 0.0) || !(g_thr > 0.0)) return -1;
  for (int d = 0; d < 3; ++d)
    if (kmesh[d] < 1) return -1;
  orc_basis bs = {nbs, bs_atom, bs_l, bs_nprim, bs_ptr, bs_exps, bs_coefs};
  orc_basis ax = {nax, ax_atom, ax_l, ax_nprim, ax_ptr, ax_exps, ax_coefs};
  (void)natm;

  int *aoff = (int *)malloc(sizeof(int) * (nbs + 1));
  int *xoff = (int *)malloc(sizeof(int) * (nax + 1));
  const int nao = basis_offsets(&bs, aoff);
  const int naux = basis_offsets(&ax, xoff);
  const int nk = kmesh[0] * kmesh[1] * kmesh[2];

  /* k-points (Gamma-centred uniform mesh) and pairs */
  double *kv = (double *)malloc(sizeof(double) * 3 * nk);
  int *kj = (int *)malloc(sizeof(int) * 3 * nk);
  for (int j0 = 0; j0 < kmesh[0]; ++j0)
    for (int j1 = 0; j1 < kmesh[1]; ++j1)
      for (int j2 = 0; j2 < kmesh[2]; ++j2) {
        int k = (j0 * kmesh[1] + j1) * kmesh[2] + j2;
        kj[3 * k] = j0; kj[3 * k + 1] = j1; kj[3 * k + 2] = j2;
        for (int d = 0; d < 3; ++d)
          kv[3 * k + d] = (double)j0 / kmesh[0] * L.b[0][d] + (double)j1 / kmesh[1] * L.b[1][d] +
                          (double)j2 / kmesh[2] * L.b[2][d];
      }
  int nkp = all_pairs ? nk * nk : nk * (nk + 1) / 2;
  int *kp1 = (int *)malloc(sizeof(int) * nkp), *kp2 = (int *)malloc(sizeof(int) * nkp);
  {
    int t = 0;
    for (int k1 = 0; k1 < nk; ++k1)
      for (int k2 = all_pairs ? 0 : k1; k2 < nk; ++k2) {
        kp1[t] = k1; kp2[t] = k2; ++t;
      }
  }

  /* k-pair selection mask (unselected k-pairs stay zero) */
  char *kmask = (char *)calloc((size_t)nkp, 1);
  if (nkp_sel < 0) memset(kmask, 1, (size_t)nkp);
  else
    for (int i = 0; i < nkp_sel; ++i)
      if (kp_sel[i] >= 0 && kp_sel[i] < nkp) kmask[kp_sel[i]] = 1;

  /* pair selection mask */
  char *pmask = (char *)calloc((size_t)nbs * nbs, 1);
  if (npair_sel < 0) memset(pmask, 1, (size_t)nbs * nbs);
  else
    for (int i = 0; i < npair_sel; ++i) pmask[pair_sel[2 * i] * nbs + pair_sel[2 * i + 1]] = 1;

  const size_t plane = (size_t)naux * nao * nao; /* per k-pair, complex */
  int64_t nsr = 0, nlr = 0;
  int err = 0;

#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nsr) reduction(| : err)
  for (int isel = 0; isel < naux_sel; ++isel) {
    const int P = aux_sel[isel];
    const int lP = ax.l[P], ncP = ncart(lP);
    int pwP[64][3];
    cart_powers(lP, pwP);
    const double *C = coords + 3 * ax.atom[P];

    for (int mu = 0; mu < nbs; ++mu)
      for (int nu = 0; nu < nbs; ++nu) {
        if (!pmask[mu * nbs + nu]) continue;
        const int la = bs.l[mu], lb = bs.l[nu], nca = ncart(la), ncb = ncart(lb);
        const double *A = coords + 3 * bs.atom[mu], *B0 = coords + 3 * bs.atom[nu];
        int pwa[64][3], pwb[64][3];
        cart_powers(la, pwa);
        cart_powers(lb, pwb);
        const int blk = ncP * nca * ncb;

        /* ---------------- SR lattice sum (Eq. M12 first term, M13a, M14) */
        if (parts & ORC_PART_SR) {
          double *X = (double *)calloc((size_t)nk * nk * blk, sizeof(double));
          double *tmp = (double *)malloc(sizeof(double) * blk);
          for (int kP = 0; kP < ax.nprim[P]; ++kP)
            for (int ka = 0; ka < bs.nprim[mu]; ++ka)
              for (int kb = 0; kb < bs.nprim[nu]; ++kb) {
                const double gP = ax.exps[ax.ptr[P] + kP], cP = ax.coefs[ax.ptr[P] + kP];
                const double ga = bs.exps[bs.ptr[mu] + ka], ca = bs.coefs[bs.ptr[mu] + ka];
                const double gb = bs.exps[bs.ptr[nu] + kb], cb = bs.coefs[bs.ptr[nu] + kb];
                const double p = ga + gb, beta = ga * gb / p;
                const double Aest = fabs(cP * ca * cb) * pow(ORC_PI, 3) / pow(gP * p, 1.5);
                const double eta1 = sqrt(gP * p / (gP + p));
                const double eta2 = 1.0 / sqrt(1.0 / (eta1 * eta1) + 1.0 / (omega * omega));
                /* radius on R_c beyond which the 1s model with polynomial growth
                 * stays below cut for any pair factor <= 1 */
                double Fstar = 0.0, Rcmax0 = 0.0;
                for (double R = 0.0; R < 1000.0; R += 0.25) {
                  double v = f_sr(R, eta1, eta2) * pow(1.0 + R, lP);
                  if (v > Fstar) Fstar = v;
                  if (Aest * v >= cut) Rcmax0 = R + 0.25;
                  if (R > 1.0 && Aest * v < 1e-3 * cut && v < Fstar) break;
                }
                double R12max = 0.0;
                for (double R = 0.0; R < 1000.0; R += 0.25) {
                  double h = exp(-beta * R * R) * pow(1.0 + R, la + lb);
                  if (Aest * h * Fstar >= cut) R12max = R + 0.25;
                  if (R * R * beta > 50.0 && Aest * h * Fstar < 1e-3 * cut) break;
                }
                const int w0 = box_halfwidth(&L, 0, R12max + 1e-9), w1 = box_halfwidth(&L, 1, R12max),
                          w2 = box_halfwidth(&L, 2, R12max);
                for (int n0 = -w0; n0 <= w0; ++n0)
                  for (int n1 = -w1; n1 <= w1; ++n1)
                    for (int n2 = -w2; n2 <= w2; ++n2) {
                      double nv[3], B[3], ABv[3];
                      lat_vec(&L, n0, n1, n2, nv);
                      double r12 = 0.0;
                      for (int d = 0; d < 3; ++d) {
                        B[d] = B0[d] + nv[d];
                        ABv[d] = A[d] - B[d];
                        r12 += ABv[d] * ABv[d];
                      }
                      r12 = sqrt(r12);
                      const double hfac = exp(-beta * r12 * r12) * pow(1.0 + r12, la + lb);
                      if (Aest * hfac * Fstar < cut) continue;
                      double Pc[3];
                      for (int d = 0; d < 3; ++d) Pc[d] = (ga * A[d] + gb * B[d]) / p;
                      const double Rm = Rcmax0;
                      const int v0 = box_halfwidth(&L, 0, Rm), v1 = box_halfwidth(&L, 1, Rm),
                                v2 = box_halfwidth(&L, 2, Rm);
                      /* nearest lattice point to C - Pc in fractional coordinates */
                      double dfrac[3];
                      for (int i = 0; i < 3; ++i) {
                        double s = 0.0;
                        for (int d = 0; d < 3; ++d) s += (C[d] - Pc[d]) * L.b[i][d];
                        dfrac[i] = s / (2.0 * ORC_PI);
                      }
                      const int c0 = (int)lround(dfrac[0]), c1 = (int)lround(dfrac[1]), c2 = (int)lround(dfrac[2]);
                      for (int m0 = c0 - v0; m0 <= c0 + v0; ++m0)
                        for (int m1 = c1 - v1; m1 <= c1 + v1; ++m1)
                          for (int m2 = c2 - v2; m2 <= c2 + v2; ++m2) {
                            /* term (P^0 | mu^m nu^{m+n'}) == (P^{-m} | mu^0 nu^{n'}): aux at C - m */
                            double mv[3], Cm[3], rc = 0.0;
                            lat_vec(&L, m0, m1, m2, mv);
                            for (int d = 0; d < 3; ++d) {
                              Cm[d] = C[d] - mv[d];
                              rc += (Pc[d] - Cm[d]) * (Pc[d] - Cm[d]);
                            }
                            rc = sqrt(rc);
                            if (rc > Rm) continue;
                            if (Aest * hfac * f_sr(rc, eta1, eta2) * pow(1.0 + rc, lP) < cut) continue;
                            if (orc_prim3c(ORC_ERFC, omega, lP, gP, Cm, la, ga, A, lb, gb, B, tmp)) {
                              err = 1;
                              continue;
                            }
                            ++nsr;
                            int mm[3] = {m0, m1, m2}, nn[3] = {m0 + n0, m1 + n1, m2 + n2}, cm, cn;
                            bvk_of(mm, kmesh, &cm);
                            bvk_of(nn, kmesh, &cn);
                            double *Xb = X + ((size_t)cm * nk + cn) * blk;
                            const double cc = cP * ca * cb;
                            for (int t = 0; t < blk; ++t) Xb[t] += cc * tmp[t];
                          }
                    }
              }
          /* direct double DFT over the BvK cells (Eq. M14) */
          for (int t = 0; t < nkp; ++t) {
            if (!kmask[t]) continue;
            const int k1 = kp1[t], k2 = kp2[t];
            for (int cm = 0; cm < nk; ++cm)
              for (int cn = 0; cn < nk; ++cn) {
                int im0 = cm / (kmesh[1] * kmesh[2]), im1 = (cm / kmesh[2]) % kmesh[1], im2 = cm % kmesh[2];
                int in0 = cn / (kmesh[1] * kmesh[2]), in1 = (cn / kmesh[2]) % kmesh[1], in2 = cn % kmesh[2];
                double ph = 2.0 * ORC_PI *
                            (-((double)kj[3 * k1] * im0 / kmesh[0] + (double)kj[3 * k1 + 1] * im1 / kmesh[1] +
                               (double)kj[3 * k1 + 2] * im2 / kmesh[2]) +
                             ((double)kj[3 * k2] * in0 / kmesh[0] + (double)kj[3 * k2 + 1] * in1 / kmesh[1] +
                              (double)kj[3 * k2 + 2] * in2 / kmesh[2]));
                const double cr = cos(ph), ci = sin(ph);
                const double *Xb = X + ((size_t)cm * nk + cn) * blk;
                for (int ic = 0; ic < ncP; ++ic)
                  for (int ia = 0; ia < nca; ++ia)
                    for (int ib = 0; ib < ncb; ++ib) {
                      double v = Xb[(ic * nca + ia) * ncb + ib];
                      size_t o = (size_t)t * plane + ((size_t)(xoff[P] + ic) * nao + aoff[mu] + ia) * nao + aoff[nu] + ib;
                      out[2 * o] += cr * v;
                      out[2 * o + 1] += ci * v;
                    }
              }
          }
          free(X);
          free(tmp);
        }

        /* ---------------- G = 0 correction on k1 == k2 (Eq. M12, M13b-c) */
        if (parts & ORC_PART_G0) {
          for (int t = 0; t < nkp; ++t) {
            if (kp1[t] != kp2[t] || !kmask[t]) continue;
            const double *k = kv + 3 * kp1[t];
            for (int ic = 0; ic < ncP; ++ic) {
              double SP = 0.0;
              for (int kP = 0; kP < ax.nprim[P]; ++kP) {
                double g = ax.exps[ax.ptr[P] + kP];
                double s = ax.coefs[ax.ptr[P] + kP];
                for (int d = 0; d < 3; ++d) s *= gauss_moment(pwP[ic][d], g);
                SP += s;
              }
              if (SP == 0.0) continue;
              for (int ia = 0; ia < nca; ++ia)
                for (int ib = 0; ib < ncb; ++ib) {
                  double sr = 0.0, si = 0.0;
                  for (int ka = 0; ka < bs.nprim[mu]; ++ka)
                    for (int kb = 0; kb < bs.nprim[nu]; ++kb) {
                      const double ga = bs.exps[bs.ptr[mu] + ka], ca = bs.coefs[bs.ptr[mu] + ka];
                      const double gb = bs.exps[bs.ptr[nu] + kb], cb = bs.coefs[bs.ptr[nu] + kb];
                      const double beta = ga * gb / (ga + gb);
                      const double Rcut = sqrt(40.0 / beta) + 10.0;
                      const int w0 = box_halfwidth(&L, 0, Rcut), w1 = box_halfwidth(&L, 1, Rcut),
                                w2 = box_halfwidth(&L, 2, Rcut);
                      for (int n0 = -w0; n0 <= w0; ++n0)
                        for (int n1 = -w1; n1 <= w1; ++n1)
                          for (int n2 = -w2; n2 <= w2; ++n2) {
                            double nv[3], B[3], r2 = 0.0;
                            lat_vec(&L, n0, n1, n2, nv);
                            for (int d = 0; d < 3; ++d) {
                              B[d] = B0[d] + nv[d];
                              r2 += (A[d] - B[d]) * (A[d] - B[d]);
                            }
                            if (beta * r2 > 60.0) continue;
                            double s = ca * cb * prim_overlap(pwa[ia], ga, A, pwb[ib], gb, B);
                            double ph = k[0] * nv[0] + k[1] * nv[1] + k[2] * nv[2];
                            sr += cos(ph) * s;
                            si += sin(ph) * s;
                          }
                    }
                  const double fac = ORC_PI / (L.vol * omega * omega) * SP;
                  size_t o = (size_t)t * plane + ((size_t)(xoff[P] + ic) * nao + aoff[mu] + ia) * nao + aoff[nu] + ib;
                  out[2 * o] -= fac * sr;
                  out[2 * o + 1] -= fac * si;
                }
            }
          }
        }

      }
  }

  /* ---------------- LR reciprocal-space sum (Eq. M10, M11), one AO shell
   * pair per task so each pair transform is evaluated once for all aux shells.
   * With ORC_PART_M15 instead, the same q sum without range separation
   * (Eq. M15): weight 4 pi/(Omega q^2) with no Gaussian damping; omega and
   * g_thr then only fix the q sphere (exp(-q^2/4w^2) >= g_thr), which the
   * caller makes large enough for the transforms to have decayed. */
  const int m15 = (parts & ORC_PART_M15) != 0;
  if (m15 && (parts & ORC_PART_LR)) err = 1;
  if ((parts & (ORC_PART_LR | ORC_PART_M15)) && !err) {
    const double q2max = -4.0 * omega * omega * log(g_thr);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nlr)
    for (int pr = 0; pr < nbs * nbs; ++pr) {
      const int mu = pr / nbs, nu = pr % nbs;
      if (!pmask[mu * nbs + nu]) continue;
      const int la = bs.l[mu], lb = bs.l[nu], nca = ncart(la), ncb = ncart(lb);
      const int npa = bs.nprim[mu], npb = bs.nprim[nu];
      const double *A = coords + 3 * bs.atom[mu], *B0 = coords + 3 * bs.atom[nu];
      /* images n kept per primitive pair: prefactor above 1e-18 */
      int *nimg = (int *)calloc((size_t)npa * npb, sizeof(int));
      double **imgs = (double **)calloc((size_t)npa * npb, sizeof(double *));
      for (int ka = 0; ka < npa; ++ka)
        for (int kb = 0; kb < npb; ++kb) {
          const double ga = bs.exps[bs.ptr[mu] + ka], ca = bs.coefs[bs.ptr[mu] + ka];
          const double gb = bs.exps[bs.ptr[nu] + kb], cb = bs.coefs[bs.ptr[nu] + kb];
          const double pp = ga + gb, beta = ga * gb / pp;
          const double pre = fabs(ca * cb) * pow(ORC_PI / pp, 1.5);
          const double Rcut = sqrt(60.0 / beta) + 10.0;
          const int w0 = box_halfwidth(&L, 0, Rcut), w1 = box_halfwidth(&L, 1, Rcut), w2 = box_halfwidth(&L, 2, Rcut);
          double *lst = (double *)malloc(sizeof(double) * 3 * (2 * w0 + 1) * (2 * w1 + 1) * (2 * w2 + 1));
          int cnt = 0;
          for (int n0 = -w0; n0 <= w0; ++n0)
            for (int n1 = -w1; n1 <= w1; ++n1)
              for (int n2 = -w2; n2 <= w2; ++n2) {
                double nv[3], r2 = 0.0;
                lat_vec(&L, n0, n1, n2, nv);
                for (int d = 0; d < 3; ++d) r2 += (A[d] - B0[d] - nv[d]) * (A[d] - B0[d] - nv[d]);
                if (pre * exp(-beta * r2) * pow(1.0 + sqrt(r2), la + lb) < 1e-18) continue;
                for (int d = 0; d < 3; ++d) lst[3 * cnt + d] = nv[d];
                ++cnt;
              }
          nimg[ka * npb + kb] = cnt;
          imgs[ka * npb + kb] = lst;
        }
      double *rho = (double *)malloc(sizeof(double) * 2 * nca * ncb);
      double *blk = (double *)malloc(sizeof(double) * 2 * nca * ncb);
      for (int t = 0; t < nkp; ++t) {
        if (!kmask[t]) continue;
        const double *k1v = kv + 3 * kp1[t], *k2v = kv + 3 * kp2[t];
        double k12[3];
        for (int d = 0; d < 3; ++d) k12[d] = k2v[d] - k1v[d];
        const double qm = sqrt(q2max) + sqrt(k12[0] * k12[0] + k12[1] * k12[1] + k12[2] * k12[2]);
        /* G range: |g_i| <= qm |a_i| / (2 pi) + 1 */
        int gw[3];
        for (int i = 0; i < 3; ++i) {
          double an = sqrt(L.a[i][0] * L.a[i][0] + L.a[i][1] * L.a[i][1] + L.a[i][2] * L.a[i][2]);
          gw[i] = (int)ceil(qm * an / (2.0 * ORC_PI)) + 1;
        }
        for (int g0i = -gw[0]; g0i <= gw[0]; ++g0i)
          for (int g1i = -gw[1]; g1i <= gw[1]; ++g1i)
            for (int g2i = -gw[2]; g2i <= gw[2]; ++g2i) {
              double q[3], q2 = 0.0;
              for (int d = 0; d < 3; ++d) {
                q[d] = g0i * L.b[0][d] + g1i * L.b[1][d] + g2i * L.b[2][d] + k12[d];
                q2 += q[d] * q[d];
              }
              if (q2 < 1e-20) continue; /* the q = 0 term is excluded */
              const double damp = exp(-q2 / (4.0 * omega * omega));
              if (damp < g_thr) continue;
              const double wgt = 4.0 * ORC_PI / L.vol * (m15 ? 1.0 : damp) / q2;
              /* rho^^{k2}_{mu nu}(q) = sum_n e^{+i k2.n} int phi_mu(r) phi_nu(r-n) e^{-iq.r} dr */
              for (int x = 0; x < 2 * nca * ncb; ++x) rho[x] = 0.0;
              for (int ka = 0; ka < npa; ++ka)
                for (int kb = 0; kb < npb; ++kb) {
                  const double ga = bs.exps[bs.ptr[mu] + ka], ca = bs.coefs[bs.ptr[mu] + ka];
                  const double gb = bs.exps[bs.ptr[nu] + kb], cb = bs.coefs[bs.ptr[nu] + kb];
                  const double *lst = imgs[ka * npb + kb];
                  for (int ii = 0; ii < nimg[ka * npb + kb]; ++ii) {
                    const double *nv = lst + 3 * ii;
                    double B[3] = {B0[0] + nv[0], B0[1] + nv[1], B0[2] + nv[2]};
                    prim_pair_ft_block(la, ga, A, lb, gb, B, q, blk);
                    ++nlr;
                    double ph = k2v[0] * nv[0] + k2v[1] * nv[1] + k2v[2] * nv[2];
                    double cr = ca * cb * cos(ph), ci = ca * cb * sin(ph);
                    for (int x = 0; x < nca * ncb; ++x) {
                      rho[2 * x] += cr * blk[2 * x] - ci * blk[2 * x + 1];
                      rho[2 * x + 1] += cr * blk[2 * x + 1] + ci * blk[2 * x];
                    }
                  }
                }
              double mq[3] = {-q[0], -q[1], -q[2]};
              for (int isel = 0; isel < naux_sel; ++isel) {
                const int P = aux_sel[isel];
                const int lP = ax.l[P], ncP = ncart(lP);
                const double *C = coords + 3 * ax.atom[P];
                for (int ic = 0; ic < ncP; ++ic) {
                  /* chi~_P(-q) */
                  double xr = 0.0, xi = 0.0;
                  for (int kP = 0; kP < ax.nprim[P]; ++kP) {
                    double reim[2];
                    orc_prim_ft(lP, ic, ax.exps[ax.ptr[P] + kP], C, mq, reim);
                    xr += ax.coefs[ax.ptr[P] + kP] * reim[0];
                    xi += ax.coefs[ax.ptr[P] + kP] * reim[1];
                  }
                  const double Ar = wgt * xr, Ai = wgt * xi;
                  for (int ia = 0; ia < nca; ++ia)
                    for (int ib = 0; ib < ncb; ++ib) {
                      const double rr = rho[2 * (ia * ncb + ib)], ri = rho[2 * (ia * ncb + ib) + 1];
                      size_t o = (size_t)t * plane + ((size_t)(xoff[P] + ic) * nao + aoff[mu] + ia) * nao + aoff[nu] + ib;
                      out[2 * o] += Ar * rr - Ai * ri;
                      out[2 * o + 1] += Ar * ri + Ai * rr;
                    }
                }
              }
            }
      }
      free(rho);
      free(blk);
      for (int x = 0; x < npa * npb; ++x) free(imgs[x]);
      free(imgs);
      free(nimg);
    }
  }

  if (counts) {
    counts[0] = nsr;
    counts[1] = nlr;
  }
  free(aoff); free(xoff); free(kv); free(kj); free(kp1); free(kp2); free(pmask); free(kmask);
  return err ? -2 : 0;
}

/*
 * orc_j2c: the two-center metric of the density fit, Eq. M5,
 *   J^k_PQ = (chi_P^{k*} | 1/r | chi_Q^k) = sum_m e^{+ik.m} (P^0 | 1/r | Q^m)
 * with the q = 0 (G = 0 at k = 0) component removed, evaluated with the
 * range separation of Eq. M9 exactly as the three-center integrals:
 *   SR = sum_m e^{+ik.m} (P^0 | erfc(w r)/r | Q^m)
 *   G0 = delta_{k0} pi/(Omega w^2) S_P S_Q
 *   LR = (4 pi/Omega) sum_{q=G+k, q!=0, exp(-q^2/4w^2)>=gthr}
 *          exp(-q^2/4w^2)/q^2 chi~_P(-q) chi~_Q(q)
 *   J = SR - G0 + LR   (ORC_PART_M15 alone: the plain q sum with 4 pi/(Omega q^2)).
 * The two-center primitive integral is the three-center one of orc_prim3c
 * with the second orbital factor set to the constant 1 (exponent 0, l = 0),
 * which its recurrences admit exactly.
 * Truncation (oracle's own rule): a term (P prim, Q prim, m) is kept while
 * |c_P c_Q| pi^3/(a_P a_Q)^{3/2} f(R; eta1, eta2) (1+R)^{l_P+l_Q} >= cut,
 * eta1 = sqrt(a_P a_Q/(a_P+a_Q)).
 *   out: complex128 [nk][naux][naux] (k in mesh order), zero-filled by the caller.
 */
int orc_j2c(const double *lattice, int natm, const double *coords, int nax, const int32_t *ax_atom,
            const int32_t *ax_l, const int32_t *ax_nprim, const int32_t *ax_ptr, const double *ax_exps,
            const double *ax_coefs, const int32_t *kmesh, double omega, double cut, double g_thr, int parts,
            double *out, int64_t *counts) {
  orc_lat L;
  if (make_lattice(lattice, &L)) return -1;
  if (!(omega > 0.0) || !(cut > 0.0) || !(g_thr > 0.0)) return -1;
  for (int d = 0; d < 3; ++d)
    if (kmesh[d] < 1) return -1;
  const int m15 = (parts & ORC_PART_M15) != 0;
  if (m15 && (parts & (ORC_PART_LR | ORC_PART_SR | ORC_PART_G0))) return -1;
  (void)natm;
  orc_basis ax = {nax, ax_atom, ax_l, ax_nprim, ax_ptr, ax_exps, ax_coefs};
  int *xoff = (int *)malloc(sizeof(int) * (nax + 1));
  const int naux = basis_offsets(&ax, xoff);
  const int nk = kmesh[0] * kmesh[1] * kmesh[2];
  double *kv = (double *)malloc(sizeof(double) * 3 * nk);
  int *kj = (int *)malloc(sizeof(int) * 3 * nk);
  for (int j0 = 0; j0 < kmesh[0]; ++j0)
    for (int j1 = 0; j1 < kmesh[1]; ++j1)
      for (int j2 = 0; j2 < kmesh[2]; ++j2) {
        int k = (j0 * kmesh[1] + j1) * kmesh[2] + j2;
        kj[3 * k] = j0; kj[3 * k + 1] = j1; kj[3 * k + 2] = j2;
        for (int d = 0; d < 3; ++d)
          kv[3 * k + d] = (double)j0 / kmesh[0] * L.b[0][d] + (double)j1 / kmesh[1] * L.b[1][d] +
                          (double)j2 / kmesh[2] * L.b[2][d];
      }
  const size_t plane = (size_t)naux * naux;
  int64_t nsr = 0, nlr = 0;
  int err = 0;

  /* ---- SR lattice sum: X[c(m)] then the DFT over the BvK cells */
  if (parts & ORC_PART_SR) {
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nsr) reduction(| : err)
    for (int pq = 0; pq < nax * nax; ++pq) {
      const int P = pq / nax, Q = pq % nax;
      const int lP = ax.l[P], lQ = ax.l[Q], ncP = ncart(lP), ncQ = ncart(lQ), blk = ncP * ncQ;
      const double *C = coords + 3 * ax.atom[P], *B0 = coords + 3 * ax.atom[Q];
      double *X = (double *)calloc((size_t)nk * blk, sizeof(double));
      double tmp[100];
      for (int iP = 0; iP < ax.nprim[P]; ++iP)
        for (int iQ = 0; iQ < ax.nprim[Q]; ++iQ) {
          const double gP = ax.exps[ax.ptr[P] + iP], cP = ax.coefs[ax.ptr[P] + iP];
          const double gQ = ax.exps[ax.ptr[Q] + iQ], cQ = ax.coefs[ax.ptr[Q] + iQ];
          const double Aest = fabs(cP * cQ) * pow(ORC_PI, 3) / pow(gP * gQ, 1.5);
          const double eta1 = sqrt(gP * gQ / (gP + gQ));
          const double eta2 = 1.0 / sqrt(1.0 / (eta1 * eta1) + 1.0 / (omega * omega));
          double Fstar = 0.0, Rmax = 0.0;
          for (double R = 0.0; R < 1000.0; R += 0.25) {
            double v = f_sr(R, eta1, eta2) * pow(1.0 + R, lP + lQ);
            if (v > Fstar) Fstar = v;
            if (Aest * v >= cut) Rmax = R + 0.25;
            if (R > 1.0 && Aest * v < 1e-3 * cut && v < Fstar) break;
          }
          /* lattice vectors m with |B0 + m - C| <= Rmax */
          double dfrac[3];
          for (int i = 0; i < 3; ++i) {
            double t = 0.0;
            for (int d = 0; d < 3; ++d) t += (C[d] - B0[d]) * L.b[i][d];
            dfrac[i] = t / (2.0 * ORC_PI);
          }
          const int c0 = (int)lround(dfrac[0]), c1 = (int)lround(dfrac[1]), c2 = (int)lround(dfrac[2]);
          const int v0 = box_halfwidth(&L, 0, Rmax), v1 = box_halfwidth(&L, 1, Rmax), v2 = box_halfwidth(&L, 2, Rmax);
          for (int m0 = c0 - v0; m0 <= c0 + v0; ++m0)
            for (int m1 = c1 - v1; m1 <= c1 + v1; ++m1)
              for (int m2 = c2 - v2; m2 <= c2 + v2; ++m2) {
                double mv[3], Bm[3], r = 0.0;
                lat_vec(&L, m0, m1, m2, mv);
                for (int d = 0; d < 3; ++d) {
                  Bm[d] = B0[d] + mv[d];
                  r += (Bm[d] - C[d]) * (Bm[d] - C[d]);
                }
                r = sqrt(r);
                if (r > Rmax) continue;
                if (Aest * f_sr(r, eta1, eta2) * pow(1.0 + r, lP + lQ) < cut) continue;
                /* (P^0 | erfc | Q^m): aux P as the "c" centre, Q^m as orbital a, b = 1 */
                if (orc_prim3c(ORC_ERFC, omega, lP, gP, C, lQ, gQ, Bm, 0, 0.0, Bm, tmp)) {
                  err = 1;
                  continue;
                }
                ++nsr;
                int mm[3] = {m0, m1, m2}, cm;
                bvk_of(mm, kmesh, &cm);
                for (int t = 0; t < blk; ++t) X[(size_t)cm * blk + t] += cP * cQ * tmp[t];
              }
        }
      /* J^k += sum_c e^{+ik.L_c} X[c] */
      for (int k = 0; k < nk; ++k)
        for (int c = 0; c < nk; ++c) {
          int i0 = c / (kmesh[1] * kmesh[2]), i1 = (c / kmesh[2]) % kmesh[1], i2 = c % kmesh[2];
          double ph = 2.0 * ORC_PI * ((double)kj[3 * k] * i0 / kmesh[0] + (double)kj[3 * k + 1] * i1 / kmesh[1] +
                                      (double)kj[3 * k + 2] * i2 / kmesh[2]);
          const double cr = cos(ph), ci = sin(ph);
          for (int iP = 0; iP < ncP; ++iP)
            for (int iQ = 0; iQ < ncQ; ++iQ) {
              double v = X[(size_t)c * blk + iP * ncQ + iQ];
              size_t o = (size_t)k * plane + (size_t)(xoff[P] + iP) * naux + xoff[Q] + iQ;
              out[2 * o] += cr * v;
              out[2 * o + 1] += ci * v;
            }
        }
      free(X);
    }
  }

  /* ---- G = 0 term at k = 0 (k index 0 is Gamma) */
  if (parts & ORC_PART_G0) {
    for (int P = 0; P < nax; ++P)
      for (int Q = 0; Q < nax; ++Q) {
        int pwP[64][3], pwQ[64][3];
        cart_powers(ax.l[P], pwP);
        cart_powers(ax.l[Q], pwQ);
        for (int iP = 0; iP < ncart(ax.l[P]); ++iP)
          for (int iQ = 0; iQ < ncart(ax.l[Q]); ++iQ) {
            double SP = 0.0, SQ = 0.0;
            for (int i = 0; i < ax.nprim[P]; ++i) {
              double t = ax.coefs[ax.ptr[P] + i];
              for (int d = 0; d < 3; ++d) t *= gauss_moment(pwP[iP][d], ax.exps[ax.ptr[P] + i]);
              SP += t;
            }
            for (int i = 0; i < ax.nprim[Q]; ++i) {
              double t = ax.coefs[ax.ptr[Q] + i];
              for (int d = 0; d < 3; ++d) t *= gauss_moment(pwQ[iQ][d], ax.exps[ax.ptr[Q] + i]);
              SQ += t;
            }
            size_t o = (size_t)(xoff[P] + iP) * naux + xoff[Q] + iQ;
            out[2 * o] -= ORC_PI / (L.vol * omega * omega) * SP * SQ;
          }
      }
  }

  /* ---- LR (or the range-separation-free sum): q = G + k */
  if (parts & (ORC_PART_LR | ORC_PART_M15)) {
    const double q2max = -4.0 * omega * omega * log(g_thr);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nlr)
    for (int k = 0; k < nk; ++k) {
      const double *kk = kv + 3 * k;
      const double qm = sqrt(q2max) + sqrt(kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2]);
      int gw[3];
      for (int i = 0; i < 3; ++i) {
        double an = sqrt(L.a[i][0] * L.a[i][0] + L.a[i][1] * L.a[i][1] + L.a[i][2] * L.a[i][2]);
        gw[i] = (int)ceil(qm * an / (2.0 * ORC_PI)) + 1;
      }
      double *ft = (double *)malloc(sizeof(double) * 4 * naux); /* chi~(-q), chi~(+q) */
      for (int g0i = -gw[0]; g0i <= gw[0]; ++g0i)
        for (int g1i = -gw[1]; g1i <= gw[1]; ++g1i)
          for (int g2i = -gw[2]; g2i <= gw[2]; ++g2i) {
            double q[3], mq[3], q2 = 0.0;
            for (int d = 0; d < 3; ++d) {
              q[d] = g0i * L.b[0][d] + g1i * L.b[1][d] + g2i * L.b[2][d] + kk[d];
              mq[d] = -q[d];
              q2 += q[d] * q[d];
            }
            if (q2 < 1e-20) continue;
            const double damp = exp(-q2 / (4.0 * omega * omega));
            if (damp < g_thr) continue;
            const double wgt = 4.0 * ORC_PI / L.vol * (m15 ? 1.0 : damp) / q2;
            ++nlr;
            for (int P = 0; P < nax; ++P)
              for (int iP = 0; iP < ncart(ax.l[P]); ++iP) {
                double am[2] = {0.0, 0.0}, ap[2] = {0.0, 0.0};
                for (int i = 0; i < ax.nprim[P]; ++i) {
                  double r1[2], r2[2];
                  orc_prim_ft(ax.l[P], iP, ax.exps[ax.ptr[P] + i], coords + 3 * ax.atom[P], mq, r1);
                  orc_prim_ft(ax.l[P], iP, ax.exps[ax.ptr[P] + i], coords + 3 * ax.atom[P], q, r2);
                  am[0] += ax.coefs[ax.ptr[P] + i] * r1[0];
                  am[1] += ax.coefs[ax.ptr[P] + i] * r1[1];
                  ap[0] += ax.coefs[ax.ptr[P] + i] * r2[0];
                  ap[1] += ax.coefs[ax.ptr[P] + i] * r2[1];
                }
                const int f = xoff[P] + iP;
                ft[4 * f] = am[0]; ft[4 * f + 1] = am[1]; ft[4 * f + 2] = ap[0]; ft[4 * f + 3] = ap[1];
              }
            for (int a = 0; a < naux; ++a)
              for (int b = 0; b < naux; ++b) {
                const double xr = ft[4 * a], xi = ft[4 * a + 1], yr = ft[4 * b + 2], yi = ft[4 * b + 3];
                size_t o = (size_t)k * plane + (size_t)a * naux + b;
                out[2 * o] += wgt * (xr * yr - xi * yi);
                out[2 * o + 1] += wgt * (xr * yi + xi * yr);
              }
          }
      free(ft);
    }
  }
  if (counts) {
    counts[0] = nsr;
    counts[1] = nlr;
  }
  free(xoff); free(kv); free(kj);
  return err ? -2 : 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
