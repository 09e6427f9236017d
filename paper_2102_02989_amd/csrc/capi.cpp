// capi.cpp -- C ABI and host planner of librsgdf (see include/rsgdf.h).
//
// The planner packs the bases, builds the lattice / k-mesh / Born-von Karman
// tables, evaluates the short-range screening bounds of the Supplementary
// Material per (aux shell, AO shell pair) (Eqs. S14, S15, S19, S23-S25),
// enumerates the pair lattice images, builds the G-vector sets of the
// long-range part per folded k12 (Eq. M10), uploads these tables and runs
// the kernels on the caller's stream:
//   per aux batch:  sr3c (SR lattice sums into BvK bins) -> fold (+ G = 0 term)
//   then:           aux transforms, per k12 class and q chunk: pair transforms
//                   -> G-space contraction accumulated into the output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rsgdf.h"
#include "kernels.h"
#include "learned.h"
#include "plan.h"

using namespace rsgdf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(RSGDF_EHIP, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
  } while (0)

// Bump allocator over caller-provided device memory (the no-allocation entry
// point's static scratch array).  While a thread has one installed, DBuf
// takes its memory from it and never calls hipMalloc or hipFree.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0, want = 0;  // want: bytes requested in all (for the error message)
  bool overflow = false;
};
thread_local Arena *t_arena = nullptr;

// Cache of large device blocks across builds.  A hipMalloc or hipFree of a
// buffer of tens of GB takes from under a millisecond to over a second (the
// long ones measured right after a large free), so the blocks of a build from
// kCacheMin bytes on go to an idle list when the build ends and the next
// request that fits reuses them: the smallest idle block of the current
// device that holds the request and wastes at most a quarter of itself.  Idle
// blocks beyond 40% of the device's memory are freed at once (oldest first),
// all of a device's when an allocation on it fails, and all by
// rsgdf_release_cache().  The budgets that follow the free memory count the
// idle blocks as free, and the part of a reused block beyond its request, so
// the planning of a build does not depend on the cache.
constexpr size_t kCacheMin = (size_t)64 << 20;
constexpr int kCacheDevs = 64;
struct CacheBlk {
  int dev;
  void *p;
  size_t n;
};
std::mutex g_cache_mu;
std::vector<CacheBlk> g_cache;          // idle blocks, oldest first
size_t g_cache_slack[kCacheDevs] = {};  // bytes of live reused blocks beyond their requests

size_t cache_idle_locked(int dev) {
  size_t b = 0;
  for (const CacheBlk &c : g_cache)
    if (c.dev == dev) b += c.n;
  return b;
}
// free the oldest idle blocks of dev until at most keep bytes stay idle
void cache_trim_locked(int dev, size_t keep) {
  size_t idle = cache_idle_locked(dev);
  for (size_t i = 0; i < g_cache.size() && idle > keep;) {
    if (g_cache[i].dev != dev) {
      ++i;
      continue;
    }
    (void)hipFree(g_cache[i].p);
    idle -= g_cache[i].n;
    g_cache.erase(g_cache.begin() + (std::ptrdiff_t)i);
  }
}
// idle bytes plus the slack of live reused blocks of the current device
size_t cache_free_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return cache_idle_locked(dev) + (dev >= 0 && dev < kCacheDevs ? g_cache_slack[dev] : 0);
}
// a block of at least bytes; *got = its size
hipError_t dev_alloc(void **p, size_t bytes, size_t *got) {
  *got = bytes;
  if (bytes < kCacheMin) return hipMalloc(p, bytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (size_t i = 0; i < g_cache.size(); ++i) {
      const CacheBlk &c = g_cache[i];
      if (c.dev == dev && c.n >= bytes && c.n - bytes <= c.n / 4 && (best < 0 || c.n < g_cache[best].n))
        best = (int)i;
    }
    if (best >= 0) {
      *p = g_cache[best].p;
      *got = g_cache[best].n;
      if (dev >= 0 && dev < kCacheDevs) g_cache_slack[dev] += *got - bytes;
      g_cache.erase(g_cache.begin() + best);
      return hipSuccess;
    }
  }
  e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      cache_trim_locked(dev, 0);
    }
    e = hipMalloc(p, bytes);
  }
  return e;
}
// give a block back: small ones are freed, large ones kept idle.  Like
// hipFree, this first waits for the device, so no kernel still uses the block
// when the next request takes it.
void dev_release(void *p, size_t n, size_t req) {
  if (n < kCacheMin) {
    (void)hipFree(p);
    return;
  }
  int dev = 0;
  size_t fr = 0, tot = 0;
  const bool ok = hipGetDevice(&dev) == hipSuccess && hipDeviceSynchronize() == hipSuccess &&
                  hipMemGetInfo(&fr, &tot) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (dev >= 0 && dev < kCacheDevs) g_cache_slack[dev] -= std::min(g_cache_slack[dev], n - std::min(n, req));
  if (!ok) {
    (void)hipFree(p);
    return;
  }
  g_cache.push_back({dev, p, n});
  cache_trim_locked(dev, (size_t)(0.4 * (double)tot));
}

// RAII device buffer
struct DBuf {
  void *p = nullptr;
  size_t n = 0;
  size_t cap = 0;  // bytes of the block behind p (>= n)
  bool owned = false;
  ~DBuf() {
    if (p && owned) dev_release(p, cap, n == 0 ? 16 : n);
  }
  hipError_t alloc(size_t bytes) {
    n = bytes;
    if (bytes == 0) bytes = 16;
    if (t_arena) {
      const size_t at = (t_arena->used + 255) / 256 * 256;
      t_arena->want = std::max(t_arena->want, at) + bytes;
      if (at + bytes > t_arena->cap) {
        t_arena->overflow = true;
        return hipErrorOutOfMemory;
      }
      p = t_arena->base + at;
      t_arena->used = at + bytes;
      owned = false;
      return hipSuccess;
    }
    owned = true;
    return dev_alloc(&p, bytes, &cap);
  }
  template <class T>
  T *as() const {
    return reinterpret_cast<T *>(p);
  }
};

template <class T>
hipError_t upload(DBuf &b, const std::vector<T> &v, hipStream_t s) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

int ncart_h(int l) { return (l + 1) * (l + 2) / 2; }

double dfact_odd(int l) {  // (2l-1)!!
  double r = 1.0;
  for (int k = 2 * l - 1; k > 1; k -= 2) r *= k;
  return r;
}

// ------------------------------------------------------------- validation
int validate_basis(const rsgdf_basis *b, int natm, int lmax, const char *what) {
  if (!b || b->nshell < 1 || !b->shell_atom || !b->shell_l || !b->shell_nprim || !b->shell_ptr || !b->exps ||
      !b->coefs)
    return fail(RSGDF_EINVAL, std::string(what) + ": null or empty basis");
  for (int s = 0; s < b->nshell; ++s) {
    if (b->shell_atom[s] < 0 || b->shell_atom[s] >= natm)
      return fail(RSGDF_EINVAL, std::string(what) + ": shell atom index out of range");
    if (b->shell_l[s] < 0) return fail(RSGDF_EINVAL, std::string(what) + ": negative angular momentum");
    if (b->shell_l[s] > lmax)
      return fail(RSGDF_EUNSUPPORTED, std::string(what) + ": angular momentum above this build's maximum");
    if (b->shell_nprim[s] < 1 || b->shell_nprim[s] > 16)
      return fail(RSGDF_EINVAL, std::string(what) + ": nprim must be in 1..16");
    if (b->shell_ptr[s] < 0) return fail(RSGDF_EINVAL, std::string(what) + ": negative primitive offset");
    for (int k = 0; k < b->shell_nprim[s]; ++k) {
      const double a = b->exps[b->shell_ptr[s] + k], c = b->coefs[b->shell_ptr[s] + k];
      if (!(a > 0.0) || !std::isfinite(a)) return fail(RSGDF_EINVAL, std::string(what) + ": exponents must be > 0");
      if (!std::isfinite(c)) return fail(RSGDF_EINVAL, std::string(what) + ": non-finite coefficient");
    }
  }
  return RSGDF_OK;
}

// free device memory for the scratch budgets: the remainder of the installed
// arena, else what the runtime reports plus the idle cached blocks
hipError_t mem_avail(size_t *free_b) {
  if (t_arena) {
    *free_b = t_arena->cap - std::min(t_arena->cap, t_arena->used);
    return hipSuccess;
  }
  size_t total_b = 0;
  const hipError_t e = hipMemGetInfo(free_b, &total_b);
  if (e == hipSuccess) *free_b += cache_free_bytes();
  return e;
}

int64_t nfunc(const rsgdf_basis *b) {
  int64_t n = 0;
  for (int s = 0; s < b->nshell; ++s) n += ncart_h(b->shell_l[s]);
  return n;
}

struct Lat {
  Lattice L;
  double an[3], bn[3];
};

int make_lattice(const rsgdf_cell *cell, const int32_t *kmesh, Lat &lt) {
  const double *a = cell->lattice;
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(a[i])) return fail(RSGDF_EINVAL, "non-finite lattice");
  const double c0[3] = {a[4] * a[8] - a[5] * a[7], a[5] * a[6] - a[3] * a[8], a[3] * a[7] - a[4] * a[6]};
  const double det = a[0] * c0[0] + a[1] * c0[1] + a[2] * c0[2];
  if (!(std::fabs(det) > 1e-8)) return fail(RSGDF_EINVAL, "singular lattice");
  const double c1[3] = {a[7] * a[2] - a[8] * a[1], a[8] * a[0] - a[6] * a[2], a[6] * a[1] - a[7] * a[0]};
  const double c2[3] = {a[1] * a[5] - a[2] * a[4], a[2] * a[3] - a[0] * a[5], a[0] * a[4] - a[1] * a[3]};
  for (int i = 0; i < 9; ++i) lt.L.a[i] = a[i];
  for (int j = 0; j < 3; ++j) {
    lt.L.b[j] = 2.0 * kPi * c0[j] / det;
    lt.L.b[3 + j] = 2.0 * kPi * c1[j] / det;
    lt.L.b[6 + j] = 2.0 * kPi * c2[j] / det;
  }
  lt.L.vol = std::fabs(det);
  for (int d = 0; d < 3; ++d) {
    if (kmesh[d] < 1 || kmesh[d] > 64) return fail(RSGDF_EINVAL, "kmesh entries must be in 1..64");
    lt.L.n[d] = kmesh[d];
    lt.an[d] = std::sqrt(a[3 * d] * a[3 * d] + a[3 * d + 1] * a[3 * d + 1] + a[3 * d + 2] * a[3 * d + 2]);
    const double *b = lt.L.b + 3 * d;
    lt.bn[d] = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  }
  lt.L.nk = kmesh[0] * kmesh[1] * kmesh[2];
  lt.L.pad = 0;
  return RSGDF_OK;
}

// ------------------------------------------------------------- Boys table
// For each order L <= kMaxL and unit interval [i, i+1) of T < kBoysSwitch, the
// Taylor coefficients of F_L about the interval centre Tc:
//   F_L(Tc + u) = sum_j (-1)^j F_{L+j}(Tc) u^j / j!   (dF_n/dT = -F_{n+1}).
// F_n(Tc) come from the power series e^{-T} sum_k (2T)^k / ((2n+1)(2n+3)...(2n+2k+1))
// at a high order in extended precision and the downward recursion
// F_n = (2T F_{n+1} + e^{-T}) / (2n+1).
const std::vector<double> &boys_poly_table() {
  static std::vector<double> tab;
  if (!tab.empty()) return tab;
  const int nc = kBoysPolyDeg + 1;
  tab.resize((size_t)(kMaxL + 1) * kBoysIntervals * nc);
  const int nmax = kMaxL + kBoysPolyDeg;
  const int ntop = nmax + 40;
  std::vector<long double> F(ntop + 1);
  for (int i = 0; i < kBoysIntervals; ++i) {
    const long double T = (long double)i + 0.5L;
    long double term = 1.0L / (2 * ntop + 1), sum = term;
    for (int k = 1; k < 10000; ++k) {
      term *= 2.0L * T / (2 * ntop + 2 * k + 1);
      sum += term;
      if (term < 1e-24L * sum) break;
    }
    const long double e = expl(-T);
    F[ntop] = e * sum;
    for (int n = ntop - 1; n >= 0; --n) F[n] = (2.0L * T * F[n + 1] + e) / (2 * n + 1);
    for (int L = 0; L <= kMaxL; ++L) {
      long double fact = 1.0L;
      for (int j = 0; j < nc; ++j) {
        if (j > 0) fact *= j;
        const long double c = ((j & 1) ? -1.0L : 1.0L) * F[L + j] / fact;
        tab[((size_t)L * kBoysIntervals + i) * nc + j] = (double)c;
      }
    }
  }
  return tab;
}

// ------------------------------------------------------------- screening
struct Screen {
  double vol, dR, eps, omega;
  double ncell_nf, r0;
  double N(double R) const {  // N_cell(R, R+dR), Eq. S19
    return (R > r0) ? 4.0 * kPi / vol * 2.0 * (R + dR) * (R + dR) * dR : ncell_nf;
  }
};

double f_sr(double R, double eta1, double eta2) {  // Eq. S7
  if (R < 1e-12) return 2.0 * (eta1 - eta2) / std::sqrt(kPi);
  return (std::erf(eta1 * R) - std::erf(eta2 * R)) / R;
}

// The cut x* of a bracket [lo, hi] with g(lo) > 0 >= g(hi), g having one sign
// change there and falling through it: Newton steps with g' from the newest
// point, a bisection whenever g' is not negative there or the step leaves the
// bracket.  Ends when a step is below 1e-14 of x (Newton converges
// quadratically, so x is then within far less of x*) and returns x (1 + 1e-12),
// at or beyond the cut like the upper end of a bisection; or the bracket's
// upper end once it is that narrow.
template <class G, class D>
double cut_root(G g, D dg, double lo, double hi) {
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double gx = g(x);
    if (gx > 0) lo = x;
    else hi = x;
    if (hi - lo <= 1e-14 * hi) return hi;
    const double d = dg(x);
    double xn = (d < 0.0) ? x - gx / d : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 1e-14 * x) return std::min(hi, xn * (1.0 + 1e-12));
    x = xn;
  }
  return hi;
}

// largest R > 0 with K (1 + 2 eta R)^L exp(-eta^2 R^2)/R >= eps: the bound of Eq. S14
// with the growth of an angular momentum L = l_P + l_a + l_b term, whose
// Gaussian tail carries a degree-L polynomial (the L-th Hermite derivative of
// exp(-eta^2 R^2) is (2 eta^2 R)^L exp(-eta^2 R^2) times 1 + O(1/R^2)), which the
// s-type model of Eq. S14 leaves out.  With t = eta R the logarithm g of the
// left side over eps has g' > 0 exactly where q(t) = 4t^3 + 2t^2 - 2(L-1)t + 1
// < 0: for L < 3 never (g falls), for larger L on the interval (t1, t2) between
// the positive roots of q when its minimum is negative (g falls, rises, falls).
// The largest cut lies beyond the local maximum t2 / eta if g is positive
// there, else before the local minimum t1 / eta; each bracket holds one.
double solve_rc(double K, double eta, double eps, int L) {
  const double c0 = std::log(K) - std::log(eps);
  auto g = [&](double R) { return c0 + L * std::log1p(2.0 * eta * R) - eta * eta * R * R - std::log(R); };
  auto dg = [&](double R) { return 2.0 * L * eta / (1.0 + 2.0 * eta * R) - 2.0 * eta * eta * R - 1.0 / R; };
  double t1 = 0.0, t2 = 0.0;
  if (L >= 3) {
    auto q = [&](double t) { return ((4.0 * t + 2.0) * t - 2.0 * (L - 1)) * t + 1.0; };
    auto dq = [&](double t) { return (12.0 * t + 4.0) * t - 2.0 * (L - 1); };
    const double ts = (-4.0 + std::sqrt(16.0 + 96.0 * (L - 1))) / 24.0;  // minimum of q on t > 0
    if (q(ts) < 0.0) {
      t1 = cut_root(q, dq, 0.0, ts);  // q falls from q(0) = 1 through zero
      double th = std::max(1.0, 2.0 * ts);
      while (q(th) <= 0.0) th *= 2.0;
      auto mq = [&](double t) { return -q(t); };
      auto dmq = [&](double t) { return -dq(t); };
      t2 = cut_root(mq, dmq, ts, th);  // q rises through zero
    }
  }
  if (t2 > 0.0 && g(t2 / eta) > 0.0) {
    const double lo = t2 / eta;
    double hi = 2.0 * lo;
    while (g(hi) > 0 && hi < 1e6) hi *= 2.0;
    if (g(hi) > 0) return hi;
    return cut_root(g, dg, lo, hi);
  }
  double lo = 1e-8, hi = 1.0;
  if (g(lo) < 0) return lo;
  if (t1 > 0.0) {
    hi = t1 / eta;  // g(hi) <= g(t2 / eta) <= 0
    if (hi <= lo) return lo;
  } else {
    while (g(hi) > 0 && hi < 1e6) hi *= 2.0;
    if (g(hi) > 0) return hi;
  }
  return cut_root(g, dg, lo, hi);
}

// largest x with NF * x exp(-beta x^2) >= eps, or 0 (Eq. S23)
double solve_r12(double NF, double beta, double eps) {
  const double xs = 1.0 / std::sqrt(2.0 * beta);
  if (!(NF > 0.0) || NF * xs * std::exp(-0.5) < eps) return 0.0;
  const double c0 = std::log(NF) - std::log(eps);
  auto g = [&](double x) { return c0 + std::log(x) - beta * x * x; };
  auto dg = [&](double x) { return 1.0 / x - 2.0 * beta * x; };
  double lo = xs, hi = 2.0 * xs;
  while (g(hi) > 0 && hi < 1e6) hi *= 2.0;
  if (g(hi) > 0) return hi;
  return cut_root(g, dg, lo, hi);
}

// largest x with NF x exp(-beta x^2) (1 + c x)^L >= eps, or 0 (Eq. S23 with the
// angular growth of an l_a + l_b = L pair factor); the left side has one
// maximum on x > 0, where its logarithmic derivative (a falling function)
// changes sign
double solve_r12_grow(double NF, double beta, double eps, int L, double c) {
  if (L == 0) return solve_r12(NF, beta, eps);
  if (!(NF > 0.0)) return 0.0;
  auto dlog = [&](double x) { return 1.0 / x - 2.0 * beta * x + L * c / (1.0 + c * x); };
  auto ddlog = [&](double x) { return -1.0 / (x * x) - 2.0 * beta - L * c * c / ((1.0 + c * x) * (1.0 + c * x)); };
  double lo = 1e-12, hi = 1.0;
  while (dlog(hi) > 0 && hi < 1e6) hi *= 2.0;
  const double xm = dlog(hi) > 0 ? hi : cut_root(dlog, ddlog, lo, hi);
  const double c0 = std::log(NF) - std::log(eps);
  auto g = [&](double x) { return c0 + std::log(x) - beta * x * x + L * std::log1p(c * x); };
  if (g(xm) < 0) return 0.0;
  lo = xm;
  hi = 2.0 * xm;
  while (g(hi) > 0 && hi < 1e6) hi *= 2.0;
  if (g(hi) > 0) return hi;
  return cut_root(g, dlog, lo, hi);
}

template <class F>
void parallel_for(int64_t n, F f, int64_t grain = 64) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = (unsigned)std::min<int64_t>(nt, (n + grain - 1) / grain);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        const int64_t i0 = next.fetch_add(grain);
        if (i0 >= n) break;
        for (int64_t i = i0; i < std::min(n, i0 + grain); ++i) f(i);
      }
    });
  for (auto &t : th) t.join();
}

struct HostPlan {
  Lat lt;
  std::vector<Shell> ao, ax;
  std::vector<double> ao_exp, ao_coef, ao_c1s, ax_exp, ax_coef, ax_c1s;
  std::vector<Pair> pairs;
  std::vector<int32_t> cls_off, nsr;
  std::vector<double> img;
  std::vector<double> rc_t;  // [naux_shell][npair] Eq. S14 bound
  std::vector<double> amp_t; // [naux_shell][npair] 1s-model amplitude
  int64_t nao = 0, naux = 0;
  bool diag_only = false;  // k-pairs (k, k) only (the Coulomb consumer needs k12 = 0)
  double acut = 0.0;       // > 0: compact/diffuse split; the short-range bounds then cover compact aux primitives
  Screen scr;
  // k-points
  std::vector<double> kvec;     // [nk][3]
  std::vector<int32_t> kp1, kp2;
};

// Packed shells of a basis: centre, l, primitive range, function offset and
// the most diffuse primitive with its 1s-equivalent amplitude (the screening
// bounds treat every function as 1s, Eq. S26).  Returns the function count.
int64_t pack_shells(const rsgdf_basis *b, const double *coords, std::vector<Shell> &sh, std::vector<double> &ex,
                    std::vector<double> &cf, std::vector<double> &c1s) {
  int64_t foff = 0;
  for (int s = 0; s < b->nshell; ++s) {
    Shell x{};
    const double *C = coords + 3 * b->shell_atom[s];
    x.x = C[0];
    x.y = C[1];
    x.z = C[2];
    x.l = b->shell_l[s];
    x.nprim = b->shell_nprim[s];
    x.pptr = (int32_t)ex.size();
    x.foff = (int32_t)foff;
    foff += ncart_h(x.l);
    double amin = 1e300, cmin = 0.0;
    for (int k = 0; k < x.nprim; ++k) {
      const double a = b->exps[b->shell_ptr[s] + k], c = b->coefs[b->shell_ptr[s] + k];
      ex.push_back(a);
      cf.push_back(c);
      // 1s function with the L2 norm of the x^l component of this primitive
      const double c1 = std::fabs(c) * std::sqrt(dfact_odd(x.l) / std::pow(4.0 * a, x.l));
      c1s.push_back(c1);
      if (a < amin) {
        amin = a;
        cmin = c1;
      }
    }
    x.a_d = amin;
    x.c_d = cmin;
    sh.push_back(x);
  }
  return foff;
}

// k-points of the Gamma-centred mesh, k_j = sum_i (j_i / n_i) b_i
std::vector<double> mesh_kvec(const Lattice &L) {
  std::vector<double> kv(3 * L.nk);
  for (int j0 = 0; j0 < L.n[0]; ++j0)
    for (int j1 = 0; j1 < L.n[1]; ++j1)
      for (int j2 = 0; j2 < L.n[2]; ++j2) {
        const int k = (j0 * L.n[1] + j1) * L.n[2] + j2;
        for (int d = 0; d < 3; ++d)
          kv[3 * k + d] = (double)j0 / L.n[0] * L.b[d] + (double)j1 / L.n[1] * L.b[3 + d] +
                          (double)j2 / L.n[2] * L.b[6 + d];
      }
  return kv;
}

// G sets per folded k12 class c (Eq. M10): q = G + k_c, q != 0,
// exp(-q^2/4w^2) >= g_thr, each sorted by |q|; qv [nq_tot][3], qoff [nk + 1]
void make_qsets(const Lat &lt, const std::vector<double> &kvec, double omega, double g_thr, std::vector<double> &qv,
                std::vector<int64_t> &qoff) {
  const Lattice &L = lt.L;
  const double q2max = -4.0 * omega * omega * std::log(g_thr);
  qv.clear();
  qoff.assign(1, 0);
  for (int c = 0; c < L.nk; ++c) {
    const double *kc = &kvec[3 * c];
    const double qm = std::sqrt(std::max(q2max, 0.0)) + std::sqrt(kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2]);
    int w[3];
    for (int d = 0; d < 3; ++d) w[d] = (int)std::ceil(qm * lt.an[d] / (2.0 * kPi)) + 1;
    std::vector<std::array<double, 4>> qc;  // (|q|^2, q)
    for (int i = -w[0]; i <= w[0]; ++i)
      for (int j = -w[1]; j <= w[1]; ++j)
        for (int k = -w[2]; k <= w[2]; ++k) {
          double q[3], q2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            q[d] = i * L.b[d] + j * L.b[3 + d] + k * L.b[6 + d] + kc[d];
            q2 += q[d] * q[d];
          }
          if (q2 < 1e-20) continue;
          if (std::exp(-q2 / (4.0 * omega * omega)) < g_thr) continue;
          qc.push_back({q2, q[0], q[1], q[2]});
        }
    // by |q|, so that neighbouring lanes of the pair-transform kernel
    // drop the same primitive pairs (the e^{-q^2/4p} factor)
    std::stable_sort(qc.begin(), qc.end(), [](const std::array<double, 4> &x, const std::array<double, 4> &y) {
      return x[0] < y[0];
    });
    for (const auto &e : qc) qv.insert(qv.end(), e.begin() + 1, e.end());
    qoff.push_back((int64_t)qv.size() / 3);
  }
}

// q sets per folded k12 class c of a plain sphere: q = G + k_c, q != 0,
// |q|^2 <= q2max, each sorted by |q| (the Eq. M15 part of the split)
void make_qsets_sphere(const Lat &lt, const std::vector<double> &kvec, double q2max, std::vector<double> &qv,
                       std::vector<int64_t> &qoff) {
  const Lattice &L = lt.L;
  qv.clear();
  qoff.assign(1, 0);
  for (int c = 0; c < L.nk; ++c) {
    const double *kc = &kvec[3 * c];
    const double qm = std::sqrt(q2max) + std::sqrt(kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2]);
    int w[3];
    for (int d = 0; d < 3; ++d) w[d] = (int)std::ceil(qm * lt.an[d] / (2.0 * kPi)) + 1;
    std::vector<std::array<double, 4>> qc;
    for (int i = -w[0]; i <= w[0]; ++i)
      for (int j = -w[1]; j <= w[1]; ++j)
        for (int k = -w[2]; k <= w[2]; ++k) {
          double q[3], q2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            q[d] = i * L.b[d] + j * L.b[3 + d] + k * L.b[6 + d] + kc[d];
            q2 += q[d] * q[d];
          }
          if (q2 < 1e-20 || q2 > q2max) continue;
          qc.push_back({q2, q[0], q[1], q[2]});
        }
    std::stable_sort(qc.begin(), qc.end(), [](const std::array<double, 4> &x, const std::array<double, 4> &y) {
      return x[0] < y[0];
    });
    for (const auto &e : qc) qv.insert(qv.end(), e.begin() + 1, e.end());
    qoff.push_back((int64_t)qv.size() / 3);
  }
}

// phase table kph[k][c] = e^{+i k.L_c} (complex, [nk][nk])
std::vector<double> mesh_phases(const Lattice &L) {
  const int nk = L.nk;
  std::vector<double> kph((size_t)2 * nk * nk);
  for (int k = 0; k < nk; ++k)
    for (int c = 0; c < nk; ++c) {
      const int j[3] = {k / (L.n[1] * L.n[2]), (k / L.n[2]) % L.n[1], k % L.n[2]};
      const int i[3] = {c / (L.n[1] * L.n[2]), (c / L.n[2]) % L.n[1], c % L.n[2]};
      long double t = 0.0L;  // 2 pi sum_d j_d i_d / n_d
      for (int d = 0; d < 3; ++d) t += (long double)(j[d] * i[d] % L.n[d]) / L.n[d];
      const double ph = (double)(2.0L * 3.14159265358979323846264338327950288L * t);
      kph[2 * ((size_t)k * nk + c)] = std::cos(ph);
      kph[2 * ((size_t)k * nk + c) + 1] = std::sin(ph);
    }
  return kph;
}

int build_plan(const rsgdf_cell *cell, const rsgdf_basis *bs, const rsgdf_basis *ax, const int32_t *kmesh,
               double omega, double thresh, HostPlan &hp) {
  int rc = make_lattice(cell, kmesh, hp.lt);
  if (rc) return rc;
  const Lattice &L = hp.lt.L;
  const int nk = L.nk;
  // shells
  hp.nao = pack_shells(bs, cell->coords, hp.ao, hp.ao_exp, hp.ao_coef, hp.ao_c1s);
  hp.naux = pack_shells(ax, cell->coords, hp.ax, hp.ax_exp, hp.ax_coef, hp.ax_c1s);
  if (hp.acut > 0.0) {
    // compact/diffuse split: only the compact primitives of an aux shell enter
    // the short-range sums, so the bounds take the most diffuse of those
    // (a_d < 0 marks a shell with none: no short-range work)
    for (Shell &x : hp.ax) {
      double amin = -1.0, cmin = 0.0;
      for (int k = 0; k < x.nprim; ++k) {
        const double a = hp.ax_exp[x.pptr + k];
        if (a >= hp.acut && (amin < 0.0 || a < amin)) {
          amin = a;
          cmin = hp.ax_c1s[x.pptr + k];
        }
      }
      x.a_d = amin;
      x.c_d = cmin;
    }
  }

  // k-points and pairs
  hp.kvec = mesh_kvec(L);
  for (int k1 = 0; k1 < nk; ++k1)
    for (int k2 = k1; k2 < nk; ++k2) {
      if (hp.diag_only && k2 != k1) continue;
      hp.kp1.push_back(k1);
      hp.kp2.push_back(k2);
    }

  // N_cell model (Eq. S19): N^NF = lattice points within 3 Omega^{1/3}
  Screen &S = hp.scr;
  S.vol = L.vol;
  S.dR = 1.0;
  S.eps = thresh;
  S.omega = omega;
  {
    const double rnf = 3.0 * std::cbrt(L.vol);
    int w[3];
    for (int d = 0; d < 3; ++d) w[d] = (int)std::ceil(rnf * hp.lt.bn[d] / (2.0 * kPi)) + 1;
    int64_t cnt = 0;
    for (int i = -w[0]; i <= w[0]; ++i)
      for (int j = -w[1]; j <= w[1]; ++j)
        for (int k = -w[2]; k <= w[2]; ++k) {
          double v[3];
          for (int d = 0; d < 3; ++d) v[d] = i * L.a[d] + j * L.a[3 + d] + k * L.a[6 + d];
          if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] <= rnf * rnf) ++cnt;
        }
    S.ncell_nf = (double)cnt;
    S.r0 = std::sqrt(S.ncell_nf * L.vol / (8.0 * kPi * S.dR)) - S.dR;
  }

  // AO shell pairs, oriented l(sa) >= l(sb)
  const int nsh = (int)hp.ao.size();
  for (int i = 0; i < nsh; ++i)
    for (int j = i; j < nsh; ++j) {
      Pair p{};
      if (hp.ao[i].l >= hp.ao[j].l) {
        p.sa = i;
        p.sb = j;
      } else {
        p.sa = j;
        p.sb = i;
      }
      p.diag = (i == j);
      const double a1 = hp.ao[p.sa].a_d, a2 = hp.ao[p.sb].a_d;
      p.beta_d = a1 * a2 / (a1 + a2);
      hp.pairs.push_back(p);
    }
  const int npair = (int)hp.pairs.size();

  // Per pair: S_h (Eq. S15, eps' = 1e-4) and R12min (Eq. S25) from the
  // eps'-truncated image sum of h = exp(-beta R12^2).  The truncation is taken
  // relative to the largest term (h >= eps' h_max), so a pair whose nearest
  // image already has h < eps' keeps its leading terms.
  const double epsp = 1e-4;
  std::vector<double> Sh(npair);
  parallel_for(npair, [&](int64_t ip) {
    Pair &p = hp.pairs[ip];
    const Shell &A = hp.ao[p.sa], &B = hp.ao[p.sb];
    const double beta = p.beta_d;
    const double AB[3] = {A.x - B.x, A.y - B.y, A.z - B.z};
    const double dab = std::sqrt(AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2]);
    const double rmax = dab + std::sqrt(std::log(1.0 / epsp) / beta) + 1.0;
    int w[3];
    for (int d = 0; d < 3; ++d) w[d] = (int)std::ceil((rmax + 1e-9) * hp.lt.bn[d] / (2.0 * kPi)) + 2;
    std::vector<double> r12all;
    for (int i = -w[0]; i <= w[0]; ++i)
      for (int j = -w[1]; j <= w[1]; ++j)
        for (int k = -w[2]; k <= w[2]; ++k) {
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            const double v = AB[d] - (i * L.a[d] + j * L.a[3 + d] + k * L.a[6 + d]);
            d2 += v * v;
          }
          r12all.push_back(std::sqrt(d2));
        }
    std::sort(r12all.begin(), r12all.end());
    const double hmax = std::exp(-beta * r12all[0] * r12all[0]);
    std::vector<double> r12s;
    double sh = 0.0;
    for (double r : r12all) {
      const double h = std::exp(-beta * r * r);
      if (h >= epsp * hmax) {
        sh += h;
        r12s.push_back(r);
      }
    }
    Sh[ip] = sh;
    std::sort(r12s.begin(), r12s.end());
    // crossing of N_cell(x) x/(2 beta) e^{-beta x^2} and sum_{R12 > x} h, the
    // tail sums taken from suffix sums over the sorted list
    double r12min = 0.0;
    const double step = 0.05;
    const double xend = r12s.back() + step;
    std::vector<double> tail(r12s.size() + 1, 0.0);
    for (size_t i = r12s.size(); i-- > 0;) tail[i] = tail[i + 1] + std::exp(-beta * r12s[i] * r12s[i]);
    size_t first = 0;  // first index with r12s[first] > x
    for (double x = 0.0; x <= xend; x += step) {
      while (first < r12s.size() && r12s[first] <= x) ++first;
      const double rhs = tail[first];
      const double lhs = S.N(x) * x / (2.0 * beta) * std::exp(-beta * x * x);
      if (lhs < rhs) r12min = x + step;
    }
    p.R12min = r12min;
  });

  // Triplets are built per call by the caller of this function (they need the
  // aux batching); here compute per (aux shell, pair) the R_c bound and the
  // largest R12 kept by any window, to size the pair image lists.
  const int nxs = (int)hp.ax.size();
  std::vector<double> r12pair(npair, 0.0);
  {
    std::vector<double> r12t((size_t)nxs * npair);
    hp.rc_t.assign((size_t)nxs * npair, 0.0);
    hp.amp_t.assign((size_t)nxs * npair, 0.0);
    // 1s-model amplitudes of Eq. S4, pi^3 C_P C_mu C_nu / (a_P p)^{3/2}, summed
    // over the primitives of contracted shells; the decay constants (eta1,
    // eta2, beta) stay those of the most diffuse primitives.
    std::vector<double> apair(npair), aaux(nxs);
    for (int ip = 0; ip < npair; ++ip) {
      const Shell &sA = hp.ao[hp.pairs[ip].sa], &sB = hp.ao[hp.pairs[ip].sb];
      double a = 0.0;
      for (int i = 0; i < sA.nprim; ++i)
        for (int j = 0; j < sB.nprim; ++j)
          a += hp.ao_c1s[sA.pptr + i] * hp.ao_c1s[sB.pptr + j] /
               std::pow(hp.ao_exp[sA.pptr + i] + hp.ao_exp[sB.pptr + j], 1.5);
      apair[ip] = a;
    }
    for (int P = 0; P < nxs; ++P) {
      double a = 0.0;
      for (int k = 0; k < hp.ax[P].nprim; ++k) {
        const double g = hp.ax_exp[hp.ax[P].pptr + k];
        if (hp.acut > 0.0 && g < hp.acut) continue;  // diffuse: Eq. M15 part
        a += hp.ax_c1s[hp.ax[P].pptr + k] / std::pow(g, 1.5);
      }
      aaux[P] = a;
    }
    parallel_for((int64_t)nxs * npair, [&](int64_t t) {
      const int P = (int)(t / npair), ip = (int)(t % npair);
      const Pair &p = hp.pairs[ip];
      const Shell &sP = hp.ax[P], &sA = hp.ao[p.sa], &sB = hp.ao[p.sb];
      if (sP.a_d <= 0.0) {  // no compact primitive (split): no short-range work
        hp.amp_t[t] = 0.0;
        hp.rc_t[t] = 0.0;
        r12t[t] = 0.0;
        return;
      }
      const double pd = sA.a_d + sB.a_d;
      const double Aamp = kPi * kPi * kPi * aaux[P] * apair[ip];
      hp.amp_t[t] = Aamp;
      const double eta1 = std::sqrt(sP.a_d * pd / (sP.a_d + pd));
      const double eta2 = 1.0 / std::sqrt(1.0 / (eta1 * eta1) + 1.0 / (omega * omega));
      const double K = Aamp * Sh[ip] * 4.0 * kPi / L.vol / (std::sqrt(kPi) * 2.0 * eta2 * eta2 * eta2);
      const double rc = solve_rc(K, eta2, thresh, sP.l + sA.l + sB.l);
      hp.rc_t[t] = rc;
      const int W = std::max(1, (int)std::ceil(rc / S.dR));
      double nfmax = 0.0;
      for (int w = 0; w < W; ++w) nfmax = std::max(nfmax, S.N(w * S.dR) * f_sr(w * S.dR, eta1, eta2));
      nfmax *= Aamp * 4.0 * kPi / L.vol / (2.0 * p.beta_d);
      r12t[t] = solve_r12_grow(nfmax, p.beta_d, thresh, sA.l + sB.l, pair_growth_c(p.beta_d));
    });
    for (int P = 0; P < nxs; ++P)
      for (int ip = 0; ip < npair; ++ip) r12pair[ip] = std::max(r12pair[ip], r12t[(size_t)P * npair + ip]);
  }

  // Pair image lists: all n' with |A - B - n'| <= max(R12 of the SR bounds,
  // overlap radius sqrt(50/beta)), grouped by BvK class, sorted by distance.
  hp.cls_off.assign((size_t)npair * (nk + 1), 0);
  hp.nsr.assign((size_t)npair * nk, 0);
  std::vector<std::vector<double>> lists(npair);
  std::vector<std::vector<int32_t>> coffs(npair), nsrs(npair);
  parallel_for(npair, [&](int64_t ip) {
    Pair &p = hp.pairs[ip];
    p.R12sr = std::max(p.R12min, r12pair[ip]);
    const Shell &A = hp.ao[p.sa], &B = hp.ao[p.sb];
    const double rlist = std::max(p.R12sr, std::sqrt(50.0 / p.beta_d));
    int w[3];
    for (int d = 0; d < 3; ++d) w[d] = (int)std::ceil(rlist * hp.lt.bn[d] / (2.0 * kPi)) + 2;
    struct Im {
      int c;
      double r;
      double v[3];
    };
    std::vector<Im> ims;
    const double AB[3] = {A.x - B.x, A.y - B.y, A.z - B.z};
    for (int i = -w[0]; i <= w[0]; ++i)
      for (int j = -w[1]; j <= w[1]; ++j)
        for (int k = -w[2]; k <= w[2]; ++k) {
          Im im;
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            im.v[d] = i * L.a[d] + j * L.a[3 + d] + k * L.a[6 + d];
            const double t = AB[d] - im.v[d];
            d2 += t * t;
          }
          im.r = std::sqrt(d2);
          if (im.r > rlist) continue;
          const int r0 = ((i % L.n[0]) + L.n[0]) % L.n[0], r1 = ((j % L.n[1]) + L.n[1]) % L.n[1],
                    r2 = ((k % L.n[2]) + L.n[2]) % L.n[2];
          im.c = (r0 * L.n[1] + r1) * L.n[2] + r2;
          ims.push_back(im);
        }
    std::sort(ims.begin(), ims.end(), [](const Im &x, const Im &y) { return x.c != y.c ? x.c < y.c : x.r < y.r; });
    coffs[ip].assign(nk + 1, 0);
    nsrs[ip].assign(nk, 0);
    for (auto &im : ims) {
      coffs[ip][im.c + 1]++;
      if (im.r <= p.R12sr) nsrs[ip][im.c]++;
    }
    for (int c = 0; c < nk; ++c) coffs[ip][c + 1] += coffs[ip][c];
    lists[ip].reserve(3 * ims.size());
    for (auto &im : ims)
      for (int d = 0; d < 3; ++d) lists[ip].push_back(im.v[d]);
  });
  for (int ip = 0; ip < npair; ++ip) {
    Pair &p = hp.pairs[ip];
    p.img_off = (int32_t)(hp.img.size() / 3);
    p.cls_off = ip * (nk + 1);
    p.nsr_off = ip * nk;
    for (int c = 0; c <= nk; ++c) hp.cls_off[(size_t)ip * (nk + 1) + c] = coffs[ip][c];
    for (int c = 0; c < nk; ++c) hp.nsr[(size_t)ip * nk + c] = nsrs[ip][c];
    hp.img.insert(hp.img.end(), lists[ip].begin(), lists[ip].end());
  }
  if (hp.img.size() / 3 > (size_t)0x7fffffff) return fail(RSGDF_EUNSUPPORTED, "too many pair images");
  return RSGDF_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

const char *rsgdf_last_error(void) { return g_err.c_str(); }

const char *rsgdf_version(void) { return "rsgdf-mi355x 0.1 (gfx950)"; }

// set by the build script from the sources it compiled
#ifndef RSGDF_SOURCE_HASH
#define RSGDF_SOURCE_HASH "unknown"
#endif
const char *rsgdf_source_hash(void) { return RSGDF_SOURCE_HASH; }

int rsgdf_release_cache(void) {
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  std::lock_guard<std::mutex> lk(g_cache_mu);
  while (!g_cache.empty()) {
    const int dev = g_cache.front().dev;
    HIPCHK(hipSetDevice(dev));
    cache_trim_locked(dev, 0);
  }
  HIPCHK(hipSetDevice(cur));
  return RSGDF_OK;
}

int64_t rsgdf_j3c_nbytes(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                         const int32_t kmesh[3]) {
  if (!cell || !basis || !auxbasis || !kmesh || cell->natm < 1 || !cell->coords) {
    fail(RSGDF_EINVAL, "null argument");
    return RSGDF_EINVAL;
  }
  int rc = validate_basis(basis, cell->natm, RSGDF_MAX_L_AO, "basis");
  if (rc) return rc;
  rc = validate_basis(auxbasis, cell->natm, RSGDF_MAX_L_AUX, "auxbasis");
  if (rc) return rc;
  for (int d = 0; d < 3; ++d)
    if (kmesh[d] < 1 || kmesh[d] > 64) {
      fail(RSGDF_EINVAL, "kmesh entries must be in 1..64");
      return RSGDF_EINVAL;
    }
  const int64_t nk = (int64_t)kmesh[0] * kmesh[1] * kmesh[2];
  const int64_t nao = nfunc(basis), naux = nfunc(auxbasis);
  return nk * (nk + 1) / 2 * naux * nao * nao * 16;
}

int rsgdf_build_j3c(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                    const int32_t kmesh[3], double omega, double thresh, rsgdf_out *out) {
  return rsgdf_build_j3c_ex(cell, basis, auxbasis, kmesh, omega, thresh, nullptr, out);
}

}  // extern "C"

namespace {

// Learned-screening hooks of one build: magnitude logging (SR only, no fold
// or LR, no output written) or the keep mask of a trained network.
struct LearnCtl {
  bool log = false;
  double sample_frac = 1.0;
  uint64_t seed = 0;
  std::vector<float> feat, tgt;   // logging results (host)
  long long ncand = 0, nskip = 0;
};

uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// n non-blocking side streams of the current device (created once per thread
// and device, default priority).  The single-cell build forks its short-range
// classes onto 3 of them: with the calling stream that is one stream per
// hardware queue at HIP's default of 4 queues per process (measured on the 8-atom
// 2x2x2 workload: 3.04 s SR with 3, 3.24 s with 4, where two streams share a queue); graph
// replays schedule their own nodes and use 4.
int side_streams(std::vector<hipStream_t> &ss, size_t n) {
  static thread_local std::vector<std::pair<int, hipStream_t>> pool;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  ss.clear();
  for (auto &pr_ : pool)
    if (pr_.first == dev && ss.size() < n) ss.push_back(pr_.second);
  while (ss.size() < n) {
    hipStream_t s_;
    HIPCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    pool.push_back({dev, s_});
    ss.push_back(s_);
  }
  return RSGDF_OK;
}

// One j3c build: host planning and every device allocation and upload in
// prepare(); then device work only (no allocation, copy or wait, so that a
// batch can be captured into a graph); results and statistics in finish().
struct Job {
  // ---- inputs
  const rsgdf_cell *cell = nullptr;
  const rsgdf_basis *basis = nullptr, *auxbasis = nullptr;
  const int32_t *kmesh = nullptr;
  double omega = 0, thresh = 0, g_thr = 0;
  rsgdf_options o{};
  rsgdf_out *out = nullptr;
  LearnCtl *ctl = nullptr;
  bool logging = false, learned = false, do_sr = false, do_g0 = false, do_lr = false;
  bool tune = false;         // autotuner trial: short-range sums only, no output
  std::vector<float> split;  // per-class work-split factors (24), empty = 1
  // ---- plan
  HostPlan hp;
  bool planned = false;      // hp already built (batches plan their cells on worker threads)
  int plan_rc = 0;
  std::string plan_err;
  int nk = 0, nkp = 0, npair = 0, nxs = 0, nb = 0;
  int64_t nao = 0, naux = 0, nao2 = 0, need = 0;
  double t_plan = 0.0;
  DBuf d_ao, d_ax, d_aoe, d_aoc, d_aoc1, d_axe, d_axc, d_axc1, d_pairs, d_coff, d_nsr, d_img, d_boys, d_plist;
  int32_t plist_grp[7] = {};  // d_plist offsets of the (l(sa), l(sb)) groups dd, dp, ds, pp, ps, ss
  DBuf d_outbuf;
  double *d_out = nullptr;
  std::vector<double> kph;
  DBuf d_kph, d_kdiag, d_SP, d_O, d_Smn, d_kp1, d_tk2, d_tkp, d_Y;
  int ftiles = 0;         // k-pair tiles of the fold's second transform
  int ftk = 4;            // k-pair slots per tile
  int64_t fchunk = 1;     // output elements per fold pass
  double *ybuf = nullptr; // the fold's intermediate: d_Y, or a batch's shared buffer
  bool own_y = true;      // false: the batch allocates one Y for all its cells (their folds run in turn)
  // SR
  std::vector<int> batch_start;
  int nbatch = 0;
  DBuf d_X, d_trip, d_cnt, d_work, d_part, d_pgrp, d_prm;
  std::vector<Triplet> trips;
  std::vector<int> tgrp_off, wgrp_off, pgrp_off;
  std::vector<double> wgrp_cost;
  std::vector<SRWork> work;
  std::vector<SRPartGroup> pgroups;
  int64_t ntrip = 0, nwork = 0, part_total = 0;
  std::vector<int64_t> cand_off;
  int64_t ncand = 0;
  SRParams base{};
  DBuf d_coffc, d_mask, d_mlp, d_nskip, d_logmag;
  // LR
  std::vector<int64_t> qoff{0};
  int64_t nq_tot = 0, qchunk = 1;
  // long-range parts: without the compact/diffuse split one range-separated
  // part (Eq. M10); with it, the range-separated part of the compact aux
  // primitives and non-diffuse-diffuse pairs, plus the Eq. M15 parts of the
  // diffuse aux primitives (every pair) and of the compact aux primitives with
  // the diffuse-diffuse pairs, on their own q sphere
  struct LRPart {
    std::vector<int64_t> qoff{0};
    int64_t nq_tot = 0;
    DBuf d_q, d_A, d_A32;
    int amode = 0, pmode = 0, undamped = 0;
  };
  std::vector<std::unique_ptr<LRPart>> lrp;
  double acut = 0.0;
  std::vector<std::vector<int>> cls_kp;
  std::vector<int64_t> kpl_off{0};
  std::vector<int64_t> ph_off;  // per class: offset (complex) of its phase table
  DBuf d_I, d_B, d_kp, d_ph, d_nterm, d_amax, d_Bhi;
  DBuf d_Asp;  // split-FP16 aux operand of one chunk (F16X3 form)
  // results
  float t_sr = 0.f, t_fold = 0.f, t_lr = 0.f, t_lr_gemm = 0.f;
  long long n_lr = 0, nskip = 0;
  double lr_flops = 0.0;
  std::vector<long long> counts;  // per work item [4], filled by finish()

  int prepare(hipStream_t st, double mem_frac);
  // elements per fold pass for a Y buffer of ybytes (at least one tile, at most
  // the largest aux batch); the bytes that takes: fchunk * nk^2 * 16
  void set_fold_chunk(double ybytes) {
    const int64_t per = (int64_t)nk * nk * 16;
    fchunk = std::max<int64_t>(64, (int64_t)(ybytes / (double)per) / 64 * 64);
    fchunk = std::min<int64_t>(fchunk, std::max<int64_t>(max_bf_el, 1));
  }
  int64_t max_bf_el = 0;  // output elements of the largest aux batch
  SRParams batch_params(int b) const;
  int enqueue_pre(hipStream_t st);
  int enqueue_zero(int b, hipStream_t st);
  int enqueue_sr(int b, hipStream_t st, const std::vector<hipStream_t> &ss, hipEvent_t evf, hipEvent_t *evj);
  int enqueue_reduce(int b, hipStream_t st);
  int enqueue_fold(int b, hipStream_t st);
  int enqueue_lr(hipStream_t st, std::vector<hipEvent_t> *gev);
  int finish(hipStream_t st, const long long *cnt_host);
};

int Job::prepare(hipStream_t st, double mem_frac) {
  const auto t_start = std::chrono::steady_clock::now();
  logging = ctl && ctl->log;
  if (!out) return fail(RSGDF_EINVAL, "null output");
  need = rsgdf_j3c_nbytes(cell, basis, auxbasis, kmesh);
  if (need < 0) return (int)need;
  if (hp.diag_only) {  // Nk k-pairs (k, k) instead of Nk (Nk + 1) / 2
    const int64_t nk_ = (int64_t)kmesh[0] * kmesh[1] * kmesh[2];
    need = need / (nk_ * (nk_ + 1) / 2) * nk_;
  }
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RSGDF_EINVAL, "omega must be > 0");
  if (!(thresh > 0.0) || !std::isfinite(thresh)) return fail(RSGDF_EINVAL, "thresh must be > 0");
  for (int i = 0; i < 3 * cell->natm; ++i)
    if (!std::isfinite(cell->coords[i])) return fail(RSGDF_EINVAL, "non-finite coordinates");
  if (!logging && !tune) {
    if (!out->data) return fail(RSGDF_EINVAL, "null output buffer");
    if (out->capacity_bytes < need) return fail(RSGDF_ESIZE, "output capacity too small");
  }
  if (o.parts == 0) o.parts = RSGDF_PART_ALL;
  g_thr = (o.g_thresh > 0.0) ? o.g_thresh : 1e-2 * thresh;
  if (o.lr_precision != RSGDF_FP64 && o.lr_precision != RSGDF_FP32 && o.lr_precision != RSGDF_F16X3)
    return fail(RSGDF_EINVAL, "unknown lr_precision");
  if (o.screening != RSGDF_SCREEN_RIGOROUS && o.screening != RSGDF_SCREEN_LEARNED)
    return fail(RSGDF_EINVAL, "unknown screening mode");
  if (!(o.alpha_cut >= 0.0) || !std::isfinite(o.alpha_cut)) return fail(RSGDF_EINVAL, "alpha_cut must be >= 0");
  acut = o.alpha_cut;
  if (!planned) hp.acut = acut;
  learned = o.screening == RSGDF_SCREEN_LEARNED && !logging;
  if (learned && !o.mlp_weights) return fail(RSGDF_EUNSUPPORTED, "learned screening needs mlp_weights");
  if (logging || tune) o.parts = RSGDF_PART_SR;
  do_sr = o.parts & RSGDF_PART_SR;
  do_g0 = o.parts & RSGDF_PART_G0;
  do_lr = o.parts & RSGDF_PART_LR;
  if (o.sr_split) {
    split.assign(o.sr_split, o.sr_split + 24);
    for (float f : split)
      if (!(f > 0.f) || !std::isfinite(f)) return fail(RSGDF_EINVAL, "sr_split factors must be > 0");
  }

  if (planned && plan_rc) return fail(plan_rc, plan_err);
  int rc = planned ? RSGDF_OK : build_plan(cell, basis, auxbasis, kmesh, omega, thresh, hp);
  if (rc) return rc;
  // host sources of asynchronous uploads stay alive until the final synchronise
  std::vector<SRParams> prms;
  std::vector<double> qv, phl;
  std::vector<int32_t> kpl;
  const Lattice &L = hp.lt.L;
  nk = L.nk;
  nkp = (int)hp.kp1.size();
  nao = hp.nao;
  naux = hp.naux;
  nao2 = nao * nao;
  npair = (int)hp.pairs.size();
  nxs = (int)hp.ax.size();
  nb = nk * nk;  // rows of X: (c1, c2)

  // ---------------------------------------------------------- device tables
  HIPCHK(upload(d_ao, hp.ao, st));
  HIPCHK(upload(d_ax, hp.ax, st));
  HIPCHK(upload(d_aoe, hp.ao_exp, st));
  HIPCHK(upload(d_aoc, hp.ao_coef, st));
  HIPCHK(upload(d_aoc1, hp.ao_c1s, st));
  HIPCHK(upload(d_axe, hp.ax_exp, st));
  HIPCHK(upload(d_axc, hp.ax_coef, st));
  HIPCHK(upload(d_axc1, hp.ax_c1s, st));
  HIPCHK(upload(d_pairs, hp.pairs, st));
  {  // pair indices grouped by angular momenta for the per-group transform kernels
    static const int key_of_grp[6] = {8, 7, 6, 4, 3, 0};  // 3 l(sa) + l(sb)
    std::vector<int32_t> plist;
    for (int g = 0; g < 6; ++g) {
      plist_grp[g] = (int32_t)plist.size();
      for (int ip = 0; ip < npair; ++ip) {
        const Pair &p = hp.pairs[ip];
        const int la = hp.ao[p.sa].l, lb = hp.ao[p.sb].l;
        if (la > 2 || lb > la) return fail(RSGDF_EINVAL, "internal: AO pair not oriented with l(sa) >= l(sb)");
        if (3 * la + lb == key_of_grp[g]) plist.push_back(ip);
      }
    }
    plist_grp[6] = (int32_t)plist.size();
    if (plist_grp[6] != npair) return fail(RSGDF_EINVAL, "internal: AO pair outside the angular groups");
    HIPCHK(upload(d_plist, plist, st));
  }
  HIPCHK(upload(d_coff, hp.cls_off, st));
  HIPCHK(upload(d_nsr, hp.nsr, st));
  HIPCHK(upload(d_img, hp.img, st));
  const std::vector<double> boys = boys_poly_table();
  HIPCHK(upload(d_boys, boys, st));

  if (logging || tune) {
    d_out = nullptr;  // magnitude logging and tuning trials write no output
  } else if (out->on_device) {
    d_out = reinterpret_cast<double *>(out->data);
  } else {
    HIPCHK(d_outbuf.alloc((size_t)need));
    d_out = d_outbuf.as<double>();
  }

  // phase table kphase[k][c] = e^{+i k.L_c}; the fold's k-pair tiles: up to
  // ftk (a multiple of 4, at most 64) k-pairs (k1, k2) of one k2 each, as many
  // as the k2 with the most k-pairs has
  kph = mesh_phases(L);
  {
    std::vector<std::vector<int32_t>> by_k2(nk);
    for (int t = 0; t < nkp; ++t) by_k2[hp.kp2[t]].push_back(t);
    size_t most = 1;
    for (auto &v : by_k2) most = std::max(most, v.size());
    ftk = (int)std::min<size_t>(64, (most + 3) / 4 * 4);
    std::vector<int32_t> tk2, tkp;
    for (int k2 = 0; k2 < nk; ++k2)
      for (size_t i = 0; i < by_k2[k2].size(); i += ftk) {
        tk2.push_back(k2);
        for (size_t j = i; j < i + ftk; ++j) tkp.push_back(j < by_k2[k2].size() ? by_k2[k2][j] : -1);
      }
    ftiles = (int)tk2.size();
    std::vector<int32_t> kp1(hp.kp1.begin(), hp.kp1.end());
    HIPCHK(upload(d_tk2, tk2, st));
    HIPCHK(upload(d_tkp, tkp, st));
    HIPCHK(upload(d_kp1, kp1, st));
  }
  std::vector<int32_t> kdiag(nkp);
  for (int t = 0; t < nkp; ++t) kdiag[t] = (hp.kp1[t] == hp.kp2[t]) ? hp.kp1[t] : -1;
  // S_P = int chi_P over all space (aux functions), Eq. M13b
  std::vector<double> SP(naux, 0.0);
  for (int s = 0; s < nxs; ++s) {
    const Shell &x = hp.ax[s];
    int ic = 0;
    for (int lx = x.l; lx >= 0; --lx)
      for (int ly = x.l - lx; ly >= 0; --ly, ++ic) {
        const int lz = x.l - lx - ly;
        if ((lx | ly | lz) & 1) continue;
        double v = 0.0;
        for (int k = 0; k < x.nprim; ++k) {
          const double g = hp.ax_exp[x.pptr + k];
          if (acut > 0.0 && g < acut) continue;  // the G = 0 term belongs to the range-separated part
          double m = hp.ax_coef[x.pptr + k] * std::pow(kPi / g, 1.5);
          const int pw[3] = {lx, ly, lz};
          for (int d = 0; d < 3; ++d) {
            double df = 1.0;
            for (int q = pw[d] - 1; q > 1; q -= 2) df *= q;
            m *= df / std::pow(2.0 * g, pw[d] / 2);
          }
          v += m;
        }
        SP[x.foff + ic] = v;
      }
  }
  HIPCHK(upload(d_kph, kph, st));
  HIPCHK(upload(d_kdiag, kdiag, st));
  HIPCHK(upload(d_SP, SP, st));
  if (do_g0) {
    HIPCHK(d_O.alloc((size_t)npair * nk * 36 * sizeof(double)));
    HIPCHK(d_Smn.alloc((size_t)nk * nao2 * 2 * sizeof(double)));
  }

  // ---------------------------------------------------------- SR plan
  // aux batches bounded by the scratch budget of X
  size_t free_b = 0;
  HIPCHK(mem_avail(&free_b));
  const double budget = std::min(mem_frac * (double)free_b, 64e9);
  batch_start.assign(1, 0);
  {
    int64_t nf = 0;
    for (int s = 0; s < nxs; ++s) {
      const int64_t add = ncart_h(hp.ax[s].l);
      if (nf > 0 && (double)(nf + add) * nb * nao2 * 8.0 > budget) {
        batch_start.push_back(s);
        nf = 0;
      }
      nf += add;
    }
    batch_start.push_back(nxs);
  }
  nbatch = (int)batch_start.size() - 1;
  int64_t max_bf = 0;
  for (int b = 0; b < nbatch; ++b) {
    int64_t nf = 0;
    for (int s = batch_start[b]; s < batch_start[b + 1]; ++s) nf += ncart_h(hp.ax[s].l);
    max_bf = std::max(max_bf, nf);
  }
  if (do_sr && (double)max_bf * nb * nao2 * 8.0 > 0.9 * (double)free_b)
    return fail(RSGDF_ENOMEM, "one aux shell's short-range scratch does not fit in device memory");
  if (do_sr) HIPCHK(d_X.alloc((size_t)max_bf * nb * nao2 * sizeof(double)));
  max_bf_el = max_bf * nao2;
  if (do_sr && own_y) {  // the fold's intermediate Y: nk^2 complex values per element of a pass
    size_t fr = 0;
    HIPCHK(mem_avail(&fr));
    set_fold_chunk(std::min(0.25 * mem_frac * (double)fr, 8e9));
    HIPCHK(d_Y.alloc((size_t)fchunk * nk * nk * 16));
    ybuf = d_Y.as<double>();
  }

  // triplets for all batches, grouped by (batch, lP, pair class)
  {
    const Screen &S = hp.scr;
    std::vector<std::vector<Triplet>> grp((size_t)nbatch * 24);
    for (int64_t t = 0; t < (int64_t)nxs * npair; ++t) {
      Triplet tr{};
      tr.aux = (int32_t)(t / npair);
      tr.pair = (int32_t)(t % npair);
      if (acut > 0.0) {  // split: aux shells with no compact primitive, pairs of diffuse shells
        const Pair &pq = hp.pairs[tr.pair];
        if (hp.ax[tr.aux].a_d <= 0.0) continue;
        bool anyc = false;
        for (int k = 0; k < hp.ao[pq.sa].nprim && !anyc; ++k) anyc = hp.ao_exp[hp.ao[pq.sa].pptr + k] >= acut;
        for (int k = 0; k < hp.ao[pq.sb].nprim && !anyc; ++k) anyc = hp.ao_exp[hp.ao[pq.sb].pptr + k] >= acut;
        if (!anyc) continue;
      }
      tr.rc_cut = hp.rc_t[t];
      tr.amp = hp.amp_t[t];
      tr.nwin = std::max(1, (int)std::ceil(tr.rc_cut / S.dR));
      if (tr.nwin > 256) return fail(RSGDF_EUNSUPPORTED, "R_c bound exceeds the window table (omega too small)");
      int b = 0;
      while (tr.aux >= batch_start[b + 1]) ++b;
      const Pair &p = hp.pairs[tr.pair];
      const int g = hp.ax[tr.aux].l * 6 + pair_class(hp.ao[p.sa].l, hp.ao[p.sb].l);
      grp[(size_t)b * 24 + g].push_back(tr);
    }
    tgrp_off.assign(1, 0);
    for (auto &g : grp) {
      trips.insert(trips.end(), g.begin(), g.end());
      tgrp_off.push_back((int)trips.size());
    }
  }
  ntrip = (int64_t)trips.size();
  {
    // the SR kernel packs lattice coordinates into 10-bit fields (|M| < 500)
    double rcmax = 0.0, r12max = 0.0, diam = 0.0;
    for (const Triplet &t : trips) rcmax = std::max(rcmax, t.rc_cut);
    for (const Pair &p : hp.pairs) r12max = std::max(r12max, p.R12sr);
    for (int d = 0; d < 3; ++d) diam += hp.lt.an[d];
    for (int d = 0; d < 3; ++d)
      if ((rcmax + r12max + 2.0 * diam) * hp.lt.bn[d] / (2.0 * kPi) + L.n[d] + 2 > 500.0)
        return fail(RSGDF_EUNSUPPORTED, "screening radius too large for the packed image coordinates");
  }
  // learned-screening candidates: (triplet t, pair image ii) has index
  // cand_off[t] + ii, ii over all images of the pair
  if (learned || logging) {
    cand_off.resize(ntrip);
    for (int64_t t = 0; t < ntrip; ++t) {
      cand_off[t] = ncand;
      ncand += hp.cls_off[(size_t)trips[t].pair * (nk + 1) + nk];
    }
  }
  // SR work list: a cost estimate per item (primitive triplets x pair images x
  // lattice vectors in the R_c ball x per-term operations) decides how many
  // waves share it, first by BvK cell ranges (disjoint outputs), then by
  // interleaved pair-image slices with private partial blocks.  The per-class
  // factors `split` (autotuner output) scale the target work per wave.
  pgrp_off.assign(1, 0);
  {
    // pair images inside R12 (all classes) per pair
    std::vector<int64_t> nimg_pair(npair, 0);
    for (int ip = 0; ip < npair; ++ip)
      for (int c = 0; c < nk; ++c) nimg_pair[ip] += hp.nsr[(size_t)ip * nk + c];
    std::vector<double> est(ntrip);
    parallel_for(ntrip, [&](int64_t t) {
      const Triplet &tr = trips[t];
      const Pair &pp = hp.pairs[tr.pair];
      const Shell &sA = hp.ao[pp.sa], &sB = hp.ao[pp.sb], &sP = hp.ax[tr.aux];
      const int64_t nimg = nimg_pair[tr.pair];
      const double nm = 4.18879020478639098 * tr.rc_cut * tr.rc_cut * tr.rc_cut / L.vol + 1.0;
      const int Lt = sP.l + sA.l + sB.l;
      // per (primitive triple, pair image, cell range): the group reduction, the
      // W table and the Cartesian components of the contraction, in flops; the
      // weight 13.6 is the least-squares ratio of the two costs over the 24
      // classes' standalone durations on the 8-atom 2x2x2 workload
      const int lab = sA.l + sB.l, nkx = (sP.l / 2 + 1) * (sP.l / 2 + 1) * (sP.l / 2 + 1);
      const int nblk = ncart_h(sP.l) * ncart_h(sA.l) * ncart_h(sB.l);
      const double ev = 2.0 * nherm(Lt) + 2.0 * ncart_h(sP.l) * nherm(lab) * nkx + 2.0 * nblk * nherm(lab);
      const double nranges = std::ceil((double)nk / std::min(nk, sr_cells_per_wave(nblk)));
      est[t] = (double)sA.nprim * sB.nprim * sP.nprim * (double)nimg * (nm * sr_term_flops(Lt) + 13.6 * nranges * ev);
    }, 1024);
    double tot = 0.0;
    for (int64_t t = 0; t < ntrip; ++t) tot += est[t];
    // target cost per wave: 8 waves per SIMD over the build
    const double target0 = std::max(tot / (8.0 * 1024.0), 1.0);
    const double part_budget = std::min(1.0e9, 0.05 * (double)free_b);  // bytes of partial blocks
    double part_bytes = 0.0;
    // per triplet: cell ranges of ncbw cells, nsl slices each, the first
    // partial group (if sliced) and the cost of each of its waves
    std::vector<int32_t> t_ncbw(ntrip), t_nsl(ntrip);
    std::vector<int64_t> t_pbase(ntrip, -1);
    std::vector<double> t_cost(ntrip);
    for (int b = 0; b < nbatch; ++b) {
      for (int g = 0; g < 24; ++g) {
        const double target = target0 * (split.empty() ? 1.0 : (double)split[g]);
        for (int t = tgrp_off[(size_t)b * 24 + g]; t < tgrp_off[(size_t)b * 24 + g + 1]; ++t) {
          const Triplet &tr = trips[t];
          const Pair &pp = hp.pairs[tr.pair];
          const int nblk = ncart_h(hp.ax[tr.aux].l) * ncart_h(hp.ao[pp.sa].l) * ncart_h(hp.ao[pp.sb].l);
          const int64_t want = std::max<int64_t>(1, (int64_t)std::ceil(est[t] / target));
          const int nsplit = (int)std::min<int64_t>(want, nk);
          int ncbw = (nk + nsplit - 1) / nsplit;
          ncbw = std::min(ncbw, sr_cells_per_wave(nblk));  // lane groups per wave (LDS accumulators)
          const int nranges = (nk + ncbw - 1) / ncbw;
          int nsl = (int)std::min<int64_t>(64, (want + nranges - 1) / nranges);
          if (nsl > 1 && part_bytes + (double)nsl * nk * nk * nblk * 8.0 > part_budget) nsl = 1;
          t_ncbw[t] = ncbw;
          t_nsl[t] = nsl;
          t_cost[t] = est[t] / ((double)nranges * nsl);
          if (nsl > 1) {
            t_pbase[t] = part_total;
            for (int r = 0; r < nranges; ++r) {
              const int cb0 = r * ncbw, ncb = std::min(ncbw, nk - cb0);
              SRPartGroup pg{};
              pg.trip = t;
              pg.cb0 = cb0;
              pg.ncb = ncb;
              pg.nslice = nsl;
              pg.part = part_total;
              pgroups.push_back(pg);
              part_total += (int64_t)nsl * ncb * nk * nblk;
              part_bytes += (double)nsl * ncb * nk * nblk * 8.0;
            }
          }
        }
      }
      pgrp_off.push_back((int)pgroups.size());
    }
    // the waves of a class launch, heaviest first (a triplet's waves share one
    // cost, so the triplets are sorted and their waves kept in range, slice
    // order); the class groups are independent and filled in parallel
    const int ngrp = (int)tgrp_off.size() - 1;
    wgrp_off.assign(ngrp + 1, 0);
    for (int g = 0; g < ngrp; ++g) {
      int64_t n = 0;
      for (int t = tgrp_off[g]; t < tgrp_off[g + 1]; ++t) n += (int64_t)((nk + t_ncbw[t] - 1) / t_ncbw[t]) * t_nsl[t];
      wgrp_off[g + 1] = (int)(wgrp_off[g] + n);
    }
    work.resize(wgrp_off[ngrp]);
    wgrp_cost.assign(ngrp, 0.0);
    parallel_for(ngrp, [&](int64_t g) {
      std::vector<int> idx;
      idx.reserve(tgrp_off[g + 1] - tgrp_off[g]);
      for (int t = tgrp_off[g]; t < tgrp_off[g + 1]; ++t) idx.push_back(t);
      std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return t_cost[x] > t_cost[y]; });
      double c = 0.0;
      SRWork *w = work.data() + wgrp_off[g];
      for (int t : idx) {
        const Triplet &tr = trips[t];
        const Pair &pp = hp.pairs[tr.pair];
        const int nblk = ncart_h(hp.ax[tr.aux].l) * ncart_h(hp.ao[pp.sa].l) * ncart_h(hp.ao[pp.sb].l);
        const int ncbw = t_ncbw[t], nsl = t_nsl[t], nranges = (nk + ncbw - 1) / ncbw;
        int64_t pbase = t_pbase[t];
        for (int r = 0; r < nranges; ++r) {
          const int cb0 = r * ncbw, ncb = std::min(ncbw, nk - cb0);
          for (int sl = 0; sl < nsl; ++sl, ++w) {
            *w = SRWork{};
            w->trip = t;
            w->cb0 = (int16_t)cb0;
            w->ncb = (int16_t)ncb;
            w->slice = (int16_t)sl;
            w->nslice = (int16_t)nsl;
            w->cell = 0;
            w->part = (nsl > 1) ? pbase + (int64_t)sl * ncb * nk * nblk : -1;
            c += t_cost[t];
          }
          if (nsl > 1) pbase += (int64_t)nsl * ncb * nk * nblk;
        }
      }
      wgrp_cost[g] = c;
    }, 1);
    // element prefix sums of the partial groups (per batch)
    for (int b = 0; b < nbatch; ++b) {
      int64_t off = 0;
      for (int i = pgrp_off[b]; i < pgrp_off[b + 1]; ++i) {
        SRPartGroup &pg = pgroups[i];
        const Pair &pp = hp.pairs[trips[pg.trip].pair];
        const int nblk = ncart_h(hp.ax[trips[pg.trip].aux].l) * ncart_h(hp.ao[pp.sa].l) * ncart_h(hp.ao[pp.sb].l);
        pg.elem_off = off;
        off += (int64_t)pg.ncb * nk * nblk;
      }
    }
  }
  nwork = (int64_t)work.size();
  if (do_sr) {
    HIPCHK(upload(d_trip, trips, st));
    HIPCHK(upload(d_work, work, st));
    HIPCHK(upload(d_pgrp, pgroups, st));
    HIPCHK(d_part.alloc((size_t)std::max<int64_t>(part_total, 1) * sizeof(double)));
    HIPCHK(d_cnt.alloc((size_t)std::max<int64_t>(nwork, 1) * 4 * sizeof(long long)));
  }
  base.ao = d_ao.as<Shell>();
  base.ax = d_ax.as<Shell>();
  base.ao_exp = d_aoe.as<double>();
  base.ao_coef = d_aoc.as<double>();
  base.ax_exp = d_axe.as<double>();
  base.ax_coef = d_axc.as<double>();
  base.ao_c1s = d_aoc1.as<double>();
  base.ax_c1s = d_axc1.as<double>();
  base.pairs = d_pairs.as<Pair>();
  base.cls_off = d_coff.as<int32_t>();
  base.nsr = d_nsr.as<int32_t>();
  base.img = d_img.as<double>();
  base.trip = d_trip.as<Triplet>();
  base.part = d_part.as<double>();
  base.lat = L;
  base.omega = omega;
  base.eps = thresh;
  base.dR = hp.scr.dR;
  base.ncell_nf = hp.scr.ncell_nf;
  base.ncell_r0 = hp.scr.r0;
  base.boys = d_boys.as<double>();
  base.acut = acut;
  base.X = d_X.as<double>();
  base.nao = (int32_t)nao;
  if (do_sr && (learned || logging)) {
    HIPCHK(upload(d_coffc, cand_off, st));
    base.cand_off = d_coffc.as<int64_t>();
  }
  if (do_sr && learned) {
    HIPCHK(d_mask.alloc((size_t)std::max<int64_t>(ncand, 1)));
    HIPCHK(d_mlp.alloc(kMlpNParam * sizeof(float)));
    HIPCHK(hipMemcpyAsync(d_mlp.p, o.mlp_weights, kMlpNParam * sizeof(float), hipMemcpyHostToDevice, st));
    HIPCHK(d_nskip.alloc(sizeof(long long)));
    base.mask = d_mask.as<uint8_t>();
  }
  if (do_sr && logging) {
    HIPCHK(d_logmag.alloc((size_t)std::max<int64_t>(ncand, 1) * nk * sizeof(float)));
    base.logmag = d_logmag.as<float>();
  }
  // per-batch parameter blocks of the SR kernels (one cell)
  if (do_sr) {
    prms.resize(nbatch);
    for (int b = 0; b < nbatch; ++b) prms[b] = batch_params(b);
    HIPCHK(upload(d_prm, prms, st));
  }

  // ---------------------------------------------------------- LR plan
  if (do_lr) {
    std::vector<double> qv15d, qv15c;
    std::vector<int64_t> qoff15d, qoff15c;
    make_qsets(hp.lt, hp.kvec, omega, g_thr, qv, qoff);
    if (acut > 0.0) {
      // q spheres of Eq. M15: a diffuse aux function (exponent < acut) has
      // decayed to g_thr at q^2 = 4 acut ln(1/g_thr); a diffuse-diffuse pair
      // density (exponent sum < 2 acut) at twice that
      make_qsets_sphere(hp.lt, hp.kvec, 4.0 * acut * std::log(1.0 / g_thr), qv15d, qoff15d);
      make_qsets_sphere(hp.lt, hp.kvec, 8.0 * acut * std::log(1.0 / g_thr), qv15c, qoff15c);
    }
    {
      auto add = [&](const std::vector<int64_t> &qo, int amode, int pmode, int undamped) {
        auto pt = std::make_unique<LRPart>();
        pt->qoff = qo;
        pt->nq_tot = qo.back();
        pt->amode = amode;
        pt->pmode = pmode;
        pt->undamped = undamped;
        lrp.push_back(std::move(pt));
      };
      if (acut > 0.0) {
        add(qoff, 1, 1, 0);     // (C | cc + cd), range-separated long range
        add(qoff15d, 2, 0, 1);  // (D | all pairs), Eq. M15
        add(qoff15c, 1, 2, 1);  // (C | dd), Eq. M15
      } else {
        add(qoff, 0, 0, 0);
      }
    }
    nq_tot = 0;
    for (auto &pt : lrp) nq_tot += pt->nq_tot;
    // k-pairs per class
    cls_kp.assign(nk, {});
    for (int t = 0; t < nkp; ++t) {
      const int k1 = hp.kp1[t], k2 = hp.kp2[t];
      const int j1[3] = {k1 / (L.n[1] * L.n[2]), (k1 / L.n[2]) % L.n[1], k1 % L.n[2]};
      const int j2[3] = {k2 / (L.n[1] * L.n[2]), (k2 / L.n[2]) % L.n[1], k2 % L.n[2]};
      int c = 0;
      for (int d = 0; d < 3; ++d) c = c * L.n[d] + ((j2[d] - j1[d]) % L.n[d] + L.n[d]) % L.n[d];
      cls_kp[c].push_back(t);
    }
    for (size_t ip = 0; ip < lrp.size(); ++ip) {
      LRPart &pt = *lrp[ip];
      HIPCHK(upload(pt.d_q, (ip == 0) ? qv : (ip == 1 ? qv15d : qv15c), st));
      HIPCHK(pt.d_A.alloc((size_t)naux * std::max<int64_t>(pt.nq_tot, 1) * 2 * sizeof(double)));
      if (o.lr_precision == RSGDF_FP32)  // FP32 operands
        HIPCHK(pt.d_A32.alloc((size_t)naux * std::max<int64_t>(pt.nq_tot, 1) * 2 * sizeof(float)));
    }
    // per q chunk: pair transforms binned by BvK class (I), the k2 phases of
    // the class's k-pairs (B), then the G-space contraction
    int max_kpi = 0;
    for (auto &v : cls_kp) max_kpi = std::max<int>(max_kpi, (int)v.size());
    // I and B per q chunk.  Every chunk's contraction reads and writes the
    // class's output rows once more, so the chunks are long: a fixed 48 GB
    // when half the memory share allows it (on the 3x3x3 workload 16 GB gave
    // 16 chunks per class, 1.6 TB of output traffic per build), else the
    // largest power of two of q that fits.  The chunk boundaries set the
    // order in which the q sums are added, so they must not follow the free
    // memory from call to call: this keeps builds bit-reproducible.
    const double per_q = (double)(nk + std::max(1, max_kpi)) * nao2 * 16.0;
    const double avail = 0.5 * mem_frac * (double)free_b, fixed = 48e9;
    if (avail >= fixed) {
      qchunk = (int64_t)(fixed / per_q);
    } else {
      const int64_t fit = (int64_t)(avail / per_q);
      qchunk = 1;
      while (qchunk * 2 <= fit) qchunk *= 2;
    }
    qchunk = std::max<int64_t>(1, std::min<int64_t>(qchunk, 8192));
    int64_t max_nq = 0;
    for (auto &pt : lrp)
      for (int c = 0; c < nk; ++c) max_nq = std::max(max_nq, pt->qoff[c + 1] - pt->qoff[c]);
    qchunk = std::min(qchunk, std::max<int64_t>(max_nq, 1));
    if (o.lr_precision == RSGDF_F16X3)  // whole 32-q blocks per chunk (the split format's unit)
      qchunk = std::max<int64_t>(kF16Blk * kF16Grp, qchunk / (kF16Blk * kF16Grp) * (kF16Blk * kF16Grp));
    HIPCHK(d_amax.alloc((size_t)qchunk * sizeof(double)));
    HIPCHK(d_I.alloc((size_t)nk * qchunk * nao2 * 2 * sizeof(double)));
    HIPCHK(d_B.alloc((size_t)max_kpi * qchunk * nao2 * 2 * sizeof(double)));
    if (o.lr_precision != RSGDF_FP64)  // the FP64 innermost columns
      HIPCHK(d_Bhi.alloc((size_t)max_kpi * kLrNqHi * nao2 * 2 * sizeof(double)));
    if (o.lr_precision == RSGDF_F16X3)  // halves [nb][naux][4][32], then exponents [nb][naux]
      HIPCHK(d_Asp.alloc(f16_split_bytes(naux, qchunk)));
    HIPCHK(d_kp.alloc((size_t)std::max(nkp, 1) * sizeof(int32_t)));
    HIPCHK(d_nterm.alloc(sizeof(long long)));
    // k-pair lists and the phases e^{+i k2.L_c} of every class, as a table
    // [cell c][k-pair of the class] with the k-pairs contiguous and padded with
    // zeros to whole passes of the k2-phase kernels
    for (int c = 0; c < nk; ++c) {
      const int nkpi = (int)cls_kp[c].size(), kpad = kphase_kpad(std::max(nkpi, 1));
      for (int t : cls_kp[c]) kpl.push_back(t);
      kpl_off.push_back((int64_t)kpl.size());
      ph_off.push_back((int64_t)(phl.size() / 2));
      for (int cell = 0; cell < nk; ++cell)
        for (int k = 0; k < kpad; ++k) {
          const int k2 = k < nkpi ? hp.kp2[cls_kp[c][k]] : -1;
          phl.push_back(k2 >= 0 ? kph[2 * ((size_t)k2 * nk + cell)] : 0.0);
          phl.push_back(k2 >= 0 ? kph[2 * ((size_t)k2 * nk + cell) + 1] : 0.0);
        }
    }
    HIPCHK(d_ph.alloc(std::max<size_t>(phl.size(), 2) * sizeof(double)));
    if (!kpl.empty())
      HIPCHK(hipMemcpyAsync(d_kp.p, kpl.data(), kpl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!phl.empty())
      HIPCHK(hipMemcpyAsync(d_ph.p, phl.data(), phl.size() * sizeof(double), hipMemcpyHostToDevice, st));
  }
  // uploads read host vectors that live in this object; make them complete
  HIPCHK(hipStreamSynchronize(st));
  t_plan = ms_since(t_start);
  return RSGDF_OK;
}

SRParams Job::batch_params(int b) const {
  SRParams p = base;
  p.aux_f0 = (int32_t)hp.ax[batch_start[b]].foff;
  int64_t nf = 0;
  for (int s = batch_start[b]; s < batch_start[b + 1]; ++s) nf += ncart_h(hp.ax[s].l);
  p.naux_b = (int32_t)nf;
  return p;
}

// device work before the SR sums: G = 0 overlaps, learned keep mask, zeroed counters
int Job::enqueue_pre(hipStream_t st) {
  if (do_g0) {
    OvlParams op{d_ao.as<Shell>(), d_aoe.as<double>(), d_aoc.as<double>(), d_pairs.as<Pair>(),
                 d_coff.as<int32_t>(), d_img.as<double>(), npair, hp.lt.L.nk, d_O.as<double>()};
    op.acut = acut;
    SmnParams sp{d_ao.as<Shell>(), d_pairs.as<Pair>(), d_O.as<double>(), d_kph.as<double>(), npair, nk,
                 (int32_t)nao, 0, d_Smn.as<double>()};
    HIPCHK(launch_overlaps(op, sp, st));
  }
  if (do_sr) {
    HIPCHK(launch_zero(d_cnt.p, (size_t)std::max<int64_t>(nwork, 1) * 4 * sizeof(long long), st));
    if (learned) {
      // drop iff inside the training range and prediction + margin < log10(thresh)
      HIPCHK(launch_zero(d_nskip.p, sizeof(long long), st));
      const float cut = (float)(std::log10(thresh) - o.mlp_margin);
      HIPCHK(launch_mlp_mask(base, (int)ntrip, ncand, d_mlp.as<float>(), cut, d_mask.as<uint8_t>(),
                             d_nskip.as<long long>(), st));
    }
    if (logging)  // NaN marks candidates the image loop never reached
      HIPCHK(hipMemsetAsync(d_logmag.p, 0xff, (size_t)std::max<int64_t>(ncand, 1) * nk * sizeof(float), st));
  }
  return RSGDF_OK;
}

// SR sums of aux batch b: zero X and the partial blocks, class launches in
// decreasing cost order round-robin over the side streams, joined back to st
int Job::enqueue_zero(int b, hipStream_t st) {
  if (!do_sr) return RSGDF_OK;
  const SRParams prm = batch_params(b);
  HIPCHK(launch_zero(d_X.p, (size_t)prm.naux_b * nb * nao2 * sizeof(double), st));
  if (part_total > 0) HIPCHK(launch_zero(d_part.p, (size_t)part_total * sizeof(double), st));
  return RSGDF_OK;
}

int Job::enqueue_sr(int b, hipStream_t st, const std::vector<hipStream_t> &ss, hipEvent_t evf, hipEvent_t *evj) {
  if (!do_sr) return RSGDF_OK;
  int rc = enqueue_zero(b, st);
  if (rc) return rc;
  if (ss.empty()) {  // no side streams: the classes in turn on st, no events
    for (int g = 0; g < 24; ++g) {
      const int w0 = wgrp_off[(size_t)b * 24 + g], w1 = wgrp_off[(size_t)b * 24 + g + 1];
      if (w1 > w0)
        HIPCHK(launch_sr3c(g / 6, g % 6, d_prm.as<SRParams>() + b, d_work.as<SRWork>(), d_cnt.as<long long>(), w0,
                           w1 - w0, st));
    }
    return enqueue_reduce(b, st);
  }
  HIPCHK(hipEventRecord(evf, st));
  for (auto s_ : ss) HIPCHK(hipStreamWaitEvent(s_, evf, 0));
  std::vector<int> order(24);
  for (int g = 0; g < 24; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return wgrp_cost[(size_t)b * 24 + x] > wgrp_cost[(size_t)b * 24 + y]; });
  // heaviest class first, each onto the side stream with the least estimated work so far
  std::vector<double> load(ss.size(), 0.0);
  for (int g : order) {
    const int w0 = wgrp_off[(size_t)b * 24 + g], w1 = wgrp_off[(size_t)b * 24 + g + 1];
    if (w1 == w0) continue;
    const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += wgrp_cost[(size_t)b * 24 + g];
    HIPCHK(launch_sr3c(g / 6, g % 6, d_prm.as<SRParams>() + b, d_work.as<SRWork>(), d_cnt.as<long long>(), w0,
                       w1 - w0, ss[k]));
  }
  for (size_t i = 0; i < ss.size(); ++i) {
    HIPCHK(hipEventRecord(evj[i], ss[i]));
    HIPCHK(hipStreamWaitEvent(st, evj[i], 0));
  }
  return enqueue_reduce(b, st);
}

// sum the split items of batch b into X
int Job::enqueue_reduce(int b, hipStream_t st) {
  const int pg0 = pgrp_off[b], pg1 = pgrp_off[b + 1];
  if (!do_sr || pg1 <= pg0) return RSGDF_OK;
  const SRPartGroup &last = pgroups[pg1 - 1];
  const Pair &pp = hp.pairs[trips[last.trip].pair];
  const int nblk = ncart_h(hp.ax[trips[last.trip].aux].l) * ncart_h(hp.ao[pp.sa].l) * ncart_h(hp.ao[pp.sb].l);
  const int64_t nelem = last.elem_off + (int64_t)last.ncb * nk * nblk;
  HIPCHK(launch_sr_reduce(batch_params(b), d_pgrp.as<SRPartGroup>() + pg0, pg1 - pg0, nelem, st));
  return RSGDF_OK;
}

// Bloch fold (+ G = 0 term) of aux batch b into the output
int Job::enqueue_fold(int b, hipStream_t st) {
  const SRParams prm = batch_params(b);
  const int64_t f0 = prm.aux_f0, nf = prm.naux_b;
  FoldParams fp{};
  fp.kph = d_kph.as<double>();
  fp.X = do_sr ? d_X.as<double>() : nullptr;
  fp.Y = do_sr ? ybuf : nullptr;
  fp.out = d_out;
  fp.kdiag = d_kdiag.as<int32_t>();
  fp.kp1 = d_kp1.as<int32_t>();
  fp.tile_k2 = d_tk2.as<int32_t>();
  fp.tile_kp = d_tkp.as<int32_t>();
  fp.SP = d_SP.as<double>() + f0;
  fp.Smn = do_g0 ? d_Smn.as<double>() : nullptr;
  fp.g0fac = do_g0 ? kPi / (hp.lt.L.vol * omega * omega) : 0.0;
  fp.ne = nf * nao2;
  fp.echunk = do_sr ? fchunk : std::max<int64_t>(fp.ne, 1);
  fp.out_off = f0 * nao2;
  fp.plane = naux * nao2;
  fp.nkp = nkp;
  fp.nk = nk;
  fp.nao2 = (int32_t)nao2;
  fp.ntile = ftiles;
  fp.tk = ftk;
  HIPCHK(launch_fold(fp, st));
  return RSGDF_OK;
}

// long-range part, accumulated into the output; gev (optional) receives
// event pairs around each contraction launch
int Job::enqueue_lr(hipStream_t st, std::vector<hipEvent_t> *gev) {
  if (!do_lr) return RSGDF_OK;
  const Lattice &L = hp.lt.L;
  HIPCHK(launch_zero(d_nterm.p, sizeof(long long), st));
  const bool f32 = o.lr_precision != RSGDF_FP64;
  const int lr_nq_hi = kLrNqHi;
  for (auto &ptp : lrp) {
    LRPart &pt = *ptp;
    if (pt.nq_tot == 0) continue;
    AuxFTParams ap{d_ax.as<Shell>(), d_axe.as<double>(), d_axc.as<double>(), pt.d_q.as<double>(), (int32_t)pt.nq_tot,
                   (int32_t)nxs, (int32_t)naux, 0, 4.0 * kPi / L.vol, omega, pt.d_A.as<double>()};
    ap.acut = acut;
    ap.amode = pt.amode;
    ap.undamped = pt.undamped;
    HIPCHK(launch_auxft(ap, st));
    if (o.lr_precision == RSGDF_FP32)
      HIPCHK(launch_to_f32(pt.d_A.as<double>(), pt.d_A32.as<float>(), naux * pt.nq_tot * 2, st));
    for (int c = 0; c < nk; ++c) {
      const int nkpi = (int)cls_kp[c].size();
      const int64_t nqc = pt.qoff[c + 1] - pt.qoff[c];
      if (nkpi == 0 || nqc == 0) continue;
      for (int64_t q0 = 0; q0 < nqc; q0 += qchunk) {
        const int nq = (int)std::min<int64_t>(qchunk, nqc - q0);
        HIPCHK(launch_amax(pt.d_A.as<double>() + 2 * (pt.qoff[c] + q0), pt.nq_tot, (int)naux, nq,
                           d_amax.as<double>(), st));
        PairFTParams pp{};
        pp.ao = d_ao.as<Shell>();
        pp.ao_exp = d_aoe.as<double>();
        pp.ao_coef = d_aoc.as<double>();
        pp.pairs = d_pairs.as<Pair>();
        pp.plist = d_plist.as<int32_t>();
        for (int g = 0; g < 7; ++g) pp.pgrp[g] = plist_grp[g];
        pp.cls_off = d_coff.as<int32_t>();
        pp.img = d_img.as<double>();
        pp.q = pt.d_q.as<double>() + 3 * (pt.qoff[c] + q0);
        pp.amax = d_amax.as<double>();
        pp.npair = npair;
        pp.nq = nq;
        pp.nao = (int32_t)nao;
        pp.nk = nk;
        for (int d = 0; d < 3; ++d) pp.kn[d] = L.n[d];
        pp.kcls[0] = c / (L.n[1] * L.n[2]);
        pp.kcls[1] = (c / L.n[2]) % L.n[1];
        pp.kcls[2] = c % L.n[2];
        pp.eps = 1e-8 * thresh;
        pp.B = d_I.as<double>();
        pp.nterm = d_nterm.as<long long>();
        pp.acut = acut;
        pp.pmode = pt.pmode;
        HIPCHK(launch_pairft_binned(pp, st));
        // A class of at most 4 nq_hi q is contracted in FP64 in every form: the
        // reduced-precision kernels would take its first nq_hi q (or all of them)
        // in FP64 on the vector ALUs, slower than the FP64 matrix-core kernel,
        // and FP64 is the more accurate.
        const int prec = (f32 && q0 == 0 && nqc <= 4 * lr_nq_hi) ? RSGDF_FP64 : o.lr_precision;
        const int nq_hi = (q0 == 0 && prec != RSGDF_FP64) ? lr_nq_hi : 0;  // q sorted by |q|: the class's innermost shell
        const bool split = prec == RSGDF_F16X3;
        const int nb = f16_nblk(nq);
        // split format: halves, then the exponents at a 256-byte boundary
        uint16_t *Xa = d_Asp.as<uint16_t>(), *Xb = d_B.as<uint16_t>();
        int32_t *Ea = reinterpret_cast<int32_t *>(d_Asp.as<char>() + f16_split_eoff(naux, nb));
        int32_t *Eb = reinterpret_cast<int32_t *>(d_B.as<char>() + f16_split_eoff((int64_t)nkpi * nao2, nb));
        if (split) {
          HIPCHK(launch_asplit(pt.d_A.as<double>() + 2 * (pt.qoff[c] + q0), pt.nq_tot, (int)naux, nq, nq_hi, Xa, Ea,
                               st));
          HIPCHK(launch_kphase_split(d_I.as<double>(), d_ph.as<double>() + 2 * ph_off[c], Xb, Eb,
                                     nq_hi ? d_Bhi.as<double>() : nullptr, nq_hi, nk, nkpi, nq, nao2, st));
        } else {
          HIPCHK(launch_kphase(d_I.as<double>(), d_ph.as<double>() + 2 * ph_off[c], d_B.p, prec == RSGDF_FP32,
                               nq_hi ? d_Bhi.as<double>() : nullptr, nq_hi, nk, nkpi, nq, nao2, st));
        }
        LRGemmParams gp{};
        gp.A = pt.d_A.as<double>() + 2 * (pt.qoff[c] + q0);
        gp.lda = pt.nq_tot;
        gp.B = d_B.as<double>();
        gp.A32 = prec == RSGDF_FP32 ? pt.d_A32.as<float>() + 2 * (pt.qoff[c] + q0) : nullptr;
        gp.B32 = prec == RSGDF_FP32 ? d_B.as<float>() : nullptr;
        if (split) {
          gp.Xa = Xa;
          gp.Ea = Ea;
          gp.Xb = Xb;
          gp.Eb = Eb;
          gp.nb = nb;
        }
        gp.Bhi = nq_hi ? d_Bhi.as<double>() : nullptr;
        gp.out = d_out;
        gp.kp_of = d_kp.as<int32_t>() + kpl_off[c];
        gp.plane = naux * nao2;
        gp.naux = (int32_t)naux;
        gp.nq = nq;
        gp.nmn = (int32_t)nao2;
        gp.nq_hi = nq_hi;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (gev) {
          HIPCHK(hipEventCreate(&e0));
          HIPCHK(hipEventCreate(&e1));
          gev->push_back(e0);
          gev->push_back(e1);
          HIPCHK(hipEventRecord(e0, st));
        }
        HIPCHK(launch_lr_gemm_tiled(prec, gp, 0, nkpi, st));
        if (gev) HIPCHK(hipEventRecord(e1, st));
        lr_flops += 8.0 * (double)naux * nq * (double)nao2 * nkpi;
      }
    }
  }
  return RSGDF_OK;
}

// read back counters (after the device work has completed) and fill stats;
// cnt_host: per-work-item counters if already copied (batch), else read here
int Job::finish(hipStream_t st, const long long *cnt_host) {
  if (!logging && !tune && !out->on_device)
    HIPCHK(hipMemcpyAsync(out->data, d_out, (size_t)need, hipMemcpyDeviceToHost, st));
  if (do_lr) HIPCHK(hipMemcpyAsync(&n_lr, d_nterm.p, sizeof(long long), hipMemcpyDeviceToHost, st));
  if (learned && do_sr) HIPCHK(hipMemcpyAsync(&nskip, d_nskip.p, sizeof(long long), hipMemcpyDeviceToHost, st));
  counts.assign((size_t)nwork * 4, 0);
  if (do_sr && nwork > 0) {
    if (cnt_host) std::copy(cnt_host, cnt_host + nwork * 4, counts.begin());
    else HIPCHK(hipMemcpyAsync(counts.data(), d_cnt.p, counts.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (ctl) {
    ctl->ncand = ncand;
    ctl->nskip = nskip;
  }
  if (logging && do_sr && ncand > 0) {
    // targets of the candidates the image loop reached, a seeded sample of
    // them, and their features; below log10(thresh) - 4 every candidate is
    // equally negligible
    DBuf d_tgt;
    HIPCHK(d_tgt.alloc((size_t)ncand * sizeof(float)));
    HIPCHK(launch_log_target(d_logmag.as<float>(), nk, ncand, (float)(std::log10(thresh) - 4.0), d_tgt.as<float>(),
                             st));
    std::vector<float> tgt(ncand);
    HIPCHK(hipMemcpyAsync(tgt.data(), d_tgt.p, (size_t)ncand * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int64_t> sel;
    const uint64_t lim = (ctl->sample_frac >= 1.0) ? ~0ull : (uint64_t)(ctl->sample_frac * 18446744073709551616.0);
    for (int64_t c = 0; c < ncand; ++c)
      if (std::isfinite(tgt[c]) && splitmix64(ctl->seed ^ (uint64_t)c) <= lim) sel.push_back(c);
    ctl->tgt.resize(sel.size());
    for (size_t i = 0; i < sel.size(); ++i) ctl->tgt[i] = tgt[sel[i]];
    ctl->feat.resize(sel.size() * kMlpF);
    if (!sel.empty()) {
      DBuf d_sel, d_feat;
      HIPCHK(upload(d_sel, sel, st));
      HIPCHK(d_feat.alloc(sel.size() * kMlpF * sizeof(float)));
      HIPCHK(launch_features(base, (int)ntrip, d_sel.as<int64_t>(), (int64_t)sel.size(), d_feat.as<float>(), st));
      HIPCHK(hipMemcpyAsync(ctl->feat.data(), d_feat.p, sel.size() * kMlpF * sizeof(float), hipMemcpyDeviceToHost,
                            st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  if (out) {
    out->nkpair = nkp;
    out->naux = naux;
    out->nao = nao;
  }
  if (out && out->stats) {
    rsgdf_stats &s = *out->stats;
    std::memset(&s, 0, sizeof(s));
    s.t_plan_ms = t_plan;
    s.t_sr_ms = t_sr;
    s.t_fold_ms = t_fold;
    s.t_lr_ms = t_lr;
    s.n_lr_terms = n_lr;
    s.t_lr_gemm_ms = t_lr_gemm;
    s.lr_gemm_flops = lr_flops;
    s.n_g_total = nq_tot;
    s.n_triplets = ntrip;
    s.n_aux_batches = nbatch;
    s.bytes_out = need;
    s.n_screen_candidates = ncand;
    s.n_screen_skipped = nskip;
    if (do_sr && ntrip > 0) {
      std::vector<long long> tterms(ntrip, 0), tshell(ntrip, 0), tcontr(ntrip, 0);
      for (int64_t w = 0; w < nwork; ++w) {
        tterms[work[w].trip] += counts[(size_t)w * 4];
        tcontr[work[w].trip] += counts[(size_t)w * 4 + 1];
        tshell[work[w].trip] += counts[(size_t)w * 4 + 2];
      }
      double flops = 0.0;
      for (int b = 0; b < nbatch; ++b)
        for (int g = 0; g < 24; ++g) {
          const int lP = g / 6, pc = g % 6;
          static const int la_of[6] = {0, 1, 1, 2, 2, 2}, lb_of[6] = {0, 0, 1, 0, 1, 2};
          const int Lt = lP + la_of[pc] + lb_of[pc];
          long long nt = 0, nc = 0;
          for (int t = tgrp_off[(size_t)b * 24 + g]; t < tgrp_off[(size_t)b * 24 + g + 1]; ++t) {
            nt += tterms[t];
            nc += tcontr[t];
            s.n_sr_shell_terms += tshell[t];
          }
          s.n_sr_terms += nt;
          flops += (double)nt * sr_term_flops(Lt) + (double)nc * sr_contr_flops(lP, la_of[pc], lb_of[pc]);
        }
      s.sr_flops = flops;
      // optional per-item dump (aux shell, pair, l_P, l_a, l_b, terms, contractions, shell terms,
      // R_c cut) for workload analysis
      if (const char *fn = std::getenv("RSGDF_COUNTS_FILE")) {
        if (FILE *f = std::fopen(fn, "w")) {
          for (int64_t t = 0; t < ntrip; ++t) {
            const Pair &pr = hp.pairs[trips[t].pair];
            std::fprintf(f, "%d %d %d %d %d %lld %lld %lld %.3f\n", trips[t].aux, trips[t].pair, hp.ax[trips[t].aux].l,
                         hp.ao[pr.sa].l, hp.ao[pr.sb].l, tterms[t], tcontr[t], tshell[t], trips[t].rc_cut);
          }
          std::fclose(f);
        }
      }
    }
  }
  return RSGDF_OK;
}

struct EventSet {
  std::vector<hipEvent_t> e;
  ~EventSet() {
    for (hipEvent_t x : e) (void)hipEventDestroy(x);
  }
  int make(int n, unsigned flags) {
    for (int i = 0; i < n; ++i) {
      hipEvent_t x;
      HIPCHK(hipEventCreateWithFlags(&x, flags));
      e.push_back(x);
    }
    return RSGDF_OK;
  }
};

// one build on one stream, timed per phase with events
int build_impl(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
               const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt, rsgdf_out *out,
               LearnCtl *ctl, bool diag_only = false) {
  const auto t_start = std::chrono::steady_clock::now();
  g_err.clear();
  Job j;
  j.hp.diag_only = diag_only;
  j.cell = cell;
  j.basis = basis;
  j.auxbasis = auxbasis;
  j.kmesh = kmesh;
  j.omega = omega;
  j.thresh = thresh;
  j.out = out;
  j.ctl = ctl;
  j.o.g_thresh = -1.0;
  j.o.lr_precision = RSGDF_FP64;
  j.o.screening = RSGDF_SCREEN_RIGOROUS;
  j.o.parts = RSGDF_PART_ALL;
  if (opt) j.o = *opt;
  hipStream_t st = out ? reinterpret_cast<hipStream_t>(out->stream) : nullptr;
  int rc = j.prepare(st, 0.45);
  if (rc) return rc;
  std::vector<hipStream_t> ss;
  if ((rc = side_streams(ss, 3))) return rc;
  EventSet ev, evs;
  if ((rc = ev.make(6, 0))) return rc;
  if ((rc = evs.make((int)ss.size() + 1, hipEventDisableTiming))) return rc;
  if ((rc = j.enqueue_pre(st))) return rc;
  for (int b = 0; b < j.nbatch; ++b) {
    HIPCHK(hipEventRecord(ev.e[0], st));
    if ((rc = j.enqueue_sr(b, st, ss, evs.e[0], &evs.e[1]))) return rc;
    HIPCHK(hipEventRecord(ev.e[1], st));
    if (!j.logging && (rc = j.enqueue_fold(b, st))) return rc;
    HIPCHK(hipEventRecord(ev.e[2], st));
    HIPCHK(hipEventSynchronize(ev.e[2]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    j.t_sr += ms;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[1], ev.e[2]));
    j.t_fold += ms;
  }
  if (j.do_lr) {
    EventSet gev;
    HIPCHK(hipEventRecord(ev.e[3], st));
    if ((rc = j.enqueue_lr(st, &gev.e))) return rc;
    HIPCHK(hipEventRecord(ev.e[4], st));
    HIPCHK(hipEventSynchronize(ev.e[4]));
    HIPCHK(hipEventElapsedTime(&j.t_lr, ev.e[3], ev.e[4]));
    for (size_t i = 0; i < gev.e.size(); i += 2) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, gev.e[i], gev.e[i + 1]));
      j.t_lr_gemm += ms;
    }
  }
  if ((rc = j.finish(st, nullptr))) return rc;
  if (out && out->stats) out->stats->t_total_ms = ms_since(t_start);
  return RSGDF_OK;
}


// rigorous, short-range-only trial of one cell with uniform split factor f:
// per-class kernel times, classes launched one after another on st
int tune_trial(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis, const int32_t kmesh[3],
               double omega, double thresh, float f, hipStream_t st, double *class_ms) {
  Job j;
  rsgdf_out dummy{};
  dummy.stream = st;
  std::vector<float> fs(24, f);
  j.cell = cell;
  j.basis = basis;
  j.auxbasis = auxbasis;
  j.kmesh = kmesh;
  j.omega = omega;
  j.thresh = thresh;
  j.out = &dummy;
  j.tune = true;
  j.o.g_thresh = -1.0;
  j.o.parts = RSGDF_PART_SR;
  j.o.sr_split = fs.data();
  int rc = j.prepare(st, 0.45);
  if (rc) return rc;
  if ((rc = j.enqueue_pre(st))) return rc;
  EventSet ev;
  if ((rc = ev.make(2 * 24, 0))) return rc;
  for (int g = 0; g < 24; ++g) class_ms[g] = 0.0;
  for (int b = 0; b < j.nbatch; ++b) {
    if ((rc = j.enqueue_zero(b, st))) return rc;
    for (int g = 0; g < 24; ++g) {
      const int w0 = j.wgrp_off[(size_t)b * 24 + g], w1 = j.wgrp_off[(size_t)b * 24 + g + 1];
      HIPCHK(hipEventRecord(ev.e[2 * g], st));
      if (w1 > w0)
        HIPCHK(launch_sr3c(g / 6, g % 6, j.d_prm.as<SRParams>() + b, j.d_work.as<SRWork>(), j.d_cnt.as<long long>(),
                           w0, w1 - w0, st));
      HIPCHK(hipEventRecord(ev.e[2 * g + 1], st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int g = 0; g < 24; ++g) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev.e[2 * g], ev.e[2 * g + 1]));
      class_ms[g] += ms;
    }
  }
  return RSGDF_OK;
}

}  // namespace

// Batch of cells: the SR work items of all cells are merged into one launch
// per angular-momentum class (a cost-sorted (cell, item) queue drained by the
// hardware dispatcher); reduce, fold and the long-range part follow per cell.
// The whole device sequence is captured once into a graph and replayed.
struct rsgdf_batch {
  std::vector<std::unique_ptr<Job>> jobs;
  DBuf d_prm, d_work, d_cnt, d_Y;  // d_Y: the fold intermediate shared by the cells
  std::vector<int> cls_off;                   // [25] merged work offsets per class
  std::vector<double> cls_cost;               // [24]
  std::vector<std::pair<int, int64_t>> from;  // merged item -> (job, local item)
  hipStream_t st = nullptr;      // the caller's stream: uploads and replays
  hipStream_t cap = nullptr;     // library stream the sequence is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  EventSet evs;
  ~rsgdf_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

int batch_capture(rsgdf_batch &B) {
  // the caller's stream may be the null stream, which cannot be captured
  HIPCHK(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
  hipStream_t st = B.cap;
  std::vector<hipStream_t> ss;
  int rc = side_streams(ss, 4);
  if (rc) return rc;
  if ((rc = B.evs.make((int)ss.size() + 1, hipEventDisableTiming))) return rc;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  auto body = [&]() -> int {
    int r;
    for (auto &j : B.jobs)
      if ((r = j->enqueue_pre(st)) || (r = j->enqueue_zero(0, st))) return r;
    HIPCHK(launch_zero(B.d_cnt.p, std::max<size_t>(B.from.size(), 1) * 4 * sizeof(long long), st));
    HIPCHK(hipEventRecord(B.evs.e[0], st));
    for (auto s_ : ss) HIPCHK(hipStreamWaitEvent(s_, B.evs.e[0], 0));
    std::vector<int> order(24);
    for (int g = 0; g < 24; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return B.cls_cost[x] > B.cls_cost[y]; });
    std::vector<double> load(ss.size(), 0.0);  // least-loaded side stream first
    for (int g : order) {
      const int w0 = B.cls_off[g], w1 = B.cls_off[g + 1];
      if (w1 == w0) continue;
      const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += B.cls_cost[g];
      HIPCHK(launch_sr3c(g / 6, g % 6, B.d_prm.as<SRParams>(), B.d_work.as<SRWork>(), B.d_cnt.as<long long>(), w0,
                         w1 - w0, ss[k]));
    }
    for (size_t i = 0; i < ss.size(); ++i) {
      HIPCHK(hipEventRecord(B.evs.e[1 + i], ss[i]));
      HIPCHK(hipStreamWaitEvent(st, B.evs.e[1 + i], 0));
    }
    for (auto &j : B.jobs)
      if ((r = j->enqueue_reduce(0, st)) || (r = j->enqueue_fold(0, st)) || (r = j->enqueue_lr(st, nullptr))) return r;
    return RSGDF_OK;
  };
  rc = body();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(RSGDF_EHIP, std::string("HIP error: ") + hipGetErrorString(e) + " at capture");
  B.graph = g;
  HIPCHK(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
  return RSGDF_OK;
}

}  // namespace

extern "C" {

int rsgdf_batch_create(int32_t ncell, const rsgdf_cell *cells, const rsgdf_basis *bases, const rsgdf_basis *auxes,
                       const int32_t (*kmeshes)[3], double omega, double thresh, const rsgdf_options *opt,
                       rsgdf_out *outs, rsgdf_batch **batch) {
  g_err.clear();
  if (!batch) return fail(RSGDF_EINVAL, "null batch handle");
  *batch = nullptr;
  if (ncell < 1 || !cells || !bases || !auxes || !kmeshes || !outs) return fail(RSGDF_EINVAL, "invalid batch arguments");
  auto B = std::make_unique<rsgdf_batch>();
  B->st = reinterpret_cast<hipStream_t>(outs[0].stream);
  for (int i = 0; i < ncell; ++i) {
    if (!outs[i].on_device) return fail(RSGDF_EINVAL, "batched outputs must be device memory");
    if (outs[i].stream != outs[0].stream) return fail(RSGDF_EINVAL, "batched outputs must share one stream");
    auto j = std::make_unique<Job>();
    j->cell = &cells[i];
    j->basis = &bases[i];
    j->auxbasis = &auxes[i];
    j->kmesh = kmeshes[i];
    j->omega = omega;
    j->thresh = thresh;
    j->out = &outs[i];
    j->o.g_thresh = -1.0;
    j->o.parts = RSGDF_PART_ALL;
    if (opt) j->o = *opt;
    B->jobs.push_back(std::move(j));
  }
  // inputs are validated here, before any planning thread reads them
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RSGDF_EINVAL, "omega must be > 0");
  if (!(thresh > 0.0) || !std::isfinite(thresh)) return fail(RSGDF_EINVAL, "thresh must be > 0");
  for (int i = 0; i < ncell; ++i) {
    const int64_t nb = rsgdf_j3c_nbytes(&cells[i], &bases[i], &auxes[i], kmeshes[i]);
    if (nb < 0) return fail((int)nb, "cell " + std::to_string(i) + ": " + g_err);
    for (int q = 0; q < 3 * cells[i].natm; ++q)
      if (!std::isfinite(cells[i].coords[q])) return fail(RSGDF_EINVAL, "cell " + std::to_string(i) + ": non-finite coordinates");
  }
  // host planning of the cells is independent: up to 8 worker threads (each
  // plan may itself fan out); device allocations and uploads stay in order
  {
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    const int nt = std::min<int>(ncell, 8);
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&]() {
        for (int i; (i = next.fetch_add(1)) < ncell;) {
          Job &j = *B->jobs[i];
          j.hp.acut = opt ? opt->alpha_cut : 0.0;
          j.plan_rc = build_plan(j.cell, j.basis, j.auxbasis, j.kmesh, j.omega, j.thresh, j.hp);
          if (j.plan_rc) j.plan_err = g_err;  // this worker's message
          j.planned = true;
        }
      });
    for (auto &t : th) t.join();
  }
  for (int i = 0; i < ncell; ++i) {
    Job &j = *B->jobs[i];
    // all cells' short-range scratch is resident at once (one merged launch),
    // so a cell may take what is left; one needing more is built alone
    j.own_y = false;
    int rc = j.prepare(B->st, 0.9);
    if (rc) return fail(rc, "cell " + std::to_string(i) + ": " + g_err);
    if (j.do_sr && j.nbatch != 1)
      return fail(RSGDF_EUNSUPPORTED, "cell " + std::to_string(i) + " needs aux batching; build it alone");
  }
  {  // one fold intermediate for all cells: the folds run one after another on one stream
    double ymax = 0.0;
    for (auto &j : B->jobs)
      if (j->do_sr) ymax = std::max(ymax, (double)j->max_bf_el * j->nk * j->nk * 16.0);
    if (ymax > 0.0) {
      size_t fr = 0;
      HIPCHK(mem_avail(&fr));
      const double ybytes = std::min({ymax, 0.25 * 0.9 * (double)fr, 8e9});
      size_t need_b = 0;
      for (auto &j : B->jobs)
        if (j->do_sr) {
          j->set_fold_chunk(ybytes);
          need_b = std::max(need_b, (size_t)j->fchunk * j->nk * j->nk * 16);
        }
      HIPCHK(B->d_Y.alloc(need_b));
      for (auto &j : B->jobs) j->ybuf = B->d_Y.as<double>();
    }
  }
  // merged SR queue: per class, all cells' items, heaviest first
  std::vector<SRParams> prms;
  std::vector<SRWork> work;
  B->cls_off.assign(1, 0);
  B->cls_cost.assign(24, 0.0);
  for (size_t c = 0; c < B->jobs.size(); ++c) prms.push_back(B->jobs[c]->batch_params(0));
  for (int g = 0; g < 24; ++g) {
    for (size_t c = 0; c < B->jobs.size(); ++c) {
      Job &j = *B->jobs[c];
      if (!j.do_sr) continue;
      for (int w = j.wgrp_off[g]; w < j.wgrp_off[g + 1]; ++w) {
        SRWork x = j.work[w];
        x.cell = (int32_t)c;
        work.push_back(x);
        B->from.push_back({(int)c, (int64_t)w});
      }
      B->cls_cost[g] += j.wgrp_cost[g];
    }
    B->cls_off.push_back((int)work.size());
  }
  HIPCHK(upload(B->d_prm, prms, B->st));
  HIPCHK(upload(B->d_work, work, B->st));
  HIPCHK(B->d_cnt.alloc(std::max<size_t>(work.size(), 1) * 4 * sizeof(long long)));
  HIPCHK(hipStreamSynchronize(B->st));
  int rc = batch_capture(*B);
  if (rc) return rc;
  *batch = B.release();
  return RSGDF_OK;
}

int rsgdf_batch_run(rsgdf_batch *batch) {
  g_err.clear();
  if (!batch || !batch->exec) return fail(RSGDF_EINVAL, "invalid batch handle");
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipGraphLaunch(batch->exec, batch->st));
  HIPCHK(hipStreamSynchronize(batch->st));
  const double ms = ms_since(t0);
  std::vector<long long> cnt(std::max<size_t>(batch->from.size(), 1) * 4);
  HIPCHK(hipMemcpy(cnt.data(), batch->d_cnt.p, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost));
  std::vector<std::vector<long long>> per(batch->jobs.size());
  for (size_t c = 0; c < batch->jobs.size(); ++c) per[c].assign((size_t)batch->jobs[c]->nwork * 4 + 4, 0);
  for (size_t m = 0; m < batch->from.size(); ++m)
    for (int q = 0; q < 4; ++q) per[batch->from[m].first][(size_t)batch->from[m].second * 4 + q] = cnt[m * 4 + q];
  for (size_t c = 0; c < batch->jobs.size(); ++c) {
    Job &j = *batch->jobs[c];
    int rc = j.finish(batch->st, per[c].data());
    if (rc) return rc;
    if (j.out->stats) j.out->stats->t_total_ms = ms;  // the whole batch
  }
  return RSGDF_OK;
}

void rsgdf_batch_destroy(rsgdf_batch *batch) { delete batch; }

int rsgdf_build_j3c_batch(int32_t ncell, const rsgdf_cell *cells, const rsgdf_basis *bases, const rsgdf_basis *auxes,
                          const int32_t (*kmeshes)[3], double omega, double thresh, const rsgdf_options *opt,
                          rsgdf_out *outs) {
  rsgdf_batch *b = nullptr;
  int rc = rsgdf_batch_create(ncell, cells, bases, auxes, kmeshes, omega, thresh, opt, outs, &b);
  if (rc) return rc;
  rc = rsgdf_batch_run(b);
  rsgdf_batch_destroy(b);
  return rc;
}

int rsgdf_autotune_sr(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                      const int32_t kmesh[3], double omega, double thresh, float *split, double *class_ms,
                      void *stream) {
  g_err.clear();
  if (!split) return fail(RSGDF_EINVAL, "null split table");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  static const float cand[5] = {0.25f, 0.5f, 1.0f, 2.0f, 4.0f};
  double best[24];
  for (int g = 0; g < 24; ++g) {
    best[g] = 1e300;
    split[g] = 1.0f;
  }
  for (float f : cand) {
    double ms[24];
    int rc = tune_trial(cell, basis, auxbasis, kmesh, omega, thresh, f, st, ms);
    if (rc) return rc;
    for (int g = 0; g < 24; ++g)
      if (ms[g] < best[g]) {
        best[g] = ms[g];
        split[g] = f;
      }
  }
  if (class_ms)
    for (int g = 0; g < 24; ++g) class_ms[g] = best[g];
  return RSGDF_OK;
}

}  // extern "C"

extern "C" {

int rsgdf_build_j3c_ex(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                       const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                       rsgdf_out *out) {
  return build_impl(cell, basis, auxbasis, kmesh, omega, thresh, opt, out, nullptr);
}

}  // extern "C"

namespace {

// Device scratch of rsgdf_build_j3c_noalloc: one copy per GPU, held until the
// process ends.  In host code the name `scratch` is a host-side stand-in, not
// a device address; the address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that pointer is used.
constexpr size_t kNoallocScratchBytes = (size_t)RSGDF_NOALLOC_SCRATCH_MB << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchSlot {
  std::once_flag once;
  void *ptr = nullptr;
  hipError_t err = hipSuccess;
  std::mutex mu;  // serialises the calls of this process on the device
};
ScratchSlot g_scratch[kMaxDevices];

struct ArenaGuard {
  explicit ArenaGuard(Arena *a) { t_arena = a; }
  ~ArenaGuard() { t_arena = nullptr; }
};

}  // namespace

extern "C" {

int rsgdf_build_j3c_noalloc(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                            const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                            rsgdf_out *out) {
  const auto t_start = std::chrono::steady_clock::now();
  g_err.clear();
  if (!out) return fail(RSGDF_EINVAL, "null output");
  if (!out->on_device) return fail(RSGDF_EINVAL, "rsgdf_build_j3c_noalloc writes device memory only (on_device = 1)");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RSGDF_EUNSUPPORTED, "device index beyond the scratch table");
  ScratchSlot &slot = g_scratch[dev];
  std::call_once(slot.once, [&] { slot.err = hipGetSymbolAddress(&slot.ptr, HIP_SYMBOL(scratch)); });
  if (slot.err != hipSuccess || !slot.ptr)
    return fail(RSGDF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(slot.err));
  std::lock_guard<std::mutex> lock(slot.mu);
  Arena ar;
  ar.base = static_cast<char *>(slot.ptr);
  ar.cap = kNoallocScratchBytes;
  ArenaGuard guard(&ar);
  Job j;
  j.cell = cell;
  j.basis = basis;
  j.auxbasis = auxbasis;
  j.kmesh = kmesh;
  j.omega = omega;
  j.thresh = thresh;
  j.out = out;
  j.o.g_thresh = -1.0;
  j.o.lr_precision = RSGDF_FP64;
  j.o.screening = RSGDF_SCREEN_RIGOROUS;
  j.o.parts = RSGDF_PART_ALL;
  if (opt) j.o = *opt;
  hipStream_t st = reinterpret_cast<hipStream_t>(out->stream);
  int rc = j.prepare(st, 0.45);
  if (ar.overflow || rc == RSGDF_ENOMEM)
    return fail(RSGDF_ENOMEM, "rsgdf_build_j3c_noalloc: this build needs more device scratch than the " +
                                  std::to_string(RSGDF_NOALLOC_SCRATCH_MB) + " MiB static buffer (at least " +
                                  std::to_string(ar.want >> 20) + " MiB requested" +
                                  (g_err.empty() ? std::string(")") : "; " + g_err + ")"));
  if (rc) return rc;
  const std::vector<hipStream_t> none;  // no side streams, no events
  if ((rc = j.enqueue_pre(st))) return rc;
  for (int b = 0; b < j.nbatch; ++b) {
    if ((rc = j.enqueue_sr(b, st, none, nullptr, nullptr))) return rc;
    if ((rc = j.enqueue_fold(b, st))) return rc;
  }
  if ((rc = j.enqueue_lr(st, nullptr))) return rc;
  if ((rc = j.finish(st, nullptr))) return rc;
  if (out->stats) out->stats->t_total_ms = ms_since(t_start);
  return RSGDF_OK;
}

int rsgdf_screen_log(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                     const int32_t kmesh[3], double omega, double thresh, double sample_frac, uint64_t seed,
                     float *feat, float *target, int64_t capacity, int64_t *n_out, void *stream) {
  g_err.clear();
  if (!n_out) return fail(RSGDF_EINVAL, "null n_out");
  if (!(sample_frac > 0.0) || sample_frac > 1.0) return fail(RSGDF_EINVAL, "sample_frac must be in (0, 1]");
  if (capacity < 0 || (capacity > 0 && (!feat || !target))) return fail(RSGDF_EINVAL, "null feature/target buffer");
  LearnCtl ctl;
  ctl.log = true;
  ctl.sample_frac = sample_frac;
  ctl.seed = seed;
  rsgdf_out out{};
  out.stream = stream;
  out.on_device = 1;
  rsgdf_options o{};
  o.g_thresh = -1.0;
  o.parts = RSGDF_PART_SR;
  const int rc = build_impl(cell, basis, auxbasis, kmesh, omega, thresh, &o, &out, &ctl);
  if (rc) return rc;
  const int64_t n = (int64_t)ctl.tgt.size();
  *n_out = n;
  if (n > capacity) return fail(RSGDF_ESIZE, "capacity below the number of logged candidates");
  std::memcpy(feat, ctl.feat.data(), (size_t)n * kMlpF * sizeof(float));
  std::memcpy(target, ctl.tgt.data(), (size_t)n * sizeof(float));
  return RSGDF_OK;
}

// full-data loss (and gradient) of the network on device-resident samples
static int mlp_eval(float *d_params, const float *d_X, const float *d_y, const int64_t *d_iota, int64_t n,
                    float kappa, DBuf &gpart, DBuf &lpart, float *grad_host, float *loss_host, hipStream_t st) {
  DBuf d_grad;
  if (grad_host) HIPCHK(d_grad.alloc(kMlpNTrain * sizeof(float)));
  HIPCHK(launch_mlp_step(d_params, d_X, d_y, d_iota, n, kappa, gpart.as<float>(), lpart.as<float>(),
                         grad_host ? d_grad.as<float>() : nullptr, nullptr, nullptr, 0.f, 0, st));
  const int nblk = (int)((n + 63) / 64);
  std::vector<float> lp(nblk);
  HIPCHK(hipMemcpyAsync(lp.data(), lpart.p, nblk * sizeof(float), hipMemcpyDeviceToHost, st));
  if (grad_host) HIPCHK(hipMemcpyAsync(grad_host, d_grad.p, kMlpNTrain * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double l = 0.0;
  for (float v : lp) l += v;
  if (loss_host) *loss_host = (float)l;
  return RSGDF_OK;
}

int rsgdf_mlp_train(float *params, const float *X, const float *y, int64_t n, int32_t epochs, int32_t batch,
                    float lr, float kappa, uint64_t seed, int32_t init, float *loss_history, void *stream) {
  g_err.clear();
  if (!params || !X || !y || n < 1 || epochs < 0 || batch < 1 || !(lr > 0.f) || !(kappa >= 1.f))
    return fail(RSGDF_EINVAL, "invalid training arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (init) {
    // standardisation and training range from the data, He-initialised weights
    for (int k = 0; k < kMlpF; ++k) {
      double s = 0.0, s2 = 0.0, lo = 1e300, hi = -1e300;
      for (int64_t i = 0; i < n; ++i) {
        const double v = X[i * kMlpF + k];
        s += v;
        s2 += v * v;
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      const double mean = s / n, var = std::max(s2 / n - mean * mean, 0.0);
      params[kMlpOffMean + k] = (float)mean;
      params[kMlpOffIstd + k] = var > 1e-20 ? (float)(1.0 / std::sqrt(var)) : 0.f;
      const double pad = 0.02 * (hi - lo) + 1e-6;
      params[kMlpOffLo + k] = (float)(lo - pad);
      params[kMlpOffHi + k] = (float)(hi + pad);
    }
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < kMlpH * kMlpF; ++i) params[kMlpOffW1 + i] = (float)(nd(rng) * std::sqrt(2.0 / kMlpF));
    for (int i = 0; i < kMlpH * kMlpH; ++i) params[kMlpOffW2 + i] = (float)(nd(rng) * std::sqrt(2.0 / kMlpH));
    for (int i = 0; i < kMlpH; ++i) {
      params[kMlpOffB1 + i] = 0.f;
      params[kMlpOffB2 + i] = 0.f;
      params[kMlpOffW3 + i] = (float)(nd(rng) * std::sqrt(1.0 / kMlpH));
    }
    double ym = 0.0;
    for (int64_t i = 0; i < n; ++i) ym += y[i];
    params[kMlpOffB3] = (float)(ym / n);
  }
  DBuf d_p, d_X, d_y, d_idx, d_iota, d_m, d_v, d_gpart, d_lpart;
  HIPCHK(d_p.alloc(kMlpNParam * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_p.p, params, kMlpNParam * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_X.alloc((size_t)n * kMlpF * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_X.p, X, (size_t)n * kMlpF * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_y.alloc((size_t)n * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_y.p, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  HIPCHK(upload(d_iota, perm, st));
  HIPCHK(d_idx.alloc((size_t)n * sizeof(int64_t)));
  HIPCHK(d_m.alloc(kMlpNTrain * sizeof(float)));
  HIPCHK(d_v.alloc(kMlpNTrain * sizeof(float)));
  HIPCHK(hipMemsetAsync(d_m.p, 0, kMlpNTrain * sizeof(float), st));
  HIPCHK(hipMemsetAsync(d_v.p, 0, kMlpNTrain * sizeof(float), st));
  const int64_t nblk_max = (n + 63) / 64;
  HIPCHK(d_gpart.alloc((size_t)nblk_max * kMlpNTrain * sizeof(float)));
  HIPCHK(d_lpart.alloc((size_t)nblk_max * sizeof(float)));
  std::mt19937_64 rng(seed ^ 0x5bd1e995ull);
  int step = 0;
  for (int e = 0; e < epochs; ++e) {
    std::shuffle(perm.begin(), perm.end(), rng);
    HIPCHK(hipMemcpyAsync(d_idx.p, perm.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, st));
    for (int64_t s0 = 0; s0 < n; s0 += batch) {
      const int64_t nb = std::min<int64_t>(batch, n - s0);
      HIPCHK(launch_mlp_step(d_p.as<float>(), d_X.as<float>(), d_y.as<float>(), d_idx.as<int64_t>() + s0, nb, kappa,
                             d_gpart.as<float>(), d_lpart.as<float>(), nullptr, d_m.as<float>(), d_v.as<float>(), lr,
                             ++step, st));
    }
    if (loss_history) {
      const int rc = mlp_eval(d_p.as<float>(), d_X.as<float>(), d_y.as<float>(), d_iota.as<int64_t>(), n, kappa,
                              d_gpart, d_lpart, nullptr, &loss_history[e], st);
      if (rc) return rc;
    } else {
      HIPCHK(hipStreamSynchronize(st));  // perm is rewritten next epoch
    }
  }
  HIPCHK(hipMemcpyAsync(params, d_p.p, kMlpNParam * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return RSGDF_OK;
}

int rsgdf_mlp_grad(const float *params, const float *X, const float *y, int64_t n, float kappa, float *grad,
                   float *loss, void *stream) {
  g_err.clear();
  if (!params || !X || !y || n < 1 || !grad || !loss) return fail(RSGDF_EINVAL, "invalid gradient arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DBuf d_p, d_X, d_y, d_iota, d_gpart, d_lpart;
  HIPCHK(d_p.alloc(kMlpNParam * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_p.p, params, kMlpNParam * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_X.alloc((size_t)n * kMlpF * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_X.p, X, (size_t)n * kMlpF * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_y.alloc((size_t)n * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_y.p, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<int64_t> iota(n);
  for (int64_t i = 0; i < n; ++i) iota[i] = i;
  HIPCHK(upload(d_iota, iota, st));
  const int64_t nblk = (n + 63) / 64;
  HIPCHK(d_gpart.alloc((size_t)nblk * kMlpNTrain * sizeof(float)));
  HIPCHK(d_lpart.alloc((size_t)nblk * sizeof(float)));
  return mlp_eval(d_p.as<float>(), d_X.as<float>(), d_y.as<float>(), d_iota.as<int64_t>(), n, kappa, d_gpart, d_lpart,
                  grad, loss, st);
}

int rsgdf_mlp_predict(const float *params, const float *X, int64_t n, int32_t mode, float *pred, void *stream) {
  g_err.clear();
  if (!params || !X || !pred || n < 1 || (mode != 0 && mode != 1)) return fail(RSGDF_EINVAL, "invalid predict arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DBuf d_p, d_X, d_pred;
  HIPCHK(d_p.alloc(kMlpNParam * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_p.p, params, kMlpNParam * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_X.alloc((size_t)n * kMlpF * sizeof(float)));
  HIPCHK(hipMemcpyAsync(d_X.p, X, (size_t)n * kMlpF * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(d_pred.alloc((size_t)n * sizeof(float)));
  HIPCHK(launch_mlp_predict(d_p.as<float>(), d_X.as<float>(), n, mode, d_pred.as<float>(), st));
  HIPCHK(hipMemcpyAsync(pred, d_pred.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return RSGDF_OK;
}

int rsgdf_mlp_margin(const float *params, const float *X, const float *y, int64_t n, double quantile,
                     double *margin, void *stream) {
  g_err.clear();
  if (!margin || !(quantile > 0.0) || quantile > 1.0) return fail(RSGDF_EINVAL, "invalid margin arguments");
  std::vector<float> pred(std::max<int64_t>(n, 1));
  const int rc = rsgdf_mlp_predict(params, X, n, 1, pred.data(), stream);
  if (rc) return rc;
  std::vector<double> r(n);
  for (int64_t i = 0; i < n; ++i) r[i] = (double)y[i] - (double)pred[i];
  std::sort(r.begin(), r.end());
  const int64_t k = std::min<int64_t>(n - 1, (int64_t)std::ceil(quantile * n) - 1);
  *margin = std::max(0.0, r[std::max<int64_t>(k, 0)]);
  return RSGDF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Two-center metric J^k (Eq. M5) and the density-fitting solve (Eq. M4)
// ---------------------------------------------------------------------------
namespace {

int64_t j2c_nbytes_impl(const rsgdf_cell *cell, const rsgdf_basis *auxbasis, const int32_t kmesh[3]) {
  if (!cell || !kmesh) return fail(RSGDF_EINVAL, "null argument");
  if (cell->natm < 1 || !cell->coords) return fail(RSGDF_EINVAL, "cell needs at least one atom");
  int rc = validate_basis(auxbasis, cell->natm, RSGDF_MAX_L_AUX, "auxbasis");
  if (rc) return rc;
  for (int d = 0; d < 3; ++d)
    if (kmesh[d] < 1 || kmesh[d] > 64) return fail(RSGDF_EINVAL, "kmesh entries must be in 1..64");
  const int64_t nk = (int64_t)kmesh[0] * kmesh[1] * kmesh[2];
  const int64_t n = nfunc(auxbasis);
  return nk * n * n * 16;
}

}  // namespace

extern "C" {

int64_t rsgdf_j2c_nbytes(const rsgdf_cell *cell, const rsgdf_basis *auxbasis, const int32_t kmesh[3]) {
  g_err.clear();
  return j2c_nbytes_impl(cell, auxbasis, kmesh);
}

int rsgdf_build_j2c(const rsgdf_cell *cell, const rsgdf_basis *auxbasis, const int32_t kmesh[3], double omega,
                    double thresh, const rsgdf_options *opt, rsgdf_out *out) {
  const auto t_start = std::chrono::steady_clock::now();
  g_err.clear();
  if (!out) return fail(RSGDF_EINVAL, "null output");
  const int64_t need = j2c_nbytes_impl(cell, auxbasis, kmesh);
  if (need < 0) return (int)need;
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RSGDF_EINVAL, "omega must be > 0");
  if (!(thresh > 0.0) || !std::isfinite(thresh)) return fail(RSGDF_EINVAL, "thresh must be > 0");
  for (int i = 0; i < 3 * cell->natm; ++i)
    if (!std::isfinite(cell->coords[i])) return fail(RSGDF_EINVAL, "non-finite coordinates");
  if (!out->data) return fail(RSGDF_EINVAL, "null output buffer");
  if (out->capacity_bytes < need) return fail(RSGDF_ESIZE, "output capacity too small");
  int parts = (opt && opt->parts) ? opt->parts : RSGDF_PART_ALL;
  const double g_thr = (opt && opt->g_thresh > 0.0) ? opt->g_thresh : 1e-2 * thresh;
  Lat lt;
  int rc = make_lattice(cell, kmesh, lt);
  if (rc) return rc;
  const Lattice &L = lt.L;
  const int nk = L.nk;
  std::vector<Shell> ax;
  std::vector<double> ax_exp, ax_coef, ax_c1s;
  const int64_t naux = pack_shells(auxbasis, cell->coords, ax, ax_exp, ax_coef, ax_c1s);
  const int nxs = (int)ax.size();
  // (P, Q) shell pairs grouped by (l_P, l_Q), each with the radius beyond which
  // every term (P^0 | erfc | Q^m) of the 1s model (Eqs. S4-S9 with one AO
  // factor replaced by the aux function), with its angular growth, stays
  // below 1e-2 thresh (solve_rc, Eq. S14)
  std::vector<J2Pair> pairs;
  int cls_off[17] = {0};
  for (int lp = 0; lp <= 3; ++lp)
    for (int lq = 0; lq <= 3; ++lq) {
      for (int P = 0; P < nxs; ++P) {
        if (ax[P].l != lp) continue;
        for (int Q = 0; Q < nxs; ++Q) {
          if (ax[Q].l != lq) continue;
          double K = 0.0;
          for (int i = 0; i < ax[P].nprim; ++i)
            for (int j = 0; j < ax[Q].nprim; ++j) {
              const double a = ax_exp[ax[P].pptr + i], b = ax_exp[ax[Q].pptr + j];
              K += kPi * kPi * kPi * ax_c1s[ax[P].pptr + i] * ax_c1s[ax[Q].pptr + j] / std::pow(a * b, 1.5);
            }
          const double a = ax[P].a_d, b = ax[Q].a_d;
          const double e1 = std::sqrt(a * b / (a + b));
          const double e2 = 1.0 / std::sqrt(1.0 / (e1 * e1) + 1.0 / (omega * omega));
          J2Pair jp{};
          jp.P = P;
          jp.Q = Q;
          jp.rmax = solve_rc(K, e2, 1e-2 * thresh, lp + lq) + 1e-9;
          pairs.push_back(jp);
        }
      }
      cls_off[4 * lp + lq + 1] = (int)pairs.size();
    }
  // S_P = int chi_P (all space) for the G = 0 term
  std::vector<double> SP(naux, 0.0);
  for (int s_ = 0; s_ < nxs; ++s_) {
    const Shell &x = ax[s_];
    int ic = 0;
    for (int lx = x.l; lx >= 0; --lx)
      for (int ly = x.l - lx; ly >= 0; --ly, ++ic) {
        const int lz = x.l - lx - ly;
        if ((lx | ly | lz) & 1) continue;
        double v = 0.0;
        for (int k = 0; k < x.nprim; ++k) {
          const double g = ax_exp[x.pptr + k];
          double m = ax_coef[x.pptr + k] * std::pow(kPi / g, 1.5);
          const int pw[3] = {lx, ly, lz};
          for (int d = 0; d < 3; ++d) {
            double df = 1.0;
            for (int q = pw[d] - 1; q > 1; q -= 2) df *= q;
            m *= df / std::pow(2.0 * g, pw[d] / 2);
          }
          v += m;
        }
        SP[x.foff + ic] = v;
      }
  }
  const std::vector<double> kvec = mesh_kvec(L);
  const std::vector<double> kph = mesh_phases(L);
  std::vector<double> qv;
  std::vector<int64_t> qoff;
  if (parts & RSGDF_PART_LR) make_qsets(lt, kvec, omega, g_thr, qv, qoff);
  const int64_t nq_tot = qoff.empty() ? 0 : qoff.back();
  const double t_plan = ms_since(t_start);

  hipStream_t st = reinterpret_cast<hipStream_t>(out->stream);
  DBuf d_ax, d_axe, d_axc, d_pairs, d_boys, d_kph, d_SP, d_X2, d_nterm, d_q, d_A, d_B, d_kidx, d_J;
  HIPCHK(upload(d_ax, ax, st));
  HIPCHK(upload(d_axe, ax_exp, st));
  HIPCHK(upload(d_axc, ax_coef, st));
  HIPCHK(upload(d_pairs, pairs, st));
  const std::vector<double> boys = boys_poly_table();
  HIPCHK(upload(d_boys, boys, st));
  HIPCHK(upload(d_kph, kph, st));
  HIPCHK(upload(d_SP, SP, st));
  std::vector<int32_t> kidx(nk);
  for (int k = 0; k < nk; ++k) kidx[k] = k;
  HIPCHK(upload(d_kidx, kidx, st));
  HIPCHK(d_X2.alloc((size_t)nk * naux * naux * sizeof(double)));
  HIPCHK(d_nterm.alloc(sizeof(long long)));
  double *J = nullptr;
  if (out->on_device) {
    J = static_cast<double *>(out->data);
  } else {
    HIPCHK(d_J.alloc((size_t)need));
    J = d_J.as<double>();
  }
  EventSet ev;
  if ((rc = ev.make(4, 0))) return rc;
  HIPCHK(hipEventRecord(ev.e[0], st));
  HIPCHK(launch_zero(d_nterm.p, sizeof(long long), st));
  J2Params jp{};
  jp.ax = d_ax.as<Shell>();
  jp.ax_exp = d_axe.as<double>();
  jp.ax_coef = d_axc.as<double>();
  jp.pairs = d_pairs.as<J2Pair>();
  jp.lat = L;
  jp.omega = omega;
  jp.boys = d_boys.as<double>();
  jp.X2 = d_X2.as<double>();
  jp.nterm = d_nterm.as<long long>();
  jp.naux = (int32_t)naux;
  if (parts & RSGDF_PART_SR) {
    for (int g = 0; g < 16; ++g)
      HIPCHK(launch_j2c_sr(g / 4, g % 4, jp, cls_off[g], cls_off[g + 1] - cls_off[g], st));
  } else {
    HIPCHK(launch_zero(d_X2.p, (size_t)nk * naux * naux * sizeof(double), st));
  }
  const double g0fac = (parts & RSGDF_PART_G0) ? kPi / (L.vol * omega * omega) : 0.0;
  HIPCHK(launch_j2c_fold(d_X2.as<double>(), d_kph.as<double>(), d_SP.as<double>(), g0fac, nk, (int)naux, J, st));
  HIPCHK(hipEventRecord(ev.e[1], st));
  double lr_flops = 0.0;
  if ((parts & RSGDF_PART_LR) && nq_tot > 0) {
    HIPCHK(upload(d_q, qv, st));
    HIPCHK(d_A.alloc((size_t)naux * nq_tot * 2 * sizeof(double)));
    int64_t max_nq = 0;
    for (int c = 0; c < nk; ++c) max_nq = std::max(max_nq, qoff[c + 1] - qoff[c]);
    HIPCHK(d_B.alloc((size_t)naux * std::max<int64_t>(max_nq, 1) * 2 * sizeof(double)));
    AuxFTParams ap{d_ax.as<Shell>(), d_axe.as<double>(), d_axc.as<double>(), d_q.as<double>(), (int32_t)nq_tot,
                   (int32_t)nxs, (int32_t)naux, 0, 4.0 * kPi / L.vol, omega, d_A.as<double>()};
    HIPCHK(launch_auxft(ap, st));
    for (int c = 0; c < nk; ++c) {
      const int64_t nqc = qoff[c + 1] - qoff[c];
      if (nqc == 0) continue;
      HIPCHK(launch_j2c_lr_operand(d_A.as<double>() + 2 * qoff[c], nq_tot, d_q.as<double>() + 3 * qoff[c], (int)nqc,
                                   (int)naux, 4.0 * kPi / L.vol, omega, d_B.as<double>(), st));
      LRGemmParams gp{};
      gp.A = d_A.as<double>() + 2 * qoff[c];
      gp.lda = nq_tot;
      gp.B = d_B.as<double>();
      gp.out = J;
      gp.kp_of = d_kidx.as<int32_t>() + c;
      gp.plane = naux * naux;
      gp.naux = (int32_t)naux;
      gp.nq = (int32_t)nqc;
      gp.nmn = (int32_t)naux;
      gp.nq_hi = 0;
      HIPCHK(launch_lr_gemm_tiled(RSGDF_FP64, gp, 0, 1, st));
      lr_flops += 8.0 * (double)naux * naux * nqc;
    }
  }
  HIPCHK(hipEventRecord(ev.e[2], st));
  long long nterm = 0;
  HIPCHK(hipMemcpyAsync(&nterm, d_nterm.p, sizeof(long long), hipMemcpyDeviceToHost, st));
  if (!out->on_device) HIPCHK(hipMemcpyAsync(out->data, J, (size_t)need, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out->nkpair = nk;
  out->naux = naux;
  out->nao = naux;
  if (out->stats) {
    rsgdf_stats &s_ = *out->stats;
    std::memset(&s_, 0, sizeof(s_));
    float ms = 0.f;
    s_.t_plan_ms = t_plan;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    s_.t_sr_ms = ms;
    HIPCHK(hipEventElapsedTime(&ms, ev.e[1], ev.e[2]));
    s_.t_lr_ms = ms;
    s_.n_sr_terms = nterm;
    s_.n_g_total = nq_tot;
    s_.n_triplets = (int64_t)pairs.size();
    s_.bytes_out = need;
    s_.lr_gemm_flops = lr_flops;
    s_.t_total_ms = ms_since(t_start);
  }
  return RSGDF_OK;
}

int rsgdf_df_solve(const int32_t kmesh[3], int64_t naux, int64_t ncol, const void *j2c, const void *j3c, void *d,
                   void *stream) {
  g_err.clear();
  if (!kmesh || !j2c || !j3c || !d) return fail(RSGDF_EINVAL, "null argument");
  for (int k = 0; k < 3; ++k)
    if (kmesh[k] < 1 || kmesh[k] > 64) return fail(RSGDF_EINVAL, "kmesh entries must be in 1..64");
  if (naux < 1 || naux > 65535 || ncol < 1) return fail(RSGDF_EINVAL, "naux must be in 1..65535 and ncol >= 1");
  const int n[3] = {kmesh[0], kmesh[1], kmesh[2]};
  const int nk = n[0] * n[1] * n[2];
  const int nkp = nk * (nk + 1) / 2;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // class of each k-pair: the mesh index of k2 - k1
  std::vector<int32_t> cls;
  for (int k1 = 0; k1 < nk; ++k1)
    for (int k2 = k1; k2 < nk; ++k2) {
      const int j1[3] = {k1 / (n[1] * n[2]), (k1 / n[2]) % n[1], k1 % n[2]};
      const int j2[3] = {k2 / (n[1] * n[2]), (k2 / n[2]) % n[1], k2 % n[2]};
      int c = 0;
      for (int q = 0; q < 3; ++q) c = c * n[q] + ((j2[q] - j1[q]) % n[q] + n[q]) % n[q];
      cls.push_back(c);
    }
  DBuf d_L, d_W, d_bad, d_cls, d_tmp;
  const size_t mat = (size_t)naux * naux * 16;
  HIPCHK(d_L.alloc(mat * nk));
  HIPCHK(d_W.alloc(mat * nk));
  HIPCHK(d_bad.alloc((size_t)nk * sizeof(int)));
  HIPCHK(upload(d_cls, cls, st));
  HIPCHK(launch_df_factor(static_cast<const double *>(j2c), d_L.as<double>(), d_W.as<double>(), d_bad.as<int>(), nk,
                          (int)naux, st));
  std::vector<int> bad(nk, 0);
  HIPCHK(hipMemcpyAsync(bad.data(), d_bad.p, (size_t)nk * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < nk; ++k)
    if (bad[k])
      return fail(RSGDF_EINVAL, "J^k is numerically singular at k index " + std::to_string(k) +
                                    " (a Cholesky pivot below 1e-12 of its diagonal entry: linearly dependent aux functions)");
  // per chunk of k-pairs: Y = W V into the temporary, then d = W^H Y (in place
  // allowed: V of the chunk is consumed by the first product before the second
  // writes it)
  const size_t per = (size_t)naux * ncol * 16;  // bytes of one k-pair's block
  size_t free_b = 0;
  HIPCHK(mem_avail(&free_b));
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nkp, (size_t)(0.25 * free_b) / per));
  HIPCHK(d_tmp.alloc(per * chunk));
  const double *V = static_cast<const double *>(j3c);
  double *D = static_cast<double *>(d);
  for (int t0 = 0; t0 < nkp; t0 += chunk) {
    const int nt = std::min(chunk, nkp - t0);
    const size_t off = 2 * (size_t)t0 * naux * ncol;
    HIPCHK(launch_df_gemm(false, d_W.as<double>(), d_cls.as<int32_t>() + t0, V + off, d_tmp.as<double>(), (int)naux,
                          ncol, nt, st));
    HIPCHK(launch_df_gemm(true, d_W.as<double>(), d_cls.as<int32_t>() + t0, d_tmp.as<double>(), D + off, (int)naux,
                          ncol, nt, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return RSGDF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Integral-direct density-fitted Coulomb matrix (a consumer of the
// three-center integrals that never stores them)
// ---------------------------------------------------------------------------
extern "C" {

int rsgdf_coulomb_direct(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                         const int32_t kmesh[3], double omega, double thresh, const rsgdf_options *opt,
                         int32_t aux_group, const void *dm, void *vj, void *stream, rsgdf_stats *stats) {
  const auto t_start = std::chrono::steady_clock::now();
  g_err.clear();
  if (!dm || !vj) return fail(RSGDF_EINVAL, "null density or output");
  if (aux_group < 0) return fail(RSGDF_EINVAL, "aux_group must be >= 0");
  const int64_t need = rsgdf_j3c_nbytes(cell, basis, auxbasis, kmesh);
  if (need < 0) return (int)need;
  if (opt && opt->parts && opt->parts != RSGDF_PART_ALL) return fail(RSGDF_EINVAL, "the Coulomb build needs all parts");
  const int nk = kmesh[0] * kmesh[1] * kmesh[2];
  const int64_t nao = nfunc(basis), naux = nfunc(auxbasis), ne = nao * nao;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  rsgdf_stats acc{};
  // J^{k12 = 0} and its factor
  DBuf d_J0, d_L, d_W, d_bad, d_cls, d_rho, d_y, d_c, d_V;
  HIPCHK(d_J0.alloc((size_t)naux * naux * 16));
  {
    rsgdf_out o{};
    o.data = d_J0.p;
    o.capacity_bytes = (int64_t)naux * naux * 16;
    o.on_device = 1;
    o.stream = stream;
    rsgdf_stats s2{};
    o.stats = &s2;
    const int32_t gam[3] = {1, 1, 1};
    int rc = rsgdf_build_j2c(cell, auxbasis, gam, omega, thresh, opt, &o);
    if (rc) return rc;
  }
  HIPCHK(d_L.alloc((size_t)naux * naux * 16));
  HIPCHK(d_W.alloc((size_t)naux * naux * 16));
  HIPCHK(d_bad.alloc(sizeof(int)));
  HIPCHK(launch_df_factor(d_J0.as<double>(), d_L.as<double>(), d_W.as<double>(), d_bad.as<int>(), 1, (int)naux, st));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return fail(RSGDF_EINVAL, "J^0 is numerically singular (linearly dependent aux functions)");
  const std::vector<int32_t> zero1(1, 0);
  HIPCHK(upload(d_cls, zero1, st));
  HIPCHK(d_rho.alloc((size_t)naux * 16));
  HIPCHK(d_y.alloc((size_t)naux * 16));
  HIPCHK(d_c.alloc((size_t)naux * 16));
  // aux shell groups: the V tile of a group [nk][naux_g][nao^2] within a budget
  std::vector<int> gstart(1, 0);
  {
    size_t free_b = 0;
    HIPCHK(mem_avail(&free_b));
    const double budget = std::min(0.1 * (double)free_b, 8e9);
    int64_t nf = 0;
    int ns = 0;
    for (int s_ = 0; s_ < auxbasis->nshell; ++s_) {
      const int64_t add = ncart_h(auxbasis->shell_l[s_]);
      const bool full = aux_group > 0 ? ns >= aux_group : (nf > 0 && (double)(nf + add) * nk * ne * 16 > budget);
      if (full) {
        gstart.push_back(s_);
        nf = 0;
        ns = 0;
      }
      nf += add;
      ++ns;
    }
    gstart.push_back(auxbasis->nshell);
  }
  int64_t max_nf = 0;
  for (size_t g = 0; g + 1 < gstart.size(); ++g) {
    int64_t nf = 0;
    for (int s_ = gstart[g]; s_ < gstart[g + 1]; ++s_) nf += ncart_h(auxbasis->shell_l[s_]);
    max_nf = std::max(max_nf, nf);
  }
  HIPCHK(d_V.alloc((size_t)nk * max_nf * ne * 16));
  HIPCHK(launch_zero(vj, (size_t)nk * ne * 16, st));
  // one pass: rebuild the diagonal-k-pair tiles of every group; pass 0 forms
  // rho, pass 1 accumulates J
  for (int pass = 0; pass < 2; ++pass) {
    int64_t f0 = 0;
    for (size_t g = 0; g + 1 < gstart.size(); ++g) {
      const int s0 = gstart[g], s1 = gstart[g + 1];
      rsgdf_basis sub = *auxbasis;
      sub.nshell = s1 - s0;
      sub.shell_atom = auxbasis->shell_atom + s0;
      sub.shell_l = auxbasis->shell_l + s0;
      sub.shell_nprim = auxbasis->shell_nprim + s0;
      sub.shell_ptr = auxbasis->shell_ptr + s0;
      int64_t nf = 0;
      for (int s_ = s0; s_ < s1; ++s_) nf += ncart_h(auxbasis->shell_l[s_]);
      rsgdf_out o{};
      o.data = d_V.p;
      o.capacity_bytes = (int64_t)nk * nf * ne * 16;
      o.on_device = 1;
      o.stream = stream;
      rsgdf_stats s2{};
      o.stats = &s2;
      int rc = build_impl(cell, basis, &sub, kmesh, omega, thresh, opt, &o, nullptr, true);
      if (rc) return rc;
      acc.t_plan_ms += s2.t_plan_ms;
      acc.t_sr_ms += s2.t_sr_ms;
      acc.t_fold_ms += s2.t_fold_ms;
      acc.t_lr_ms += s2.t_lr_ms;
      acc.t_lr_gemm_ms += s2.t_lr_gemm_ms;
      acc.n_sr_terms += s2.n_sr_terms;
      acc.n_lr_terms += s2.n_lr_terms;
      acc.n_aux_batches += 1;
      if (pass == 0) {
        HIPCHK(launch_dm_contract(d_V.as<double>(), static_cast<const double *>(dm), nk, (int)nf, (int)nao,
                                  d_rho.as<double>() + 2 * f0, st));
      } else {
        HIPCHK(launch_vj_accum(d_V.as<double>(), d_c.as<double>() + 2 * f0, nk, (int)nf, ne, 1.0 / nk,
                               static_cast<double *>(vj), st));
      }
      f0 += nf;
    }
    if (pass == 0) {  // c = (J^0)^{-1} rho = W^H (W rho)
      HIPCHK(launch_df_gemm(false, d_W.as<double>(), d_cls.as<int32_t>(), d_rho.as<double>(), d_y.as<double>(),
                            (int)naux, 1, 1, st));
      HIPCHK(launch_df_gemm(true, d_W.as<double>(), d_cls.as<int32_t>(), d_y.as<double>(), d_c.as<double>(),
                            (int)naux, 1, 1, st));
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  if (stats) {
    *stats = acc;
    stats->bytes_out = (int64_t)nk * ne * 16;
    stats->t_total_ms = ms_since(t_start);
  }
  return RSGDF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Work features of a build for the cost model of the automatic choice of
// omega (host planning only, no device work)
// ---------------------------------------------------------------------------
extern "C" {

int rsgdf_plan_features_acut(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                             const int32_t kmesh[3], double omega, double alpha_cut, double thresh, double g_thresh,
                             double feat[RSGDF_NFEATURES]) {
  g_err.clear();
  if (!feat) return fail(RSGDF_EINVAL, "null feature array");
  const int64_t need = rsgdf_j3c_nbytes(cell, basis, auxbasis, kmesh);
  if (need < 0) return (int)need;
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RSGDF_EINVAL, "omega must be > 0");
  if (!(thresh > 0.0) || !std::isfinite(thresh)) return fail(RSGDF_EINVAL, "thresh must be > 0");
  if (!(alpha_cut >= 0.0) || !std::isfinite(alpha_cut)) return fail(RSGDF_EINVAL, "alpha_cut must be >= 0");
  const double g_thr = g_thresh > 0.0 ? g_thresh : 1e-2 * thresh;
  const double acut = alpha_cut;
  HostPlan hp;
  hp.acut = acut;
  int rc = build_plan(cell, basis, auxbasis, kmesh, omega, thresh, hp);
  if (rc) return rc;
  const Lattice &L = hp.lt.L;
  const int nk = L.nk, npair = (int)hp.pairs.size(), nxs = (int)hp.ax.size();
  // primitives below the cut (the diffuse ones of the split, R28)
  auto ndiff = [&](const Shell &s_, const std::vector<double> &ex) {
    int n = 0;
    if (acut > 0.0)
      for (int k = 0; k < s_.nprim; ++k) n += ex[s_.pptr + k] < acut;
    return n;
  };
  // short range: the planner's per-item cost (primitive triples x pair images
  // x lattice vectors in the R_c ball x per-term operations, plus the
  // per-(triple, image) contraction), summed over every (aux shell, pair);
  // with the split only compact aux primitives and pairs of primitives not
  // both diffuse
  double sr = 0.0, sr_terms = 0.0;
  for (int P = 0; P < nxs; ++P)
    for (int ip = 0; ip < npair; ++ip) {
      const size_t t = (size_t)P * npair + ip;
      const Pair &pp = hp.pairs[ip];
      const Shell &sA = hp.ao[pp.sa], &sB = hp.ao[pp.sb], &sP = hp.ax[P];
      if (acut > 0.0 && sP.a_d <= 0.0) continue;  // no compact primitive
      int64_t nimg = 0;
      for (int c = 0; c < nk; ++c) nimg += hp.nsr[(size_t)ip * nk + c];
      const double rc_cut = hp.rc_t[t];
      const double nm = 4.18879020478639098 * rc_cut * rc_cut * rc_cut / L.vol + 1.0;
      const int Lt = sP.l + sA.l + sB.l;
      const int lab = sA.l + sB.l, nkx = (sP.l / 2 + 1) * (sP.l / 2 + 1) * (sP.l / 2 + 1);
      const int nblk = ncart_h(sP.l) * ncart_h(sA.l) * ncart_h(sB.l);
      const double ev = 2.0 * nherm(Lt) + 2.0 * ncart_h(sP.l) * nherm(lab) * nkx + 2.0 * nblk * nherm(lab);
      const double nranges = std::ceil((double)nk / std::min(nk, sr_cells_per_wave(nblk)));
      const double npp = (double)sA.nprim * sB.nprim - (double)ndiff(sA, hp.ao_exp) * ndiff(sB, hp.ao_exp);
      const double np3 = npp * (sP.nprim - ndiff(sP, hp.ax_exp)) * (double)nimg;
      sr += np3 * (nm * sr_term_flops(Lt) + 13.6 * nranges * ev);
      sr_terms += np3 * nm;
    }
  // long range: q vectors, pair-transform candidates, contraction flops, per
  // part (one part without the split; with it the range-separated part and
  // the two Eq. M15 parts on their q spheres, R28)
  std::vector<int> kp_of_cls(nk, 0);
  for (size_t t = 0; t < hp.kp1.size(); ++t) {
    const int k1 = hp.kp1[t], k2 = hp.kp2[t];
    const int j1[3] = {k1 / (L.n[1] * L.n[2]), (k1 / L.n[2]) % L.n[1], k1 % L.n[2]};
    const int j2[3] = {k2 / (L.n[1] * L.n[2]), (k2 / L.n[2]) % L.n[1], k2 % L.n[2]};
    int c = 0;
    for (int d = 0; d < 3; ++d) c = c * L.n[d] + ((j2[d] - j1[d]) % L.n[d] + L.n[d]) % L.n[d];
    kp_of_cls[c]++;
  }
  // (primitive pair, image, component) units of the pair transforms per q:
  // every pair (pmode 0), not both diffuse (1), both diffuse (2)
  double img_pp[3] = {0.0, 0.0, 0.0};
  for (int ip = 0; ip < npair; ++ip) {
    const Pair &pp = hp.pairs[ip];
    const Shell &sA = hp.ao[pp.sa], &sB = hp.ao[pp.sb];
    const double w = (double)hp.cls_off[(size_t)ip * (nk + 1) + nk] * ncart_h(sA.l) * ncart_h(sB.l);
    const double all = (double)sA.nprim * sB.nprim, dd = (double)ndiff(sA, hp.ao_exp) * ndiff(sB, hp.ao_exp);
    img_pp[0] += all * w;
    img_pp[1] += (all - dd) * w;
    img_pp[2] += dd * w;
  }
  struct Part {
    std::vector<int64_t> qoff;
    int pmode;
  };
  std::vector<Part> parts;
  {
    std::vector<double> qv;
    Part rs;
    make_qsets(hp.lt, hp.kvec, omega, g_thr, qv, rs.qoff);
    rs.pmode = acut > 0.0 ? 1 : 0;
    parts.push_back(rs);
    if (acut > 0.0) {
      Part d, c;
      make_qsets_sphere(hp.lt, hp.kvec, 4.0 * acut * std::log(1.0 / g_thr), qv, d.qoff);
      d.pmode = 0;
      make_qsets_sphere(hp.lt, hp.kvec, 8.0 * acut * std::log(1.0 / g_thr), qv, c.qoff);
      c.pmode = 2;
      parts.push_back(d);
      parts.push_back(c);
    }
  }
  double nq = 0.0, gemm = 0.0, kphase = 0.0, cand = 0.0;
  for (const Part &pt : parts)
    for (int c = 0; c < nk; ++c) {
      const double nqc = (double)(pt.qoff[c + 1] - pt.qoff[c]);
      if (kp_of_cls[c] == 0) continue;
      nq += nqc;
      cand += nqc * img_pp[pt.pmode];
      gemm += 8.0 * (double)hp.naux * nqc * (double)hp.nao * hp.nao * kp_of_cls[c];
      kphase += nqc * (double)hp.nao * hp.nao * (nk + kp_of_cls[c]);
    }
  feat[0] = sr;                                              // SR operations (cost estimate)
  feat[1] = cand;                                            // pair-transform candidate components
  feat[2] = gemm;                                            // contraction flops
  feat[3] = kphase;                                          // k2-phase elements read + written
  feat[4] = (double)hp.kp1.size() * hp.naux * hp.nao * hp.nao;  // output elements (fold, write-out)
  feat[5] = (double)nk * nk * hp.naux * hp.nao * hp.nao;     // short-range intermediate elements
  feat[6] = nq;                                              // q vectors summed over the classes
  feat[7] = sr_terms;                                        // SR primitive terms (estimate)
  feat[8] = 1.0;                                             // per-build fixed cost
  return RSGDF_OK;
}

int rsgdf_plan_features(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                        const int32_t kmesh[3], double omega, double thresh, double g_thresh,
                        double feat[RSGDF_NFEATURES]) {
  return rsgdf_plan_features_acut(cell, basis, auxbasis, kmesh, omega, 0.0, thresh, g_thresh, feat);
}

// argmin over the (omega, alpha_cut) grid of the predicted time sum_i coef[i] feat[i]
int rsgdf_choose_params(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                        const int32_t kmesh[3], double thresh, double g_thresh, const double *omegas, int32_t nomega,
                        const double *acuts, int32_t nacut, const double coef[RSGDF_NFEATURES], double *best_omega,
                        double *best_acut, double *predicted_ms) {
  g_err.clear();
  if (!omegas || nomega < 1 || !acuts || nacut < 1 || !coef || !best_omega || !best_acut)
    return fail(RSGDF_EINVAL, "null argument or no candidates");
  double best = 1e300;
  int ib = -1;
  for (int i = 0; i < nomega; ++i)
    for (int j = 0; j < nacut; ++j) {
      double f[RSGDF_NFEATURES];
      const int rc = rsgdf_plan_features_acut(cell, basis, auxbasis, kmesh, omegas[i], acuts[j], thresh, g_thresh, f);
      if (rc) return rc;
      double t = 0.0;
      for (int k = 0; k < RSGDF_NFEATURES; ++k) t += coef[k] * f[k];
      if (predicted_ms) predicted_ms[(size_t)i * nacut + j] = t;
      if (t < best) {
        best = t;
        ib = i * nacut + j;
      }
    }
  *best_omega = omegas[ib / nacut];
  *best_acut = acuts[ib % nacut];
  return RSGDF_OK;
}

// argmin over the candidate omegas of the predicted time sum_i coef[i] feat[i]
int rsgdf_choose_omega(const rsgdf_cell *cell, const rsgdf_basis *basis, const rsgdf_basis *auxbasis,
                       const int32_t kmesh[3], double thresh, double g_thresh, const double *omegas, int32_t nomega,
                       const double coef[RSGDF_NFEATURES], double *best_omega, double *predicted_ms) {
  g_err.clear();
  if (!omegas || nomega < 1 || !coef || !best_omega) return fail(RSGDF_EINVAL, "null argument or no candidates");
  double best = 1e300;
  int ib = -1;
  for (int i = 0; i < nomega; ++i) {
    double f[RSGDF_NFEATURES];
    const int rc = rsgdf_plan_features(cell, basis, auxbasis, kmesh, omegas[i], thresh, g_thresh, f);
    if (rc) return rc;
    double t = 0.0;
    for (int j = 0; j < RSGDF_NFEATURES; ++j) t += coef[j] * f[j];
    if (predicted_ms) predicted_ms[i] = t;
    if (t < best) {
      best = t;
      ib = i;
    }
  }
  *best_omega = omegas[ib];
  return RSGDF_OK;
}

}  // extern "C"
