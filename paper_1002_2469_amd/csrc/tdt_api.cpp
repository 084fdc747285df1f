// tdt_api.cpp -- host side of the C ABI declared in include/tdt.h: the
// once-per-matrix preliminary step (plan), workspace management and the
// launch sequence of a solve.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <limits>
#include <new>
#include <numeric>
#include <queue>
#include <exception>
#include <vector>

#include "tdt.h"
#include "tdt_internal.h"
#include "tdt_strided.h"


using tdt::SysDesc;
typedef long double ld;

// tdt_last_info reports TDT_ERR_NOT_CONVERGED above this estimated remaining
// relative error of a refinement.
constexpr float kNotConvergedRel = 1e-7f;

struct tdt_plan_s {
  // work shape (index into tdt::kShapes): B rows per lane, NT lanes, tiles of L rows
  int shape = 0;
  int B = tdt::kShapes[0].B, NT = tdt::kShapes[0].NT;
  int64_t L = (int64_t)tdt::kShapes[0].B * tdt::kShapes[0].NT;
  // the creation arguments (a change of shape rebuilds the plan from them)
  std::vector<double> in_tm1, in_t0, in_t1;
  std::vector<double> in_psi, in_chi;   // quasi-Toeplitz corner terms (quasi plans)
  std::vector<int64_t> in_sizes, in_offs;
  bool quasi = false;     // every system is quasi-Toeplitz (eq. (21))
  bool chunks = false;    // series of 2049..16384 tiles: interface pass in chunks of 64 tiles
  // general (per-row) matrix of a series plan: its rows, and per direction the
  // per-row LU and per-block constants (compute precision), per-tile end values
  bool general = false;
  std::vector<double> in_ga, in_gb, in_gc;
  void* dgrow[2] = {nullptr, nullptr};
  void* dgblk[2] = {nullptr, nullptr};
  double* dgtK[2] = {nullptr, nullptr};
  // first and last row of each tile's inverse, in double: with supports
  // (gen_kf > 0, the widest over all tiles) only their entries,
  // [tile][gen_kf + gen_kl]; without, double plans keep whole rows,
  // [tile][2][L], and float plans none
  void* dggreen[2] = {nullptr, nullptr};
  int gen_kf[2] = {0, 0}, gen_kl[2] = {0, 0};
  int64_t reserved_M = 0;
  // strided batch plan (systems along a slow axis): P classes of order N
  bool strided = false;
  int64_t sP = 0;
  int sC = 0;
  double* dstr = nullptr;   // iu [kStrB][P] | sc [kStrScalarN][P] | pos [2][C][P]
  // a system longer than one column: sK tiles (tdt::strided_tiles), the
  // full tile's tables, the last tile's and the end values one after
  // another at dstr
  int64_t sK = 1;
  bool varlen = false;
  tdt_dtype_t dtype = TDT_F64;
  int64_t N = 0;          // series: order of the system (with its corner rows)
  int64_t S = 1;          // number of systems
  int64_t total = 0;      // varlen: packed length
  std::vector<SysDesc> hsys[2];   // [0]: T, [1]: T^T (adjoint)
  SysDesc* dsys[2] = {nullptr, nullptr};
  double* dvec64[2] = {nullptr, nullptr};
  float* dvec32[2] = {nullptr, nullptr};
  double* dtab64[2] = {nullptr, nullptr};
  float* dtab32[2] = {nullptr, nullptr};
  double* dgreen[2] = {nullptr, nullptr};   // series with several tiles: [2][L]
  // rows of a tile the first pass reads from the head and the tail (0: all)
  int green_kf[2] = {0, 0}, green_kl[2] = {0, 0};
  // varlen: the systems' Green row supports, packed (SysDesc goff, gkf, gkl)
  double* dgpack[2] = {nullptr, nullptr};
  double* dttab[2] = {nullptr, nullptr};    // per tile position table [2][ttab_n]
  int64_t ttab_n = 0;
  // varlen launch lists: [0] forward solves, [1] the adjoint, which solves
  // only one-tile systems whole (its whole-system kernel holds no prefetched
  // tile: the register budget goes to the gradient sums, so it streams
  // multi-tile systems slower than the tile kernels)
  std::vector<int64_t> order;   // systems, largest first
  int sys_max_tiles = tdt::kSysMaxTilesDefault;
  struct Lists {
    int2* p1 = nullptr;     // first pass by sweeps: (system, tile)
    int2* ends = nullptr;   // first pass from the Green rows' supports: (system, full tile)
    int2* fin = nullptr;    // final pass: (system, tile)
    int* grid = nullptr;    // systems with an interface pass across tiles
    int* whole = nullptr;   // systems solved whole by one workgroup each, by bins
    int* bins = nullptr;
    int64_t n_p1 = 0, n_ends = 0, n_fin = 0, n_grid = 0, n_whole = 0, n_bins = 0;
  } lists[2];
  int64_t vslots = 0, vfslots = 0;
  // workspace
  int64_t ws_slots = 0, ws_fslots = 0;
  double* summ = nullptr;
  double* ghost = nullptr;
  double* gscr = nullptr;
  double* gpart = nullptr;
  int* iters = nullptr;
  double dominance = 0.0, kappa = 0.0;
  int max_iter = 40;
  double refine_tol = 1e-13;
  int wg_per_cu = 0;
  // measurement
  bool profile = false;
  std::vector<hipEvent_t> prof_ev;   // 4 per recorded solve
};

// ---------------------------------------------------------------------------
// Preliminary step (host, long double).
// ---------------------------------------------------------------------------
namespace {

// LU multipliers of the B x B block and its responses to unit outside values
// (the forward sweep d_i = (q_i - t_-1 d_{i-1}) / u_i and back substitution
// y_i = d_i - (t_1/u_i) y_{i+1} the kernels run).  Returns false on a zero pivot.
bool block_vectors(ld a, ld b, ld c, int B, ld* iu, ld* cp, ld* phi, ld* chi) {
  ld u = b;
  if (u == 0.0L) return false;
  iu[0] = 1.0L / u;
  cp[0] = c * iu[0];
  for (int i = 1; i < B; ++i) {
    u = b - a * cp[i - 1];
    if (u == 0.0L) return false;
    iu[i] = 1.0L / u;
    cp[i] = c * iu[i];
  }
  // phi: T_B phi = -t_-1 e_0
  phi[0] = -a * iu[0];
  for (int i = 1; i < B; ++i) phi[i] = -a * phi[i - 1] * iu[i];
  for (int i = B - 2; i >= 0; --i) phi[i] -= cp[i] * phi[i + 1];
  // chi: T_B chi = -t_1 e_{B-1}
  for (int i = 0; i + 1 < B; ++i) chi[i] = 0.0L;
  chi[B - 1] = -c * iu[B - 1];
  for (int i = B - 2; i >= 0; --i) chi[i] -= cp[i] * chi[i + 1];
  return true;
}

// End values (phi_first, phi_last, chi_first, chi_last) of a run of L rows,
// by an O(L) long double elimination.  Returns false on a zero pivot.
bool segment_ends_sweep(ld a, ld b, ld c, int64_t L, ld out[4]) {
  std::vector<ld> cpv((size_t)L), d1((size_t)L), d2((size_t)L);
  ld u = b;
  if (u == 0.0L) return false;
  ld iu = 1.0L / u;
  cpv[0] = c * iu;
  d1[0] = -a * iu;
  d2[0] = L == 1 ? -c * iu : 0.0L;
  for (int64_t i = 1; i < L; ++i) {
    u = b - a * cpv[i - 1];
    if (u == 0.0L) return false;
    iu = 1.0L / u;
    cpv[i] = c * iu;
    d1[i] = (0.0L - a * d1[i - 1]) * iu;
    d2[i] = ((i == L - 1 ? -c : 0.0L) - a * d2[i - 1]) * iu;
  }
  for (int64_t i = L - 2; i >= 0; --i) {
    d1[i] -= cpv[i] * d1[i + 1];
    d2[i] -= cpv[i] * d2[i + 1];
  }
  out[0] = d1[0];
  out[1] = d1[L - 1];
  out[2] = d2[0];
  out[3] = d2[L - 1];
  return std::isfinite((double)out[0]) && std::isfinite((double)out[1]) &&
         std::isfinite((double)out[2]) && std::isfinite((double)out[3]);
}

struct SegLD {
  ld yf, yl, pf, pl, cf, cl;
};
bool merge_ld(const SegLD& L, const SegLD& R, SegLD& M);

// The same end values by the merge of the dichotomy step (eqs. (6)-(8)):
// the run of one row is (phi, chi) = (-t_-1/t_0, -t_1/t_0) at both ends, and
// runs of 2k rows are two runs of k merged, so L rows take O(log L) merges
// instead of L elimination steps.  Every merge divides by 1 - chi_last phi_first
// of its two halves; under diagonal dominance both factors are below 1 in
// magnitude (a maximum principle), so the divisor loses at most a few of the
// 64 bits of long double.  Used at dominance ratio >= 1.001; below that (and
// if a merge is refused) the elimination above gives the values.
bool segment_ends(ld a, ld b, ld c, int64_t L, ld out[4]) {
  const ld off = std::fabs(a) + std::fabs(c);
  if (L >= 32 && std::fabs(b) >= 1.001L * off && b != 0.0L) {
    SegLD acc{0, 0, 0, 1, 1, 0};   // the run of no rows: merging with it changes nothing
    SegLD pw{0, 0, -a / b, -a / b, -c / b, -c / b};
    bool ok = true;
    for (int64_t k = L; k > 0 && ok; k >>= 1) {
      SegLD t;
      if (k & 1) {
        ok = merge_ld(acc, pw, t);
        acc = t;
      }
      if (ok && k > 1) {
        ok = merge_ld(pw, pw, t);
        pw = t;
      }
    }
    if (ok) {
      out[0] = acc.pf;
      out[1] = acc.pl;
      out[2] = acc.cf;
      out[3] = acc.cl;
      if (std::isfinite((double)out[0]) && std::isfinite((double)out[1]) &&
          std::isfinite((double)out[2]) && std::isfinite((double)out[3]))
        return true;
    }
  }
  return segment_ends_sweep(a, b, c, L, out);
}

// First and last row of T_L^{-1} (T = tridiag{a, b, c} of order L): the rows
// r solve T^T r = e_0 and T^T r = e_{L-1}, T^T = tridiag{c, b, a}.
bool green_rows_ld(ld a, ld b, ld c, int64_t L, std::vector<ld>& r1, std::vector<ld>& r2) {
  std::vector<ld> cpv((size_t)L);
  r1.assign((size_t)L, 0.0L);
  r2.assign((size_t)L, 0.0L);
  ld u = b;
  if (u == 0.0L) return false;
  cpv[0] = a / u;                 // super-diagonal of T^T is a
  r1[0] = 1.0L / u;
  r2[0] = L == 1 ? 1.0L / u : 0.0L;
  for (int64_t i = 1; i < L; ++i) {
    u = b - c * cpv[i - 1];       // sub-diagonal of T^T is c
    if (u == 0.0L) return false;
    cpv[i] = a / u;
    r1[i] = (0.0L - c * r1[i - 1]) / u;
    r2[i] = ((i == L - 1 ? 1.0L : 0.0L) - c * r2[i - 1]) / u;
  }
  for (int64_t i = L - 2; i >= 0; --i) {
    r1[i] -= cpv[i] * r1[i + 1];
    r2[i] -= cpv[i] * r2[i + 1];
  }
  return true;
}

bool green_rows(ld a, ld b, ld c, int64_t L, double* first, double* last) {
  std::vector<ld> r1, r2;
  if (!green_rows_ld(a, b, c, L, r1, r2)) return false;
  for (int64_t i = 0; i < L; ++i) {
    first[i] = (double)r1[i];
    last[i] = (double)r2[i];
    if (!std::isfinite(first[i]) || !std::isfinite(last[i])) return false;
  }
  return true;
}

// Where the two Green rows carry their mass (the decay of the inverse's
// entries away from the diagonal under dominance, Sec. 3.4): kf = the
// fewest leading entries of the first row, kl = the fewest trailing entries
// of the last row, such that the rest of the row has 1-norm at most
// kGreenDrop times the row's.  Sums in long double from the small end.
constexpr long double kGreenDrop = 0x1p-60L;
void green_support(const std::vector<ld>& r1, const std::vector<ld>& r2, int64_t& kf,
                   int64_t& kl) {
  const int64_t L = (int64_t)r1.size();
  ld n1 = 0.0L, n2 = 0.0L;
  for (int64_t i = L - 1; i >= 0; --i) n1 += std::fabs(r1[i]);
  for (int64_t i = 0; i < L; ++i) n2 += std::fabs(r2[i]);
  // first row: grow the dropped tail from the far end while it stays small
  ld drop = 0.0L;
  kf = L;
  while (kf > 1 && drop + std::fabs(r1[kf - 1]) <= kGreenDrop * n1) drop += std::fabs(r1[--kf]);
  drop = 0.0L;
  kl = L;
  while (kl > 1 && drop + std::fabs(r2[L - kl]) <= kGreenDrop * n2) drop += std::fabs(r2[L - kl--]);
}

// The supports the first pass of a series plan uses: kf, kl rounded up to
// the kernel's 64-row runs, or 0 (read whole tiles) when they would cover a
// quarter of the tile or more.
void green_support_rounded(int64_t L, int64_t kf, int64_t kl, int& rkf, int& rkl) {
  const int64_t f = (kf + 63) / 64 * 64, l = (kl + 63) / 64 * 64;
  if (4 * (f + l) > L) {
    rkf = rkl = 0;
  } else {
    rkf = (int)f;
    rkl = (int)l;
  }
}

// The same supports without forming the rows (for the many matrices of a
// varlen plan), with their entries.  The rows are ratios of leading minors:
//   (T_L^{-1})_{0,j}         = (-t_1)^j  / (u_{L-1-j} ... u_{L-1}),
//   (T_L^{-1})_{L-1,L-1-m}   = (-t_-1)^m / (u_{L-1-m} ... u_{L-1}),
// u_i the pivots of the elimination (u_0 = t_0, u_i = t_0 - t_-1 t_1 / u_{i-1}).
// Under dominance the pivots settle at u* (the larger root of
// u^2 - t_0 u + t_-1 t_1 = 0); once two agree to long double rounding (at C),
// the entries within L-1-C of the row's own end are geometric,
// (-t_1)^j / u*^(j+1), and every entry is at most |t_1|^j / umin^(j+1),
// umin the smallest |u_i|.  So the mass beyond entry k is at most
// s^k / (umin (1 - s)), s = |t_1| / umin, against a total of at least the
// first entry, 1 / |u*|: kf is the least k with s^k |u*| / (umin (1 - s))
// <= kGreenDrop (the same with t_-1 for kl), a support at least as long as
// the minimal one of green_support.  head: kf entries of the first row from
// its start, tail: kl entries of the last row up to its end, in row order.
// Returns false (no truncation) unless the pivots settle, s < 1 for both
// rows and both supports lie where they have settled.
bool green_support_bound(ld a, ld b, ld c, int64_t L, int64_t& kf, int64_t& kl, ld* ustar,
                         int64_t* settled_at) {
  if (b == 0.0L || L < 2) return false;
  ld u = b, umin = std::fabs(b);
  int64_t C = -1;
  for (int64_t i = 1; i < L; ++i) {
    const ld un = b - a * c / u;
    if (un == 0.0L || !std::isfinite((double)un)) return false;
    umin = std::min(umin, std::fabs(un));
    const bool settled = std::fabs(un - u) <= 0x1p-62L * std::fabs(un);
    u = un;
    if (settled) {
      C = i;
      break;
    }
  }
  if (C < 0) return false;
  auto support = [&](ld t, int64_t& k) {
    const ld sr = std::fabs(t) / umin;
    if (!(sr < 1.0L)) return false;
    if (sr == 0.0L) {
      k = 1;
      return true;
    }
    const ld factor = std::fabs(u) / (umin * (1.0L - sr));
    const ld kk = std::ceil((std::log(kGreenDrop) - std::log(factor)) / std::log(sr));
    k = std::max<int64_t>(1, (int64_t)kk);
    return k <= L - C;
  };
  if (!support(c, kf) || !support(a, kl)) return false;
  if (ustar) *ustar = u;
  if (settled_at) *settled_at = C;
  return true;
}

// The supports a varlen plan's first pass uses for a full tile of L rows
// (green_support_bound rounded up to 64-row runs; false when they would
// cover a quarter of the tile, or reach past where the pivots settled) and
// their entries: head = the first rf entries of the first row, tail = the
// last rl entries of the last row, (-t_1)^j / u*^(j+1) and
// (-t_-1)^m / u*^(m+1) at distance j, m from the row's own end.  These are
// the entries of every order n >= max(rf, rl) + C (C = *settled, where the
// pivots settle): the entries within them involve only the pivots
// u_{n-1-j} .. u_{n-1}, all past C.
bool green_ends(ld a, ld b, ld c, int64_t L, int& rf, int& rl, std::vector<ld>& head,
                std::vector<ld>& tail, int64_t* settled) {
  int64_t kf = 0, kl = 0, C = 0;
  ld us = 0.0L;
  if (!green_support_bound(a, b, c, L, kf, kl, &us, &C)) return false;
  green_support_rounded(L, kf, kl, rf, rl);
  if (rf == 0 || rf > L - C || rl > L - C) return false;
  *settled = C;
  head.assign((size_t)rf, 0.0L);
  tail.assign((size_t)rl, 0.0L);
  ld e = 1.0L / us;
  for (int j = 0; j < rf; ++j, e *= -c / us) head[(size_t)j] = e;
  e = 1.0L / us;
  for (int m = 0; m < rl; ++m, e *= -a / us) tail[(size_t)(rl - 1 - m)] = e;
  return true;
}

bool merge_ld(const SegLD& L, const SegLD& R, SegLD& M) {
  const ld D = 1.0L - L.cl * R.pf;
  if (!(std::fabs((double)D) > 1e-13)) return false;
  const ld iD = 1.0L / D;
  const ld xk0 = (L.yl + L.cl * R.yf) * iD;
  const ld xk10 = R.yf + R.pf * xk0;
  const ld tl = L.pl * iD, ur = R.cf * iD;
  M.yf = L.yf + xk10 * L.cf;
  M.yl = R.yl + xk0 * R.pl;
  M.pf = L.pf + L.cf * R.pf * tl;
  M.pl = tl * R.pl;
  M.cf = L.cf * ur;
  M.cl = R.cl + L.cl * ur * R.pl;
  return true;
}

// The interface merges the kernels perform divide by 1 - chi_last(L) phi_first(R)
// for runs of full blocks of every length up to a wavefront and beyond; check
// them for runs of up to 64 + 64 blocks.  Under diagonal dominance they are
// bounded away from zero (|chi_last|, |phi_first| < 1 by the maximum
// principle, and the divisor of two runs of m and n rows of tridiag{-1,2,-1},
// the weakest dominant case, is (m+n+1)/((m+1)(n+1)) >= 1/1025 here), so the
// check runs only without dominance, where a sub-block may be (nearly)
// singular.
bool merges_ok(const ld blk4[4]) {
  std::vector<SegLD> run(65);
  run[1] = SegLD{0, 0, blk4[0], blk4[1], blk4[2], blk4[3]};
  for (int k = 2; k <= 64; ++k)
    if (!merge_ld(run[k - 1], run[1], run[k])) return false;
  SegLD tmp;
  for (int j = 1; j <= 64; ++j)
    for (int k = 1; k <= 64; ++k)
      if (!merge_ld(run[j], run[k], tmp)) return false;
  return true;
}

double dominance_ratio(double a, double b, double c) {
  const double off = std::fabs(a) + std::fabs(c);
  return off == 0.0 ? std::numeric_limits<double>::infinity() : std::fabs(b) / off;
}

// Row dominance of a quasi-Toeplitz matrix: the inner rows and the two
// corner rows (t0+psi next to t_1, t0+chi next to t_-1).
double quasi_dominance(double a, double b, double c, double psi, double chi) {
  const double inf = std::numeric_limits<double>::infinity();
  auto ratio = [&](double d, double off) { return off == 0.0 ? inf : std::fabs(d) / off; };
  return std::min(dominance_ratio(a, b, c),
                  std::min(ratio(b + psi, std::fabs(c)), ratio(b + chi, std::fabs(a))));
}

// Upper bound of the 2-norm condition number of a quasi-Toeplitz matrix of
// order n >= 3: kappa_2 <= sqrt(kappa_1 kappa_inf), each bounded by the norm
// times the inverse-norm bound of a strictly dominant matrix (the smallest
// diagonal excess over its row's, resp. column's, off-diagonal sum);
// infinite without strict row and column dominance.
double quasi_condition_bound(double a, double b, double c, double psi, double chi) {
  const double inf = std::numeric_limits<double>::infinity();
  const double A = std::fabs(a), C = std::fabs(c), d = std::fabs(b);
  const double d0 = std::fabs(b + psi), d1 = std::fabs(b + chi);
  // rows: first (d0, C), inner (d, A + C), last (d1, A); columns: first
  // (d0, A), inner (d, A + C), last (d1, C)
  const double rex = std::min(d0 - C, std::min(d - A - C, d1 - A));
  const double cex = std::min(d0 - A, std::min(d - A - C, d1 - C));
  if (!(rex > 0.0) || !(cex > 0.0)) return inf;
  const double rnorm = std::max(d0 + C, std::max(d + A + C, d1 + A));
  const double cnorm = std::max(d0 + A, std::max(d + A + C, d1 + C));
  return std::sqrt((rnorm / rex) * (cnorm / cex));
}

// 2-norm condition number from the closed-form spectrum when t_1 t_-1 > 0
// (T is similar to a symmetric matrix), else the infinity-norm bound.
double condition_number(double a, double b, double c, int64_t n) {
  if (a * c > 0.0) {
    const double s = std::sqrt(a * c) * (c > 0 ? 1.0 : -1.0);
    const double pi = 3.14159265358979323846;
    auto lam = [&](double k) { return b + 2.0 * s * std::cos(k * pi / (double)(n + 1)); };
    double lmax = std::max(std::fabs(lam(1)), std::fabs(lam((double)n)));
    double lmin = std::min(std::fabs(lam(1)), std::fabs(lam((double)n)));
    if (std::fabs(b) < 2.0 * std::fabs(s)) {   // the spectrum straddles zero
      const double th = std::acos(-b / (2.0 * s));
      const double k0 = th * (double)(n + 1) / pi;
      for (double k = std::floor(k0) - 1; k <= std::floor(k0) + 2; k += 1.0)
        if (k >= 1 && k <= (double)n) lmin = std::min(lmin, std::fabs(lam(k)));
    }
    return lmin > 0 ? lmax / lmin : std::numeric_limits<double>::infinity();
  }
  const double off = std::fabs(a) + std::fabs(c);
  if (std::fabs(b) > off) return (std::fabs(b) + off) / (std::fabs(b) - off);
  if (n == 1) return 1.0;
  return std::numeric_limits<double>::infinity();
}

// Fill the descriptor and the block vectors of one system.
tdt_status_t build_system(double a, double b, double c, int64_t n, bool quasi, int kB, int kNT,
                          SysDesc& D, double* v64, float* v32, double* t64, float* t32) {
  const int64_t kTile = (int64_t)kB * kNT;
  ld iu[tdt::kMaxB], cp[tdt::kMaxB], phi[tdt::kMaxB], chi[tdt::kMaxB];
  if (!block_vectors(a, b, c, kB, iu, cp, phi, chi)) return TDT_ERR_SINGULAR;
  for (int i = 0; i < kB; ++i) {
    ld vv[tdt::kVecN];
    vv[tdt::kVecIU] = iu[i];
    vv[tdt::kVecCP] = cp[i];
    vv[tdt::kVecPHI] = phi[i];
    vv[tdt::kVecCHI] = chi[i];
    vv[tdt::kVecAIU] = (ld)a * iu[i];
    for (int k = 0; k < tdt::kVecN; ++k) {
      v64[k * kB + i] = (double)vv[k];
      v32[k * kB + i] = (float)vv[k];
      if (!std::isfinite(v64[k * kB + i])) return TDT_ERR_SINGULAR;
    }
  }
  D.a = a;
  D.b = b;
  D.c = c;
  D.n = n;
  D.ntiles = (int32_t)((n + kTile - 1) / kTile);
  const ld blk[4] = {phi[0], phi[kB - 1], chi[0], chi[kB - 1]};
  for (int k = 0; k < 4; ++k) D.blk[k] = (double)blk[k];
  if (std::fabs(b) < std::fabs(a) + std::fabs(c) && !merges_ok(blk)) return TDT_ERR_SINGULAR;
  // per-position table of the left-to-right interface elimination over the
  // NT blocks of a tile: beta_{m-1} and 1/(1 - phi_first beta_{m-1})
  // (beta_m contracts to a fixed point, under dominance within a few
  // blocks; once it repeats exactly, so does every later entry)
  D.tfix = 0;
  {
    ld beta = 0.0L;
    bool fixed = false;
    ld iD = 1.0L;
    for (int m = 0; m < kNT; ++m) {
      if (!fixed) {
        const ld D = 1.0L - blk[0] * beta;
        if (!(std::fabs((double)D) > 1e-13)) return TDT_ERR_SINGULAR;
        iD = 1.0L / D;
      }
      t64[tdt::kTabBeta * kNT + m] = (double)beta;
      t64[tdt::kTabInvD * kNT + m] = (double)iD;
      t32[tdt::kTabBeta * kNT + m] = (float)beta;
      t32[tdt::kTabInvD * kNT + m] = (float)iD;
      if (!fixed) {
        const ld next = blk[3] + blk[1] * beta * blk[2] * iD;
        if (!std::isfinite((double)next)) return TDT_ERR_SINGULAR;
        fixed = next == beta;
        if (fixed) D.tfix = m;   // entries m, m + 1, ... are equal
        beta = next;
      }
    }
  }
  // last block of the system
  const int bt = (int)((n - 1) % kB) + 1;
  if (bt == kB) {
    D.tail_pf = D.blk[0];
    D.tail_pl = D.blk[1];
    D.tail_cf = D.blk[2];
  } else {
    ld e[4];
    if (!segment_ends(a, b, c, bt, e)) return TDT_ERR_SINGULAR;
    D.tail_pf = (double)e[0];
    D.tail_pl = (double)e[1];
    D.tail_cf = (double)e[2];
    for (int m = 0; m < kNT; ++m)   // the last block may sit at any position
      if (!(std::fabs(1.0 - D.tail_pf * t64[tdt::kTabBeta * kNT + m]) > 1e-13))
        return TDT_ERR_SINGULAR;
  }
  // end values of a full tile and of the last tile (its real length), which
  // the interface pass needs when the system has several tiles or corner rows
  for (int k = 0; k < 4; ++k) D.tileK[k] = D.ltileK[k] = 0.0;
  if (D.ntiles > 1 || quasi) {
    ld e[4];
    const int64_t lt = n - (int64_t)(D.ntiles - 1) * kTile;
    if (D.ntiles > 1) {
      if (!segment_ends(a, b, c, kTile, e)) return TDT_ERR_SINGULAR;
      for (int k = 0; k < 4; ++k) D.tileK[k] = (double)e[k];
    }
    if (lt == kTile && D.ntiles > 1) {
      for (int k = 0; k < 4; ++k) D.ltileK[k] = D.tileK[k];
    } else {
      if (!segment_ends(a, b, c, lt, e)) return TDT_ERR_SINGULAR;
      for (int k = 0; k < 4; ++k) D.ltileK[k] = (double)e[k];
    }
  }
  return TDT_OK;
}

// Corner constants of a quasi-Toeplitz system (first diagonal entry t0+psi,
// last t0+chi; a, c the sub- and super-diagonal of the matrix being solved):
// each corner row alone, and its response to the unknown next to it.
tdt_status_t corner_constants(double a, double b, double c, double psi, double chi, SysDesc& D) {
  const ld d0 = (ld)b + (ld)psi, d1 = (ld)b + (ld)chi;
  if (d0 == 0.0L || d1 == 0.0L) return TDT_ERR_SINGULAR;
  D.quasi = 1;
  D.qc[0] = (double)(1.0L / d0);
  D.qc[1] = (double)(-(ld)c / d0);
  D.qc[2] = (double)(1.0L / d1);
  D.qc[3] = (double)(-(ld)a / d1);
  D.qc[4] = D.qc[5] = 0.0;   // set with the interface table
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(D.qc[k])) return TDT_ERR_SINGULAR;
  return TDT_OK;
}

// A system goes through the interface pass when it has several tiles or
// corner rows.
bool needs_interface(const SysDesc& D) { return D.ntiles > 1 || D.quasi != 0; }

bool finite3(double a, double b, double c) {
  return std::isfinite(a) && std::isfinite(b) && std::isfinite(c);
}

template <typename T>
tdt_status_t dev_upload(T** dst, const T* src, size_t count) {
  *dst = nullptr;
  if (count == 0) return TDT_OK;
  if (hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return TDT_ERR_OOM;
  }
  if (hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return TDT_ERR_HIP;
  return TDT_OK;
}

void free_workspace(tdt_plan_s* p) {
  (void)hipFree(p->summ);
  (void)hipFree(p->ghost);
  (void)hipFree(p->gscr);
  (void)hipFree(p->gpart);
  p->summ = p->ghost = p->gscr = p->gpart = nullptr;
  p->ws_slots = p->ws_fslots = 0;
}

// Make sure the workspace holds `slots` tile slots and `fslots` adjoint
// partial-sum slots.  Never allocates while the stream is being captured.
tdt_status_t ensure_workspace(tdt_plan_s* p, int64_t slots, int64_t fslots, hipStream_t st) {
  // the kernels read the values just outside a tile unconditionally (slot 0
  // for a one-tile system), so every array holds at least one slot
  slots = std::max<int64_t>(slots, 1);
  fslots = std::max<int64_t>(fslots, 1);
  if (slots <= p->ws_slots && fslots <= p->ws_fslots) return TDT_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return TDT_ERR_CAPTURE;
  const int64_t ns = std::max(slots, p->ws_slots), nf = std::max(fslots, p->ws_fslots);
  (void)hipDeviceSynchronize();
  free_workspace(p);
  if (hipMalloc(&p->summ, (size_t)ns * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->ghost, (size_t)ns * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->gscr, (size_t)ns * 3 * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->gpart, (size_t)nf * tdt::kGradN * sizeof(double)) != hipSuccess) {
    free_workspace(p);
    return TDT_ERR_OOM;
  }
  if (hipMemset(p->ghost, 0, (size_t)ns * 2 * sizeof(double)) != hipSuccess) {
    free_workspace(p);
    return TDT_ERR_HIP;
  }
  p->ws_slots = ns;
  p->ws_fslots = nf;
  return TDT_OK;
}

void clear_profile(tdt_plan_s* p) {
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  p->prof_ev.clear();
}

void destroy(tdt_plan_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  clear_profile(p);
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(p->dsys[k]);
    (void)hipFree(p->dvec64[k]);
    (void)hipFree(p->dvec32[k]);
    (void)hipFree(p->dtab64[k]);
    (void)hipFree(p->dtab32[k]);
    (void)hipFree(p->dgreen[k]);
    (void)hipFree(p->dttab[k]);
    (void)hipFree(p->dgrow[k]);
    (void)hipFree(p->dgblk[k]);
    (void)hipFree(p->dgtK[k]);
    (void)hipFree(p->dggreen[k]);
  }
  (void)hipFree(p->dstr);
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(p->dgpack[k]);
    tdt_plan_s::Lists& q = p->lists[k];
    (void)hipFree(q.p1);
    (void)hipFree(q.ends);
    (void)hipFree(q.fin);
    (void)hipFree(q.grid);
    (void)hipFree(q.whole);
    (void)hipFree(q.bins);
  }
  (void)hipFree(p->iters);
  free_workspace(p);
  delete p;
}

// Work lists of a varlen plan.  Systems of at most sys_max_tiles tiles are
// solved whole by one workgroup each (largest first); the others go through
// the three kernels: first pass over their tiles, interface pass, final pass
// over their tiles in the reverse of the first pass's order (the most
// recently read, still cached, tiles first).
tdt_status_t build_lists(tdt_plan_s* p, int dir, int max_tiles) {
  tdt_plan_s::Lists& q = p->lists[dir];
  std::vector<int2> p1, fin;
  std::vector<int> grid, whole_sys;
  for (int64_t s : p->order) {
    const int nt = p->hsys[0][s].ntiles;
    if (nt <= max_tiles) {
      whole_sys.push_back((int)s);
    } else {
      for (int t = 0; t < nt; ++t) p1.push_back(make_int2((int)s, t));
      if (needs_interface(p->hsys[0][s])) grid.push_back((int)s);
    }
  }
  // systems outside the whole-system list without an interface pass (one
  // tile, no corner rows): no first pass
  std::vector<int2> single;
  auto alone = [&](const int2& it) { return !needs_interface(p->hsys[0][it.x]); };
  for (const int2& it : p1)
    if (alone(it)) single.push_back(it);
  p1.erase(std::remove_if(p1.begin(), p1.end(), alone), p1.end());
  fin.assign(p1.rbegin(), p1.rend());
  fin.insert(fin.end(), single.begin(), single.end());
  // full tiles of systems whose Green rows decay (in both directions), and
  // their last tiles where long enough: their summaries are dot products
  // with the rows' supports, not sweeps
  std::vector<int2> ends;
  auto by_ends = [&](const int2& it) {
    const SysDesc& D0 = p->hsys[0][it.x];
    const SysDesc& D1 = p->hsys[1][it.x];
    const bool full = (int64_t)(it.y + 1) * p->L <= D0.n;
    return D0.gkf > 0 && D1.gkf > 0 && (full || (D0.glast && D1.glast));
  };
  for (const int2& it : p1)
    if (by_ends(it)) {
      // long supports: a wavefront per tile end
      const SysDesc& D = p->hsys[dir][it.x];
      if (D.gkf + D.gkl > tdt::kEndsSplitRows) {
        ends.push_back(make_int2(it.x, it.y | (1 << tdt::kEndsPartShift)));
        ends.push_back(make_int2(it.x, it.y | (2 << tdt::kEndsPartShift)));
      } else {
        ends.push_back(it);
      }
    }
  p1.erase(std::remove_if(p1.begin(), p1.end(), by_ends), p1.end());
  // Whole systems: by default one workgroup each, largest first, so that
  // the hardware starts the next system wherever a workgroup finishes (the
  // longest-processing-time order, scheduled dynamically).  With a cap of
  // persistent workgroups per CU, the systems go to that many lists instead,
  // each system (largest first) to the least loaded list; a system of nt
  // tiles costs about 2 nt tile steps (summaries, then the solve), a
  // one-tile system one.
  std::vector<int> whole, bins;
  if (!whole_sys.empty() && p->wg_per_cu == 0) {
    whole = whole_sys;
    for (size_t b = 0; b <= whole.size(); ++b) bins.push_back((int)b);
  } else if (!whole_sys.empty()) {
    const int64_t G = std::min<int64_t>(
        (int64_t)whole_sys.size(),
        std::max(1, tdt::sys_wg_capacity(p->shape, (int)p->dtype, p->wg_per_cu,
                                         p->quasi ? 1 : 0)));
    std::vector<std::vector<int>> lists((size_t)G);
    typedef std::pair<int64_t, int64_t> Load;   // (cost so far, list)
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int64_t b = 0; b < G; ++b) heap.push(Load(0, b));
    for (int s : whole_sys) {
      const int nt = p->hsys[0][s].ntiles;
      Load l = heap.top();
      heap.pop();
      lists[(size_t)l.second].push_back(s);
      l.first += needs_interface(p->hsys[0][s]) ? 2 * nt : 1;
      heap.push(l);
    }
    bins.push_back(0);
    for (const auto& l : lists) {
      whole.insert(whole.end(), l.begin(), l.end());
      bins.push_back((int)whole.size());
    }
  }
  (void)hipFree(q.p1);
  (void)hipFree(q.ends);
  (void)hipFree(q.fin);
  (void)hipFree(q.grid);
  (void)hipFree(q.whole);
  (void)hipFree(q.bins);
  q = tdt_plan_s::Lists{};
  q.n_p1 = (int64_t)p1.size();
  q.n_ends = (int64_t)ends.size();
  q.n_fin = (int64_t)fin.size();
  q.n_grid = (int64_t)grid.size();
  q.n_whole = (int64_t)whole.size();
  q.n_bins = bins.empty() ? 0 : (int64_t)bins.size() - 1;
  tdt_status_t st = dev_upload(&q.p1, p1.data(), p1.size());
  if (st == TDT_OK) st = dev_upload(&q.ends, ends.data(), ends.size());
  if (st == TDT_OK) st = dev_upload(&q.fin, fin.data(), fin.size());
  if (st == TDT_OK) st = dev_upload(&q.grid, grid.data(), grid.size());
  if (st == TDT_OK) st = dev_upload(&q.whole, whole.data(), whole.size());
  if (st == TDT_OK) st = dev_upload(&q.bins, bins.data(), bins.size());
  return st;
}

tdt_status_t build_varlen_lists(tdt_plan_s* p) {
  const tdt_status_t st = build_lists(p, 0, p->sys_max_tiles);
  return st == TDT_OK ? build_lists(p, 1, std::min(p->sys_max_tiles, 1)) : st;
}

// Build both descriptor sets (T and T^T) and upload everything.  sizes and
// offs are the systems' orders and first rows; the tiles of a quasi-Toeplitz
// system cover its N - 2 inner rows.
tdt_status_t finish_plan(tdt_plan_s* p, const std::vector<double>& tm1,
                         const std::vector<double>& t0, const std::vector<double>& t1,
                         const std::vector<int64_t>& sizes, const std::vector<int64_t>& offs) {
  const int64_t S = (int64_t)sizes.size();
  const int64_t cut = p->quasi ? 2 : 0;
  double dom = std::numeric_limits<double>::infinity(), kap = 0.0;
  for (int dir = 0; dir < 2; ++dir) {
    const int kB = p->B, kNT = p->NT;
    const int64_t kTile = p->L;
    std::vector<double> v64((size_t)S * tdt::kVecN * kB);
    std::vector<float> v32((size_t)S * tdt::kVecN * kB);
    std::vector<double> t64((size_t)S * tdt::kTabN * kNT);
    std::vector<float> t32((size_t)S * tdt::kTabN * kNT);
    p->hsys[dir].assign((size_t)S, SysDesc());
    for (int64_t s = 0; s < S; ++s) {
      const double a = dir == 0 ? tm1[s] : t1[s];
      const double c = dir == 0 ? t1[s] : tm1[s];
      SysDesc& D = p->hsys[dir][s];
      std::memset(&D, 0, sizeof(D));
      tdt_status_t st = build_system(a, t0[s], c, sizes[s] - cut, p->quasi, kB, kNT, D,
                                     v64.data() + (size_t)s * tdt::kVecN * kB,
                                     v32.data() + (size_t)s * tdt::kVecN * kB,
                                     t64.data() + (size_t)s * tdt::kTabN * kNT,
                                     t32.data() + (size_t)s * tdt::kTabN * kNT);
      if (st != TDT_OK) return st;
      if (p->quasi) {
        st = corner_constants(a, t0[s], c, p->in_psi[s], p->in_chi[s], D);
        if (st != TDT_OK) return st;
      }
      D.off = offs[s] + cut / 2;
      D.stride = sizes[s];
      D.cidx = (int32_t)s;
      if (dir == 0) {
        if (p->quasi) {
          dom = std::min(dom, quasi_dominance(tm1[s], t0[s], t1[s], p->in_psi[s], p->in_chi[s]));
          kap = std::max(kap, quasi_condition_bound(tm1[s], t0[s], t1[s], p->in_psi[s],
                                                    p->in_chi[s]));
        } else {
          dom = std::min(dom, dominance_ratio(tm1[s], t0[s], t1[s]));
          kap = std::max(kap, condition_number(tm1[s], t0[s], t1[s], sizes[s]));
        }
      }
    }
    // varlen bookkeeping: adjoint partial-sum slots, one per tile and one
    // per corner row
    int64_t fs = 0;
    for (int64_t s = 0; s < S; ++s) {
      p->hsys[dir][s].fslot0 = (int32_t)fs;
      fs += p->hsys[dir][s].ntiles + (p->quasi ? 2 : 0);
    }
    p->vfslots = fs;
    // varlen: Green row supports of each multi-tile system's full tiles
    if (p->varlen) {
      std::vector<double> pack;
      std::vector<ld> head, tail;
      for (int64_t s = 0; s < S; ++s) {
        SysDesc& D = p->hsys[dir][s];
        D.goff = 0;
        D.gkf = D.gkl = D.glast = 0;
        if (!needs_interface(D)) continue;
        const double a = dir == 0 ? tm1[s] : t1[s], c = dir == 0 ? t1[s] : tm1[s];
        int rf = 0, rl = 0;
        int64_t C = 0;
        if (!green_ends(a, t0[s], c, kTile, rf, rl, head, tail, &C)) continue;
        const int64_t tl = D.n - (int64_t)(D.ntiles - 1) * kTile;
        D.glast = tl < kTile && tl >= std::max(rf, rl) + C ? 1 : 0;
        // a quasi-Toeplitz system of one shorter tile: only if that tile is
        // long enough for the entries
        if (D.n < kTile && !D.glast) continue;
        D.goff = (int64_t)pack.size();
        D.gkf = (int32_t)rf;
        D.gkl = (int32_t)rl;
        for (ld v : head) pack.push_back((double)v);
        for (ld v : tail) pack.push_back((double)v);
      }
      (void)hipFree(p->dgpack[dir]);
      p->dgpack[dir] = nullptr;
      if (!pack.empty()) {
        tdt_status_t sg = dev_upload(&p->dgpack[dir], pack.data(), pack.size());
        if (sg != TDT_OK) return sg;
      }
    }
    p->green_kf[dir] = p->green_kl[dir] = 0;
    if (!p->varlen && needs_interface(p->hsys[dir][0])) {
      std::vector<double> g(2 * (size_t)kTile);
      const double a = dir == 0 ? tm1[0] : t1[0], c = dir == 0 ? t1[0] : tm1[0];
      std::vector<ld> r1, r2;
      if (!green_rows_ld(a, t0[0], c, kTile, r1, r2)) return TDT_ERR_SINGULAR;
      for (int64_t i = 0; i < kTile; ++i) {
        g[(size_t)i] = (double)r1[(size_t)i];
        g[(size_t)(kTile + i)] = (double)r2[(size_t)i];
        if (!std::isfinite(g[(size_t)i]) || !std::isfinite(g[(size_t)(kTile + i)]))
          return TDT_ERR_SINGULAR;
      }
      int64_t kf = 0, kl = 0;
      green_support(r1, r2, kf, kl);
      green_support_rounded(kTile, kf, kl, p->green_kf[dir], p->green_kl[dir]);
      tdt_status_t sg = dev_upload(&p->dgreen[dir], g.data(), g.size());
      if (sg != TDT_OK) return sg;
    }
    tdt_status_t st = dev_upload(&p->dvec64[dir], v64.data(), v64.size());
    if (st == TDT_OK) st = dev_upload(&p->dvec32[dir], v32.data(), v32.size());
    if (st == TDT_OK) st = dev_upload(&p->dtab64[dir], t64.data(), t64.size());
    if (st == TDT_OK) st = dev_upload(&p->dtab32[dir], t32.data(), t32.size());
    if (st != TDT_OK) return st;
  }
  p->dominance = dom;
  p->kappa = kap;
  // interface-pass layout: tiles per thread of the variant the most tiled
  // system selects (see launch_solve), and the run-interleaved slot counts
  {
    int maxp = 1;
    for (const SysDesc& D : p->hsys[0]) maxp = std::max(maxp, (int)D.ntiles);
    // (the same thresholds as launch_grid: <64,1>, <256,1>, <256,8>,
    // <512,16>, <1024,16>, then the segment-merge kernel; a series Toeplitz
    // plan of 2049..16384 tiles takes the chunked pass, one tile per slot)
    p->chunks = !p->varlen && !p->quasi && maxp > 2048 && maxp <= 16384;
    const int tr = p->chunks ? 1
                             : (maxp <= 256 ? 1 : (maxp <= 2048 ? 8 : (maxp <= 16384 ? 16 : 1)));
    for (int dir = 0; dir < 2; ++dir)
      for (SysDesc& D : p->hsys[dir]) {
        D.tr = tr;
        D.tq = (D.ntiles + tr - 1) / tr;
        D.tslots = D.tq * tr;
      }
  }
  if (p->varlen) {
    // workspace slots of the multi-tile systems, largest system first
    p->order.resize((size_t)S);
    std::iota(p->order.begin(), p->order.end(), 0);
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int64_t x, int64_t y) { return sizes[x] > sizes[y]; });
    int64_t slot = 0;
    for (int64_t s : p->order) {
      if (needs_interface(p->hsys[0][s])) {
        for (int dir = 0; dir < 2; ++dir) p->hsys[dir][s].slot0 = (int32_t)slot;
        slot += p->hsys[0][s].tslots;
      }
    }
    p->vslots = slot;
    const tdt_status_t st = build_varlen_lists(p);
    if (st != TDT_OK) return st;
  }
  // interface pass across tiles: beta_{t-1} and 1/(1 - Pf_t beta_{t-1}) for
  // every tile position of every system with an interface pass (a series
  // indexes by tile, a varlen plan by workspace slot), in long double.  A
  // quasi-Toeplitz system starts from its first corner row (beta_{-1} is that
  // row's response to the unknown right of it) and ends with its last.
  p->ttab_n = p->varlen ? std::max<int64_t>(p->vslots, 1)
                        : std::max<int64_t>(p->hsys[0][0].tslots, 1);
  for (int dir = 0; dir < 2; ++dir) {
    std::vector<double> tt(2 * (size_t)p->ttab_n, 0.0);
    for (int64_t s = 0; s < S; ++s) {
      SysDesc& D = p->hsys[dir][s];
      if (!needs_interface(D)) continue;
      const int64_t base = p->varlen ? D.slot0 : 0;
      ld beta = D.quasi ? (ld)D.qc[1] : 0.0L;
      for (int t = 0; t < D.ntiles; ++t) {
        const double* K = t + 1 < D.ntiles ? D.tileK : D.ltileK;
        const ld den = 1.0L - (ld)K[0] * beta;
        if (!(std::fabs((double)den) > 1e-13)) return TDT_ERR_SINGULAR;
        const ld iD = 1.0L / den;
        const int64_t pos = (int64_t)(t % D.tr) * D.tq + t / D.tr;
        tt[base + pos] = (double)beta;
        tt[p->ttab_n + base + pos] = (double)iD;
        beta = (ld)K[3] + (ld)K[1] * beta * (ld)K[2] * iD;
      }
      if (D.quasi) {
        const ld den = 1.0L - (ld)D.qc[3] * beta;
        if (!(std::fabs((double)den) > 1e-13)) return TDT_ERR_SINGULAR;
        D.qc[4] = (double)beta;
        D.qc[5] = (double)(1.0L / den);
      }
    }
    tdt_status_t st = dev_upload(&p->dttab[dir], tt.data(), tt.size());
    if (st != TDT_OK) return st;
  }
  for (int dir = 0; dir < 2; ++dir) {
    tdt_status_t st = dev_upload(&p->dsys[dir], p->hsys[dir].data(), p->hsys[dir].size());
    if (st != TDT_OK) return st;
  }
  {
    const tdt_status_t ws = ensure_workspace(p, 1, 1, nullptr);
    if (ws != TDT_OK) return ws;
  }
  if (hipMalloc(&p->iters, 2 * sizeof(int)) != hipSuccess) return TDT_ERR_OOM;
  if (hipMemset(p->iters, 0, 2 * sizeof(int)) != hipSuccess) return TDT_ERR_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  return p->dominance < 1.0 ? TDT_WARN_NOT_DOMINANT : TDT_OK;
}

// Rebuild the plan for another work shape from its creation arguments,
// keeping its options and reservation.  On failure the plan is unchanged.
tdt_status_t rebuild_plan(tdt_plan_s* p, int shape) {
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  tdt_plan_s* q = new (std::nothrow) tdt_plan_s();
  if (!q) return TDT_ERR_OOM;
  q->shape = shape;
  q->B = tdt::kShapes[shape].B;
  q->NT = tdt::kShapes[shape].NT;
  q->L = (int64_t)q->B * q->NT;
  q->in_tm1 = p->in_tm1;
  q->in_t0 = p->in_t0;
  q->in_t1 = p->in_t1;
  q->in_psi = p->in_psi;
  q->in_chi = p->in_chi;
  q->quasi = p->quasi;
  q->in_sizes = p->in_sizes;
  q->in_offs = p->in_offs;
  q->varlen = p->varlen;
  q->dtype = p->dtype;
  q->N = p->N;
  q->S = p->S;
  q->total = p->total;
  q->sys_max_tiles = p->sys_max_tiles;
  q->max_iter = p->max_iter;
  q->refine_tol = p->refine_tol;
  q->wg_per_cu = p->wg_per_cu;
  tdt_status_t st = finish_plan(q, q->in_tm1, q->in_t0, q->in_t1, q->in_sizes, q->in_offs);
  if (st >= 0 && p->reserved_M > 0) st = tdt_plan_reserve(q, p->reserved_M);
  if (st < 0) {
    destroy(q);
    return st;
  }
  q->profile = p->profile;
  std::swap(*p, *q);
  destroy(q);   // the old buffers
  return TDT_OK;
}

// ---------------------------------------------------------------------------
// General (per-row) matrices.  The system is padded to whole tiles with
// decoupled rows (b = 1, a = c = 0), so every tile is full.  Everything below
// is long double, rounded once on upload.
// ---------------------------------------------------------------------------
// First and last row of the inverse of the L-row matrix with rows
// (a_i, b_i, c_i), i.e. the solutions of T^T r = e_0 and T^T r = e_{L-1}
// (T^T has c_{i-1} left of its diagonal and a_{i+1} right of it).
bool green_rows_general(const ld* a, const ld* b, const ld* c, int64_t L, double* first,
                        double* last) {
  std::vector<ld> cpv((size_t)L), r1((size_t)L), r2((size_t)L);
  ld u = b[0];
  if (u == 0.0L) return false;
  cpv[0] = L > 1 ? a[1] / u : 0.0L;
  r1[0] = 1.0L / u;
  r2[0] = L == 1 ? 1.0L / u : 0.0L;
  for (int64_t i = 1; i < L; ++i) {
    u = b[i] - c[i - 1] * cpv[i - 1];
    if (u == 0.0L) return false;
    cpv[i] = i + 1 < L ? a[i + 1] / u : 0.0L;
    r1[i] = (0.0L - c[i - 1] * r1[i - 1]) / u;
    r2[i] = ((i == L - 1 ? 1.0L : 0.0L) - c[i - 1] * r2[i - 1]) / u;
  }
  for (int64_t i = L - 2; i >= 0; --i) {
    r1[i] -= cpv[i] * r1[i + 1];
    r2[i] -= cpv[i] * r2[i + 1];
  }
  for (int64_t i = 0; i < L; ++i) {
    first[i] = (double)r1[i];
    last[i] = (double)r2[i];
    if (!std::isfinite(first[i]) || !std::isfinite(last[i])) return false;
  }
  return true;
}

template <typename Tc>
tdt_status_t build_general_dir(tdt_plan_s* p, int dir, double& dom, double& kap) {
  const int B = p->B, NT = p->NT;
  const int64_t L = p->L, N = p->N;
  const int64_t P = (N + L - 1) / L, Np = P * L;
  // rows of the matrix being solved: A (dir 0) or A^T (dir 1)
  std::vector<ld> a((size_t)Np, 0.0L), b((size_t)Np, 1.0L), c((size_t)Np, 0.0L);
  for (int64_t i = 0; i < N; ++i) {
    b[i] = p->in_gb[i];
    if (dir == 0) {
      a[i] = i > 0 ? p->in_ga[i] : 0.0;
      c[i] = i + 1 < N ? p->in_gc[i] : 0.0;
    } else {
      a[i] = i > 0 ? p->in_gc[i - 1] : 0.0;
      c[i] = i + 1 < N ? p->in_ga[i + 1] : 0.0;
    }
  }
  if (dir == 0) {
    // row dominance, and the 2-norm condition bound sqrt(kappa_1 kappa_inf)
    // from strict row and column dominance (infinite without it)
    double rmin = std::numeric_limits<double>::infinity();
    double rex = rmin, cex = rmin, rn = 0.0, cn = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      const double ai = std::fabs((double)a[i]), bi = std::fabs((double)b[i]);
      const double ci = std::fabs((double)c[i]);
      if (ai + ci > 0.0) rmin = std::min(rmin, bi / (ai + ci));
      // column i: c_{i-1} above the diagonal, a_{i+1} below
      const double up = i > 0 ? std::fabs((double)c[i - 1]) : 0.0;
      const double dn = i + 1 < N ? std::fabs((double)a[i + 1]) : 0.0;
      rex = std::min(rex, bi - ai - ci);
      cex = std::min(cex, bi - up - dn);
      rn = std::max(rn, bi + ai + ci);
      cn = std::max(cn, bi + up + dn);
    }
    dom = rmin;
    kap = (rex > 0.0 && cex > 0.0) ? std::sqrt((rn / rex) * (cn / cex))
                                   : std::numeric_limits<double>::infinity();
  }
  std::vector<Tc> row((size_t)P * tdt::kGenRowN * L), blk((size_t)P * tdt::kGenBlkN * NT);
  std::vector<double> tK((size_t)P * 4);
  // the tiles' Green rows (the first pass's summaries are their dot
  // products with the tile's F) and their supports: with several tiles,
  // all of them full (no tail to mask), the first pass reads the widest
  // supports over the tiles
  std::vector<double> green(P > 1 ? (size_t)P * 2 * L : 0);
  int64_t kfmax = 0, klmax = 0;
  for (int64_t t = 0; !green.empty() && t < P; ++t) {
    double* g1 = green.data() + (size_t)t * 2 * L;
    if (!green_rows_general(a.data() + t * L, b.data() + t * L, c.data() + t * L, L, g1,
                            g1 + L))
      return TDT_ERR_SINGULAR;
    std::vector<ld> r1(g1, g1 + L), r2(g1 + L, g1 + 2 * L);
    int64_t kf = 0, kl = 0;
    green_support(r1, r2, kf, kl);
    kfmax = std::max(kfmax, kf);
    klmax = std::max(klmax, kl);
  }
  int gkf = 0, gkl = 0;
  if (!green.empty() && N % L == 0) green_support_rounded(L, kfmax, klmax, gkf, gkl);
  p->gen_kf[dir] = gkf;
  p->gen_kl[dir] = gkl;
  if (gkf > 0) {
    // only the supports' entries: the head of the first row, the tail of the last
    std::vector<double> packed((size_t)P * (gkf + gkl));
    for (int64_t t = 0; t < P; ++t) {
      const double* g1 = green.data() + (size_t)t * 2 * L;
      double* o = packed.data() + (size_t)t * (gkf + gkl);
      std::copy(g1, g1 + gkf, o);
      std::copy(g1 + 2 * L - gkl, g1 + 2 * L, o + gkf);
    }
    green.swap(packed);
  } else if (sizeof(Tc) == 4) {
    green.clear();   // float plans sweep whole tiles: the rows would weigh as much as F
  }
  std::vector<ld> iu(B), aiu(B), cp(B), ph(B), ch(B);
  for (int64_t t = 0; t < P; ++t) {
    ld beta = 0.0L;
    SegLD tile{0, 0, 0, 0, 0, 0};
    for (int j = 0; j < NT; ++j) {
      const int64_t r0 = t * L + (int64_t)j * B;
      // block-local LU: u_0 = b, u_i = b_i - a_i c_{i-1}/u_{i-1}
      ld u = b[r0];
      for (int i = 0; i < B; ++i) {
        const int64_t r = r0 + i;
        if (i > 0) u = b[r] - a[r] * cp[i - 1];
        if (u == 0.0L) return TDT_ERR_SINGULAR;
        iu[i] = 1.0L / u;
        aiu[i] = a[r] * iu[i];
        cp[i] = c[r] * iu[i];
      }
      // responses to unit values just left (phi) and right (chi) of the block
      ph[0] = -aiu[0];
      for (int i = 1; i < B; ++i) ph[i] = -aiu[i] * ph[i - 1];
      for (int i = B - 2; i >= 0; --i) ph[i] -= cp[i] * ph[i + 1];
      for (int i = 0; i + 1 < B; ++i) ch[i] = 0.0L;
      ch[B - 1] = -cp[B - 1];
      for (int i = B - 2; i >= 0; --i) ch[i] -= cp[i] * ch[i + 1];
      const ld pf = ph[0], pl = ph[B - 1], cf = ch[0], cl = ch[B - 1];
      for (int i = 0; i < B; ++i) {
        Tc* rw = row.data() + (size_t)t * tdt::kGenRowN * L + (size_t)i * NT + j;
        rw[(size_t)tdt::kGenIU * L] = (Tc)iu[i];
        rw[(size_t)tdt::kGenAIU * L] = (Tc)aiu[i];
        rw[(size_t)tdt::kGenCP * L] = (Tc)cp[i];
        if (!std::isfinite((double)iu[i]) || !std::isfinite((double)cp[i]))
          return TDT_ERR_SINGULAR;
      }
      // in-tile left-to-right elimination across the blocks
      const ld den = 1.0L - pf * beta;
      if (!(std::fabs((double)den) > 1e-13)) return TDT_ERR_SINGULAR;
      const ld iD = 1.0L / den;
      Tc* bk = blk.data() + (size_t)t * tdt::kGenBlkN * NT + j;
      bk[(size_t)tdt::kGenPF * NT] = (Tc)pf;
      bk[(size_t)tdt::kGenPL * NT] = (Tc)pl;
      bk[(size_t)tdt::kGenCF * NT] = (Tc)cf;
      bk[(size_t)tdt::kGenBP * NT] = (Tc)beta;
      bk[(size_t)tdt::kGenID * NT] = (Tc)iD;
      beta = cl + pl * beta * cf * iD;
      if (!std::isfinite((double)beta)) return TDT_ERR_SINGULAR;
      // the tile's end values: its blocks merged left to right
      const SegLD s{0, 0, pf, pl, cf, cl};
      if (j == 0) {
        tile = s;
      } else {
        SegLD mrg;
        if (!merge_ld(tile, s, mrg)) return TDT_ERR_SINGULAR;
        tile = mrg;
      }
    }
    tK[4 * t + 0] = (double)tile.pf;
    tK[4 * t + 1] = (double)tile.pl;
    tK[4 * t + 2] = (double)tile.cf;
    tK[4 * t + 3] = (double)tile.cl;
  }
  // the system descriptor (the interface pass and the item geometry use it)
  SysDesc D;
  std::memset(&D, 0, sizeof(D));
  D.n = N;
  D.ntiles = (int32_t)P;
  D.stride = N;
  const int maxp = (int)P;
  D.tr = maxp <= 256 ? 1 : (maxp <= 2048 ? 8 : (maxp <= 16384 ? 16 : 1));
  D.tq = (D.ntiles + D.tr - 1) / D.tr;
  D.tslots = D.tq * D.tr;
  p->hsys[dir].assign(1, D);
  // interface pass across tiles: beta_{t-1}, 1/(1 - Pf_t beta_{t-1}) per tile
  p->ttab_n = std::max<int64_t>(D.tslots, 1);
  std::vector<double> tt(2 * (size_t)p->ttab_n, 0.0);
  if (P > 1) {
    ld beta = 0.0L;
    for (int64_t t = 0; t < P; ++t) {
      const double* K = tK.data() + 4 * t;
      const ld den = 1.0L - (ld)K[0] * beta;
      if (!(std::fabs((double)den) > 1e-13)) return TDT_ERR_SINGULAR;
      const ld iD = 1.0L / den;
      const int64_t pos = (t % D.tr) * D.tq + t / D.tr;
      tt[pos] = (double)beta;
      tt[p->ttab_n + pos] = (double)iD;
      beta = (ld)K[3] + (ld)K[1] * beta * (ld)K[2] * iD;
    }
  }
  tdt_status_t st = dev_upload(reinterpret_cast<Tc**>(&p->dgrow[dir]), row.data(), row.size());
  if (st == TDT_OK) st = dev_upload(reinterpret_cast<Tc**>(&p->dgblk[dir]), blk.data(), blk.size());
  if (st == TDT_OK) st = dev_upload(&p->dgtK[dir], tK.data(), tK.size());
  if (st == TDT_OK)
    st = dev_upload(reinterpret_cast<double**>(&p->dggreen[dir]), green.data(), green.size());
  if (st == TDT_OK) st = dev_upload(&p->dttab[dir], tt.data(), tt.size());
  if (st == TDT_OK) st = dev_upload(&p->dsys[dir], p->hsys[dir].data(), 1);
  return st;
}

tdt_status_t finish_general_plan(tdt_plan_s* p) {
  double dom = 0.0, kap = 0.0;
  for (int dir = 0; dir < 2; ++dir) {
    const tdt_status_t st = p->dtype == TDT_F32 ? build_general_dir<float>(p, dir, dom, kap)
                                                : build_general_dir<double>(p, dir, dom, kap);
    if (st != TDT_OK) return st;
  }
  p->dominance = dom;
  p->kappa = kap;
  {
    const tdt_status_t ws = ensure_workspace(p, 1, 1, nullptr);
    if (ws != TDT_OK) return ws;
  }
  if (hipMalloc(&p->iters, 2 * sizeof(int)) != hipSuccess) return TDT_ERR_OOM;
  if (hipMemset(p->iters, 0, 2 * sizeof(int)) != hipSuccess) return TDT_ERR_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  return p->dominance < 1.0 ? TDT_WARN_NOT_DOMINANT : TDT_OK;
}

bool overlaps(const void* x, size_t nx, const void* y, size_t ny) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(x), b = reinterpret_cast<uintptr_t>(y);
  return a < b + ny && b < a + nx;
}

size_t elem_size(tdt_dtype_t d) { return d == TDT_F32 ? sizeof(float) : sizeof(double); }

// Adjoint partial-sum slots of a series of M right-hand sides: one per tile,
// then two per right-hand side for the corner rows of a quasi-Toeplitz plan.
int64_t series_fslots(const tdt_plan_s* p, int64_t M) {
  return M * p->hsys[0][0].ntiles + (p->quasi ? 2 * M : 0);
}

// The launch set of a solve (everything but the workspace and the profile
// events) and the tile slots / adjoint partial-sum slots it needs.
tdt_status_t launch_set(tdt_plan_s* p, int dir, bool adjoint, int64_t M, tdt::LaunchSet& L,
                        int64_t& slots, int64_t& fslots) {
  L = tdt::LaunchSet{};
  L.ends_items = nullptr;
  L.n_ends = 0;
  L.gpack = nullptr;
  L.sys = p->dsys[dir];
  L.vec64 = p->dvec64[dir];
  L.vec32 = p->dvec32[dir];
  L.tab64 = p->dtab64[dir];
  L.tab32 = p->dtab32[dir];
  L.iters = p->iters;
  L.max_iter = p->max_iter;
  L.refine_tol = p->refine_tol;
  L.wg_per_cu = p->wg_per_cu;
  L.shape = p->shape;
  L.quasi = p->quasi ? 1 : 0;
  L.ttab = p->dttab[dir];
  L.ttab_n = p->ttab_n;
  L.max_ntiles = 1;
  for (const SysDesc& D : p->hsys[0]) L.max_ntiles = std::max(L.max_ntiles, (int)D.ntiles);
  L.chunks = p->chunks ? 1 : 0;
  L.general = p->general ? 1 : 0;
  L.gen_row = p->dgrow[dir];
  L.gen_blk = p->dgblk[dir];
  L.gen_tK = p->dgtK[dir];
  L.gen_M = M;
  if (p->general) {
    const SysDesc& D0 = p->hsys[0][0];
    const int64_t nt = D0.ntiles;
    L.green = nullptr;
    L.green_kf = L.green_kl = 0;
    L.gen_green = p->dggreen[dir];
    L.gen_kf = p->gen_kf[dir];
    L.gen_kl = p->gen_kl[dir];
    L.p1_items = L.fin_items = nullptr;
    L.grid_items = L.sys_items = L.sys_bins = nullptr;
    L.n_bins = L.n_sys = 0;
    L.n_beta = L.n_last = 0;
    L.nfull = 0;
    // right-hand sides per item: up to 8 share one load of a tile's
    // constants, as long as at least 4 items per compute unit remain
    int R = (int)std::min<int64_t>(M, 8);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    while (R > 1 && nt * ((M + R - 1) / R) < 4 * (int64_t)cus) --R;
    L.gen_R = R;
    const int64_t groups = (M + R - 1) / R;
    L.n_p1 = nt > 1 ? groups * nt : 0;
    L.n_grid = nt > 1 ? M : 0;
    L.n_fin = groups * nt;
    L.corner0 = 0;
    slots = nt > 1 ? M * D0.tslots : 0;
    fslots = 0;
  } else if (p->varlen) {
    L.green = nullptr;
    L.green_kf = L.green_kl = 0;
    L.n_beta = L.n_last = 0;
    L.nfull = 0;
    const tdt_plan_s::Lists& q = p->lists[dir];
    L.p1_items = q.p1;
    L.fin_items = q.fin;
    L.grid_items = q.grid;
    L.sys_items = q.whole;
    L.sys_bins = q.bins;
    L.n_bins = q.n_bins;
    L.n_p1 = q.n_p1;
    L.n_fin = q.n_fin;
    L.n_grid = q.n_grid;
    L.n_sys = q.n_whole;
    L.ends_items = q.n_ends > 0 ? q.ends : nullptr;
    L.n_ends = q.n_ends;
    L.gpack = p->dgpack[dir];
    slots = p->vslots;
    fslots = adjoint ? p->vfslots : 0;
    L.corner0 = 0;
  } else {
    const SysDesc& D0 = p->hsys[0][0];
    const int64_t nt = D0.ntiles;
    const bool itf = needs_interface(D0);
    L.p1_items = nullptr;
    L.fin_items = nullptr;
    L.grid_items = nullptr;
    L.sys_items = nullptr;
    L.sys_bins = nullptr;
    L.n_bins = 0;
    L.n_sys = 0;
    L.green = p->dgreen[dir];
    L.green_kf = p->green_kf[dir];
    L.green_kl = p->green_kl[dir];
    L.nfull = (int)(D0.n % p->L == 0 ? nt : nt - 1);
    L.n_beta = itf ? M * L.nfull : 0;
    L.n_last = (itf && D0.n % p->L != 0) ? M : 0;
    L.n_p1 = itf ? M * nt : 0;
    L.n_grid = itf ? M : 0;
    L.n_fin = M * nt;
    slots = itf ? M * D0.tslots : 0;
    fslots = adjoint ? series_fslots(p, M) : 0;
    L.corner0 = M * nt;
  }
  if (L.n_fin > 0x7fffffffLL) return TDT_ERR_INVALID_ARG;
  return TDT_OK;
}

tdt_status_t run(tdt_plan_s* p, int dir, const void* F, void* X, const void* Xfwd, int64_t M,
                 hipStream_t st) {
  tdt::LaunchSet L;
  int64_t slots = 0, fslots = 0;
  tdt_status_t s = launch_set(p, dir, Xfwd != nullptr, M, L, slots, fslots);
  if (s != TDT_OK) return s;
  s = ensure_workspace(p, slots, fslots, st);
  if (s != TDT_OK) return s;
  if (!p->summ || !p->ghost || !p->gscr || !p->gpart) return TDT_ERR_OOM;
  L.summ = p->summ;
  L.ghost = p->ghost;
  L.gscr = p->gscr;
  L.gpart = p->gpart;
  L.ev = nullptr;
  if (p->profile) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      const size_t k = p->prof_ev.size();
      p->prof_ev.resize(k + 4);
      for (size_t j = 0; j < 4; ++j)
        if (hipEventCreate(&p->prof_ev[k + j]) != hipSuccess) return TDT_ERR_HIP;
      L.ev = p->prof_ev.data() + k;
    }
  }
  if (tdt::launch_solve((int)p->dtype, Xfwd != nullptr, L, F, X, Xfwd, st) != hipSuccess)
    return TDT_ERR_HIP;
  return TDT_OK;
}

}  // namespace

namespace tdt {
// The checks of tdt_solve and its launch set, for the entry point whose
// workspace is the library's static device scratch (tdt_solve_noalloc).
int series_solve_prepare(tdt_plan_s* p, const void* F, void* X, int64_t M, LaunchSet& L,
                         int64_t& slots, int& dtype) {
  if (!p || p->varlen || p->strided || !F || !X || M < 1) return TDT_ERR_INVALID_ARG;
  const size_t bytes = (size_t)M * (size_t)p->N * elem_size(p->dtype);
  if (overlaps(F, bytes, X, bytes)) return TDT_ERR_INVALID_ARG;
  int64_t fslots = 0;
  dtype = (int)p->dtype;
  return launch_set(p, 0, false, M, L, slots, fslots);
}
}  // namespace tdt


// Tables of a strided batch (systems along a slow axis, one workgroup per
// column of adjacent systems): per class the block LU pivots, the end values
// of a full block and of the last block, and the left-to-right interface
// table over the C block positions of a column (beta_{c-1} and
// 1/(1 - phi_first(c) beta_{c-1}), each block with its own end values).
namespace tdt {
int strided_tables(int64_t N, int64_t P, const double* tm1, const double* t0, const double* t1,
                   double* iu, double* sc, double* pos, double* dominance) {
  if (N < 1 || N > (int64_t)kStrMaxChunks * kStrB || P < 1 || !tm1 || !t0 || !t1)
    return TDT_ERR_INVALID_ARG;
  const int C = strided_chunks(N);
  const int bt = (int)(N - (int64_t)(C - 1) * kStrB);
  double dom = std::numeric_limits<double>::infinity();
  ld iuv[kStrB], cp[kStrB], phi[kStrB], chi[kStrB];
  for (int64_t k = 0; k < P; ++k) {
    const double a = tm1[k], b = t0[k], c = t1[k];
    if (!finite3(a, b, c)) return TDT_ERR_INVALID_ARG;
    dom = std::min(dom, dominance_ratio(a, b, c));
    if (!block_vectors(a, b, c, kStrB, iuv, cp, phi, chi)) return TDT_ERR_SINGULAR;
    for (int i = 0; i < kStrB; ++i) {
      iu[(int64_t)i * P + k] = (double)iuv[i];
      if (!std::isfinite(iu[(int64_t)i * P + k])) return TDT_ERR_SINGULAR;
    }
    const ld full[4] = {phi[0], phi[kStrB - 1], chi[0], chi[kStrB - 1]};
    ld tail[4];
    if (bt == kStrB) {
      for (int e = 0; e < 4; ++e) tail[e] = full[e];
    } else if (!segment_ends(a, b, c, bt, tail)) {
      return TDT_ERR_SINGULAR;
    }
    sc[kStrTM1 * P + k] = a;
    sc[kStrT1 * P + k] = c;
    sc[kStrPF * P + k] = (double)full[0];
    sc[kStrPL * P + k] = (double)full[1];
    sc[kStrCF * P + k] = (double)full[2];
    sc[kStrTPF * P + k] = (double)tail[0];
    sc[kStrTPL * P + k] = (double)tail[1];
    sc[kStrTCF * P + k] = (double)tail[2];
    ld beta = 0.0L;
    for (int m = 0; m < C; ++m) {
      const ld* e = m == C - 1 ? tail : full;
      const ld D = 1.0L - e[0] * beta;
      if (!(std::fabs((double)D) > 1e-13)) return TDT_ERR_SINGULAR;
      const ld iD = 1.0L / D;
      pos[(int64_t)m * P + k] = (double)beta;
      pos[((int64_t)C + m) * P + k] = (double)iD;
      beta = e[3] + e[1] * e[2] * beta * iD;
      if (!std::isfinite((double)beta)) return TDT_ERR_SINGULAR;
    }
  }
  if (dominance) *dominance = dom;
  return TDT_OK;
}

StridedTiles strided_tiles(int64_t N, int64_t P) {
  StridedTiles g{};
  // one column up to kStrMaxChunks blocks, tiles of kStrTile rows beyond
  g.K = N > (int64_t)kStrMaxChunks * kStrB ? (N + kStrTile - 1) / kStrTile : 1;
  g.NL = N - (g.K - 1) * kStrTile;
  g.C = strided_chunks(g.K > 1 ? kStrTile : N);
  g.CL = strided_chunks(g.NL);
  g.n_full = (int64_t)(kStrB + kStrScalarN + 2 * g.C) * P;
  g.n_last = (int64_t)(kStrB + kStrScalarN + 2 * g.CL) * P;
  g.n_ends = (int64_t)kTileEndN * P;
  return g;
}

// Tables of a system in tiles: a full tile's and the last tile's column
// tables, and per class the end values (phi_f, phi_l, chi_f, chi_l) of both
// tile lengths.  The pivots D_m = 1 - phi_f s_{m-1} of the tiles'
// elimination depend on the class only and are checked here; s_m settles
// quickly, so the full tiles stop at its fixed point.
int strided_tiled_tables(int64_t N, int64_t P, const double* tm1, const double* t0,
                         const double* t1, double* out, double* dominance) {
  const StridedTiles g = strided_tiles(N, P);
  if (g.K < 2) return TDT_ERR_INVALID_ARG;
  auto tables = [&](int64_t n, double* t) {
    double* iu = t;
    double* sc = iu + (int64_t)kStrB * P;
    double* pos = sc + (int64_t)kStrScalarN * P;
    return strided_tables(n, P, tm1, t0, t1, iu, sc, pos, dominance);
  };
  int st = tables(kStrTile, out);
  if (st < 0) return st;
  st = tables(g.NL, out + g.n_full);
  if (st < 0) return st;
  double* ends = out + g.n_full + g.n_last;
  for (int64_t k = 0; k < P; ++k) {
    ld full[4], lastv[4];
    if (!segment_ends(tm1[k], t0[k], t1[k], kStrTile, full) ||
        !segment_ends(tm1[k], t0[k], t1[k], g.NL, lastv))
      return TDT_ERR_SINGULAR;
    for (int e = 0; e < 4; ++e) {
      ends[(int64_t)e * P + k] = (double)full[e];
      ends[(int64_t)(4 + e) * P + k] = (double)lastv[e];
    }
    ld sv = 0.0L;
    for (int64_t m = 0; m < g.K; ++m) {
      const ld* e = m == g.K - 1 ? lastv : full;
      const ld D = 1.0L - e[0] * sv;
      if (!(std::fabs((double)D) > 1e-13)) return TDT_ERR_SINGULAR;
      const ld sn = e[1] * sv * e[2] / D + e[3];
      if (!std::isfinite((double)sn)) return TDT_ERR_SINGULAR;
      if (m < g.K - 2 && sn == sv) m = g.K - 2;   // the full tiles left repeat it
      sv = sn;
    }
  }
  return TDT_OK;
}
}  // namespace tdt

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// Autotuner support: choice record, cache key, JSON cache file.
namespace tune {

struct Choice {
  int shape;
  int whole_max_tiles;
  int wg_per_cu;
  double ms;
};

int64_t pow2_ceil(int64_t v) {
  int64_t r = 1;
  while (r < v) r <<= 1;
  return r;
}

std::string key_of(const tdt_plan_s* p, int64_t M) {
  int dev = 0, cus = 0;
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  const char* dt = p->dtype == TDT_F64 ? "f64" : (p->dtype == TDT_F32 ? "f32" : "f32_refine");
  const char* kind = p->quasi ? "q" : (p->general ? "g" : "");
  // (the leading version tag changes when the meaning of a choice does)
  char buf[256];
  if (p->varlen) {
    int maxt = 1;
    for (const SysDesc& D : p->hsys[0]) maxt = std::max(maxt, (int)D.ntiles);
    std::snprintf(buf, sizeof(buf), "v2|%s|cu%d|varlen%s|%s|S%lld|U%lld|P%lld", arch.c_str(), cus,
                  kind, dt,
                  (long long)pow2_ceil(p->S), (long long)pow2_ceil(p->total),
                  (long long)pow2_ceil(maxt));
  } else {
    std::snprintf(buf, sizeof(buf), "v2|%s|cu%d|series%s|%s|N%lld|M%lld", arch.c_str(), cus, kind,
                  dt,
                  (long long)pow2_ceil(p->N), (long long)pow2_ceil(M));
  }
  return buf;
}

std::string cache_path() {
  if (const char* e = std::getenv("TDT_TUNE_CACHE")) return e;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : ".") + "/.cache/tdt/autotune.json";
}

// The file holds one entry per line:
//   "key": {"shape": S, "whole_max_tiles": W, "wg_per_cu": C, "ms": T},
// inside {"format": "tdt-autotune-1", "entries": { ... }}.
std::vector<std::pair<std::string, Choice>> read_all() {
  std::vector<std::pair<std::string, Choice>> out;
  FILE* f = std::fopen(cache_path().c_str(), "r");
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    const char* b = std::strstr(q1, "{\"shape\":");
    if (!b) continue;
    Choice c{0, 0, 0, 0.0};
    if (std::sscanf(b, "{\"shape\": %d, \"whole_max_tiles\": %d, \"wg_per_cu\": %d, \"ms\": %lf",
                    &c.shape, &c.whole_max_tiles, &c.wg_per_cu, &c.ms) == 4 &&
        c.shape >= 0 && c.shape < tdt::kNumShapes)
      out.emplace_back(std::string(q0 + 1, q1), c);
  }
  std::fclose(f);
  return out;
}

bool lookup(const std::string& key, Choice& c) {
  for (const auto& e : read_all())
    if (e.first == key) {
      c = e.second;
      return true;
    }
  return false;
}

void store(const std::string& key, const Choice& c) {
  auto all = read_all();
  bool found = false;
  for (auto& e : all)
    if (e.first == key) {
      e.second = c;
      found = true;
    }
  if (!found) all.emplace_back(key, c);
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directories on the way (best effort)
    for (size_t i = 1; i <= slash; ++i)
      if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\"format\": \"tdt-autotune-1\", \"entries\": {\n");
  for (size_t i = 0; i < all.size(); ++i)
    std::fprintf(f,
                 "  \"%s\": {\"shape\": %d, \"whole_max_tiles\": %d, \"wg_per_cu\": %d, "
                 "\"ms\": %.6f}%s\n",
                 all[i].first.c_str(), all[i].second.shape, all[i].second.whole_max_tiles,
                 all[i].second.wg_per_cu, all[i].second.ms, i + 1 < all.size() ? "," : "");
  std::fprintf(f, "}}\n");
  std::fclose(f);
  (void)std::rename(tmp.c_str(), path.c_str());
}

tdt_status_t apply(tdt_plan_s* p, const Choice& c) {
  tdt_status_t st = tdt_plan_set_option(p, TDT_OPT_SHAPE, c.shape);
  if (st == TDT_OK) st = tdt_plan_set_option(p, TDT_OPT_WG_PER_CU, c.wg_per_cu);
  if (st == TDT_OK && p->varlen)
    st = tdt_plan_set_option(p, TDT_OPT_WHOLE_MAX_TILES, c.whole_max_tiles);
  return st;
}

}  // namespace tune

namespace {

bool valid_dtype(tdt_dtype_t d) { return d == TDT_F64 || d == TDT_F32 || d == TDT_F32_REFINE; }

// One system (or a series sharing it); psi/chi non-null: quasi-Toeplitz.
tdt_status_t create_series(double t_m1, double t_0, double t_1, const double* psi,
                           const double* chi, int64_t N, tdt_dtype_t dtype, tdt_plan_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  const bool quasi = psi != nullptr;
  if (N < (quasi ? 3 : 1) || N > ((int64_t)1 << 40) || !finite3(t_m1, t_0, t_1) ||
      !valid_dtype(dtype) || (quasi && !(std::isfinite(*psi) && std::isfinite(*chi))))
    return TDT_ERR_INVALID_ARG;
  tdt_plan_s* p = new (std::nothrow) tdt_plan_s();
  if (!p) return TDT_ERR_OOM;
  p->dtype = dtype;
  p->N = N;
  p->S = 1;
  p->in_tm1 = {t_m1};
  p->in_t0 = {t_0};
  p->in_t1 = {t_1};
  p->in_sizes = {N};
  p->in_offs = {0};
  if (quasi) {
    p->quasi = true;
    p->in_psi = {*psi};
    p->in_chi = {*chi};
  }
  tdt_status_t st = finish_plan(p, p->in_tm1, p->in_t0, p->in_t1, p->in_sizes, p->in_offs);
  if (st < 0) {
    destroy(p);
    return st;
  }
  *out = p;
  return st;
}

// Packed systems of their own sizes; h_psi/h_chi non-null: quasi-Toeplitz.
tdt_status_t create_varlen(int64_t S, const int64_t* h_offsets, const double* h_tm1,
                           const double* h_t0, const double* h_t1, const double* h_psi,
                           const double* h_chi, tdt_dtype_t dtype, tdt_plan_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  const bool quasi = h_psi != nullptr;
  if (S < 1 || S > 0x7fffffffLL || !h_offsets || !h_tm1 || !h_t0 || !h_t1 ||
      !valid_dtype(dtype) || h_offsets[0] != 0)
    return TDT_ERR_INVALID_ARG;
  std::vector<int64_t> sizes((size_t)S), offs((size_t)S);
  std::vector<double> tm1(h_tm1, h_tm1 + S), t0(h_t0, h_t0 + S), t1(h_t1, h_t1 + S);
  for (int64_t s = 0; s < S; ++s) {
    sizes[s] = h_offsets[s + 1] - h_offsets[s];
    offs[s] = h_offsets[s];
    if (sizes[s] < (quasi ? 3 : 1) || !finite3(tm1[s], t0[s], t1[s]) ||
        (quasi && !(std::isfinite(h_psi[s]) && std::isfinite(h_chi[s]))))
      return TDT_ERR_INVALID_ARG;
  }
  tdt_plan_s* p = new (std::nothrow) tdt_plan_s();
  if (!p) return TDT_ERR_OOM;
  p->varlen = true;
  p->dtype = dtype;
  p->S = S;
  p->total = h_offsets[S];
  p->in_tm1 = tm1;
  p->in_t0 = t0;
  p->in_t1 = t1;
  p->in_sizes = sizes;
  p->in_offs = offs;
  if (quasi) {
    p->quasi = true;
    p->in_psi.assign(h_psi, h_psi + S);
    p->in_chi.assign(h_chi, h_chi + S);
  }
  tdt_status_t st = finish_plan(p, tm1, t0, t1, sizes, offs);
  if (st < 0) {
    destroy(p);
    return st;
  }
  *out = p;
  return st;
}

}  // namespace

extern "C" {

const char* tdt_status_string(tdt_status_t s) {
  switch (s) {
    case TDT_OK: return "ok";
    case TDT_WARN_NOT_DOMINANT: return "solved; matrix not diagonally dominant";
    case TDT_ERR_INVALID_ARG: return "invalid argument";
    case TDT_ERR_SINGULAR: return "singular matrix or sub-block";
    case TDT_ERR_HIP: return "HIP runtime error";
    case TDT_ERR_OOM: return "out of memory";
    case TDT_ERR_NOT_CONVERGED: return "refinement did not converge";
    case TDT_ERR_CAPTURE: return "allocation needed during stream capture";
  }
  return "unknown status";
}

tdt_status_t tdt_plan_create(double t_m1, double t_0, double t_1, int64_t N, tdt_dtype_t dtype,
                             tdt_plan_t* out) {
  return create_series(t_m1, t_0, t_1, nullptr, nullptr, N, dtype, out);
}

tdt_status_t tdt_plan_quasi_create(double t_m1, double t_0, double t_1, double psi, double chi,
                                   int64_t N, tdt_dtype_t dtype, tdt_plan_t* out) {
  return create_series(t_m1, t_0, t_1, &psi, &chi, N, dtype, out);
}

tdt_status_t tdt_plan_varlen_create(int64_t S, const int64_t* h_offsets, const double* h_tm1,
                                    const double* h_t0, const double* h_t1, tdt_dtype_t dtype,
                                    tdt_plan_t* out) {
  return create_varlen(S, h_offsets, h_tm1, h_t0, h_t1, nullptr, nullptr, dtype, out);
}

tdt_status_t tdt_plan_general_create(int64_t N, const double* h_a, const double* h_b,
                                     const double* h_c, tdt_dtype_t dtype, tdt_plan_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  if (N < 1 || N > ((int64_t)1 << 40) || !h_a || !h_b || !h_c ||
      (dtype != TDT_F64 && dtype != TDT_F32))
    return TDT_ERR_INVALID_ARG;
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(h_b[i]) || (i > 0 && !std::isfinite(h_a[i])) ||
        (i + 1 < N && !std::isfinite(h_c[i])))
      return TDT_ERR_INVALID_ARG;
  tdt_plan_s* p = new (std::nothrow) tdt_plan_s();
  if (!p) return TDT_ERR_OOM;
  p->general = true;
  p->dtype = dtype;
  p->N = N;
  p->S = 1;
  p->shape = tdt::kGeneralShape;
  p->B = tdt::kShapes[p->shape].B;
  p->NT = tdt::kShapes[p->shape].NT;
  p->L = (int64_t)p->B * p->NT;
  p->in_ga.assign(h_a, h_a + N);
  p->in_gb.assign(h_b, h_b + N);
  p->in_gc.assign(h_c, h_c + N);
  tdt_status_t st = finish_general_plan(p);
  if (st < 0) {
    destroy(p);
    return st;
  }
  *out = p;
  return st;
}

tdt_status_t tdt_plan_strided_create(int64_t N, int64_t P, const double* h_tm1,
                                     const double* h_t0, const double* h_t1, tdt_dtype_t dtype,
                                     tdt_plan_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  if (N < 1 || N > tdt::kStrMaxN || P < 1 || P > ((int64_t)1 << 31) || !h_tm1 || !h_t0 ||
      !h_t1 || dtype != TDT_F64)
    return TDT_ERR_INVALID_ARG;
  // one column, or tiles of kStrTile rows and a shorter last tile
  const tdt::StridedTiles g = tdt::strided_tiles(N, P);
  const int64_t K = g.K;
  const int C = g.C;
  const int64_t n1 = g.n_full, n2 = K > 1 ? g.n_last : 0, n3 = K > 1 ? g.n_ends : 0;
  std::vector<double> tab;
  try {
    tab.resize((size_t)(n1 + n2 + n3));
  } catch (const std::exception&) {   // P too large for the host tables
    return TDT_ERR_OOM;
  }
  double dom = 0.0;
  const int st =
      K > 1 ? tdt::strided_tiled_tables(N, P, h_tm1, h_t0, h_t1, tab.data(), &dom)
            : tdt::strided_tables(N, P, h_tm1, h_t0, h_t1, tab.data(),
                                  tab.data() + (int64_t)tdt::kStrB * P,
                                  tab.data() + (int64_t)(tdt::kStrB + tdt::kStrScalarN) * P, &dom);
  if (st < 0) return (tdt_status_t)st;
  tdt_plan_s* p = new (std::nothrow) tdt_plan_s();
  if (!p) return TDT_ERR_OOM;
  p->strided = true;
  p->dtype = dtype;
  p->N = N;
  p->S = P;
  p->sP = P;
  p->sC = C;
  p->sK = K;
  p->dominance = dom;
  p->kappa = 0.0;
  tdt_status_t s2 = dev_upload(&p->dstr, tab.data(), tab.size());
  if (s2 != TDT_OK) {
    destroy(p);
    return s2;
  }
  *out = p;
  return dom < 1.0 ? TDT_WARN_NOT_DOMINANT : TDT_OK;
}

tdt_status_t tdt_solve_strided(tdt_plan_t p, const double* F, double* X, int64_t M, int64_t ld,
                               int64_t nb, int64_t ldb, hipStream_t stream) {
  if (!p || !p->strided || !F || !X || M < 1 || M > p->sP || nb < 1 || ld < 1 || ldb < 0)
    return TDT_ERR_INVALID_ARG;
  const int64_t N = p->N;
  // the two layouts whose addresses b*ldb + i*ld + s are all distinct: batches
  // one after the other, or batches interleaved inside each row
  const bool outer = ld >= M && (nb == 1 || ldb >= (N - 1) * ld + M);
  const bool inner = ldb >= M && ld >= (nb - 1) * ldb + M;
  if (!outer && !inner) return TDT_ERR_INVALID_ARG;
  const int64_t extent = (nb - 1) * ldb + (N - 1) * ld + M;
  const size_t bytes = (size_t)extent * sizeof(double);
  if (F != X && overlaps(F, bytes, X, bytes)) return TDT_ERR_INVALID_ARG;
  const int64_t K = p->sK;
  if (K > 1) {
    // the tiles' end values and outside values, [nb][K][2][M] each
    const tdt_status_t ws = ensure_workspace(p, nb * K * M, 0, stream);
    if (ws != TDT_OK) return ws;
  }
  tdt::StridedArgs a{};
  auto set_tables = [&](const double* t) {
    a.iu = t;
    a.sc = a.iu + (int64_t)tdt::kStrB * p->sP;
    a.pos = a.sc + (int64_t)tdt::kStrScalarN * p->sP;
  };
  a.R = F;
  a.O = X;
  a.G = nullptr;
  a.epi = nullptr;
  set_tables(p->dstr);
  a.N = K > 1 ? tdt::kStrTile : N;
  a.P = p->sP;
  a.M = M;
  a.Mg = M;
  a.ld = ld;
  a.nb = nb;
  a.ldb = ldb;
  a.C = p->sC;
  hipEvent_t* ev = nullptr;
  if (p->profile) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      const size_t k = p->prof_ev.size();
      p->prof_ev.resize(k + 4);
      for (size_t j = 0; j < 4; ++j)
        if (hipEventCreate(&p->prof_ev[k + j]) != hipSuccess) return TDT_ERR_HIP;
      ev = p->prof_ev.data() + k;
      for (int j = 0; j < 3; ++j) (void)hipEventRecord(ev[j], stream);
    }
  }
  if (K == 1) {
    if (tdt::launch_strided(a, stream) != hipSuccess) return TDT_ERR_HIP;
  } else {
    // pass 1 and pass 2 over the full tiles, then over the last one
    if (tdt::launch_strided_tiled(a, tdt::strided_tiles(N, p->sP), p->dstr, p->summ, p->ghost,
                                  stream) != hipSuccess)
      return TDT_ERR_HIP;
  }
  if (ev) (void)hipEventRecord(ev[3], stream);
  return TDT_OK;
}

tdt_status_t tdt_plan_varlen_quasi_create(int64_t S, const int64_t* h_offsets,
                                          const double* h_tm1, const double* h_t0,
                                          const double* h_t1, const double* h_psi,
                                          const double* h_chi, tdt_dtype_t dtype,
                                          tdt_plan_t* out) {
  if (!h_psi || !h_chi) {
    if (out) *out = nullptr;
    return TDT_ERR_INVALID_ARG;
  }
  return create_varlen(S, h_offsets, h_tm1, h_t0, h_t1, h_psi, h_chi, dtype, out);
}

tdt_status_t tdt_plan_reserve(tdt_plan_t p, int64_t M_max) {
  if (!p || M_max < 1) return TDT_ERR_INVALID_ARG;
  if (p->strided)   // workspace only for systems of several tiles
    return p->sK > 1 ? ensure_workspace(p, M_max * p->sK, 0, nullptr) : TDT_OK;
  p->reserved_M = std::max(p->reserved_M, M_max);
  int64_t slots, fslots;
  if (p->general) {
    slots = p->hsys[0][0].ntiles > 1 ? M_max * p->hsys[0][0].tslots : 0;
    fslots = 0;
  } else if (p->varlen) {
    slots = p->vslots;
    fslots = p->vfslots;
  } else {
    slots = needs_interface(p->hsys[0][0]) ? M_max * p->hsys[0][0].tslots : 0;
    fslots = series_fslots(p, M_max);
  }
  return ensure_workspace(p, slots, fslots, nullptr);
}

tdt_status_t tdt_solve(tdt_plan_t p, const void* F, void* X, int64_t M, hipStream_t stream) {
  if (!p || p->varlen || p->strided || !F || !X || M < 1) return TDT_ERR_INVALID_ARG;
  const size_t bytes = (size_t)M * (size_t)p->N * elem_size(p->dtype);
  if (overlaps(F, bytes, X, bytes)) return TDT_ERR_INVALID_ARG;
  return run(p, 0, F, X, nullptr, M, stream);
}

tdt_status_t tdt_solve_varlen(tdt_plan_t p, const void* F, void* X, hipStream_t stream) {
  if (!p || !p->varlen || p->strided || !F || !X) return TDT_ERR_INVALID_ARG;
  const size_t bytes = (size_t)p->total * elem_size(p->dtype);
  if (overlaps(F, bytes, X, bytes)) return TDT_ERR_INVALID_ARG;
  return run(p, 0, F, X, nullptr, 1, stream);
}

tdt_status_t tdt_solve_backward(tdt_plan_t p, const void* gX, const void* X, void* gF,
                                double* d_gt, int64_t M, hipStream_t stream) {
  if (!p || p->strided || !gX || !X || !gF) return TDT_ERR_INVALID_ARG;
  if (p->varlen) M = 1;
  if (M < 1) return TDT_ERR_INVALID_ARG;
  const size_t bytes =
      (size_t)(p->varlen ? p->total : M * p->N) * elem_size(p->dtype);
  if (overlaps(gF, bytes, gX, bytes) || overlaps(gF, bytes, X, bytes)) return TDT_ERR_INVALID_ARG;
  if (p->general) {
    // gF = A^{-T} gX, then the entry gradients from gF and X
    tdt_status_t st = run(p, 1, gX, gF, nullptr, M, stream);
    if (st != TDT_OK) return st;
    if (d_gt && tdt::launch_general_grad(p->dtype == TDT_F32 ? 1 : 0, gF, X, p->N, M, d_gt,
                                         stream) != hipSuccess)
      return TDT_ERR_HIP;
    return TDT_OK;
  }
  tdt_status_t st = run(p, 1, gX, gF, X, M, stream);
  if (st != TDT_OK) return st;
  if (d_gt) {
    const int64_t nparts = p->varlen ? p->vfslots : series_fslots(p, M);
    if (tdt::launch_gt_reduce(p->gpart, p->dsys[1], p->S, nparts, p->varlen ? 1 : 0,
                              p->quasi ? tdt::kGradN : 3, d_gt, stream) != hipSuccess)
      return TDT_ERR_HIP;
  }
  return TDT_OK;
}

tdt_status_t tdt_plan_destroy(tdt_plan_t p) {
  if (!p) return TDT_ERR_INVALID_ARG;
  destroy(p);
  return TDT_OK;
}

tdt_status_t tdt_last_info(tdt_plan_t p, int* n_refine_iters, double* last_rel_update,
                           double* dominance, double* kappa2) {
  if (!p) return TDT_ERR_INVALID_ARG;
  if (dominance) *dominance = p->dominance;
  if (kappa2) *kappa2 = p->kappa;
  if (!n_refine_iters && !last_rel_update) return TDT_OK;
  if (!p->iters) {   // no refinement in this kind of plan
    if (n_refine_iters) *n_refine_iters = 0;
    if (last_rel_update) *last_rel_update = 0.0;
    return TDT_OK;
  }
  int v[2] = {0, 0};
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(v, p->iters, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(p->iters, 0, sizeof(v)) != hipSuccess)
    return TDT_ERR_HIP;
  float rel;
  std::memcpy(&rel, &v[1], sizeof(rel));
  if (n_refine_iters) *n_refine_iters = v[0];
  if (last_rel_update) *last_rel_update = (double)rel;
  // refinement stopped (cap, or updates no longer shrinking) while its
  // remaining error was still above float resolution relative to the solution
  if (p->dtype == TDT_F32_REFINE && v[0] > 0 && !(rel <= kNotConvergedRel))
    return TDT_ERR_NOT_CONVERGED;
  return TDT_OK;
}

tdt_status_t tdt_plan_set_option(tdt_plan_t p, tdt_option_t opt, int64_t value) {
  if (!p || p->strided) return TDT_ERR_INVALID_ARG;
  switch (opt) {
    case TDT_OPT_WHOLE_MAX_TILES: {
      if (!p->varlen || value < 0 || value > tdt::kSysMaxTiles) return TDT_ERR_INVALID_ARG;
      if ((int)value == p->sys_max_tiles) return TDT_OK;
      if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
      p->sys_max_tiles = (int)value;
      return build_varlen_lists(p);
    }
    case TDT_OPT_WG_PER_CU:
      if (value < 0 || value > 64) return TDT_ERR_INVALID_ARG;
      if ((int)value == p->wg_per_cu) return TDT_OK;
      p->wg_per_cu = (int)value;
      if (!p->varlen) return TDT_OK;
      if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
      return build_varlen_lists(p);   // the whole-system lists follow the grid
    case TDT_OPT_MAX_REFINE:
      if (value < 1 || value > 100) return TDT_ERR_INVALID_ARG;
      p->max_iter = (int)value;
      return TDT_OK;
    case TDT_OPT_SHAPE:
      if (value < 0 || value >= tdt::kNumShapes) return TDT_ERR_INVALID_ARG;
      if ((int)value == p->shape) return TDT_OK;
      if (p->general) return TDT_ERR_INVALID_ARG;   // built for kGeneralShape only
      return rebuild_plan(p, (int)value);
  }
  return TDT_ERR_INVALID_ARG;
}

tdt_status_t tdt_plan_get_option(tdt_plan_t p, tdt_option_t opt, int64_t* value) {
  if (!p || !value) return TDT_ERR_INVALID_ARG;
  switch (opt) {
    case TDT_OPT_WHOLE_MAX_TILES: *value = p->sys_max_tiles; return TDT_OK;
    case TDT_OPT_WG_PER_CU: *value = p->wg_per_cu; return TDT_OK;
    case TDT_OPT_MAX_REFINE: *value = p->max_iter; return TDT_OK;
    case TDT_OPT_SHAPE: *value = p->shape; return TDT_OK;
  }
  return TDT_ERR_INVALID_ARG;
}

tdt_status_t tdt_plan_autotune(tdt_plan_t p, const void* F, void* X, int64_t M,
                               hipStream_t stream, int flags, double* best_ms) {
  if (best_ms) *best_ms = 0.0;
  if (!p || p->strided || !F || !X) return TDT_ERR_INVALID_ARG;
  if (p->varlen) M = 1;
  if (M < 1) return TDT_ERR_INVALID_ARG;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return TDT_ERR_CAPTURE;
  const bool adjoint = (flags & TDT_TUNE_ADJOINT) != 0;
  const std::string key = tune::key_of(p, M) + (adjoint ? "|adj" : "");
  const bool use_cache = !(flags & TDT_TUNE_NO_CACHE);
  if (use_cache && !(flags & TDT_TUNE_FORCE)) {
    tune::Choice c;
    if (tune::lookup(key, c)) return tune::apply(p, c);
  }
  // with the adjoint, each trial also runs tdt_solve_backward (gX = F, the
  // forward solution X) into buffers of the tuner's own
  void* gF = nullptr;
  double* gt = nullptr;
  if (adjoint) {
    const size_t n = (size_t)(p->varlen ? p->total : M * p->N);
    if (hipMalloc(&gF, n * elem_size(p->dtype)) != hipSuccess) return TDT_ERR_OOM;
    if (hipMalloc(reinterpret_cast<void**>(&gt), (size_t)p->S * tdt::kGradN * sizeof(double) +
                                                     (p->general ? 3 * (size_t)p->N * 8 : 0)) !=
        hipSuccess) {
      (void)hipFree(gF);
      return TDT_ERR_OOM;
    }
  }
  struct Free {
    void* a;
    void* b;
    ~Free() {
      if (a || b) (void)hipDeviceSynchronize();
      (void)hipFree(a);
      (void)hipFree(b);
    }
  } free_bufs{gF, gt};
  auto solve = [&]() {
    tdt_status_t st =
        p->varlen ? tdt_solve_varlen(p, F, X, stream) : tdt_solve(p, F, X, M, stream);
    if (st >= 0 && adjoint) st = tdt_solve_backward(p, F, X, gF, gt, M, stream);
    return st;
  };
  std::vector<tune::Choice> cands;
  const int whole[] = {0, 1, 2, 4, 8, 16};
  for (int sh = 0; sh < tdt::kNumShapes; ++sh)
    for (int wpc : {0, 1, 2}) {
      if (p->general && sh != tdt::kGeneralShape) continue;
      if (p->varlen)
        for (int w : whole) cands.push_back(tune::Choice{sh, w, wpc, 0.0});
      else
        cands.push_back(tune::Choice{sh, p->sys_max_tiles, wpc, 0.0});
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TDT_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TDT_ERR_HIP;
  }
  tdt_status_t st = TDT_OK;
  int best = -1;
  for (size_t i = 0; i < cands.size() && st >= 0; ++i) {
    st = tune::apply(p, cands[i]);
    if (st < 0) break;
    st = solve();   // warm-up (also grows the workspace outside the timing)
    if (st < 0) break;
    // the median of five timed samples (single solves of a few hundred us
    // vary by several per cent); a sample is one solve, or back-to-back
    // solves filling about 0.2 ms where one solve is shorter (a solve of
    // 10-20 us timed alone is mostly the events' own overhead and jitter)
    constexpr int kReps = 5;
    float t[kReps] = {};
    int per = 1;
    for (int r = -1; r < kReps && st >= 0; ++r) {   // r = -1: sizes the samples
      float ms = 0.0f;
      (void)hipEventRecord(e0, stream);
      for (int k = 0; k < per && st >= 0; ++k) st = solve();
      (void)hipEventRecord(e1, stream);
      if (hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = TDT_ERR_HIP;
      if (r < 0)
        per = ms > 0.0f ? std::min(64, std::max(1, (int)std::ceil(0.2f / ms))) : 64;
      else
        t[r] = ms / (float)per;
    }
    std::sort(t, t + kReps);
    cands[i].ms = t[kReps / 2];
    if (st >= 0 && (best < 0 || cands[i].ms < cands[best].ms)) best = (int)i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st < 0) return st;
  st = tune::apply(p, cands[best]);
  if (st < 0) return st;
  if (best_ms) *best_ms = cands[best].ms;
  if (use_cache) tune::store(key, cands[best]);
  // leave X holding the solution under the chosen shape
  return p->varlen ? tdt_solve_varlen(p, F, X, stream) : tdt_solve(p, F, X, M, stream);
}

tdt_status_t tdt_block_constants(double t_m1, double t_0, double t_1, int B, double* out) {
  if (!out || B < 1 || B > 64 || !finite3(t_m1, t_0, t_1)) return TDT_ERR_INVALID_ARG;
  ld iu[64], cp[64], phi[64], chi[64];
  if (!block_vectors(t_m1, t_0, t_1, B, iu, cp, phi, chi)) return TDT_ERR_SINGULAR;
  for (int i = 0; i < B; ++i) {
    out[i] = (double)iu[i];
    out[B + i] = (double)cp[i];
    out[2 * B + i] = (double)phi[i];
    out[3 * B + i] = (double)chi[i];
  }
  out[4 * B + 0] = (double)phi[0];
  out[4 * B + 1] = (double)phi[B - 1];
  out[4 * B + 2] = (double)chi[0];
  out[4 * B + 3] = (double)chi[B - 1];
  return TDT_OK;
}

tdt_status_t tdt_green_rows(double t_m1, double t_0, double t_1, int64_t L, double* first,
                            double* last) {
  if (!first || !last || L < 1 || L > ((int64_t)1 << 26) || !finite3(t_m1, t_0, t_1))
    return TDT_ERR_INVALID_ARG;
  return green_rows(t_m1, t_0, t_1, L, first, last) ? TDT_OK : TDT_ERR_SINGULAR;
}

tdt_status_t tdt_green_support(double t_m1, double t_0, double t_1, int64_t L, int64_t* kf,
                               int64_t* kl, int64_t* bound2) {
  if (!kf || !kl || L < 1 || L > ((int64_t)1 << 26) || !finite3(t_m1, t_0, t_1))
    return TDT_ERR_INVALID_ARG;
  std::vector<ld> r1, r2;
  if (!green_rows_ld(t_m1, t_0, t_1, L, r1, r2)) return TDT_ERR_SINGULAR;
  green_support(r1, r2, *kf, *kl);
  if (bound2) {
    int64_t bf = 0, bl = 0;
    if (!green_support_bound(t_m1, t_0, t_1, L, bf, bl, nullptr, nullptr)) bf = bl = 0;
    bound2[0] = bf;
    bound2[1] = bl;
  }
  return TDT_OK;
}

tdt_status_t tdt_plan_green_support(tdt_plan_t p, int64_t* rows4) {
  if (!p || !rows4) return TDT_ERR_INVALID_ARG;
  for (int dir = 0; dir < 2; ++dir) {
    rows4[2 * dir] = p->general ? p->gen_kf[dir] : p->green_kf[dir];
    rows4[2 * dir + 1] = p->general ? p->gen_kl[dir] : p->green_kl[dir];
  }
  return TDT_OK;
}

tdt_status_t tdt_segment_merge(const double* l, const double* r, double* out) {
  if (!l || !r || !out) return TDT_ERR_INVALID_ARG;
  const double D = 1.0 - l[5] * r[2];
  if (D == 0.0) return TDT_ERR_SINGULAR;
  const double iD = 1.0 / D;
  const double xk0 = (l[1] + l[5] * r[0]) * iD;
  const double xk10 = r[0] + r[2] * xk0;
  const double tl = l[3] * iD, ur = r[4] * iD;
  out[0] = l[0] + xk10 * l[4];
  out[1] = r[1] + xk0 * r[3];
  out[2] = l[2] + l[4] * r[2] * tl;
  out[3] = tl * r[3];
  out[4] = l[4] * ur;
  out[5] = r[5] + l[5] * ur * r[3];
  return TDT_OK;
}

tdt_status_t tdt_plan_profile(tdt_plan_t p, int enable) {
  if (!p) return TDT_ERR_INVALID_ARG;
  if (!enable) {
    (void)hipDeviceSynchronize();
    clear_profile(p);
  }
  p->profile = enable != 0;
  return TDT_OK;
}

tdt_status_t tdt_plan_profile_read(tdt_plan_t p, double* ms3, int64_t* nsolves) {
  if (!p || !ms3) return TDT_ERR_INVALID_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  ms3[0] = ms3[1] = ms3[2] = 0.0;
  const size_t ns = p->prof_ev.size() / 4;
  for (size_t k = 0; k < ns; ++k) {
    for (int j = 0; j < 3; ++j) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p->prof_ev[4 * k + j], p->prof_ev[4 * k + j + 1]) !=
          hipSuccess)
        return TDT_ERR_HIP;
      ms3[j] += (double)ms;
    }
  }
  if (nsolves) *nsolves = (int64_t)ns;
  clear_profile(p);
  return TDT_OK;
}

tdt_status_t tdt_build_info(int* block_f64, int* block_f32, int* wg_threads, int64_t* tile_len) {
  if (block_f64) *block_f64 = tdt::kShapes[0].B;
  if (block_f32) *block_f32 = tdt::kShapes[0].B;
  if (wg_threads) *wg_threads = tdt::kShapes[0].NT;
  if (tile_len) *tile_len = (int64_t)tdt::kShapes[0].B * tdt::kShapes[0].NT;
  return TDT_OK;
}

}  // extern "C"
