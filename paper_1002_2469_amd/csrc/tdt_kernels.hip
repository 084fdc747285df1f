// tdt_kernels.hip -- gfx950 kernels of the partitioned dichotomy solve.
//
// Formulation (Sec. 2.2-2.3 of the paper, restated for one GPU).  The system
// is cut into blocks of kB consecutive unknowns, one block per lane; kNT
// lanes form a workgroup tile of kTile unknowns; a long system is a sequence
// of tiles.  Every block of a Toeplitz matrix is the same
// kB x kB matrix T_B, so its LU multipliers and its responses to unit values
// just outside it (phi: left, chi: right) are computed once per T on the host
// (the economical preliminary step of Sec. 3.1) and read here as
// wave-uniform scalars.
//
// For any run of consecutive rows S, with y = T_S^{-1} f_S its local
// (zero-boundary) solution, the exact solution on S is
//      x_S = y + x_left * phi_S + x_right * chi_S,                    (*)
// x_left / x_right being the unknowns just outside S (the superposition
// principle of Sec. 2.3).  A segment is summarised by six numbers
//      (y_first, y_last, phi_first, phi_last, chi_first, chi_last).
// Knowing the two values outside a segment made of two halves, (*) written
// at the two rows where the halves meet is a 2x2 system: solving it gives the
// two unknowns at the junction and splits the segment into two independent
// problems -- the dichotomy step of Sec. 2.2 (eqs. (6)-(8)).  The same 2x2
// elimination with zero outside values merges the two half summaries into the
// summary of the whole (the segment's own "beta" of eq. (16): its first and
// last unknown when the right-hand side vanishes outside it, restricted to
// the segment taken as the whole system).  Merging is associative (the
// reordering argument of Sec. 2.5), so all block summaries of a wavefront are
// combined by two Kogge-Stone scans (prefix and suffix) over lanes, the
// wavefront summaries through LDS, and tile summaries in a separate grid
// kernel.  Each lane then knows the solution just outside its block and
// finishes with (*): the final correction with the shared basis phi, chi.
//
// The last block of a system (length Bt < kB) is handled as a kB block whose
// rows beyond Bt are decoupled zeros; lanes past the end are all-zero
// segments.  The merge formulas treat both consistently.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tdt_internal.h"

namespace tdt {

// Compile-time work shape of the tile kernels: B rows per lane, NT lanes per
// workgroup (NW wavefronts), tiles of L = B*NT rows, occupancy target WAVES.
template <int B_, int NT_, int WAVES_>
struct Shape {
  static constexpr int B = B_;
  static constexpr int NT = NT_;
  static constexpr int NW = NT_ / 64;
  static constexpr int L = B_ * NT_;
  static constexpr int WAVES = WAVES_;
};
// The names the shape-generic code uses for its shape's sizes.
#define TDT_SHAPE(SH)                          \
  [[maybe_unused]] constexpr int kB = SH::B;   \
  [[maybe_unused]] constexpr int kNT = SH::NT; \
  [[maybe_unused]] constexpr int kNW = SH::NW; \
  [[maybe_unused]] constexpr int kTile = SH::L;

// The grid-level kernels (interface fallback, gradient reduction) use a
// fixed workgroup of their own.
constexpr int kGridNT = 512;
constexpr int kGridNW = kGridNT / 64;

template <typename T>
struct Seg {
  T yf, yl, pf, pl, cf, cl;
};

// Read-only per-plan data (block vectors, system descriptors, work lists) is
// read through the constant address space: with a wave-uniform address the
// compiler then uses scalar loads into SGPRs, which the sweeps take as
// operands, instead of vector loads into VGPRs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(uintptr_t)p;
}

// Hides a value from the optimiser (an empty asm that "modifies" a register)
// so that per-element offsets derived from it are recomputed next to each
// access instead of being hoisted out of the tile loop and kept live.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The same for a pointer to per-plan constants: loads through the returned
// pointer cannot be merged with, or hoisted above, earlier loads of the same
// data, so each phase of a solve re-reads (with cheap scalar loads) the
// constants it uses instead of keeping all of them live in SGPRs.
template <typename T>
__device__ __forceinline__ cptr<T> fresh(cptr<T> p) {
  uint64_t v = (uint64_t)(uintptr_t)p;
  asm volatile("" : "+s"(v));
  return (cptr<T>)(uintptr_t)v;
}

// Raw buffer accesses: a wave-uniform resource (base, size in bytes) held in
// SGPRs plus one per-lane byte offset.  The hardware range check returns 0
// for reads at or past `bytes` (and for "negative" offsets, which wrap to
// huge unsigned ones) and drops such writes, which is how partial tiles and
// the rows just outside a system are handled.
// The base and size are wave-uniform by construction; readfirstlane states it
// to the compiler, which otherwise may not prove it and would wrap every
// access in a loop over distinct descriptors.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const uint64_t a = reinterpret_cast<uintptr_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const int nb = __builtin_amdgcn_readfirstlane((int)bytes);
  void* ub = reinterpret_cast<void*>((uintptr_t)(((uint64_t)hi << 32) | lo));
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, nb, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// AUX: the instruction's cache-policy bits (0: default; 2: non-temporal).
template <typename T, int AUX = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, T v) {
  if constexpr (sizeof(T) == 8) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, off, 0, AUX);
  } else {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), r, off, 0, AUX);
  }
}
// The solution is stored non-temporal: it is not read again by this solve,
// and lines that do not linger dirty in the caches leave the next read of the
// right-hand side (the first pass of the next solve) at full speed.
constexpr int kStoreAux = 2;

// The segment of no rows: its "first row" is the value right of it and its
// "last row" the value left of it, so that merging it on either side of a
// segment changes nothing and outside values pass through it.
template <typename T>
__device__ __forceinline__ Seg<T> seg_identity() {
  return Seg<T>{T(0), T(0), T(0), T(1), T(1), T(0)};
}

// Summary of L followed by R (the 2x2 elimination at their junction with zero
// values outside L u R).
template <typename T>
__device__ __forceinline__ Seg<T> seg_merge(const Seg<T>& L, const Seg<T>& R) {
  const T iD = T(1) / (T(1) - L.cl * R.pf);
  const T xk0 = (L.yl + L.cl * R.yf) * iD;   // last row of L
  const T xk10 = R.yf + R.pf * xk0;          // first row of R
  const T tl = L.pl * iD;
  const T ur = R.cf * iD;
  Seg<T> M;
  M.yf = L.yf + xk10 * L.cf;
  M.yl = R.yl + xk0 * R.pl;
  M.pf = L.pf + L.cf * R.pf * tl;
  M.pl = tl * R.pl;
  M.cf = L.cf * ur;
  M.cl = R.cl + L.cl * ur * R.pl;
  return M;
}

// Unknowns at the junction of A (left) and B (right) when the values just
// outside A u B are XL and XR: xk = last row of A, xk1 = first row of B.
template <typename T>
__device__ __forceinline__ void junction(T a_yl, T a_pl, T a_cl, T b_yf, T b_pf, T b_cf,
                                         T XL, T XR, T& xk, T& xk1) {
  const T iD = T(1) / (T(1) - a_cl * b_pf);
  xk = (a_yl + a_cl * b_yf + XL * a_pl + XR * a_cl * b_cf) * iD;
  xk1 = b_yf + b_pf * xk + XR * b_cf;
}

template <typename T>
__device__ __forceinline__ Seg<T> shfl_up_seg(const Seg<T>& s, int d) {
  return Seg<T>{__shfl_up(s.yf, d, 64), __shfl_up(s.yl, d, 64), __shfl_up(s.pf, d, 64),
                __shfl_up(s.pl, d, 64), __shfl_up(s.cf, d, 64), __shfl_up(s.cl, d, 64)};
}
template <typename T>
__device__ __forceinline__ Seg<T> shfl_down_seg(const Seg<T>& s, int d) {
  return Seg<T>{__shfl_down(s.yf, d, 64), __shfl_down(s.yl, d, 64), __shfl_down(s.pf, d, 64),
                __shfl_down(s.pl, d, 64), __shfl_down(s.cf, d, 64), __shfl_down(s.cl, d, 64)};
}

// Inclusive prefix (lanes 0..l) and suffix (lanes l..63) summaries.
template <typename T>
__device__ __forceinline__ void wave_scan(const Seg<T>& own, Seg<T>& pre, Seg<T>& suf) {
  const int lane = threadIdx.x & 63;
  pre = own;
  suf = own;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Seg<T> rp = shfl_up_seg(pre, d);
    const Seg<T> rs = shfl_down_seg(suf, d);
    if (lane >= d) pre = seg_merge(rp, pre);
    if (lane + d < 64) suf = seg_merge(suf, rs);
  }
}

// Workgroup level: wavefront summaries go through LDS; every thread derives
// the values just outside its own wavefront from the chain's outside values,
// which outer(summary of the whole chain, XLt, XRt) supplies.  Returns the
// chain's summary.  Contains one barrier (all threads must call).
template <typename T, class Outer>
__device__ __forceinline__ Seg<T> wg_level(const Seg<T>& pre, T (*wsum)[6], Outer outer,
                                           T& XLw, T& XRw) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) {
    wsum[w][0] = pre.yf; wsum[w][1] = pre.yl; wsum[w][2] = pre.pf;
    wsum[w][3] = pre.pl; wsum[w][4] = pre.cf; wsum[w][5] = pre.cl;
  }
  __syncthreads();
  Seg<T> W[kGridNW];
#pragma unroll
  for (int k = 0; k < kGridNW; ++k)
    W[k] = Seg<T>{wsum[k][0], wsum[k][1], wsum[k][2], wsum[k][3], wsum[k][4], wsum[k][5]};
  Seg<T> P[kGridNW], Q[kGridNW];   // P[k] = W[0..k], Q[k] = W[k..kGridNW-1]
  P[0] = W[0];
#pragma unroll
  for (int k = 1; k < kGridNW; ++k) P[k] = seg_merge(P[k - 1], W[k]);
  Q[kGridNW - 1] = W[kGridNW - 1];
#pragma unroll
  for (int k = kGridNW - 2; k >= 0; --k) Q[k] = seg_merge(W[k], Q[k + 1]);
  T XLt, XRt;
  outer(P[kGridNW - 1], XLt, XRt);
  XLw = XLt;
  XRw = XRt;
#pragma unroll
  for (int k = 0; k + 1 < kGridNW; ++k) {   // junction between waves k and k+1
    T xk, xk1;
    junction(P[k].yl, P[k].pl, P[k].cl, Q[k + 1].yf, Q[k + 1].pf, Q[k + 1].cf, XLt, XRt, xk, xk1);
    if (w == k) XRw = xk1;
    if (w == k + 1) XLw = xk;
  }
  return P[kGridNW - 1];
}

// Values just outside this lane's block, from the scans and the wavefront's
// outside values.
template <typename T>
__device__ __forceinline__ void lane_ghosts(const Seg<T>& pre, const Seg<T>& suf, T XLw, T XRw,
                                            T& xl, T& xr) {
  const int lane = threadIdx.x & 63;
  const T p_yl = __shfl_up(pre.yl, 1, 64);
  const T p_pl = __shfl_up(pre.pl, 1, 64);
  const T p_cl = __shfl_up(pre.cl, 1, 64);
  T xk, xk1;
  junction(p_yl, p_pl, p_cl, suf.yf, suf.pf, suf.cf, XLw, XRw, xk, xk1);
  const T nx = __shfl_down(xk1, 1, 64);
  xl = lane == 0 ? XLw : xk;
  xr = lane == 63 ? XRw : nx;
}

// Cross-lane moves inside a wavefront.  DPP row shifts move a value by d lanes
// within each row of 16 lanes (lanes whose source falls outside the row keep
// `old`); readlane copies one lane's value to all lanes.
template <int CTRL>
__device__ __forceinline__ float dpp(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, src),
                                                               CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double old, double src) {
  const uint64_t o = __builtin_bit_cast(uint64_t, old), v = __builtin_bit_cast(uint64_t, src);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v,
                                                            CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32),
                                                            (int)(uint32_t)(v >> 32), CTRL, 0xf,
                                                            0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// Maximum over the 64 lanes (all lanes receive it).
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp<0x111>(v, v));
  v = fmaxf(v, dpp<0x112>(v, v));
  v = fmaxf(v, dpp<0x114>(v, v));
  v = fmaxf(v, dpp<0x118>(v, v));
  return fmaxf(fmaxf(readlane(v, 15), readlane(v, 31)), fmaxf(readlane(v, 47), readlane(v, 63)));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp<0x111>(v, v));
  v = fmax(v, dpp<0x112>(v, v));
  v = fmax(v, dpp<0x114>(v, v));
  v = fmax(v, dpp<0x118>(v, v));
  return fmax(fmax(readlane(v, 15), readlane(v, 31)), fmax(readlane(v, 47), readlane(v, 63)));
}

constexpr int kDppRowShr = 0x110;   // + d: row_shr:d
constexpr int kDppRowShl = 0x100;   // + d: row_shl:d

// Inclusive left-to-right scan over the 64 lanes of affine maps x -> A x + g
// (composition: the map of lane l applied after those of lanes < l): four
// in-row DPP steps, then the four row totals (readlane) carried across rows.
template <typename T>
__device__ __forceinline__ void wave_scan_affine_fwd(T& A, T& g) {
#define TDT_FWD_STEP(D)                                    \
  {                                                        \
    const T As = dpp<kDppRowShr + D>(T(1), A);             \
    const T gs = dpp<kDppRowShr + D>(T(0), g);             \
    g = A * gs + g;                                        \
    A = A * As;                                            \
  }
  TDT_FWD_STEP(1) TDT_FWD_STEP(2) TDT_FWD_STEP(4) TDT_FWD_STEP(8)
#undef TDT_FWD_STEP
  const int row = (threadIdx.x & 63) >> 4;
  const T A0 = readlane(A, 15), g0 = readlane(g, 15);
  const T A1 = readlane(A, 31), g1 = readlane(g, 31);
  const T A2 = readlane(A, 47), g2 = readlane(g, 47);
  // carry into row r: rows 0..r-1 composed
  const T cA1 = A0, cg1 = g0;
  const T cA2 = A1 * cA1, cg2 = A1 * cg1 + g1;
  const T cA3 = A2 * cA2, cg3 = A2 * cg2 + g2;
  const T cA = row == 0 ? T(1) : (row == 1 ? cA1 : (row == 2 ? cA2 : cA3));
  const T cg = row == 0 ? T(0) : (row == 1 ? cg1 : (row == 2 ? cg2 : cg3));
  g = A * cg + g;
  A = A * cA;
}

// Inclusive right-to-left scan of affine maps u -> C u + h (the map of lane l
// applied after those of lanes > l).
template <typename T>
__device__ __forceinline__ void wave_scan_affine_bwd(T& C, T& h) {
#define TDT_BWD_STEP(D)                                    \
  {                                                        \
    const T Cs = dpp<kDppRowShl + D>(T(1), C);             \
    const T hs = dpp<kDppRowShl + D>(T(0), h);             \
    h = C * hs + h;                                        \
    C = C * Cs;                                            \
  }
  TDT_BWD_STEP(1) TDT_BWD_STEP(2) TDT_BWD_STEP(4) TDT_BWD_STEP(8)
#undef TDT_BWD_STEP
  const int row = (threadIdx.x & 63) >> 4;
  const T C1 = readlane(C, 16), h1 = readlane(h, 16);
  const T C2 = readlane(C, 32), h2 = readlane(h, 32);
  const T C3 = readlane(C, 48), h3 = readlane(h, 48);
  // carry into row r from the right: rows r+1..3 composed
  const T eC2 = C3, eh2 = h3;
  const T eC1 = C2 * eC2, eh1 = C2 * eh2 + h2;
  const T eC0 = C1 * eC1, eh0 = C1 * eh1 + h1;
  const T eC = row == 3 ? T(1) : (row == 2 ? eC2 : (row == 1 ? eC1 : eC0));
  const T eh = row == 3 ? T(0) : (row == 2 ? eh2 : (row == 1 ? eh1 : eh0));
  h = C * eh + h;
  C = C * eC;
}

// Per-system constants in compute precision.
template <typename Tc>
struct Consts {
  cptr<Tc> iu;
  cptr<Tc> aiu;
  cptr<Tc> cp;
  cptr<Tc> phi;
  cptr<Tc> chi;
  Tc a;
  Tc pf, pl, cf;          // phi_first, phi_last, chi_first of a full block
  Tc tail_pf, tail_pl, tail_cf;   // the same of the system's last block
};

// Solve the tile's local problem for this lane's block q (in: right-hand
// side, out: solution) given the values XLt, XRt just outside the tile.
// len: real rows of the lane's block (kB full, 1..kB-1 last block of the
// system, 0 past its end).  bp, iDf: this lane's entries of the per-position
// table (beta_{m-1} and 1/(1 - phi_first beta_{m-1}) for a full block m).
//
// Interface pass.  With u_m, v_m the first and last unknown of block m and
// y its local solution, (*) at those two rows reads
//     u_m = y_f + phi_f v_{m-1} + chi_f u_{m+1},
//     v_m = y_l + phi_l v_{m-1} + chi_l u_{m+1}.
// Eliminating left to right gives v_m = alpha_m + beta_m u_{m+1} with
//     alpha_m = A_m alpha_{m-1} + g_m,  A_m = phi_l iD_m,
//     g_m = y_l + A_m beta_{m-1} y_f,   iD_m = 1/(1 - phi_f beta_{m-1}),
// where beta_m = chi_l + phi_l chi_f beta_{m-1} iD_m depends on T only (the
// table), and then right to left
//     u_m = C_m u_{m+1} + h_m,  C_m = chi_f iD_m,  h_m = (y_f + phi_f alpha_{m-1}) iD_m.
// alpha_m is a sum over blocks j <= m of each block's own contribution g_j
// carried by products of A's, u_m a sum over blocks j >= m of the h_j
// carried by products of C's: the two sums of eq. (15) (contributions from
// the left and from the right, weighted by the exterior responses Z of
// eqs. (10)-(12)), evaluated as affine scans.  Associativity (Sec. 2.5) lets the
// scans run as Kogge-Stone steps inside a wavefront and as one LDS level
// across wavefronts instead of the recursive halving of Sec. 2.4.
// If yfo/ylo are non-null the tile summary (first and last unknown of the
// tile with zero outside values) is written by the owning threads and the
// correction is skipped.  Two workgroup barriers inside.
// FULL: every block of the tile has kB rows (the caller has checked it for
// the whole workgroup), which removes the tail handling from the code.
// Otherwise the rows past the system's last block (1..kB-1 rows) are 0 and
// nothing is taken from the right of it (a right outside value of a tile
// that ends inside a block is folded into its right-hand side by the caller).
// TAILV (summaries): the last block takes the end values of its own length,
// and the lanes past the end pass both recurrences through unchanged
// (A = C = 1, g = h = 0), so that the tile's last unknown is the one of its
// real last row.
template <class SH, typename Tc, bool FULL, bool TAILV = false>
__device__ __forceinline__ void tile_solve(Tc (&q)[SH::B], int len_in, Tc XLt, Tc XRt,
                                           const Consts<Tc>& K, Tc bp, Tc iDf,
                                           Tc (*fw)[2], Tc (*bw)[2], double* yfo,
                                           double* ylo) {
  TDT_SHAPE(SH)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int len = FULL ? kB : len_in;
  const bool tail = len > 0 && len < kB;
  const bool wave_tail = FULL ? false : __ballot(tail) != 0;
  // local Thomas sweep with the shared multipliers (T_B^{-1} q); the forward
  // step d_i = q_i/u_i - (t_-1/u_i) d_{i-1} keeps one dependent FMA per row
  const cptr<Tc> iu = fresh(K.iu), aiu = fresh(K.aiu);
#pragma unroll
  for (int i = 0; i < kB; ++i) q[i] *= iu[i];
  if (!wave_tail) {
#pragma unroll
    for (int i = 1; i < kB; ++i) q[i] -= aiu[i] * q[i - 1];
  } else {
#pragma unroll
    for (int i = 1; i < kB; ++i) {
      const Tc d = q[i] - aiu[i] * q[i - 1];
      q[i] = i < len ? d : Tc(0);
    }
  }
  const cptr<Tc> cpb = fresh(K.cp);
#pragma unroll
  for (int i = kB - 2; i >= 0; --i) q[i] -= cpb[i] * q[i + 1];

  // this block's coefficients
  Tc pf = K.pf, pl = K.pl, cf = K.cf, iD = iDf, yf = q[0], yl = q[kB - 1];
  if (!FULL && len < kB) {
    if (len > 0) {
      pf = K.tail_pf;
      iD = Tc(1) / (Tc(1) - pf * bp);
      if (TAILV) {
        pl = K.tail_pl;
        cf = K.tail_cf;
#pragma unroll
        for (int i = 0; i + 1 < kB; ++i)
          if (i == len - 1) yl = q[i];
      } else {
        pl = Tc(0);
        cf = Tc(0);
        yl = Tc(0);
      }
    } else {   // past the end
      pf = Tc(0);
      pl = TAILV ? Tc(1) : Tc(0);
      cf = TAILV ? Tc(1) : Tc(0);
      iD = Tc(1);
      yf = Tc(0);
      yl = Tc(0);
    }
  }
  // left-to-right sums
  Tc A = pl * iD;
  Tc g = yl + A * bp * yf;
  wave_scan_affine_fwd(A, g);
  if (lane == 63) { fw[w][0] = A; fw[w][1] = g; }
  __syncthreads();
  Tc cin = XLt;
  for (int k = 0; k < w; ++k) cin = fw[k][0] * cin + fw[k][1];
  const Tc alpha = A * cin + g;
  Tc alpha_prev = __shfl_up(alpha, 1, 64);
  if (lane == 0) alpha_prev = cin;
  // right-to-left sums
  Tc C = cf * iD;
  Tc h = (yf + pf * alpha_prev) * iD;
  wave_scan_affine_bwd(C, h);
  if (lane == 0) { bw[w][0] = C; bw[w][1] = h; }
  __syncthreads();
  Tc ein = XRt;
  for (int k = kNW - 1; k > w; --k) ein = bw[k][0] * ein + bw[k][1];
  const Tc u = C * ein + h;
  if (TAILV || yfo) {
    if (threadIdx.x == 0) *yfo = (double)u;
    if (threadIdx.x == kNT - 1) *ylo = (double)alpha;
    return;
  }
  Tc u_next = __shfl_down(u, 1, 64);
  if (lane == 63) u_next = ein;
  const Tc xl = alpha_prev + bp * u;   // last unknown of the previous block
  const Tc xr = u_next;                // first unknown of the next block
  if (len == kB) {
    const cptr<Tc> phi = fresh(K.phi), chi = fresh(K.chi);
#pragma unroll
    for (int i = 0; i < kB; ++i) q[i] += xl * phi[i] + xr * chi[i];
  } else if (len > 0) {
    // last block: re-sweep T_Bt x = q_orig - t_-1 xl e_0 in place, recovering
    // the forward-sweep values d_i = y_i + cp_i y_{i+1} from y (nothing comes
    // from the right: see above)
    Tc delta = -K.a * xl * K.iu[0];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const Tc ynext = i + 1 < kB ? q[i + 1] : Tc(0);
      const Tc dp = q[i] + K.cp[i] * ynext + delta;
      q[i] = i < len ? dp : Tc(0);
      if (i + 1 < kB) delta = -K.aiu[i + 1] * delta;
    }
#pragma unroll
    for (int i = kB - 2; i >= 0; --i) q[i] -= K.cp[i] * q[i + 1];
  } else {
#pragma unroll
    for (int i = 0; i < kB; ++i) q[i] = Tc(0);
  }
}

template <typename Tio>
struct TileArgs {
  const Tio* __restrict__ F;
  Tio* __restrict__ X;
  const SysDesc* __restrict__ sys;
  const double* __restrict__ vec64;   // [ncidx][kVecN][kB]
  const float* __restrict__ vec32;
  const double* __restrict__ tab64;   // [ncidx][2][kNT] per-position table
  const float* __restrict__ tab32;
  const int2* __restrict__ items;     // varlen: (system, tile) per item; null for a series
  int64_t nitems;
  int reverse;                        // process items last to first
  int last_only;                      // series: item m is the last tile of right-hand side m
  double* __restrict__ summ;          // [slot][2] tile summaries (y_first, y_last)
  const double* __restrict__ ghost;   // [slot][2] values just outside each tile
  const Tio* __restrict__ Xfwd;       // adjoint: forward solution
  double* __restrict__ gpart;         // adjoint: [final slot][3] partial t-gradients
  int* __restrict__ iters;            // refinement: max iterations used (atomicMax)
  int max_iter;
  double refine_tol;
  // summary launch of a varlen plan: workgroups past the nitems tiles take
  // the first pass's support items (k_beta_ends' varlen items), a wavefront
  // each, so that the two halves of the first pass share one launch
  const int2* __restrict__ ends_items;
  int64_t n_ends;
  const double* __restrict__ gpack;
  // final pass of a plan whose multi-tile systems have at most 64 tiles:
  // each wavefront runs its system's interface pass itself (lane t takes
  // tile t) instead of reading the ghosts of a separate launch, and the
  // workgroups of a quasi-Toeplitz system's end tiles store its corner rows
  int itf_inline;
  const double* __restrict__ ttab;    // as the interface pass's table ([2][ttab_n])
  int64_t ttab_n;
  int64_t corner0;                    // series, quasi-Toeplitz: first corner slot (2 per
                                      // right-hand side) of the adjoint partials
  // final pass of a small series whose Green rows have short supports (the
  // P1 kernels): each workgroup also computes its system's tile summaries
  // (no first-pass launch); the supports' entries as the first pass's
  // ([2][tile length])
  const double* __restrict__ green;
  int gkf, gkl;
};

// Copy of a system descriptor read with scalar loads (wave-uniform index).
__device__ __forceinline__ SysDesc load_sys(const SysDesc* sys, int s) {
  SysDesc D;
  const cptr<uint64_t> src = as_const(reinterpret_cast<const uint64_t*>(sys + s));
  uint64_t* dst = reinterpret_cast<uint64_t*>(&D);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(SysDesc) / 8); ++k) dst[k] = src[k];
  return D;
}

struct ItemInfo {
  int s, t;
  int64_t m;
};

__device__ __forceinline__ ItemInfo decode_item(const int2* items, const SysDesc* sys,
                                                int64_t it, int last_only) {
  ItemInfo r;
  if (last_only) {
    r.s = 0; r.m = it; r.t = *as_const(&sys[0].ntiles) - 1;
  } else if (items) {
    const cptr<int> iv = as_const(reinterpret_cast<const int*>(items)) + 2 * it;
    r.s = iv[0]; r.t = iv[1]; r.m = 0;
  } else {
    const int nt = *as_const(&sys[0].ntiles);
    r.s = 0; r.m = it / nt; r.t = (int)(it - r.m * nt);
  }
  return r;
}

template <class SH, typename Tc>
__device__ __forceinline__ Consts<Tc> make_consts(const SysDesc& S, const double* vec64,
                                                  const float* vec32) {
  TDT_SHAPE(SH)
  Consts<Tc> K;
  const Tc* v;
  if constexpr (sizeof(Tc) == 8)
    v = reinterpret_cast<const Tc*>(vec64) + (int64_t)S.cidx * kVecN * kB;
  else
    v = reinterpret_cast<const Tc*>(vec32) + (int64_t)S.cidx * kVecN * kB;
  const cptr<Tc> c = as_const(v);
  K.iu = c + kVecIU * kB;
  K.aiu = c + kVecAIU * kB;
  K.cp = c + kVecCP * kB;
  K.phi = c + kVecPHI * kB;
  K.chi = c + kVecCHI * kB;
  K.a = (Tc)S.a;
  K.pf = (Tc)S.blk[0]; K.pl = (Tc)S.blk[1]; K.cf = (Tc)S.blk[2];
  K.tail_pf = (Tc)S.tail_pf; K.tail_pl = (Tc)S.tail_pl; K.tail_cf = (Tc)S.tail_cf;
  return K;
}

struct TileGeom {
  ItemInfo I;
  int64_t base;   // element offset of the tile's first row
  int64_t t0;     // row of the tile's first element within its system
  int tl;         // rows in the tile
};

template <class SH>
__device__ __forceinline__ TileGeom tile_geom(const int2* items, const SysDesc* sys,
                                              int64_t it, int last_only) {
  TDT_SHAPE(SH)
  TileGeom G;
  G.I = decode_item(items, sys, it, last_only);
  const SysDesc S = load_sys(sys, G.I.s);
  G.t0 = (int64_t)G.I.t * kTile;
  G.base = S.off + G.I.m * S.stride + G.t0;
  G.tl = (int)(S.n - G.t0 < kTile ? S.n - G.t0 : kTile);
  return G;
}

// Everything a workgroup needs from global memory for one tile, issued
// together at the top of its iteration: the tile's rows (coalesced, element
// j*kNT + tid), this lane's table entries and the values just outside the
// tile.  Every load is unconditional (rows past the tile read as 0 through
// the buffer range check) so that all of them are in flight together.
template <class SH, typename Tio, typename Tc>
struct TileLoad {
  Tio v[SH::B];
  Tc bp, iD;
  double XL, XR;
};

// A corner row of a quasi-Toeplitz system once the interface pass has its
// value v: which = 0 is row 0 (stored at X[base - 1], base = the first inner
// row), which = 1 row N-1 (at X[base + n]).  With Xfwd (adjoint, v = gF of
// that row) the row's own t-gradient terms go to the corner slot cg[0..4]:
// row 0 holds t_0 + psi and t_1, row N-1 holds t_-1 and t_0 + chi.
template <typename Tio>
__device__ __forceinline__ void store_corner(Tio* X, const Tio* Xfwd, double* cg, int64_t base,
                                             int64_t n, int which, double v) {
  if (which == 0) {
    X[base - 1] = (Tio)v;
    if (Xfwd) {
      const double x0 = (double)Xfwd[base - 1], x1 = (double)Xfwd[base];
      cg[0] = 0.0;
      cg[1] = -v * x0;
      cg[2] = -v * x1;
      cg[3] = -v * x0;
      cg[4] = 0.0;
    }
  } else {
    X[base + n] = (Tio)v;
    if (Xfwd) {
      const double xn = (double)Xfwd[base + n], xp = (double)Xfwd[base + n - 1];
      cg[0] = -v * xp;
      cg[1] = -v * xn;
      cg[2] = 0.0;
      cg[3] = 0.0;
      cg[4] = -v * xn;
    }
  }
}

// The values just outside tile t of a system of at most 64 tiles, by the
// system's interface pass (the scans of eq. (15), one tile per lane) from
// the tile summaries and table entries this lane loaded for tile `lane`.
// Outside the chain of tiles: zero, or for a quasi-Toeplitz system the two
// corner rows, whose equations close the chain at both ends (fl, fr: their
// right-hand sides).
template <bool QUASI>
__device__ __forceinline__ void inline_ghosts(const SysDesc& S, int t, double u, double v,
                                              double b0, double i0, double fl, double fr,
                                              double& XL, double& XR) {
  const int lane = threadIdx.x & 63;
  const int P = S.ntiles;
  const bool real = lane < P, last = lane == P - 1;
  const double yf = real ? u : 0.0, yl = real ? v : 0.0;
  const double bp = real ? b0 : 0.0, iD = real ? i0 : 1.0;
  const double pf = real ? (last ? S.ltileK[0] : S.tileK[0]) : 0.0;
  const double pl = real ? (last ? S.ltileK[1] : S.tileK[1]) : 1.0;
  const double cf = real ? (last ? S.ltileK[2] : S.tileK[2]) : 1.0;
  const double alpha_in = QUASI ? fl * S.qc[0] : 0.0;   // alpha_{-1}
  double Ai = pl * iD, gi = yl + pl * iD * bp * yf;
  wave_scan_affine_fwd(Ai, gi);
  const double at = Ai * alpha_in + gi;           // alpha_lane
  double am = __shfl_up(at, 1, 64);               // alpha_{lane-1}
  if (lane == 0) am = alpha_in;
  const double u_right =                          // u_P
      QUASI ? (fr * S.qc[2] + S.qc[3] * __shfl(at, P - 1, 64)) * S.qc[5] : 0.0;
  double Ct = cf * iD, ht = (yf + pf * am) * iD;
  wave_scan_affine_bwd(Ct, ht);
  const double ut = Ct * u_right + ht;            // u_lane
  double un = __shfl_down(ut, 1, 64);             // u_{lane+1}
  if (lane == 63) un = u_right;
  XL = __shfl(am + bp * ut, t, 64);
  XR = __shfl(un, t, 64);
}

//   INLINE: the kernel can run the interface pass inline (when A.itf_inline)
//   P1: the system's tile summaries are in LDS (ps), computed by the workgroup
template <class SH, typename Tio, typename Tc, bool SUMMARY, bool QUASI, bool INLINE, bool P1>
__device__ __forceinline__ void load_tile_item(const TileArgs<Tio>& A, int64_t item,
                                               TileLoad<SH, Tio, Tc>& P, const double* ps) {
  TDT_SHAPE(SH)
  const int tid = threadIdx.x;
  const TileGeom G = tile_geom<SH>(A.items, A.sys, item, A.last_only);
  const SysDesc S = load_sys(A.sys, G.I.s);
  // the inline interface pass: its loads first, so that its scans can run
  // while the tile's rows are still on their way
  const bool inl = INLINE && !SUMMARY && A.itf_inline && (S.ntiles > 1 || QUASI);
  const int64_t sbase = G.base - G.t0;   // the system's first row (inside the corners)
  double iu = 0.0, iv = 0.0, ib = 0.0, ii = 1.0, fl = 0.0, fr = 0.0;
  if (inl) {
    const int lane = tid & 63;
    const int tc = lane < S.ntiles ? lane : 0;
    const bool varlen = A.items != nullptr;
    const int64_t sl = tile_slot(S, G.I.m, tc, varlen);
    const int64_t tb = varlen ? sl : tile_slot(S, 0, tc, false);
    iu = P1 ? ps[2 * tc] : A.summ[2 * sl];
    iv = P1 ? ps[2 * tc + 1] : A.summ[2 * sl + 1];
    ib = A.ttab[tb];
    ii = A.ttab[A.ttab_n + tb];
    if (QUASI) {
      fl = (double)A.F[sbase - 1];
      fr = (double)A.F[sbase + S.n];
    }
  }
  const __amdgpu_buffer_rsrc_t src = make_rsrc(A.F + G.base, (int64_t)G.tl * sizeof(Tio));
  const int vb = opaque(tid * (int)sizeof(Tio));
#pragma unroll
  for (int j = 0; j < kB; ++j) P.v[j] = buf_load<Tio>(src, vb + j * kNT * (int)sizeof(Tio));
  const int ti = S.tfix > 0 && tid > S.tfix ? S.tfix : tid;   // repeated entries: one address
  if constexpr (sizeof(Tc) == 8) {
    const double* tb = A.tab64 + (int64_t)S.cidx * kTabN * kNT;
    P.bp = tb[kTabBeta * kNT + ti];
    P.iD = tb[kTabInvD * kNT + ti];
  } else {
    const float* tb = A.tab32 + (int64_t)S.cidx * kTabN * kNT;
    P.bp = tb[kTabBeta * kNT + ti];
    P.iD = tb[kTabInvD * kNT + ti];
  }
  if (inl) {
    inline_ghosts<QUASI>(S, G.I.t, iu, iv, ib, ii, fl, fr, P.XL, P.XR);
    if (QUASI && tid == 0 && (G.I.t == 0 || G.I.t == S.ntiles - 1)) {
      // the corner rows (and, in the adjoint, their t-gradient partials)
      const int64_t cs0 = A.items ? (int64_t)S.fslot0 + S.ntiles : A.corner0 + 2 * G.I.m;
      if (G.I.t == 0)
        store_corner<Tio>(A.X, A.Xfwd, A.gpart + kGradN * cs0, sbase, S.n, 0, P.XL);
      if (G.I.t == S.ntiles - 1)
        store_corner<Tio>(A.X, A.Xfwd, A.gpart + kGradN * (cs0 + 1), sbase, S.n, 1, P.XR);
    }
  } else if (!SUMMARY) {
    // a one-tile system has no interface pass (zero outside values) unless
    // it has corner rows
    const bool has_ghosts = S.ntiles > 1 || QUASI;
    const int64_t slot = tile_slot(S, G.I.m, G.I.t, A.items != nullptr);
    const int64_t gs = has_ghosts ? slot : 0;   // the ghost array always has slot 0
    const double xl = A.ghost[2 * gs], xr = A.ghost[2 * gs + 1];
    P.XL = has_ghosts ? xl : 0.0;
    P.XR = has_ghosts ? xr : 0.0;
  } else {
    P.XL = P.XR = 0.0;
  }
}

// Occupancy target of the refinement kernels.  They hold no prefetched next
// tile: the register budget goes to the double iterate, and a build that
// prefetched (16 more doubles per lane) spilled and ran the 2^26-row final
// pass at 330-370 us against 213-228 us without.
constexpr int kRefineWaves = kMinWavesPerSimd;

// A workgroup's refinement record, published once when it exits: rec[0] =
// most float solves of any tile, rec[1] = bits of the largest estimated
// remaining relative error (non-negative floats order like their bits).
// Thousands of workgroups publish to the same two words, and atomics on one
// address serialise; the record only grows, so a plain read that already
// shows a value at least as large (a stale read can only show a smaller one)
// makes the atomic unnecessary, and most workgroups skip it.
__device__ __forceinline__ void publish_refine_record(int* rec, int it_max, float est_max) {
  if (threadIdx.x == 0 && rec && it_max > 0) {
    const int e = __float_as_int(est_max);
    if (__atomic_load_n(rec, __ATOMIC_RELAXED) < it_max) atomicMax(rec, it_max);
    if (__atomic_load_n(rec + 1, __ATOMIC_RELAXED) < e) atomicMax(rec + 1, e);
  }
}

// Workgroup-shared scratch of a tile solve.
template <class SH, typename Tio, typename Tc>
struct TileShared {
  static constexpr int RP = SH::B + 16 / (int)sizeof(Tio);   // padded LDS row pitch
  __align__(16) Tio lds[SH::NT * RP];
  Tc fw[SH::NW][2], bw[SH::NW][2];
  double red[SH::NW][4];
  double edge[SH::NW][2];
  double ps[64][2];   // a small series system's tile summaries (final pass)
};

// The tile summaries of one system of a small series from the Green rows'
// supports (the dot products of the first pass, eq. (13)), computed by the
// final pass's workgroup itself: wavefront w takes tiles w, w + NW, ...,
// four at a time with all their loads in flight; lanes stride the support
// rows and the lane sums are added by the same butterfly as in the first
// pass.  Results to ps (LDS); the caller's barrier publishes them.
template <class SH, typename Tio>
__device__ __forceinline__ void system_summaries(const TileArgs<Tio>& A, const SysDesc& S,
                                                 int64_t sbase, double (*ps)[2]) {
  TDT_SHAPE(SH)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nf = A.gkf / 64, nl = A.gkl / 64;
  const double* gf = A.green + lane;
  const double* gl = A.green + 2 * kTile - A.gkl + lane;
  for (int t0 = w; t0 < S.ntiles; t0 += 4 * kNW) {
    double s1[4], s2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) s1[q] = s2[q] = 0.0;
    for (int j = 0; j < nf || j < nl; ++j) {
      const double g1 = j < nf ? gf[j * 64] : 0.0, g2 = j < nl ? gl[j * 64] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + q * kNW;
        const Tio* head = A.F + sbase + (int64_t)(t < S.ntiles ? t : 0) * kTile + lane;
        const double h = j < nf ? (double)head[j * 64] : 0.0;
        const double l = j < nl ? (double)head[kTile - A.gkl + j * 64] : 0.0;
        s1[q] += h * g1;
        s2[q] += l * g2;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        s1[q] += __shfl_xor(s1[q], d, 64);
        s2[q] += __shfl_xor(s2[q], d, 64);
      }
      const int t = t0 + q * kNW;
      if (lane == 0 && t < S.ntiles) {
        ps[t][0] = s1[q];
        ps[t][1] = s2[q];
      }
    }
  }
}

// Element j*kNT + tid of a tile lives in LDS row j*(kNT/kB) + tid/kB, column
// tid%kB: after the coalesced loads each lane owns kB consecutive rows.
template <class SH, typename Tio>
__device__ __forceinline__ int lds_base() {
  TDT_SHAPE(SH)
  constexpr int RP = kB + 16 / (int)sizeof(Tio);
  return (threadIdx.x / kB) * RP + (threadIdx.x % kB);
}
template <class SH, typename Tio>
constexpr int lds_stride() {
  return (SH::NT / SH::B) * (SH::B + 16 / (int)sizeof(Tio));
}

// Rows of the lane's block that exist in a tile of tl rows.
template <class SH>
__device__ __forceinline__ int block_len(int tl) {
  TDT_SHAPE(SH)
  const int r = tl - (int)threadIdx.x * kB;
  return r >= kB ? kB : (r > 0 ? r : 0);
}

// Solves the tile held in LDS in place (each lane's kB rows at myrow), given
// the values just outside it.  With yfo/ylo non-null (SUMMARY, outside values
// zero) it writes the tile's first and last unknown instead.  FULL: every
// block has kB rows.  REFINE: Tio = double data, Tc = float sweeps; residual
// and update in double, repeated until converged (see below).
template <class SH, typename Tio, typename Tc, bool REFINE, bool SUMMARY, bool FULL,
          bool TAILV = false>
__device__ __forceinline__ void solve_in_lds(TileShared<SH, Tio, Tc>& sh, Tio* myrow, int len, int tl,
                                             double XLt, double XRt, const SysDesc& S,
                                             const Consts<Tc>& K, Tc bp, Tc iDf,
                                             double* yfo, double* ylo, int& it_max,
                                             float& est_max, int max_iter, double refine_tol) {
  TDT_SHAPE(SH)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if constexpr (!REFINE) {
    Tc q[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) q[i] = (Tc)myrow[i];
    if constexpr (SUMMARY) {
      tile_solve<SH, Tc, FULL, TAILV>(q, len, Tc(0), Tc(0), K, bp, iDf, sh.fw, sh.bw, yfo, ylo);
    } else {
      tile_solve<SH, Tc, FULL>(q, len, (Tc)XLt, (Tc)XRt, K, bp, iDf, sh.fw, sh.bw, (double*)nullptr,
                           (double*)nullptr);
#pragma unroll
      for (int i = 0; i < kB; ++i) myrow[i] = (Tio)q[i];
    }
  } else {
    // iterative refinement: x_1 = solve_float(f with the tile's outside
    // values); then repeat r = f - T x (double), d = solve_float(r) with
    // zero outside values, x += d (double).  After update k >= 2 the next
    // update is predicted as |d_k| rho with rho = |d_k| / |d_{k-1}|
    // (|d_1| = |x_1|); stop when that is below tol |x_1|, when updates stop
    // shrinking, or at the cap.  The maxima only steer the stopping test, so
    // they are taken in float.  One barrier per update carries both the
    // wavefront edges for the next residual and the wavefront maxima of the
    // last update.
    const double a = S.a, b = S.b, c = S.c;
    double x[kB];
    float xloc = 0.0f;
    {
      Tc q[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        double r = (double)myrow[i];
        if (i == 0 && tid == 0) r -= a * XLt;
        if (i == kB - 1 && tid == kNT - 1) r -= c * XRt;
        q[i] = (FULL || i < len) ? (Tc)r : Tc(0);
      }
      tile_solve<SH, Tc, FULL>(q, len, Tc(0), Tc(0), K, bp, iDf, sh.fw, sh.bw, (double*)nullptr,
                           (double*)nullptr);
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        x[i] = (double)q[i];
        xloc = fmaxf(xloc, fabsf((float)q[i]));
      }
    }
    int it = 1;
    float dprev = 0.0f, dloc = 0.0f, xmax = 0.0f;
    float est = 1.0f;   // estimated remaining relative error (1: no update ran)
    for (;;) {
      float dmax = 0.0f;
      if (it >= 2) dmax = wave_max(dloc);
      else xmax = wave_max(xloc);
      if (lane == 0) { sh.edge[w][0] = x[0]; sh.red[w][0] = it >= 2 ? dmax : xmax; }
      if (lane == 63) sh.edge[w][1] = x[kB - 1];
      __syncthreads();
      if (it >= 2) {
        dmax = (float)sh.red[0][0];
#pragma unroll
        for (int q = 1; q < kNW; ++q) dmax = fmaxf(dmax, (float)sh.red[q][0]);
        const float rho = it == 2 ? dmax / xmax : dmax / dprev;
        dprev = dmax;
        // the next update, predicted (or, once updates stop shrinking, the
        // last one), relative to |x|
        est = dmax == 0.0f ? 0.0f
                           : (xmax > 0.0f ? (rho > 0.9f ? dmax : dmax * rho) / xmax : 1.0f);
        if (dmax == 0.0f || (double)dmax * rho <= refine_tol * xmax || rho > 0.9f) break;
      } else {
        xmax = (float)sh.red[0][0];
#pragma unroll
        for (int q = 1; q < kNW; ++q) xmax = fmaxf(xmax, (float)sh.red[q][0]);
      }
      if (it >= max_iter) break;
      double xm = __shfl_up(x[kB - 1], 1, 64);
      double xp = __shfl_down(x[0], 1, 64);
      if (lane == 0) xm = w == 0 ? XLt : sh.edge[w > 0 ? w - 1 : 0][1];
      if (lane == 63) xp = w == kNW - 1 ? XRt : sh.edge[w + 1 < kNW ? w + 1 : kNW - 1][0];
      Tc q[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const double left = i == 0 ? xm : x[i - 1];
        const double right = i + 1 < kB ? x[i + 1] : xp;
        // r = f - (t_0 x_i + t_-1 x_{i-1} + t_1 x_{i+1}), three fused steps
        double r = fma(-b, x[i], (double)myrow[i]);
        r = fma(-a, left, r);
        r = fma(-c, right, r);
        q[i] = (FULL || i < len) ? (Tc)r : Tc(0);
      }
      tile_solve<SH, Tc, FULL>(q, len, Tc(0), Tc(0), K, bp, iDf, sh.fw, sh.bw, (double*)nullptr,
                           (double*)nullptr);
      dloc = 0.0f;
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        x[i] += (double)q[i];
        dloc = fmaxf(dloc, fabsf((float)q[i]));
      }
      ++it;
      // the next barrier rewrites red[] and edge[]: every wavefront has read
      // them once it is past the barriers inside tile_solve
    }
    // the workgroup's record (kept by every lane; the kernel publishes it once)
    it_max = it > it_max ? it : it_max;
    est_max = fmaxf(est_max, est);
    if constexpr (SUMMARY) {
      if (tid == 0) *yfo = x[0];
      if (tid == (tl - 1) / kB) {
        double xl = x[kB - 1];
#pragma unroll
        for (int i = 0; i + 1 < kB; ++i)
          if (i == (tl - 1) % kB) xl = x[i];
        *ylo = xl;
      }
    } else {
      __syncthreads();   // every lane is done reading f from LDS
#pragma unroll
      for (int i = 0; i < kB; ++i) myrow[i] = (Tio)x[i];
    }
  }
}

template <class SH, typename Tio, typename Tc, bool REFINE, bool SUMMARY, bool TAILV = false>
__device__ __forceinline__ void solve_tile_lds(TileShared<SH, Tio, Tc>& sh, int tl, double XLt,
                                               double XRt, const SysDesc& S,
                                               const Consts<Tc>& K, Tc bp, Tc iDf, double* yfo,
                                               double* ylo, int& it_max, float& est_max,
                                               int max_iter, double refine_tol) {
  TDT_SHAPE(SH)
  Tio* myrow = sh.lds + threadIdx.x * TileShared<SH, Tio, Tc>::RP;
  // a separate full-tile copy of the solve (no tail masking) pays in the
  // refinement kernel; in the double ones it measured the same time
  if (REFINE && tl == kTile)
    solve_in_lds<SH, Tio, Tc, REFINE, SUMMARY, true, TAILV>(sh, myrow, kB, tl, XLt, XRt, S, K, bp, iDf, yfo, ylo,
                                        it_max, est_max, max_iter, refine_tol);
  else
    solve_in_lds<SH, Tio, Tc, REFINE, SUMMARY, false, TAILV>(sh, myrow, block_len<SH>(tl), tl, XLt, XRt, S, K, bp, iDf,
                                         yfo, ylo, it_max, est_max, max_iter, refine_tol);
}

// Stores the solved tile from LDS (coalesced).  BWD: also forms this tile's
// t-gradient partial sums against the forward solution Xfwd and writes their
// negatives to gpart[0..2].  Each lane loads the forward solution at its own
// elements; the neighbours x_{e-1}, x_{e+1} come from the adjacent lanes by
// shuffles, and only the first and last lane of a wavefront load theirs.  QUASI (quasi-Toeplitz plans, whose partials have 5
// components): 0 to the corner components gpart[3..4], and the rows next to
// the corner rows read those rows' forward solution; the corner rows
// themselves are stored by the interface pass (inline: by the workgroups of
// the system's end tiles).  One barrier inside (BWD).
//   PRE (adjoint): the forward solution's first rows are requested before
//   the stores, so that their latency overlaps them (costs registers)
template <class SH, typename Tio, typename Tc, bool BWD, bool QUASI, bool PRE = false>
__device__ __forceinline__ void store_tile(TileShared<SH, Tio, Tc>& sh, Tio* X, const Tio* Xfwd,
                                           int64_t base, int64_t t0, int tl, int64_t n,
                                           double* gpart) {
  TDT_SHAPE(SH)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int lstride = lds_stride<SH, Tio>();
  const __amdgpu_buffer_rsrc_t dst = make_rsrc(X + base, (int64_t)tl * sizeof(Tio));
  // adjoint: the forward solution over this tile and one row on each side
  // that lies inside the system (rows outside read as 0)
  const int lo = t0 > 0 || QUASI ? 1 : 0, hi = t0 + tl < n || QUASI ? 1 : 0;
  const __amdgpu_buffer_rsrc_t xf =
      make_rsrc(BWD ? Xfwd + base - lo : X + base, BWD ? (int64_t)(lo + tl + hi) * sizeof(Tio) : 0);
  const Tio* lr = sh.lds + opaque(lds_base<SH, Tio>());
  const int vs = opaque(tid * (int)sizeof(Tio));
  // where the tile starts within a 128-byte line (packed varlen systems
  // start anywhere)
  constexpr int kLine = 128 / (int)sizeof(Tio);
  const int mis = __builtin_amdgcn_readfirstlane(
      (int)((reinterpret_cast<uintptr_t>(X + base) / sizeof(Tio)) & (kLine - 1)));
  constexpr int kPre = BWD && PRE ? 8 : 0;
  Tio xpre[kPre > 0 ? kPre : 1];
  if constexpr (kPre > 0) {
#pragma unroll
    for (int j = 0; j < kPre; ++j)
      xpre[j] = buf_load<Tio>(xf, vs + (j * kNT + lo) * (int)sizeof(Tio));
  }
  if (mis == 0) {
#pragma unroll
    for (int j = 0; j < kB; ++j)
      buf_store<Tio, kStoreAux>(dst, vs + j * kNT * (int)sizeof(Tio), lr[j * lstride]);
  } else {
    // Lanes rotated by the offset, so that every wavefront's store covers
    // whole lines (stores begun mid-line wrote partial lines: 7 % more bytes
    // in the counters on the separation-of-variables batch).  Store j of lane
    // tid writes row j kNT + tid - mis of the tile; rows outside the tile
    // get an offset past the buffer's range, which drops the store.
    constexpr int RP = kB + 16 / (int)sizeof(Tio);
    constexpr int kDrop = 1 << 30;
    const __amdgpu_buffer_rsrc_t dsta =
        make_rsrc(X + base - mis, (int64_t)(tl + mis) * sizeof(Tio));
    int u = tid - mis, jo = 0;
    if (u < 0) {
      u += kNT;
      jo = -1;
    }
    const Tio* lu = sh.lds + opaque((u / kB) * RP + u % kB);
#pragma unroll
    for (int j = 0; j <= kB; ++j) {
      const int jj = j + jo;   // the row's place in the lane-major LDS tile
      const bool ok = jj >= 0 && jj < kB && jj * kNT + u < tl;
      const Tio v = lu[(jj < 0 ? 0 : (jj < kB ? jj : kB - 1)) * lstride];
      buf_store<Tio, kStoreAux>(dsta, ok ? vs + j * kNT * (int)sizeof(Tio) : kDrop, v);
    }
  }
  if constexpr (BWD) {
    // eight rows at a time (88.5 against 90.8 us with four on the
    // differentiable batch): all sixteen at once would hold too many loads
    // in registers (spills)
    double s0 = 0.0, s1 = 0.0, sm1 = 0.0;
#pragma unroll 8
    for (int j = 0; j < kB; ++j) {
      const int xo = vs + (j * kNT + lo) * (int)sizeof(Tio);
      const Tio xt = j < kPre ? xpre[j < kPre ? j : 0] : buf_load<Tio>(xf, xo);
      Tio xn = __shfl_down(xt, 1, 64);   // element e + 1
      Tio xq = __shfl_up(xt, 1, 64);     // element e - 1
      if (lane == 63) xn = buf_load<Tio>(xf, xo + (int)sizeof(Tio));
      if (lane == 0) xq = buf_load<Tio>(xf, xo - (int)sizeof(Tio));
      const double gv = j * kNT + tid < tl ? (double)lr[j * lstride] : 0.0;
      s0 += gv * (double)xt;
      s1 += gv * (double)xn;
      sm1 += gv * (double)xq;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      s0 += __shfl_xor(s0, d, 64);
      s1 += __shfl_xor(s1, d, 64);
      sm1 += __shfl_xor(sm1, d, 64);
    }
    if (lane == 0) { sh.red[w][0] = sm1; sh.red[w][1] = s0; sh.red[w][2] = s1; }
    __syncthreads();
    if (tid == 0) {
      double u = 0.0, v = 0.0, z = 0.0;
      for (int q = 0; q < kNW; ++q) { u += sh.red[q][0]; v += sh.red[q][1]; z += sh.red[q][2]; }
      gpart[0] = -u;
      gpart[1] = -v;
      gpart[2] = -z;
      if (QUASI) {
        gpart[3] = 0.0;
        gpart[4] = 0.0;
      }
    }
  }
}

// The last tile of a quasi-Toeplitz system, when it ends inside a block: the
// corner row's value XR right of it is folded into the tile's last
// right-hand side row (f - t_1 XR), and the tile is then solved with 0 on
// its right.  One thread changes the LDS copy; the caller's next barrier
// publishes it.
template <class SH, typename Tio, typename Tc>
__device__ __forceinline__ void fold_right(TileShared<SH, Tio, Tc>& sh, int tl, double c,
                                           double XR) {
  TDT_SHAPE(SH)
  const int e = tl - 1;
  if ((int)threadIdx.x == e % kNT) {
    Tio* p = sh.lds + lds_base<SH, Tio>() + (e / kNT) * lds_stride<SH, Tio>();
    *p = (Tio)((double)*p - c * XR);
  }
}

// One wavefront's dot product of k rows of a tile with k entries of a Green
// row's support (k a multiple of 64; both pointers already offset by the
// lane), U rows in flight per lane.  The lane sums are added by a fixed
// butterfly, so the result is repeatable and the same in every lane.
// Both ends of a tile in one wavefront: H rows of the head and H of the tail
// in flight together per lane (for short supports, where a wavefront per end
// would cost more to launch than it saves in waiting).
template <typename Tio, int H>
__device__ __forceinline__ void support_dot2(const Tio* head, const double* gf, int kf,
                                             const Tio* tail, const double* gl, int kl,
                                             double& s1, double& s2) {
  const int nf = kf / 64, nl = kl / 64;
  s1 = 0.0;
  s2 = 0.0;
  for (int j0 = 0; j0 < nf || j0 < nl; j0 += H) {
    double v[H], w[H], x[H], y[H];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      v[u] = j0 + u < nf ? (double)head[(j0 + u) * 64] : 0.0;
      w[u] = j0 + u < nf ? gf[(j0 + u) * 64] : 0.0;
      x[u] = j0 + u < nl ? (double)tail[(j0 + u) * 64] : 0.0;
      y[u] = j0 + u < nl ? gl[(j0 + u) * 64] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      s1 += v[u] * w[u];
      s2 += x[u] * y[u];
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    s1 += __shfl_xor(s1, d, 64);
    s2 += __shfl_xor(s2, d, 64);
  }
}

template <typename Tio, int U>
__device__ __forceinline__ double support_dot(const Tio* rows, const double* g, int k) {
  const int nr = k / 64;
  double s = 0.0;
  for (int j0 = 0; j0 < nr; j0 += U) {
    double v[U], w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = j0 + u < nr ? (double)rows[(j0 + u) * 64] : 0.0;
      w[u] = j0 + u < nr ? g[(j0 + u) * 64] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u] * w[u];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  return s;
}

// The same first pass when the two Green rows decay fast (a diagonally
// dominant T, Sec. 3.4: the entries fall geometrically away from the row's
// own end): the plan has found the head of the first row (kf entries) and
// the tail of the last row (kl entries) outside which a row's mass is below
// 2^-60 of its 1-norm, so each summary reads only those rows of its tile.
// What is dropped is at most 2^-60 |row|_1 |F|_inf, below the rounding of
// the dot product itself.  A wavefront takes a tile, or for long supports
// one end of a tile (the head's dot product and the tail's are independent,
// so two wavefronts halve the chain of loads each waits on); lanes stride
// the rows 64 at a time (kf, kl are multiples of 64), and the lane sums are
// added by a fixed butterfly, so results are repeatable.
// (kEndsSplitRows, kEndsPartShift: tdt_internal.h)
constexpr int kEndsNT = 256;
constexpr int kEndsNW = kEndsNT / 64;
template <typename Tio>
struct BetaEndsArgs {
  const Tio* __restrict__ F;
  const SysDesc* __restrict__ sys;
  const double* __restrict__ green;   // series: [2][kTile]: first row, last row
  int64_t nitems;                     // series: right-hand sides x full tiles per right-hand side
                                      // (varlen: items)
  int split;                          // series: a wavefront per tile end (else per tile)
  int nfull;                          // series: full tiles per right-hand side
  int kf, kl;                         // series: head of the first row, tail of the last row
  double* __restrict__ summ;          // [slot][2]
  int64_t gstride;                    // series: 0, one matrix, green = [2][kTile]; else a
                                      // general matrix, [tile][kf + kl] (the supports'
                                      // entries of each tile's own rows)
  const int2* __restrict__ items;     // varlen: (system, tile | part << kEndsPartShift) per
                                      // item, else null
  const double* __restrict__ gpack;   // varlen: each system's head and tail entries
};

// One wavefront's share of the first pass from the supports: wavefront
// item iw (a tile, or one end of a tile).  Used by k_beta_ends and by the
// summary launch of the tile kernel, whose extra workgroups take these items
// next to the tiles it sweeps.
template <class SH, typename Tio>
__device__ __forceinline__ void beta_ends_item(const BetaEndsArgs<Tio>& A, int64_t iw, int lane) {
  TDT_SHAPE(SH)
  const int64_t it = A.items || !A.split ? iw : iw >> 1;
  int part = A.items || !A.split ? 0 : 1 + (int)(iw & 1);
  // this item's tile, the supports and their entries
  const Tio* head;
  const double *gf, *gl;
  int kf, kl;
  int64_t sl;
  int tl = kTile;
  if (A.items) {
    const cptr<int> iv = as_const(reinterpret_cast<const int*>(A.items)) + 2 * it;
    const int s = iv[0], t = iv[1] & ((1 << kEndsPartShift) - 1);
    part = iv[1] >> kEndsPartShift;
    const SysDesc S = load_sys(A.sys, s);
    kf = S.gkf;
    kl = S.gkl;
    gf = A.gpack + S.goff;
    gl = gf + kf;
    head = A.F + S.off + (int64_t)t * kTile;
    sl = tile_slot(S, 0, t, true);
    const int64_t rest = S.n - (int64_t)t * kTile;   // a shorter last tile (glast)
    tl = rest < kTile ? (int)rest : kTile;
  } else {
    const SysDesc S = load_sys(A.sys, 0);
    const int64_t m = it / A.nfull;
    const int t = (int)(it - m * A.nfull);
    kf = A.kf;
    kl = A.kl;
    gf = A.green + t * A.gstride;
    gl = A.gstride ? gf + kf : gf + 2 * kTile - kl;
    head = A.F + S.off + m * S.stride + (int64_t)t * kTile;
    sl = tile_slot(S, m, t, false);
  }
  // the first row's head against the tile's first rows, the last row's
  // tail against its last rows
  if (part == 0) {
    double s1, s2;
    support_dot2<Tio, 4>(head + lane, gf + lane, kf, head + tl - kl + lane, gl + lane, kl, s1,
                         s2);
    if (lane == 0) {
      A.summ[2 * sl] = s1;
      A.summ[2 * sl + 1] = s2;
    }
  } else {
    const double s = part == 1 ? support_dot<Tio, 8>(head + lane, gf + lane, kf)
                               : support_dot<Tio, 8>(head + tl - kl + lane, gl + lane, kl);
    if (lane == 0) A.summ[2 * sl + part - 1] = s;
  }
}

// Workgroups over tiles: by default one tile each (latency hidden by the
// other resident workgroups, whose loads overlap this one's solve and
// stores), or a grid capped per CU whose workgroups loop over tiles.  Each
// iteration loads its tile at the top; a copy that held the next tile in
// registers ran no faster with one tile per workgroup and spilled in the
// refinement and adjoint variants.
//   SUMMARY = true : first pass over a tile of a multi-tile system: writes the
//                    tile's (y_first, y_last) of its zero-boundary problem.
//   SUMMARY = false: solves the tile given the values just outside it (zero
//                    for a one-tile system) and stores X.
//   REFINE         : Tio = double data, Tc = float sweeps; residual and update
//                    in double, repeated until converged.
//   BWD            : also accumulates the t-gradient partial sums against the
//                    forward solution Xfwd (the tile solves T^T gF = gX).
//   P1             : final pass of a small series that computes its
//                    system's tile summaries itself (no first pass)
template <class SH, typename Tio, typename Tc, bool REFINE, bool SUMMARY, bool BWD, bool QUASI,
          bool P1 = false>
__global__ __launch_bounds__(SH::NT, REFINE ? kRefineWaves : SH::WAVES) void k_tile(
    TileArgs<Tio> A) {
  TDT_SHAPE(SH)
  __shared__ TileShared<SH, Tio, Tc> sh;
  const int tid = threadIdx.x;
  if constexpr (SUMMARY) {
    if (A.n_ends > 0 && (int64_t)blockIdx.x >= A.nitems) {
      // a workgroup of support items (the launch has one tile per workgroup)
      BetaEndsArgs<Tio> B{};
      B.F = A.F;
      B.sys = A.sys;
      B.nitems = A.n_ends;
      B.summ = A.summ;
      B.items = A.ends_items;
      B.gpack = A.gpack;
      const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
      const int64_t iw = ((int64_t)blockIdx.x - A.nitems) * kNW + w;
      if (iw < A.n_ends) beta_ends_item<SH, Tio>(B, iw, tid & 63);
      return;
    }
  }
  const int lbase = lds_base<SH, Tio>();
  constexpr int lstride = lds_stride<SH, Tio>();
  auto item_of = [&](int64_t k) { return A.reverse ? A.nitems - 1 - k : k; };
  int it_max = 0;        // refinement record of this workgroup
  float est_max = 0.0f;
  int64_t k = blockIdx.x;
  TileLoad<SH, Tio, Tc> P;

  while (k < A.nitems) {
    if constexpr (P1) {
      const TileGeom G0 = tile_geom<SH>(A.items, A.sys, item_of(k), A.last_only);
      const SysDesc S0 = load_sys(A.sys, G0.I.s);
      system_summaries<SH, Tio>(A, S0, G0.base - G0.t0, sh.ps);
      __syncthreads();
    }
    load_tile_item<SH, Tio, Tc, SUMMARY, QUASI, !(REFINE && QUASI), P1>(A, item_of(k), P,
                                                                        &sh.ps[0][0]);
    const int64_t item = item_of(k);
    const TileGeom G = tile_geom<SH>(A.items, A.sys, item, A.last_only);
    const SysDesc S = load_sys(A.sys, G.I.s);
    const int64_t slot = tile_slot(S, G.I.m, G.I.t, A.items != nullptr);
    const double XLt = P.XL, XRt = P.XR;
    const Tc bp = P.bp, iDf = P.iD;
    const Consts<Tc> K = make_consts<SH, Tc>(S, A.vec64, A.vec32);
    const int tl = G.tl;

    __syncthreads();   // the previous tile is done with LDS
    {
      Tio* lw = sh.lds + opaque(lbase);
#pragma unroll
      for (int j = 0; j < kB; ++j) lw[j * lstride] = P.v[j];
    }
    const int64_t kn = k + gridDim.x;
    __syncthreads();
    const bool fold = QUASI && !SUMMARY && tl < kTile;
    if (fold) {
      fold_right<SH>(sh, tl, S.c, XRt);
      __syncthreads();
    }

    if constexpr (SUMMARY) {
      solve_tile_lds<SH, Tio, Tc, REFINE, true, QUASI>(sh, tl, 0.0, 0.0, S, K, bp, iDf, A.summ + 2 * slot,
                                      A.summ + 2 * slot + 1, it_max, est_max, A.max_iter, A.refine_tol);
    } else {
      solve_tile_lds<SH, Tio, Tc, REFINE, false>(sh, tl, XLt, fold ? 0.0 : XRt, S, K, bp, iDf,
                                                 (double*)nullptr, (double*)nullptr, it_max,
                                                 est_max, A.max_iter, A.refine_tol);
      __syncthreads();
      const int64_t fs = A.items ? (int64_t)S.fslot0 + G.I.t : G.I.m * S.ntiles + G.I.t;
      store_tile<SH, Tio, Tc, BWD, QUASI, true>(sh, A.X, A.Xfwd, G.base, G.t0, tl, S.n,
                                          A.gpart + (QUASI ? kGradN : 3) * fs);
    }
    k = kn;
  }
  publish_refine_record(A.iters, it_max, est_max);
}

template <typename Tio>
struct SysArgs {
  const Tio* __restrict__ F;
  Tio* __restrict__ X;
  const SysDesc* __restrict__ sys;
  const double* __restrict__ vec64;
  const float* __restrict__ vec32;
  const double* __restrict__ tab64;
  const float* __restrict__ tab32;
  const int* __restrict__ items;      // systems, grouped by workgroup
  const int* __restrict__ bins;       // workgroup b takes items[bins[b] .. bins[b+1])
  const double* __restrict__ ttab;    // [2][tile slot]: beta_{t-1}, 1/(1 - Pf_t beta_{t-1})
  int64_t ttab_n;
  const Tio* __restrict__ Xfwd;       // adjoint: forward solution
  double* __restrict__ gpart;         // adjoint: [final slot][3] partial t-gradients
  int* __restrict__ iters;
  int max_iter;
  double refine_tol;
  const double* __restrict__ gpack;   // Green row supports of the systems (SysDesc goff)
};

// Coalesced load of rows [base, base + tl) into the LDS tile (rows past tl
// read as 0).  The caller brackets it with barriers.
template <class SH, typename Tio, typename Tc>
__device__ __forceinline__ void load_tile(TileShared<SH, Tio, Tc>& sh, const Tio* F, int64_t base,
                                          int tl) {
  TDT_SHAPE(SH)
  const __amdgpu_buffer_rsrc_t src = make_rsrc(F + base, (int64_t)tl * sizeof(Tio));
  const int vb = opaque((int)threadIdx.x * (int)sizeof(Tio));
  Tio v[kB];
#pragma unroll
  for (int j = 0; j < kB; ++j) v[j] = buf_load<Tio>(src, vb + j * kNT * (int)sizeof(Tio));
  Tio* lw = sh.lds + opaque(lds_base<SH, Tio>());
  constexpr int lstride = lds_stride<SH, Tio>();
#pragma unroll
  for (int j = 0; j < kB; ++j) lw[j * lstride] = v[j];
}

template <class SH, typename T>
__device__ __forceinline__ void lane_table(const SysDesc& S, const double* tab64,
                                           const float* tab32, T& bp, T& iD) {
  TDT_SHAPE(SH)
  const int tid = threadIdx.x;
  const int ti = S.tfix > 0 && tid > S.tfix ? S.tfix : tid;   // repeated entries: one address
  if constexpr (sizeof(T) == 8) {
    const double* tb = tab64 + (int64_t)S.cidx * kTabN * kNT;
    bp = tb[kTabBeta * kNT + ti];
    iD = tb[kTabInvD * kNT + ti];
  } else {
    const float* tb = tab32 + (int64_t)S.cidx * kTabN * kNT;
    bp = tb[kTabBeta * kNT + ti];
    iD = tb[kTabInvD * kNT + ti];
  }
}

// One workgroup per system of at most kSysMaxTiles tiles; each workgroup
// works through its own list of systems (the host balances the lists).  All three steps of the method run inside the workgroup:
//   1. every tile's summary (its first and last unknown with zero outside
//      values), tile by tile, kept in LDS;
//   2. the interface across the tiles: the same left-to-right and
//      right-to-left affine recurrences as the grid interface pass (the two
//      sums of eq. (15)), walked by one thread over the few tiles;
//   3. the tiles solved with their outside values and stored, last tile
//      first, so that the rows read last in step 1 are re-read from cache.
// Summaries are computed in double for the refinement path (as in the
// multi-kernel path), in the data precision otherwise.
template <class SH, typename Tio, typename Tc, bool REFINE, bool BWD, bool QUASI>
__global__ __launch_bounds__(SH::NT, REFINE ? kRefineWaves : SH::WAVES) void k_sys(
    SysArgs<Tio> A) {
  TDT_SHAPE(SH)
  using Ts = typename std::conditional<REFINE, double, Tc>::type;
  __shared__ TileShared<SH, Tio, Tc> sh;
  __shared__ Ts sfw[kNW][2], sbw[kNW][2];
  __shared__ double tsum[kSysMaxTiles][2];
  __shared__ double tgh[kSysMaxTiles][2];
  __shared__ double tap[kSysMaxTiles], th[kSysMaxTiles], tbp[kSysMaxTiles], tiD[kSysMaxTiles];
  const int tid = threadIdx.x;
  // Each tile is loaded when its turn comes: holding the next one in
  // registers spilled the double kernel (120-148 B per lane) and made it
  // slower than without (differentiable batch forward, 4 tiles per system:
  // 54.6 -> 47.1 us).
  auto tile_len = [](const SysDesc& S, int t) {
    const int64_t t0 = (int64_t)t * kTile;
    return (int)(S.n - t0 < kTile ? S.n - t0 : kTile);
  };

  int it_max = 0;        // refinement record of this workgroup
  float est_max = 0.0f;
  const int kb = as_const(A.bins)[blockIdx.x], ke = as_const(A.bins)[blockIdx.x + 1];
  for (int k = kb; k < ke; ++k) {
    const int s = as_const(A.items)[k];
    const SysDesc S = load_sys(A.sys, s);
    const int nt = S.ntiles;
    if (nt > kSysMaxTiles) continue;   // never listed here (the host checks it)
    // the last tile is still in LDS after the summaries unless they came
    // from the Green rows' supports
    bool last_in_lds = true;
    if (nt > 1 || QUASI) {
      const Consts<Ts> KS = make_consts<SH, Ts>(S, A.vec64, A.vec32);
      Ts sbp, siD;
      lane_table<SH, Ts>(S, A.tab64, A.tab32, sbp, siD);
      auto sweep_summary = [&](int t) {
        const int tl = tile_len(S, t);
        __syncthreads();   // LDS free
        load_tile<SH>(sh, A.F, S.off + (int64_t)t * kTile, tl);
        __syncthreads();
        Ts q[kB];
        const Tio* myrow = sh.lds + tid * TileShared<SH, Tio, Tc>::RP;
#pragma unroll
        for (int i = 0; i < kB; ++i) q[i] = (Ts)myrow[i];
        tile_solve<SH, Ts, false, QUASI>(q, block_len<SH>(tl), Ts(0), Ts(0), KS, sbp, siD, sfw,
                                        sbw, &tsum[t][0], &tsum[t][1]);
      };
      if (S.gkf > 0) {
        // full tiles, and a shorter last tile with the same entries
        // (glast): one wavefront per tile end reads only the rows under the
        // supports; another shorter last tile is swept (and stays in LDS)
        const int nfull = (int)(S.n / kTile);
        const int nends = nfull < nt && S.glast ? nt : nfull;
        if (nends < nt) sweep_summary(nt - 1);
        else last_in_lds = false;
        const int lane = tid & 63, w = tid >> 6;
        const double* gf = A.gpack + S.goff + lane;
        const double* gl = gf + S.gkf;
        for (int iw = w; iw < 2 * nends; iw += kNW) {
          const int t = iw >> 1;
          const Tio* hd = A.F + S.off + (int64_t)t * kTile + lane;
          const double sv = (iw & 1) == 0
                                ? support_dot<Tio, 4>(hd, gf, S.gkf)
                                : support_dot<Tio, 4>(hd + tile_len(S, t) - S.gkl, gl, S.gkl);
          if (lane == 0) tsum[t][iw & 1] = sv;
        }
      } else {
        for (int t = 0; t < nt; ++t) sweep_summary(t);
      }
      __syncthreads();
      if (tid == 0) {
        // beta_{t-1} and 1/(1 - Pf_t beta_{t-1}) from the plan's table
        // (slot order of the grid interface pass); a quasi-Toeplitz system
        // starts from its first corner row (alpha = its local solution) and
        // ends with its last (u = its solution)
        double alpha = QUASI ? (double)A.F[S.off - 1] * S.qc[0] : 0.0;
        for (int t = 0; t < nt; ++t) {
          const double* Kt = t + 1 < nt ? S.tileK : S.ltileK;
          const int64_t pos = S.slot0 + (int64_t)(t % S.tr) * S.tq + t / S.tr;
          const double bt = A.ttab[pos], iD = A.ttab[A.ttab_n + pos];
          tbp[t] = bt;
          tiD[t] = iD;
          tap[t] = alpha;
          th[t] = (tsum[t][0] + Kt[0] * alpha) * iD;
          const double At = Kt[1] * iD;
          alpha = At * alpha + (tsum[t][1] + At * bt * tsum[t][0]);
        }
        double u = QUASI ? ((double)A.F[S.off + S.n] * S.qc[2] + S.qc[3] * alpha) * S.qc[5]
                           : 0.0;
        for (int t = nt - 1; t >= 0; --t) {
          const double* Kt = t + 1 < nt ? S.tileK : S.ltileK;
          const double un = u;
          u = Kt[2] * tiD[t] * u + th[t];
          tgh[t][0] = tap[t] + tbp[t] * u;
          tgh[t][1] = un;
        }
        if (QUASI) {   // the corner rows (slots after the system's tiles)
          double* cg = A.gpart + kGradN * ((int64_t)S.fslot0 + nt);
          const Tio* xf = BWD ? A.Xfwd : nullptr;
          store_corner<Tio>(A.X, xf, cg, S.off, S.n, 0, tgh[0][0]);
          store_corner<Tio>(A.X, xf, cg + kGradN, S.off, S.n, 1, tgh[nt - 1][1]);
        }
      }
      __syncthreads();
    }
    const Consts<Tc> K = make_consts<SH, Tc>(S, A.vec64, A.vec32);
    Tc bp, iD;
    lane_table<SH, Tc>(S, A.tab64, A.tab32, bp, iD);
    for (int t = nt - 1; t >= 0; --t) {
      const int64_t t0 = (int64_t)t * kTile;
      const int tl = tile_len(S, t);
      const double XLt = nt > 1 || QUASI ? tgh[t][0] : 0.0;
      const double XRt = nt > 1 || QUASI ? tgh[t][1] : 0.0;
      // the last tile summarised may still be in LDS
      if ((!QUASI && nt == 1) || t < nt - 1 || !last_in_lds) {
        __syncthreads();   // LDS free
        load_tile<SH>(sh, A.F, S.off + t0, tl);
        __syncthreads();
      }
      const bool fold = QUASI && tl < kTile;   // only the last tile can be short
      if (fold) {
        fold_right<SH>(sh, tl, S.c, XRt);
        __syncthreads();
      }
      solve_tile_lds<SH, Tio, Tc, REFINE, false>(sh, tl, XLt, fold ? 0.0 : XRt, S, K, bp, iD,
                                                 (double*)nullptr, (double*)nullptr, it_max,
                                                 est_max, A.max_iter, A.refine_tol);
      __syncthreads();
      store_tile<SH, Tio, Tc, BWD, QUASI>(sh, A.X, A.Xfwd, S.off + t0, t0, tl, S.n,
                                          A.gpart + (QUASI ? kGradN : 3) * ((int64_t)S.fslot0 + t));
    }
  }
  publish_refine_record(A.iters, it_max, est_max);
}

// First pass of a series plan over its full tiles: the tile summary is the
// pair of sums of eqs. (13) and (16),
//     y_first = sum_j f_j (T_L^{-1})_{0,j},   y_last = sum_j f_j (T_L^{-1})_{L-1,j},
// i.e. the right-hand side weighted by the first and last row of the inverse
// of the tile's matrix (the Green's function rows of eq. (9) for a tile taken
// as the whole system).  Every full tile of one Toeplitz matrix has the same
// rows, so each lane keeps the entries of its own element positions in
// registers and the pass is a streaming dot product with no transposition
// and no sweeps.  Wavefront w of a workgroup always reads slice w (kTile/kNW
// consecutive rows, 16 bytes per lane per load) of the workgroup's tiles; the
// kNW partial sums of a tile meet in LDS and are added in a fixed order one
// tile later, after the next tile's loads are in flight, so the barrier never
// stalls the stream.  Double arithmetic for every data type.
constexpr int kBetaNT = 1024;                  // threads per workgroup of this pass
constexpr int kBetaNW = kBetaNT / 64;
template <typename Tio>
struct BetaArgs {
  const Tio* __restrict__ F;
  const SysDesc* __restrict__ sys;
  const double* __restrict__ green;   // [2][kTile]: first row, last row
  int64_t nitems;                     // right-hand sides x full tiles per right-hand side
  int nfull;                          // full tiles per right-hand side
  double* __restrict__ summ;          // [slot][2]
};

template <class SH, typename Tio>
__global__ __launch_bounds__(kBetaNT) void k_beta(BetaArgs<Tio> A) {
  TDT_SHAPE(SH)
  constexpr int kSlice = kTile / kBetaNW;           // rows per wavefront slice
  constexpr int kBetaPerLane = kSlice / 64;         // rows per lane
  constexpr int V = 16 / (int)sizeof(Tio);          // elements per 16-byte load
  constexpr int NL = kBetaPerLane / V;              // loads per lane per slice
  __shared__ double part[2][kBetaNW][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const SysDesc S0 = load_sys(A.sys, 0);
  const int64_t base0 = S0.off, stride = S0.stride;
  // rows of this lane inside its slice: (j*64 + lane)*V + v
  double g1[kBetaPerLane], gl[kBetaPerLane];
#pragma unroll
  for (int j = 0; j < NL; ++j)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int e = w * kSlice + (j * 64 + lane) * V + v;
      g1[j * V + v] = A.green[e];
      gl[j * V + v] = A.green[kTile + e];
    }
  auto slot_of = [&](int64_t it) {
    const int64_t m = it / A.nfull;
    return tile_slot(S0, m, (int)(it - m * A.nfull), false);
  };
  int par = 0;
  int64_t prev = -1;
  for (int64_t it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const int64_t m = it / A.nfull;
    const int t = (int)(it - m * A.nfull);
    const __amdgpu_buffer_rsrc_t src = make_rsrc(
        A.F + base0 + m * stride + (int64_t)t * kTile + w * kSlice,
        (int64_t)kSlice * sizeof(Tio));
    const int vb = opaque(lane * 16);
    using R4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(src, 0, 0, 0));
    R4 raw[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) raw[j] = __builtin_amdgcn_raw_buffer_load_b128(src, vb + j * 1024, 0, 0);
    // the previous tile's partials are complete in LDS once every wavefront
    // has passed this barrier (its loads for this tile are already issued)
    __syncthreads();
    if (tid == 0 && prev >= 0) {
      double u = 0.0, v = 0.0;
      for (int k = 0; k < kBetaNW; ++k) { u += part[par ^ 1][k][0]; v += part[par ^ 1][k][1]; }
      const int64_t sl = slot_of(prev);
      A.summ[2 * sl] = u;
      A.summ[2 * sl + 1] = v;
    }
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      if constexpr (sizeof(Tio) == 8) {
        const double2 f2 = __builtin_bit_cast(double2, raw[j]);
        s1 += f2.x * g1[2 * j] + f2.y * g1[2 * j + 1];
        s2 += f2.x * gl[2 * j] + f2.y * gl[2 * j + 1];
      } else {
        const float4 f4 = __builtin_bit_cast(float4, raw[j]);
        const float fv[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          s1 += (double)fv[v] * g1[4 * j + v];
          s2 += (double)fv[v] * gl[4 * j + v];
        }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      s1 += __shfl_xor(s1, d, 64);
      s2 += __shfl_xor(s2, d, 64);
    }
    if (lane == 0) { part[par][w][0] = s1; part[par][w][1] = s2; }
    prev = it;
    par ^= 1;
  }
  __syncthreads();
  if (tid == 0 && prev >= 0) {
    double u = 0.0, v = 0.0;
    for (int k = 0; k < kBetaNW; ++k) { u += part[par ^ 1][k][0]; v += part[par ^ 1][k][1]; }
    const int64_t sl = slot_of(prev);
    A.summ[2 * sl] = u;
    A.summ[2 * sl + 1] = v;
  }
}

template <class SH, typename Tio>
__global__ __launch_bounds__(kEndsNT) void k_beta_ends(BetaEndsArgs<Tio> A) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t nw = A.items || !A.split ? A.nitems : 2 * A.nitems;   // wavefront items
  for (int64_t iw = (int64_t)blockIdx.x * kEndsNW + w; iw < nw;
       iw += (int64_t)gridDim.x * kEndsNW)
    beta_ends_item<SH, Tio>(A, iw, lane);
}

// First pass of a general double series plan: the same Green-row dot
// products as k_beta, with the rows of each tile's own inverse
// ([tile][2][kTile], from the plan).  An item is a tile and a group of R
// right-hand sides: the lane loads its entries of the tile's two rows once and
// streams the group.  (A float plan sweeps its tiles instead: its Green rows
// would weigh as much as its data and measured slower.)
template <typename Tio>
struct GBetaArgs {
  const Tio* __restrict__ F;
  const SysDesc* __restrict__ sys;
  const Tio* __restrict__ green;      // [tile][2][kTile]
  int64_t M;
  int R;
  int64_t G;                          // groups per tile, ceil(M / R)
  int64_t nitems;                     // G * tiles
  double* __restrict__ summ;          // [slot][2]
};

template <class SH, typename Tio>
__global__ __launch_bounds__(kBetaNT) void k_gbeta(GBetaArgs<Tio> A) {
  TDT_SHAPE(SH)
  constexpr int kSlice = kTile / kBetaNW;
  constexpr int kBetaPerLane = kSlice / 64;
  constexpr int V = 16 / (int)sizeof(Tio);
  constexpr int NL = kBetaPerLane / V;
  constexpr int U = 1;   // right-hand sides per step (more in flight did not pay)
  __shared__ double part[2][U][kBetaNW][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const SysDesc S0 = load_sys(A.sys, 0);
  const int64_t stride = S0.stride;
  // partials of the previous step: tile pt, right-hand sides pm .. pm+pc-1
  auto flush = [&](int pt, int64_t pm, int pc, int pp) {
    for (int u = 0; u < pc; ++u) {
      double y1 = 0.0, y2 = 0.0;
      for (int k = 0; k < kBetaNW; ++k) { y1 += part[pp][u][k][0]; y2 += part[pp][u][k][1]; }
      const int64_t sl = tile_slot(S0, pm + u, pt, false);
      A.summ[2 * sl] = y1;
      A.summ[2 * sl + 1] = y2;
    }
  };
  int par = 0, pt = -1, pc = 0;
  int64_t pm = -1;
  for (int64_t k = blockIdx.x; k < A.nitems; k += gridDim.x) {
    const int t = (int)(k / A.G);
    const int64_t m0 = (k - (int64_t)t * A.G) * A.R;
    const int64_t m1 = m0 + A.R < A.M ? m0 + A.R : A.M;
    const Tio* gr = A.green + (int64_t)t * 2 * kTile;
    double g1[kBetaPerLane], gl[kBetaPerLane];
#pragma unroll
    for (int j = 0; j < NL; ++j)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int e = w * kSlice + (j * 64 + lane) * V + v;
        g1[j * V + v] = (double)gr[e];
        gl[j * V + v] = (double)gr[kTile + e];
      }
    // rows of this wavefront's slice that lie inside the system: all of them
    // but in the last tile, whose rows past the end read as 0 (loaded one
    // element at a time there, so that the range check applies to each)
    const int64_t r0 = (int64_t)t * kTile + w * kSlice;
    const int64_t avail = S0.n - r0;
    const int nrows = avail <= 0 ? 0 : (avail < kSlice ? (int)avail : kSlice);
    for (int64_t m = m0; m < m1; m += U) {
      const int cnt = m1 - m < U ? (int)(m1 - m) : U;
      using R4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(
          make_rsrc(A.F, 0), 0, 0, 0));
      R4 raw[U][NL];
      const int vb = opaque(lane * 16);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // right-hand sides past the group read nothing (empty range)
        const __amdgpu_buffer_rsrc_t src = make_rsrc(
            A.F + (m + (u < cnt ? u : 0)) * stride + r0,
            u < cnt ? (int64_t)nrows * sizeof(Tio) : 0);
        if (nrows == kSlice) {
#pragma unroll
          for (int j = 0; j < NL; ++j)
            raw[u][j] = __builtin_amdgcn_raw_buffer_load_b128(src, vb + j * 1024, 0, 0);
        } else {
#pragma unroll
          for (int j = 0; j < NL; ++j) {
            Tio e[V];
#pragma unroll
            for (int v = 0; v < V; ++v)
              e[v] = buf_load<Tio>(src, vb + j * 1024 + v * (int)sizeof(Tio));
            raw[u][j] = __builtin_bit_cast(R4, e);
          }
        }
      }
      __syncthreads();   // the previous step's partials are in LDS
      if (tid == 0 && pt >= 0) flush(pt, pm, pc, par ^ 1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          if constexpr (sizeof(Tio) == 8) {
            const double2 f2 = __builtin_bit_cast(double2, raw[u][j]);
            s1 += f2.x * g1[2 * j] + f2.y * g1[2 * j + 1];
            s2 += f2.x * gl[2 * j] + f2.y * gl[2 * j + 1];
          } else {
            const float4 f4 = __builtin_bit_cast(float4, raw[u][j]);
            const float fv[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              s1 += (double)fv[v] * g1[4 * j + v];
              s2 += (double)fv[v] * gl[4 * j + v];
            }
          }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
          s1 += __shfl_xor(s1, d, 64);
          s2 += __shfl_xor(s2, d, 64);
        }
        if (lane == 0) { part[par][u][w][0] = s1; part[par][u][w][1] = s2; }
      }
      pt = t;
      pm = m;
      pc = cnt;
      par ^= 1;
    }
  }
  __syncthreads();
  if (tid == 0 && pt >= 0) flush(pt, pm, pc, par ^ 1);
}

struct GridArgs {
  // quasi-Toeplitz systems: the corner rows of the right-hand side are read,
  // and those of the solution written, here
  const void* F;
  void* X;
  const void* Xfwd;                   // adjoint: forward solution (else null)
  double* gpart;                      // adjoint: t-gradient slots (corner rows)
  int64_t corner0;                    // series: first corner slot (2 per right-hand side)
  int f32;                            // F, X hold floats
  const double* tK;                   // general matrices: end values of every tile [tile][4]
  const SysDesc* __restrict__ sys;
  const int* __restrict__ gitems;     // varlen: system of each workgroup; null for a series
  const double* __restrict__ ttab;    // [2][tile slot]: beta_{t-1}, 1/(1 - Pf_t beta_{t-1})
  int64_t ttab_n;                     // entries per row of ttab
  const double* __restrict__ summ;
  double* __restrict__ ghost;
  double* __restrict__ gscr;          // [slot][3] suffix (y_first, phi_first, chi_first)
};

__device__ __forceinline__ double grid_f(const GridArgs& A, int64_t i) {
  return A.f32 ? (double)static_cast<const float*>(A.F)[i] : static_cast<const double*>(A.F)[i];
}

// The two corner rows of a quasi-Toeplitz system in the interface pass: the
// first one enters the left-to-right recurrence as alpha = its local solution
// f_0 / (t0 + psi) (its beta is part of the plan's table); the last one
// closes the right-to-left recurrence with u = (f_{N-1} / (t0 + chi) +
// Pf alpha_{P-1}) / (1 - Pf beta_{P-1}), Pf = -t_-1 / (t0 + chi), which is
// the solution in that row.
template <bool QUASI>
__device__ __forceinline__ double corner_alpha(const GridArgs& A, const SysDesc& S,
                                               int64_t base) {
  return QUASI ? grid_f(A, base - 1) * S.qc[0] : 0.0;
}
template <bool QUASI>
__device__ __forceinline__ double corner_u(const GridArgs& A, const SysDesc& S, int64_t base,
                                           double alpha_last) {
  return QUASI ? (grid_f(A, base + S.n) * S.qc[2] + S.qc[3] * alpha_last) * S.qc[5] : 0.0;
}
// Stores corner row `which` (0: row 0, 1: row N-1) with value v; a series
// keeps the corner slots of right-hand side m at corner0 + 2m, a varlen
// system right after its tiles' slots.
__device__ __forceinline__ void grid_corner(const GridArgs& A, const SysDesc& S, int64_t base,
                                            int which, double v) {
  const int64_t cs =
      (A.gitems ? (int64_t)S.fslot0 + S.ntiles : A.corner0 + 2 * (int64_t)blockIdx.x) + which;
  double* cg = A.gpart + kGradN * cs;
  if (A.f32)
    store_corner<float>(static_cast<float*>(A.X), static_cast<const float*>(A.Xfwd), cg, base,
                        S.n, which, v);
  else
    store_corner<double>(static_cast<double*>(A.X), static_cast<const double*>(A.Xfwd), cg, base,
                         S.n, which, v);
}

// Interface pass across the tiles of one system (one workgroup per system
// and right-hand side): every thread folds a run of consecutive tile
// summaries, the runs are combined by the same wavefront scans and LDS level
// as inside a tile, and each thread then walks its run left to right to give
// every tile the values just outside it.
template <bool QUASI, bool GEN>
__global__ __launch_bounds__(kGridNT) void k_grid(GridArgs A) {
  __shared__ double wsum[kGridNW][6];
  const int tid = threadIdx.x;
  int s = 0;
  int64_t slot0;
  if (A.gitems) {
    s = A.gitems[blockIdx.x];
    slot0 = A.sys[s].slot0;
  } else {
    slot0 = (int64_t)blockIdx.x * A.sys[0].tslots;
  }
  const SysDesc& S = A.sys[s];
  const int P = S.ntiles;
  const double* summ = A.summ + 2 * slot0;
  double* ghost = A.ghost + 2 * slot0;
  double* scr = A.gscr + 3 * slot0;
  const int ch = (P + kGridNT - 1) / kGridNT;
  const int ta = tid * ch < P ? tid * ch : P;
  const int tb = ta + ch < P ? ta + ch : P;

  auto tile_seg = [&](int t) {
    const double* k = GEN ? A.tK + 4 * (int64_t)t : (t + 1 < P ? S.tileK : S.ltileK);
    return Seg<double>{summ[2 * t], summ[2 * t + 1], k[0], k[1], k[2], k[3]};
  };

  Seg<double> acc = seg_identity<double>();   // an empty run
  for (int t = tb - 1; t >= ta; --t) {
    const Seg<double> ts = tile_seg(t);
    acc = t == tb - 1 ? ts : seg_merge(ts, acc);
    scr[3 * t] = acc.yf;
    scr[3 * t + 1] = acc.pf;
    scr[3 * t + 2] = acc.cf;
  }
  Seg<double> pre, suf;
  wave_scan(acc, pre, suf);
  // values outside the chain of tiles: 0, or for a quasi-Toeplitz system the
  // two corner rows, from their equations and the chain's end responses
  //   x_0     = f_0 qc0     + qc1 (yf + pf x_0 + cf x_N-1),
  //   x_{N-1} = f_{N-1} qc2 + qc3 (yl + pl x_0 + cl x_N-1)
  const int64_t base = S.off + (A.gitems ? 0 : (int64_t)blockIdx.x) * S.stride;
  auto outer = [&](const Seg<double>& W, double& xl0, double& xr0) {
    if (!QUASI) {
      xl0 = xr0 = 0.0;
      return;
    }
    const double l = grid_f(A, base - 1) * S.qc[0] + S.qc[1] * W.yf;
    const double r = grid_f(A, base + S.n) * S.qc[2] + S.qc[3] * W.yl;
    const double m00 = 1.0 - S.qc[1] * W.pf, m01 = -S.qc[1] * W.cf;
    const double m10 = -S.qc[3] * W.pl, m11 = 1.0 - S.qc[3] * W.cl;
    const double idet = 1.0 / (m00 * m11 - m01 * m10);
    xl0 = (l * m11 - m01 * r) * idet;
    xr0 = (m00 * r - m10 * l) * idet;
  };
  double XLw, XRw;
  wg_level(pre, wsum, outer, XLw, XRw);
  double xl, xr;
  lane_ghosts(pre, suf, XLw, XRw, xl, xr);
  if (QUASI && ta == 0 && tb > 0) grid_corner(A, S, base, 0, xl);
  for (int t = ta; t < tb; ++t) {
    if (t == tb - 1) {
      ghost[2 * t] = xl;
      ghost[2 * t + 1] = xr;
      if (QUASI && t == P - 1) grid_corner(A, S, base, 1, xr);
    } else {
      const Seg<double> ts = tile_seg(t);
      double xk, xk1;
      junction(ts.yl, ts.pl, ts.cl, scr[3 * (t + 1)], scr[3 * (t + 1) + 1], scr[3 * (t + 1) + 2],
               xl, xr, xk, xk1);
      ghost[2 * t] = xl;
      ghost[2 * t + 1] = xk1;
      xl = xk;
    }
  }
}

// Interface pass across the tiles of one system, affine form (one workgroup
// of NTG threads per system and right-hand side, runs of R consecutive tiles
// per thread).  Tiles play the role blocks play inside a tile: with
// (yf_t, yl_t) the tile summaries and (Pf, Pl, Cf, Cl) the end values of a
// full tile (the last tile has those of its own length), the left-to-right
// elimination coefficient
//     beta_t = Cl + Pl Cf beta_{t-1} / (1 - Pf beta_{t-1}),  beta_{-1} = 0,
// depends on T only and comes, with 1/(1 - Pf beta_{t-1}), from the plan's
// table.  Then, as in a tile,
//     alpha_t = A_t alpha_{t-1} + g_t   (left to right, alpha_{-1} = 0),
//     u_t     = C_t u_{t+1} + h_t       (right to left, u_P = 0),
// evaluated as two affine scans over the runs, and tile t's outside values
// are alpha_{t-1} + beta_{t-1} u_t and u_{t+1}.
template <int NTG>
struct GridShared {
  double f[NTG / 64][2];   // wave aggregates (left-to-right affine map)
  double b[NTG / 64][2];   // wave aggregates (right-to-left affine map)
  double alast;            // alpha of the last tile (quasi-Toeplitz systems)
};

// alpha of the last tile, from the thread that holds it to all (one
// barrier, quasi-Toeplitz systems only)
template <int NTG, bool QUASI>
__device__ __forceinline__ double share_alpha_last(GridShared<NTG>& sh, bool mine,
                                                   double alast) {
  if (!QUASI) return 0.0;
  if (mine) sh.alast = alast;
  __syncthreads();
  return sh.alast;
}

// Exclusive left-to-right scan of affine maps x -> A x + g over the threads
// of a workgroup; returns the value entering this thread given x_in for
// thread 0.
template <int NTG>
__device__ __forceinline__ double scan_affine_fwd(double A, double g, double x_in,
                                                  double (*ws)[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  wave_scan_affine_fwd(A, g);
  if (lane == 63) { ws[w][0] = A; ws[w][1] = g; }
  __syncthreads();
  double c = x_in;
  for (int k = 0; k < w; ++k) c = ws[k][0] * c + ws[k][1];
  const double incl = A * c + g;
  const double ex = __shfl_up(incl, 1, 64);
  return lane == 0 ? c : ex;
}

// Exclusive right-to-left scan of affine maps x -> C x + h; returns the value
// entering this thread from the right given x_in after the last thread.
template <int NTG>
__device__ __forceinline__ double scan_affine_bwd(double C, double h, double x_in,
                                                  double (*ws)[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NTG / 64;
  wave_scan_affine_bwd(C, h);
  if (lane == 0) { ws[w][0] = C; ws[w][1] = h; }
  __syncthreads();
  double e = x_in;
  for (int k = NW - 1; k > w; --k) e = ws[k][0] * e + ws[k][1];
  const double incl = C * e + h;
  const double ex = __shfl_down(incl, 1, 64);
  return lane == 63 ? e : ex;
}

// Runs are held in registers: every input of the run is loaded up front.
template <int NTG, int R, bool QUASI, bool GEN>
__global__ __launch_bounds__(NTG) void k_grid_affine(GridArgs A) {
  __shared__ GridShared<NTG> sh;
  const int tid = threadIdx.x;
  int s = 0;
  int64_t slot0;
  if (A.gitems) {
    s = as_const(A.gitems)[blockIdx.x];
    slot0 = *as_const(&A.sys[s].slot0);
  } else {
    slot0 = (int64_t)blockIdx.x * *as_const(&A.sys[0].tslots);
  }
  const SysDesc S = load_sys(A.sys, s);
  const int P = S.ntiles;
  const int tq = S.tq;
  const double* summ = A.summ + 2 * slot0;
  double* ghost = A.ghost + 2 * slot0;
  const int64_t base = S.off + (A.gitems ? 0 : (int64_t)blockIdx.x) * S.stride;
  const int ta = tid * R;
  // this thread's tiles: ta .. ta+R-1 (those >= P are empty), tile ta+r at
  // slot r*tq + tid (run-interleaved).  Full tiles share (Pf, Pl, Cf, Cl);
  // the last one has its own.
  auto pos = [&](int r) { return ta + r < P ? r * tq + tid : 0; };
  double yf[R], yl[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = ta + r;
    const int pc = pos(r);
    const double u = summ[2 * pc], v = summ[2 * pc + 1];
    yf[r] = t < P ? u : 0.0;
    yl[r] = t < P ? v : 0.0;
  }
  // an empty tile passes both recurrences through (A = C = 1, g = h = 0),
  // so that the value entering from the right reaches the last tile
  // (a general matrix has end values per tile)
  auto kofs = [&](int t, double& pf, double& pl, double& cf, double& cl) {
    const bool real = t < P, last = t == P - 1;
    const double* K = GEN ? A.tK + 4 * (int64_t)(real ? t : 0) : (last ? S.ltileK : S.tileK);
    pf = real ? K[0] : 0.0;
    pl = real ? K[1] : 1.0;
    cf = real ? K[2] : 1.0;
    cl = real ? K[3] : 0.0;
  };
  // 1. beta_{t-1} and 1/(1 - Pf_t beta_{t-1}) at every tile, from the plan's
  //    table (they depend on T only)
  const int64_t tb0 = A.gitems ? slot0 : 0;
  double bp[R], iD[R];
  double Af = 1.0, gf = 0.0;   // composite left-to-right map of the run
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = ta + r;
    const int64_t tc = tb0 + pos(r);
    const double b0 = A.ttab[tc], i0 = A.ttab[A.ttab_n + tc];
    bp[r] = t < P ? b0 : 0.0;
    iD[r] = t < P ? i0 : 1.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double pf, pl, cf, cl;
    kofs(ta + r, pf, pl, cf, cl);
    const double At = pl * iD[r];
    const double gt = yl[r] + At * bp[r] * yf[r];
    gf = At * gf + gt;
    Af = At * Af;
  }
  // 2. alpha (left to right)
  double alpha = scan_affine_fwd<NTG>(Af, gf, corner_alpha<QUASI>(A, S, base), sh.f);   // alpha_{ta-1}
  double ap[R], h[R];
  double alast = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double pf, pl, cf, cl;
    kofs(ta + r, pf, pl, cf, cl);
    ap[r] = alpha;
    h[r] = (yf[r] + pf * alpha) * iD[r];
    alpha = pl * iD[r] * alpha + (yl[r] + pl * iD[r] * bp[r] * yf[r]);
    if (ta + r == P - 1) alast = alpha;
  }
  alast = share_alpha_last<NTG, QUASI>(sh, ta <= P - 1 && P - 1 < ta + R, alast);
  // 3. u (right to left)
  double Cb = 1.0, hb = 0.0;   // composite right-to-left map of the run
#pragma unroll
  for (int r = R - 1; r >= 0; --r) {
    double pf, pl, cf, cl;
    kofs(ta + r, pf, pl, cf, cl);
    const double Cr = cf * iD[r];
    hb = Cr * hb + h[r];
    Cb = Cr * Cb;
  }
  double u = scan_affine_bwd<NTG>(Cb, hb, corner_u<QUASI>(A, S, base, alast), sh.b);   // u_{ta+R}
#pragma unroll
  for (int r = R - 1; r >= 0; --r) {
    const int t = ta + r;
    double pf, pl, cf, cl;
    kofs(t, pf, pl, cf, cl);
    const double un = u;                 // u_{t+1}
    u = cf * iD[r] * u + h[r];           // u_t
    if (t < P) {
      const int pc = pos(r);
      const double xl = ap[r] + bp[r] * u;
      ghost[2 * pc] = xl;
      ghost[2 * pc + 1] = un;
      if (QUASI && t == 0) grid_corner(A, S, base, 0, xl);
      if (QUASI && t == P - 1) grid_corner(A, S, base, 1, un);
    }
  }
}

// The same pass for the widest workgroup (1024 threads, whose register
// budget cannot hold a run's inputs): each pass re-reads a tile's inputs from
// L2, and alpha_{t-1} and h_t wait in the tile's ghost slot between passes.
template <int NTG, int R, bool QUASI, bool GEN>
__global__ __launch_bounds__(NTG) void k_grid_affine_lean(GridArgs A) {
  __shared__ GridShared<NTG> sh;
  const int tid = threadIdx.x;
  int s = 0;
  int64_t slot0;
  if (A.gitems) {
    s = as_const(A.gitems)[blockIdx.x];
    slot0 = *as_const(&A.sys[s].slot0);
  } else {
    slot0 = (int64_t)blockIdx.x * *as_const(&A.sys[0].tslots);
  }
  const SysDesc S = load_sys(A.sys, s);
  const int P = S.ntiles;
  const int tq = S.tq;
  const double* summ = A.summ + 2 * slot0;
  double* ghost = A.ghost + 2 * slot0;
  const int64_t tb0 = A.gitems ? slot0 : 0;
  const int64_t base = S.off + (A.gitems ? 0 : (int64_t)blockIdx.x) * S.stride;
  const int ta = tid * R;
  // This thread's tiles ta .. ta+R-1 (those >= P are empty); tile ta+r sits
  // at slot r*tq + tid (run-interleaved).  Each pass re-reads a tile's
  // inputs (L2-resident) instead of holding them in registers: the summary
  // (yf, yl), beta_{t-1} and 1/(1 - Pf_t beta_{t-1}) from the plan's table
  // (they depend on T only), and the end values (Pf, Pl, Cf) of a full tile
  // (the last tile has its own).
  auto pos = [&](int r) { return ta + r < P ? r * tq + tid : 0; };
  struct TileIn { double yf, yl, bp, iD, pf, pl, cf; };
  auto tile_in = [&](int r) {
    const int t = ta + r;
    const int pc = pos(r);
    const bool real = t < P, last = t == P - 1;
    const double* K = GEN ? A.tK + 4 * (int64_t)(real ? t : 0) : (last ? S.ltileK : S.tileK);
    const double u = summ[2 * pc], v = summ[2 * pc + 1];
    const double b0 = A.ttab[tb0 + pc], i0 = A.ttab[A.ttab_n + tb0 + pc];
    TileIn x;
    x.yf = real ? u : 0.0;
    x.yl = real ? v : 0.0;
    x.bp = real ? b0 : 0.0;
    x.iD = real ? i0 : 1.0;
    // an empty tile passes both recurrences through (A = C = 1, g = h = 0)
    x.pf = real ? K[0] : 0.0;
    x.pl = real ? K[1] : 1.0;
    x.cf = real ? K[2] : 1.0;
    return x;
  };
  // 1. composite left-to-right map of the run: alpha_t = A_t alpha_{t-1} + g_t
  double Af = 1.0, gf = 0.0;
#pragma unroll 4
  for (int r = 0; r < R; ++r) {
    const TileIn x = tile_in(r);
    const double At = x.pl * x.iD;
    const double gt = x.yl + At * x.bp * x.yf;
    gf = At * gf + gt;
    Af = At * Af;
  }
  // 2. alpha entering the run; walk it, keeping alpha_{t-1} and h_t of every
  //    tile in its ghost slot until step 3, and compose the run's right-to-left
  //    map u_t = C_t u_{t+1} + h_t front to back (u_ta = Cb u_{ta+R} + hb)
  double alpha = scan_affine_fwd<NTG>(Af, gf, corner_alpha<QUASI>(A, S, base), sh.f);   // alpha_{ta-1}
  double Cb = 1.0, hb = 0.0;
  double alast = 0.0;
#pragma unroll 4
  for (int r = 0; r < R; ++r) {
    const TileIn x = tile_in(r);
    const double h = (x.yf + x.pf * alpha) * x.iD;
    if (ta + r < P) {
      const int pc = pos(r);
      ghost[2 * pc] = alpha;
      ghost[2 * pc + 1] = h;
    }
    hb += Cb * h;
    Cb *= x.cf * x.iD;
    alpha = x.pl * x.iD * alpha + (x.yl + x.pl * x.iD * x.bp * x.yf);
    if (ta + r == P - 1) alast = alpha;
  }
  alast = share_alpha_last<NTG, QUASI>(sh, ta <= P - 1 && P - 1 < ta + R, alast);
  // 3. u (right to left) and the values just outside every tile:
  //    alpha_{t-1} + beta_{t-1} u_t and u_{t+1}
  double u = scan_affine_bwd<NTG>(Cb, hb, corner_u<QUASI>(A, S, base, alast), sh.b);   // u_{ta+R}
#pragma unroll 4
  for (int r = R - 1; r >= 0; --r) {
    if (ta + r >= P) continue;
    const TileIn x = tile_in(r);
    const int pc = pos(r);
    const double ap = ghost[2 * pc], h = ghost[2 * pc + 1];
    const double un = u;                 // u_{t+1}
    u = x.cf * x.iD * u + h;             // u_t
    const double xl = ap + x.bp * u;
    ghost[2 * pc] = xl;
    ghost[2 * pc + 1] = un;
    if (QUASI && ta + r == 0) grid_corner(A, S, base, 0, xl);
    if (QUASI && ta + r == P - 1) grid_corner(A, S, base, 1, un);
  }
}

// Deterministic second stage of the t-gradient sums: series plans sum all
// partials (one workgroup, fixed tree); varlen plans sum each system's tiles
// in order (one thread per system).  A partial slot holds ncomp values: 3
// (t_-1, t_0, t_1), or 5 with (psi, chi) for quasi-Toeplitz plans.
__global__ __launch_bounds__(kGridNT) void k_gt_reduce(const double* __restrict__ gpart,
                                                   const SysDesc* __restrict__ sys,
                                                   int64_t nsys, int64_t nparts, int varlen,
                                                   int ncomp, double* __restrict__ gt) {
  if (varlen) {
    const int64_t s = (int64_t)blockIdx.x * kGridNT + threadIdx.x;
    if (s >= nsys) return;
    const int64_t f0 = sys[s].fslot0;
    // the system's tiles, then its two corner rows (quasi-Toeplitz)
    const int nf = sys[s].ntiles + (sys[s].quasi ? 2 : 0);
    double acc[kGradN] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < nf; ++t)
      for (int c = 0; c < ncomp; ++c) acc[c] += gpart[ncomp * (f0 + t) + c];
    for (int c = 0; c < ncomp; ++c) gt[ncomp * s + c] = acc[c];
    return;
  }
  __shared__ double red[kGridNT][kGradN];
  double acc[kGradN] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < nparts; k += kGridNT)
    for (int c = 0; c < ncomp; ++c) acc[c] += gpart[ncomp * k + c];
  for (int c = 0; c < kGradN; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int h = kGridNT / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < kGradN; ++c) red[threadIdx.x][c] += red[threadIdx.x + h][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < ncomp; ++c) gt[c] = red[0][c];
}


// ---------------------------------------------------------------------------
// General tridiagonal matrices: row i reads a_i x_{i-1} + b_i x_i + c_i
// x_{i+1} = f_i with entries of its own, for a series of right-hand sides
// sharing the matrix (eq. (2) with any A; the preliminary step of Sec. 2.3
// is written for such A).  The method is unchanged: B-row blocks per lane,
// the two affine recurrences of eq. (15) across the blocks of a tile and
// across tiles; only the constants become per block and per tile.  The plan
// pads the system to whole tiles with decoupled rows (b = 1, a = c = 0, f =
// 0), so every tile is full, and lays its per-row and per-block constants
// out [tile][value][row in block][lane], so that each lane loads its own with
// loads that are coalesced across the workgroup.  An item is a tile and a
// group of R right-hand sides: the workgroup loads the tile's constants once
// and keeps them in registers while it solves the group (the items run
// tile-major, so neighbouring items find the constants in L2).
// ---------------------------------------------------------------------------

template <typename Tio, typename Tc>
struct GenArgs {
  const Tio* __restrict__ F;
  Tio* __restrict__ X;
  const Tc* __restrict__ row;    // [tile][kGenRowN][B][NT]: 1/u, a/u, c/u of the block-local LU
  const Tc* __restrict__ blk;    // [tile][kGenBlkN][NT]: block end values, beta_{m-1}, 1/(1 - pf beta_{m-1})
  const SysDesc* __restrict__ sys;
  int64_t M;                     // right-hand sides
  int R;                         // right-hand sides per item
  int64_t G;                     // groups of R right-hand sides per tile, ceil(M / R)
  int64_t nitems;                // G * tiles
  int reverse;
  double* __restrict__ summ;     // [slot][2] tile summaries
  const double* __restrict__ ghost;
};

// One tile of a general matrix for one right-hand side, this lane's block in
// q (in: right-hand side, out: solution, or with yfo/ylo the tile summary).
// The correction re-sweeps each block with its outside values folded into
// its first and last right-hand side rows, so that only the LU of the block
// is needed (no stored basis vectors): with y the block's own solution, the
// forward-sweep values are d_i = y_i + (c/u)_i y_{i+1}; the left value xl
// adds -(a/u)_0 xl to d_0, carried down by d_i -= (a/u)_i times the previous
// change, and the right value xr adds -(c/u)_{B-1} xr to d_{B-1}.
template <class SH, typename Tc>
__device__ __forceinline__ void gen_tile_solve(Tc (&q)[SH::B], const Tc (&iu)[SH::B],
                                               const Tc (&aiu)[SH::B], const Tc (&cp)[SH::B],
                                               Tc pf, Tc pl, Tc cf, Tc bp, Tc iD, Tc XLt, Tc XRt,
                                               Tc (*fw)[2], Tc (*bw)[2], double* yfo,
                                               double* ylo) {
  TDT_SHAPE(SH)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  q[0] *= iu[0];
#pragma unroll
  for (int i = 1; i < kB; ++i) q[i] = q[i] * iu[i] - aiu[i] * q[i - 1];
#pragma unroll
  for (int i = kB - 2; i >= 0; --i) q[i] -= cp[i] * q[i + 1];
  const Tc yf = q[0], yl = q[kB - 1];
  // left-to-right and right-to-left sums (eq. (15)), as in the Toeplitz tile
  Tc A = pl * iD;
  Tc g = yl + A * bp * yf;
  wave_scan_affine_fwd(A, g);
  if (lane == 63) { fw[w][0] = A; fw[w][1] = g; }
  __syncthreads();
  Tc cin = XLt;
  for (int k = 0; k < w; ++k) cin = fw[k][0] * cin + fw[k][1];
  const Tc alpha = A * cin + g;
  Tc alpha_prev = __shfl_up(alpha, 1, 64);
  if (lane == 0) alpha_prev = cin;
  Tc C = cf * iD;
  Tc h = (yf + pf * alpha_prev) * iD;
  wave_scan_affine_bwd(C, h);
  if (lane == 0) { bw[w][0] = C; bw[w][1] = h; }
  __syncthreads();
  Tc ein = XRt;
  for (int k = kNW - 1; k > w; --k) ein = bw[k][0] * ein + bw[k][1];
  const Tc u = C * ein + h;
  if (yfo) {
    if (threadIdx.x == 0) *yfo = (double)u;
    if (threadIdx.x == kNT - 1) *ylo = (double)alpha;
    return;
  }
  Tc u_next = __shfl_down(u, 1, 64);
  if (lane == 63) u_next = ein;
  const Tc xl = alpha_prev + bp * u;   // last unknown of the previous block
  const Tc xr = u_next;                // first unknown of the next block
  Tc delta = -aiu[0] * xl;
#pragma unroll
  for (int i = 0; i < kB; ++i) {
    Tc d = i + 1 < kB ? q[i] + cp[i] * q[i + 1] : q[i];
    d += delta;
    if (i == kB - 1) d -= cp[kB - 1] * xr;
    q[i] = d;
    if (i + 1 < kB) delta = -aiu[i + 1] * delta;
  }
#pragma unroll
  for (int i = kB - 2; i >= 0; --i) q[i] -= cp[i] * q[i + 1];
}

// Persistent workgroups over the (tile, group of right-hand sides) items of a
// general series plan, tile-major; each right-hand side's rows are loaded
// when its turn comes (holding the next one in registers spilled the double
// kernel and cost the float one occupancy: final pass 226 -> 220 us in
// double, 113 -> 105 us in float without it).
//   SUMMARY = true : first pass, the tile summaries (y_first, y_last);
//   SUMMARY = false: solve with the values just outside the tile and store.
template <class SH, typename Tio, typename Tc, bool SUMMARY>
__global__ __launch_bounds__(SH::NT, SH::WAVES) void k_gtile(GenArgs<Tio, Tc> A) {
  TDT_SHAPE(SH)
  __shared__ TileShared<SH, Tio, Tc> sh;
  const int tid = threadIdx.x;
  const SysDesc S = load_sys(A.sys, 0);
  const int nt = S.ntiles;
  // Workgroup b runs on XCD b % 8 (the hardware deals workgroups out round
  // robin), and an XCD's L2 serves only its own compute units: in every full
  // round of gridDim.x items the workgroups of one XCD take a contiguous run
  // of items, so that the groups of one tile, which share its constants,
  // mostly meet in one L2 instead of fetching the constants once per XCD.
  const int64_t cap = gridDim.x;
  auto item_of = [&](int64_t k) {
    const int64_t rd = k / cap, b = k - rd * cap;
    int64_t l = k;
    if ((cap & 7) == 0 && (rd + 1) * cap <= A.nitems) l = rd * cap + (b & 7) * (cap >> 3) + (b >> 3);
    return A.reverse ? A.nitems - 1 - l : l;
  };
  // item it: tile t, right-hand sides g R .. min(g R + R, M) - 1
  auto tile_of = [&](int64_t it) { return (int)(it / A.G); };
  auto first_of = [&](int64_t it) { return (it - (int64_t)tile_of(it) * A.G) * A.R; };
  auto tile_rows = [&](int t) {
    return (int)(S.n - (int64_t)t * kTile < kTile ? S.n - (int64_t)t * kTile : kTile);
  };
  Tio pv[kB];
  auto issue = [&](int t, int64_t m) {
    const int64_t base = m * S.stride + (int64_t)t * kTile;
    const __amdgpu_buffer_rsrc_t src =
        make_rsrc(A.F + base, (int64_t)tile_rows(t) * sizeof(Tio));
    const int vb = opaque(tid * (int)sizeof(Tio));
#pragma unroll
    for (int j = 0; j < kB; ++j) pv[j] = buf_load<Tio>(src, vb + j * kNT * (int)sizeof(Tio));
  };
  int64_t k = blockIdx.x;
  while (k < A.nitems) {
    const int64_t it = item_of(k);
    const int t = tile_of(it), tl = tile_rows(t);
    const int64_t m0 = first_of(it);
    const int64_t m1 = m0 + A.R < A.M ? m0 + A.R : A.M;
    const int64_t kn = k + gridDim.x;
    // this lane's constants, kept for the item's right-hand sides
    const Tc* rw = A.row + (int64_t)t * kGenRowN * kTile + tid;
    Tc iu[kB], aiu[kB], cp[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      iu[i] = rw[(kGenIU * kB + i) * kNT];
      aiu[i] = rw[(kGenAIU * kB + i) * kNT];
      cp[i] = rw[(kGenCP * kB + i) * kNT];
    }
    const Tc* bk = A.blk + (int64_t)t * kGenBlkN * kNT + tid;
    const Tc pf = bk[kGenPF * kNT], pl = bk[kGenPL * kNT], cf = bk[kGenCF * kNT];
    const Tc bp = bk[kGenBP * kNT], iD = bk[kGenID * kNT];
    for (int64_t m = m0; m < m1; ++m) {
      const int64_t slot = tile_slot(S, m, t, false);
      double XLt = 0.0, XRt = 0.0;
      if (!SUMMARY && nt > 1) {
        XLt = A.ghost[2 * slot];
        XRt = A.ghost[2 * slot + 1];
      }
      issue(t, m);
      __syncthreads();   // the previous right-hand side is done with LDS
      {
        Tio* lw = sh.lds + opaque(lds_base<SH, Tio>());
#pragma unroll
        for (int j = 0; j < kB; ++j) lw[j * lds_stride<SH, Tio>()] = pv[j];
      }
      __syncthreads();
      Tio* myrow = sh.lds + tid * TileShared<SH, Tio, Tc>::RP;
      Tc q[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) q[i] = (Tc)myrow[i];
      if constexpr (SUMMARY) {
        gen_tile_solve<SH, Tc>(q, iu, aiu, cp, pf, pl, cf, bp, iD, Tc(0), Tc(0), sh.fw, sh.bw,
                               A.summ + 2 * slot, A.summ + 2 * slot + 1);
      } else {
        gen_tile_solve<SH, Tc>(q, iu, aiu, cp, pf, pl, cf, bp, iD, (Tc)XLt, (Tc)XRt, sh.fw,
                               sh.bw, (double*)nullptr, (double*)nullptr);
#pragma unroll
        for (int i = 0; i < kB; ++i) myrow[i] = (Tio)q[i];
        __syncthreads();
        store_tile<SH, Tio, Tc, false, false>(sh, A.X, (const Tio*)nullptr,
                                              m * S.stride + (int64_t)t * kTile,
                                              (int64_t)t * kTile, tl, S.n, (double*)nullptr);
      }
    }
    k = kn;
  }
}

// Entry gradients of a general series plan after its adjoint solve:
// g[0][i] = dL/da_i = -sum_m gF_{m,i} x_{m,i-1}, g[1][i] = dL/db_i =
// -sum_m gF_{m,i} x_{m,i}, g[2][i] = dL/dc_i = -sum_m gF_{m,i} x_{m,i+1}
// (0 for the unused a_0 and c_{n-1}); one thread per row, right-hand sides
// in order (deterministic).
template <typename Tio>
__global__ __launch_bounds__(kGridNT) void k_ggrad(const Tio* __restrict__ gF,
                                                const Tio* __restrict__ X, int64_t n, int64_t M,
                                                double* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * kGridNT + threadIdx.x;
  if (i >= n) return;
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    const Tio* gp = gF + m * n;
    const Tio* xp = X + m * n;
    const double gv = (double)gp[i];
    sb += gv * (double)xp[i];
    if (i > 0) sa += gv * (double)xp[i - 1];
    if (i + 1 < n) sc += gv * (double)xp[i + 1];
  }
  g[i] = -sa;
  g[n + i] = -sb;
  g[2 * n + i] = -sc;
}
}  // namespace tdt

// ---------------------------------------------------------------------------
// Launch helpers used by the host API (C++ linkage, internal).
// ---------------------------------------------------------------------------
namespace tdt {


// Resident workgroups per CU of a kernel (queried once per variant).
template <typename KernelT>
static int resident_per_cu(KernelT kern, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

static int num_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 1;
  }
  return cus;
}

// Persistent grid: as many workgroups as fit on the device at once, or the
// plan's cap per CU if lower.
static int64_t grid_cap(int per_cu, int wg_per_cu) {
  const int n = wg_per_cu > 0 && wg_per_cu < per_cu ? wg_per_cu : per_cu;
  return (int64_t)n * num_cus();
}

// One workgroup per tile by default: the hardware keeps as many resident as
// fit and starts new ones as others finish, so one workgroup's stores
// overlap the next ones' loads (measured on a 512 MiB solve: 5.8 TB/s
// against 5.3 TB/s for the same tile code run by resident workgroups that
// loop over tiles).  With a cap per CU the workgroups persist and loop.
template <class SH, typename Tio, typename Tc, bool REFINE, bool SUMMARY, bool BWD, bool QUASI,
          bool P1 = false>
static void launch_tile(TileArgs<Tio>& A, int64_t nitems, int reverse, int last_only,
                        int wg_per_cu, hipStream_t st, int64_t extra_wg = 0) {
  auto kern = k_tile<SH, Tio, Tc, REFINE, SUMMARY, BWD, QUASI, P1>;
  static int per_cu = resident_per_cu(kern, SH::NT);
  const int64_t cap = wg_per_cu > 0 ? grid_cap(per_cu, wg_per_cu) : nitems;
  A.nitems = nitems;
  A.reverse = reverse;
  A.last_only = last_only;
  // extra_wg: workgroups past the tiles (support items of the summary
  // launch; only with one tile per workgroup)
  const unsigned grid = (unsigned)((nitems < cap ? nitems : cap) + extra_wg);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(SH::NT), 0, st, A);
}

template <class SH, typename Tio, typename Tc, bool REFINE, bool BWD, bool QUASI>
static void launch_sys(const LaunchSet& L, const TileArgs<Tio>& T, hipStream_t st) {
  SysArgs<Tio> A{T.F,         T.X,         T.sys,      T.vec64,  T.vec32,   T.tab64,
                 T.tab32,     L.sys_items, L.sys_bins, L.ttab,   L.ttab_n,  T.Xfwd,
                 T.gpart,     T.iters,     T.max_iter, T.refine_tol, L.gpack};
  hipLaunchKernelGGL((k_sys<SH, Tio, Tc, REFINE, BWD, QUASI>), dim3((unsigned)L.n_bins), dim3(SH::NT),
                     0, st, A);
}

template <class SH, bool QUASI>
static int sys_capacity(int dtype, int wg_per_cu) {
  int per_cu;
  switch (dtype) {
    case 0: per_cu = resident_per_cu(k_sys<SH, double, double, false, false, QUASI>, SH::NT); break;
    case 1: per_cu = resident_per_cu(k_sys<SH, float, float, false, false, QUASI>, SH::NT); break;
    default: per_cu = resident_per_cu(k_sys<SH, double, float, true, false, QUASI>, SH::NT); break;
  }
  return (int)grid_cap(per_cu, wg_per_cu);
}

template <class SH, typename Tio>
static void launch_beta(const LaunchSet& L, const Tio* F, hipStream_t st) {
  auto kern = k_beta<SH, Tio>;
  static int per_cu = resident_per_cu(kern, kBetaNT);
  const int64_t cap = grid_cap(per_cu, L.wg_per_cu);
  BetaArgs<Tio> B{F, L.sys, L.green, L.n_beta, L.nfull, L.summ};
  const unsigned grid = (unsigned)(L.n_beta < cap ? L.n_beta : cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBetaNT), 0, st, B);
}

// The first pass over the Green rows' supports only (the plan found them
// short enough): one wavefront per tile (with a cap per CU, persistent
// workgroups loop over the tiles).
template <class SH, typename Tio>
static void launch_beta_ends(const LaunchSet& L, const Tio* F, hipStream_t st) {
  auto kern = k_beta_ends<SH, Tio>;
  static int per_cu = resident_per_cu(kern, kEndsNT);
  const int64_t cap = grid_cap(per_cu, L.wg_per_cu);
  const bool varlen = L.ends_items != nullptr;
  const int64_t n = varlen ? L.n_ends : L.n_beta;
  const int split = !varlen && L.green_kf + L.green_kl > kEndsSplitRows ? 1 : 0;
  BetaEndsArgs<Tio> B{F,      L.sys,  L.green, n,     split, L.nfull,
                      L.green_kf, L.green_kl, L.summ, 0,     varlen ? L.ends_items : nullptr,
                      L.gpack};
  const int64_t want = ((split ? 2 : 1) * n + kEndsNW - 1) / kEndsNW;
  const int64_t lim = L.wg_per_cu > 0 ? cap : ((int64_t)1 << 30);
  const unsigned grid = (unsigned)(want < lim ? want : lim);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kEndsNT), 0, st, B);
}

// Interface pass of a series Toeplitz plan of 2049 to 16384 tiles, in two
// launches over chunks of 64 tiles, one wavefront per chunk and right-hand
// side, instead of one workgroup per system (whose single compute unit the
// 16384-tile pass left waiting on its loads and stores).  With the tiles'
// maps of eq. (15) written as in the affine variants,
//   alpha_t = A_t alpha_{t-1} + g_t,   u_t = C_t u_{t+1} + h_t,
//   h_t = (y_f + Pf alpha_{t-1}) iD_t,
// a chunk's alpha_{t-1} is affine in the alpha entering the chunk, so its
// h_t are too, and the chunk composes to alpha_out = Ac alpha_in + gc and
//   u_first = Cc u_right + Hq + Hp alpha_in.
// The first launch writes these five numbers per chunk; the second scans
// them over the chunks (every wavefront redundantly: at most 256 chunks, in
// L2), then its own chunk's tiles, and writes their outside values.  No
// atomics and no waiting between workgroups.  Slots are plain (a run of one
// tile per thread), so a chunk's summaries are contiguous.
constexpr int kChunkNT = 256;
constexpr int kChunkRC = 4;   // chunks per lane in the chunk scan (up to 64 x 4 chunks)

// Tile t's summaries, table entries and end values (identity maps past the
// last tile).
__device__ __forceinline__ void chunk_tile(const GridArgs& A, const SysDesc& S, int64_t slot0,
                                           int t, double& yf, double& yl, double& bp,
                                           double& iD, double& pf, double& pl, double& cf) {
  const int P = S.ntiles;
  const bool real = t < P;
  const int tc = real ? t : 0;
  const double* K = t == P - 1 ? S.ltileK : S.tileK;
  const double u = A.summ[2 * (slot0 + tc)], v = A.summ[2 * (slot0 + tc) + 1];
  const double b0 = A.ttab[tc], i0 = A.ttab[A.ttab_n + tc];
  yf = real ? u : 0.0;
  yl = real ? v : 0.0;
  bp = real ? b0 : 0.0;
  iD = real ? i0 : 1.0;
  pf = real ? K[0] : 0.0;
  pl = real ? K[1] : 1.0;
  cf = real ? K[2] : 1.0;
}

// The tiles of chunk c (64 tiles, one per lane) given the alpha entering the
// chunk and the u right of it: the scans of eq. (15) over the chunk, and
// every tile's values just outside it.
__device__ __forceinline__ void chunk_tiles_apply(const GridArgs& A, const SysDesc& S,
                                                  int64_t slot0, int c, double alpha_in,
                                                  double u_right, int lane) {
  const int t = c * 64 + lane;
  double yf, yl, bp, iD, pf, pl, cf;
  chunk_tile(A, S, slot0, t, yf, yl, bp, iD, pf, pl, cf);
  double Ai = pl * iD, gi = yl + pl * iD * bp * yf;
  wave_scan_affine_fwd(Ai, gi);
  const double ainc = Ai * alpha_in + gi;                    // alpha_t
  double am = __shfl_up(ainc, 1, 64);                        // alpha_{t-1}
  if (lane == 0) am = alpha_in;
  double Ct = cf * iD, ht = (yf + pf * am) * iD;
  wave_scan_affine_bwd(Ct, ht);
  const double ut = Ct * u_right + ht;                       // u_t
  double un = __shfl_down(ut, 1, 64);                        // u_{t+1}
  if (lane == 63) un = u_right;
  if (t < S.ntiles) {
    A.ghost[2 * (slot0 + t)] = am + bp * ut;
    A.ghost[2 * (slot0 + t) + 1] = un;
  }
}

__global__ __launch_bounds__(kChunkNT) void k_grid_chunk_reduce(GridArgs A, int64_t M) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (kChunkNT / 64) +
                     __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const SysDesc S = load_sys(A.sys, 0);
  const int NC = (S.ntiles + 63) / 64;
  const int64_t m = gw / NC;
  const int c = (int)(gw - m * NC);
  if (m >= M) return;
  double yf, yl, bp, iD, pf, pl, cf;
  chunk_tile(A, S, m * S.tslots, c * 64 + lane, yf, yl, bp, iD, pf, pl, cf);
  double Ai = pl * iD, gi = yl + pl * iD * bp * yf;
  wave_scan_affine_fwd(Ai, gi);   // alpha_t = Ai alpha_in + gi
  double Pe = __shfl_up(Ai, 1, 64), Qe = __shfl_up(gi, 1, 64);   // alpha_{t-1}
  if (lane == 0) {
    Pe = 1.0;
    Qe = 0.0;
  }
  double C1 = cf * iD, C2 = C1;
  double hq = (yf + pf * Qe) * iD, hp = pf * Pe * iD;
  wave_scan_affine_bwd(C1, hq);
  wave_scan_affine_bwd(C2, hp);
  const double Ac = readlane(Ai, 63), gc = readlane(gi, 63);
  if (lane == 0) {
    double* o = A.gscr + 5 * (m * NC + c);
    o[0] = Ac;
    o[1] = gc;
    o[2] = C1;
    o[3] = hq;
    o[4] = hp;
  }
}

__global__ __launch_bounds__(kChunkNT) void k_grid_chunk_apply(GridArgs A, int64_t M) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (kChunkNT / 64) +
                     __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const SysDesc S = load_sys(A.sys, 0);
  const int NC = (S.ntiles + 63) / 64;
  const int64_t m = gw / NC;
  const int c = (int)(gw - m * NC);
  if (m >= M) return;
  // 1. the chunks: lane k holds chunks k RC .. k RC + RC - 1
  const double* ch = A.gscr + 5 * m * NC;
  double Ac[kChunkRC], gc[kChunkRC], Cc[kChunkRC], Hq[kChunkRC], Hp[kChunkRC];
#pragma unroll
  for (int r = 0; r < kChunkRC; ++r) {
    const int q = lane * kChunkRC + r;
    const bool real = q < NC;
    const double* e = ch + 5 * (real ? q : 0);
    const double e0 = e[0], e1 = e[1], e2 = e[2], e3 = e[3], e4 = e[4];
    Ac[r] = real ? e0 : 1.0;
    gc[r] = real ? e1 : 0.0;
    Cc[r] = real ? e2 : 1.0;
    Hq[r] = real ? e3 : 0.0;
    Hp[r] = real ? e4 : 0.0;
  }
  double Ar = 1.0, gr = 0.0;
#pragma unroll
  for (int r = 0; r < kChunkRC; ++r) {
    gr = Ac[r] * gr + gc[r];
    Ar = Ac[r] * Ar;
  }
  wave_scan_affine_fwd(Ar, gr);
  double a = __shfl_up(gr, 1, 64);   // alpha entering the lane's chunks (alpha_{-1} = 0)
  if (lane == 0) a = 0.0;
  double ain[kChunkRC], hb[kChunkRC];
#pragma unroll
  for (int r = 0; r < kChunkRC; ++r) {
    ain[r] = a;
    hb[r] = Hq[r] + Hp[r] * a;
    a = Ac[r] * a + gc[r];
  }
  double Cr = 1.0, hr = 0.0;
#pragma unroll
  for (int r = kChunkRC - 1; r >= 0; --r) {
    hr = Cc[r] * hr + hb[r];
    Cr = Cc[r] * Cr;
  }
  wave_scan_affine_bwd(Cr, hr);
  double u = __shfl_down(hr, 1, 64);   // u entering the lane's chunks from the right (u_P = 0)
  if (lane == 63) u = 0.0;
  double ur[kChunkRC];
#pragma unroll
  for (int r = kChunkRC - 1; r >= 0; --r) {
    ur[r] = u;
    u = Cc[r] * u + hb[r];
  }
  // this wavefront's chunk c: held by lane c / RC as its entry c % RC
  const int rc = c % kChunkRC;
  double ai = ain[0], uo = ur[0];
#pragma unroll
  for (int r = 1; r < kChunkRC; ++r) {
    ai = rc == r ? ain[r] : ai;
    uo = rc == r ? ur[r] : uo;
  }
  const double alpha_in = __shfl(ai, c / kChunkRC, 64);
  const double u_right = __shfl(uo, c / kChunkRC, 64);
  // 2. the chunk's tiles
  chunk_tiles_apply(A, S, m * S.tslots, c, alpha_in, u_right, lane);
}

// Interface pass across tiles: the affine variant sized for the most tiled
// system (up to 16384 tiles), beyond that the segment-merge kernel.  The
// plan lays out its workspace slots for the same choice (interface_run).
template <bool QUASI, bool GEN = false>
static void launch_grid(const LaunchSet& L, const void* F, void* X, const void* Xfwd, int f32,
                        hipStream_t st) {
  GridArgs G{F,     X,          Xfwd,   L.gpart,  L.corner0, f32,    L.gen_tK, L.sys,
             L.grid_items, L.ttab, L.ttab_n, L.summ,   L.ghost, L.gscr};
  const dim3 gg((unsigned)L.n_grid);
  if (!QUASI && !GEN && L.chunks) {
    const int64_t nw = L.n_grid * ((L.max_ntiles + 63) / 64);   // chunks of all right-hand sides
    const dim3 cg((unsigned)((nw + kChunkNT / 64 - 1) / (kChunkNT / 64)));
    hipLaunchKernelGGL(k_grid_chunk_reduce, cg, dim3(kChunkNT), 0, st, G, (int64_t)L.n_grid);
    hipLaunchKernelGGL(k_grid_chunk_apply, cg, dim3(kChunkNT), 0, st, G, (int64_t)L.n_grid);
  } else if (L.max_ntiles <= 64)   // one wavefront per system: no idle waves, no LDS level
    hipLaunchKernelGGL((k_grid_affine<64, 1, QUASI, GEN>), gg, dim3(64), 0, st, G);
  else if (L.max_ntiles <= 256)
    hipLaunchKernelGGL((k_grid_affine<256, 1, QUASI, GEN>), gg, dim3(256), 0, st, G);
  else if (L.max_ntiles <= 2048)
    hipLaunchKernelGGL((k_grid_affine<256, 8, QUASI, GEN>), gg, dim3(256), 0, st, G);
  else if (!GEN && L.max_ntiles <= 8192) {
    // (a general matrix's end values per tile, 16 tiles per thread, would
    // not fit 512 threads' registers: it takes the lean kernel from here on)
    if constexpr (!GEN)
      hipLaunchKernelGGL((k_grid_affine<512, 16, QUASI, false>), gg, dim3(512), 0, st, G);
  } else if (L.max_ntiles <= 16384)
    hipLaunchKernelGGL((k_grid_affine_lean<1024, 16, QUASI, GEN>), gg, dim3(1024), 0, st, G);
  else
    hipLaunchKernelGGL((k_grid<QUASI, GEN>), gg, dim3(kGridNT), 0, st, G);
}

template <class SH, typename Tio, typename Tc, bool REFINE, bool BWD, bool QUASI>
static hipError_t run_solve(const LaunchSet& L, const void* F, void* X, const void* Xfwd,
                            hipStream_t st) {
  TileArgs<Tio> A{};
  A.F = static_cast<const Tio*>(F);
  A.X = static_cast<Tio*>(X);
  A.sys = L.sys;
  A.vec64 = L.vec64;
  A.vec32 = L.vec32;
  A.tab64 = L.tab64;
  A.tab32 = L.tab32;
  A.summ = L.summ;
  A.ghost = L.ghost;
  A.Xfwd = static_cast<const Tio*>(Xfwd);
  A.gpart = L.gpart;
  A.iters = L.iters;
  A.max_iter = L.max_iter;
  A.refine_tol = L.refine_tol;
  A.ttab = L.ttab;
  A.ttab_n = L.ttab_n;
  A.corner0 = L.corner0;
  if (L.ev) (void)hipEventRecord(L.ev[0], st);
  // Tile summaries of the refinement path are computed in double (one
  // double sweep costs less than a float solve plus refinement, and the
  // values outside each tile then come out exact in double).
  using Ts = typename std::conditional<REFINE, double, Tc>::type;
  // every multi-tile system of at most 64 tiles: the final pass runs the
  // interface pass itself, and there is no interface launch (except in the
  // refinement of quasi-Toeplitz systems, whose final pass lost more to it
  // than the launch costs)
  const bool inl = L.n_grid > 0 && L.max_ntiles <= 64 && !(REFINE && QUASI);
  // a small series (few tiles in all, at most four per wavefront of a
  // workgroup) of whole tiles with short supports: the final pass computes
  // the summaries too, and the solve is one launch
  const bool p1i = inl && !QUASI && !BWD && L.green && L.green_kf > 0 && L.n_last == 0 &&
                   L.n_beta > 0 && L.n_beta <= 256 && L.max_ntiles <= 4 * SH::NW &&
                   L.green_kf + L.green_kl <= kEndsSplitRows;
  if (L.n_grid > 0) {
    if (L.green) {
      if (L.n_beta > 0 && !p1i) {
        if (L.green_kf > 0)
          launch_beta_ends<SH, Tio>(L, static_cast<const Tio*>(F), st);
        else
          launch_beta<SH, Tio>(L, static_cast<const Tio*>(F), st);
      }
      if (L.n_last > 0) {
        A.items = nullptr;
        launch_tile<SH, Tio, Ts, false, true, false, QUASI>(A, L.n_last, 0, 1, L.wg_per_cu, st);
      }
    } else {
      // support items and swept tiles in one launch (one tile per
      // workgroup), else the support items first
      const bool fuse = L.n_ends > 0 && L.n_p1 > 0 && L.wg_per_cu == 0;
      if (L.n_ends > 0 && !fuse) launch_beta_ends<SH, Tio>(L, static_cast<const Tio*>(F), st);
      A.items = L.p1_items;
      if (L.n_p1 > 0) {
        if (fuse) {
          A.ends_items = L.ends_items;
          A.n_ends = L.n_ends;
          A.gpack = L.gpack;
        }
        launch_tile<SH, Tio, Ts, false, true, false, QUASI>(
            A, L.n_p1, 0, 0, L.wg_per_cu, st, fuse ? (L.n_ends + SH::NW - 1) / SH::NW : 0);
        A.n_ends = 0;
      }
    }
    if (L.ev) (void)hipEventRecord(L.ev[1], st);
    if (!inl) launch_grid<QUASI>(L, F, X, Xfwd, sizeof(Tio) == 4 ? 1 : 0, st);
    if (L.ev) (void)hipEventRecord(L.ev[2], st);
  } else if (L.ev) {
    (void)hipEventRecord(L.ev[1], st);
    (void)hipEventRecord(L.ev[2], st);
  }
  // systems solved whole by one workgroup each (varlen plans)
  if (L.n_sys > 0) launch_sys<SH, Tio, Tc, REFINE, BWD, QUASI>(L, A, st);
  A.items = L.fin_items;
  A.itf_inline = inl ? 1 : 0;
  A.green = L.green;
  A.gkf = L.green_kf;
  A.gkl = L.green_kl;
  // after a first pass the final pass re-reads the tiles the first pass read
  // last while they are still cached: a series runs last-tile-first, a varlen
  // plan's list already starts with the first pass's tiles in reverse
  if (L.n_fin > 0) {
    if constexpr (!BWD && !QUASI) {
      if (p1i) {
        launch_tile<SH, Tio, Tc, REFINE, false, false, false, true>(A, L.n_fin, 0, 0,
                                                                   L.wg_per_cu, st);
        if (L.ev) (void)hipEventRecord(L.ev[3], st);
        return hipGetLastError();
      }
    }
    launch_tile<SH, Tio, Tc, REFINE, false, BWD, QUASI>(
        A, L.n_fin, (L.n_p1 > 0 && !L.fin_items) ? 1 : 0, 0, L.wg_per_cu, st);
  }
  if (L.ev) (void)hipEventRecord(L.ev[3], st);
  return hipGetLastError();
}

template <class SH>
static hipError_t launch_shape(int dtype, bool bwd, const LaunchSet& L, const void* F, void* X,
                               const void* Xfwd, hipStream_t st) {
  // quasi-Toeplitz plans run their own instantiations, so that the corner
  // handling costs the Toeplitz kernels nothing
  auto go = [&](auto quasi) -> hipError_t {
    constexpr bool Q = decltype(quasi)::value;
    switch (dtype) {
      case 0:
        return bwd ? run_solve<SH, double, double, false, true, Q>(L, F, X, Xfwd, st)
                   : run_solve<SH, double, double, false, false, Q>(L, F, X, Xfwd, st);
      case 1:
        return bwd ? run_solve<SH, float, float, false, true, Q>(L, F, X, Xfwd, st)
                   : run_solve<SH, float, float, false, false, Q>(L, F, X, Xfwd, st);
      default:
        return bwd ? run_solve<SH, double, float, true, true, Q>(L, F, X, Xfwd, st)
                   : run_solve<SH, double, float, true, false, Q>(L, F, X, Xfwd, st);
    }
  };
  return L.quasi ? go(std::true_type()) : go(std::false_type());
}

using Shape0 = Shape<kShapes[0].B, kShapes[0].NT, kShapes[0].waves>;
using Shape1 = Shape<kShapes[1].B, kShapes[1].NT, kShapes[1].waves>;
using Shape2 = Shape<kShapes[2].B, kShapes[2].NT, kShapes[2].waves>;
static_assert(kNumShapes == 3, "one Shape alias per entry of kShapes");

// General matrices (series plans, work shape kGeneralShape): first pass over
// the (tile, right-hand side) items, interface pass with per-tile end values,
// final pass in reverse item order (the most recently read tiles first).
template <class SH, typename Tio, typename Tc, bool SUMMARY>
static void launch_gtile(GenArgs<Tio, Tc>& A, int64_t nitems, int reverse, int wg_per_cu,
                         hipStream_t st) {
  auto kern = k_gtile<SH, Tio, Tc, SUMMARY>;
  static int per_cu = resident_per_cu(kern, SH::NT);
  const int64_t cap = grid_cap(per_cu, wg_per_cu);
  A.nitems = nitems;
  A.reverse = reverse;
  hipLaunchKernelGGL(kern, dim3((unsigned)(nitems < cap ? nitems : cap)), dim3(SH::NT), 0, st,
                     A);
}

template <typename Tio, typename Tc>
static hipError_t run_general(const LaunchSet& L, const void* F, void* X, hipStream_t st) {
  using SH = Shape<kShapes[kGeneralShape].B, kShapes[kGeneralShape].NT,
                   kShapes[kGeneralShape].waves>;
  GenArgs<Tio, Tc> A{static_cast<const Tio*>(F), static_cast<Tio*>(X),
                     static_cast<const Tc*>(L.gen_row), static_cast<const Tc*>(L.gen_blk),
                     L.sys, L.gen_M, L.gen_R, (L.gen_M + L.gen_R - 1) / L.gen_R, 0, 0,
                     L.summ, L.ghost};
  if (L.ev) (void)hipEventRecord(L.ev[0], st);
  if (L.n_p1 > 0) {
    if (L.gen_kf > 0) {
      // the rows' supports are short (dominance, Sec. 3.4): one wavefront
      // per tile and right-hand side reads the two ends only
      auto kern = k_beta_ends<SH, Tio>;
      const int64_t nt = L.n_p1 / A.G, n = L.gen_M * nt;
      const int split = L.gen_kf + L.gen_kl > kEndsSplitRows ? 1 : 0;
      BetaEndsArgs<Tio> B{static_cast<const Tio*>(F),
                          L.sys,
                          static_cast<const double*>(L.gen_green),
                          n,
                          split,
                          (int)nt,
                          L.gen_kf,
                          L.gen_kl,
                          L.summ,
                          (int64_t)L.gen_kf + L.gen_kl,
                          nullptr,
                          nullptr};
      int64_t grid = ((split ? 2 : 1) * n + kEndsNW - 1) / kEndsNW;
      if (L.wg_per_cu > 0) {
        static int per_cu = resident_per_cu(kern, kEndsNT);
        const int64_t cap = grid_cap(per_cu, L.wg_per_cu);
        grid = grid < cap ? grid : cap;
      }
      hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kEndsNT), 0, st, B);
    } else if constexpr (sizeof(Tio) == 8) {
      // tile summaries as Green-row dot products over whole tiles
      auto kern = k_gbeta<SH, Tio>;
      static int per_cu = resident_per_cu(kern, kBetaNT);
      const int64_t cap = grid_cap(per_cu, L.wg_per_cu);
      GBetaArgs<Tio> B{static_cast<const Tio*>(F), L.sys, static_cast<const Tio*>(L.gen_green),
                       L.gen_M, L.gen_R, A.G, L.n_p1, L.summ};
      hipLaunchKernelGGL(kern, dim3((unsigned)(L.n_p1 < cap ? L.n_p1 : cap)), dim3(kBetaNT), 0,
                         st, B);
    } else {
      // by sweeps (float plans: whole Green rows would weigh as much as F)
      launch_gtile<SH, Tio, Tc, true>(A, L.n_p1, 0, L.wg_per_cu, st);
    }
    if (L.ev) (void)hipEventRecord(L.ev[1], st);
    launch_grid<false, true>(L, F, X, nullptr, sizeof(Tio) == 4 ? 1 : 0, st);
    if (L.ev) (void)hipEventRecord(L.ev[2], st);
  } else if (L.ev) {
    (void)hipEventRecord(L.ev[1], st);
    (void)hipEventRecord(L.ev[2], st);
  }
  launch_gtile<SH, Tio, Tc, false>(A, L.n_fin, L.n_p1 > 0 ? 1 : 0, L.wg_per_cu, st);
  if (L.ev) (void)hipEventRecord(L.ev[3], st);
  return hipGetLastError();
}

hipError_t launch_general_grad(int f32, const void* gF, const void* X, int64_t n, int64_t M,
                               double* g, hipStream_t st) {
  const unsigned grid = (unsigned)((n + kGridNT - 1) / kGridNT);
  if (f32)
    hipLaunchKernelGGL(k_ggrad<float>, dim3(grid), dim3(kGridNT), 0, st,
                       static_cast<const float*>(gF), static_cast<const float*>(X), n, M, g);
  else
    hipLaunchKernelGGL(k_ggrad<double>, dim3(grid), dim3(kGridNT), 0, st,
                       static_cast<const double*>(gF), static_cast<const double*>(X), n, M, g);
  return hipGetLastError();
}

hipError_t launch_solve(int dtype, bool bwd, const LaunchSet& L, const void* F, void* X,
                        const void* Xfwd, hipStream_t st) {
  if (L.general)
    return dtype == 1 ? run_general<float, float>(L, F, X, st)
                      : run_general<double, double>(L, F, X, st);
  switch (L.shape) {
    case 1: return launch_shape<Shape1>(dtype, bwd, L, F, X, Xfwd, st);
    case 2: return launch_shape<Shape2>(dtype, bwd, L, F, X, Xfwd, st);
    default: return launch_shape<Shape0>(dtype, bwd, L, F, X, Xfwd, st);
  }
}

int sys_wg_capacity(int shape, int dtype, int wg_per_cu, int quasi) {
  switch (shape) {
    case 1:
      return quasi ? sys_capacity<Shape1, true>(dtype, wg_per_cu)
                   : sys_capacity<Shape1, false>(dtype, wg_per_cu);
    case 2:
      return quasi ? sys_capacity<Shape2, true>(dtype, wg_per_cu)
                   : sys_capacity<Shape2, false>(dtype, wg_per_cu);
    default:
      return quasi ? sys_capacity<Shape0, true>(dtype, wg_per_cu)
                   : sys_capacity<Shape0, false>(dtype, wg_per_cu);
  }
}

hipError_t launch_gt_reduce(const double* gpart, const SysDesc* sys, int64_t nsys,
                            int64_t nparts, int varlen, int ncomp, double* gt, hipStream_t st) {
  const unsigned grid = varlen ? (unsigned)((nsys + kGridNT - 1) / kGridNT) : 1u;
  hipLaunchKernelGGL(k_gt_reduce, dim3(grid), dim3(kGridNT), 0, st, gpart, sys, nsys, nparts,
                     varlen, ncomp, gt);
  return hipGetLastError();
}

}  // namespace tdt

// ---------------------------------------------------------------------------
// Solve without allocation: the workspace is a static device array of this
// file instead of the plan's.  Layout in doubles: tile summaries [slot][2],
// values outside the tiles [slot][2], the segment-merge suffixes [slot][3],
// then one adjoint partial-sum slot (passed, never used by a forward solve).
// No part of it needs to start at zero: a solve reads only what it wrote
// earlier in the same call (the one unconditional read, slot 0 of the values
// outside a one-tile system, is discarded).
// ---------------------------------------------------------------------------
#include <mutex>

#include "tdt.h"

namespace {
constexpr int64_t kScratchSlots = (int64_t)1 << 17;
constexpr int64_t kScratchDoubles = 7 * kScratchSlots + tdt::kGradN;   // 7 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

// The array's device address on the current device, looked up once per
// device (the host-side symbol is not a device address).
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

double* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" tdt_status_t tdt_solve_noalloc(tdt_plan_t plan, const void* F, void* X, int64_t M,
                                          hipStream_t stream) {
  tdt::LaunchSet L;
  int64_t slots = 0;
  int dtype = 0;
  const int st = tdt::series_solve_prepare(plan, F, X, M, L, slots, dtype);
  if (st != TDT_OK) return (tdt_status_t)st;
  if (slots > kScratchSlots) return TDT_ERR_INVALID_ARG;
  double* base = scratch_on_current_device();
  if (!base) return TDT_ERR_HIP;
  L.summ = base;
  L.ghost = base + 2 * kScratchSlots;
  L.gscr = base + 4 * kScratchSlots;
  L.gpart = base + 7 * kScratchSlots;
  L.ev = nullptr;
  return tdt::launch_solve(dtype, false, L, F, X, nullptr, stream) == hipSuccess ? TDT_OK
                                                                                : TDT_ERR_HIP;
}
