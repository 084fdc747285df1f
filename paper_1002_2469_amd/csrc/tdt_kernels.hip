// tdt_kernels.hip -- gfx950 kernels of the partitioned dichotomy solve.
//
// Formulation (Sec. 2.2-2.3 of the paper, restated for one GPU).  The system
// is cut into blocks of kB consecutive unknowns, one block per lane; 256
// lanes (4 wavefronts) form a workgroup tile of 8192 unknowns; a long system
// is a sequence of tiles.  Every block of a Toeplitz matrix is the same
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
// problems -- the dichotomy step of Sec. 2.2 (eqs. (4)-(6)).  The same 2x2
// elimination with zero outside values merges the two half summaries into the
// summary of the whole (the segment's own "beta" of eq. (10): its first and
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

#include "tdt_internal.h"

namespace tdt {

template <typename T>
struct Seg {
  T yf, yl, pf, pl, cf, cl;
};

template <typename T>
__device__ __forceinline__ Seg<T> seg_zero() {
  return Seg<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
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
// the values just outside its own wavefront from the tile's outside values.
// Returns the tile summary.  Contains one barrier (all threads must call).
template <typename T>
__device__ __forceinline__ Seg<T> wg_level(const Seg<T>& pre, T (*wsum)[6], T XLt, T XRt,
                                           T& XLw, T& XRw) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) {
    wsum[w][0] = pre.yf; wsum[w][1] = pre.yl; wsum[w][2] = pre.pf;
    wsum[w][3] = pre.pl; wsum[w][4] = pre.cf; wsum[w][5] = pre.cl;
  }
  __syncthreads();
  Seg<T> W[kNW];
#pragma unroll
  for (int k = 0; k < kNW; ++k)
    W[k] = Seg<T>{wsum[k][0], wsum[k][1], wsum[k][2], wsum[k][3], wsum[k][4], wsum[k][5]};
  Seg<T> P[kNW], Q[kNW];   // P[k] = W[0..k], Q[k] = W[k..kNW-1]
  P[0] = W[0];
#pragma unroll
  for (int k = 1; k < kNW; ++k) P[k] = seg_merge(P[k - 1], W[k]);
  Q[kNW - 1] = W[kNW - 1];
#pragma unroll
  for (int k = kNW - 2; k >= 0; --k) Q[k] = seg_merge(W[k], Q[k + 1]);
  XLw = XLt;
  XRw = XRt;
#pragma unroll
  for (int k = 0; k + 1 < kNW; ++k) {   // junction between waves k and k+1
    T xk, xk1;
    junction(P[k].yl, P[k].pl, P[k].cl, Q[k + 1].yf, Q[k + 1].pf, Q[k + 1].cf, XLt, XRt, xk, xk1);
    if (w == k) XRw = xk1;
    if (w == k + 1) XLw = xk;
  }
  return P[kNW - 1];
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

// Per-system constants in compute precision.
template <typename Tc>
struct Consts {
  const Tc* __restrict__ iu;
  const Tc* __restrict__ cp;
  const Tc* __restrict__ phi;
  const Tc* __restrict__ chi;
  Tc a;
  Tc bpf, bpl, bcf, bcl;
  Tc tail_pf;
};

// Solve the tile's local problem for this lane's block q (in: right-hand
// side, out: solution) given the values just outside the tile.  len: real
// rows of the lane's block (kB full, 1..kB-1 last block, 0 past the end).
// If tile_seg is non-null the tile summary is returned there and the
// correction is skipped.  One workgroup barrier inside.
template <typename Tc>
__device__ __forceinline__ void tile_solve(Tc (&q)[kB], int len, Tc XLt, Tc XRt,
                                           const Consts<Tc>& K, Tc (*wsum)[6],
                                           Seg<Tc>* tile_seg) {
  const bool tail = len > 0 && len < kB;
  const bool wave_tail = __ballot(tail) != 0;
  // local Thomas sweep with the shared multipliers (T_B^{-1} q)
  q[0] *= K.iu[0];
  if (!wave_tail) {
#pragma unroll
    for (int i = 1; i < kB; ++i) q[i] = (q[i] - K.a * q[i - 1]) * K.iu[i];
  } else {
#pragma unroll
    for (int i = 1; i < kB; ++i) {
      const Tc d = (q[i] - K.a * q[i - 1]) * K.iu[i];
      q[i] = i < len ? d : Tc(0);
    }
  }
#pragma unroll
  for (int i = kB - 2; i >= 0; --i) q[i] -= K.cp[i] * q[i + 1];

  Seg<Tc> own = seg_zero<Tc>();
  if (len == kB) {
    own = Seg<Tc>{q[0], q[kB - 1], K.bpf, K.bpl, K.bcf, K.bcl};
  } else if (len > 0) {
    own = Seg<Tc>{q[0], Tc(0), K.tail_pf, Tc(0), Tc(0), Tc(0)};
  }
  Seg<Tc> pre, suf;
  wave_scan(own, pre, suf);
  Tc XLw, XRw;
  const Seg<Tc> ts = wg_level(pre, wsum, XLt, XRt, XLw, XRw);
  if (tile_seg) {
    *tile_seg = ts;
    return;
  }
  Tc xl, xr;
  lane_ghosts(pre, suf, XLw, XRw, xl, xr);
  if (len == kB) {
#pragma unroll
    for (int i = 0; i < kB; ++i) q[i] += xl * K.phi[i] + xr * K.chi[i];
  } else if (len > 0) {
    // last block: re-sweep T_Bt x = q_orig - t_-1 xl e_0 in place, recovering
    // the forward-sweep values d_i = y_i + cp_i y_{i+1} from y (xr is 0 here:
    // the next row is past the end of the system)
    Tc delta = -K.a * xl * K.iu[0];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const Tc ynext = i + 1 < kB ? q[i + 1] : Tc(0);
      const Tc dp = q[i] + K.cp[i] * ynext + delta;
      q[i] = i < len ? dp : Tc(0);
      if (i + 1 < kB) delta = -K.a * delta * K.iu[i + 1];
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
  const int2* __restrict__ items;     // varlen: (system, tile) per workgroup; null for a series
  double* __restrict__ summ;          // [slot][2] tile summaries (y_first, y_last)
  const double* __restrict__ ghost;   // [slot][2] values just outside each tile
  const Tio* __restrict__ Xfwd;       // adjoint: forward solution
  double* __restrict__ gpart;         // adjoint: [final slot][3] partial t-gradients
  int* __restrict__ iters;            // refinement: max iterations used (atomicMax)
  int max_iter;
  double refine_tol;
};

struct ItemInfo {
  int s, t;
  int64_t m;
};

__device__ __forceinline__ ItemInfo decode_item(const int2* items, const SysDesc* sys,
                                                int64_t it) {
  ItemInfo r;
  if (items) {
    const int2 v = items[it];
    r.s = v.x; r.t = v.y; r.m = 0;
  } else {
    const int nt = sys[0].ntiles;
    r.s = 0; r.m = it / nt; r.t = (int)(it - r.m * nt);
  }
  return r;
}

template <typename Tc>
__device__ __forceinline__ Consts<Tc> load_consts(const SysDesc& S, const double* vec64,
                                                  const float* vec32) {
  Consts<Tc> K;
  const Tc* v;
  if constexpr (sizeof(Tc) == 8)
    v = reinterpret_cast<const Tc*>(vec64) + (int64_t)S.cidx * kVecN * kB;
  else
    v = reinterpret_cast<const Tc*>(vec32) + (int64_t)S.cidx * kVecN * kB;
  K.iu = v + kVecIU * kB;
  K.cp = v + kVecCP * kB;
  K.phi = v + kVecPHI * kB;
  K.chi = v + kVecCHI * kB;
  K.a = (Tc)S.a;
  K.bpf = (Tc)S.blk[0]; K.bpl = (Tc)S.blk[1]; K.bcf = (Tc)S.blk[2]; K.bcl = (Tc)S.blk[3];
  K.tail_pf = (Tc)S.tail_pf;
  return K;
}

// Workgroup max of two non-negative values (fixed order, all threads get it).
__device__ __forceinline__ void wg_max2(double& u, double& v, double (*red)[4]) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    u = fmax(u, __shfl_xor(u, d, 64));
    v = fmax(v, __shfl_xor(v, d, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { red[w][0] = u; red[w][1] = v; }
  __syncthreads();
  u = red[0][0]; v = red[0][1];
#pragma unroll
  for (int k = 1; k < kNW; ++k) { u = fmax(u, red[k][0]); v = fmax(v, red[k][1]); }
}

// One workgroup per tile.
//   SUMMARY = true : first pass over a tile of a multi-tile system: writes the
//                    tile's (y_first, y_last) of its zero-boundary problem.
//   SUMMARY = false: solves the tile given the values just outside it (zero
//                    for a one-tile system) and stores X.
//   REFINE         : Tio = double data, Tc = float sweeps; residual and update
//                    in double, repeated until converged.
//   BWD            : also accumulates the t-gradient partial sums against the
//                    forward solution Xfwd (the tile solves T^T gF = gX).
template <typename Tio, typename Tc, bool REFINE, bool SUMMARY, bool BWD>
__global__ __launch_bounds__(kNT) void k_tile(TileArgs<Tio> A) {
  constexpr int RP = kB + 16 / (int)sizeof(Tio);   // padded LDS row pitch
  __shared__ __align__(16) Tio lds[kNT * RP];
  __shared__ Tc wsum[kNW][6];
  __shared__ double red[kNW][4];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const ItemInfo I = decode_item(A.items, A.sys, blockIdx.x);
  const SysDesc& S = A.sys[I.s];
  const int64_t n = S.n;
  const int64_t t0 = (int64_t)I.t * kTile;
  const int64_t base = S.off + I.m * n + t0;
  const int tl = (int)(n - t0 < kTile ? n - t0 : kTile);
  const int64_t slot = A.items ? (int64_t)S.slot0 + I.t : I.m * S.ntiles + I.t;
  double XLt = 0.0, XRt = 0.0;
  if (!SUMMARY && S.ntiles > 1) {
    XLt = A.ghost[2 * slot];
    XRt = A.ghost[2 * slot + 1];
  }

  // coalesced load, transposed through LDS into one row of kB per lane
#pragma unroll 8
  for (int j = 0; j < kB; ++j) {
    const int e = j * kNT + tid;
    const Tio v = e < tl ? A.F[base + e] : Tio(0);
    lds[(e / kB) * RP + (e % kB)] = v;
  }
  __syncthreads();

  const Consts<Tc> K = load_consts<Tc>(S, A.vec64, A.vec32);
  const int len = tl - tid * kB >= kB ? kB : (tl - tid * kB > 0 ? tl - tid * kB : 0);
  Tio* myrow = lds + tid * RP;

  if constexpr (!REFINE) {
    Tc q[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) q[i] = (Tc)myrow[i];
    if constexpr (SUMMARY) {
      Seg<Tc> ts;
      tile_solve(q, len, Tc(0), Tc(0), K, wsum, &ts);
      if (tid == 0) {
        A.summ[2 * slot] = (double)ts.yf;
        A.summ[2 * slot + 1] = (double)ts.yl;
      }
      return;
    } else {
      tile_solve(q, len, (Tc)XLt, (Tc)XRt, K, wsum, (Seg<Tc>*)nullptr);
#pragma unroll
      for (int i = 0; i < kB; ++i) myrow[i] = (Tio)q[i];
    }
  } else {
    // iterative refinement: x = 0; repeat r = f - T x (double, with the
    // tile's outside values), d = solve_float(r) with zero outside values,
    // x += d (double)
    __shared__ double edge[kNW][2];
    const double a = S.a, b = S.b, c = S.c;
    double x[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) x[i] = 0.0;
    double dprev = 0.0;
    int it = 0;
    for (;;) {
      // neighbours of this lane's block
      if (lane == 0) edge[w][0] = x[0];
      if (lane == 63) edge[w][1] = x[kB - 1];
      __syncthreads();
      double xm = __shfl_up(x[kB - 1], 1, 64);
      double xp = __shfl_down(x[0], 1, 64);
      if (lane == 0) xm = w == 0 ? XLt : edge[w - 1][1];
      if (lane == 63) xp = w == kNW - 1 ? XRt : edge[w + 1][0];
      Tc q[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const double left = i == 0 ? xm : x[i - 1];
        const double right = i + 1 < kB ? x[i + 1] : xp;
        const double r = (double)myrow[i] - (b * x[i] + a * left + c * right);
        q[i] = i < len ? (Tc)r : Tc(0);
      }
      tile_solve(q, len, Tc(0), Tc(0), K, wsum, (Seg<Tc>*)nullptr);
      double dmax = 0.0, xmax = 0.0;
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        x[i] += (double)q[i];
        dmax = fmax(dmax, fabs((double)q[i]));
        xmax = fmax(xmax, fabs(x[i]));
      }
      wg_max2(dmax, xmax, red);
      ++it;
      // stop when the next update is predicted below tol (contraction
      // estimate dmax/dprev), when updates stop shrinking, or at the cap
      bool stop = it >= A.max_iter || dmax == 0.0;
      if (it >= 2) {
        const double rho = dmax / dprev;
        stop = stop || dmax * rho <= A.refine_tol * xmax || rho > 0.9;
      }
      dprev = dmax;
      if (stop) break;
    }
    if (tid == 0 && A.iters) atomicMax(A.iters, it);
    if constexpr (SUMMARY) {
      if (tid == 0) A.summ[2 * slot] = x[0];
      __syncthreads();
      if (tid == kNT - 1) A.summ[2 * slot + 1] = tl == kTile ? x[kB - 1] : 0.0;
      return;
    } else {
      __syncthreads();   // every lane is done reading f from LDS
#pragma unroll
      for (int i = 0; i < kB; ++i) myrow[i] = (Tio)x[i];
    }
  }

  if constexpr (!SUMMARY) {
    __syncthreads();
    double s0 = 0.0, s1 = 0.0, sm1 = 0.0;
#pragma unroll 8
    for (int j = 0; j < kB; ++j) {
      const int e = j * kNT + tid;
      if (e < tl) {
        const Tio g = lds[(e / kB) * RP + (e % kB)];
        A.X[base + e] = g;
        if constexpr (BWD) {
          const int64_t gi = t0 + e;   // row in the system
          const double xe = (double)A.Xfwd[base + e];
          const double xn = gi + 1 < n ? (double)A.Xfwd[base + e + 1] : 0.0;
          const double xq = gi > 0 ? (double)A.Xfwd[base + e - 1] : 0.0;
          s0 += (double)g * xe;
          s1 += (double)g * xn;
          sm1 += (double)g * xq;
        }
      }
    }
    if constexpr (BWD) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        s0 += __shfl_xor(s0, d, 64);
        s1 += __shfl_xor(s1, d, 64);
        sm1 += __shfl_xor(sm1, d, 64);
      }
      __syncthreads();
      if (lane == 0) { red[w][0] = sm1; red[w][1] = s0; red[w][2] = s1; }
      __syncthreads();
      if (tid == 0) {
        double u = 0.0, v = 0.0, z = 0.0;
        for (int k = 0; k < kNW; ++k) { u += red[k][0]; v += red[k][1]; z += red[k][2]; }
        const int64_t fs = A.items ? (int64_t)S.fslot0 + I.t : I.m * S.ntiles + I.t;
        A.gpart[3 * fs + 0] = -u;
        A.gpart[3 * fs + 1] = -v;
        A.gpart[3 * fs + 2] = -z;
      }
    }
  }
}

struct GridArgs {
  const SysDesc* __restrict__ sys;
  const int* __restrict__ gitems;     // varlen: system of each workgroup; null for a series
  const double* __restrict__ summ;
  double* __restrict__ ghost;
  double* __restrict__ gscr;          // [slot][3] suffix (y_first, phi_first, chi_first)
};

// Interface pass across the tiles of one system (one workgroup per system
// and right-hand side): every thread folds a run of consecutive tile
// summaries, the runs are combined by the same wavefront scans and LDS level
// as inside a tile, and each thread then walks its run left to right to give
// every tile the values just outside it.
__global__ __launch_bounds__(kNT) void k_grid(GridArgs A) {
  __shared__ double wsum[kNW][6];
  const int tid = threadIdx.x;
  int s = 0;
  int64_t slot0;
  if (A.gitems) {
    s = A.gitems[blockIdx.x];
    slot0 = A.sys[s].slot0;
  } else {
    slot0 = (int64_t)blockIdx.x * A.sys[0].ntiles;
  }
  const SysDesc& S = A.sys[s];
  const int P = S.ntiles;
  const double* summ = A.summ + 2 * slot0;
  double* ghost = A.ghost + 2 * slot0;
  double* scr = A.gscr + 3 * slot0;
  const int ch = (P + kNT - 1) / kNT;
  const int ta = tid * ch < P ? tid * ch : P;
  const int tb = ta + ch < P ? ta + ch : P;

  auto tile_seg = [&](int t) {
    const double* k = t + 1 < P ? S.tileK : S.ltileK;
    return Seg<double>{summ[2 * t], summ[2 * t + 1], k[0], k[1], k[2], k[3]};
  };

  Seg<double> acc = seg_zero<double>();
  for (int t = tb - 1; t >= ta; --t) {
    const Seg<double> ts = tile_seg(t);
    acc = t == tb - 1 ? ts : seg_merge(ts, acc);
    scr[3 * t] = acc.yf;
    scr[3 * t + 1] = acc.pf;
    scr[3 * t + 2] = acc.cf;
  }
  Seg<double> pre, suf;
  wave_scan(acc, pre, suf);
  double XLw, XRw;
  wg_level(pre, wsum, 0.0, 0.0, XLw, XRw);
  double xl, xr;
  lane_ghosts(pre, suf, XLw, XRw, xl, xr);
  for (int t = ta; t < tb; ++t) {
    if (t == tb - 1) {
      ghost[2 * t] = xl;
      ghost[2 * t + 1] = xr;
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

// Deterministic second stage of the t-gradient sums: series plans sum all
// partials (one workgroup, fixed tree); varlen plans sum each system's tiles
// in order (one thread per system).
__global__ __launch_bounds__(kNT) void k_gt_reduce(const double* __restrict__ gpart,
                                                   const SysDesc* __restrict__ sys,
                                                   int64_t nsys, int64_t nparts, int varlen,
                                                   double* __restrict__ gt) {
  if (varlen) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s >= nsys) return;
    const int64_t f0 = sys[s].fslot0;
    double u = 0.0, v = 0.0, z = 0.0;
    for (int t = 0; t < sys[s].ntiles; ++t) {
      u += gpart[3 * (f0 + t)];
      v += gpart[3 * (f0 + t) + 1];
      z += gpart[3 * (f0 + t) + 2];
    }
    gt[3 * s] = u; gt[3 * s + 1] = v; gt[3 * s + 2] = z;
    return;
  }
  __shared__ double red[kNT][3];
  double u = 0.0, v = 0.0, z = 0.0;
  for (int64_t k = threadIdx.x; k < nparts; k += kNT) {
    u += gpart[3 * k]; v += gpart[3 * k + 1]; z += gpart[3 * k + 2];
  }
  red[threadIdx.x][0] = u; red[threadIdx.x][1] = v; red[threadIdx.x][2] = z;
  __syncthreads();
  for (int h = kNT / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[threadIdx.x][0] += red[threadIdx.x + h][0];
      red[threadIdx.x][1] += red[threadIdx.x + h][1];
      red[threadIdx.x][2] += red[threadIdx.x + h][2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { gt[0] = red[0][0]; gt[1] = red[0][1]; gt[2] = red[0][2]; }
}

}  // namespace tdt

// ---------------------------------------------------------------------------
// Launch helpers used by the host API (C++ linkage, internal).
// ---------------------------------------------------------------------------
namespace tdt {


template <typename Tio, typename Tc, bool REFINE, bool BWD>
static hipError_t run_solve(const LaunchSet& L, const void* F, void* X, const void* Xfwd,
                            hipStream_t st) {
  TileArgs<Tio> A;
  A.F = static_cast<const Tio*>(F);
  A.X = static_cast<Tio*>(X);
  A.sys = L.sys;
  A.vec64 = L.vec64;
  A.vec32 = L.vec32;
  A.summ = L.summ;
  A.ghost = L.ghost;
  A.Xfwd = static_cast<const Tio*>(Xfwd);
  A.gpart = L.gpart;
  A.iters = L.iters;
  A.max_iter = L.max_iter;
  A.refine_tol = L.refine_tol;
  if (L.n_p1 > 0) {
    A.items = L.p1_items;
    hipLaunchKernelGGL((k_tile<Tio, Tc, REFINE, true, false>), dim3((unsigned)L.n_p1),
                       dim3(kNT), 0, st, A);
    GridArgs G{L.sys, L.grid_items, L.summ, L.ghost, L.gscr};
    hipLaunchKernelGGL(k_grid, dim3((unsigned)L.n_grid), dim3(kNT), 0, st, G);
  }
  A.items = L.fin_items;
  hipLaunchKernelGGL((k_tile<Tio, Tc, REFINE, false, BWD>), dim3((unsigned)L.n_fin), dim3(kNT),
                     0, st, A);
  return hipGetLastError();
}

hipError_t launch_solve(int dtype, bool bwd, const LaunchSet& L, const void* F, void* X,
                        const void* Xfwd, hipStream_t st) {
  switch (dtype) {
    case 0:
      return bwd ? run_solve<double, double, false, true>(L, F, X, Xfwd, st)
                 : run_solve<double, double, false, false>(L, F, X, Xfwd, st);
    case 1:
      return bwd ? run_solve<float, float, false, true>(L, F, X, Xfwd, st)
                 : run_solve<float, float, false, false>(L, F, X, Xfwd, st);
    default:
      return bwd ? run_solve<double, float, true, true>(L, F, X, Xfwd, st)
                 : run_solve<double, float, true, false>(L, F, X, Xfwd, st);
  }
}

hipError_t launch_gt_reduce(const double* gpart, const SysDesc* sys, int64_t nsys,
                            int64_t nparts, int varlen, double* gt, hipStream_t st) {
  const unsigned grid = varlen ? (unsigned)((nsys + kNT - 1) / kNT) : 1u;
  hipLaunchKernelGGL(k_gt_reduce, dim3(grid), dim3(kNT), 0, st, gpart, sys, nsys, nparts, varlen,
                     gt);
  return hipGetLastError();
}

}  // namespace tdt
