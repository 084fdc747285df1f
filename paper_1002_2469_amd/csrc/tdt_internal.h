// tdt_internal.h -- layout shared by the host plan code and the gfx950 kernels.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

struct tdt_plan_s;

namespace tdt {

// Work shape of the tile kernels: B contiguous unknowns per lane (the
// paper's sub-vector U_m of Sec. 2.1 held by one processing element), NT
// lanes per workgroup, and the tile of L = B*NT unknowns one workgroup holds
// on chip at once.  A plan is built for one shape; the shapes below are
// compiled in and the autotuner may pick any of them.
struct ShapeInfo {
  int B, NT, waves;   // waves: occupancy (waves per SIMD) the kernels target
};
constexpr ShapeInfo kShapes[] = {{16, 512, 4}, {8, 512, 4}, {16, 256, 4}};
constexpr int kNumShapes = 3;
constexpr int kMaxB = 16;
constexpr int kMaxNT = 512;
constexpr int kMinWavesPerSimd = 4;    // occupancy of the other kernels
// varlen plans: systems of at most this many tiles are solved whole by one
// workgroup each (default; the plan option can lower it, or raise it up to
// kSysMaxTiles)
constexpr int kSysMaxTilesDefault = 8;
constexpr int kSysMaxTiles = 16;

// One Toeplitz system as the kernels see it.  All constants are double; the
// float kernels round them on load.  Segment end values use the order
// (phi_first, phi_last, chi_first, chi_last): phi is the segment's response
// to a unit value just left of it, chi to a unit value just right of it.
struct SysDesc {
  double a, b, c;        // t_-1 (sub-diagonal), t_0, t_1 (super-diagonal)
  int64_t n;             // order of the system
  int64_t off;           // element offset of the system (varlen) or 0 (series)
  int32_t ntiles;        // number of tiles (last one may be partial)
  int32_t slot0;         // first workspace slot of the system (varlen)
  int32_t cidx;          // index of the block-constant vectors of this system
  int32_t fslot0;         // first adjoint partial-sum slot of the system (varlen)
  double tail_pf;        // phi_first of the last block of the system (length (n-1)%B+1)
  double blk[4];         // end values of a full block (length B)
  double tileK[4];       // end values of a full tile (length L)
  double ltileK[4];      // end values of the last tile (its real length)
  // Workspace slots of a multi-tile system are "run-interleaved" for the
  // interface pass, whose thread j walks tiles j*tr .. j*tr+tr-1: tile t
  // lives at slot (t % tr) * tq + t / tr, so that the r-th access of
  // consecutive threads touches consecutive slots.
  int32_t tr;            // tiles per thread of the interface pass
  int32_t tq;            // threads of the interface pass in use, ceil(ntiles / tr)
  int32_t tslots;        // slots per right-hand side (tq * tr)
  // Quasi-Toeplitz systems (t0+psi and t0+chi in the first and last diagonal
  // entry): the tiles cover the n = N - 2 inner rows, which start one row
  // after the system's first row; the two corner rows are one-row segments
  // at both ends of the interface pass.
  int32_t quasi;         // 1 for a quasi-Toeplitz system
  int64_t stride;        // rows between right-hand sides of a series (N)
  double tail_pl;        // phi_last and chi_first of the system's last block
  double tail_cf;        //   (tile summaries of quasi-Toeplitz systems)
  // corner constants: [0] 1/(t0+psi); [1] -t1/(t0+psi), the first corner's
  // response to a unit value right of it (and its beta); [2] 1/(t0+chi);
  // [3] -t_-1/(t0+chi), the last corner's response to a unit value left of
  // it; [4] beta of the last inner tile; [5] 1/(1 - [3] [4])
  double qc[6];
  // varlen plans: the supports of a full tile's two Green rows (gkf leading
  // entries of the first row, then gkl trailing entries of the last, at
  // goff of the plan's packed array), or gkf = gkl = 0 (summaries by sweeps);
  // glast = 1: a shorter last tile has the same entries (its rows under the
  // supports meet only settled pivots) and is summarised from them too
  int64_t goff;
  int32_t gkf, gkl;
  int32_t glast;
  // the per-position table's entries repeat from position tfix on (its
  // recurrence reached its fixed point): lanes past it read entry tfix, so
  // a workgroup's table loads touch a few cache lines (0: every lane reads
  // its own entry)
  int32_t tfix;
};
// First pass from the Green rows' supports: supports longer than this many
// rows (head and tail together) take a wavefront per tile end, shorter ones
// a wavefront per tile.  Varlen items carry the part of the tile in the bits
// of the tile index from kEndsPartShift up: 0 both ends, 1 head, 2 tail.
constexpr int kEndsSplitRows = 256;
constexpr int kEndsPartShift = 24;

// Slot of tile t of a system: a varlen plan adds the system's slot0; a
// series plan uses tslots slots per right-hand side m.
__host__ __device__ inline int64_t tile_slot(const SysDesc& S, int64_t m, int t, bool varlen) {
  const int64_t pos = (int64_t)(t % S.tr) * S.tq + t / S.tr;
  return varlen ? (int64_t)S.slot0 + pos : m * S.tslots + pos;
}

// Per-system table over the NT block positions of a tile: beta_{m-1} (the
// coefficient that carries the next block's first unknown into block m-1's
// last one, from the left-to-right elimination) and 1/(1 - phi_first beta_{m-1}).
enum { kTabBeta = 0, kTabInvD = 1, kTabN = 2 };

// Per-system block vectors, B each, in this order.
//   IU: 1/u_i (inverse pivots), AIU: t_-1/u_i, CP: t_1/u_i, PHI, CHI: the
//   block's responses to unit values just left / right of it.
enum { kVecIU = 0, kVecCP = 1, kVecPHI = 2, kVecCHI = 3, kVecAIU = 4, kVecN = 5 };

// General (per-row) matrices: per row of a block, the block-local LU
// (1/u_i, a_i/u_i, c_i/u_i), laid out [tile][value][row in block][lane]; per
// block, its end values, beta_{m-1} and 1/(1 - pf beta_{m-1}) of the in-tile
// elimination, laid out [tile][value][lane].
enum { kGenIU = 0, kGenAIU = 1, kGenCP = 2, kGenRowN = 3 };
enum { kGenPF = 0, kGenPL = 1, kGenCF = 2, kGenBP = 3, kGenID = 4, kGenBlkN = 5 };

// Everything one solve launch sequence needs (device pointers).
struct LaunchSet {
  const SysDesc* sys;
  const double* vec64;
  const float* vec32;
  int shape;               // index into kShapes
  const double* tab64;     // per-position table [ncidx][2][NT]
  const float* tab32;
  const int2* p1_items;    // varlen: (system, tile) of the first pass; null for a series
  const int2* fin_items;   // varlen: (system, tile) of the final pass
  const int* grid_items;   // varlen: systems with more than one tile
  const int* sys_items;    // varlen: systems solved whole by one workgroup each,
  const int* sys_bins;     //   grouped by workgroup: bin b = sys_items[sys_bins[b] ..
  int64_t n_bins;          //   sys_bins[b+1]), one workgroup per bin
  int64_t n_p1, n_fin, n_grid, n_sys;
  // series plans with more than one tile: the first pass is a dot product of
  // every full tile with the tile's Green rows (n_beta items), plus the
  // sweep-based pass over the partial last tile of each right-hand side
  // (n_last items); varlen plans use the sweep-based pass over p1_items
  const double* green;     // [2][L] or null
  int green_kf, green_kl;  // supports of the Green rows (multiples of 64), or 0: whole tile
  int64_t n_beta, n_last;
  // varlen plans: full tiles whose summaries come from their system's Green
  // row supports (packed entries at gpack + goff of the system)
  const int2* ends_items;
  int64_t n_ends;
  const double* gpack;
  int nfull;
  int max_ntiles;          // most tiles of any system (selects the interface kernel)
  int chunks;              // series of 2049..16384 tiles: interface pass in chunks of 64 tiles
  const double* ttab;      // per tile position: beta_{t-1}, 1/(1 - Pf beta_{t-1}) ([2][ttab_n])
  int64_t ttab_n;
  double* summ;
  double* ghost;
  double* gscr;
  double* gpart;
  int64_t corner0;        // series, quasi-Toeplitz: first corner t-gradient slot
  int quasi;              // the plan's systems are quasi-Toeplitz
  // general (per-row) matrix, series plans: per-row LU and per-block constants
  // in the compute precision, per-tile end values; gen_M right-hand sides
  int general;
  const void* gen_row;
  const void* gen_blk;
  const double* gen_tK;
  const void* gen_green;   // Green rows of the tiles, double (the plan's dggreen)
  int gen_kf, gen_kl;      // double plans: the rows' supports over all tiles, or 0
  int64_t gen_M;
  int gen_R;               // right-hand sides per item (the item counts below are per item)
  int* iters;
  int max_iter;
  double refine_tol;
  int wg_per_cu;           // cap of persistent workgroups per CU (0: as many as fit)
  hipEvent_t* ev;          // measurement: 4 events (before pass 1, after pass 1,
                           // after the interface pass, after the final pass) or null
};

// The argument checks of a forward solve of a series plan (those of
// tdt_solve) and its launch set without workspace; slots = the tile slots
// its workspace needs, dtype = the plan's.  Returns a tdt_status_t.
int series_solve_prepare(tdt_plan_s* p, const void* F, void* X, int64_t M, LaunchSet& L,
                         int64_t& slots, int& dtype);
// dtype: 0 double, 1 float, 2 float sweeps with double refinement.
hipError_t launch_solve(int dtype, bool bwd, const LaunchSet& L, const void* F, void* X,
                        const void* Xfwd, hipStream_t st);
// Workgroups of the whole-system kernel that are resident at once (the
// plan spreads its systems over this many lists).
int sys_wg_capacity(int shape, int dtype, int wg_per_cu, int quasi);
// Partial t-gradient sums per tile of the adjoint: (t_-1, t_0, t_1, psi, chi).
constexpr int kGradN = 5;
// Sums the partials per system (varlen) or over all (series) into gt,
// ncomp (3, or 5 for quasi-Toeplitz plans) values per system.
hipError_t launch_gt_reduce(const double* gpart, const SysDesc* sys, int64_t nsys,
                            int64_t nparts, int varlen, int ncomp, double* gt, hipStream_t st);
// General matrices: the work shape their kernels are built for (index into
// kShapes), and the entry gradients [3][n] from the adjoint solution gF and
// the forward solution X ([M][n], floats if f32).
constexpr int kGeneralShape = 1;
hipError_t launch_general_grad(int f32, const void* gF, const void* X, int64_t n, int64_t M,
                               double* g, hipStream_t st);

}  // namespace tdt
