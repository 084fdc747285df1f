// tdt_internal.h -- layout shared by the host plan code and the gfx950 kernels.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace tdt {

// Block of contiguous unknowns owned by one lane (the paper's sub-vector U_m
// of Sec. 2.1 held by one processing element), threads per workgroup, and the
// tile: the unknowns one workgroup holds on chip at once.
constexpr int kB = 32;
constexpr int kNT = 256;
constexpr int kNW = kNT / 64;          // wavefronts per workgroup
constexpr int kTile = kB * kNT;        // 8192 unknowns per tile

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
  double tail_pf;        // phi_first of the last block of the system (length (n-1)%kB+1)
  double blk[4];         // end values of a full block (length kB)
  double tileK[4];       // end values of a full tile (length kTile)
  double ltileK[4];      // last tile, padded form: full-tile values if full,
                         // else (phi_first of its real length, 0, 0, 0)
};

// Per-system table over the kNT block positions of a tile: beta_{m-1} (the
// coefficient that carries the next block's first unknown into block m-1's
// last one, from the left-to-right elimination) and 1/(1 - phi_first beta_{m-1}).
enum { kTabBeta = 0, kTabInvD = 1, kTabN = 2 };

// Per-system block vectors, kB each, in this order.
enum { kVecIU = 0, kVecCP = 1, kVecPHI = 2, kVecCHI = 3, kVecN = 4 };

// Everything one solve launch sequence needs (device pointers).
struct LaunchSet {
  const SysDesc* sys;
  const double* vec64;
  const float* vec32;
  const double* tab64;     // per-position table [ncidx][2][kNT]
  const float* tab32;
  const int2* p1_items;    // varlen: (system, tile) of the first pass; null for a series
  const int2* fin_items;   // varlen: (system, tile) of the final pass
  const int* grid_items;   // varlen: systems with more than one tile
  int64_t n_p1, n_fin, n_grid;
  double* summ;
  double* ghost;
  double* gscr;
  double* gpart;
  int* iters;
  int max_iter;
  double refine_tol;
  hipEvent_t* ev;          // measurement: 4 events (before pass 1, after pass 1,
                           // after the interface pass, after the final pass) or null
};

// dtype: 0 double, 1 float, 2 float sweeps with double refinement.
hipError_t launch_solve(int dtype, bool bwd, const LaunchSet& L, const void* F, void* X,
                        const void* Xfwd, hipStream_t st);
hipError_t launch_gt_reduce(const double* gpart, const SysDesc* sys, int64_t nsys,
                            int64_t nparts, int varlen, double* gt, hipStream_t st);

}  // namespace tdt
