// tdt_strided.h -- the strided batch solve (systems along a slow axis of an
// array) shared by the host plan code, the 3D Poisson driver and its kernel.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace tdt {

// Strided batches: systems whose consecutive unknowns lie ld elements apart
// and whose neighbouring systems are adjacent in memory (the lines along a
// slow axis of a 2D or 3D array).  A workgroup holds the whole column of SW
// adjacent systems, kStrB rows per lane in registers, and runs the three
// steps of the method on it: the lanes of one system are its blocks.
constexpr int kStrB = 16;             // rows per lane (one block)
constexpr int kStrMaxChunks = 64;     // blocks per column: 1024 rows
// Longer systems are cut into tiles of kStrTile rows (the last one shorter),
// each a column of the kernel above: a first pass keeps every tile's end
// values with zero outside values, one thread per system eliminates the
// tiles' interface values, and a second pass re-solves every tile with its
// two outside values.  Tiles of 512 rows (512 lanes per workgroup, two
// workgroups per compute unit) measured faster than 1024 (one) and as fast
// as 256: 0.41 against 0.49 ms for the 8191 x 8191 batch.
constexpr int kStrTileChunks = 32;
constexpr int64_t kStrTile = (int64_t)kStrTileChunks * kStrB;
constexpr int64_t kStrMaxN = (int64_t)1 << 24;
// Per-class end values of a tile's responses to unit outside values,
// [field][P]: phi_first, phi_last, chi_first, chi_last of a full tile, then
// of the last tile.
enum { kTilePF, kTilePL, kTileCF, kTileCL, kTileEndN = 8 };
// Per-class scalars, [field][P]: t_-1, t_1, the end values
// (phi_first, phi_last, chi_first) of a full block and of the last block.
enum { kStrTM1, kStrT1, kStrPF, kStrPL, kStrCF, kStrTPF, kStrTPL, kStrTCF, kStrScalarN };
// Per-class epilogue, [field][P]: with r the array read and g a second
// input, the system solved is T x = scale (r + c_q g), and the output is
// c_x x + c_r r + c_g g.
enum { kEpiScale, kEpiCQ, kEpiCX, kEpiCR, kEpiCG, kEpiN };
struct StridedArgs {
  const double* R;          // right-hand sides (read)
  double* O;                // output (may be R itself)
  const double* G;          // second input of the epilogue (or null)
  const double* epi;        // [kEpiN][P] or null (plain solve: O = x)
  const double* iu;         // [kStrB][P] 1/u_i of the block LU
  const double* sc;         // [kStrScalarN][P]
  const double* pos;        // [2][C][P] per block position: beta_{c-1}, 1/(1 - phi_f beta_{c-1})
  int64_t N, P, M, ld, nb, ldb;
  int64_t Mg;               // systems s < Mg read G (the others take g = 0)
  int C;                    // blocks per system, ceil(N / kStrB)
  // Tiles of a longer system (pass 0: none).  Column b of a launch is tile
  // m0 + b % tiles of batch b / tiles, at (b / tiles) ldb + (b % tiles) ldt.
  // Pass 1 writes the tile's first and last unknown to Y, pass 2 folds the
  // outside values of Gh into the tile's end rows; both index
  // [(batch K + tile) 2 + end][M].
  int pass;
  int64_t tiles, ldt, K, m0;
  double* Y;
  const double* Gh;
};
hipError_t launch_strided(const StridedArgs& a, hipStream_t st);
// The tiles' interface values of every system (one thread each), from the
// tiles' end values Y: Gh receives every tile's left and right outside
// value; Y is overwritten with intermediate coefficients.
hipError_t launch_strided_interface(const double* ends, double* Y, double* Gh, int64_t M,
                                    int64_t P, int64_t K, int64_t nb, hipStream_t st);
// A system of N > 1024 rows in tiles: K tiles, the last of NL rows; C (CL)
// blocks per full (last) tile; the sizes of the full tile's tables
// [iu|sc|pos], the last tile's, and the end values [kTileEndN][P], which lie
// one after another in that order.
struct StridedTiles {
  int64_t K, NL;
  int C, CL;
  int64_t n_full, n_last, n_ends;
};
StridedTiles strided_tiles(int64_t N, int64_t P);
// The tables of a tiled system (host, long double; n_full + n_last + n_ends
// doubles at out), with the tiles' interface pivots checked per class.
int strided_tiled_tables(int64_t N, int64_t P, const double* tm1, const double* t0,
                         const double* t1, double* out, double* dominance);
// The passes of a tiled system: a carries R, O, G, epi, P, M, Mg, ld, nb,
// ldb; tabs the tables above; Y and Gh hold nb K M 2 doubles each.
hipError_t launch_strided_tiled(StridedArgs a, const StridedTiles& g, const double* tabs,
                                double* Y, double* Gh, hipStream_t st);
// Host tables of P classes (t_-1, t_0, t_1)[k] for systems of order N, in
// long double: iu [kStrB][P], sc [kStrScalarN][P], pos [2][C][P].  Returns a
// negative status on a singular class or bad arguments; *dominance is the
// smallest |t_0| / (|t_-1| + |t_1|) over the classes.
int strided_tables(int64_t N, int64_t P, const double* tm1, const double* t0, const double* t1,
                   double* iu, double* sc, double* pos, double* dominance);
inline int strided_chunks(int64_t N) { return (int)((N + kStrB - 1) / kStrB); }

}  // namespace tdt
