// tdt_strided.hip -- the dichotomy solve of Toeplitz systems laid out along a
// slow axis: unknown i of system s at b * ldb + i * ld + s (batch b).
//
// Lanes map to systems, so each row of a load is SW consecutive doubles of
// SW adjacent systems; the SW * CW lanes of a workgroup hold the whole
// column of SW systems, CW blocks of kStrB rows each, in registers.  The
// three steps of the method (Sec. 2.1-2.5) run inside the workgroup:
//   1. every lane solves its block with zero outside values by the block LU
//      of its system's class (T_B^{-1} of eq. (7), shared by all blocks of
//      the class);
//   2. the interface values follow from the affine recurrences of eq. (15)
//      (the same elimination as the tile kernels: v_c = alpha_c + beta_c
//      u_{c+1} left to right, then u_c = C_c u_{c+1} + h_c right to left),
//      evaluated as Kogge-Stone scans across the blocks through LDS;
//   3. every lane re-sweeps its block with its two outside values folded
//      into the first and last right-hand side row.
// Columns of at most kStrMaxChunks * kStrB = 1024 rows; a longer system is
// cut into tiles of kStrTile rows, solved in two passes over the columns
// with the tiles' interface values eliminated between them (the same steps
// one level up: the end values of every tile's zero-outside solution, the
// recurrences of eq. (15) over the tiles, the re-solve).  Optionally the
// right-hand side is scale (r + c_q g) and the output c_x x + c_r r + c_g g
// per class (r the array read, g a second array): an ADI half-step's
// right-hand side and update fused into its solve.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdt_internal.h"
#include "tdt_strided.h"

namespace tdt {
namespace {

constexpr int B = kStrB;

// Raw buffer access with a wave-uniform base (SGPRs), one per-lane byte
// offset for all rows and the row's byte offset as the uniform soffset, so
// that no per-row 64-bit address is kept in VGPRs.  The range is 2^31
// bytes: the host keeps every real offset below it, and a lane that must
// not touch a row passes kBad as its offset, which the hardware range check
// turns into a load of 0 or a dropped store (with or without the uniform
// offset added, the sum stays in [2^31, 2^32)).  So the loads of a column
// are issued back to back, without a branch per row.
constexpr uint32_t kRange = 0x80000000u;
constexpr uint32_t kBad = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const void* base) {
  const uint64_t a = reinterpret_cast<uintptr_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* ub = reinterpret_cast<void*>((uintptr_t)(((uint64_t)hi << 32) | lo));
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)kRange, 0x00020000);
}
__device__ __forceinline__ double ld64(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void st64(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                     double v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}
// An LDS address hidden from the optimiser: reads through it are issued
// next to their use instead of being merged with earlier reads and kept live.
typedef __attribute__((address_space(3))) const double lds_cdouble;
__device__ __forceinline__ lds_cdouble* lds_fresh(const double* p) {
  uint32_t v = (uint32_t)(uintptr_t)(lds_cdouble*)p;
  asm volatile("" : "+v"(v));
  return (lds_cdouble*)(uintptr_t)v;
}

// EPI: 0 plain solve, 1 epilogue without the second input (g = 0, not
// read), 2 epilogue with it
template <int CW, int SW, int EPI, int PASS>
__global__ __launch_bounds__(CW * SW, 4)
void k_strided(StridedArgs a) {
  constexpr int NT = CW * SW;
  __shared__ double s0[2][NT], s1[2][NT];
  // the class tables of this workgroup's SW systems, staged once
  __shared__ double tIU[B][SW], tSC[kStrScalarN][SW], tEP[EPI ? kEpiN : 1][SW];
  __shared__ double tPOS[2][CW][SW];
  const int t = threadIdx.x, sl = t % SW, c = t / SW;
  const int64_t s = (int64_t)blockIdx.x * SW + sl;
  const bool live = s < a.M && c < a.C;
  const int len = live ? (int)(a.N - (int64_t)c * B < B ? a.N - (int64_t)c * B : B) : 0;
  const bool last = c == a.C - 1;
  // the wave's first lane: its system and block give the uniform bases
  const int t0 = t & ~63, sl0 = t0 % SW, c0 = t0 / SW;
  const int64_t s_w = (int64_t)blockIdx.x * SW + sl0;
  // data: unknown i of this lane at (c - c0) * B * ld + (sl - sl0) + i * ld
  // elements from the wave's base
  const uint32_t ldb8 = (uint32_t)(a.ld * 8);
  const uint32_t voff = (uint32_t)((c - c0) * B) * ldb8 + (uint32_t)(sl - sl0) * 8u;
  const bool with_g = EPI == 2 && a.G != nullptr && s < a.Mg;

  // columns of the launch: batches, or (batch, tile) pairs of a tiled system
  const int64_t ncol = PASS ? a.nb * a.tiles : a.nb;
  auto col_off = [&](int64_t bb) -> int64_t {
    if constexpr (PASS == 0) {
      return bb * a.ldb;
    } else {
      const int64_t q2 = bb / a.tiles;
      return q2 * a.ldb + (bb - q2 * a.tiles) * a.ldt;
    }
  };
  // this lane's system in the tiles' end arrays, [(batch K + tile) 2 + end][M]
  auto end_idx = [&](int64_t bb) -> int64_t {
    const int64_t q2 = bb / a.tiles;
    return ((q2 * a.K + a.m0 + (bb - q2 * a.tiles)) * 2) * a.M + s;
  };
  int64_t b = blockIdx.y;
  if (b >= ncol) return;   // uniform over the workgroup
  double q[B], w[B];
  // the column's loads (0 past len), raw: r in q, g in w
  // Only the system's last block can end inside a lane's rows: a wavefront
  // without such a lane addresses every row through one per-lane offset
  // (kBad for lanes without a block); one with it masks the rows past len.
  const bool part = __builtin_amdgcn_ballot_w64(len > 0 && len < B) != 0;   // uniform
  const uint32_t vo = len > 0 ? voff : kBad;
  const uint32_t vg = (len > 0 && with_g) ? voff : kBad;
  auto load = [&](int64_t bb) {
    const int64_t wbase = col_off(bb) + (int64_t)c0 * B * a.ld + s_w;
    const __amdgpu_buffer_rsrc_t rR = wave_rsrc(a.R + wbase);
    const __amdgpu_buffer_rsrc_t rG = wave_rsrc(EPI == 2 && a.G ? a.G + wbase : a.R + wbase);
    if (!part) {
#pragma unroll
      for (int i = 0; i < B; ++i) q[i] = ld64(rR, vo, (uint32_t)i * ldb8);
      if (EPI == 2) {
#pragma unroll
        for (int i = 0; i < B; ++i) w[i] = ld64(rG, vg, (uint32_t)i * ldb8);
      }
    } else {
#pragma unroll
      for (int i = 0; i < B; ++i) {
        q[i] = 0.0;
        if (i < len) q[i] = ld64(rR, vo, (uint32_t)i * ldb8);
      }
      if (EPI == 2) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
          w[i] = 0.0;
          if (i < len) w[i] = ld64(rG, vg, (uint32_t)i * ldb8);
        }
      }
    }
  };
  load(b);
  {
    // the class tables into LDS, once, while the first column is in flight
    // (classes past M read the last one)
    const int64_t k0 = (int64_t)blockIdx.x * SW;
#pragma unroll 1
    for (int e = t; e < (B + kStrScalarN + (EPI ? kEpiN : 0) + 2 * CW) * SW; e += NT) {
      const int row = e / SW, col = e % SW;
      const int64_t k = k0 + col < a.M ? k0 + col : a.M - 1;
      if (row < B) {
        tIU[row][col] = a.iu[row * a.P + k];
      } else if (row < B + kStrScalarN) {
        tSC[row - B][col] = a.sc[(row - B) * a.P + k];
      } else if (EPI && row < B + kStrScalarN + kEpiN) {
        tEP[row - B - kStrScalarN][col] = a.epi[(row - B - kStrScalarN) * a.P + k];
      } else {
        const int r2 = row - B - kStrScalarN - (EPI ? kEpiN : 0);   // [2][CW]
        const int half = r2 / CW, cpos = r2 % CW;
        tPOS[half][cpos][col] = cpos < a.C ? a.pos[((int64_t)half * a.C + cpos) * a.P + k]
                                           : (half == 0 ? 0.0 : 1.0);
      }
    }
    __syncthreads();
  }
  for (;;) {
    const int64_t wbase = col_off(b) + (int64_t)c0 * B * a.ld + s_w;
    const __amdgpu_buffer_rsrc_t rO = wave_rsrc(a.O + wbase);
    const double tm1 = tSC[kStrTM1][sl], t1 = tSC[kStrT1][sl];
    if (EPI) {
      const double scale = tEP[kEpiScale][sl], cq = tEP[kEpiCQ][sl];
      const double cr = tEP[kEpiCR][sl], cg = tEP[kEpiCG][sl];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double r = q[i], gi = EPI == 2 ? w[i] : 0.0;
        w[i] = cr * r + cg * gi;
        q[i] = scale * (r + cq * gi);
        asm volatile("" : "+v"(w[i]));   // formed here: r and g are not kept to the store
      }
    }
    if constexpr (PASS == 2) {
      // the tile's outside values moved to the right-hand side (after the
      // epilogue formed it): f_0 - t_-1 x_left and f_last - t_1 x_right
      if (live) {
        const int64_t gi = end_idx(b);
        if (c == 0) q[0] -= tm1 * a.Gh[gi];
        if (last) {
          const double gr = t1 * a.Gh[gi + a.M];
#pragma unroll
          for (int i = 0; i < B; ++i)
            if (i == len - 1) q[i] -= gr;
        }
      }
    }
    // 1. local solve: d_i = q_i / u_i - (t_-1 / u_i) d_{i-1}, y_i = d_i - (t_1 / u_i) y_{i+1};
    //    rows past len stay 0
    {
      lds_cdouble* iu = lds_fresh(&tIU[0][sl]);
      q[0] *= iu[0];
#pragma unroll
      for (int i = 1; i < B; ++i) {
        const double d = (q[i] - tm1 * q[i - 1]) * iu[i * SW];
        q[i] = i < len ? d : 0.0;
      }
    }
    {
      lds_cdouble* iu = lds_fresh(&tIU[0][sl]);
#pragma unroll
      for (int i = B - 2; i >= 0; --i) q[i] -= t1 * iu[i * SW] * q[i + 1];
    }
    double yl = q[0];
#pragma unroll
    for (int i = 1; i < B; ++i)
      if (i == len - 1) yl = q[i];
    const double yf = q[0];

    // 2. interface: alpha_c = A alpha_{c-1} + g, left to right
    const int kind = last ? kStrTPF : kStrPF;
    const double pf = tSC[kind][sl], pl = tSC[kind + 1][sl], cf = tSC[kind + 2][sl];
    const double bp = tPOS[0][c][sl], iD = tPOS[1][c][sl];
    double A = live ? pl * iD : 1.0;
    double g = live ? yl + A * bp * yf : 0.0;
    double alpha_prev, Cc, h, u_next;
    if constexpr (SW <= 64) {
      // CPW blocks of each system per wavefront, 16/32/64 lanes apart: the
      // scan steps inside a wavefront are shuffles, the wavefronts' totals
      // go through LDS once per direction
      constexpr int CPW = 64 / SW, NW = NT / 64;
      const int j = (t & 63) / SW, wv = t >> 6;
#pragma unroll
      for (int d = 1; d < CPW; d <<= 1) {
        const double Ap = __shfl_up(A, d * SW, 64), gp = __shfl_up(g, d * SW, 64);
        if (j >= d) {
          g = A * gp + g;
          A = A * Ap;
        }
      }
      if (j == CPW - 1) {
        s0[0][wv * SW + sl] = A;
        s1[0][wv * SW + sl] = g;
      }
      __syncthreads();
      double cin = 0.0;   // alpha of the last block before this wavefront's
#pragma unroll 1
      for (int k = 0; k < wv; ++k) cin = s0[0][k * SW + sl] * cin + s1[0][k * SW + sl];
      const double alpha = A * cin + g;
      alpha_prev = __shfl_up(alpha, SW, 64);
      if (j == 0) alpha_prev = cin;
      // u_c = C u_{c+1} + h, right to left (blocks past the end pass u = 0 through)
      Cc = live ? cf * iD : 1.0;
      h = live ? (yf + pf * alpha_prev) * iD : 0.0;
#pragma unroll
      for (int d = 1; d < CPW; d <<= 1) {
        const double Cn = __shfl_down(Cc, d * SW, 64), hn = __shfl_down(h, d * SW, 64);
        if (j + d < CPW) {
          h = Cc * hn + h;
          Cc = Cc * Cn;
        }
      }
      if (j == 0) {
        s0[1][wv * SW + sl] = Cc;
        s1[1][wv * SW + sl] = h;
      }
      __syncthreads();
      double ein = 0.0;   // u of the first block after this wavefront's
#pragma unroll 1
      for (int k = NW - 1; k > wv; --k) ein = s0[1][k * SW + sl] * ein + s1[1][k * SW + sl];
      h = Cc * ein + h;   // u_c
      u_next = __shfl_down(h, SW, 64);
      if (j == CPW - 1) u_next = ein;
    } else {
      // a system's block spans SW / 64 wavefronts: Kogge-Stone through LDS
      int p = 0;
#pragma unroll
      for (int d = 1; d < CW; d <<= 1) {
        s0[p][t] = A;
        s1[p][t] = g;
        __syncthreads();
        if (c >= d) {
          const double Ap = s0[p][t - d * SW], gp = s1[p][t - d * SW];
          g = A * gp + g;
          A = A * Ap;
        }
        p ^= 1;
      }
      s1[p][t] = g;   // alpha_c
      __syncthreads();
      alpha_prev = c > 0 ? s1[p][t - SW] : 0.0;
      p ^= 1;
      Cc = live ? cf * iD : 1.0;
      h = live ? (yf + pf * alpha_prev) * iD : 0.0;
#pragma unroll
      for (int d = 1; d < CW; d <<= 1) {
        s0[p][t] = Cc;
        s1[p][t] = h;
        __syncthreads();
        if (c + d < CW) {
          const double Cn = s0[p][t + d * SW], hn = s1[p][t + d * SW];
          h = Cc * hn + h;
          Cc = Cc * Cn;
        }
        p ^= 1;
      }
      s1[p][t] = h;   // u_c
      __syncthreads();
      u_next = c + 1 < CW ? s1[p][t + SW] : 0.0;
    }
    const double xl = alpha_prev + bp * h;   // last unknown of the block on the left
    const double xr = u_next;                // first unknown of the block on the right

    if constexpr (PASS == 1) {
      // only the tile's first and last unknown are kept, and they need no
      // re-sweep: x_0 = y_0 + phi_f xl + chi_f xr and
      // x_last = y_last + phi_l xl + chi_l xr, with xl = 0 in the first
      // block and xr = 0 in the last (the tile's outside values are zero)
      if (live) {
        const int64_t gi = end_idx(b);
        if (c == 0)
          a.Y[gi] = yf + tSC[last ? kStrTCF : kStrCF][sl] * xr +
                    tSC[last ? kStrTPF : kStrPF][sl] * xl;
        if (last) a.Y[gi + a.M] = yl + tSC[kStrTPL][sl] * xl;
      }
    } else {
      // 3. correction: recover d_i = y_i + (t_1/u_i) y_{i+1}, add the outside
      //    values' contributions (-t_-1 xl carried down from row 0, -t_1 xr at
      //    the last row), back-substitute
      double delta = -tm1 * xl;
      lds_cdouble* iu3 = lds_fresh(&tIU[0][sl]);
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double ui = iu3[i * SW];
        delta *= ui;
        const double ynext = i + 1 < B ? q[i + 1] : 0.0;
        double dv = q[i] + t1 * ui * ynext + delta;
        if (i == len - 1) dv -= t1 * xr * ui;
        q[i] = i < len ? dv : 0.0;
        delta = -tm1 * delta;
      }
      lds_cdouble* iu4 = lds_fresh(&tIU[0][sl]);
#pragma unroll
      for (int i = B - 2; i >= 0; --i) q[i] -= t1 * iu4[i * SW] * q[i + 1];
      const double cx = EPI ? tEP[kEpiCX][sl] : 1.0;
      if (!part) {
#pragma unroll
        for (int i = 0; i < B; ++i)
          st64(rO, vo, (uint32_t)i * ldb8, EPI ? cx * q[i] + w[i] : q[i]);
      } else {
#pragma unroll
        for (int i = 0; i < B; ++i)
          if (i < len) st64(rO, vo, (uint32_t)i * ldb8, EPI ? cx * q[i] + w[i] : q[i]);
      }
    }
    b += gridDim.y;
    if (b >= ncol) break;
    __syncthreads();   // the LDS of this batch is read before the next one writes it
    load(b);
  }
}

// Each workgroup takes two batches of its system group in turn (the class
// tables staged once for both): the ADI of the 511^3 Poisson problem took
// 14.6 ms with one batch per workgroup, 13.8 ms with two, 14.3 with four.
template <int CW, int SW>
hipError_t go(const StridedArgs& a, hipStream_t st) {
  const unsigned gx = (unsigned)((a.M + SW - 1) / SW);
  const int64_t ncol = a.pass ? a.nb * a.tiles : a.nb, gyv = (ncol + 1) / 2;
  const unsigned gy = (unsigned)(gyv < 65535 ? gyv : 65535);
  if (a.epi && a.G && a.Mg > 0)
    hipLaunchKernelGGL((k_strided<CW, SW, 2, 0>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  else if (a.epi)
    hipLaunchKernelGGL((k_strided<CW, SW, 1, 0>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  else
    hipLaunchKernelGGL((k_strided<CW, SW, 0, 0>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  return hipGetLastError();
}

// A tiled system's passes: every tile (the last one too, whatever its block
// count) is a column of the full tile's shape.
// Each workgroup takes two of the columns (tiles) of its system group in
// turn, so that the group's class tables, staged in LDS once, serve both:
// with thousands of classes the tables do not stay in L2 between tiles, and
// reading them per tile cost 1.3x the data's bytes (counters) and 10 % of
// the time on the 8191 x 8191 batch (0.39 -> 0.35 ms).  The workgroups in
// flight still take neighbouring groups of the same tiles, which keeps the
// rows' 128-byte runs together in DRAM (an order that gave each XCD the
// tiles of one group fetched no extra bytes but ran slower, 0.42 ms).
template <int PASS>
hipError_t go_tiles(const StridedArgs& a, hipStream_t st) {
  constexpr int CW = kStrTileChunks, SW = 16;
  const unsigned gx = (unsigned)((a.M + SW - 1) / SW);
  const int64_t ncol = a.nb * a.tiles, gyv = (ncol + 1) / 2;
  const unsigned gy = (unsigned)(gyv < 65535 ? gyv : 65535);
  if (a.epi && a.G && a.Mg > 0)
    hipLaunchKernelGGL((k_strided<CW, SW, 2, PASS>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  else if (a.epi)
    hipLaunchKernelGGL((k_strided<CW, SW, 1, PASS>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  else
    hipLaunchKernelGGL((k_strided<CW, SW, 0, PASS>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  return hipGetLastError();
}

// The tiles' interface values, one thread per (batch, system).  With
// (phi, chi) a tile's responses to unit outside values (first and last entry
// each) and y its zero-outside solution, the first and last unknowns a_m,
// z_m of tile m satisfy
//     a_m = yf_m + phif z_{m-1} + chif a_{m+1},
//     z_m = yl_m + phil z_{m-1} + chil a_{m+1},     z_{-1} = a_K = 0.
// Left to right, z_{m-1} = r_{m-1} + s_{m-1} a_m gives
//     a_m = p_m + q_m a_{m+1},  p_m = (yf_m + phif r_{m-1}) / D_m,
//     q_m = chif / D_m,  D_m = 1 - phif s_{m-1},
//     r_m = yl_m + phil (r_{m-1} + s_{m-1} p_m),  s_m = phil s_{m-1} q_m + chil;
// right to left the a_m and z_m follow, and tile m's outside values are
// z_{m-1} and a_{m+1}.  (p, r) are kept in Gh and (q, s) in Y until the
// backward sweep.
__global__ __launch_bounds__(256) void k_strided_interface(
    const double* __restrict__ ends, double* __restrict__ Y, double* __restrict__ Gh, int64_t M,
    int64_t P, int64_t K, int64_t nb) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= nb * M) return;
  const int64_t bb = id / M, s = id - bb * M;
  const double fpf = ends[kTilePF * P + s], fpl = ends[kTilePL * P + s];
  const double fcf = ends[kTileCF * P + s], fcl = ends[kTileCL * P + s];
  const double lpf = ends[(4 + kTilePF) * P + s], lpl = ends[(4 + kTilePL) * P + s];
  const double lcf = ends[(4 + kTileCF) * P + s], lcl = ends[(4 + kTileCL) * P + s];
  const int64_t base = bb * K * 2 * M + s;
  // eight tiles at a time: their loads are issued together
  constexpr int G = 8;
  double r = 0.0, sp = 0.0;
  for (int64_t m0 = 0; m0 < K; m0 += G) {
    double yf[G], yl[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t i0 = base + (m0 + u) * 2 * M;
      yf[u] = m0 + u < K ? Y[i0] : 0.0;
      yl[u] = m0 + u < K ? Y[i0 + M] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t m = m0 + u;
      if (m >= K) break;
      const bool lt = m == K - 1;
      const double pf = lt ? lpf : fpf, pl = lt ? lpl : fpl;
      const double cf = lt ? lcf : fcf, cl = lt ? lcl : fcl;
      const int64_t i0 = base + m * 2 * M, i1 = i0 + M;
      const double iD = 1.0 / (1.0 - pf * sp);
      const double pm = (yf[u] + pf * r) * iD, qm = cf * iD;
      const double rn = yl[u] + pl * (r + sp * pm);
      const double sn = pl * sp * qm + cl;
      Gh[i0] = pm;
      Gh[i1] = rn;
      Y[i0] = qm;
      Y[i1] = sn;
      r = rn;
      sp = sn;
    }
  }
  double an = 0.0;   // a_{m+1}
  for (int64_t m1 = K - 1; m1 >= 0; m1 -= G) {
    double pm[G], rm[G], qm[G], sm[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t m = m1 - u, i0 = base + m * 2 * M, i1 = i0 + M;
      const bool in = m >= 0;
      pm[u] = in ? Gh[i0] : 0.0;
      rm[u] = in ? Gh[i1] : 0.0;
      qm[u] = in ? Y[i0] : 0.0;
      sm[u] = in ? Y[i1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t m = m1 - u;
      if (m < 0) break;
      const int64_t i0 = base + m * 2 * M, i1 = i0 + M;
      const double am = pm[u] + qm[u] * an, zm = rm[u] + sm[u] * an;
      Gh[i1] = an;                           // right outside value of tile m
      if (m + 1 < K) Gh[i0 + 2 * M] = zm;    // left outside value of tile m + 1
      an = am;
    }
  }
  Gh[base] = 0.0;
}

}  // namespace

hipError_t launch_strided_interface(const double* ends, double* Y, double* Gh, int64_t M,
                                    int64_t P, int64_t K, int64_t nb, hipStream_t st) {
  if (M <= 0 || nb <= 0 || K <= 0) return hipSuccess;
  if (M > P) return hipErrorInvalidValue;
  const int64_t n = nb * M;
  hipLaunchKernelGGL(k_strided_interface, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     ends, Y, Gh, M, P, K, nb);
  return hipGetLastError();
}

hipError_t launch_strided_tiled(StridedArgs a, const StridedTiles& g, const double* tabs,
                                double* Y, double* Gh, hipStream_t st) {
  if (a.M <= 0 || a.nb <= 0) return hipSuccess;
  const double* R = a.R;
  double* O = a.O;
  const double* G = a.G;
  const int64_t off = (g.K - 1) * kStrTile * a.ld;   // the last tile's first row
  a.K = g.K;
  a.ldt = kStrTile * a.ld;
  a.Y = Y;
  a.Gh = Gh;
  auto tables = [&](const double* t) {
    a.iu = t;
    a.sc = t + (int64_t)kStrB * a.P;
    a.pos = a.sc + (int64_t)kStrScalarN * a.P;
  };
  auto pass = [&](int which) {
    a.pass = which;
    tables(tabs);
    a.R = R;
    a.O = O;
    a.G = G;
    a.N = kStrTile;
    a.C = g.C;
    a.tiles = g.K - 1;
    a.m0 = 0;
    hipError_t e = launch_strided(a, st);
    if (e != hipSuccess) return e;
    tables(tabs + g.n_full);
    a.R = R + off;
    a.O = O + off;
    a.G = G ? G + off : nullptr;
    a.N = g.NL;
    a.C = g.CL;
    a.tiles = 1;
    a.m0 = g.K - 1;
    return launch_strided(a, st);
  };
  hipError_t e = pass(1);
  if (e != hipSuccess) return e;
  e = launch_strided_interface(tabs + g.n_full + g.n_last, Y, Gh, a.M, a.P, g.K, a.nb, st);
  if (e != hipSuccess) return e;
  return pass(2);
}

hipError_t launch_strided(const StridedArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.nb <= 0 || a.N <= 0) return hipSuccess;
  // buffer offsets below 2^31: a lane reaches at most (4 + 1) * kStrB rows
  // past its wave's base row (four blocks per wave when SW = 16), plus 64
  // systems; the tables at most 2 kStrMaxChunks + kStrB rows of P classes
  if ((int64_t)(5 * kStrB) * a.ld * 8 + 64 * 8 >= ((int64_t)1 << 31) ||
      (int64_t)(kEpiN + 2 * kStrMaxChunks + kStrB) * a.P * 8 >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  // 16 adjacent systems (128 contiguous bytes of a row) per workgroup once
  // the column needs 16 or more blocks: on rows that start on a cache line
  // this measured faster than 32 or 64 (ADI of the 511^3 Poisson problem:
  // 15.6 ms with 16, 16.9 ms with 32), while rows that do not start on one
  // favour the wider runs (22.7 ms with 16, 20.6 ms with 32).
  const int C = a.C;
  if (a.pass) {
    if (a.tiles < 1 || a.K < 1 || C > kStrTileChunks ||
        (a.pass == 1 && !a.Y) || (a.pass == 2 && !a.Gh) || a.pass > 2)
      return hipErrorInvalidValue;
    return a.pass == 1 ? go_tiles<1>(a, st) : go_tiles<2>(a, st);
  }
  if (C <= 1) return go<1, 256>(a, st);
  if (C <= 2) return go<2, 128>(a, st);
  if (C <= 4) return go<4, 64>(a, st);
  if (C <= 8) return go<8, 32>(a, st);
  if (C <= 16) return go<16, 16>(a, st);
  if (C <= 32) return go<32, 16>(a, st);
  return go<64, 16>(a, st);
}

}  // namespace tdt
