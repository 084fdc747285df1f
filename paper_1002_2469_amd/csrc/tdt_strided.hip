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
// Systems of at most kStrMaxChunks * kStrB = 1024 rows.  An optional
// epilogue writes c_x x + c_r r + c_g g per class instead of x (r the
// right-hand side as read, g a second array): the update of an ADI
// half-step fused into its solve.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdt_internal.h"

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
// Hides a value from the optimiser so that loads through it are issued where
// they are written instead of being hoisted and kept live.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <int CW, int SW, bool EPI>
__global__ __launch_bounds__(CW * SW, (CW * SW >= 1024 ? 1 : 1024 / (CW * SW)))
void k_strided(StridedArgs a) {
  constexpr int NT = CW * SW;
  __shared__ double s0[2][NT], s1[2][NT];
  const int t = threadIdx.x, sl = t % SW, c = t / SW;
  const int64_t s = (int64_t)blockIdx.x * SW + sl;
  const bool live = s < a.M && c < a.C;
  const int64_t P = a.P;
  const int len = live ? (int)(a.N - (int64_t)c * B < B ? a.N - (int64_t)c * B : B) : 0;
  const bool last = c == a.C - 1;
  // the wave's first lane: its system and block give the uniform bases
  const int t0 = t & ~63, sl0 = t0 % SW, c0 = t0 / SW;
  const int64_t s_w = (int64_t)blockIdx.x * SW + sl0;
  // per-class tables: the lane's class is its system, clamped to the last
  // one for lanes past M (their loads still read a valid class), at a byte
  // offset from the wave's first (clamped) class
  const int64_t k_w = s_w < a.M ? s_w : a.M - 1;
  const uint32_t koff = (uint32_t)((s < a.M ? s : a.M - 1) - k_w) * 8u;
  const uint32_t rowP = (uint32_t)(P * 8);
  const __amdgpu_buffer_rsrc_t tiu = wave_rsrc(a.iu + k_w);
  const __amdgpu_buffer_rsrc_t tsc = wave_rsrc(a.sc + k_w);
  const __amdgpu_buffer_rsrc_t tpos = wave_rsrc(a.pos + k_w);
  const __amdgpu_buffer_rsrc_t tepi = wave_rsrc(EPI ? a.epi + k_w : a.sc);
  const int cc = c < a.C ? c : 0;
  // data: unknown i of this lane at (c - c0) * B * ld + (sl - sl0) + i * ld
  // elements from the wave's base
  const uint32_t ldb8 = (uint32_t)(a.ld * 8);
  const uint32_t voff = (uint32_t)((c - c0) * B) * ldb8 + (uint32_t)(sl - sl0) * 8u;

  for (int64_t b = blockIdx.y; b < a.nb; b += gridDim.y) {
    const int64_t wbase = b * a.ldb + (int64_t)c0 * B * a.ld + s_w;
    const __amdgpu_buffer_rsrc_t rR = wave_rsrc(a.R + wbase);
    const __amdgpu_buffer_rsrc_t rO = wave_rsrc(a.O + wbase);
    double q[B], w[B];
    double scale = 1.0, cr = 0.0, cg = 0.0;
    if (EPI) {
      scale = ld64(tepi, koff, kEpiScale * rowP);
      cr = ld64(tepi, koff, kEpiCR * rowP);
      cg = ld64(tepi, koff, kEpiCG * rowP);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const double r = ld64(rR, i < len ? voff : kBad, (uint32_t)i * ldb8);   // 0 past len
      q[i] = EPI ? scale * r : r;
      w[i] = EPI ? cr * r : 0.0;
    }
    if (EPI && a.G != nullptr && cg != 0.0) {
      const __amdgpu_buffer_rsrc_t rG = wave_rsrc(a.G + wbase);
#pragma unroll
      for (int i = 0; i < B; ++i)
        w[i] += cg * ld64(rG, i < len ? voff : kBad, (uint32_t)i * ldb8);
    }
    const double tm1 = ld64(tsc, koff, kStrTM1 * rowP), t1 = ld64(tsc, koff, kStrT1 * rowP);
    // 1. local solve: d_i = q_i / u_i - (t_-1 / u_i) d_{i-1}, y_i = d_i - (t_1 / u_i) y_{i+1};
    //    rows past len stay 0
    {
      const uint32_t ko = opaque(koff);
      q[0] *= ld64(tiu, ko, 0);
#pragma unroll
      for (int i = 1; i < B; ++i) {
        const double d = (q[i] - tm1 * q[i - 1]) * ld64(tiu, ko, (uint32_t)i * rowP);
        q[i] = i < len ? d : 0.0;
      }
    }
    {
      const uint32_t ko = opaque(koff);
#pragma unroll
      for (int i = B - 2; i >= 0; --i) q[i] -= t1 * ld64(tiu, ko, (uint32_t)i * rowP) * q[i + 1];
    }
    double yl = q[0];
#pragma unroll
    for (int i = 1; i < B; ++i)
      if (i == len - 1) yl = q[i];
    const double yf = q[0];

    // 2. interface: alpha_c = A alpha_{c-1} + g, left to right
    // (per-lane rows: the lane's own block kind and position go into the
    // per-lane offset, the uniform offset stays 0)
    const uint32_t ko2 = opaque(koff);
    const uint32_t kb = ko2 + (uint32_t)(last ? kStrTPF : kStrPF) * rowP;
    const double pf = ld64(tsc, kb, 0);
    const double pl = ld64(tsc, kb, (uint32_t)(kStrPL - kStrPF) * rowP);
    const double cf = ld64(tsc, kb, (uint32_t)(kStrCF - kStrPF) * rowP);
    const uint32_t kp = ko2 + (uint32_t)cc * rowP;
    const double bp = ld64(tpos, kp, 0);
    const double iD = ld64(tpos, kp, (uint32_t)a.C * rowP);
    double A = live ? pl * iD : 1.0;
    double g = live ? yl + A * bp * yf : 0.0;
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
    const double alpha_prev = c > 0 ? s1[p][t - SW] : 0.0;
    p ^= 1;
    // u_c = C u_{c+1} + h, right to left (blocks past the end pass u = 0 through)
    double Cc = live ? cf * iD : 1.0;
    double h = live ? (yf + pf * alpha_prev) * iD : 0.0;
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
    const double u_next = c + 1 < CW ? s1[p][t + SW] : 0.0;
    const double xl = alpha_prev + bp * h;   // last unknown of the block on the left
    const double xr = u_next;                // first unknown of the block on the right

    // 3. correction: recover d_i = y_i + (t_1/u_i) y_{i+1}, add the outside
    //    values' contributions (-t_-1 xl carried down from row 0, -t_1 xr at
    //    the last row), back-substitute
    {
      const uint32_t ko = opaque(koff);
      double delta = -tm1 * xl;
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double ui = ld64(tiu, ko, (uint32_t)i * rowP);
        delta *= ui;
        const double ynext = i + 1 < B ? q[i + 1] : 0.0;
        double dv = q[i] + t1 * ui * ynext + delta;
        if (i == len - 1) dv -= t1 * xr * ui;
        q[i] = i < len ? dv : 0.0;
        delta = -tm1 * delta;
      }
    }
    {
      const uint32_t ko = opaque(koff);
#pragma unroll
      for (int i = B - 2; i >= 0; --i) q[i] -= t1 * ld64(tiu, ko, (uint32_t)i * rowP) * q[i + 1];
    }
    const double cx = EPI ? ld64(tepi, opaque(koff), kEpiCX * rowP) : 1.0;
#pragma unroll
    for (int i = 0; i < B; ++i)
      st64(rO, i < len ? voff : kBad, (uint32_t)i * ldb8, EPI ? cx * q[i] + w[i] : q[i]);
    __syncthreads();   // the LDS of this batch is read before the next one writes it
  }
}

template <int CW, int SW>
hipError_t go(const StridedArgs& a, hipStream_t st) {
  const unsigned gx = (unsigned)((a.M + SW - 1) / SW);
  const unsigned gy = (unsigned)(a.nb < 65535 ? a.nb : 65535);
  if (a.epi)
    hipLaunchKernelGGL((k_strided<CW, SW, true>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  else
    hipLaunchKernelGGL((k_strided<CW, SW, false>), dim3(gx, gy), dim3(CW * SW), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_strided(const StridedArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.nb <= 0 || a.N <= 0) return hipSuccess;
  // buffer offsets below 2^31: a lane reaches at most (4 + 1) * kStrB rows
  // past its wave's base row (four blocks per wave when SW = 16), plus 64
  // systems; the tables at most 2 kStrMaxChunks + kStrB rows of P classes
  if ((int64_t)(5 * kStrB) * a.ld * 8 + 64 * 8 >= ((int64_t)1 << 31) ||
      (int64_t)(kEpiN + 2 * kStrMaxChunks + kStrB) * a.P * 8 >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  const int C = a.C;
  if (C <= 1) return go<1, 256>(a, st);
  if (C <= 2) return go<2, 128>(a, st);
  if (C <= 4) return go<4, 64>(a, st);
  if (C <= 8) return go<8, 32>(a, st);
  if (C <= 16) return go<16, 16>(a, st);
  if (C <= 32) return go<32, 16>(a, st);
  return go<64, 16>(a, st);
}

}  // namespace tdt
