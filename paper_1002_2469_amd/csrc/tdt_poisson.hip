// tdt_poisson.hip -- 2D Poisson solve by separation of variables on one
// MI355X (the application of Sec. 3.2): sine transform along x, one
// tridiagonal Toeplitz system per mode along y (the varlen solver of this
// library), inverse sine transform.
//
// Problem: the five-point system (2u_ij - u_{i-1,j} - u_{i+1,j}) / hx^2 +
// (2u_ij - u_{i,j-1} - u_{i,j+1}) / hy^2 = f_ij on the Nx x Ny interior
// points, u = 0 on the boundary; F and U are [Ny][Nx] (x contiguous).  With
// u_ij = sum_k v_kj sin(pi k i / (Nx+1)) every mode k satisfies
//     -v_{k,j-1} + (2 + hy^2 mu_k) v_kj - v_{k,j+1} = hy^2 fhat_kj,
//     mu_k = (4 / hx^2) sin^2(pi k / (2 (Nx+1))),
//     fhat_kj = (2 / (Nx+1)) sum_i f_ij sin(pi k i / (Nx+1)).
// The sine transform S_m = sum_{j=1}^{n-1} f_j sin(pi j m / n) (n = Nx + 1)
// is taken from a real FFT of length n of the folded sequence
//     y_0 = 0,  y_j = sin(pi j / n) (f_j + f_{n-j}) + (f_j - f_{n-j}) / 2
// (the sine transform through a half-length real transform; Makhoul, IEEE
// Trans. ASSP 28, 1980): with Y_k = sum_j y_j e^{-2 pi i j k / n},
//     S_{2k} = -Im Y_k,   S_1 = Re Y_0 / 2,   S_{2k+1} = S_{2k-1} + Re Y_k,
// the odd coefficients a prefix sum along k.  The FFTs are hipFFT's; the
// folding, the prefix sums, the scaled transposes into and out of mode-major
// order and the line solves are this library's kernels.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "tdt.h"
#include "tdt_internal.h"
#include "tdt_strided.h"

struct tdt_poisson_s {
  int64_t nx = 0, ny = 0;
  double hx = 0.0, hy = 0.0;
  tdt_plan_t line = nullptr;     // Nx Toeplitz systems of Ny rows (mode-major), or
  bool strided = false;          // the same systems in place in the row-major
  int64_t ldw = 0;               // transformed rows (a strided plan), rows ldw apart
  hipfftHandle fft = 0;          // Ny real transforms of length Nx + 1
  bool fft_made = false;
  double* sn = nullptr;          // sin(pi j / (Nx + 1)), j = 0 .. Nx
  double* y = nullptr;           // [Ny][Nx + 1] folded rows
  double* spec = nullptr;        // [Ny][(Nx + 1) / 2 + 1] complex spectra
  double* T = nullptr;           // [Nx][Ny] mode-major right-hand sides
  double* V = nullptr;           // [Nx][Ny] mode-major solutions
  bool fused = false;            // Nx + 1 = 2 N2 (N2 a power of two): k_dst_rows
  double* tw = nullptr;          // its twiddle tables
  double* pw = nullptr;
  bool profile = false;
  std::vector<hipEvent_t> ev;    // 4 per recorded solve
};

namespace {

constexpr int kTileP = 32;       // transpose tile (kTileP x kTileP, kTileP x 8 threads)
constexpr unsigned kMaxGridY = 32768;   // the y dimension of a launch walks the rest
constexpr int kScanNT = 256;     // threads of the per-row prefix sum

// y[j][.] = the folded row j of F (n = Nx + 1 entries)
__global__ void k_fold_rows(const double* __restrict__ F, const double* __restrict__ sn,
                            double* __restrict__ y, int64_t nx, int64_t ny) {
  const int64_t n = nx + 1;
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= n) return;
  for (int64_t r = blockIdx.y; r < ny; r += gridDim.y) {
    const double* f = F + r * nx;
    double v = 0.0;
    if (jj > 0) {
      const double a = f[jj - 1], b = f[n - jj - 1];
      v = sn[jj] * (a + b) + 0.5 * (a - b);
    }
    y[r * n + jj] = v;
  }
}

// In place on each spectrum row: Re Y_k -> S_{2k+1} (Re Y_0 / 2 plus the
// inclusive prefix sum of Re Y_1..Re Y_k); Im Y_k (= -S_{2k}) is kept.  With
// U non-null the row's coefficients S_1..S_Nx, times scale, are written to
// U's row instead.  One workgroup per row walks it in
// segments of 4 kScanNT entries: each thread takes 4 consecutive entries
// (coalesced), the thread totals are scanned across the wavefront by
// shuffles and across the wavefronts through LDS, and a carry runs from
// segment to segment (a fixed summation order).
__global__ __launch_bounds__(kScanNT) void k_scan_rows(double* __restrict__ spec,
                                                       int64_t nx, int64_t ny,
                                                       double* __restrict__ U,
                                                       double scale) {
  constexpr int E = 4, NW = kScanNT / 64;
  __shared__ double wtot[NW];
  const int64_t K = (nx + 1) / 2 + 1;                  // complex entries per row
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int64_t r = blockIdx.x; r < ny; r += gridDim.x) {
    double* row = spec + 2 * r * K;
    double carry = 0.0;
    for (int64_t base = 0; base < K; base += (int64_t)E * kScanNT) {
      const int64_t k0 = base + (int64_t)E * tid;
      double v[E], im[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t k = k0 + e;
        const double re = k < K ? row[2 * k] : 0.0;
        im[e] = k < K ? row[2 * k + 1] : 0.0;
        v[e] = k == 0 ? 0.5 * re : re;
      }
#pragma unroll
      for (int e = 1; e < E; ++e) v[e] += v[e - 1];   // inclusive within the thread
      // exclusive prefix of the thread totals across the wavefront
      double x = v[E - 1];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      if (lane == 63) wtot[w] = x;
      __syncthreads();
      double off = carry, seg = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        if (q < w) off += wtot[q];
        seg += wtot[q];
      }
      off += x - v[E - 1];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t k = k0 + e;
        if (k >= K) break;
        const double acc = off + v[e];
        if (U) {
          // S_{2k+1} = acc, S_{2k} = -Im Y_k; U[m-1] = S_m for m = 1..Nx
          double* u = U + r * nx;
          if (2 * k + 1 <= nx) u[2 * k] = scale * acc;
          if (k >= 1 && 2 * k <= nx) u[2 * k - 1] = -scale * im[e];
        } else {
          row[2 * k] = acc;
        }
      }
      carry += seg;
      __syncthreads();   // wtot is rewritten by the next segment
    }
  }
}

// The same for rows of at most 64 E spectrum entries (Nx < 128 E): one
// wavefront per row, four rows per workgroup.  Entry k is taken by lane
// k % 64 in round k / 64, so that every load and store of a round is
// contiguous across the lanes; each round is a wavefront scan by shuffles
// plus the carry of the rounds before it.  A lane writes the adjacent pair
// (S_{2k}, S_{2k+1}) = (U[2k-1], U[2k]).
template <int E>
__global__ __launch_bounds__(256) void k_scan_rows_wave(double* __restrict__ spec, int64_t nx,
                                                        int64_t ny, double* __restrict__ U,
                                                        double scale) {
  const int64_t K = (nx + 1) / 2 + 1;
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < ny;
       r += (int64_t)gridDim.x * 4) {
    double2* row = reinterpret_cast<double2*>(spec) + r * K;
    double2 z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t k = (int64_t)64 * e + lane;
      z[e] = k < K ? row[k] : make_double2(0.0, 0.0);
    }
    double carry = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t k = (int64_t)64 * e + lane;
      double x = k == 0 ? 0.5 * z[e].x : z[e].x;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      const double acc = carry + x;
      carry += __shfl(x, 63, 64);
      if (k < K) {
        if (U) {
          double* u = U + r * nx;
          // U[2k] = S_{2k+1} = acc, U[2k-1] = S_{2k} = -Im Y_k (m = 1 .. Nx)
          if (k >= 1 && 2 * k <= nx) u[2 * k - 1] = -scale * z[e].y;
          if (2 * k + 1 <= nx) u[2 * k] = scale * acc;
        } else {
          row[k].x = acc;
        }
      }
    }
  }
}

// T[m-1][j] = s * S_m of spectrum row j (S_m = Re' Y_{(m-1)/2} for odd m,
// -Im Y_{m/2} for even m): the scaled coefficients transposed to mode-major
// order through an LDS tile.
__global__ void k_modes_from_rows(const double* __restrict__ spec, double* __restrict__ T,
                                  int64_t nx, int64_t ny, double s) {
  __shared__ double tile[kTileP][kTileP + 1];
  const int64_t K = (nx + 1) / 2 + 1;
  const int64_t m0 = (int64_t)blockIdx.x * kTileP;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int64_t j0 = (int64_t)blockIdx.y * kTileP; j0 < ny; j0 += (int64_t)gridDim.y * kTileP) {
    __syncthreads();   // the previous tile is read
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t j = j0 + r, m = m0 + tx + 1;
      if (j < ny && m <= nx) {
        const double* row = spec + 2 * j * K;
        tile[r][tx] = s * ((m & 1) ? row[2 * ((m - 1) / 2)] : -row[2 * (m / 2) + 1]);
      }
    }
    __syncthreads();
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t m = m0 + r, j = j0 + tx;
      if (m < nx && j < ny) T[m * ny + j] = tile[tx][r];
    }
  }
}

// y[j][.] = the folded mode coefficients of row j (v_m = V[m-1][j]): the
// transpose back to row-major order, with each block reading the tile of its
// mode range and the tile of the mirrored range n - m.
__global__ void k_fold_modes(const double* __restrict__ V, const double* __restrict__ sn,
                             double* __restrict__ y, int64_t nx, int64_t ny) {
  __shared__ double ta[kTileP][kTileP + 1], tb[kTileP][kTileP + 1];
  const int64_t n = nx + 1;
  const int64_t m0 = (int64_t)blockIdx.x * kTileP;   // folded positions m0 .. m0 + 31
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int64_t j0 = (int64_t)blockIdx.y * kTileP; j0 < ny; j0 += (int64_t)gridDim.y * kTileP) {
    __syncthreads();
    for (int q = ty; q < kTileP; q += blockDim.y) {
      const int64_t m = m0 + q, j = j0 + tx;
      if (j < ny && m >= 1 && m < n) {
        ta[q][tx] = V[(m - 1) * ny + j];          // v_m
        tb[q][tx] = V[(n - m - 1) * ny + j];      // v_{n-m}
      }
    }
    __syncthreads();
    for (int q = ty; q < kTileP; q += blockDim.y) {
      const int64_t j = j0 + q, m = m0 + tx;
      if (j < ny && m < n) {
        double v = 0.0;
        if (m >= 1) {
          const double a = ta[tx][q], b = tb[tx][q];
          v = sn[m] * (a + b) + 0.5 * (a - b);
        }
        y[j * n + m] = v;
      }
    }
  }
}

// The per-row prefix sums of a batch of spectra (see k_scan_rows).
void launch_scan_rows(double* spec, int64_t nx, int64_t ny, double* U, double scale,
                      hipStream_t st) {
  const int64_t K = (nx + 1) / 2 + 1;
  const int E = (int)((K + 63) / 64);
  const unsigned gw = (unsigned)std::min<int64_t>((ny + 3) / 4, kMaxGridY);
  switch (E) {
#define TDT_SCAN_CASE(e) \
  case e: hipLaunchKernelGGL(k_scan_rows_wave<e>, dim3(gw), dim3(256), 0, st, spec, nx, ny, U, scale); return;
    TDT_SCAN_CASE(1) TDT_SCAN_CASE(2) TDT_SCAN_CASE(3) TDT_SCAN_CASE(4)
    TDT_SCAN_CASE(5) TDT_SCAN_CASE(6) TDT_SCAN_CASE(7) TDT_SCAN_CASE(8)
#undef TDT_SCAN_CASE
    default: {
      const unsigned g = (unsigned)std::min<int64_t>(ny, kMaxGridY);
      hipLaunchKernelGGL(k_scan_rows, dim3(g), dim3(kScanNT), 0, st, spec, nx, ny, U, scale);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused sine transform of rows, for n = Nx + 1 = 2 N2 with N2 a power of two
// in [64, 4096]: out[m-1] = scale S_m, S_m = sum_{j=1}^{n-1} f_j sin(pi j m / n),
// in one pass over HBM (read a row, write a row).  Per row, in LDS: the
// folded sequence y (the same fold as k_fold_rows) packed as
// z_k = y_2k + i y_2k+1, its complex FFT of length N2 by Stockham autosort
// passes (radix 4, one radix-2 pass first when log2 N2 is odd; Govindaraju
// et al., SC 2008), the split into the real FFT Y of length n,
// Y_k = E_k + e^{-2 pi i k / n} O_k with E_k = (Z_k + conj Z_{N2-k}) / 2 and
// O_k = -i (Z_k - conj Z_{N2-k}) / 2, then S_2k = -Im Y_k and the odd
// coefficients as the prefix sum of Re Y_k (as in k_scan_rows).  Twiddles
// come from tables made in long double on the host: tw[q] = e^{-2 pi i q/N2},
// pw[k] = e^{-2 pi i k/n}.  N2/4 threads per row, 256/(N2/4) rows per
// workgroup for N2 <= 1024.
constexpr int kDstMinN2 = 64, kDstMaxN2 = 4096;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// 4-point DFT in place: y_s = sum_t x_t e^{-2 pi i t s / 4}
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
  const double2 s0 = cadd(x0, x2), d0 = csub(x0, x2), s1 = cadd(x1, x3), d1 = csub(x1, x3);
  x0 = cadd(s0, s1);
  x1 = make_double2(d0.x + d1.y, d0.y - d1.x);   // d0 - i d1
  x2 = csub(s0, s1);
  x3 = make_double2(d0.x - d1.y, d0.y + d1.x);   // d0 + i d1
}
// 8-point DFT in place, X_s = sum_r a_r w^{r s}, w = e^{-i pi / 4}: the
// 4-point DFTs E, O of the even and odd inputs, X_s = E_s + w^s O_s,
// X_{s+4} = E_s - w^s O_s.
__device__ __forceinline__ void dft8(double2 (&a)[8]) {
  dft4(a[0], a[2], a[4], a[6]);
  dft4(a[1], a[3], a[5], a[7]);
  constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
  const double2 o1 = make_double2(h * (a[3].x + a[3].y), h * (a[3].y - a[3].x));
  const double2 o2 = make_double2(a[5].y, -a[5].x);
  const double2 o3 = make_double2(h * (a[7].y - a[7].x), -h * (a[7].x + a[7].y));
  const double2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}
// LDS positions that spread strided accesses over the banks.  A wavefront's
// 16-byte accesses are served eight lanes (128 bytes) at a time, 8-byte ones
// sixteen at a time; the lanes k = E j + e (fixed e) of the real split, and
// the first pass's outputs E j + r, would fall on one bank group (E = 8) or
// four (E = 4).  Element k of the complex buffer sits at
// k ^ ((k >> S) & 7) and double d of the output staging at
// d ^ ((d >> (S + 1)) & 15): a bijection that keeps each aligned group of 8
// (16) slots, so consecutive indices stay conflict-free too.  S = 3 for the
// radix-8 passes and for log2 N2 odd, S = 2 for the even radix-4 sizes,
// whose passes then have no conflicts at all (one 2-way pass remains for
// the odd sizes).
template <int S>
__device__ __forceinline__ int swz16(int k) { return k ^ ((k >> S) & 7); }
template <int S>
__device__ __forceinline__ int swz8(int d) { return d ^ ((d >> (S + 1)) & 15); }

template <int N2>
struct DstShape {
  // complex values per thread: 4 (one radix-4 butterfly per pass), 8 for
  // the 4096-point rows, whose 512 threads then fit two rows per compute
  // unit in one LDS buffer each
  static constexpr int E = N2 >= 4096 ? 8 : 4;
  static constexpr int TR = N2 / E;                      // threads per row
  static constexpr int RW = TR >= 256 ? 1 : 256 / TR;    // rows per workgroup
  static constexpr int NT = TR * RW;
  static constexpr int NWR = TR >= 64 ? TR / 64 : 1;     // wavefronts per row
};

// Raw buffer accesses with a wave-uniform base and range (SGPRs), a per-lane
// byte offset and a uniform byte offset: no 64-bit address per access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uintptr_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const uint32_t nb = __builtin_amdgcn_readfirstlane(bytes);
  void* ub = reinterpret_cast<void*>((uintptr_t)(((uint64_t)hi << 32) | lo));
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)nb, 0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, double x) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, v, s, 0);
}

template <int N2>
__global__ __launch_bounds__(DstShape<N2>::NT, N2 == 256 ? 5 : 4) void k_dst_rows(
    const double* __restrict__ in, double* __restrict__ out, int64_t rows, int64_t ldi,
    int64_t ldo, double scale, const double* __restrict__ sn, const double2* __restrict__ tw,
    const double2* __restrict__ pw) {
  using S = DstShape<N2>;
  constexpr int E = S::E, TR = S::TR, RW = S::RW, n = 2 * N2, nx = n - 1;
  constexpr int Q = E / 4;   // radix-4 butterflies per thread and pass
  // One LDS buffer per row: the row, then the transform, every pass reading
  // its inputs into registers before any thread writes (two barriers per
  // pass) -- half the LDS of ping-pong buffers, so more rows per compute
  // unit overlap their loads, arithmetic and stores.
  __shared__ double2 buf[RW][N2];
  __shared__ double wt[RW][S::NWR];
  const int t = threadIdx.x, rr = t / TR;
  // the rows of a wavefront: its first row's base, the lane's row offset
  const int rr0 = (t & ~63) / TR;
  const uint32_t lri = (uint32_t)((rr - rr0) * ldi) * 8u, lro = (uint32_t)((rr - rr0) * ldo) * 8u;
  const __amdgpu_buffer_rsrc_t tsn = row_rsrc(sn, (uint32_t)n * 8u);
  constexpr int L2 = __builtin_ctz(N2), ODD = L2 & 1, NP = L2 / 2;
  constexpr int NS0 = ODD ? 2 : 4;   // Ns of the first pass taken from LDS
  constexpr int NPL = NP - (ODD ? 0 : 1);
  // eight values per thread and a power of 8: radix-8 passes (one in
  // registers, L2 / 3 - 1 through LDS) instead of radix 4
  constexpr bool R8 = E == 8 && L2 % 3 == 0;
  constexpr int NP8 = L2 / 3 - 1;
  // swizzled positions of the complex buffer and of the output staging
  constexpr int SZ = (R8 || ODD) ? 3 : 2;
  auto pz = [](int k) { return swz16<SZ>(k); };
  auto pd = [](int d) { return swz8<SZ>(d); };
  const int64_t rstep = (int64_t)gridDim.x * RW;
  // a row block's input, coalesced, into registers (rows past the end read
  // 0): the next block's is requested while this one's spectrum is written
  // out, so its latency is hidden behind the scan and the stores
  const uint32_t lrj = lri + (uint32_t)(t % TR) * 8u;
  auto load_rows = [&](int64_t rb, double (&nv)[2 * E]) {
    const int64_t w0 = rb + rr0;
    uint32_t nb = 0u;
    if (w0 < rows) {
      const int64_t b = ((rows - w0 - 1) * ldi + nx) * 8;
      nb = b < ((int64_t)1 << 31) ? (uint32_t)b : 0x7fffffffu;
    }
    const __amdgpu_buffer_rsrc_t rin = row_rsrc(in + (w0 < rows ? w0 : 0) * ldi, nb);
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) nv[i] = bload(rin, lrj, (uint32_t)(TR * i) * 8u);
  };
  double nv[2 * E];
  load_rows((int64_t)blockIdx.x * RW, nv);
  for (int64_t r0 = (int64_t)blockIdx.x * RW; r0 < rows; r0 += rstep) {
    const int64_t r = r0 + rr;
    const bool live = r < rows;
    // the row into LDS (f_m+1 at m)
    const int64_t rw0 = r0 + rr0;
    // the bytes from the wavefront's first row to the end of the array
    auto avail = [&](int64_t ld) {
      if (rw0 >= rows) return 0u;
      const int64_t b = ((rows - rw0 - 1) * ld + nx) * 8;
      return b < ((int64_t)1 << 31) ? (uint32_t)b : 0x7fffffffu;
    };
    double* fl = reinterpret_cast<double*>(buf[rr]);
    // the lane's index, opaque to the compiler, for the table loads: their
    // values repeat from row to row, and held across rows they would take
    // more registers than reloading them (from cache) costs
    int jt = t % TR;
    asm volatile("" : "+v"(jt));
    const int j = jt;
    __builtin_assume(j >= 0 && j < TR);
    // one twiddle per butterfly and pass (W^q; W^2q and W^3q follow from
    // it), loaded one pass ahead, the first and the real split's with the row
    auto twq = [&](int ps, int q) {
      const int lg = __builtin_ctz(NS0) + 2 * ps;   // Ns = NS0 4^ps
      return tw[((jt + TR * q) & ((1 << lg) - 1)) << (L2 - 2 - lg)];
    };
    // the radix-8 passes' twiddle W^k, k = j mod Ns, Ns = 8^(ps + 1)
    auto tw8 = [&](int ps) {
      const int lg = 3 * (ps + 1);
      return tw[(jt & ((1 << lg) - 1)) << (L2 - 3 - lg)];
    };
    double2 wcur[Q];
    if constexpr (R8) {
      wcur[0] = tw8(0);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) wcur[q] = twq(0, q);
    }
    const double2 pw0 = pw[E * jt];
    // the fold's sines, with the row too
    double sv[E][2];
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        sv[e][h] = bload(tsn, (uint32_t)(2 * jt) * 8u, (uint32_t)(2 * TR * e + h) * 8u);
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int m = j + TR * i;
      if (m < nx) fl[m] = nv[i];
    }
    __syncthreads();
    // fold, packed in pairs: z_k = y_2k + i y_2k+1 for k = j + TR e
    double2 z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = j + TR * e;
      double y2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jj = 2 * k + h;
        const double a = jj > 0 ? fl[jj - 1] : 0.0, b = jj > 0 ? fl[n - jj - 1] : 0.0;
        y2[h] = jj > 0 ? sv[e][h] * (a + b) + 0.5 * (a - b) : 0.0;
      }
      z[e] = make_double2(y2[0], y2[1]);
    }
    __syncthreads();   // the row is read
    // complex FFT of length N2, Stockham autosort; its first pass works on
    // the thread's own z (butterfly b = j + TR q takes z_{b + r N2/R})
    if constexpr (R8) {
      // butterfly b = j: inputs at b + r N2/8 (the thread's z), outputs at
      // (b / Ns) 8 Ns + (b mod Ns) + r Ns
      dft8(z);
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[rr][pz(8 * j + r)] = z[r];
      __syncthreads();
#pragma unroll 1
      for (int ps = 0; ps < NP8; ++ps) {
        const int lg = 3 * (ps + 1), Ns = 1 << lg;
        const double2 wnext = tw8(ps + 1 < NP8 ? ps + 1 : ps);
        double2 a8[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a8[r] = buf[rr][pz(j + r * (N2 / 8))];
        const double2 w1 = wcur[0], w2 = cmul(w1, w1), w3 = cmul(w2, w1), w4 = cmul(w2, w2);
        wcur[0] = wnext;
        a8[1] = cmul(a8[1], w1);
        a8[2] = cmul(a8[2], w2);
        a8[3] = cmul(a8[3], w3);
        a8[4] = cmul(a8[4], w4);
        a8[5] = cmul(a8[5], cmul(w4, w1));
        a8[6] = cmul(a8[6], cmul(w4, w2));
        a8[7] = cmul(a8[7], cmul(w4, w3));
        dft8(a8);
        const int idx = ((j >> lg) << (lg + 3)) + (j & (Ns - 1));
        __syncthreads();   // every thread has read the pass's inputs
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[rr][pz(idx + r * Ns)] = a8[r];
        __syncthreads();
      }
    } else if constexpr (ODD) {   // radix 2, Ns = 1
#pragma unroll
      for (int q = 0; q < E / 2; ++q) {
        const int b = j + TR * q;
        buf[rr][pz(2 * b)] = cadd(z[q], z[q + E / 2]);
        buf[rr][pz(2 * b + 1)] = csub(z[q], z[q + E / 2]);
      }
    } else {               // radix 4, Ns = 1 (no twiddles)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = j + TR * q;
        const double2 s0 = cadd(z[q], z[q + 2 * Q]), d0 = csub(z[q], z[q + 2 * Q]);
        const double2 s1 = cadd(z[q + Q], z[q + 3 * Q]), d1 = csub(z[q + Q], z[q + 3 * Q]);
        buf[rr][pz(4 * b)] = cadd(s0, s1);
        buf[rr][pz(4 * b + 1)] = make_double2(d0.x + d1.y, d0.y - d1.x);
        buf[rr][pz(4 * b + 2)] = csub(s0, s1);
        buf[rr][pz(4 * b + 3)] = make_double2(d0.x - d1.y, d0.y + d1.x);
      }
    }
    if constexpr (!R8) __syncthreads();
    int Ns = NS0;
#pragma unroll 1
    for (int ps = 0; ps < (R8 ? 0 : NPL); ++ps, Ns *= 4) {
      const int lg = __builtin_ctz(NS0) + 2 * ps;
      double2 X[Q][4];
      int idx[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = j + TR * q;
        const int k = b & (Ns - 1);
        const double2 wnext = twq(ps + 1 < NPL ? ps + 1 : ps, q);
        double2 v0 = buf[rr][pz(b)], v1 = buf[rr][pz(b + N2 / 4)];
        double2 v2 = buf[rr][pz(b + N2 / 2)], v3 = buf[rr][pz(b + 3 * (N2 / 4))];
        const double2 w1 = wcur[q], w2 = cmul(w1, w1), w3 = cmul(w2, w1);
        wcur[q] = wnext;
        v1 = cmul(v1, w1);
        v2 = cmul(v2, w2);
        v3 = cmul(v3, w3);
        const double2 s0 = cadd(v0, v2), d0 = csub(v0, v2), s1 = cadd(v1, v3), d1 = csub(v1, v3);
        X[q][0] = cadd(s0, s1);
        X[q][1] = make_double2(d0.x + d1.y, d0.y - d1.x);       // d0 - i d1
        X[q][2] = csub(s0, s1);
        X[q][3] = make_double2(d0.x - d1.y, d0.y + d1.x);       // d0 + i d1
        idx[q] = ((b >> lg) << (lg + 2)) + k;
      }
      __syncthreads();   // every thread has read the pass's inputs
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int rj = 0; rj < 4; ++rj) buf[rr][pz(idx[q] + rj * Ns)] = X[q][rj];
      __syncthreads();
    }
    // the real transform Y_k for k = E j .. E j + E - 1, and the prefix sum of Re Y
    const double2* Z = buf[rr];
    double v[E], im[E];
    double2 pwk = pw0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = E * j + e;
      const double2 zk = Z[pz(k)], zm = Z[pz((N2 - k) & (N2 - 1))];
      const double2 Ev = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
      const double2 O = make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x));
      const double2 Y = cadd(Ev, cmul(pwk, O));
      v[e] = k == 0 ? 0.5 * Y.x : Y.x;
      im[e] = Y.y;
      pwk = cmul(pwk, pw[1]);   // e^{-2 pi i (k + 1) / n}
    }
    __syncthreads();   // the spectrum is read
    if (r0 + rstep < rows) load_rows(r0 + rstep, nv);
    // S in natural order (m - 1) in LDS: the odd terms now, the even ones
    // after the scan, then coalesced stores
    double* ob = reinterpret_cast<double*>(buf[rr]);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = E * j + e;
      if (k >= 1) ob[pd(2 * k - 1)] = -im[e];
    }
#pragma unroll
    for (int e = 1; e < E; ++e) v[e] += v[e - 1];
    double x = v[E - 1];
    constexpr int W = TR < 64 ? TR : 64;
    const int lw = t % W;
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
      const double yv = __shfl_up(x, d, W);
      if (lw >= d) x += yv;
    }
    double carry = 0.0;
    if constexpr (TR > 64) {
      const int wv = j / 64;
      if (lw == 63) wt[rr][wv] = x;
      __syncthreads();
      for (int q2 = 0; q2 < wv; ++q2) carry += wt[rr][q2];
    }
    const double off = carry + x - v[E - 1];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = E * j + e;
      if (2 * k + 1 <= nx) ob[pd(2 * k)] = off + v[e];
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rout =
        row_rsrc(out + (rw0 < rows ? rw0 : 0) * ldo, avail(ldo));
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int m = j + TR * i;
      if (m < nx && live)
        bstore(rout, lro + (uint32_t)j * 8u, (uint32_t)(TR * i) * 8u, scale * ob[pd(m)]);
    }
    __syncthreads();   // the buffer is rewritten by the next rows
  }
}

bool dst_supported(int64_t nx) {
  const int64_t n2 = (nx + 1) / 2;
  return (nx + 1) % 2 == 0 && n2 >= kDstMinN2 && n2 <= kDstMaxN2 && (n2 & (n2 - 1)) == 0;
}

// The twiddle tables of k_dst_rows (long double): tw [N2], pw [N2] complex.
void dst_tables(int64_t nx, std::vector<double>& tw, std::vector<double>& pw) {
  const int64_t n = nx + 1, n2 = n / 2;
  const long double pi = 3.141592653589793238462643383279502884L;
  tw.assign((size_t)(2 * n2), 0.0);
  pw.assign((size_t)(2 * n2), 0.0);
  for (int64_t q = 0; q < n2; ++q) {
    const long double a = -2.0L * pi * (long double)q / (long double)n2;
    tw[(size_t)(2 * q)] = (double)std::cos(a);
    tw[(size_t)(2 * q + 1)] = (double)std::sin(a);
    const long double b = -2.0L * pi * (long double)q / (long double)n;
    pw[(size_t)(2 * q)] = (double)std::cos(b);
    pw[(size_t)(2 * q + 1)] = (double)std::sin(b);
  }
}

void launch_dst_rows(const double* in, double* out, int64_t nx, int64_t rows, int64_t ldi,
                     int64_t ldo, double scale,
                     const double* sn, const double* tw, const double* pw, hipStream_t st) {
  const int n2 = (int)((nx + 1) / 2);
  const auto* t2 = reinterpret_cast<const double2*>(tw);
  const auto* p2 = reinterpret_cast<const double2*>(pw);
  switch (n2) {
#define TDT_DST_CASE(N)                                                                    \
  case N: {                                                                                \
    const int64_t g = (rows + DstShape<N>::RW - 1) / DstShape<N>::RW;                      \
    hipLaunchKernelGGL(k_dst_rows<N>, dim3((unsigned)std::min<int64_t>(g, 1 << 20)),       \
                       dim3(DstShape<N>::NT), 0, st, in, out, rows, ldi, ldo, scale, sn,  \
                       t2, p2);                                                            \
    return;                                                                                \
  }
    TDT_DST_CASE(64) TDT_DST_CASE(128) TDT_DST_CASE(256) TDT_DST_CASE(512)
    TDT_DST_CASE(1024) TDT_DST_CASE(2048) TDT_DST_CASE(4096)
#undef TDT_DST_CASE
    default: return;
  }
}

// out[c][r] = s in[r][c] for an R x C row-major array, through 32 x 33 LDS tiles.
__global__ void k_transpose_scale(const double* __restrict__ in, double* __restrict__ out,
                                  int64_t R, int64_t C, double s) {
  __shared__ double tile[kTileP][kTileP + 1];
  const int64_t c0 = (int64_t)blockIdx.x * kTileP;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int64_t r0 = (int64_t)blockIdx.y * kTileP; r0 < R; r0 += (int64_t)gridDim.y * kTileP) {
    __syncthreads();   // the previous tile is read
    for (int q = ty; q < kTileP; q += blockDim.y) {
      const int64_t r = r0 + q, c = c0 + tx;
      if (r < R && c < C) tile[q][tx] = s * in[r * C + c];
    }
    __syncthreads();
    for (int q = ty; q < kTileP; q += blockDim.y) {
      const int64_t c = c0 + q, r = r0 + tx;
      if (c < C && r < R) out[c * R + r] = tile[tx][q];
    }
  }
}

void destroy_poisson(tdt_poisson_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->line) (void)tdt_plan_destroy(p->line);
  if (p->fft_made) (void)hipfftDestroy(p->fft);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  (void)hipFree(p->sn);
  (void)hipFree(p->y);
  (void)hipFree(p->spec);
  (void)hipFree(p->T);
  (void)hipFree(p->V);
  (void)hipFree(p->tw);
  (void)hipFree(p->pw);
  delete p;
}

}  // namespace

extern "C" {

// Largest condition number of a mode system a TDT_F32_REFINE handle accepts.
constexpr double kRefineKappaMax = 8.0e6;

tdt_status_t tdt_poisson2d_create(int64_t nx, int64_t ny, double hx, double hy,
                                  tdt_dtype_t dtype, tdt_poisson_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 26) || nx * ny > ((int64_t)1 << 31) ||
      !(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy) ||
      (dtype != TDT_F64 && dtype != TDT_F32_REFINE))
    return TDT_ERR_INVALID_ARG;
  tdt_poisson_s* p = new (std::nothrow) tdt_poisson_s();
  if (!p) return TDT_ERR_OOM;
  p->nx = nx;
  p->ny = ny;
  p->hx = hx;
  p->hy = hy;
  // one system per mode: t_-1 = t_1 = -1, t_0 = 2 + hy^2 mu_k (long double)
  std::vector<int64_t> off((size_t)nx + 1);
  std::vector<double> tm1((size_t)nx, -1.0), t0((size_t)nx), t1((size_t)nx, -1.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int64_t k = 1; k <= nx; ++k) {
    const long double sn = std::sin(pi * (long double)k / (2.0L * (long double)(nx + 1)));
    const long double mu = 4.0L / ((long double)hx * hx) * sn * sn;
    t0[(size_t)k - 1] = (double)(2.0L + (long double)hy * hy * mu);
  }
  for (int64_t k = 0; k <= nx; ++k) off[(size_t)k] = k * ny;
  // Float sweeps contract a refinement by about c kappa_2 2^-24 per step.
  // The mode systems' condition numbers are known in closed form (spectrum
  // t_0 - 2 cos(j pi / (Ny+1))); the lowest mode's is the largest.  Above
  // kRefineKappaMax the contraction is too slow to reach the double tier
  // (measured: systems up to kappa_2 = 6.8e6 reach it, the lowest modes of
  // the 8191 x 8191 grid, kappa_2 = 1.4e7, do not), so such a plan is refused.
  if (dtype == TDT_F32_REFINE) {
    const long double cs = std::cos(pi / (long double)(ny + 1));
    for (int64_t k = 0; k < nx; ++k) {
      const long double lo = (long double)t0[(size_t)k] - 2.0L * cs;
      const long double hi = (long double)t0[(size_t)k] + 2.0L * cs;
      if (!(lo > 0.0L) || (double)(hi / lo) > kRefineKappaMax) {
        delete p;
        return TDT_ERR_NOT_CONVERGED;
      }
    }
  }
  const int64_t n = nx + 1, K = n / 2 + 1;
  p->fused = dst_supported(nx);
  // In float64 with the fused row transform, the mode systems are solved in
  // place in the transformed rows, as a strided batch (system k: column k),
  // with rows padded to a multiple of 16 doubles plus 16, so that each
  // starts on a cache line and consecutive rows fall on different channels.
  // Otherwise transposes to and from mode-major order around a varlen plan.
  p->strided = p->fused && dtype == TDT_F64;
  p->ldw = p->strided ? (nx + 15) / 16 * 16 + 16 : n;
  tdt_status_t st =
      p->strided
          ? tdt_plan_strided_create(ny, nx, tm1.data(), t0.data(), t1.data(), dtype, &p->line)
          : tdt_plan_varlen_create(nx, off.data(), tm1.data(), t0.data(), t1.data(), dtype,
                                   &p->line);
  if (st < 0) {
    destroy_poisson(p);
    return st;
  }
  st = tdt_plan_reserve(p->line, p->strided ? nx : 1);
  if (st == TDT_OK &&
      (hipMalloc(&p->sn, (size_t)n * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->y, (size_t)(ny * p->ldw) * sizeof(double)) != hipSuccess ||
       (!p->fused &&
        hipMalloc(&p->spec, (size_t)(ny * K) * 2 * sizeof(double)) != hipSuccess) ||
       (!p->strided && hipMalloc(&p->T, (size_t)(nx * ny) * sizeof(double)) != hipSuccess) ||
       (!p->strided && hipMalloc(&p->V, (size_t)(nx * ny) * sizeof(double)) != hipSuccess)))
    st = TDT_ERR_OOM;
  if (st == TDT_OK) {
    std::vector<double> sn((size_t)n);
    for (int64_t j = 0; j < n; ++j) sn[(size_t)j] = (double)std::sin(pi * (long double)j / n);
    if (hipMemcpy(p->sn, sn.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess)
      st = TDT_ERR_HIP;
  }
  if (st == TDT_OK && p->fused) {
    std::vector<double> tw, pw;
    dst_tables(nx, tw, pw);
    if (hipMalloc(&p->tw, tw.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->pw, pw.size() * sizeof(double)) != hipSuccess)
      st = TDT_ERR_OOM;
    else if (hipMemcpy(p->tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice) !=
                 hipSuccess ||
             hipMemcpy(p->pw, pw.data(), pw.size() * sizeof(double), hipMemcpyHostToDevice) !=
                 hipSuccess)
      st = TDT_ERR_HIP;
  }
  if (st == TDT_OK && !p->fused) {
    int len[1] = {(int)n};
    if (hipfftPlanMany(&p->fft, 1, len, nullptr, 1, (int)n, nullptr, 1, (int)K, HIPFFT_D2Z,
                       (int)ny) != HIPFFT_SUCCESS)
      st = TDT_ERR_HIP;
    else
      p->fft_made = true;
  }
  if (st < 0) {
    destroy_poisson(p);
    return st;
  }
  *out = p;
  return TDT_OK;
}

tdt_status_t tdt_poisson2d_solve(tdt_poisson_t p, const double* F, double* U,
                                 hipStream_t stream) {
  if (!p || !F || !U) return TDT_ERR_INVALID_ARG;
  const int64_t nx = p->nx, ny = p->ny, n = nx + 1;
  auto gy = [](int64_t v) { return (unsigned)(v < (int64_t)kMaxGridY ? v : kMaxGridY); };
  hipEvent_t* ev = nullptr;
  if (p->profile) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      const size_t k = p->ev.size();
      p->ev.resize(k + 4);
      for (size_t j = 0; j < 4; ++j)
        if (hipEventCreate(&p->ev[k + j]) != hipSuccess) return TDT_ERR_HIP;
      ev = p->ev.data() + k;
    }
  }
  auto mark = [&](int j) {
    if (ev) (void)hipEventRecord(ev[j], stream);
  };
  const double s = p->hy * p->hy * 2.0 / (double)(nx + 1);
  if (p->strided) {
    // rows' sine transforms (the forward one scaled) into the padded work
    // rows, the mode systems solved in place down the columns, the inverse
    // transforms into U
    mark(0);
    launch_dst_rows(F, p->y, nx, ny, nx, p->ldw, s, p->sn, p->tw, p->pw, stream);
    mark(1);
    tdt_status_t st = tdt_solve_strided(p->line, p->y, p->y, nx, p->ldw, 1, 0, stream);
    if (st < 0) return st;
    mark(2);
    launch_dst_rows(p->y, U, nx, ny, p->ldw, nx, 1.0, p->sn, p->tw, p->pw, stream);
    mark(3);
    return hipGetLastError() == hipSuccess ? TDT_OK : TDT_ERR_HIP;
  }
  if (p->fused) {
    // rows' sine transforms in one pass each, transposes to and from
    // mode-major order (the forward one scaled)
    const dim3 trow((unsigned)((nx + kTileP - 1) / kTileP), gy((ny + kTileP - 1) / kTileP));
    const dim3 tcol((unsigned)((ny + kTileP - 1) / kTileP), gy((nx + kTileP - 1) / kTileP));
    mark(0);
    launch_dst_rows(F, p->y, nx, ny, nx, nx, 1.0, p->sn, p->tw, p->pw, stream);
    hipLaunchKernelGGL(k_transpose_scale, trow, dim3(kTileP, 8), 0, stream, p->y, p->T, ny, nx,
                       s);
    mark(1);
    tdt_status_t st = tdt_solve_varlen(p->line, p->T, p->V, stream);
    if (st < 0) return st;
    mark(2);
    hipLaunchKernelGGL(k_transpose_scale, tcol, dim3(kTileP, 8), 0, stream, p->V, p->y, nx, ny,
                       1.0);
    launch_dst_rows(p->y, U, nx, ny, nx, nx, 1.0, p->sn, p->tw, p->pw, stream);
    mark(3);
    return hipGetLastError() == hipSuccess ? TDT_OK : TDT_ERR_HIP;
  }
  if (hipfftSetStream(p->fft, stream) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  const dim3 tiles((unsigned)((nx + 1 + kTileP - 1) / kTileP), gy((ny + kTileP - 1) / kTileP));
  auto* spec = reinterpret_cast<hipfftDoubleComplex*>(p->spec);
  // sine transform of the rows, scaled and transposed to mode-major order
  mark(0);
  hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((n + 255) / 256), gy(ny)), dim3(256), 0,
                     stream, F, p->sn, p->y, nx, ny);
  if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  launch_scan_rows(p->spec, nx, ny, nullptr, 1.0, stream);
  hipLaunchKernelGGL(k_modes_from_rows, tiles, dim3(kTileP, 8), 0, stream, p->spec, p->T, nx,
                     ny, s);
  mark(1);
  // one Toeplitz system per mode
  tdt_status_t st = tdt_solve_varlen(p->line, p->T, p->V, stream);
  if (st < 0) return st;
  mark(2);
  // inverse transform: the same sine transform of the mode coefficients
  hipLaunchKernelGGL(k_fold_modes, tiles, dim3(kTileP, 8), 0, stream, p->V, p->sn, p->y, nx,
                     ny);
  if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  launch_scan_rows(p->spec, nx, ny, U, 1.0, stream);
  mark(3);
  return hipGetLastError() == hipSuccess ? TDT_OK : TDT_ERR_HIP;
}

tdt_status_t tdt_poisson2d_profile(tdt_poisson_t p, int enable) {
  if (!p) return TDT_ERR_INVALID_ARG;
  if (!enable) {
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
  }
  p->profile = enable != 0;
  return TDT_OK;
}

tdt_status_t tdt_poisson2d_profile_read(tdt_poisson_t p, double* ms3, int64_t* nsolves) {
  if (!p || !ms3) return TDT_ERR_INVALID_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  ms3[0] = ms3[1] = ms3[2] = 0.0;
  const size_t ns = p->ev.size() / 4;
  for (size_t k = 0; k < ns; ++k)
    for (int j = 0; j < 3; ++j) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p->ev[4 * k + j], p->ev[4 * k + j + 1]) != hipSuccess)
        return TDT_ERR_HIP;
      ms3[j] += (double)ms;
    }
  if (nsolves) *nsolves = (int64_t)ns;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  return TDT_OK;
}

tdt_status_t tdt_poisson2d_line_plan(tdt_poisson_t p, tdt_plan_t* line) {
  if (!p || !line) return TDT_ERR_INVALID_ARG;
  *line = p->line;
  return TDT_OK;
}

tdt_status_t tdt_poisson2d_destroy(tdt_poisson_t p) {
  if (!p) return TDT_ERR_INVALID_ARG;
  destroy_poisson(p);
  return TDT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// 3D Poisson problem (Sec. 3.5): a sine transform along x leaves, for every
// mode k, a 2D problem on the (y, z) plane,
//     (A_y + A_z + mu_k) v_k = fhat_k,   A_y v = (2 v_j - v_{j-1} - v_{j+1}) / hy^2 (A_z alike),
// solved by Peaceman-Rachford ADI with the shift split evenly, A1 = A_y + mu_k/2
// and A2 = A_z + mu_k/2, from v = 0:
//     (w_j + A1) v'  = (w_j - A2) v  + fhat,
//     (w_j + A2) v'' = (w_j - A1) v' + fhat,       j = 1 .. J_k.
// Each half-step is one strided batch of Toeplitz line systems (lines along
// y, then along z, all modes of a plane at once; no transposes).  Its
// right-hand side never needs the other direction's operator: with R1 the
// first half-step's right-hand side, (w - A1) v' + fhat = 2 w v' - R1 + fhat,
// and the next iteration's (w' - A2) v'' + fhat = (w' + w) v'' - R2 + fhat.
// So the first half-step writes P2 = 2 w v' - R1, the second solves with
// P2 + fhat (R2) and writes R1' = (w' + w) v'' - P2, or v'' in a mode's last
// iteration: fhat is read once per iteration, by the second half-step.
// Parameters: the optimal set of Jordan and Wachspress for the interval
// [a_k, b_k] holding both spectra, w_j = b dn((2j - 1) K / (2J), m),
// m = 1 - (a/b)^2; J_k is the smallest J whose error bound d_J^2 <= eps,
// d_J = prod_j (w_j - a) / (w_j + a), the largest error factor of one
// direction on [a, b] for this set.
// ---------------------------------------------------------------------------
struct tdt_poisson3d_s {
  int64_t nx = 0, ny = 0, nz = 0;
  double hx = 0.0, hy = 0.0, hz = 0.0, eps = 0.0;
  hipfftHandle fft = 0;
  bool fft_made = false;
  double* sn = nullptr;     // sin(pi j / (Nx + 1)), j = 0 .. Nx
  double* y = nullptr;      // [Ny Nz][Nx + 1] folded rows
  double* spec = nullptr;   // [Ny Nz][(Nx + 1) / 2 + 1] complex spectra; the ADI work array
  double* tabs = nullptr;   // per iteration and direction: iu | sc | pos | epi of its modes
  bool fused = false;       // Nx + 1 = 2 N2 (N2 a power of two): k_dst_rows, no FFT buffers
  double* tw = nullptr;     // its twiddle tables
  double* pw = nullptr;
  double* W = nullptr;      // the ADI work array (the spectrum buffer otherwise)
  double* Yt = nullptr;     // lines of more than 1024 rows: the tiles' end values
  double* Gt = nullptr;     // and outside values, [nb][K][2][modes] each
  double* fh = nullptr;     // fhat (U otherwise)
  int64_t ldx = 0;          // row stride of W and fhat: Nx rounded up to 16 (128-byte rows)
  std::vector<int> count;                  // J_k
  std::vector<double> omega;               // [k][jmax]
  int jmax = 0;
  std::vector<int64_t> active;             // modes in iteration j (a prefix: J_k falls with k)
  std::vector<int64_t> toff[2];            // table offset per iteration, y and z sweeps
  bool profile = false;
  std::vector<hipEvent_t> ev;              // 4 per recorded solve
};

namespace {

const long double kPi = 3.141592653589793238462643383279502884L;

// Complete elliptic integral of the first kind from the complementary
// modulus kp = sqrt(1 - m): K = pi / (2 AGM(1, kp)) (Gauss).
long double ellip_K(long double kp) {
  long double a = 1.0L, b = kp;
  for (int it = 0; it < 64 && std::fabs(a - b) > 1e-19L * a; ++it) {
    const long double an = 0.5L * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return kPi / (2.0L * a);
}

// Jacobi dn(u | m), kp = sqrt(1 - m), by the arithmetic-geometric mean
// scheme (Abramowitz and Stegun 16.4): a_0 = 1, b_0 = kp, c_0 = sqrt(m);
// phi_N = 2^N a_N u, phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2;
// dn = cos(phi_0) / cos(phi_1 - phi_0).
long double ellip_dn(long double u, long double kp) {
  long double a[64], c[64];
  a[0] = 1.0L;
  c[0] = std::sqrt((1.0L - kp) * (1.0L + kp));
  long double b = kp;
  int n = 0;
  while (n < 62 && std::fabs(c[n]) > 1e-19L * a[n]) {
    a[n + 1] = 0.5L * (a[n] + b);
    c[n + 1] = 0.5L * (a[n] - b);
    b = std::sqrt(a[n] * b);
    ++n;
  }
  if (n == 0) return 1.0L;   // m = 0
  long double phi = std::ldexp(a[n] * u, n), prev = phi;
  for (int i = n; i >= 1; --i) {
    prev = phi;
    phi = 0.5L * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
  }
  return std::cos(phi) / std::cos(prev - phi);
}

// The J optimal parameters for [a, b] (largest first).  The half with
// u <= K/2 comes from dn, where dn >= sqrt(a/b) keeps its relative accuracy;
// the others from the pairing w_j w_{J+1-j} = a b (dn(K - u) = kp / dn(u)).
void adi_parameters(long double a, long double b, int J, std::vector<long double>& w) {
  w.assign((size_t)J, 0.0L);
  const long double kp = a / b, K = ellip_K(kp);
  for (int j = 1; 2 * j <= J + 1; ++j) {
    w[(size_t)j - 1] = b * ellip_dn((2 * j - 1) * K / (2.0L * J), kp);
    w[(size_t)(J - j)] = a * b / w[(size_t)j - 1];
  }
  if (J % 2 == 1) w[(size_t)(J / 2)] = std::sqrt(a * b);
}

long double adi_bound(long double a, long double b, int J) {
  std::vector<long double> w;
  adi_parameters(a, b, J, w);
  long double d = 1.0L;
  for (long double x : w) d *= std::fabs((x - a) / (x + a));
  return d;
}

long double line_eig(int64_t n, double h, int64_t q) {
  const long double s = std::sin(kPi * (long double)q / (2.0L * (long double)(n + 1)));
  return 4.0L / ((long double)h * h) * s * s;
}

void destroy_poisson3d(tdt_poisson3d_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->fft_made) (void)hipfftDestroy(p->fft);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  (void)hipFree(p->sn);
  (void)hipFree(p->y);
  (void)hipFree(p->spec);
  (void)hipFree(p->tabs);
  (void)hipFree(p->tw);
  (void)hipFree(p->pw);
  (void)hipFree(p->W);
  (void)hipFree(p->fh);
  (void)hipFree(p->Yt);
  (void)hipFree(p->Gt);
  delete p;
}

constexpr int kAdiCap = 400;

}  // namespace

extern "C" {

tdt_status_t tdt_poisson3d_create(int64_t nx, int64_t ny, int64_t nz, double hx, double hy,
                                  double hz, double eps, tdt_poisson3d_t* out) {
  if (!out) return TDT_ERR_INVALID_ARG;
  *out = nullptr;
  const int64_t lmax = tdt::kStrMaxN;
  if (nx < 1 || ny < 1 || nz < 1 || ny > lmax || nz > lmax || nx > (1 << 20) ||
      nx * ny * nz > ((int64_t)1 << 34) || ny * nz > ((int64_t)1 << 31) ||
      (int64_t)(5 * tdt::kStrB) * nx * ny * 8 + 512 >= ((int64_t)1 << 31) ||
      !(hx > 0.0) || !(hy > 0.0) || !(hz > 0.0) || !std::isfinite(hx) || !std::isfinite(hy) ||
      !std::isfinite(hz) || !(eps > 0.0) || !(eps < 1.0))
    return TDT_ERR_INVALID_ARG;
  tdt_poisson3d_s* p = new (std::nothrow) tdt_poisson3d_s();
  if (!p) return TDT_ERR_OOM;
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->hx = hx;
  p->hy = hy;
  p->hz = hz;
  p->eps = eps;
  // ADI schedule per mode (long double)
  const long double ly0 = line_eig(ny, hy, 1), ly1 = line_eig(ny, hy, ny);
  const long double lz0 = line_eig(nz, hz, 1), lz1 = line_eig(nz, hz, nz);
  std::vector<long double> mu((size_t)nx);
  std::vector<std::vector<long double>> w((size_t)nx);
  p->count.assign((size_t)nx, 0);
  int J = 1;
  for (int64_t k = 0; k < nx; ++k) {
    mu[(size_t)k] = line_eig(nx, hx, k + 1);
    const long double a = 0.5L * mu[(size_t)k] + std::min(ly0, lz0);
    const long double b = 0.5L * mu[(size_t)k] + std::max(ly1, lz1);
    auto ok = [&](int j) {
      const long double d = adi_bound(a, b, j);
      return d * d <= (long double)eps;
    };
    // J_k falls with k (b/a does): start from the previous mode's count
    while (J > 1 && ok(J - 1)) --J;
    while (J < kAdiCap && !ok(J)) ++J;
    if (!ok(J)) {
      destroy_poisson3d(p);
      return TDT_ERR_INVALID_ARG;   // eps out of reach within the cap
    }
    p->count[(size_t)k] = J;
    adi_parameters(a, b, J, w[(size_t)k]);
  }
  // counts must not rise with k for the prefix structure of the iterations
  for (int64_t k = nx - 1; k > 0; --k)
    if (p->count[(size_t)k] > p->count[(size_t)k - 1]) {
      destroy_poisson3d(p);
      return TDT_ERR_SINGULAR;
    }
  p->jmax = p->count[0];
  p->omega.assign((size_t)(nx * p->jmax), 0.0);
  for (int64_t k = 0; k < nx; ++k)
    for (int j = 0; j < p->count[(size_t)k]; ++j)
      p->omega[(size_t)(k * p->jmax + j)] = (double)w[(size_t)k][(size_t)j];
  p->active.assign((size_t)p->jmax, 0);
  for (int j = 0; j < p->jmax; ++j) {
    int64_t K = 0;
    while (K < nx && p->count[(size_t)K] > j) ++K;
    p->active[(size_t)j] = K;
  }
  // tables of every half-step: classes k < K_j with t_+-1 = -1,
  // t_0 = 2 + h^2 (w_kj + mu_k / 2), and the epilogue of the step
  std::vector<double> tab;
  tdt_status_t st = TDT_OK;
  for (int d = 0; d < 2 && st == TDT_OK; ++d) {
    const int64_t N = d == 0 ? ny : nz;
    const long double h2 = d == 0 ? (long double)hy * hy : (long double)hz * hz;
    const int C = tdt::strided_chunks(N);
    p->toff[d].assign((size_t)p->jmax, 0);
    for (int j = 0; j < p->jmax && st == TDT_OK; ++j) {
      const int64_t P = p->active[(size_t)j];
      std::vector<double> tm1((size_t)P, -1.0), t0((size_t)P), t1((size_t)P, -1.0);
      const size_t base = tab.size();
      p->toff[d][(size_t)j] = (int64_t)base;
      // one column: iu | sc | pos | epi; tiles: full | last | ends | epi
      const tdt::StridedTiles g = tdt::strided_tiles(N, P);
      const int64_t ncol = g.K > 1 ? g.n_full + g.n_last + g.n_ends
                                   : (int64_t)(tdt::kStrB + tdt::kStrScalarN + 2 * C) * P;
      tab.resize(base + (size_t)(ncol + tdt::kEpiN * P));
      double* epi = tab.data() + base + ncol;
      for (int64_t k = 0; k < P; ++k) {
        const long double wk = w[(size_t)k][(size_t)j];
        t0[(size_t)k] = (double)(2.0L + h2 * (wk + 0.5L * mu[(size_t)k]));
        epi[tdt::kEpiScale * P + k] = (double)h2;
        const bool fin = d == 1 && j + 1 == p->count[(size_t)k];
        // y: solve R1, write P2 = 2w v' - R1; z: solve P2 + fhat, write
        // R1' = (w' + w) v'' - P2, or v'' at the mode's last iteration
        long double cx = d == 0 ? 2.0L * wk
                                : (fin ? 1.0L : w[(size_t)k][(size_t)j + 1] + wk);
        epi[tdt::kEpiCQ * P + k] = d == 0 ? 0.0 : 1.0;
        epi[tdt::kEpiCX * P + k] = (double)cx;
        epi[tdt::kEpiCR * P + k] = fin ? 0.0 : -1.0;
        epi[tdt::kEpiCG * P + k] = 0.0;
      }
      double dom = 0.0;
      double* iu = tab.data() + base;
      double* sc = iu + tdt::kStrB * P;
      double* pos = sc + tdt::kStrScalarN * P;
      const int r =
          g.K > 1 ? tdt::strided_tiled_tables(N, P, tm1.data(), t0.data(), t1.data(), iu, &dom)
                  : tdt::strided_tables(N, P, tm1.data(), t0.data(), t1.data(), iu, sc, pos, &dom);
      if (r < 0) st = (tdt_status_t)r;
    }
  }
  const int64_t n = nx + 1, Kc = n / 2 + 1, rows = ny * nz;
  p->fused = dst_supported(nx);
  // With the fused transform the ADI arrays get rows of a multiple of 128
  // bytes, so that a workgroup's 256-byte run of a row starts on a cache
  // line, and 128 bytes more, so that the rows do not step through memory
  // in a power of two (at 511^3 the ADI half-steps take 19.3 ms with
  // 511-double rows, 17.1 ms with 512 and 16.9 ms with 528)
  p->ldx = p->fused ? (nx + 15) / 16 * 16 + 16 : nx;
  if (st == TDT_OK && (int64_t)(5 * tdt::kStrB) * p->ldx * ny * 8 + 512 >= ((int64_t)1 << 31))
    st = TDT_ERR_INVALID_ARG;
  if (st == TDT_OK &&
      (hipMalloc(&p->sn, (size_t)n * sizeof(double)) != hipSuccess ||
       (p->fused &&
        hipMalloc(&p->W, (size_t)(rows * p->ldx) * sizeof(double)) != hipSuccess) ||
       (p->fused &&
        hipMalloc(&p->fh, (size_t)(rows * p->ldx) * sizeof(double)) != hipSuccess) ||
       (!p->fused && hipMalloc(&p->y, (size_t)(rows * n) * sizeof(double)) != hipSuccess) ||
       (!p->fused &&
        hipMalloc(&p->spec, (size_t)(rows * Kc) * 2 * sizeof(double)) != hipSuccess) ||
       hipMalloc(&p->tabs, tab.size() * sizeof(double)) != hipSuccess))
    st = TDT_ERR_OOM;
  // lines of more than 1024 rows run in tiles, with the tiles' end and
  // outside values of every (batch, mode) in two work arrays
  {
    const int64_t ky = tdt::strided_tiles(ny, 1).K, kz = tdt::strided_tiles(nz, 1).K;
    const int64_t slots = std::max(ky > 1 ? nz * ky : 0, kz > 1 ? ny * kz : 0) * nx * 2;
    if (st == TDT_OK && slots > 0 &&
        (hipMalloc(&p->Yt, (size_t)slots * sizeof(double)) != hipSuccess ||
         hipMalloc(&p->Gt, (size_t)slots * sizeof(double)) != hipSuccess))
      st = TDT_ERR_OOM;
  }
  if (st == TDT_OK && p->fused) {
    std::vector<double> tw, pw;
    dst_tables(nx, tw, pw);
    if (hipMalloc(&p->tw, tw.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->pw, pw.size() * sizeof(double)) != hipSuccess)
      st = TDT_ERR_OOM;
    else if (hipMemcpy(p->tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice) !=
                 hipSuccess ||
             hipMemcpy(p->pw, pw.data(), pw.size() * sizeof(double), hipMemcpyHostToDevice) !=
                 hipSuccess)
      st = TDT_ERR_HIP;
  }
  if (st == TDT_OK) {
    std::vector<double> sn((size_t)n);
    for (int64_t j = 0; j < n; ++j) sn[(size_t)j] = (double)std::sin(kPi * (long double)j / n);
    if (hipMemcpy(p->sn, sn.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->tabs, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess)
      st = TDT_ERR_HIP;
  }
  if (st == TDT_OK && !p->fused) {
    int len[1] = {(int)n};
    if (hipfftPlanMany(&p->fft, 1, len, nullptr, 1, (int)n, nullptr, 1, (int)Kc, HIPFFT_D2Z,
                       (int)rows) != HIPFFT_SUCCESS)
      st = TDT_ERR_HIP;
    else
      p->fft_made = true;
  }
  if (st < 0) {
    destroy_poisson3d(p);
    return st;
  }
  *out = p;
  return TDT_OK;
}

tdt_status_t tdt_poisson3d_solve(tdt_poisson3d_t p, const double* F, double* U,
                                 hipStream_t stream) {
  if (!p || !F || !U) return TDT_ERR_INVALID_ARG;
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz, n = nx + 1, rows = ny * nz;
  const size_t bytes = (size_t)(nx * rows) * sizeof(double);
  if (F == U || (reinterpret_cast<const char*>(F) < reinterpret_cast<const char*>(U) + bytes &&
                 reinterpret_cast<const char*>(U) < reinterpret_cast<const char*>(F) + bytes))
    return TDT_ERR_INVALID_ARG;
  if (!p->fused && hipfftSetStream(p->fft, stream) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  hipEvent_t* ev = nullptr;
  if (p->profile) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      const size_t k = p->ev.size();
      p->ev.resize(k + 4);
      for (size_t j = 0; j < 4; ++j)
        if (hipEventCreate(&p->ev[k + j]) != hipSuccess) return TDT_ERR_HIP;
      ev = p->ev.data() + k;
    }
  }
  auto gy = [](int64_t v) { return (unsigned)(v < (int64_t)kMaxGridY ? v : kMaxGridY); };
  auto* spec = reinterpret_cast<hipfftDoubleComplex*>(p->spec);
  if (ev) (void)hipEventRecord(ev[0], stream);
  // fhat: the scaled sine transform of every row along x (into its own
  // array with padded rows, or into U on the hipFFT path)
  if (p->fused) {
    launch_dst_rows(F, p->fh, nx, rows, nx, p->ldx, 2.0 / (double)(nx + 1), p->sn, p->tw, p->pw,
                    stream);
  } else {
    hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((n + 255) / 256), gy(rows)), dim3(256), 0,
                       stream, F, p->sn, p->y, nx, rows);
    if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
    launch_scan_rows(p->spec, nx, rows, U, 2.0 / (double)(nx + 1), stream);
  }
  if (ev) (void)hipEventRecord(ev[1], stream);
  // ADI: W (its own array, or the spectrum buffer) holds each mode's current
  // right-hand side
  double* W = p->fused ? p->W : p->spec;
  const double* fh = p->fused ? p->fh : U;
  const int64_t lx = p->ldx;
  for (int j = 0; j < p->jmax; ++j) {
    const int64_t P = p->active[(size_t)j];
    for (int d = 0; d < 2; ++d) {
      const int64_t N = d == 0 ? ny : nz;
      const int C = tdt::strided_chunks(N);
      const tdt::StridedTiles g = tdt::strided_tiles(N, P);
      const double* tb = p->tabs + p->toff[d][(size_t)j];
      tdt::StridedArgs a{};
      a.R = (j == 0 && d == 0) ? fh : W;
      a.O = W;
      a.G = fh;
      a.iu = tb;
      a.sc = a.iu + tdt::kStrB * P;
      a.pos = a.sc + tdt::kStrScalarN * P;
      a.epi = g.K > 1 ? tb + g.n_full + g.n_last + g.n_ends : a.pos + 2 * C * P;
      a.N = N;
      a.P = P;
      a.M = P;
      a.Mg = d == 0 ? 0 : P;   // fhat: read by the second half-step only
      a.C = C;
      if (d == 0) {   // lines along y: rows lx apart, one batch per z plane
        a.ld = lx;
        a.nb = nz;
        a.ldb = lx * ny;
      } else {        // lines along z: rows lx ny apart, one batch per y row
        a.ld = lx * ny;
        a.nb = ny;
        a.ldb = lx;
      }
      if (g.K > 1) {
        if (tdt::launch_strided_tiled(a, g, tb, p->Yt, p->Gt, stream) != hipSuccess)
          return TDT_ERR_HIP;
      } else if (tdt::launch_strided(a, stream) != hipSuccess) {
        return TDT_ERR_HIP;
      }
    }
  }
  if (ev) (void)hipEventRecord(ev[2], stream);
  // U: the (unscaled) sine transform of the mode coefficients of every row
  if (p->fused) {
    launch_dst_rows(W, U, nx, rows, p->ldx, nx, 1.0, p->sn, p->tw, p->pw, stream);
  } else {
    hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((n + 255) / 256), gy(rows)), dim3(256), 0,
                       stream, W, p->sn, p->y, nx, rows);
    if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
    launch_scan_rows(p->spec, nx, rows, U, 1.0, stream);
  }
  if (ev) (void)hipEventRecord(ev[3], stream);
  return hipGetLastError() == hipSuccess ? TDT_OK : TDT_ERR_HIP;
}

tdt_status_t tdt_poisson3d_schedule(tdt_poisson3d_t p, int* h_counts, double* h_omega,
                                    int64_t omega_len, int* jmax) {
  if (!p) return TDT_ERR_INVALID_ARG;
  if (jmax) *jmax = p->jmax;
  if (h_counts)
    for (int64_t k = 0; k < p->nx; ++k) h_counts[k] = p->count[(size_t)k];
  if (h_omega) {
    if (omega_len < (int64_t)p->omega.size()) return TDT_ERR_INVALID_ARG;
    for (size_t i = 0; i < p->omega.size(); ++i) h_omega[i] = p->omega[i];
  }
  return TDT_OK;
}

tdt_status_t tdt_poisson3d_profile(tdt_poisson3d_t p, int enable) {
  if (!p) return TDT_ERR_INVALID_ARG;
  if (!enable) {
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
  }
  p->profile = enable != 0;
  return TDT_OK;
}

tdt_status_t tdt_poisson3d_profile_read(tdt_poisson3d_t p, double* ms3, int64_t* nsolves) {
  if (!p || !ms3) return TDT_ERR_INVALID_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return TDT_ERR_HIP;
  ms3[0] = ms3[1] = ms3[2] = 0.0;
  const size_t ns = p->ev.size() / 4;
  for (size_t k = 0; k < ns; ++k)
    for (int j = 0; j < 3; ++j) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p->ev[4 * k + j], p->ev[4 * k + j + 1]) != hipSuccess)
        return TDT_ERR_HIP;
      ms3[j] += (double)ms;
    }
  if (nsolves) *nsolves = (int64_t)ns;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  return TDT_OK;
}

tdt_status_t tdt_adi_parameters(double a, double b, int J, double* out, double* bound) {
  if (!(a > 0.0) || !(b >= a) || !std::isfinite(b) || J < 1 || J > kAdiCap || !out)
    return TDT_ERR_INVALID_ARG;
  std::vector<long double> w;
  adi_parameters(a, b, J, w);
  long double d = 1.0L;
  for (int j = 0; j < J; ++j) {
    out[j] = (double)w[(size_t)j];
    d *= std::fabs((w[(size_t)j] - a) / (w[(size_t)j] + a));
  }
  if (bound) *bound = (double)d;
  return TDT_OK;
}

tdt_status_t tdt_poisson3d_destroy(tdt_poisson3d_t p) {
  if (!p) return TDT_ERR_INVALID_ARG;
  destroy_poisson3d(p);
  return TDT_OK;
}

}  // extern "C"
