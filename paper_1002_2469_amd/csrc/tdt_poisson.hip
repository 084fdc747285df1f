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

#include <cmath>
#include <new>
#include <vector>

#include "tdt.h"

struct tdt_poisson_s {
  int64_t nx = 0, ny = 0;
  double hx = 0.0, hy = 0.0;
  tdt_plan_t line = nullptr;     // Nx Toeplitz systems of Ny rows (mode-major)
  hipfftHandle fft = 0;          // Ny real transforms of length Nx + 1
  bool fft_made = false;
  double* sn = nullptr;          // sin(pi j / (Nx + 1)), j = 0 .. Nx
  double* y = nullptr;           // [Ny][Nx + 1] folded rows
  double* spec = nullptr;        // [Ny][(Nx + 1) / 2 + 1] complex spectra
  double* T = nullptr;           // [Nx][Ny] mode-major right-hand sides
  double* V = nullptr;           // [Nx][Ny] mode-major solutions
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
// U non-null (the inverse transform) the row's coefficients S_1..S_Nx are
// written to U's row instead, unscaled.  One workgroup per row walks it in
// segments of 4 kScanNT entries: each thread takes 4 consecutive entries
// (coalesced), the thread totals are scanned across the wavefront by
// shuffles and across the wavefronts through LDS, and a carry runs from
// segment to segment (a fixed summation order).
__global__ __launch_bounds__(kScanNT) void k_scan_rows(double* __restrict__ spec,
                                                       int64_t nx, int64_t ny,
                                                       double* __restrict__ U) {
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
          if (2 * k + 1 <= nx) u[2 * k] = acc;
          if (k >= 1 && 2 * k <= nx) u[2 * k - 1] = -im[e];
        } else {
          row[2 * k] = acc;
        }
      }
      carry += seg;
      __syncthreads();   // wtot is rewritten by the next segment
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

void destroy_poisson(tdt_poisson_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->line) (void)tdt_plan_destroy(p->line);
  if (p->fft_made) (void)hipfftDestroy(p->fft);
  (void)hipFree(p->sn);
  (void)hipFree(p->y);
  (void)hipFree(p->spec);
  (void)hipFree(p->T);
  (void)hipFree(p->V);
  delete p;
}

}  // namespace

extern "C" {

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
  tdt_status_t st = tdt_plan_varlen_create(nx, off.data(), tm1.data(), t0.data(), t1.data(),
                                           dtype, &p->line);
  if (st < 0) {
    destroy_poisson(p);
    return st;
  }
  st = tdt_plan_reserve(p->line, 1);
  const int64_t n = nx + 1, K = n / 2 + 1;
  if (st == TDT_OK &&
      (hipMalloc(&p->sn, (size_t)n * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->y, (size_t)(ny * n) * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->spec, (size_t)(ny * K) * 2 * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->T, (size_t)(nx * ny) * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->V, (size_t)(nx * ny) * sizeof(double)) != hipSuccess))
    st = TDT_ERR_OOM;
  if (st == TDT_OK) {
    std::vector<double> sn((size_t)n);
    for (int64_t j = 0; j < n; ++j) sn[(size_t)j] = (double)std::sin(pi * (long double)j / n);
    if (hipMemcpy(p->sn, sn.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess)
      st = TDT_ERR_HIP;
  }
  if (st == TDT_OK) {
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
  if (hipfftSetStream(p->fft, stream) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  auto gy = [](int64_t v) { return (unsigned)(v < (int64_t)kMaxGridY ? v : kMaxGridY); };
  const dim3 tiles((unsigned)((nx + 1 + kTileP - 1) / kTileP), gy((ny + kTileP - 1) / kTileP));
  auto* spec = reinterpret_cast<hipfftDoubleComplex*>(p->spec);
  // sine transform of the rows, scaled and transposed to mode-major order
  hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((n + 255) / 256), gy(ny)), dim3(256), 0,
                     stream, F, p->sn, p->y, nx, ny);
  if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  hipLaunchKernelGGL(k_scan_rows, dim3(gy(ny)), dim3(kScanNT), 0, stream, p->spec, nx, ny,
                     (double*)nullptr);
  const double s = p->hy * p->hy * 2.0 / (double)(nx + 1);
  hipLaunchKernelGGL(k_modes_from_rows, tiles, dim3(kTileP, 8), 0, stream, p->spec, p->T, nx,
                     ny, s);
  // one Toeplitz system per mode
  tdt_status_t st = tdt_solve_varlen(p->line, p->T, p->V, stream);
  if (st < 0) return st;
  // inverse transform: the same sine transform of the mode coefficients
  hipLaunchKernelGGL(k_fold_modes, tiles, dim3(kTileP, 8), 0, stream, p->V, p->sn, p->y, nx,
                     ny);
  if (hipfftExecD2Z(p->fft, p->y, spec) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  hipLaunchKernelGGL(k_scan_rows, dim3(gy(ny)), dim3(kScanNT), 0, stream, p->spec, nx, ny, U);
  return hipGetLastError() == hipSuccess ? TDT_OK : TDT_ERR_HIP;
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
