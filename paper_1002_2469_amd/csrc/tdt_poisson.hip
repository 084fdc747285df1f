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
// The sine transform of a row of length n is taken from a real FFT of its
// odd extension (0, f_1..f_n, 0, -f_n..-f_1) of length 2(n+1): the FFT's
// imaginary part at k is -2 sum_i f_i sin(pi k i / (n+1)).  The FFTs are
// hipFFT's; packing, the scaled transposes into and out of mode-major order,
// and the line solves are this library's kernels.
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
  hipfftHandle fft = 0;          // Ny real transforms of length 2 (Nx + 1)
  bool fft_made = false;
  double* ext = nullptr;         // [Ny][2 (Nx + 1)] odd extensions
  double* spec = nullptr;        // [Ny][Nx + 2] complex spectra
  double* T = nullptr;           // [Nx][Ny] mode-major right-hand sides
  double* V = nullptr;           // [Nx][Ny] mode-major solutions
};

namespace {

constexpr int kTileP = 32;       // transpose tile (kTileP x kTileP, kTileP x 8 threads)
constexpr unsigned kMaxGridY = 32768;   // the y dimension of a launch walks the rest

// ext[j][n] = the odd extension of row j of F (n = 0 .. 2 Nx + 1)
__global__ void k_pack_rows(const double* __restrict__ F, double* __restrict__ ext, int64_t nx,
                            int64_t ny) {
  const int64_t w = 2 * (nx + 1);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= w) return;
  for (int64_t j = blockIdx.y; j < ny; j += gridDim.y) {
    const double* f = F + j * nx;
    double v = 0.0;
    if (n >= 1 && n <= nx) v = f[n - 1];
    else if (n >= nx + 2) v = -f[2 * nx + 1 - n];
    ext[j * w + n] = v;
  }
}

// T[k][j] = s * (-Im spec[j][k+1] / 2), k < Nx, j < Ny: the scaled sine
// coefficients, transposed to mode-major order through an LDS tile.
__global__ void k_extract_modes(const double* __restrict__ spec, double* __restrict__ T,
                                int64_t nx, int64_t ny, double s) {
  __shared__ double tile[kTileP][kTileP + 1];
  const int64_t k0 = (int64_t)blockIdx.x * kTileP;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t cw = nx + 2;   // complex entries per spectrum row
  for (int64_t j0 = (int64_t)blockIdx.y * kTileP; j0 < ny; j0 += (int64_t)gridDim.y * kTileP) {
    __syncthreads();   // the previous tile is read
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t j = j0 + r, k = k0 + tx;
      if (j < ny && k < nx) tile[r][tx] = -0.5 * s * spec[2 * (j * cw + k + 1) + 1];
    }
    __syncthreads();
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t k = k0 + r, j = j0 + tx;
      if (k < nx && j < ny) T[k * ny + j] = tile[tx][r];
    }
  }
}

// ext[j][n] = the odd extension of the mode coefficients of row j: V[n-1][j]
// at n = 1..Nx, -V[2Nx+1-n][j] at n = Nx+2..2Nx+1, 0 at n = 0 and Nx+1
// (the transpose back to row-major order through an LDS tile).
__global__ void k_pack_modes(const double* __restrict__ V, double* __restrict__ ext, int64_t nx,
                             int64_t ny) {
  __shared__ double tile[kTileP][kTileP + 1];
  const int64_t k0 = (int64_t)blockIdx.x * kTileP;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t w = 2 * (nx + 1);
  for (int64_t j0 = (int64_t)blockIdx.y * kTileP; j0 < ny; j0 += (int64_t)gridDim.y * kTileP) {
    __syncthreads();   // the previous tile is read
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t k = k0 + r, j = j0 + tx;
      if (k < nx && j < ny) tile[r][tx] = V[k * ny + j];
    }
    __syncthreads();
    for (int r = ty; r < kTileP; r += blockDim.y) {
      const int64_t j = j0 + r, k = k0 + tx;
      if (j < ny && k < nx) {
        const double v = tile[tx][r];
        ext[j * w + k + 1] = v;
        ext[j * w + 2 * nx + 1 - k] = -v;
        if (k == 0) {
          ext[j * w] = 0.0;
          ext[j * w + nx + 1] = 0.0;
        }
      }
    }
  }
}

// U[j][i] = -Im spec[j][i+1] / 2: the inverse sine transform of row j
__global__ void k_extract_rows(const double* __restrict__ spec, double* __restrict__ U,
                               int64_t nx, int64_t ny) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  for (int64_t j = blockIdx.y; j < ny; j += gridDim.y)
    U[j * nx + i] = -0.5 * spec[2 * (j * (nx + 2) + i + 1) + 1];
}

void destroy_poisson(tdt_poisson_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->line) (void)tdt_plan_destroy(p->line);
  if (p->fft_made) (void)hipfftDestroy(p->fft);
  (void)hipFree(p->ext);
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
  const int64_t w = 2 * (nx + 1);
  if (st == TDT_OK &&
      (hipMalloc(&p->ext, (size_t)(ny * w) * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->spec, (size_t)(ny * (nx + 2)) * 2 * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->T, (size_t)(nx * ny) * sizeof(double)) != hipSuccess ||
       hipMalloc(&p->V, (size_t)(nx * ny) * sizeof(double)) != hipSuccess))
    st = TDT_ERR_OOM;
  if (st == TDT_OK) {
    int n[1] = {(int)w};
    if (hipfftPlanMany(&p->fft, 1, n, nullptr, 1, (int)w, nullptr, 1, (int)(nx + 2),
                       HIPFFT_D2Z, (int)ny) != HIPFFT_SUCCESS)
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
  const int64_t nx = p->nx, ny = p->ny, w = 2 * (nx + 1);
  if (hipfftSetStream(p->fft, stream) != HIPFFT_SUCCESS) return TDT_ERR_HIP;
  auto gy = [](int64_t n) { return (unsigned)(n < (int64_t)kMaxGridY ? n : kMaxGridY); };
  hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)((w + 255) / 256), gy(ny)), dim3(256), 0,
                     stream, F, p->ext, nx, ny);
  if (hipfftExecD2Z(p->fft, p->ext, reinterpret_cast<hipfftDoubleComplex*>(p->spec)) !=
      HIPFFT_SUCCESS)
    return TDT_ERR_HIP;
  const double s = p->hy * p->hy * 2.0 / (double)(nx + 1);
  hipLaunchKernelGGL(k_extract_modes,
                     dim3((unsigned)((nx + kTileP - 1) / kTileP), gy((ny + kTileP - 1) / kTileP)),
                     dim3(kTileP, 8), 0, stream, p->spec, p->T, nx, ny, s);
  tdt_status_t st = tdt_solve_varlen(p->line, p->T, p->V, stream);
  if (st < 0) return st;
  hipLaunchKernelGGL(k_pack_modes,
                     dim3((unsigned)((nx + kTileP - 1) / kTileP), gy((ny + kTileP - 1) / kTileP)),
                     dim3(kTileP, 8), 0, stream, p->V, p->ext, nx, ny);
  if (hipfftExecD2Z(p->fft, p->ext, reinterpret_cast<hipfftDoubleComplex*>(p->spec)) !=
      HIPFFT_SUCCESS)
    return TDT_ERR_HIP;
  hipLaunchKernelGGL(k_extract_rows, dim3((unsigned)((nx + 255) / 256), gy(ny)), dim3(256), 0,
                     stream, p->spec, U, nx, ny);
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
