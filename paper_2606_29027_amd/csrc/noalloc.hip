// Allocation-free variant of the spectral Poisson solve (slar_poisson):
// the same kernels (DFT/FFT lines, the Poisson symbol, inverse transform)
// run on scratch memory taken from a file-scope device array instead of a
// workspace, for callers that cannot allocate device memory.
//
// The array's host-side name is only a handle: every use goes through the
// device address obtained once per device with hipGetSymbolAddress.  Calls
// that overlap in time on one device share that device's array and race;
// a call writes every scratch element it reads, so nothing carries over
// from the previous call.
#include <array>
#include <cmath>
#include <mutex>

#include "slar_internal.h"
#include "fields.h"

namespace slar {

// twiddles of the two axes (2 SLAR_NLINE doubles each), then the transform
// buffers of the largest grid (2D, Nx = 128^2): rho, the forward transform,
// the symbol output (1 + dx fields), the line-transform temporaries
// (2 (1 + dx) complex fields) and the real output (1 + dx fields)
constexpr size_t NOALLOC_TW = 4 * (size_t)SLAR_NLINE;
constexpr size_t NOALLOC_PER_NX = 1 + 2 + 2 * 3 + 4 * 3 + 3;   // dx = 2
constexpr size_t NOALLOC_ELEMS = NOALLOC_TW + NOALLOC_PER_NX * (size_t)SLAR_NMAX * SLAR_NMAX;

static __device__ __align__(256) double scratch[NOALLOC_ELEMS];

constexpr int NOALLOC_MAXDEV = 64;
static std::mutex g_mu;
static std::array<double*, NOALLOC_MAXDEV> g_ptr{};

// device address of this device's scratch array (resolved once per device)
static hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAXDEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

__global__ void k_twiddles(int n, double* tw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double a = 2.0 * M_PI * (double)t / (double)n;
  tw[2 * t] = cos(a);
  tw[2 * t + 1] = sin(a);
}

__global__ void k_rho_of_ne(int n, const double* __restrict__ ne, double ni, double* __restrict__ rho) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) rho[e] = ni - ne[e];
}

size_t noalloc_scratch_elems(const GridDev& G) {
  const size_t per = 1 + 2 + 2 * (1 + G.dx) + 4 * (1 + G.dx) + (1 + G.dx);
  return NOALLOC_TW + per * (size_t)G.nx;
}

slar_status poisson_noalloc_run(hipStream_t s, const slar_grid& grid, const double* n_e, double n_i,
                                double* phi, double* E) {
  const GridDev G = make_grid(grid);
  if (noalloc_scratch_elems(G) > NOALLOC_ELEMS) return SLAR_E_NOMEM;
  double* base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) return SLAR_E_HIP;
  const int Nx = G.nx, B = 1 + G.dx;
  double* tw0 = base;
  double* tw1 = base + 2 * SLAR_NLINE;
  double* p = base + NOALLOC_TW;
  double* rho = p; p += Nx;
  double2* c0 = (double2*)p; p += 2 * (size_t)Nx;
  double2* c1 = (double2*)p; p += 2 * (size_t)B * Nx;
  double2* tmp = (double2*)p; p += 4 * (size_t)B * Nx;
  double* out = p;
  // a view of the grid for the shared transform helpers: no device memory
  // of its own (only the grid, the twiddle pointers and the lengths are read)
  Workspace view;
  view.grid = grid;
  view.G = G;
  view.tw[0] = tw0;
  view.tw[1] = tw1;
  k_twiddles<<<(G.n[0] + 255) / 256, 256, 0, s>>>(G.n[0], tw0);
  if (G.dx == 2) k_twiddles<<<(G.n[1] + 255) / 256, 256, 0, s>>>(G.n[1], tw1);
  k_rho_of_ne<<<(Nx + 255) / 256, 256, 0, s>>>(Nx, n_e, n_i, rho);
  if (hipGetLastError() != hipSuccess) return SLAR_E_HIP;
  if (dft_forward(s, &view, 1, rho, c0, tmp) != hipSuccess) return SLAR_E_HIP;
  if (spectral_symbol(s, &view, 0, 1, c0, c1) != hipSuccess) return SLAR_E_HIP;
  if (dft_inverse(s, &view, B, c1, out, tmp) != hipSuccess) return SLAR_E_HIP;
  if (phi && hipMemcpyAsync(phi, out, sizeof(double) * Nx, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return SLAR_E_HIP;
  if (hipMemcpyAsync(E, out + Nx, sizeof(double) * Nx * G.dx, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return SLAR_E_HIP;
  return SLAR_OK;
}

}  // namespace slar
