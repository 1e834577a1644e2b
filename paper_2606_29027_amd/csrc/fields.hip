// Fields on the x-grid: velocity moments of a frame-form tensor and the
// spectral (DFT) Poisson solve / derivatives (eqs. (Poisson), (Efromphi);
// section 3.2.3 uses FFT-based differentiation for all field terms).
//
// The transforms are direct DFTs along each axis, one block per line with
// the line and the twiddle table in LDS: N <= 128 per axis, so a line is
// N^2 <= 16384 complex FMAs and the whole 2D transform of a 128^2 field is
// spread over 2 x 128 blocks.  This handles every N (the batched workload
// has N = 48, 96), not only powers of two.
#include <cmath>

#include "slar_internal.h"
#include "dense.h"
#include "fields.h"
#include "group.h"

namespace slar {

// ---------------------------------------------------------- twiddles
void host_twiddles(int n, std::vector<double>& tw) {
  tw.resize(2 * n);
  for (int t = 0; t < n; ++t) {
    // reduce the angle exactly: 2 pi t / n
    const double a = 2.0 * M_PI * (double)t / (double)n;
    tw[2 * t] = std::cos(a);
    tw[2 * t + 1] = std::sin(a);
  }
}

// line transform along the last axis (axis = 1) or the first (axis = 0)
// of [B][n0][n1] complex (double2) data; sign -1 forward, +1 inverse.
__device__ __forceinline__ void dft_line_dev(int n0, int n1, int axis, double sign, const double2* __restrict__ in,
                                             const double* __restrict__ realin, double2* __restrict__ out,
                                             const double* __restrict__ tw, int other, int b) {
  __shared__ double2 line[SLAR_NLINE];
  __shared__ double2 w[SLAR_NLINE];
  const int L = axis == 1 ? n1 : n0;          // line length
  const long long base = (long long)b * n0 * n1;
  const int t = threadIdx.x;
  for (int e = t; e < L; e += blockDim.x) {
    const long long off = axis == 1 ? base + (long long)other * n1 + e : base + (long long)e * n1 + other;
    line[e] = realin ? make_double2(realin[off], 0.0) : in[off];
    w[e] = make_double2(tw[2 * e], sign * tw[2 * e + 1]);
  }
  __syncthreads();
  for (int kk = t; kk < L; kk += blockDim.x) {
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int i = 0; i < L; ++i) {
      const double2 x = line[i], ww = w[idx];
      re += x.x * ww.x - x.y * ww.y;
      im += x.x * ww.y + x.y * ww.x;
      idx += kk;
      if (idx >= L) idx -= L;
    }
    const long long off = axis == 1 ? base + (long long)other * n1 + kk : base + (long long)kk * n1 + other;
    out[off] = make_double2(re, im);
  }
}

__global__ void k_dft_line(int n0, int n1, int axis, double sign, const double2* __restrict__ in,
                           const double* __restrict__ realin, double2* __restrict__ out,
                           const double* __restrict__ tw) {
  dft_line_dev(n0, n1, axis, sign, in, realin, out, tw, blockIdx.x, blockIdx.y);
}

// Radix-2 Cooley--Tukey stages over `nl` lines of length L = 2^logL held
// in LDS in bit-reversed order (line l at a + l * L); the block's threads
// share the butterflies of all lines, one barrier per stage.
__device__ void fft_stages(double2* a, int nl, int L, const double* __restrict__ tw, double sign) {
  const int nt = blockDim.x, t = threadIdx.x;
  for (int len = 2; len <= L; len <<= 1) {
    const int hl = len >> 1;
    for (int q = t; q < nl * (L / 2); q += nt) {
      const int l = q / (L / 2), bt = q % (L / 2);
      const int grp = bt / hl, pos = bt % hl;
      const int i = l * L + grp * len + pos, j = i + hl;
      const int ti = pos * (L / len);
      const double wr = tw[2 * ti], wi = sign * tw[2 * ti + 1];
      const double2 u = a[i], x = a[j];
      const double2 v = make_double2(x.x * wr - x.y * wi, x.x * wi + x.y * wr);
      a[i] = make_double2(u.x + v.x, u.y + v.y);
      a[j] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

// FFT of one line (n a power of two <= SLAR_NLINE) per block: bit-reversed
// load, log2(n) butterfly stages.  With realout set, the scaled real part
// is stored instead of the complex line.
__device__ __forceinline__ void fft_line_dev(int n0, int n1, int axis, double sign, const double2* __restrict__ in,
                                             const double* __restrict__ realin, double2* __restrict__ out,
                                             double* __restrict__ realout, double scale,
                                             const double* __restrict__ tw, int logL, int other, int b) {
  __shared__ double2 a[SLAR_NLINE];
  const int L = axis == 1 ? n1 : n0;
  const long long base = (long long)b * n0 * n1;
  const int t = threadIdx.x;
  for (int e = t; e < L; e += blockDim.x) {
    const long long off = axis == 1 ? base + (long long)other * n1 + e : base + (long long)e * n1 + other;
    const double2 v = realin ? make_double2(realin[off], 0.0) : in[off];
    const int r = __brev((unsigned)e) >> (32 - logL);
    a[r] = v;
  }
  __syncthreads();
  fft_stages(a, 1, L, tw, sign);
  for (int e = t; e < L; e += blockDim.x) {
    const long long off = axis == 1 ? base + (long long)other * n1 + e : base + (long long)e * n1 + other;
    if (realout) realout[off] = a[e].x * scale;
    else out[off] = a[e];
  }
}

__global__ void k_fft_line(int n0, int n1, int axis, double sign, const double2* __restrict__ in,
                           const double* __restrict__ realin, double2* __restrict__ out,
                           double* __restrict__ realout, double scale,
                           const double* __restrict__ tw, int logL) {
  fft_line_dev(n0, n1, axis, sign, in, realin, out, realout, scale, tw, logL, blockIdx.x, blockIdx.y);
}

// grouped line transforms: problem d owns others x B blocks (line, field)
__global__ __launch_bounds__(64) void k_fft_line_group(const LineDesc* __restrict__ D, const int* __restrict__ first,
                                                       int nd) {
  const int bk = blockIdx.x;
  const int d = group_find(first, nd, bk);
  const LineDesc g = D[d];
  const int local = bk - first[d];
  const int others = g.axis == 1 ? g.n0 : g.n1;
  fft_line_dev(g.n0, g.n1, g.axis, g.sign, g.in, g.realin, g.out, nullptr, 0.0, g.tw, g.logL, local % others,
               local / others);
}
__global__ __launch_bounds__(128) void k_dft_line_group(const LineDesc* __restrict__ D, const int* __restrict__ first,
                                                        int nd) {
  const int bk = blockIdx.x;
  const int d = group_find(first, nd, bk);
  const LineDesc g = D[d];
  const int local = bk - first[d];
  const int others = g.axis == 1 ? g.n0 : g.n1;
  dft_line_dev(g.n0, g.n1, g.axis, g.sign, g.in, g.realin, g.out, g.tw, local % others, local / others);
}

static int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return ((1 << l) == n) ? l : -1;
}

// one batch of line transforms along an axis: FFT for powers of two, DFT otherwise
static void line_transform(hipStream_t s, int n0, int n1, int axis, double sign, const double2* in,
                           const double* realin, double2* out, const double* tw, int B) {
  const int L = axis == 1 ? n1 : n0;
  const int others = axis == 1 ? n0 : n1;
  const int lg = log2_exact(L);
  if (lg >= 1)
    k_fft_line<<<dim3(others, B), 64, 0, s>>>(n0, n1, axis, sign, in, realin, out, nullptr, 0.0, tw, lg);
  else
    k_dft_line<<<dim3(others, B), 128, 0, s>>>(n0, n1, axis, sign, in, realin, out, tw);
}

__global__ void k_take_real(long long n, const double2* __restrict__ in, double scale,
                            double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = in[e].x * scale;
}


// Forward 2D DFT of B real fields [B][Nx] into complex [B][Nx].
hipError_t dft_forward(hipStream_t s, Workspace* ws, int B, const double* in, double2* out,
                       double2* tmp) {
  const GridDev& G = ws->G;
  const int n0 = G.n[0], n1 = (G.dx == 2) ? G.n[1] : 1;
  if (G.dx == 2) {
    line_transform(s, n0, n1, 1, -1.0, nullptr, in, tmp, ws->tw[1], B);
    line_transform(s, n0, n1, 0, -1.0, tmp, nullptr, out, ws->tw[0], B);
  } else {
    line_transform(s, n0, 1, 0, -1.0, nullptr, in, out, ws->tw[0], B);
  }
  return hipGetLastError();
}

// Inverse 2D DFT of B complex fields, real part, scaled by 1/Nx.
hipError_t dft_inverse(hipStream_t s, Workspace* ws, int B, const double2* in, double* out,
                       double2* tmp) {
  const GridDev& G = ws->G;
  const int n0 = G.n[0], n1 = (G.dx == 2) ? G.n[1] : 1;
  const long long tot = (long long)B * G.nx;
  if (G.dx == 2) {
    line_transform(s, n0, n1, 0, 1.0, in, nullptr, tmp, ws->tw[0], B);
    line_transform(s, n0, n1, 1, 1.0, tmp, nullptr, (double2*)tmp + tot, ws->tw[1], B);
    k_take_real<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(tot, (double2*)tmp + tot, 1.0 / G.nx, out);
  } else {
    line_transform(s, n0, 1, 0, 1.0, in, nullptr, tmp, ws->tw[0], B);
    k_take_real<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(tot, tmp, 1.0 / G.nx, out);
  }
  return hipGetLastError();
}

// wavenumber of index i on an axis of n cells and length L, Nyquist -> 0
__device__ __forceinline__ double wavenum(int i, int n, double L) {
  if ((n % 2) == 0 && i == n / 2) return 0.0;
  const int m = (i < (n + 1) / 2) ? i : i - n;
  return 2.0 * M_PI * (double)m / L;
}

struct Kgrid { int n0, n1, dx; double L0, L1; };

__device__ __forceinline__ void kvec(const Kgrid& K, long long e, double* k) {
  const int i0 = (int)(e / K.n1), i1 = (int)(e % K.n1);
  k[0] = wavenum(i0, K.n0, K.L0);
  k[1] = K.dx == 2 ? wavenum(i1, K.n1, K.L1) : 0.0;
}

// Symbol application.  op: 0 Poisson (rho^ -> phi^, E^_m = -i k_m phi^),
// 1 gradient (f^ -> i k_m f^), 2 divergence (F^[m] -> sum i k_m F^_m),
// 3 inverse negative Laplacian (f^ -> f^ / |k|^2, 0 on null modes).
// in/out strides are in fields of Nx complex values.
__device__ __forceinline__ void symbol_dev(const Kgrid& K, int op, int nvec, const double2* __restrict__ in,
                                           double2* __restrict__ out, int Nx, long long e) {
  if (e >= (long long)Nx * nvec) return;
  const int v = (int)(e / Nx);
  const long long p = e % Nx;
  double k[2];
  kvec(K, p, k);
  const double k2 = k[0] * k[0] + k[1] * k[1];
  if (op == 0) {
    const double2 r = in[(long long)v * Nx + p];
    const double2 ph = k2 > 0.0 ? make_double2(r.x / k2, r.y / k2) : make_double2(0.0, 0.0);
    double2* o = out + (long long)v * (1 + K.dx) * Nx;
    o[p] = ph;
    for (int m = 0; m < K.dx; ++m)  // -i k ph
      o[(long long)(1 + m) * Nx + p] = make_double2(k[m] * ph.y, -k[m] * ph.x);
  } else if (op == 1) {
    const double2 f = in[(long long)v * Nx + p];
    for (int m = 0; m < K.dx; ++m)
      out[((long long)v * K.dx + m) * Nx + p] = make_double2(-k[m] * f.y, k[m] * f.x);
  } else if (op == 2) {
    double re = 0.0, im = 0.0;
    for (int m = 0; m < K.dx; ++m) {
      const double2 f = in[((long long)v * K.dx + m) * Nx + p];
      re += -k[m] * f.y;
      im += k[m] * f.x;
    }
    out[(long long)v * Nx + p] = make_double2(re, im);
  } else {
    const double2 f = in[(long long)v * Nx + p];
    out[(long long)v * Nx + p] = k2 > 0.0 ? make_double2(f.x / k2, f.y / k2) : make_double2(0.0, 0.0);
  }
}

__global__ void k_symbol(Kgrid K, int op, int nvec, const double2* __restrict__ in,
                         double2* __restrict__ out, int Nx) {
  symbol_dev(K, op, nvec, in, out, Nx, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// grouped pointwise field steps (FieldDesc.op): rho = n_i - n_e, the
// scaled real part, or the symbol map; one element per thread
__global__ __launch_bounds__(256) void k_field_group(const FieldDesc* __restrict__ D, const int* __restrict__ first,
                                                     int nd) {
  const int bk = blockIdx.x;
  const int d = group_find(first, nd, bk);
  const FieldDesc g = D[d];
  const long long e = (long long)(bk - first[d]) * 256 + threadIdx.x;
  if (g.op == FIELD_RHO) {
    if (e < g.n) g.rout[e] = g.ni - g.rin[e];
  } else if (g.op == FIELD_REAL) {
    if (e < g.n) g.rout[e] = g.cin[e].x * g.scale;
  } else {
    const Kgrid K{g.n0, g.n1, g.dx, g.L0, g.L1};
    symbol_dev(K, g.sym, g.nvec, g.cin, g.cout, g.Nx, e);
  }
}

hipError_t spectral_symbol(hipStream_t s, Workspace* ws, int op, int nvec, const double2* in,
                           double2* out) {
  const GridDev& G = ws->G;
  Kgrid K{G.n[0], G.dx == 2 ? G.n[1] : 1, G.dx, ws->grid.hi[0] - ws->grid.lo[0],
          G.dx == 2 ? ws->grid.hi[1] - ws->grid.lo[1] : 1.0};
  const long long n = (long long)G.nx * nvec;
  k_symbol<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(K, op, nvec, in, out, G.nx);
  return hipGetLastError();
}

// ------------------------------------------------------ spectral stages
// A spectral stage maps Bin real fields to Bout real fields through one
// pointwise operation per Fourier mode (all field terms of the macroscopic
// residual and the per-mode preconditioner are of this form):
//   SPEC_POISSON  rho -> (phi, E_m = -i k_m phi), phi = rho / |k|^2
//   SPEC_DTPHI    J_m -> i k_m dtphi, dtphi = -(sum_m i k_m J_m) / |k|^2
//   SPEC_DIV      F[q][m] -> sum_m i k_m F[q][m]
//   SPEC_PRECOND  x_b -> sum_b Minv[a][b] x_b (per-mode K x K inverse; the
//                 modes stored transposed, pm = i1 n0 + i0 for p = i0 n1 + i1)
//   SPEC_FILTER   x_q -> sigma x_q, sigma = prod_d exp(-36 kappa_d^8),
//                 kappa_d = |m_d| / (n_d / 2) the mode index of axis d
//                 relative to the Nyquist index (1 on the zero mode)
// Null modes (|k| = 0) and Nyquist wavenumbers map to zero as in k_symbol.
constexpr int SPEC_MAXIN = 8, SPEC_MAXOUT = 4;

// one axis of the exponential filter exp(-36 kappa^8), kappa = |m| / (n / 2),
// from the mode index i of n cells
__device__ __forceinline__ double filt_axis(int i, int n) {
  if (n <= 1) return 1.0;
  const int m = i < n - i ? i : n - i;
  const double kap = (double)m / (0.5 * n);
  const double k2 = kap * kap, k4 = k2 * k2;
  return exp(-36.0 * (k4 * k4));
}

__device__ __forceinline__ void spec_map(int op, int dx, int K, const double* k, const double2* x,
                                         double2* y, const double2* __restrict__ Minv, long long pm,
                                         int Nx, double sigma) {
  const double k2 = k[0] * k[0] + k[1] * k[1];
  if (op == SPEC_FILTER) {
    for (int q = 0; q < K; ++q) y[q] = make_double2(sigma * x[q].x, sigma * x[q].y);
    return;
  }
  if (op == SPEC_POISSON) {
    const double2 ph = k2 > 0.0 ? make_double2(x[0].x / k2, x[0].y / k2) : make_double2(0.0, 0.0);
    y[0] = ph;
    for (int m = 0; m < dx; ++m) y[1 + m] = make_double2(k[m] * ph.y, -k[m] * ph.x);
  } else if (op == SPEC_DTPHI) {
    double dre = 0.0, dim = 0.0;
    for (int m = 0; m < dx; ++m) {
      dre += -k[m] * x[m].y;
      dim += k[m] * x[m].x;
    }
    double pre = 0.0, pim = 0.0;
    if (k2 > 0.0) { pre = -dre / k2; pim = -dim / k2; }
    for (int m = 0; m < dx; ++m) y[m] = make_double2(-k[m] * pim, k[m] * pre);
  } else if (op == SPEC_DIV) {
    for (int q = 0; q < K; ++q) {
      double re = 0.0, im = 0.0;
      for (int m = 0; m < dx; ++m) {
        re += -k[m] * x[q * dx + m].y;
        im += k[m] * x[q * dx + m].x;
      }
      y[q] = make_double2(re, im);
    }
  } else {
    for (int a = 0; a < K; ++a) {
      double sr = 0.0, si = 0.0;
      for (int b = 0; b < K; ++b) {
        const double2 m = Minv[(size_t)(a * K + b) * Nx + pm];
        sr += m.x * x[b].x - m.y * x[b].y;
        si += m.x * x[b].y + m.y * x[b].x;
      }
      y[a] = make_double2(sr, si);
    }
  }
}

static void spec_counts(int op, int dx, int K, int* bin, int* bout) {
  switch (op) {
    case SPEC_POISSON: *bin = 1; *bout = 1 + dx; break;
    case SPEC_DTPHI: *bin = dx; *bout = dx; break;
    case SPEC_DIV: *bin = K * dx; *bout = K; break;
    default: *bin = K; *bout = K; break;
  }
}

// Fused axis-0 part of a stage: per block one line (index `other` along
// axis 1) of every input field: forward FFT, the pointwise map (outputs
// written in bit-reversed order), inverse FFT, store.  Inputs complex
// (after the axis-1 forward pass) or real (1D); outputs complex (before
// the axis-1 inverse pass) or scaled real (1D).  Dynamic LDS:
// (Bin + Bout) lines of n0 complex values.
__global__ __launch_bounds__(256) void k_spec_line(Kgrid Kg, int op, int K, int Bin, int Bout,
                                                   const double2* __restrict__ cin,
                                                   const double* __restrict__ realin,
                                                   double2* __restrict__ cout, double* __restrict__ realout,
                                                   double scale, const double2* __restrict__ Minv,
                                                   const double* __restrict__ tw, int logL) {
  extern __shared__ double2 sl[];
  const int L = Kg.n0, n1 = Kg.n1, Nx = Kg.n0 * Kg.n1;
  const int other = blockIdx.x, t = threadIdx.x;
  double2* a = sl;
  double2* b = sl + (size_t)Bin * L;
  for (int q = t; q < Bin * L; q += blockDim.x) {
    const int f = q / L, e = q % L;
    const long long off = (long long)f * Nx + (long long)e * n1 + other;
    const int r = __brev((unsigned)e) >> (32 - logL);
    a[f * L + r] = realin ? make_double2(realin[off], 0.0) : cin[off];
  }
  __syncthreads();
  fft_stages(a, Bin, L, tw, -1.0);
  for (int e = t; e < L; e += blockDim.x) {
    const long long p = (long long)e * n1 + other;
    double k[2];
    kvec(Kg, p, k);
    double2 x[SPEC_MAXIN], y[SPEC_MAXOUT];
    for (int f = 0; f < Bin; ++f) x[f] = a[f * L + e];
    const double sg = (op == SPEC_FILTER) ? filt_axis(e, Kg.n0) * (Kg.dx == 2 ? filt_axis(other, n1) : 1.0) : 1.0;
    spec_map(op, Kg.dx, K, k, x, y, Minv, (long long)other * L + e, Nx, sg);
    const int r = __brev((unsigned)e) >> (32 - logL);
    for (int g = 0; g < Bout; ++g) b[g * L + r] = y[g];
  }
  __syncthreads();
  fft_stages(b, Bout, L, tw, 1.0);
  for (int q = t; q < Bout * L; q += blockDim.x) {
    const int g = q / L, e = q % L;
    const long long off = (long long)g * Nx + (long long)e * n1 + other;
    if (realout) realout[off] = b[g * L + e].x * scale;
    else cout[off] = b[g * L + e];
  }
}

// the pointwise map alone, for grids the fused path does not take
__global__ void k_spec_point(Kgrid Kg, int op, int K, int Bin, int Bout, const double2* __restrict__ in,
                             double2* __restrict__ out, const double2* __restrict__ Minv, int Nx) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Nx) return;
  double k[2];
  kvec(Kg, p, k);
  double2 x[SPEC_MAXIN], y[SPEC_MAXOUT];
  for (int f = 0; f < Bin; ++f) x[f] = in[(size_t)f * Nx + p];
  const double sg = (op == SPEC_FILTER)
                        ? filt_axis(p / Kg.n1, Kg.n0) * (Kg.dx == 2 ? filt_axis(p % Kg.n1, Kg.n1) : 1.0) : 1.0;
  spec_map(op, Kg.dx, K, k, x, y, Minv, (long long)(p % Kg.n1) * Kg.n0 + p / Kg.n1, Nx, sg);
  for (int g = 0; g < Bout; ++g) out[(size_t)g * Nx + p] = y[g];
}

hipError_t spectral_stage(hipStream_t s, Workspace* ws, int op, const double* in, double* out,
                          const double2* Minv, double2* scr) {
  const GridDev& G = ws->G;
  const int Nx = G.nx, dx = G.dx, K = G.dv + 2;
  int Bin = 0, Bout = 0;
  spec_counts(op, dx, K, &Bin, &Bout);
  if (Bin > SPEC_MAXIN || Bout > SPEC_MAXOUT || (op == SPEC_PRECOND && !Minv)) return hipErrorInvalidValue;
  const Kgrid Kg{G.n[0], dx == 2 ? G.n[1] : 1, dx, ws->grid.hi[0] - ws->grid.lo[0],
                 dx == 2 ? ws->grid.hi[1] - ws->grid.lo[1] : 1.0};
  const int lg0 = log2_exact(Kg.n0), lg1 = dx == 2 ? log2_exact(Kg.n1) : 0;
  double2* c0 = scr;                          // Bin fields
  double2* c1 = scr + (size_t)Bin * Nx;       // Bout fields
  const size_t lds = sizeof(double2) * (size_t)(Bin + Bout) * Kg.n0;
  if (lg0 >= 1 && lg1 >= (dx == 2 ? 1 : 0)) {
    if (dx == 2) {
      k_fft_line<<<dim3(Kg.n0, Bin), 64, 0, s>>>(Kg.n0, Kg.n1, 1, -1.0, nullptr, in, c0, nullptr, 0.0,
                                                ws->tw[1], lg1);
      k_spec_line<<<Kg.n1, 256, lds, s>>>(Kg, op, K, Bin, Bout, c0, nullptr, c1, nullptr, 0.0, Minv,
                                          ws->tw[0], lg0);
      k_fft_line<<<dim3(Kg.n0, Bout), 64, 0, s>>>(Kg.n0, Kg.n1, 1, 1.0, c1, nullptr, nullptr, out,
                                                 1.0 / Nx, ws->tw[1], lg1);
    } else {
      k_spec_line<<<1, 256, lds, s>>>(Kg, op, K, Bin, Bout, nullptr, in, nullptr, out, 1.0 / Nx, Minv,
                                      ws->tw[0], lg0);
    }
    return hipGetLastError();
  }
  double2* tmp = c1 + (size_t)Bout * Nx;      // max(Bin, 2 Bout) fields
  HIP_CHK(dft_forward(s, ws, Bin, in, c0, tmp));
  k_spec_point<<<(Nx + 255) / 256, 256, 0, s>>>(Kg, op, K, Bin, Bout, c0, c1, Minv, Nx);
  HIP_CHK(hipGetLastError());
  return dft_inverse(s, ws, Bout, c1, out, tmp);
}

__global__ void k_rho(int n, const double* ne, double ni, double* rho) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) rho[e] = ni - ne[e];
}

// phi (may be null) and E [dx][Nx] from n_e.
hipError_t poisson_run(hipStream_t s, Workspace* ws, const double* n_e, double n_i, double* phi,
                       double* E) {
  const GridDev& G = ws->G;
  const int Nx = G.nx;
  double2* c0 = (double2*)ws->cbuf;
  double2* c1 = c0 + (size_t)4 * Nx;
  double2* tmp = c0 + (size_t)12 * Nx;
  double* rho = ws->cbuf + (size_t)2 * 40 * Nx;
  k_rho<<<(Nx + 255) / 256, 256, 0, s>>>(Nx, n_e, n_i, rho);
  hipError_t e = dft_forward(s, ws, 1, rho, c0, tmp);
  if (e != hipSuccess) return e;
  e = spectral_symbol(s, ws, 0, 1, c0, c1);
  if (e != hipSuccess) return e;
  double* out = rho + Nx;
  e = dft_inverse(s, ws, 1 + G.dx, c1, out, tmp);
  if (e != hipSuccess) return e;
  if (phi) HIP_CHK(hipMemcpyAsync(phi, out, sizeof(double) * Nx, hipMemcpyDeviceToDevice, s));
  HIP_CHK(hipMemcpyAsync(E, out + Nx, sizeof(double) * Nx * G.dx, hipMemcpyDeviceToDevice, s));
  return hipSuccess;
}

// ----------------------------------------------------------- moments
// Psi[J][q]: test functions times the velocity cell volume, order
// 1, v_mu, |v|^2, v_mu v_nu (mu <= nu), |v|^2 v_mu.
__global__ void k_psi(GridDev g, int nmom, double* psi) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= g.nv) return;
  const int dx = g.dx, dv = g.dv;
  double v[2];
  double vol = 1.0;
  if (dv == 1) {
    v[0] = g.lo[1] + ((double)J + 0.5) * g.h[1];
    vol = g.h[1];
  } else {
    v[0] = g.lo[2] + ((double)(J / g.n[3]) + 0.5) * g.h[2];
    v[1] = g.lo[3] + ((double)(J % g.n[3]) + 0.5) * g.h[3];
    vol = g.h[2] * g.h[3];
  }
  double v2 = 0.0;
  for (int m = 0; m < dv; ++m) v2 += v[m] * v[m];
  double* o = psi + (size_t)J * nmom;
  int q = 0;
  o[q++] = vol;
  for (int m = 0; m < dv; ++m) o[q++] = v[m] * vol;
  o[q++] = v2 * vol;
  for (int a = 0; a < dv; ++a)
    for (int b = a; b < dv; ++b) o[q++] = v[a] * v[b] * vol;
  for (int m = 0; m < dv; ++m) o[q++] = v2 * v[m] * vol;
  (void)dx;
}

int nmom_of(int dv) { return dv == 1 ? 5 : 9; }

hipError_t psi_build(hipStream_t s, Workspace* ws) {
  const GridDev& G = ws->G;
  k_psi<<<(G.nv + 255) / 256, 256, 0, s>>>(G, nmom_of(G.dv), ws->psi);
  return hipGetLastError();
}

// C (rows x cols) = A^T B with A = [n][lda] (first `rows` cols), B = [n][ldb],
// reduction over long n, deterministic split: chunks of `chunk` rows as one
// batched product (a single product over n runs on one tile), then a fixed
// order sum of the chunk products.
__device__ __forceinline__ void sum_batches_dev(const double* __restrict__ P, int M, int N, int batch,
                                                double* __restrict__ C, int ldc, double beta, int e) {
  if (e >= M * N) return;
  double acc = 0.0;
  for (int b = 0; b < batch; ++b) acc += P[(long long)b * M * N + e];
  double* c = C + (long long)(e / N) * ldc + (e % N);
  *c = (beta == 0.0) ? acc : acc + beta * (*c);
}

__global__ void k_sum_batches(const double* __restrict__ P, int M, int N, int batch,
                              double* __restrict__ C, int ldc, double beta) {
  sum_batches_dev(P, M, N, batch, C, ldc, beta, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_sum_batches_group(const SumDesc* __restrict__ D,
                                                           const int* __restrict__ first, int nd) {
  const int bk = blockIdx.x;
  const int d = group_find(first, nd, bk);
  const SumDesc g = D[d];
  sum_batches_dev(g.P, g.M, g.N, g.batch, g.C, g.ldc, 0.0, (bk - first[d]) * 256 + (int)threadIdx.x);
}

hipError_t gemm_tn_long(hipStream_t s, Workspace* ws, int rows, int cols, int n, const double* A,
                        int lda, const double* B, int ldb, double* C, int ldc) {
  int chunk = 256;
  while ((size_t)((n + chunk - 1) / chunk) * rows * cols > ws->dwork_elems) chunk *= 2;
  const int full = n / chunk, tail = n - full * chunk;
  if (full > 0) {
    hipError_t e = gemm_f64(s, true, false, rows, cols, chunk, 1.0, A, lda, (long long)chunk * lda, B, ldb,
                            (long long)chunk * ldb, 0.0, ws->dwork, cols, (long long)rows * cols, full);
    if (e != hipSuccess) return e;
    k_sum_batches<<<(rows * cols + 255) / 256, 256, 0, s>>>(ws->dwork, rows, cols, full, C, ldc, 0.0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (tail > 0)
    return gemm_f64(s, true, false, rows, cols, tail, 1.0, A + (long long)full * chunk * lda, lda,
                    0, B + (long long)full * chunk * ldb, ldb, 0, full > 0 ? 1.0 : 0.0, C, ldc, 0, 1);
  return hipSuccess;
}

// M [nmom][Nx] = X (Psi^T P)^T restricted to r columns.
hipError_t moments_run(hipStream_t s, Workspace* ws, const slar_frames& F, double* M) {
  const GridDev& G = ws->G;
  const int nmom = nmom_of(G.dv);
  double* m = ws->cbuf + (size_t)2 * 40 * G.nx + (size_t)8 * G.nx;   // [r][nmom]
  hipError_t e = gemm_tn_long(s, ws, F.r, nmom, G.nv, F.P, F.ld, ws->psi, nmom, m, nmom);
  if (e != hipSuccess) return e;
  // M^T = m^T X^T  -> [nmom][Nx]
  return gemm_f64(s, true, true, nmom, G.nx, F.r, 1.0, m, nmom, 0, F.X, F.ld, 0, 0.0, M, G.nx, 0, 1);
}

hipError_t line_group_launch(hipStream_t s, bool fft, const LineDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  if (fft) k_fft_line_group<<<nblocks, 64, 0, s>>>(d, first, nd);
  else k_dft_line_group<<<nblocks, 128, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t field_group_launch(hipStream_t s, const FieldDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_field_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t sum_group_launch(hipStream_t s, const SumDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_sum_batches_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

// moments_run and poisson_run for n problems, every step one grouped launch
// (the scratch of each problem as in the one-problem calls)
hipError_t efield_group(GroupQueue& q, int n, Workspace* const* ws, const slar_frames* F, const double* n_i,
                        double* const* M, double* const* E) {
  std::vector<GemmArgs> m1, m3, m4;
  std::vector<SumDesc> m2;
  std::vector<FieldDesc> rho, real;
  std::vector<FieldDesc> sym;
  std::vector<LineDesc> f1, f0, i0, i1;
  std::vector<CopyDesc> cpE;
  for (int j = 0; j < n; ++j) {
    Workspace* w = ws[j];
    const GridDev& G = w->G;
    const int Nx = G.nx, nmom = nmom_of(G.dv), r = F[j].r;
    // moments: m = P^T Psi (chunked, fixed-order sum), M = m^T X^T
    double* m = w->cbuf + (size_t)2 * 40 * Nx + (size_t)8 * Nx;
    {
      const int n_ = G.nv;
      int chunk = 256;
      while ((size_t)((n_ + chunk - 1) / chunk) * r * nmom > w->dwork_elems) chunk *= 2;
      const int full = n_ / chunk, tail = n_ - full * chunk;
      if (full > 0) {
        m1.push_back(GemmArgs{r, nmom, chunk, 1.0, F[j].P, F[j].ld, (long long)chunk * F[j].ld, w->psi, nmom,
                              (long long)chunk * nmom, 0.0, w->dwork, nmom, (long long)r * nmom, full});
        m2.push_back(SumDesc{r, nmom, full, nmom, w->dwork, m});
      }
      if (tail > 0)
        m3.push_back(GemmArgs{r, nmom, tail, 1.0, F[j].P + (long long)full * chunk * F[j].ld, F[j].ld, 0,
                              w->psi + (long long)full * chunk * nmom, nmom, 0, full > 0 ? 1.0 : 0.0, m, nmom, 0,
                              1});
    }
    m4.push_back(GemmArgs{nmom, Nx, r, 1.0, m, nmom, 0, F[j].X, F[j].ld, 0, 0.0, M[j], Nx, 0, 1});
    // Poisson: rho = n_i - n_e, forward transform, symbol, inverse of
    // (phi, E), real part, E copied out
    double2* c0 = (double2*)w->cbuf;
    double2* c1 = c0 + (size_t)4 * Nx;
    double2* tmp = c0 + (size_t)12 * Nx;
    double* rh = w->cbuf + (size_t)2 * 40 * Nx;
    double* out = rh + Nx;
    const int n0 = G.n[0], n1 = G.dx == 2 ? G.n[1] : 1;
    const int lg0 = log2_exact(n0), lg1 = G.dx == 2 ? log2_exact(n1) : 0;
    FieldDesc fr{};
    fr.op = FIELD_RHO; fr.n = Nx; fr.ni = n_i[j]; fr.rin = M[j]; fr.rout = rh;
    rho.push_back(fr);
    const int B = 1 + G.dx;
    const long long tot = (long long)B * Nx;
    if (G.dx == 2) {
      f1.push_back(LineDesc{n0, n1, 1, lg1, 1, -1.0, nullptr, rh, tmp, w->tw[1]});
      f0.push_back(LineDesc{n0, n1, 0, lg0, 1, -1.0, tmp, nullptr, c0, w->tw[0]});
      i0.push_back(LineDesc{n0, n1, 0, lg0, B, 1.0, c1, nullptr, tmp, w->tw[0]});
      i1.push_back(LineDesc{n0, n1, 1, lg1, B, 1.0, tmp, nullptr, tmp + tot, w->tw[1]});
    } else {
      f0.push_back(LineDesc{n0, 1, 0, lg0, 1, -1.0, nullptr, rh, c0, w->tw[0]});
      i0.push_back(LineDesc{n0, 1, 0, lg0, B, 1.0, c1, nullptr, tmp, w->tw[0]});
    }
    FieldDesc fs{};
    fs.op = FIELD_SYMBOL; fs.sym = 0; fs.nvec = 1; fs.Nx = Nx; fs.n0 = n0; fs.n1 = n1; fs.dx = G.dx;
    fs.L0 = w->grid.hi[0] - w->grid.lo[0];
    fs.L1 = G.dx == 2 ? w->grid.hi[1] - w->grid.lo[1] : 1.0;
    fs.cin = c0; fs.cout = c1;
    sym.push_back(fs);
    FieldDesc fx{};
    fx.op = FIELD_REAL; fx.n = tot; fx.scale = 1.0 / Nx; fx.cin = G.dx == 2 ? tmp + tot : tmp; fx.rout = out;
    real.push_back(fx);
    cpE.push_back(CopyDesc{1, Nx * G.dx, Nx * G.dx, Nx * G.dx, out + Nx, E[j], nullptr});
  }
  HIP_CHK(q.gemm(true, false, m1));
  HIP_CHK(q.sums(m2));
  HIP_CHK(q.gemm(true, false, m3));
  HIP_CHK(q.gemm(true, true, m4));
  HIP_CHK(q.field(rho));
  HIP_CHK(q.lines(f1));
  HIP_CHK(q.lines(f0));
  HIP_CHK(q.field(sym));
  HIP_CHK(q.lines(i0));
  HIP_CHK(q.lines(i1));
  HIP_CHK(q.field(real));
  return q.copy2d(cpE);
}

__global__ void k_conserved(int Nx, int dv, const double* M, const double* E, int dx, double* U) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx) return;
  double ep = 0.0;
  for (int m = 0; m < dx; ++m) ep += E[(size_t)m * Nx + e] * E[(size_t)m * Nx + e];
  ep *= 0.5;
  for (int q = 0; q <= dv; ++q) U[(size_t)q * Nx + e] = M[(size_t)q * Nx + e];
  U[(size_t)(dv + 1) * Nx + e] = 0.5 * M[(size_t)(dv + 1) * Nx + e] + ep;
}

hipError_t conserved_from_moments(hipStream_t s, Workspace* ws, const double* M, double n_i,
                                  double* U) {
  const GridDev& G = ws->G;
  double* E = ws->cbuf + (size_t)2 * 40 * G.nx + (size_t)10 * G.nx;
  hipError_t e = poisson_run(s, ws, M, n_i, nullptr, E);
  if (e != hipSuccess) return e;
  k_conserved<<<(G.nx + 255) / 256, 256, 0, s>>>(G.nx, G.dv, M, E, G.dx, U);
  return hipGetLastError();
}

}  // namespace slar
