// Internal declarations of the gfx950 SLAR library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "../../include/slar.h"

#define SLAR_KMAX 72      // largest cross rank / frame width handled
#define SLAR_NMAX 128     // largest cells per dimension
#define SLAR_MAXMOM 9     // moments for dv = 2

#define HIP_TRY(expr)                                       \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return SLAR_E_HIP;                \
  } while (0)

// same, for functions returning hipError_t
#define HIP_CHK(expr)                                       \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return e_;                        \
  } while (0)

namespace slar {

// ------------------------------------------------------------------ grid
struct GridDev {
  int dx, dv, d;
  int n[4];
  double lo[4];
  double h[4];
  int nx;   // prod n_x
  int nv;   // prod n_v
};

inline GridDev make_grid(const slar_grid& g) {
  GridDev G{};
  G.dx = g.dx; G.dv = g.dv; G.d = g.dx + g.dv;
  G.nx = 1; G.nv = 1;
  for (int m = 0; m < G.d; ++m) {
    G.n[m] = g.n[m];
    G.lo[m] = g.lo[m];
    G.h[m] = (g.hi[m] - g.lo[m]) / (double)g.n[m];
    if (m < g.dx) G.nx *= g.n[m]; else G.nv *= g.n[m];
  }
  return G;
}

struct AdvDev {
  int kind;
  int order;
  double tau;
  double cv;
  const double* E;    // frozen field [dx][Nx] = cE0 * E + cE1 * E1
  const double* E1;   // may be null
  double cE0, cE1;
};

__device__ __forceinline__ double efield_node(const AdvDev& a, size_t off) {
  double v = a.cE0 * a.E[off];
  if (a.E1 != nullptr) v = v + a.cE1 * a.E1[off];
  return v;
}

__device__ __forceinline__ int wrap(int j, int n) {
  int r = j % n;
  return r < 0 ? r + n : r;
}

// Lagrange weights on nodes -(w/2)..(w/2) evaluated at xi:
// l_m(xi) = prod_{n != m} (xi - n) / (m - n); the constant denominators are
// folded into one reciprocal per weight.
template <int W>
__device__ __forceinline__ void lagrange(double xi, double* w) {
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int m = a - W / 2;
    double p = 1.0;
    double den = 1.0;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int nn = b - W / 2;
      if (nn != m) { p = p * (xi - (double)nn); den *= (double)(m - nn); }
    }
    w[a] = p * (1.0 / den);
  }
}

__device__ __forceinline__ void quad_weights(double xi, double* w) {
  w[0] = 0.5 * xi * (xi - 1.0);
  w[1] = 1.0 - xi * xi;
  w[2] = 0.5 * xi * (xi + 1.0);
}

// Degree-4 periodic tensor-product interpolation of component c of the
// frozen field at spatial point X[0..dx-1].
__device__ __forceinline__ double efield_at(const GridDev& g, const AdvDev& ad, int c,
                                            const double* X) {
  if (g.dx == 1) {
    const double s = (X[0] - g.lo[0]) / g.h[0];
    const double jf = floor(s);
    const double xi = s - jf - 0.5;
    double w[5];
    lagrange<5>(xi, w);
    const int j = (int)jf;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) acc += w[a] * efield_node(ad, (size_t)c * g.n[0] + wrap(j + a - 2, g.n[0]));
    return acc;
  }
  const double s0 = (X[0] - g.lo[0]) / g.h[0];
  const double s1 = (X[1] - g.lo[1]) / g.h[1];
  const double j0f = floor(s0), j1f = floor(s1);
  double w0[5], w1[5];
  lagrange<5>(s0 - j0f - 0.5, w0);
  lagrange<5>(s1 - j1f - 0.5, w1);
  const int j0 = (int)j0f, j1 = (int)j1f;
  const size_t cb = (size_t)c * g.nx;
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int r0 = wrap(j0 + a - 2, g.n[0]) * g.n[1];
    double row = 0.0;
#pragma unroll
    for (int b = 0; b < 5; ++b) row += w1[b] * efield_node(ad, cb + r0 + wrap(j1 + b - 2, g.n[1]));
    acc += w0[a] * row;
  }
  return acc;
}

// Foot of the characteristic through grid point idx (section 3.1).
__device__ __forceinline__ void foot_of(const GridDev& g, const AdvDev& a, const int* idx,
                                        double* out) {
  double X[2], V[2];
  const int dx = g.dx;
  for (int m = 0; m < dx; ++m) {
    X[m] = g.lo[m] + ((double)idx[m] + 0.5) * g.h[m];
    V[m] = g.lo[dx + m] + ((double)idx[dx + m] + 0.5) * g.h[dx + m];
  }
  if (a.kind == 0) {
    for (int m = 0; m < dx; ++m) { out[m] = X[m] - a.cv * a.tau * V[m]; out[dx + m] = V[m]; }
    return;
  }
  if (a.kind == 1) {
    int lin = idx[0];
    if (dx == 2) lin = idx[0] * g.n[1] + idx[1];
    for (int m = 0; m < dx; ++m) { out[m] = X[m]; out[dx + m] = V[m] + a.tau * efield_node(a, (size_t)m * g.nx + lin); }
    return;
  }
  // RK4 backwards: d/ds (X, V) = (-c V, +E(X)), s in [0, tau]
  const double t = a.tau, c = a.cv;
  double k1x[2], k1v[2], k2x[2], k2v[2], k3x[2], k3v[2], k4x[2], k4v[2], Y[2];
  for (int m = 0; m < dx; ++m) { k1x[m] = -c * V[m]; k1v[m] = efield_at(g, a, m, X); }
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + 0.5 * t * k1x[m];
  for (int m = 0; m < dx; ++m) { k2x[m] = -c * (V[m] + 0.5 * t * k1v[m]); k2v[m] = efield_at(g, a, m, Y); }
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + 0.5 * t * k2x[m];
  for (int m = 0; m < dx; ++m) { k3x[m] = -c * (V[m] + 0.5 * t * k2v[m]); k3v[m] = efield_at(g, a, m, Y); }
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + t * k3x[m];
  for (int m = 0; m < dx; ++m) { k4x[m] = -c * (V[m] + t * k3v[m]); k4v[m] = efield_at(g, a, m, Y); }
  for (int m = 0; m < dx; ++m) {
    out[m] = X[m] + (t / 6.0) * (k1x[m] + 2.0 * k2x[m] + 2.0 * k3x[m] + k4x[m]);
    out[dx + m] = V[m] + (t / 6.0) * (k1v[m] + 2.0 * k2v[m] + 2.0 * k3v[m] + k4v[m]);
  }
}

// Stencil rows (wrapped) and weights of dimension m for a foot coordinate.
template <int W>
__device__ __forceinline__ void stencil_of(const GridDev& g, const AdvDev& a, int m, double xf,
                                           int gidx, int* rows, double* w) {
  const bool moving = (a.kind == 2) || (a.kind == 0 && m < g.dx) || (a.kind == 1 && m >= g.dx);
  int j;
  if (moving) {
    const double s = (xf - g.lo[m]) / g.h[m];
    const double jf = floor(s);
    const double xi = s - jf - 0.5;
    j = (int)jf;
    if (W == 3) quad_weights(xi, w); else lagrange<W>(xi, w);
  } else {
    j = gidx;
#pragma unroll
    for (int b = 0; b < W; ++b) w[b] = (b == W / 2) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int b = 0; b < W; ++b) rows[b] = wrap(j + b - W / 2, g.n[m]);
}

// ------------------------------------------------------------- workspace
struct Workspace {
  slar_grid grid;
  GridDev G;
  int rmax;
  // sampling
  double* Eeff = nullptr;        // [dx][Nx]
  float* X32 = nullptr;          // [Nx][LD32]
  float* P32 = nullptr;          // [Nv][LD32]
  int ld32 = 0;
  // cross approximation
  void* aca_ctl = nullptr;       // AcaCtl
  void* aca_ctl_host = nullptr;  // pinned copy
  double* aca_part = nullptr;    // partial reductions
  unsigned char* used = nullptr; // [Nx]
  double* resid = nullptr;       // [max(Nx,Nv)]
  // dense linear algebra scratch
  double* dwork = nullptr;
  size_t dwork_elems = 0;
  double* small = nullptr;       // small matrices (k x k etc.)
  size_t small_elems = 0;
  int* ismall = nullptr;
  void* host_pinned = nullptr;   // pinned host staging
  // spectral
  double* tw[2] = {nullptr, nullptr};   // twiddles per x-dimension [N][2]
  double* cbuf = nullptr;               // complex scratch
  size_t cbuf_elems = 0;
  // moments
  double* psi = nullptr;         // [Nv][nmom]
  // LoMaC closure
  double* lm = nullptr;          // packed closure arrays
  size_t lm_elems = 0;
  double lm_scal[64];            // host copy of 1D scalars
  double n_i = 1.0;
  bool lm_ready = false;
  // macro / Krylov
  double* kry = nullptr;
  size_t kry_elems = 0;
  // optional in-stream event timing of the cross-approximation sampling
  // kernels: [0] row ms, [1] row launches, [2] row bytes, [3] col ms,
  // [4] col launches, [5] col bytes
  bool timing = false;
  std::vector<hipEvent_t> events;
  double tstat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // optional recording of (J z, z) pairs for training the preconditioner
  float* rec_feat = nullptr;
  float* rec_targ = nullptr;
  int rec_cap = 0;
  int rec_count = 0;
};

// launchers implemented across the .hip files
hipError_t gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                    double beta, double* C, int ldc, long long sC, int batch);
// C = sum over batch of op(A_b) op(B_b) (deterministic); partial buffer in ws
hipError_t gemm_f64_sumbatch(hipStream_t s, Workspace* ws, bool ta, bool tb, int M, int N, int K,
                             const double* A, int lda, long long sA, const double* B, int ldb,
                             long long sB, double* C, int ldc, int batch);
hipError_t combine_field(hipStream_t s, const GridDev& G, const slar_adv* a, double* out);

}  // namespace slar

struct slar_workspace {
  slar::Workspace w;
};
