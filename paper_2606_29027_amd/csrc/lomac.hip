// Adaptive-weight LoMaC projection and the implicit macroscopic solve
// (section 3.2 and Supplement B), FP64 throughout.
//
//  prepare : omega^(mu) = max(|U^(v_mu)[:,0]|, delta); 1D weighted
//            Gram--Schmidt (gamma, q1, eta, beta, q2, norms), one block per
//            velocity dimension; Q_0, Q_{1,mu}, Q_2 on the velocity grid;
//            <psi, Q_k>; moments and projection coefficients of F*.
//  residual: G(U) = U - U_hist + beta (D.F(U) - S(U)) with the LoMaC
//            closure; spectral Poisson / d_t phi / divergence.
//  solve   : Newton with finite-difference Jacobian-vector products and
//            restarted (flexible) GMRES with CGS2; each Newton step is
//            corrected exactly on the per-component mean, where the Jacobian
//            is the identity (the divergence and the source have zero mean).
//  project : F^{n+1} = F* + sum_k dC_k (x) Q_k appended to the frames.
#include <cmath>
#include <vector>

#include "slar_internal.h"
#include "dense.h"
#include "fields.h"
#include "lomac.h"

namespace slar {

static void flux_jacobian(const GridDev& G, const double* scal, const double* psiQ, double* A);

// ---------------------------------------------------------------- layout
LmLayout lm_layout(const GridDev& G) {
  LmLayout L{};
  const int K = G.dv + 2, nm = nmom_of(G.dv);
  size_t o = 0;
  L.gs = o; o += 2 * 3 * SLAR_NLINE;
  L.scal = o; o += 32;
  L.Q = o; o += (size_t)K * G.nv;
  L.psiQ = o; o += (size_t)nm * K;
  L.Mstar = o; o += (size_t)nm * G.nx;
  L.Cstar = o; o += (size_t)K * G.nx;
  L.U0 = o; o += (size_t)K * G.nx;
  L.Aflux = o; o += 2 * 4 * 4;
  L.total = o;
  return L;
}

// 1D weighted Gram--Schmidt, one block per velocity dimension.
// scal layout per mu (8 slots): gamma, eta, beta, n0, n1, n2.
__global__ void k_gram_schmidt(GridDev g, const double* u0, int ld0, const double* u1, int ld1,
                               double delta, double* gs, double* scal) {
  const int mu = blockIdx.x;
  const int dim = g.dx + mu;
  const int n = g.n[dim];
  const double h = g.h[dim];
  const double* u = mu == 0 ? u0 : u1;
  const int ld = mu == 0 ? ld0 : ld1;
  double* om = gs + (size_t)mu * 3 * SLAR_NLINE;
  double* q1 = om + SLAR_NLINE;
  double* q2 = q1 + SLAR_NLINE;
  __shared__ double red[256];
  const int t = threadIdx.x;
  auto bsum = [&](double v) -> double {
    red[t] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] += red[t + o];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };
  // cells c = t, t + blockDim.x, ... (n <= SLAR_NLINE); a thread's partial
  // sums run over its cells in order, then over the block
  const int nb = blockDim.x;
  auto wof = [&](int c) { return fmax(fabs(u[(size_t)c * ld]), delta); };
  auto vof = [&](int c) { return g.lo[dim] + ((double)c + 0.5) * h; };
  double p0 = 0.0, pg = 0.0, pe = 0.0;
  for (int c = t; c < n; c += nb) {
    const double w = wof(c), vv = vof(c);
    const double vo = vv * w, v2o = vv * vv * w;
    om[c] = w;
    p0 += w * w * h / w;
    pg += vo * w * h / w;
    pe += v2o * w * h / w;
  }
  const double n0 = bsum(p0);
  const double gamma = bsum(pg) / n0;
  const double eta = bsum(pe) / n0;
  double p1 = 0.0, pb = 0.0;
  for (int c = t; c < n; c += nb) {
    const double w = wof(c), vv = vof(c);
    const double vo = vv * w, v2o = vv * vv * w;
    const double q1v = vo - gamma * w;
    p1 += q1v * q1v * h / w;
    pb += v2o * q1v * h / w;
  }
  const double n1 = bsum(p1);
  const double beta = bsum(pb) / n1;
  double p2 = 0.0;
  for (int c = t; c < n; c += nb) {
    const double w = wof(c), vv = vof(c);
    const double vo = vv * w, v2o = vv * vv * w;
    const double q1v = vo - gamma * w;
    const double q2v = v2o - eta * w - beta * q1v;
    q1[c] = q1v;
    q2[c] = q2v;
    p2 += q2v * q2v * h / w;
  }
  const double n2 = bsum(p2);
  if (t == 0) {
    double* sc = scal + mu * 8;
    sc[0] = gamma; sc[1] = eta; sc[2] = beta; sc[3] = n0; sc[4] = n1; sc[5] = n2;
  }
}

// Q tensors (stored [Nv][K]) and squared norms NQ (scal[16 + k]).
__global__ void k_qbasis(GridDev g, const double* gs, double* scal, double* Q) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int dv = g.dv, K = dv + 2;
  if (J == 0) {
    const double* s0 = scal;
    const double* s1 = scal + 8;
    double* NQ = scal + 16;
    if (dv == 1) {
      NQ[0] = s0[3]; NQ[1] = s0[4]; NQ[2] = s0[5];
    } else {
      NQ[0] = s0[3] * s1[3];
      NQ[1] = s0[4] * s1[3];
      NQ[2] = s0[3] * s1[4];
      NQ[3] = s0[5] * s1[3] + s1[5] * s0[3];
    }
  }
  if (J >= g.nv) return;
  double* q = Q + (size_t)J * K;     // Q stored [Nv][K]
  if (dv == 1) {
    const double* om = gs;
    q[0] = om[J];
    q[1] = om[SLAR_NLINE + J];
    q[2] = om[2 * SLAR_NLINE + J];
    return;
  }
  const int a = J / g.n[3], b = J % g.n[3];
  const double* A = gs;                    // mu = 0: omega, q1, q2
  const double* B = gs + 3 * SLAR_NLINE;    // mu = 1
  const double w0 = A[a], w1 = B[b];
  q[0] = w0 * w1;
  q[1] = A[SLAR_NLINE + a] * w1;
  q[2] = w0 * B[SLAR_NLINE + b];
  q[3] = A[2 * SLAR_NLINE + a] * w1 + w0 * B[2 * SLAR_NLINE + b];
  (void)K;
}

// Projection coefficients eqs. (C0_def)-(C2_def) from raw moments
// Mraw = (M0, M1_mu, M2) -> C [K][Nx].
__device__ __forceinline__ void coeffs_at(int dv, const double* scal, const double* Mr, double* C) {
  const double* NQ = scal + 16;
  const double M0 = Mr[0];
  C[0] = M0 / NQ[0];
  double etas = 0.0, num = Mr[dv + 1];
  for (int m = 0; m < dv; ++m) {
    const double* sc = scal + 8 * m;
    const double d1 = Mr[1 + m] - sc[0] * M0;
    C[1 + m] = d1 / NQ[1 + m];
    etas += sc[1];
  }
  num = num - etas * M0;
  for (int m = 0; m < dv; ++m) {
    const double* sc = scal + 8 * m;
    num = num - sc[2] * (Mr[1 + m] - sc[0] * M0);
  }
  C[dv + 1] = num / NQ[dv + 1];
}

__global__ void k_cstar(int Nx, int dv, const double* scal, const double* M, double* C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx) return;
  double Mr[4], c[4];
  for (int q = 0; q < dv + 2; ++q) Mr[q] = M[(size_t)q * Nx + e];
  coeffs_at(dv, scal, Mr, c);
  for (int q = 0; q < dv + 2; ++q) C[(size_t)q * Nx + e] = c[q];
}

slar_status lomac_prepare_run(hipStream_t s, Workspace* ws, const slar_ht& Fs,
                              const slar_frames& Ff, double delta, double n_i) {
  const GridDev& G = ws->G;
  const LmLayout L = lm_layout(G);
  double* lm = ws->lm;
  const int dv = G.dv, K = dv + 2, nm = nmom_of(dv);
  const double* u0 = (const double*)Fs.leaf[G.dx];
  const int ld0 = Fs.rank[G.dx];
  const double* u1 = dv == 2 ? (const double*)Fs.leaf[G.dx + 1] : u0;
  const int ld1 = dv == 2 ? Fs.rank[G.dx + 1] : ld0;
  k_gram_schmidt<<<dv, 256, 0, s>>>(G, u0, ld0, u1, ld1, delta, lm + L.gs, lm + L.scal);
  k_qbasis<<<(G.nv + 255) / 256, 256, 0, s>>>(G, lm + L.gs, lm + L.scal, lm + L.Q);
  HIP_TRY(hipGetLastError());
  // <psi_q, Q_k> -> psiQ [nm][K]: sum_J Psi[J][q] Q[J][k]
  if (gemm_tn_long(s, ws, nm, K, G.nv, ws->psi, nm, lm + L.Q, K, lm + L.psiQ, K) != hipSuccess)
    return SLAR_E_HIP;
  if (moments_run(s, ws, Ff, lm + L.Mstar) != hipSuccess) return SLAR_E_HIP;
  k_cstar<<<(G.nx + 255) / 256, 256, 0, s>>>(G.nx, dv, lm + L.scal, lm + L.Mstar, lm + L.Cstar);
  if (conserved_from_moments(s, ws, lm + L.Mstar, n_i, lm + L.U0) != hipSuccess) return SLAR_E_HIP;
  HIP_TRY(hipMemcpyAsync(ws->lm_scal, lm + L.scal, 32 * sizeof(double), hipMemcpyDeviceToHost, s));
  std::vector<double> psiQ_h((size_t)nm * K), Af(2 * 4 * 4, 0.0);
  HIP_TRY(hipMemcpyAsync(psiQ_h.data(), lm + L.psiQ, sizeof(double) * nm * K, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < 20; ++i)
    if (!std::isfinite(ws->lm_scal[i])) return SLAR_E_NUMERIC;
  flux_jacobian(G, ws->lm_scal, psiQ_h.data(), Af.data());
  HIP_TRY(hipMemcpyAsync(lm + L.Aflux, Af.data(), sizeof(double) * Af.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  ws->n_i = n_i;
  ws->lm_ready = true;
  return SLAR_OK;
}

// ------------------------------------------------------------ residual
struct MacroBufs {
  double *rho, *phiE, *J, *gdt, *Mall, *flux, *divF;
  double2* c0;
};

static MacroBufs macro_bufs(Workspace* ws) {
  const GridDev& G = ws->G;
  const size_t Nx = G.nx;
  MacroBufs b;
  double* p = ws->kry;   // first region of kry
  b.rho = p; p += Nx;
  b.phiE = p; p += 3 * Nx;
  b.J = p; p += 2 * Nx;
  b.gdt = p; p += 2 * Nx;
  b.Mall = p; p += 9 * Nx;
  b.flux = p; p += 8 * Nx;
  b.divF = p; p += 4 * Nx;
  double2* c = (double2*)ws->cbuf;
  b.c0 = c;   // spectral-stage scratch, 20 Nx complex
  return b;
}

size_t macro_fixed_elems(int Nx) { return (size_t)29 * Nx; }

__global__ void k_rho_of(int Nx, const double* U, double ni, double* rho) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < Nx) rho[e] = ni - U[e];
}

// e_p, raw moments from U, dC, all corrected moments, J = -M1
__global__ void k_closure(int Nx, int dx, int dv, int nm, const double* __restrict__ U,
                          const double* __restrict__ phiE, const double* __restrict__ scal,
                          const double* __restrict__ Cstar, const double* __restrict__ Mstar,
                          const double* __restrict__ psiQ, double* __restrict__ Mall,
                          double* __restrict__ J) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx) return;
  const int K = dv + 2;
  double ep = 0.0;
  for (int m = 0; m < dx; ++m) {
    const double Em = phiE[(size_t)(1 + m) * Nx + e];
    ep += Em * Em;
  }
  ep *= 0.5;
  double Mr[4], C[4];
  for (int q = 0; q <= dv; ++q) Mr[q] = U[(size_t)q * Nx + e];
  Mr[dv + 1] = 2.0 * (U[(size_t)(dv + 1) * Nx + e] - ep);
  coeffs_at(dv, scal, Mr, C);
  double dC[4];
  for (int k = 0; k < K; ++k) dC[k] = C[k] - Cstar[(size_t)k * Nx + e];
  for (int q = 0; q < nm; ++q) {
    double v = Mstar[(size_t)q * Nx + e];
    for (int k = 0; k < K; ++k) v += psiQ[q * K + k] * dC[k];
    Mall[(size_t)q * Nx + e] = v;
  }
  for (int m = 0; m < dx; ++m) J[(size_t)m * Nx + e] = -Mall[(size_t)(1 + m) * Nx + e];
}

// d_t phi gradient symbol: g_m = i k_m * ( -(sum_n i k_n J^_n) / |k|^2 )
// fluxes [K][dx][Nx]
__global__ void k_fluxes(int Nx, int dx, int dv, const double* __restrict__ Mall,
                         const double* __restrict__ phiE, const double* __restrict__ J,
                         const double* __restrict__ gdt, double* __restrict__ flux) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx) return;
  const double phi = phiE[e];
  int pair[2][2];
  int c = dv + 2;
  for (int a = 0; a < dv; ++a)
    for (int b = a; b < dv; ++b) { pair[a][b] = c; pair[b][a] = c; ++c; }
  const int off_e = c;
  for (int m = 0; m < dx; ++m) flux[(size_t)(0 * dx + m) * Nx + e] = Mall[(size_t)(1 + m) * Nx + e];
  for (int a = 0; a < dv; ++a)
    for (int m = 0; m < dx; ++m)
      flux[(size_t)((1 + a) * dx + m) * Nx + e] = Mall[(size_t)pair[a][m] * Nx + e];
  for (int m = 0; m < dx; ++m) {
    const double fep = -phi * gdt[(size_t)m * Nx + e] + J[(size_t)m * Nx + e] * phi;
    flux[(size_t)((dv + 1) * dx + m) * Nx + e] = 0.5 * Mall[(size_t)(off_e + m) * Nx + e] + fep;
  }
}

__global__ void k_gres(int Nx, int dx, int dv, const double* __restrict__ U,
                       const double* __restrict__ Uh, double bdt, const double* __restrict__ divF,
                       const double* __restrict__ phiE, double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx) return;
  const int K = dv + 2;
  for (int q = 0; q < K; ++q) {
    double S = 0.0;
    if (q >= 1 && q <= dv) S = -U[e] * phiE[(size_t)(1 + (q - 1)) * Nx + e];
    const size_t i = (size_t)q * Nx + e;
    G[i] = U[i] - Uh[i] + bdt * (divF[i] - S);
  }
}

hipError_t macro_residual(hipStream_t s, Workspace* ws, const double* U, const double* Uhist,
                          double bdt, double* Gout) {
  const GridDev& G = ws->G;
  const LmLayout L = lm_layout(G);
  const double* lm = ws->lm;
  MacroBufs b = macro_bufs(ws);
  const int Nx = G.nx, dx = G.dx, dv = G.dv, K = dv + 2, nm = nmom_of(dv);
  const unsigned nb = (Nx + 255) / 256;
  k_rho_of<<<nb, 256, 0, s>>>(Nx, U, ws->n_i, b.rho);
  hipError_t e = spectral_stage(s, ws, SPEC_POISSON, b.rho, b.phiE, nullptr, b.c0);
  if (e != hipSuccess) return e;
  k_closure<<<nb, 256, 0, s>>>(Nx, dx, dv, nm, U, b.phiE, lm + L.scal, lm + L.Cstar, lm + L.Mstar,
                               lm + L.psiQ, b.Mall, b.J);
  if ((e = spectral_stage(s, ws, SPEC_DTPHI, b.J, b.gdt, nullptr, b.c0)) != hipSuccess) return e;
  k_fluxes<<<nb, 256, 0, s>>>(Nx, dx, dv, b.Mall, b.phiE, b.J, b.gdt, b.flux);
  if ((e = spectral_stage(s, ws, SPEC_DIV, b.flux, b.divF, nullptr, b.c0)) != hipSuccess) return e;
  k_gres<<<nb, 256, 0, s>>>(Nx, dx, dv, U, Uhist, bdt, b.divF, b.phiE, Gout);
  return hipGetLastError();
}

// ------------------------------------------------------ vector kernels
constexpr int MD_CHUNK = 512;   // elements per block in the Krylov passes

// Sum of per-block partials, the same fixed order in every block that asks:
// out[v] = sum_b part[v][b] for v < nv, one wave per value, lanes over b,
// then a butterfly.  Every block gets bitwise the same sums.
__device__ __forceinline__ void reduce_parts_block(int nb, int nv, const double* __restrict__ part,
                                                   double* __restrict__ out) {
  const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int v = wv; v < nv; v += nw) {
    double acc = 0.0;
    for (int b = ln; b < nb; b += 64) acc += part[(size_t)v * nb + b];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (ln == 0) out[v] = acc;
  }
}

// One classical Gram--Schmidt pass of the Arnoldi step over V[0..nv):
//   nsub > 0: h = sum of the previous pass's partials hpart (nbk per value,
//             reduced redundantly by every block), block 0 stores h in hout;
//             w -= sum_{v < nsub} V[v] h[v]
//   then part[v][block] = V[v] . w for v < ndot, and part[ndot][block] =
//   w . w when wnorm.
__global__ __launch_bounds__(256) void k_cgs_pass(int n, int nsub, int ndot, int wnorm,
                                                  const double* __restrict__ V, long long ldv,
                                                  const double* __restrict__ hpart,
                                                  double* __restrict__ hout, double* __restrict__ w,
                                                  double* __restrict__ part) {
  __shared__ double red[4][SLAR_KMAX + 2];
  __shared__ double hs[SLAR_KMAX + 2];
  const int t = threadIdx.x;
  const int e0 = blockIdx.x * MD_CHUNK;
  if (nsub > 0) {
    reduce_parts_block(gridDim.x, nsub, hpart, hs);
    __syncthreads();
    if (blockIdx.x == 0 && hout)
      for (int v = t; v < nsub; v += 256) hout[v] = hs[v];
  }
  double wl[MD_CHUNK / 256];
  for (int q = 0; q < MD_CHUNK / 256; ++q) {
    const int e = e0 + t + q * 256;
    double x = 0.0;
    if (e < n) {
      x = w[e];
      if (nsub > 0) {
        for (int v = 0; v < nsub; ++v) x -= V[v * ldv + e] * hs[v];
        w[e] = x;
      }
    }
    wl[q] = x;
  }
  const int nd = ndot + (wnorm ? 1 : 0);
  for (int v = 0; v < nd; ++v) {
    double acc = 0.0;
    for (int q = 0; q < MD_CHUNK / 256; ++q) {
      const int e = e0 + t + q * 256;
      if (e < n) acc += (v < ndot ? V[v * ldv + e] : wl[q]) * wl[q];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((t & 63) == 0) red[t >> 6][v] = acc;
  }
  __syncthreads();
  for (int v = t; v < nd; v += 256)
    part[(size_t)v * gridDim.x + blockIdx.x] = red[0][v] + red[1][v] + red[2][v] + red[3][v];
}

// Last step of the Arnoldi orthogonalisation: ||w||^2 = sum of the partials
// (same fixed order as above), out = w / ||w|| (0 if w == 0); block 0
// stores ||w||^2 in nout.  Launched with the grid of the partials.
__global__ __launch_bounds__(256) void k_cgs_normalize(int n, const double* __restrict__ npart,
                                                       double* __restrict__ nout,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ out) {
  __shared__ double nn[1];
  reduce_parts_block(gridDim.x, 1, npart, nn);
  __syncthreads();
  const double s2 = nn[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) nout[0] = s2;
  const double nz = sqrt(s2);
  const int e0 = blockIdx.x * MD_CHUNK;
  for (int q = 0; q < MD_CHUNK / 256; ++q) {
    const int e = e0 + threadIdx.x + q * 256;
    if (e < n) out[e] = nz > 0.0 ? w[e] / nz : 0.0;
  }
}

// out[v] = sum_b part[v][b]: one wave per v, lanes over b (coalesced),
// fixed order (lane partial sums, then a butterfly)
__global__ __launch_bounds__(64) void k_reduce_parts(int nb, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  const int v = blockIdx.x, ln = threadIdx.x;
  double acc = 0.0;
  for (int b = ln; b < nb; b += 64) acc += part[(size_t)v * nb + b];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (ln == 0) out[v] = acc;
}

// y = a x + b y ; if x2: y += c x2
__global__ void k_axpby(int n, double a, const double* __restrict__ x, double b, double* __restrict__ y,
                        double c, const double* __restrict__ x2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
  if (x2) v += c * x2[e];
  y[e] = v;
}

// finite-difference point: h = cst / sqrt(nrm2) (cst if nrm2 == 0),
// Uh = U + h z; h is stored for k_fd_diff
__global__ void k_fd_point(int n, const double* __restrict__ U, const double* __restrict__ z,
                           const double* __restrict__ nrm2, double cst, double* __restrict__ Uh,
                           double* __restrict__ hout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const double nz = nrm2 ? sqrt(nrm2[0]) : 1.0;
  const double h = nz > 0.0 ? cst / nz : cst;
  if (e == 0) hout[0] = h;
  if (e < n) Uh[e] = U[e] + h * z[e];
}

// w = (Gh - g0) / h  (scale < 0 : w = -(Gh - g0)/h - g0, the true residual)
__global__ void k_fd_diff(int n, const double* __restrict__ Gh, const double* __restrict__ g0,
                          const double* __restrict__ hdev, int residual_form, double* __restrict__ w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double h = hdev[0];
  const double jv = (Gh[e] - g0[e]) / h;
  w[e] = residual_form ? -g0[e] - jv : jv;
}


// x += sum_v A[v] y[v]
__global__ void k_add_combo(int n, int nv, const double* __restrict__ A, long long lda,
                            const double* __restrict__ y, double* __restrict__ x) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc = x[e];
  for (int v = 0; v < nv; ++v) acc += A[v * lda + e] * y[v];
  x[e] = acc;
}

// per-component means of d and g: out[c] = mean(d_c), out[8 + c] = mean(g_c)
__global__ void k_comp_means(int Nx, const double* __restrict__ d, const double* __restrict__ g,
                             double* __restrict__ out) {
  __shared__ double r1[256], r2[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int e = t; e < Nx; e += 256) { a += d[(size_t)c * Nx + e]; b += g[(size_t)c * Nx + e]; }
  r1[t] = a; r2[t] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) { r1[t] += r1[t + o]; r2[t] += r2[t + o]; }
    __syncthreads();
  }
  if (t == 0) { out[c] = r1[0] / Nx; out[8 + c] = r2[0] / Nx; }
}

// per-component mean fix: d_c -= mean(d_c) + mean(g_c)  (means given)
__global__ void k_meanfix(int Nx, int K, const double* __restrict__ md, const double* __restrict__ mg,
                          double* __restrict__ d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx * K) return;
  const int c = e / Nx;
  d[e] -= md[c] + mg[c];
}

// --------------------------------------------- spectral preconditioner
// The kinetic part of the LoMaC flux is linear in U with x-independent
// coefficients (the closure basis Q_k depends on v only, the coefficient
// map of eqs. (C0_def)-(C2_def) is linear in the raw moments, and
// M2 = 2 (U2 - e_p)); with the linearised Poisson source -n_i E(dU_0) this
// gives, per Fourier mode k, the K x K system
//   (I + b dt [ sum_mu i k_mu A_mu + n_i (i k_mu / |k|^2) e_{1+mu} e_0^T ]) z^ = r^.
// The K x K matrix of each mode is inverted once per macroscopic solve
// (complex Gauss-Jordan, partial pivoting) and applied as a matrix-vector
// product; the field-energy flux and the E-dependent parts are left to the
// Krylov iteration.  A_mu [dx][K][K] is precomputed on the host.
// Minv[(a K + b) Nx + pt] holds entry (a, b) of the inverse of mode
// p = i0 n1 + i1 at the transposed position pt = i1 n0 + i0, so that the
// modes of one axis-0 line (the spectral line kernel's lanes) are adjacent.
__global__ void k_spec_setup(int n0, int n1, int dx, double L0, double L1, int K,
                             const double* __restrict__ A, double bdt, double ni,
                             double2* __restrict__ Minv, int Nx) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Nx) return;
  auto wn = [](int i, int n, double Lx) {
    if ((n % 2) == 0 && i == n / 2) return 0.0;
    const int m = (i < (n + 1) / 2) ? i : i - n;
    return 2.0 * M_PI * (double)m / Lx;
  };
  double k[2] = {wn(p / n1, n0, L0), dx == 2 ? wn(p % n1, n1, L1) : 0.0};
  const double k2 = k[0] * k[0] + k[1] * k[1];
  // [M | I] with M = I + i bdt (sum_mu k_mu A_mu + n_i k_mu / |k|^2 e_{1+mu} e_0^T)
  double Mr[4][8], Mi[4][8];
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      double im = 0.0;
      for (int mu = 0; mu < dx; ++mu) im += k[mu] * A[(mu * K + a) * K + b];
      Mr[a][b] = (a == b) ? 1.0 : 0.0;
      Mi[a][b] = bdt * im;
      Mr[a][K + b] = (a == b) ? 1.0 : 0.0;
      Mi[a][K + b] = 0.0;
    }
  if (k2 > 0.0)
    for (int mu = 0; mu < dx; ++mu) Mi[1 + mu][0] += bdt * ni * k[mu] / k2;
  for (int c = 0; c < K; ++c) {
    int piv = c;
    double best = Mr[c][c] * Mr[c][c] + Mi[c][c] * Mi[c][c];
    for (int r = c + 1; r < K; ++r) {
      const double v = Mr[r][c] * Mr[r][c] + Mi[r][c] * Mi[r][c];
      if (v > best) { best = v; piv = r; }
    }
    if (piv != c)
      for (int b = 0; b < 2 * K; ++b) {
        double t = Mr[c][b]; Mr[c][b] = Mr[piv][b]; Mr[piv][b] = t;
        t = Mi[c][b]; Mi[c][b] = Mi[piv][b]; Mi[piv][b] = t;
      }
    // scale row c by 1 / M[c][c]
    const double dr = Mr[c][c], di = Mi[c][c], dd = dr * dr + di * di;
    const double ir = dr / dd, ii = -di / dd;
    for (int b = 0; b < 2 * K; ++b) {
      const double xr = Mr[c][b], xi = Mi[c][b];
      Mr[c][b] = xr * ir - xi * ii;
      Mi[c][b] = xr * ii + xi * ir;
    }
    for (int r = 0; r < K; ++r) {
      if (r == c) continue;
      const double fr = Mr[r][c], fi = Mi[r][c];
      for (int b = 0; b < 2 * K; ++b) {
        Mr[r][b] -= fr * Mr[c][b] - fi * Mi[c][b];
        Mi[r][b] -= fr * Mi[c][b] + fi * Mr[c][b];
      }
    }
  }
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b)
      Minv[(size_t)(a * K + b) * Nx + (size_t)(p % n1) * n0 + p / n1] = make_double2(Mr[a][K + b], Mi[a][K + b]);
}

static hipError_t spectral_setup(hipStream_t s, Workspace* ws, double bdt, double2* Minv) {
  const GridDev& G = ws->G;
  const int K = G.dv + 2, Nx = G.nx;
  k_spec_setup<<<(Nx + 255) / 256, 256, 0, s>>>(G.n[0], G.dx == 2 ? G.n[1] : 1, G.dx,
                                                ws->grid.hi[0] - ws->grid.lo[0],
                                                G.dx == 2 ? ws->grid.hi[1] - ws->grid.lo[1] : 1.0,
                                                K, ws->lm + lm_layout(G).Aflux, bdt, ws->n_i, Minv, Nx);
  return hipGetLastError();
}

static hipError_t spectral_precond(hipStream_t s, Workspace* ws, const double* v, const double2* Minv,
                                   double* z) {
  // scratch above the residual's (20 Nx complex each)
  return spectral_stage(s, ws, SPEC_PRECOND, v, z, Minv, (double2*)ws->cbuf + (size_t)24 * ws->G.nx);
}

struct KryBufs {
  double *V, *Z, *w, *g0, *Uh, *Gh, *d, *r, *x, *U;
  double *partA, *partB;   // per-block partial dot products, [m + 2][nbk] each
  double2* Minv;   // spectral preconditioner inverses [K][K][Nx]
};

static KryBufs kry_bufs(Workspace* ws, int n, int m) {
  KryBufs b;
  double* p = ws->kry + macro_fixed_elems(ws->G.nx);
  b.V = p; p += (size_t)(m + 1) * n;
  b.Z = p; p += (size_t)m * n;
  b.w = p; p += n;
  b.g0 = p; p += n;
  b.Uh = p; p += n;
  b.Gh = p; p += n;
  b.d = p; p += n;
  b.r = p; p += n;
  b.x = p; p += n;
  b.U = p; p += n;
  b.Minv = (double2*)p; p += (size_t)2 * 4 * n;   // K^2 Nx complex, K <= 4
  const size_t np = (size_t)(m + 2) * ((n + MD_CHUNK - 1) / MD_CHUNK);
  b.partA = p; p += np;
  b.partB = p; p += np;
  return b;
}

size_t kry_elems_for(int Nx, int K, int m) {
  const size_t n = (size_t)Nx * K;
  return macro_fixed_elems(Nx) + (size_t)(2 * m + 1) * n + 8 * n + (size_t)8 * n +
         (size_t)2 * (m + 2) * ((n + MD_CHUNK - 1) / MD_CHUNK) + 4096;
}

// host-side flux Jacobian of the closure (see k_spec_setup)
static void flux_jacobian(const GridDev& G, const double* scal, const double* psiQ, double* A) {
  const int dv = G.dv, K = dv + 2, dx = G.dx;
  const double* NQ = scal + 16;
  double Cc[4][4] = {};
  Cc[0][0] = 1.0 / NQ[0];
  double etas = 0.0, bg = 0.0;
  for (int a = 0; a < dv; ++a) {
    const double* sc = scal + 8 * a;
    Cc[1 + a][0] = -sc[0] / NQ[1 + a];
    Cc[1 + a][1 + a] = 1.0 / NQ[1 + a];
    etas += sc[1];
    bg += sc[2] * sc[0];
  }
  Cc[dv + 1][0] = (-etas + bg) / NQ[dv + 1];
  for (int a = 0; a < dv; ++a) Cc[dv + 1][1 + a] = -scal[8 * a + 2] / NQ[dv + 1];
  Cc[dv + 1][dv + 1] = 1.0 / NQ[dv + 1];
  // dMraw/dU = diag(1, .., 1, 2)
  for (int k = 0; k < K; ++k) Cc[k][dv + 1] *= 2.0;
  int pair[2][2];
  int c = dv + 2;
  for (int a = 0; a < dv; ++a)
    for (int b = a; b < dv; ++b) { pair[a][b] = pair[b][a] = c; ++c; }
  const int off_e = c;
  for (int mu = 0; mu < dx; ++mu)
    for (int comp = 0; comp < K; ++comp) {
      int q; double wgt = 1.0;
      if (comp == 0) q = 1 + mu;
      else if (comp <= dv) q = pair[comp - 1][mu];
      else { q = off_e + mu; wgt = 0.5; }
      for (int j = 0; j < K; ++j) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += psiQ[q * K + k] * Cc[k][j];
        A[(mu * K + comp) * K + j] = wgt * acc;
      }
    }
}

// Uhist = sum_j c_j U_j - sum_j d_j R_j, accumulated in that order
__global__ void k_hist_combine(int n, MacroHist h, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = h.c[0] * h.U[0][e];
  for (int j = 1; j < h.nh; ++j) v += h.c[j] * h.U[j][e];
  for (int j = 0; j < h.nr; ++j) v -= h.d[j] * h.R[j][e];
  out[e] = v;
}

hipError_t macro_rhs(hipStream_t s, Workspace* ws, const double* U, double* Rout) {
  // G = U - U + 1 (D.F - S): the history cancels exactly
  return macro_residual(s, ws, U, U, 1.0, Rout);
}

// One JFNK solve with the given preconditioner, from U(F*).  kry_limit
// bounds the Krylov iterations of each Newton step: a linear solve that
// does not reach krylov_tol within it ends the whole solve with
// SLAR_E_NOCONV.
static slar_status macro_solve_once(hipStream_t s, Workspace* ws, const MacroHist& hist, double beta,
                                    double newton_tol, double krylov_tol, int precond,
                                    const slar_cnn* cnn, double* Uout, int* iters, int kry_limit) {
  if (!ws->lm_ready) return SLAR_E_INVAL;
  const GridDev& G = ws->G;
  const int K = G.dv + 2, Nx = G.nx, n = K * Nx;
  const int m = KRY_RESTART;
  const LmLayout L = lm_layout(G);
  KryBufs b = kry_bufs(ws, n, m);
  double* hdev = ws->small;            // [0..72] dots, [80..] second pass, [160] h, [170..] means
  double* h1 = hdev, * h2 = hdev + 80, * hval = hdev + 160, * means = hdev + 170;
  double* nrm = hdev + 200;            // norms
  double* hh = (double*)ws->host_pinned;
  const unsigned nb = (n + 255) / 256;
  const int nbk = (n + MD_CHUNK - 1) / MD_CHUNK;
  auto norm2 = [&](const double* x, double* out) {
    k_cgs_pass<<<nbk, 256, 0, s>>>(n, 0, 0, 1, nullptr, n, nullptr, nullptr, (double*)x, b.partA);
    k_reduce_parts<<<1, 64, 0, s>>>(nbk, b.partA, out);
  };
  double* Uhist = b.x;
  const double bdt = beta;
  k_hist_combine<<<nb, 256, 0, s>>>(n, hist, Uhist);
  if (precond != 0) HIP_TRY(spectral_setup(s, ws, bdt, b.Minv));
  double* U = b.U;
  HIP_TRY(hipMemcpyAsync(U, ws->lm + L.U0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const double sqeps = std::sqrt(2.220446049250313e-16);
  int newton = 0, krylov = 0;
  bool converged = false;
  ws->newton_hist_n = 0;
  const bool flexible = precond != 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
  auto apply_pc = [&](const double* v, double* z) -> hipError_t {
    if (precond == 1) return spectral_precond(s, ws, v, b.Minv, z);
    if (precond == 2) {
      HIP_CHK(spectral_precond(s, ws, v, b.Minv, z));
      return cnn_apply(s, ws, cnn, v, U, z);
    }
    return hipErrorInvalidValue;
  };
  for (int it = 0; it <= KRY_MAX_NEWTON; ++it) {
    if (macro_residual(s, ws, U, Uhist, bdt, b.g0) != hipSuccess) return SLAR_E_HIP;
    norm2(b.g0, nrm);
    norm2(U, nrm + 1);
    HIP_TRY(hipMemcpyAsync(hh, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double gn = std::sqrt(hh[0]);
    if (!std::isfinite(gn)) return SLAR_E_NUMERIC;
    const double rms = gn / std::sqrt((double)n);
    double* rec = ws->newton_hist + 4 * std::min(it, 31);
    rec[0] = rms; rec[1] = 0.0; rec[2] = 0.0; rec[3] = 0.0;
    ws->newton_hist_n = std::min(it + 1, 32);
    if (rms <= newton_tol) { converged = true; break; }
    if (it == KRY_MAX_NEWTON) break;
    const double fdc = sqeps * (1.0 + std::sqrt(hh[1]));
    HIP_TRY(hipMemsetAsync(b.d, 0, sizeof(double) * n, s));
    const double bn = gn;
    double beta = gn;
    k_axpby<<<nb, 256, 0, s>>>(n, -1.0, b.g0, 0.0, b.r, 0.0, nullptr);
    int kits = 0;
    bool done = false;
    while (!done && kits < kry_limit) {
      k_axpby<<<nb, 256, 0, s>>>(n, 1.0 / beta, b.r, 0.0, b.V, 0.0, nullptr);
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(gv.begin(), gv.end(), 0.0);
      gv[0] = beta;
      int jl = 0;
      int pre = -1;   // basis vector whose preconditioned copy is already enqueued
      for (int j = 0; j < m; ++j) {
        double* vj = b.V + (size_t)j * n;
        double* zj = flexible ? b.Z + (size_t)j * n : vj;
        if (flexible && pre != j) {
          if (apply_pc(vj, zj) != hipSuccess) return SLAR_E_HIP;
          norm2(zj, nrm + 2);
        }
        // w = J z by a finite difference with h = sqrt(eps)(1 + ||U||)/||z||
        k_fd_point<<<nb, 256, 0, s>>>(n, U, zj, flexible ? nrm + 2 : nullptr, fdc, b.Uh, hval);
        if (macro_residual(s, ws, b.Uh, Uhist, bdt, b.Gh) != hipSuccess) return SLAR_E_HIP;
        k_fd_diff<<<nb, 256, 0, s>>>(n, b.Gh, b.g0, hval, 0, b.w);
        if (flexible && ws->rec_feat && ws->rec_count < ws->rec_cap) {
          if (spectral_precond(s, ws, b.w, b.Minv, b.Uh) != hipSuccess) return SLAR_E_HIP;
          if (record_pair(s, ws, b.w, zj, U, b.Uh) != hipSuccess) return SLAR_E_HIP;
        }
        // CGS2 against V[0..j]: h1 = V^T w; w -= V h1; h2 = V^T w; w -= V h2;
        // V[j+1] = w / ||w||.  The Hessenberg column is h1 + h2.
        k_cgs_pass<<<nbk, 256, 0, s>>>(n, 0, j + 1, 0, b.V, n, nullptr, nullptr, b.w, b.partA);
        k_cgs_pass<<<nbk, 256, 0, s>>>(n, j + 1, j + 1, 0, b.V, n, b.partA, h1, b.w, b.partB);
        k_cgs_pass<<<nbk, 256, 0, s>>>(n, j + 1, 0, 1, b.V, n, b.partB, h2, b.w, b.partA);
        k_cgs_normalize<<<nbk, 256, 0, s>>>(n, b.partA, nrm + 3, b.w, b.V + (size_t)(j + 1) * n);
        HIP_TRY(hipMemcpyAsync(hh, hdev, sizeof(double) * 208, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(ws->poll_ev[0], s));
        // the next basis vector is on the device: its preconditioner runs
        // while the host waits for this column (the same launches in the
        // same order as without; wasted once, when the solve stops here)
        if (flexible && j + 1 < m) {
          double* zn = b.Z + (size_t)(j + 1) * n;
          if (apply_pc(b.V + (size_t)(j + 1) * n, zn) != hipSuccess) return SLAR_E_HIP;
          norm2(zn, nrm + 2);
          pre = j + 1;
        }
        HIP_TRY(hipEventSynchronize(ws->poll_ev[0]));
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[80 + i];
        const double hn = std::sqrt(std::max(hh[203], 0.0));
        H[(size_t)(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double t1 = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
          H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = t1;
        }
        const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
        cs[j] = den > 0 ? H[(size_t)j * m + j] / den : 1.0;
        sn[j] = den > 0 ? H[(size_t)(j + 1) * m + j] / den : 0.0;
        H[(size_t)j * m + j] = den;
        H[(size_t)(j + 1) * m + j] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        ++kits;
        jl = j;
        if (std::fabs(gv[j + 1]) <= krylov_tol * bn || kits >= kry_limit || den == 0.0) break;
      }
      const int kk = jl + 1;
      for (int i = kk - 1; i >= 0; --i) {
        double acc = gv[i];
        for (int q = i + 1; q < kk; ++q) acc -= H[(size_t)i * m + q] * y[q];
        y[i] = H[(size_t)i * m + i] != 0 ? acc / H[(size_t)i * m + i] : 0.0;
      }
      double* ydev = hdev + 256;
      for (int i = 0; i < kk; ++i) hh[256 + i] = y[i];
      HIP_TRY(hipMemcpyAsync(ydev, hh + 256, sizeof(double) * kk, hipMemcpyHostToDevice, s));
      k_add_combo<<<nb, 256, 0, s>>>(n, kk, flexible ? b.Z : b.V, n, ydev, b.d);
      // true residual r = -g0 - J d
      norm2(b.d, nrm + 4);
      k_fd_point<<<nb, 256, 0, s>>>(n, U, b.d, nrm + 4, fdc, b.Uh, hval);
      if (macro_residual(s, ws, b.Uh, Uhist, bdt, b.Gh) != hipSuccess) return SLAR_E_HIP;
      k_fd_diff<<<nb, 256, 0, s>>>(n, b.Gh, b.g0, hval, 1, b.r);
      norm2(b.r, nrm + 5);
      HIP_TRY(hipMemcpyAsync(hh, nrm + 5, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      beta = std::sqrt(std::max(hh[0], 0.0));
      rec[2] = bn > 0.0 ? beta / bn : 0.0;
      rec[3] += 1.0;
      if (beta <= krylov_tol * bn || beta == 0.0) done = true;
    }
    rec[1] = kits;
    krylov += kits;
    if (!done && kry_limit < KRY_MAXIT) {
      // a preconditioned linear solve that stalls: give up on this solve
      if (iters) { iters[0] = newton; iters[1] = krylov; }
      return SLAR_E_NOCONV;
    }
    // exact step on the per-component mean
    k_comp_means<<<K, 256, 0, s>>>(Nx, b.d, b.g0, means);
    k_meanfix<<<nb, 256, 0, s>>>(Nx, K, means, means + 8, b.d);
    k_axpby<<<nb, 256, 0, s>>>(n, 1.0, b.d, 1.0, U, 0.0, nullptr);
    ++newton;
  }
  // U^(n+1) is complete in stream order
  HIP_TRY(hipMemcpyAsync(Uout, U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (iters) { iters[0] = newton; iters[1] = krylov; }
  return converged ? SLAR_OK : SLAR_E_NOCONV;
}

// The learned preconditioner has plain GMRES as its fallback: when the
// network's solve fails (a stalled linear solve, no Newton convergence, a
// non-finite value, a failed launch), the system is solved again from
// U(F*) without preconditioning.  The answer is judged by the same Newton
// tolerance either way; iteration counts include the failed attempt.
slar_status macro_solve_run(hipStream_t s, Workspace* ws, const MacroHist& hist, double beta,
                            double newton_tol, double krylov_tol, int precond,
                            const slar_cnn* cnn, double* Uout, int* iters) {
  ws->macro_fell_back = false;
  if (precond != 2)
    return macro_solve_once(s, ws, hist, beta, newton_tol, krylov_tol, precond, cnn, Uout, iters,
                            KRY_MAXIT);
  int it1[2] = {0, 0};
  slar_status st = macro_solve_once(s, ws, hist, beta, newton_tol, krylov_tol, 2, cnn, Uout, it1,
                                    KRY_LEARNED_LIMIT);
  if (st == SLAR_OK || st == SLAR_E_INVAL) {
    if (iters) { iters[0] = it1[0]; iters[1] = it1[1]; }
    return st;
  }
  (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
  ++ws->macro_fallbacks;
  ws->macro_fell_back = true;
  int it2[2] = {0, 0};
  st = macro_solve_once(s, ws, hist, beta, newton_tol, krylov_tol, 0, nullptr, Uout, it2, KRY_MAXIT);
  if (iters) { iters[0] = it1[0] + it2[0]; iters[1] = it1[1] + it2[1]; }
  return st;
}

// ------------------------------------------------- correction filter
// U <- U(F*) + sigma (U - U(F*)) with the exponential mode filter of
// SPEC_FILTER: the LoMaC correction acts on the resolved band of x-modes
// and leaves the kinetic solution's top modes to the kinetic update.  The
// zero mode is untouched (sigma = 1), so the totals of U are kept exactly.
slar_status lomac_filter_run(hipStream_t s, Workspace* ws, double* U) {
  if (!ws->lm_ready) return SLAR_E_INVAL;
  const GridDev& G = ws->G;
  const int K = G.dv + 2, Nx = G.nx, n = K * Nx;
  const LmLayout L = lm_layout(G);
  const double* U0 = ws->lm + L.U0;
  KryBufs b = kry_bufs(ws, n, KRY_RESTART);
  const unsigned nb = (n + 255) / 256;
  k_axpby<<<nb, 256, 0, s>>>(n, 1.0, U, 0.0, b.Uh, -1.0, U0);          // d = U - U0
  HIP_TRY(spectral_stage(s, ws, SPEC_FILTER, b.Uh, b.Gh, nullptr, (double2*)ws->cbuf + (size_t)24 * Nx));
  k_axpby<<<nb, 256, 0, s>>>(n, 1.0, U0, 0.0, U, 1.0, b.Gh);           // U = U0 + sigma d
  HIP_TRY(hipGetLastError());
  return SLAR_OK;
}

// --------------------------------------------------------------- project
__global__ void k_project(int Nx, int Nv, int dv, int r, int ldo, const double* __restrict__ Uf,
                          const double* __restrict__ phiE, const double* __restrict__ scal,
                          const double* __restrict__ Cstar, const double* __restrict__ Q,
                          double* __restrict__ Xo, double* __restrict__ Po, int dx) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = dv + 2;
  if (e < Nx) {
    double ep = 0.0;
    for (int m = 0; m < dx; ++m) {
      const double Em = phiE[(size_t)(1 + m) * Nx + e];
      ep += Em * Em;
    }
    ep *= 0.5;
    double Mr[4], C[4];
    for (int q = 0; q <= dv; ++q) Mr[q] = Uf[(size_t)q * Nx + e];
    Mr[dv + 1] = 2.0 * (Uf[(size_t)(dv + 1) * Nx + e] - ep);
    coeffs_at(dv, scal, Mr, C);
    for (int k = 0; k < K; ++k) Xo[(size_t)e * ldo + r + k] = C[k] - Cstar[(size_t)k * Nx + e];
  }
  if (e < Nv)
    for (int k = 0; k < K; ++k) Po[(size_t)e * ldo + r + k] = Q[(size_t)e * K + k];
}

slar_status lomac_project_run(hipStream_t s, Workspace* ws, const slar_frames& Fs,
                              const double* Unew, slar_frames* out) {
  if (!ws->lm_ready) return SLAR_E_INVAL;
  const GridDev& G = ws->G;
  const LmLayout L = lm_layout(G);
  const int K = G.dv + 2;
  MacroBufs b = macro_bufs(ws);
  if (copy2d(s, G.nx, Fs.r, Fs.X, Fs.ld, out->X, out->ld, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (copy2d(s, G.nv, Fs.r, Fs.P, Fs.ld, out->P, out->ld, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (poisson_run(s, ws, Unew, ws->n_i, b.phiE, b.phiE + G.nx) != hipSuccess) return SLAR_E_HIP;
  const int mx = std::max(G.nx, G.nv);
  k_project<<<(mx + 255) / 256, 256, 0, s>>>(G.nx, G.nv, G.dv, Fs.r, out->ld, Unew, b.phiE,
                                             ws->lm + L.scal, ws->lm + L.Cstar, ws->lm + L.Q,
                                             out->X, out->P, G.dx);
  HIP_TRY(hipGetLastError());
  out->r = Fs.r + K;
  return SLAR_OK;
}

}  // namespace slar
