// Adaptive cross approximation of the SL-updated tensor (HTACA sampling stage,
// introduction and section 3.1; the pivoting rules are documented in slar.h).
//
// Every iteration is three launches that read and write a device control
// block, so the host can enqueue several iterations before it looks at the
// stop flag:
//   k_aca_row : sample row fiber A[i, :] (Nv entries) through the SL-FD
//               evaluator, residual r = A[i,:] - sum_l u_l[i] v_l, stored as
//               V[k]; block partials of max|r| and of v_l . r.  The last
//               block to finish picks the column pivot (lowest index within
//               a relative 1e-10 of the maximum).
//   k_aca_col : sample column fiber A[:, j] (Nx entries), residual scaled by
//               1/r_j stored as U[k]; partials of u_l . u; the last block
//               updates ||S_k||^2, applies the stopping test and chooses the
//               next row pivot among unused rows.
//   k_aca_probe: on a stop request, residuals at the host-given random
//               probe entries decide between finishing and continuing.
// The rank-1 terms are u_k v_k^T with u_k = column residual / r_j and
// v_k = row residual (the same product as the textbook v = r / r_j).
#include <cmath>

#include "slar_internal.h"
#include "frame_sampler.h"

namespace slar {

enum { ACA_RUN = 0, ACA_PROBE = 1, ACA_DONE = 2 };

struct AcaCtl {
  int phase, k, i, j;
  int iters, probe_rounds, converged, capped;
  unsigned cnt_row, cnt_col;
  int kmax, pad;
  double pivot, norm2, tol;
  long long samples;
  double gv[SLAR_KMAX + 1];
  double gu[SLAR_KMAX + 1];
};

constexpr int ACA_MAXBLK = 1024;   // partial slots

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block max of |v| over 256 threads -> returns in all threads
__device__ double block_max(double v, double* red) {
  const int t = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return m;
}

// Lowest index in [0, n) with |x[idx]| >= thr among entries with mask==0
// (mask may be null).  One block.
__device__ int block_first_at_least(const double* x, int n, double thr, const unsigned char* mask,
                                    int* redi) {
  const int t = threadIdx.x;
  int best = n;
  for (int e = t; e < n; e += blockDim.x) {
    if (mask && mask[e]) continue;
    if (fabs(x[e]) >= thr) { best = e; break; }
  }
  for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((t & 63) == 0) redi[t >> 6] = best;
  __syncthreads();
  const int b = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  __syncthreads();
  return b;
}

__device__ double block_max_masked(const double* x, int n, const unsigned char* mask, double* red) {
  double m = -1.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x)
    if (!(mask && mask[e])) m = fmax(m, fabs(x[e]));
  return block_max(m, red);
}

__device__ __forceinline__ void unravel_x(const GridDev& g, int I, int* gi) {
  if (g.dx == 1) gi[0] = I; else { gi[0] = I / g.n[1]; gi[1] = I % g.n[1]; }
}
__device__ __forceinline__ void unravel_v(const GridDev& g, int J, int* gi) {
  if (g.dv == 1) gi[1] = J; else { gi[2] = J / g.n[3]; gi[3] = J % g.n[3]; }
}

template <typename T, int W, int DX>
__global__ __launch_bounds__(FS_THREADS) void k_aca_row(GridDev g, AdvDev a, const T* __restrict__ X,
                                                         const T* __restrict__ P, int ld, int r,
                                                         AcaCtl* ctl, double* __restrict__ U,
                                                         double* __restrict__ V,
                                                         unsigned char* __restrict__ used,
                                                         double* __restrict__ part) {
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int s_phase, s_i, s_k, s_last;
  const int t = threadIdx.x;
  if (t == 0) { s_phase = ctl->phase; s_i = ctl->i; s_k = ctl->k; }
  __syncthreads();
  if (s_phase != ACA_RUN) return;
  const int i = s_i, k = s_k;
  const int Nx = g.nx, Nv = g.nv;
  const int J0 = blockIdx.x * FS_SAMPLES;
  const int ns = min(FS_SAMPLES, Nv - J0);
  if (t < ns) {
    int gi[4];
    unravel_x(g, i, gi);
    unravel_v(g, J0 + t, gi);
    fs_prepare<W, DX>(g, a, gi, L, t);
  }
  __syncthreads();
  fs_evaluate<T, W, DX>(X, P, ld, r, L, ns);
  __syncthreads();
  double rv = 0.0;
  double amax = 0.0;
  if (t < 64) {
    if (t < ns) {
      const int J = J0 + t;
      rv = L.val[t];
      for (int l = 0; l < k; ++l) rv -= U[(size_t)l * Nx + i] * V[(size_t)l * Nv + J];
      V[(size_t)k * Nv + J] = rv;
      amax = fabs(rv);
    }
    // partial dot products v_l . r (l < k) and r . r (l = k), wave 0
    for (int l = 0; l <= k; ++l) {
      double p = 0.0;
      if (t < ns) p = (l < k ? V[(size_t)l * Nv + J0 + t] : rv) * rv;
      p = wave_sum(p);
      if (t == 0) part[(size_t)(1 + l) * ACA_MAXBLK + blockIdx.x] = p;
    }
  }
  amax = block_max(amax, red);
  if (t == 0) part[blockIdx.x] = amax;
  __threadfence();
  __syncthreads();
  if (t == 0) s_last = (atomicAdd(&ctl->cnt_row, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // ---- finalize (last block)
  const int nb = gridDim.x;
  double m = 0.0;
  for (int b = t; b < nb; b += blockDim.x) m = fmax(m, part[b]);
  m = block_max(m, red);
  const double thr = ctl->tol * sqrt(ctl->norm2) / sqrt((double)Nx * (double)Nv);
  const double* vk = V + (size_t)k * Nv;
  int jp = 0;
  if (m > 0.0 && m > thr) jp = block_first_at_least(vk, Nv, m * (1.0 - 1e-10), nullptr, redi);
  for (int l = t; l <= k; l += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)(1 + l) * ACA_MAXBLK + b];
    ctl->gv[l] = acc;
  }
  if (t == 0) {
    ctl->cnt_row = 0;
    used[i] = 1;
    ctl->iters += 1;
    ctl->samples += Nv;
    if (m == 0.0 || m <= thr) {
      ctl->phase = ACA_PROBE;
    } else {
      ctl->j = jp;
      ctl->pivot = vk[jp];
    }
  }
}

template <typename T, int W, int DX>
__global__ __launch_bounds__(FS_THREADS) void k_aca_col(GridDev g, AdvDev a, const T* __restrict__ X,
                                                         const T* __restrict__ P, int ld, int r,
                                                         AcaCtl* ctl, double* __restrict__ U,
                                                         double* __restrict__ V,
                                                         unsigned char* __restrict__ used,
                                                         double* __restrict__ part) {
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int s_phase, s_j, s_k, s_last;
  __shared__ double s_piv;
  const int t = threadIdx.x;
  if (t == 0) { s_phase = ctl->phase; s_j = ctl->j; s_k = ctl->k; s_piv = ctl->pivot; }
  __syncthreads();
  if (s_phase != ACA_RUN) return;
  const int j = s_j, k = s_k;
  const double piv = s_piv;
  const int Nx = g.nx, Nv = g.nv;
  const int I0 = blockIdx.x * FS_SAMPLES;
  const int ns = min(FS_SAMPLES, Nx - I0);
  if (t < ns) {
    int gi[4];
    unravel_x(g, I0 + t, gi);
    unravel_v(g, j, gi);
    fs_prepare<W, DX>(g, a, gi, L, t);
  }
  __syncthreads();
  fs_evaluate<T, W, DX>(X, P, ld, r, L, ns);
  __syncthreads();
  if (t < 64) {
    double u = 0.0;
    if (t < ns) {
      const int I = I0 + t;
      u = L.val[t];
      for (int l = 0; l < k; ++l) u -= V[(size_t)l * Nv + j] * U[(size_t)l * Nx + I];
      u = u / piv;
      U[(size_t)k * Nx + I] = u;
    }
    for (int l = 0; l <= k; ++l) {
      double p = 0.0;
      if (t < ns) p = (l < k ? U[(size_t)l * Nx + I0 + t] : u) * u;
      p = wave_sum(p);
      if (t == 0) part[(size_t)(1 + l) * ACA_MAXBLK + blockIdx.x] = p;
    }
  }
  __threadfence();
  __syncthreads();
  if (t == 0) s_last = (atomicAdd(&ctl->cnt_col, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int nb = gridDim.x;
  for (int l = t; l <= k; l += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)(1 + l) * ACA_MAXBLK + b];
    ctl->gu[l] = acc;
  }
  __syncthreads();
  __shared__ int s_stop;
  if (t == 0) {
    ctl->cnt_col = 0;
    ctl->samples += Nx;
    double cross = 0.0;
    for (int l = 0; l < k; ++l) cross += ctl->gu[l] * ctl->gv[l];
    const double nk = ctl->gu[k] * ctl->gv[k];
    ctl->norm2 = ctl->norm2 + 2.0 * cross + nk;
    ctl->k = k + 1;
    s_stop = 0;
    if (sqrt(nk) <= ctl->tol * sqrt(fmax(ctl->norm2, 0.0))) {
      ctl->phase = ACA_PROBE;
      s_stop = 1;
    } else if (k + 1 >= ctl->kmax) {
      ctl->phase = ACA_DONE;
      ctl->capped = 1;
      s_stop = 1;
    }
  }
  __syncthreads();
  if (s_stop) return;
  const double* uk = U + (size_t)k * Nx;
  const double m = block_max_masked(uk, Nx, used, red);
  int ip = Nx;
  if (m >= 0.0) ip = block_first_at_least(uk, Nx, m * (1.0 - 1e-10), used, redi);
  if (t == 0) {
    if (ip >= Nx) ctl->phase = ACA_DONE;
    else ctl->i = ip;
  }
}

template <typename T, int W, int DX>
__global__ __launch_bounds__(FS_THREADS) void k_aca_probe(GridDev g, AdvDev a, const T* __restrict__ X,
                                                           const T* __restrict__ P, int ld, int r,
                                                           AcaCtl* ctl, const double* __restrict__ U,
                                                           const double* __restrict__ V,
                                                           const unsigned char* __restrict__ used,
                                                           int nprobe, const int* __restrict__ probes) {
  __shared__ FsLds<W, DX> L;
  __shared__ double res[1024];
  __shared__ int pi[1024];
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int s_phase, s_k;
  const int t = threadIdx.x;
  if (t == 0) { s_phase = ctl->phase; s_k = ctl->k; }
  __syncthreads();
  if (s_phase != ACA_PROBE) return;
  const int k = s_k;
  const int Nx = g.nx, Nv = g.nv;
  if (k == 0 || nprobe <= 0) {
    if (t == 0) { ctl->phase = ACA_DONE; ctl->converged = 1; }
    return;
  }
  const double thr = ctl->tol * sqrt(fmax(ctl->norm2, 0.0)) / sqrt((double)Nx * (double)Nv);
  for (int base = 0; base < nprobe; base += FS_SAMPLES) {
    const int ns = min(FS_SAMPLES, nprobe - base);
    if (t < ns) {
      int gi[4];
      unravel_x(g, probes[2 * (base + t)], gi);
      unravel_v(g, probes[2 * (base + t) + 1], gi);
      fs_prepare<W, DX>(g, a, gi, L, t);
    }
    __syncthreads();
    fs_evaluate<T, W, DX>(X, P, ld, r, L, ns);
    __syncthreads();
    if (t < ns) {
      const int I = probes[2 * (base + t)], J = probes[2 * (base + t) + 1];
      double v = L.val[t];
      for (int l = 0; l < k; ++l) v -= U[(size_t)l * Nx + I] * V[(size_t)l * Nv + J];
      const bool bad = fabs(v) > thr && !used[I];
      res[base + t] = bad ? fabs(v) : -1.0;
      pi[base + t] = I;
    }
    __syncthreads();
  }
  double m = -1.0;
  for (int e = t; e < nprobe; e += blockDim.x) m = fmax(m, res[e]);
  m = block_max(m, red);
  int best = nprobe;
  if (m > 0.0) {
    for (int e = t; e < nprobe; e += blockDim.x)
      if (res[e] > 0.0 && res[e] >= m * (1.0 - 1e-10)) { best = e; break; }
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    if ((t & 63) == 0) redi[t >> 6] = best;
    __syncthreads();
    best = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  }
  if (t == 0) {
    ctl->samples += nprobe;
    if (m <= 0.0 || best >= nprobe) {
      ctl->phase = ACA_DONE;
      ctl->converged = 1;
    } else if (k >= ctl->kmax) {
      ctl->phase = ACA_DONE;
      ctl->capped = 1;
    } else {
      ctl->probe_rounds += 1;
      ctl->i = pi[best];
      ctl->phase = ACA_RUN;
    }
  }
}

size_t aca_ctl_bytes() { return sizeof(AcaCtl); }

template <typename T, int W, int DX>
static hipError_t aca_iterate(hipStream_t s, const GridDev& G, const AdvDev& A, const T* X,
                              const T* P, int ld, int r, AcaCtl* ctl, double* U, double* V,
                              unsigned char* used, double* part, int nprobe, const int* probes) {
  const unsigned bRow = (G.nv + FS_SAMPLES - 1) / FS_SAMPLES;
  const unsigned bCol = (G.nx + FS_SAMPLES - 1) / FS_SAMPLES;
  k_aca_row<T, W, DX><<<bRow, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, ctl, U, V, used, part);
  k_aca_col<T, W, DX><<<bCol, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, ctl, U, V, used, part);
  k_aca_probe<T, W, DX><<<1, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, ctl, U, V, used, nprobe, probes);
  return hipGetLastError();
}

template <typename T>
static hipError_t aca_iter_dispatch(hipStream_t s, const GridDev& G, const AdvDev& A, const T* X,
                                    const T* P, int ld, int r, AcaCtl* ctl, double* U, double* V,
                                    unsigned char* used, double* part, int nprobe,
                                    const int* probes) {
  if (G.dx == 1) {
    if (A.order == 5) return aca_iterate<T, 5, 1>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes);
    return aca_iterate<T, 3, 1>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes);
  }
  return aca_iterate<T, 3, 2>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes);
}

hipError_t table_copy(hipStream_t s, int rows, int r, int ldin, const double* in, int ldo,
                      float* o32, double* o64);

// Host driver of the cross approximation (synchronises the stream).
slar_status cross_run(hipStream_t s, Workspace* ws, const slar_frames& src, const slar_adv& adv,
                      slar_dtype dt, double tol, int kmax, int nprobe, const int* probes,
                      slar_lowrank* out, slar_cross_info* info) {
  const GridDev& G = ws->G;
  const int r = src.r;
  const int ldt = (r + 3) & ~3;
  // tables: FP64 copies live in dwork, FP32 copies in X32/P32
  double* X64 = ws->dwork;
  double* P64 = ws->dwork + (size_t)G.nx * ldt;
  if (dt == SLAR_F32) {
    if (table_copy(s, G.nx, r, src.ld, src.X, ldt, ws->X32, nullptr) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(s, G.nv, r, src.ld, src.P, ldt, ws->P32, nullptr) != hipSuccess) return SLAR_E_HIP;
  } else {
    if (table_copy(s, G.nx, r, src.ld, src.X, ldt, nullptr, X64) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(s, G.nv, r, src.ld, src.P, ldt, nullptr, P64) != hipSuccess) return SLAR_E_HIP;
  }
  if (combine_field(s, G, &adv, ws->Eeff) != hipSuccess) return SLAR_E_HIP;
  AdvDev A{adv.kind, adv.order, adv.tau, adv.cv, ws->Eeff, nullptr, 1.0, 0.0};
  AcaCtl h{};
  h.phase = ACA_RUN; h.k = 0; h.i = 0; h.j = 0; h.kmax = kmax; h.tol = tol; h.norm2 = 0.0;
  AcaCtl* ctl = (AcaCtl*)ws->aca_ctl;
  AcaCtl* hc = (AcaCtl*)ws->aca_ctl_host;
  *hc = h;
  HIP_TRY(hipMemcpyAsync(ctl, hc, sizeof(AcaCtl), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(ws->used, 0, G.nx, s));
  const int maxit = kmax + 64;
  for (int it = 0; it < maxit; ++it) {
    hipError_t e;
    if (dt == SLAR_F32)
      e = aca_iter_dispatch<float>(s, G, A, ws->X32, ws->P32, ldt, r, ctl, out->U, out->V,
                                   ws->used, ws->aca_part, nprobe, probes);
    else
      e = aca_iter_dispatch<double>(s, G, A, X64, P64, ldt, r, ctl, out->U, out->V, ws->used,
                                    ws->aca_part, nprobe, probes);
    if (e != hipSuccess) return SLAR_E_HIP;
    if ((it % 4) == 3 || it == maxit - 1) {
      HIP_TRY(hipMemcpyAsync(hc, ctl, sizeof(AcaCtl), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (hc->phase == ACA_DONE) break;
    }
  }
  HIP_TRY(hipMemcpyAsync(hc, ctl, sizeof(AcaCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->k = hc->k;
  if (info) {
    info->rank = hc->k;
    info->iterations = hc->iters;
    info->probe_rounds = hc->probe_rounds;
    info->converged = hc->converged;
    info->samples = hc->samples;
  }
  if (!std::isfinite(hc->norm2)) return SLAR_E_NUMERIC;
  if (hc->capped || hc->phase != ACA_DONE) return SLAR_E_RANK_CAP;
  return SLAR_OK;
}

}  // namespace slar
