// Adaptive cross approximation of the SL-updated tensor (HTACA sampling stage,
// introduction and section 3.1; the pivoting rules are documented in slar.h).
//
// Every iteration is two launches that read and write a device control
// block, so the host can enqueue several iterations before it looks at the
// stop flag:
//   k_aca_row : every block derives the row pivot i (the unused row
//               maximising the last column residual, from the column
//               launch's block candidates, or the probe check's worst
//               entry), samples row fiber A[i, :] (Nv entries) through the
//               SL-FD evaluator, stores the residual
//               r = A[i,:] - sum_l u_l[i] v_l as V[k], per-block partials of
//               v_l . r and a per-block pivot candidate, and finishes the
//               sums of the column launch's dot products;
//   k_aca_col : every block runs the stopping test of the previous term
//               (||S_k||^2 update; stop, probe check or continue), derives
//               the column pivot j from the row candidates (lowest index
//               within a relative 1e-10 of the maximum), samples column
//               fiber A[:, j] (Nx entries), stores the residual scaled by
//               1/r_j as U[k], partials of u_l . u and per-block candidates
//               of the next row pivot (unused rows); or it samples the
//               probe entries when the cross wants to stop.
// A row launch samples its row before the stopping test of the previous
// term has run; the column launch discards that row when the test stops.
// Kernel boundaries order the partial sums; no inter-block fences are used.
// The rank-1 terms are u_k v_k^T with u_k = column residual / r_j and
// v_k = row residual (the same product as the textbook v = r / r_j).
#include <algorithm>
#include <cmath>
#include <vector>

#include <hip/hip_ext.h>

#include "aca.h"
#include "dense.h"

namespace slar {

size_t aca_ctl_bytes() { return 2 * sizeof(AcaCtl); }
size_t aca_part_elems() { return (size_t)ACA_PART_SLOTS * ACA_MAXBLK; }

template <typename T, int W, int DX>
static hipError_t aca_iterate(hipStream_t s, const GridDev& G, const AdvDev& A, const T* X,
                              const T* P, int ld, int r, AcaCtl* ctl, double* U, double* V,
                              unsigned char* used, double* part, int nprobe, const int* probes,
                              hipEvent_t* ev, int* phase_dev, int seq, int* piv) {
  const unsigned bRow = (G.nv + ACA_TILE - 1) / ACA_TILE;
  const unsigned bCol = (G.nx + ACA_TILE - 1) / ACA_TILE;
  AcaInst I{G, A, X, P, ld, r, ctl, U, V, used, part, (int)bRow, (int)bCol, nprobe, 16, probes};
  I.phase_host = phase_dev;
  I.seq = seq;
  I.piv = piv;
  if (ev) {
    // events attached to the dispatches themselves: start and end of the
    // kernel, without marker packets between the launches
    hipExtLaunchKernelGGL(k_aca_row<T, W, DX>, dim3(bRow), dim3(FS_THREADS), 0, s, ev[0], ev[1], 0, I);
    hipExtLaunchKernelGGL(k_aca_col<T, W, DX>, dim3(bCol), dim3(FS_THREADS), 0, s, ev[2], ev[3], 0, I);
  } else {
    k_aca_row<T, W, DX><<<bRow, FS_THREADS, 0, s>>>(I);
    k_aca_col<T, W, DX><<<bCol, FS_THREADS, 0, s>>>(I);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t aca_iter_dispatch(hipStream_t s, const GridDev& G, const AdvDev& A, const T* X,
                                    const T* P, int ld, int r, AcaCtl* ctl, double* U, double* V,
                                    unsigned char* used, double* part, int nprobe,
                                    const int* probes, hipEvent_t* ev, int* phase_dev, int seq, int* piv) {
  if (G.dx == 1) {
    if (A.order == 5)
      return aca_iterate<T, 5, 1>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes, ev, phase_dev, seq, piv);
    return aca_iterate<T, 3, 1>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes, ev, phase_dev, seq, piv);
  }
  return aca_iterate<T, 3, 2>(s, G, A, X, P, ld, r, ctl, U, V, used, part, nprobe, probes, ev, phase_dev, seq, piv);
}

hipError_t table_copy(hipStream_t s, int rows, int r, int ldin, const double* in, int ldo,
                      float* o32, double* o64);

// Wait until the device has written a sequence number >= target into ph[1]
// (host-mapped).  Every 1024 polls the stream is queried: once it has
// drained, the number must be there (else SLAR_E_HIP), and a stream error
// ends the wait as well.
static slar_status wait_seq(hipStream_t s, volatile int* ph, int target) {
  for (long n = 1;; ++n) {
    if (ph[1] >= target) return SLAR_OK;
    if ((n & 1023) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) return ph[1] >= target ? SLAR_OK : SLAR_E_HIP;
      if (q != hipErrorNotReady) return SLAR_E_HIP;
    }
  }
}

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
  AdvDev A{adv.kind, adv.order, adv.tau, adv.cv, ws->Eeff, nullptr, 1.0, 0.0, 1};
  AcaCtl h{};
  h.phase = ACA_RUN; h.k = 0; h.i = 0; h.j = 0; h.kmax = kmax; h.tol = tol; h.norm2 = 0.0;
  AcaCtl* ctl = (AcaCtl*)ws->aca_ctl;
  AcaCtl* hc = (AcaCtl*)ws->aca_ctl_host;
  *hc = h;
  HIP_TRY(hipMemcpyAsync(ctl, hc, sizeof(AcaCtl), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(ws->used, 0, G.nx, s));
  const int maxit = kmax + 64;
  // algorithmic bytes of one sampled entry: both stencil gathers, the reads
  // of the previous cross vectors (residual and dot products) and the write
  const int rx = (G.dx == 2) ? adv.order * adv.order : adv.order;
  const double gather_bytes = 2.0 * rx * ldt * (dt == SLAR_F32 ? 4.0 : 8.0) + 8.0;
  const bool timing = ws->timing && (int)ws->events.size() >= 4 * maxit;
  // Iterations are enqueued in chunks of CH.  The last column launch of
  // chunk c writes the phase and then the sequence number c + 1 to
  // host-mapped pinned words (a store that crosses to host memory delays
  // the end of its kernel, so the others skip it).  Once the next chunk is
  // queued (so the device never idles on a poll), the host waits until the
  // sequence number reaches the previous chunk's and reads the phase.  A
  // newer value than that chunk's is harmless: DONE is final.  (An event
  // recorded after each chunk for the same purpose held the next launch
  // back by ~4 us.)
  // Iterations enqueued after the stop see phase != RUN and exit at once
  // (their launches did no work and are left out of the timing below).
  constexpr int CH = 8;
  auto timed = [&](int q) { return timing && (q % ws->timing_every) == ws->timing_every - 1; };
  volatile int* ph = (volatile int*)ws->phase_host;
  ph[0] = ACA_RUN;                              // no launch of this workspace is in flight
  ph[1] = 0;
  int it = 0, pending = -1;
  bool stop = false;
  while (it < maxit && !stop) {
    const int c = it / CH;
    for (const int end = std::min(it + CH, maxit); it < end; ++it) {
      hipError_t e;
      int* pw = (it == end - 1) ? ws->phase_dev : nullptr;
      if (dt == SLAR_F32)
        e = aca_iter_dispatch<float>(s, G, A, ws->X32, ws->P32, ldt, r, ctl, out->U, out->V,
                                     ws->used, ws->aca_part, nprobe, probes,
                                     timed(it) ? &ws->events[4 * it] : nullptr, pw, c + 1, ws->aca_piv);
      else
        e = aca_iter_dispatch<double>(s, G, A, X64, P64, ldt, r, ctl, out->U, out->V, ws->used,
                                      ws->aca_part, nprobe, probes,
                                      timed(it) ? &ws->events[4 * it] : nullptr, pw, c + 1, ws->aca_piv);
      if (e != hipSuccess) return SLAR_E_HIP;
    }
    if (pending >= 0) {
      const slar_status w = wait_seq(s, ph, pending + 1);
      if (w != SLAR_OK) return w;
      stop = ph[0] == ACA_DONE;
    }
    pending = c;
  }
  HIP_TRY(hipMemcpyAsync(hc, ctl, sizeof(AcaCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (timing) {
    // iterations 0 .. iters-1 did their work; the rank grows by one per
    // iteration except in those that met a reproduced row
    for (int q = 0; q < std::min(it, hc->iters); ++q) {
      if (!timed(q)) continue;
      float ms_row = 0.f, ms_col = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms_row, ws->events[4 * q], ws->events[4 * q + 1]));
      HIP_TRY(hipEventElapsedTime(&ms_col, ws->events[4 * q + 2], ws->events[4 * q + 3]));
      const double per = gather_bytes + 16.0 * std::min(q, hc->k);
      ws->tstat[0] += ms_row; ws->tstat[1] += 1; ws->tstat[2] += per * G.nv;
      ws->tstat[3] += ms_col; ws->tstat[4] += 1; ws->tstat[5] += per * G.nx;
    }
  }
  out->k = hc->k;
  if (info) {
    info->rank = hc->k;
    info->iterations = hc->iters;
    info->probe_rounds = hc->probe_rounds;
    info->converged = hc->converged;
    info->samples = hc->samples;
  }
  if (!std::isfinite(hc->norm2)) return SLAR_E_NUMERIC;
  if (hc->capped || hc->phase != ACA_DONE) {
    // stopped at the term cap: the skeleton's pivot block gets a
    // pseudo-inverse truncated at the workspace's rank cap
    if (out->k > ws->rmax) {
      const slar_status st = cur_core_run(s, ws, out, ws->rmax);
      if (st != SLAR_OK) return st;
      if (info) info->rank = out->k;
    }
    return SLAR_E_RANK_CAP;
  }
  return SLAR_OK;
}

// Ui[l][m] = u_m[i_l], Vjt[l][m] = v_m[j_l] for the logged pivots (i_l, j_l)
__global__ void k_cur_gather(int k, const double* __restrict__ U, int Nx, const double* __restrict__ V,
                             int Nv, const int* __restrict__ piv, double* __restrict__ Ui,
                             double* __restrict__ Vjt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int l = e / k, m = e % k;
  Ui[e] = U[(size_t)m * Nx + piv[2 * l]];
  Vjt[e] = V[(size_t)m * Nv + piv[2 * l + 1]];
}

// The k terms of a capped cross are U^T V = C W^-1 R with the pivot
// columns C = U^T Vjt^T, the pivot rows R = Ui V and the pivot block
// W = Ui Vjt^T.  With W = Y diag(s) Z^T and r = min(rcap, #{s > 1e-14 s_1})
// the regularised skeleton C Z_r diag(s_r)^-1 Y_r^T R is returned as the r
// terms U' = (Z_r diag(s_r)^-1)^T Vjt U and V' = Y_r^T Ui V.
namespace {
struct CurBuf {
  double *Ui, *Vjt, *W, *Y, *Z, *sv, *Pm, *Qm, *Ut, *Vt;
};
CurBuf cur_carve(Workspace* ws, int k) {
  const GridDev& G = ws->G;
  double* p = ws->small;
  CurBuf c;
  c.Ui = p; p += (size_t)k * k;
  c.Vjt = p; p += (size_t)k * k;
  c.W = p; p += (size_t)k * k;
  c.Y = p; p += (size_t)k * k;
  c.Z = p; p += (size_t)k * k;
  c.sv = p; p += k;
  c.Pm = p; p += (size_t)k * k;
  c.Qm = p; p += (size_t)k * k;
  c.Ut = p; p += (size_t)k * G.nx;
  c.Vt = p; p += (size_t)k * G.nv;
  return c;
}
// pivot rows / columns and the pivot block W
hipError_t cur_front(hipStream_t s, Workspace* ws, const slar_lowrank* out, const CurBuf& c) {
  const int k = out->k;
  k_cur_gather<<<(k * k + 255) / 256, 256, 0, s>>>(k, out->U, ws->G.nx, out->V, ws->G.nv, ws->aca_piv, c.Ui, c.Vjt);
  HIP_CHK(hipGetLastError());
  return gemm_f64(s, false, true, k, k, k, 1.0, c.Ui, k, 0, c.Vjt, k, 0, 0.0, c.W, k, 0, 1);
}
// kept triplets: s_i > 1e-14 s_1, at most rcap, at least one; 0 if s_1 is
// not a positive finite number
int cur_rank(const double* hs, int k, int rcap) {
  if (!(hs[0] > 0.0) || !std::isfinite(hs[0])) return 0;
  int r = 0;
  while (r < k && r < rcap && hs[r] > 1e-14 * hs[0]) ++r;
  return std::max(r, 1);
}
// the r new terms, written over the first r of U and V
hipError_t cur_back(hipStream_t s, Workspace* ws, slar_lowrank* out, const CurBuf& c, int r) {
  const int k = out->k, Nx = ws->G.nx, Nv = ws->G.nv;
  if (k > 64) {
    // right vectors of the kept triplets: Z_r = W^T Y_r diag(s_r)^-1
    HIP_CHK(gemm_f64(s, true, false, k, r, k, 1.0, c.W, k, 0, c.Y, k, 0, 0.0, c.Z, k, 0, 1));
    HIP_CHK(scale_cols_inv(s, k, r, c.Z, k, c.sv));
  }
  HIP_CHK(scale_cols_inv(s, k, r, c.Z, k, c.sv));   // Z_r diag(s_r)^-1
  HIP_CHK(gemm_f64(s, true, false, r, k, k, 1.0, c.Z, k, 0, c.Vjt, k, 0, 0.0, c.Pm, k, 0, 1));
  HIP_CHK(gemm_f64(s, true, false, r, k, k, 1.0, c.Y, k, 0, c.Ui, k, 0, 0.0, c.Qm, k, 0, 1));
  HIP_CHK(gemm_f64(s, false, false, r, Nx, k, 1.0, c.Pm, k, 0, out->U, Nx, 0, 0.0, c.Ut, Nx, 0, 1));
  HIP_CHK(gemm_f64(s, false, false, r, Nv, k, 1.0, c.Qm, k, 0, out->V, Nv, 0, 0.0, c.Vt, Nv, 0, 1));
  HIP_CHK(hipMemcpyAsync(out->U, c.Ut, sizeof(double) * r * Nx, hipMemcpyDeviceToDevice, s));
  return hipMemcpyAsync(out->V, c.Vt, sizeof(double) * r * Nv, hipMemcpyDeviceToDevice, s);
}
}  // namespace

slar_status cur_core_run(hipStream_t s, Workspace* ws, slar_lowrank* out, int rcap) {
  const int k = out->k;
  const CurBuf c = cur_carve(ws, k);
  if (cur_front(s, ws, out, c) != hipSuccess) return SLAR_E_HIP;
  if (k > 64) {
    if (svd_left_big(s, k, c.W, c.Y, c.sv) != hipSuccess) return SLAR_E_HIP;
  } else if (svd_small(s, k, c.W, c.Y, c.sv, c.Z) != hipSuccess) {
    return SLAR_E_HIP;
  }
  double* hs = (double*)ws->host_pinned;
  HIP_TRY(hipMemcpyAsync(hs, c.sv, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int r = cur_rank(hs, k, rcap);
  if (r == 0) return SLAR_E_NUMERIC;
  // the new terms are complete in stream order; the host already knows r
  if (cur_back(s, ws, out, c, r) != hipSuccess) return SLAR_E_HIP;
  out->k = r;
  return SLAR_OK;
}

// The same for several capped crosses at once: the pivot-block SVDs run as
// one grouped launch per size class, and the host reads all singular
// values in one copy.  dmem / hmem: cur_core_group_bytes(n) of device /
// pinned host memory.
static size_t cg_align(size_t x) { return (x + 255) & ~(size_t)255; }
size_t cur_core_group_bytes(int n) {
  n = std::max(n, 1);
  return cg_align(sizeof(SvdDesc) * n) + cg_align(sizeof(double) * SLAR_CROSS_KMAX * n);
}

slar_status cur_core_group(hipStream_t s, int n, Workspace* const* ws, slar_lowrank* const* out,
                           const int* rcap, slar_status* st, void* dmem, void* hmem) {
  if (n <= 0) return SLAR_OK;
  const size_t CK = SLAR_CROSS_KMAX, off_sv = cg_align(sizeof(SvdDesc) * n);
  std::vector<CurBuf> cb(n);
  std::vector<SvdDesc> sm, bg;
  double* svs = (double*)((char*)dmem + off_sv);
  for (int j = 0; j < n; ++j) {
    const int k = out[j]->k;
    st[j] = SLAR_OK;
    cb[j] = cur_carve(ws[j], k);
    if (cur_front(s, ws[j], out[j], cb[j]) != hipSuccess) return SLAR_E_HIP;
    if (k > 64) bg.push_back(SvdDesc{k, cb[j].W, cb[j].Y, cb[j].sv, nullptr, svs + (size_t)j * CK});
    else sm.push_back(SvdDesc{k, cb[j].W, cb[j].Y, cb[j].sv, cb[j].Z, svs + (size_t)j * CK});
  }
  SvdDesc* hd = (SvdDesc*)hmem;
  std::copy(sm.begin(), sm.end(), hd);
  std::copy(bg.begin(), bg.end(), hd + sm.size());
  HIP_TRY(hipMemcpyAsync(dmem, hmem, sizeof(SvdDesc) * n, hipMemcpyHostToDevice, s));
  if (svd_group(s, (int)sm.size(), (const SvdDesc*)dmem, false) != hipSuccess) return SLAR_E_HIP;
  if (svd_group(s, (int)bg.size(), (const SvdDesc*)dmem + sm.size(), true) != hipSuccess) return SLAR_E_HIP;
  const double* hs = (const double*)((char*)hmem + off_sv);
  HIP_TRY(hipMemcpyAsync((char*)hmem + off_sv, svs, sizeof(double) * CK * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int> r(n);
  for (int j = 0; j < n; ++j) {
    r[j] = cur_rank(hs + (size_t)j * CK, out[j]->k, rcap[j]);
    if (r[j] == 0) { st[j] = SLAR_E_NUMERIC; continue; }
    if (cur_back(s, ws[j], out[j], cb[j], r[j]) != hipSuccess) return SLAR_E_HIP;
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (int j = 0; j < n; ++j)
    if (st[j] == SLAR_OK) out[j]->k = r[j];
  return SLAR_OK;
}

}  // namespace slar
