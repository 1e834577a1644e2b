// C ABI entry points: argument validation, workspace management and the
// host-side orchestration of the kernels in the other translation units.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "slar_internal.h"
#include "dense.h"
#include "fields.h"
#include "lomac.h"
#include "truncate.h"

namespace slar {
hipError_t ht_sample(hipStream_t st, const GridDev& G, const AdvDev& A, const slar_ht& F,
                     long long n, const int* idx, void* out);
hipError_t frames_from_ht(hipStream_t s, Workspace* ws, const GridDev& G, const slar_ht& F,
                          slar_frames* out);
hipError_t table_copy(hipStream_t s, int rows, int r, int ldin, const double* in, int ldo,
                      float* o32, double* o64);
hipError_t frame_points(hipStream_t s, const GridDev& G, const AdvDev& A, slar_dtype dt,
                        const void* X, const void* P, int ld, int r, long long n, const int* idx,
                        double* out);
slar_status cross_run(hipStream_t s, Workspace* ws, const slar_frames& src, const slar_adv& adv,
                      slar_dtype dt, double tol, int kmax, int nprobe, const int* probes,
                      slar_lowrank* out, slar_cross_info* info);
size_t aca_ctl_bytes();
size_t aca_part_elems();
slar_status poisson_noalloc_run(hipStream_t s, const slar_grid& grid, const double* n_e, double n_i,
                                double* phi, double* E);
}  // namespace slar

using namespace slar;

static bool grid_ok(const slar_grid* g) {
  if (!g) return false;
  if (g->dx != g->dv || (g->dx != 1 && g->dx != 2)) return false;
  for (int m = 0; m < g->dx + g->dv; ++m) {
    if (g->n[m] < 4 || g->n[m] > (g->dx == 1 ? SLAR_NMAX_1D : SLAR_NMAX)) return false;
    if (!(g->hi[m] > g->lo[m]) || !std::isfinite(g->lo[m]) || !std::isfinite(g->hi[m])) return false;
  }
  return true;
}

static bool same_grid(const slar_grid* a, const slar_grid* b) {
  if (a->dx != b->dx || a->dv != b->dv) return false;
  for (int m = 0; m < a->dx + a->dv; ++m)
    if (a->n[m] != b->n[m] || a->lo[m] != b->lo[m] || a->hi[m] != b->hi[m]) return false;
  return true;
}

static bool adv_ok(const slar_grid* g, const slar_adv* a) {
  if (!a) return false;
  if (a->kind < 0 || a->kind > 2) return false;
  if (a->order != 3 && a->order != 5) return false;
  if (!std::isfinite(a->tau) || !std::isfinite(a->cv)) return false;
  if (a->kind != 0 && a->E[0] == nullptr) return false;
  if (g->dx == 2 && a->order != 3) return false;
  return true;
}

static bool ht_ok(const slar_grid* g, const slar_ht* F) {
  if (!F || F->d != g->dx + g->dv) return false;
  const int nr = F->d == 2 ? 2 : 6;
  for (int m = 0; m < nr; ++m)
    if (F->rank[m] < 1 || F->rank[m] > 64) return false;
  for (int m = 0; m < F->d; ++m)
    if (!F->leaf[m]) return false;
  if (!F->root) return false;
  if (F->d == 4 && (!F->B12 || !F->B34)) return false;
  if (F->dtype != SLAR_F32 && F->dtype != SLAR_F64) return false;
  return true;
}

static bool frames_ok(const slar_frames* F) {
  return F && F->X && F->P && F->r >= 1 && F->r <= SLAR_KMAX && F->ld >= F->r;
}

static AdvDev make_adv(const slar_adv* a, const double* Eeff) {
  return AdvDev{a->kind, a->order, a->tau, a->cv, Eeff, nullptr, 1.0, 0.0, 1};
}

extern "C" {

const char* slar_status_str(slar_status s) {
  switch (s) {
    case SLAR_OK: return "ok";
    case SLAR_E_INVAL: return "invalid argument";
    case SLAR_E_NOMEM: return "out of device memory";
    case SLAR_E_RANK_CAP: return "rank cap reached";
    case SLAR_E_NOCONV: return "Newton did not converge";
    case SLAR_E_NUMERIC: return "non-finite value";
    case SLAR_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"

// Sizes of a workspace's scratch for grid g and rank cap rmax.
static void ws_sizes(Workspace& ws, const slar_grid& g, int rmax) {
  ws.grid = g;
  ws.G = make_grid(g);
  ws.rmax = rmax;
  const GridDev& G = ws.G;
  const size_t K = SLAR_KMAX;
  ws.ld32 = SLAR_KMAX;
  ws.dwork_elems = std::max({(size_t)2 * (G.nx + G.nv) * K + 64,
                             (size_t)SLAR_NMAX * K * K + (size_t)G.nv * K + 64,
                             (size_t)SLAR_NMAX * SLAR_NMAX * SLAR_NMAX + 64,
                             (size_t)(G.nx / 256 + 2) * K * 9 + (size_t)(G.nx / 512 + 2) * K * K,
                             (size_t)(SLAR_NMAX * K / 512 + 2) * SLAR_NMAX * SLAR_NMAX});
  ws.small_elems = truncate_scratch_elems(G) + 8192;
  ws.cbuf_elems = cbuf_elems_for(G.nx);
  ws.lm_elems = lm_layout(G).total;
  ws.kry_elems = kry_elems_for(G.nx, G.dv + 2, KRY_RESTART);
}

// Every device buffer of a workspace, in a fixed order: fn(slot, bytes).
template <class F>
static void ws_buffers(Workspace& ws, F&& fn) {
  const GridDev& G = ws.G;
  const int nm = nmom_of(G.dv);
  fn((void**)&ws.Eeff, sizeof(double) * G.dx * G.nx);
  fn((void**)&ws.X32, sizeof(float) * G.nx * ws.ld32);
  fn((void**)&ws.P32, sizeof(float) * G.nv * ws.ld32);
  fn(&ws.aca_ctl, aca_ctl_bytes());
  fn((void**)&ws.aca_part, sizeof(double) * aca_part_elems());
  fn((void**)&ws.aca_piv, sizeof(int) * 2 * SLAR_CROSS_KMAX);
  fn((void**)&ws.used, (size_t)G.nx);
  fn((void**)&ws.dwork, sizeof(double) * ws.dwork_elems);
  fn((void**)&ws.small, sizeof(double) * ws.small_elems);
  fn((void**)&ws.tw[0], sizeof(double) * 2 * SLAR_NLINE);
  fn((void**)&ws.tw[1], sizeof(double) * 2 * SLAR_NLINE);
  fn((void**)&ws.cbuf, sizeof(double) * ws.cbuf_elems);
  fn((void**)&ws.psi, sizeof(double) * G.nv * nm);
  fn((void**)&ws.lm, sizeof(double) * ws.lm_elems);
  fn((void**)&ws.kry, sizeof(double) * ws.kry_elems);
  if (G.d == 4) {
    const size_t NT = 16384, NL = nest_list_elems();
    fn((void**)&ws.nest_U, sizeof(double) * 64 * NT);
    fn((void**)&ws.nest_V, sizeof(double) * 64 * NT);
    fn((void**)&ws.nest_used, NT);
    fn((void**)&ws.nest_rowtab, sizeof(int) * 4 * NT);
    fn((void**)&ws.nest_coltab, sizeof(int) * 4 * NT);
    fn((void**)&ws.nest_probes, sizeof(int) * 2 * 128);
    fn((void**)&ws.nest_piv, sizeof(int) * 2 * SLAR_KMAX);
    fn((void**)&ws.nest_idx, sizeof(int) * 4 * NL);
    fn((void**)&ws.nest_vals, sizeof(double) * NL);
    fn((void**)&ws.nest_small, sizeof(double) * 6 * 64 * 64);
    fn((void**)&ws.nest_flag, sizeof(int) * 4);
    fn((void**)&ws.nest_fX, sizeof(double) * G.nx * SLAR_KMAX);
    fn((void**)&ws.nest_fP, sizeof(double) * G.nv * SLAR_KMAX);
    fn((void**)&ws.nest_X64, sizeof(double) * G.nx * SLAR_KMAX);
    fn((void**)&ws.nest_P64, sizeof(double) * G.nv * SLAR_KMAX);
  }
}

static size_t ws_align(size_t b) { return (std::max(b, (size_t)256) + 255) & ~(size_t)255; }

extern "C" {

slar_status slar_workspace_bytes(const slar_grid* g, int32_t rmax, size_t* bytes) {
  if (!bytes || !grid_ok(g) || rmax < 1 || rmax > 64) return SLAR_E_INVAL;
  Workspace ws;
  ws_sizes(ws, *g, rmax);
  size_t total = 0;
  ws_buffers(ws, [&](void**, size_t b) { total += ws_align(b); });
  *bytes = total;
  return SLAR_OK;
}

slar_status slar_workspace_destroy(slar_workspace* w) {
  if (!w) return SLAR_OK;
  Workspace& ws = w->w;
  if (ws.owns_device) ws_buffers(ws, [](void** p, size_t) { if (*p) (void)hipFree(*p); });
  for (hipEvent_t e : ws.events) (void)hipEventDestroy(e);
  if (ws.ev_fork) (void)hipEventDestroy(ws.ev_fork);
  if (ws.ev_join) (void)hipEventDestroy(ws.ev_join);
  for (hipEvent_t e : ws.poll_ev)
    if (e) (void)hipEventDestroy(e);
  if (ws.aux) {
    (void)hipStreamSynchronize(ws.aux);
    (void)hipStreamDestroy(ws.aux);
  }
  if (ws.aca_ctl_host) (void)hipHostFree(ws.aca_ctl_host);
  if (ws.host_pinned) (void)hipHostFree(ws.host_pinned);
  if (ws.phase_host) (void)hipHostFree(ws.phase_host);
  delete w;
  return SLAR_OK;
}

// work == nullptr: the library allocates the device buffers; else they are
// carved from the caller's work (work_bytes >= slar_workspace_bytes).
static slar_status ws_create(const slar_grid* g, int32_t rmax, void* work, size_t work_bytes,
                             slar_workspace** out) {
  *out = nullptr;
  size_t need = 0;
  if (work) {
    if (slar_workspace_bytes(g, rmax, &need) != SLAR_OK) return SLAR_E_INVAL;
    if (work_bytes < need || ((uintptr_t)work & 255) != 0) return work_bytes < need ? SLAR_E_NOMEM : SLAR_E_INVAL;
  }
  slar_workspace* w = new (std::nothrow) slar_workspace();
  if (!w) return SLAR_E_NOMEM;
  Workspace& ws = w->w;
  ws_sizes(ws, *g, rmax);
  const GridDev& G = ws.G;
  bool ok = true;
  if (work) {
    ws.owns_device = false;
    char* p = (char*)work;
    ws_buffers(ws, [&](void** slot, size_t b) {
      *slot = p;
      p += ws_align(b);
    });
  } else {
    ws.owns_device = true;
    ws_buffers(ws, [&](void** slot, size_t b) {
      if (ok && hipMalloc(slot, std::max(b, (size_t)256)) != hipSuccess) ok = false;
    });
  }
  if (ok && hipHostMalloc(&ws.aca_ctl_host, 3 * aca_ctl_bytes(), 0) != hipSuccess) ok = false;
  for (hipEvent_t& e : ws.poll_ev)
    if (ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) ok = false;
  if (ok && hipHostMalloc(&ws.host_pinned, 65536, 0) != hipSuccess) ok = false;
  if (ok && hipHostMalloc((void**)&ws.phase_host, 256, hipHostMallocMapped) != hipSuccess) ok = false;
  if (ok && hipHostGetDevicePointer((void**)&ws.phase_dev, ws.phase_host, 0) != hipSuccess) ok = false;
  if (ok && hipStreamCreateWithFlags(&ws.aux, hipStreamNonBlocking) != hipSuccess) ok = false;
  if (ok && hipEventCreateWithFlags(&ws.ev_fork, hipEventDisableTiming) != hipSuccess) ok = false;
  if (ok && hipEventCreateWithFlags(&ws.ev_join, hipEventDisableTiming) != hipSuccess) ok = false;
  if (!ok) {
    slar_workspace_destroy(w);
    return SLAR_E_NOMEM;
  }
  std::vector<double> tw;
  for (int m = 0; m < G.dx; ++m) {
    host_twiddles(G.n[m], tw);
    if (hipMemcpy(ws.tw[m], tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice) != hipSuccess) {
      slar_workspace_destroy(w);
      return SLAR_E_HIP;
    }
  }
  if (psi_build(0, &ws) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    slar_workspace_destroy(w);
    return SLAR_E_HIP;
  }
  *out = w;
  return SLAR_OK;
}

slar_status slar_workspace_create(const slar_grid* g, int32_t rmax, slar_workspace** out) {
  if (!out || !grid_ok(g) || rmax < 1 || rmax > 64) return SLAR_E_INVAL;
  return ws_create(g, rmax, nullptr, 0, out);
}

slar_status slar_workspace_create_in(const slar_grid* g, int32_t rmax, void* work, size_t work_bytes,
                                     slar_workspace** out) {
  if (!out || !work || !grid_ok(g) || rmax < 1 || rmax > 64) return SLAR_E_INVAL;
  return ws_create(g, rmax, work, work_bytes, out);
}

slar_status slar_ht_sample(const slar_grid* g, const slar_ht* F, const slar_adv* a, int64_t n,
                           const int32_t* idx, void* out, hipStream_t stream) {
  if (!grid_ok(g) || !ht_ok(g, F) || !adv_ok(g, a) || n < 0) return SLAR_E_INVAL;
  if (n > 0 && (!idx || !out)) return SLAR_E_INVAL;
  if (a->kind == 2 && a->E[0] == nullptr) return SLAR_E_INVAL;
  if (F->d == 4 && a->order != 3) return SLAR_E_INVAL;
  if (n == 0) return SLAR_OK;
  GridDev G = make_grid(*g);
  // the two frozen fields are combined node by node inside the kernel
  AdvDev A{a->kind, a->order, a->tau, a->cv, a->E[0], a->E[1], a->cE[0], a->cE[1], 0};
  hipError_t e = ht_sample(stream, G, A, *F, n, idx, out);
  return e == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_frames_from_ht(const slar_grid* g, const slar_ht* F, slar_frames* out,
                                slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !ht_ok(g, F) || !out || !out->X || !out->P)
    return SLAR_E_INVAL;
  if (F->dtype != SLAR_F64) return SLAR_E_INVAL;
  const int need = F->d == 2 ? F->rank[0] : F->rank[4];
  if (out->ld < need) return SLAR_E_INVAL;
  return frames_from_ht(stream, &w->w, w->w.G, *F, out) == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_frame_sample(const slar_grid* g, const slar_frames* F, const slar_adv* a,
                              slar_dtype dtype, int64_t n, const int32_t* idx, double* out,
                              slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(F) || !adv_ok(g, a) || n < 0)
    return SLAR_E_INVAL;
  if (dtype != SLAR_F32 && dtype != SLAR_F64) return SLAR_E_INVAL;
  if (n > 0 && (!idx || !out)) return SLAR_E_INVAL;
  if (n == 0) return SLAR_OK;
  Workspace& ws = w->w;
  const GridDev& G = ws.G;
  const int ldt = (F->r + 3) & ~3;
  if (combine_field(stream, G, a, ws.Eeff) != hipSuccess) return SLAR_E_HIP;
  AdvDev A = make_adv(a, ws.Eeff);
  const void *X, *P;
  if (dtype == SLAR_F32) {
    if (table_copy(stream, G.nx, F->r, F->ld, F->X, ldt, ws.X32, nullptr) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(stream, G.nv, F->r, F->ld, F->P, ldt, ws.P32, nullptr) != hipSuccess) return SLAR_E_HIP;
    X = ws.X32; P = ws.P32;
  } else {
    double* X64 = ws.dwork;
    double* P64 = ws.dwork + (size_t)G.nx * ldt;
    if (table_copy(stream, G.nx, F->r, F->ld, F->X, ldt, nullptr, X64) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(stream, G.nv, F->r, F->ld, F->P, ldt, nullptr, P64) != hipSuccess) return SLAR_E_HIP;
    X = X64; P = P64;
  }
  return frame_points(stream, G, A, dtype, X, P, ldt, F->r, n, idx, out) == hipSuccess ? SLAR_OK
                                                                                        : SLAR_E_HIP;
}

slar_status slar_nested_cross(const slar_grid* g, const slar_frames* src, const slar_adv* a,
                              slar_dtype dtype, double tol, int32_t kmax, int32_t nprobe,
                              const int32_t* probes, const int32_t* seed, slar_ht* out,
                              slar_nested_info* info, slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(src) || !adv_ok(g, a))
    return SLAR_E_INVAL;
  const GridDev& G = w->w.G;
  if (G.d != 4 || a->order != 3 || (dtype != SLAR_F32 && dtype != SLAR_F64)) return SLAR_E_INVAL;
  if (!(tol > 0.0) || kmax < 1 || kmax > 64 || nprobe < 0 || nprobe > 1024) return SLAR_E_INVAL;
  if ((nprobe > 0 && !probes) || !seed || !out) return SLAR_E_INVAL;
  if (!out->leaf[0] || !out->leaf[1] || !out->leaf[2] || !out->leaf[3] || !out->B12 || !out->B34 ||
      !out->root)
    return SLAR_E_INVAL;
  for (int m = 0; m < 4; ++m)
    if (seed[m] < 0 || seed[m] >= G.n[m]) return SLAR_E_INVAL;
  for (int q = 0; q < nprobe; ++q)
    for (int m = 0; m < 4; ++m)
      if (probes[4 * q + m] < 0 || probes[4 * q + m] >= G.n[m]) return SLAR_E_INVAL;
  return nested_run(stream, &w->w, *src, *a, dtype, tol, kmax, nprobe, probes, seed, out, info);
}

slar_status slar_cross_update(const slar_grid* g, const slar_frames* src, const slar_adv* a,
                              slar_dtype dtype, double tol, int32_t kmax, int32_t nprobe,
                              const int32_t* probes, slar_lowrank* out, slar_cross_info* info,
                              slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(src) || !adv_ok(g, a))
    return SLAR_E_INVAL;
  if (!(tol > 0.0) || kmax < 1 || kmax > SLAR_CROSS_KMAX || nprobe < 0 || nprobe > 1024) return SLAR_E_INVAL;
  if (nprobe > 0 && !probes) return SLAR_E_INVAL;
  if (!out || !out->U || !out->V) return SLAR_E_INVAL;
  if (dtype != SLAR_F32 && dtype != SLAR_F64) return SLAR_E_INVAL;
  return cross_run(stream, &w->w, *src, *a, dtype, tol, kmax, nprobe, probes, out, info);
}

slar_status slar_truncate(const slar_grid* g, const slar_lowrank* in, double tol, int32_t rmax,
                          slar_ht* out, slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !in || !in->U || !in->V) return SLAR_E_INVAL;
  if (in->k < 1 || in->k > SLAR_CROSS_KMAX || !(tol > 0.0) || rmax < 1 || rmax > 64 || !out)
    return SLAR_E_INVAL;
  const int d = g->dx + g->dv;
  for (int m = 0; m < d; ++m)
    if (!out->leaf[m]) return SLAR_E_INVAL;
  if (!out->root || (d == 4 && (!out->B12 || !out->B34))) return SLAR_E_INVAL;
  return truncate_run(stream, &w->w, *in, tol, rmax, out);
}

slar_status slar_moments(const slar_grid* g, const slar_frames* F, double* M, slar_workspace* w,
                         hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(F) || !M) return SLAR_E_INVAL;
  return moments_run(stream, &w->w, *F, M) == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_poisson(const slar_grid* g, const double* n_e, double n_i, double* phi, double* E,
                         slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !n_e || !E || !std::isfinite(n_i))
    return SLAR_E_INVAL;
  return poisson_run(stream, &w->w, n_e, n_i, phi, E) == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_conserved(const slar_grid* g, const slar_frames* F, double n_i, double* U,
                           slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(F) || !U) return SLAR_E_INVAL;
  Workspace& ws = w->w;
  // moments into the Krylov scratch (free outside slar_macro_solve)
  double* Mtmp = ws.kry;
  if (moments_run(stream, &ws, *F, Mtmp) != hipSuccess) return SLAR_E_HIP;
  return conserved_from_moments(stream, &ws, Mtmp, n_i, U) == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_lomac_prepare(const slar_grid* g, const slar_ht* Fstar,
                               const slar_frames* Fstar_frames, double delta, double n_i,
                               slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !ht_ok(g, Fstar) || !frames_ok(Fstar_frames))
    return SLAR_E_INVAL;
  if (Fstar->dtype != SLAR_F64 || !(delta > 0.0) || !std::isfinite(n_i)) return SLAR_E_INVAL;
  return lomac_prepare_run(stream, &w->w, *Fstar, *Fstar_frames, delta, n_i);
}

slar_status slar_macro_solve(const slar_grid* g, const double* U_n, const double* U_nm1,
                             double dt, int32_t bdf_order, double newton_tol, double krylov_tol,
                             int32_t precond, const slar_cnn* cnn, double* U_out, int32_t* iters,
                             slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !U_n || !U_out) return SLAR_E_INVAL;
  if (!(dt > 0.0) || (bdf_order != 1 && bdf_order != 2) || !(newton_tol > 0.0) ||
      !(krylov_tol > 0.0 && krylov_tol < 1.0))
    return SLAR_E_INVAL;
  if (bdf_order == 2 && !U_nm1) return SLAR_E_INVAL;
  if (precond < 0 || precond > 2 || (precond == 2 && !cnn)) return SLAR_E_INVAL;
  MacroHist h{};
  double beta = dt;
  h.nh = 1; h.U[0] = U_n; h.c[0] = 1.0;
  if (bdf_order == 2) {
    h.nh = 2; h.c[0] = 4.0 / 3.0; h.U[1] = U_nm1; h.c[1] = -1.0 / 3.0;
    beta = 2.0 / 3.0 * dt;
  }
  return macro_solve_run(stream, &w->w, h, beta, newton_tol, krylov_tol, precond, cnn, U_out, iters);
}

slar_status slar_macro_solve_system(const slar_grid* g, const slar_macro_system* S,
                                    double newton_tol, double krylov_tol, int32_t precond,
                                    const slar_cnn* cnn, double* U_out, int32_t* iters,
                                    slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !S || !U_out) return SLAR_E_INVAL;
  if (S->nhist < 1 || S->nhist > 3 || S->nstage < 0 || S->nstage > 3) return SLAR_E_INVAL;
  if (!(S->beta > 0.0) || !std::isfinite(S->beta) || !(newton_tol > 0.0) ||
      !(krylov_tol > 0.0 && krylov_tol < 1.0))
    return SLAR_E_INVAL;
  if (precond < 0 || precond > 2 || (precond == 2 && !cnn)) return SLAR_E_INVAL;
  MacroHist h{};
  h.nh = S->nhist;
  h.nr = S->nstage;
  for (int j = 0; j < S->nhist; ++j) {
    if (!S->U[j] || !std::isfinite(S->c[j]) || S->U[j] == U_out) return SLAR_E_INVAL;
    h.U[j] = S->U[j]; h.c[j] = S->c[j];
  }
  for (int j = 0; j < S->nstage; ++j) {
    if (!S->R[j] || !std::isfinite(S->d[j]) || S->R[j] == U_out) return SLAR_E_INVAL;
    h.R[j] = S->R[j]; h.d[j] = S->d[j];
  }
  return macro_solve_run(stream, &w->w, h, S->beta, newton_tol, krylov_tol, precond, cnn, U_out, iters);
}

slar_status slar_macro_rhs(const slar_grid* g, const double* U, double* R_out, slar_workspace* w,
                           hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !U || !R_out || U == R_out) return SLAR_E_INVAL;
  if (!w->w.lm_ready) return SLAR_E_INVAL;
  return macro_rhs(stream, &w->w, U, R_out) == hipSuccess ? SLAR_OK : SLAR_E_HIP;
}

slar_status slar_cnn_correct(const slar_grid* g, const slar_cnn* cnn, const double* v, const double* U,
                             double* z, slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !cnn || !v || !U || !z) return SLAR_E_INVAL;
  if (z == v || z == U) return SLAR_E_INVAL;
  const hipError_t e = cnn_apply(stream, &w->w, cnn, v, U, z);
  return e == hipSuccess ? SLAR_OK : (e == hipErrorInvalidValue ? SLAR_E_INVAL : SLAR_E_HIP);
}

slar_status slar_dirk3_tableau(double* A, double* c) {
  if (!A || !c) return SLAR_E_INVAL;
  // gamma: the root in (1/6, 1/2) of p(x) = 6x^3 - 18x^2 + 9x - 1, by bisection
  // (p(1/6) = 1/36 > 0 > p(1/2) = -1/4 and p has one root there)
  double lo = 1.0 / 6.0, hi = 0.5;
  auto p = [](double x) { return ((6.0 * x - 18.0) * x + 9.0) * x - 1.0; };
  for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (p(mid) > 0.0) lo = mid; else hi = mid;
  }
  const double gm = 0.5 * (lo + hi);
  const double b1 = -(6.0 * gm * gm - 16.0 * gm + 1.0) / 4.0;
  const double b2 = (6.0 * gm * gm - 20.0 * gm + 5.0) / 4.0;
  const double T[9] = {gm, 0.0, 0.0, (1.0 - gm) / 2.0, gm, 0.0, b1, b2, gm};
  for (int i = 0; i < 9; ++i) A[i] = T[i];
  c[0] = gm; c[1] = (1.0 + gm) / 2.0; c[2] = 1.0;
  return SLAR_OK;
}

slar_status slar_bdf_weights(int32_t k, const double* t, double* c, double* beta) {
  if (k < 1 || k > 3 || !t || !c || !beta) return SLAR_E_INVAL;
  for (int j = 0; j < k; ++j)
    if (!(t[j] > t[j + 1]) || !std::isfinite(t[j]) || !std::isfinite(t[j + 1])) return SLAR_E_INVAL;
  double l0 = 0.0;
  for (int m = 1; m <= k; ++m) l0 += 1.0 / (t[0] - t[m]);
  for (int j = 1; j <= k; ++j) {
    double num = 1.0, den = 1.0;
    for (int m = 1; m <= k; ++m)
      if (m != j) num *= t[0] - t[m];
    for (int m = 0; m <= k; ++m)
      if (m != j) den *= t[j] - t[m];
    c[j - 1] = -(num / den) / l0;
  }
  *beta = 1.0 / l0;
  return SLAR_OK;
}

slar_status slar_poisson_noalloc(const slar_grid* g, const double* n_e, double n_i, double* phi,
                                 double* E, hipStream_t stream) {
  if (!grid_ok(g) || !n_e || !E || !std::isfinite(n_i)) return SLAR_E_INVAL;
  return poisson_noalloc_run(stream, *g, n_e, n_i, phi, E);
}

slar_status slar_lomac_filter(const slar_grid* g, double* U, slar_workspace* w, hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !U) return SLAR_E_INVAL;
  return lomac_filter_run(stream, &w->w, U);
}

slar_status slar_lomac_project(const slar_grid* g, const slar_frames* Fstar_frames,
                               const double* U_new, slar_frames* out, slar_workspace* w,
                               hipStream_t stream) {
  if (!w || !grid_ok(g) || !same_grid(g, &w->w.grid) || !frames_ok(Fstar_frames) || !U_new || !out ||
      !out->X || !out->P)
    return SLAR_E_INVAL;
  if (out->ld < Fstar_frames->r + g->dv + 2 || Fstar_frames->r + g->dv + 2 > SLAR_KMAX) return SLAR_E_INVAL;
  return lomac_project_run(stream, &w->w, *Fstar_frames, U_new, out);
}

slar_status slar_leaf_refine(slar_workspace* w, int32_t on) {
  if (!w || (on != 0 && on != 1)) return SLAR_E_INVAL;
  w->w.leaf_refine = on != 0;
  return SLAR_OK;
}

slar_status slar_timing_enable(slar_workspace* w, int32_t on) {
  if (!w) return SLAR_E_INVAL;
  Workspace& ws = w->w;
  if (on && ws.events.empty()) {
    const int need = 4 * (SLAR_CROSS_KMAX + 64);
    ws.events.resize(need);
    for (int i = 0; i < need; ++i)
      if (hipEventCreate(&ws.events[i]) != hipSuccess) {
        ws.events.resize(i);
        return SLAR_E_HIP;
      }
  }
  if (on < 0) return SLAR_E_INVAL;
  ws.timing = on != 0;
  ws.timing_every = on > 0 ? on : 1;
  for (double& v : ws.tstat) v = 0.0;
  return SLAR_OK;
}

slar_status slar_timing_read(const slar_workspace* w, double* out /* host [8] */) {
  if (!w || !out) return SLAR_E_INVAL;
  for (int i = 0; i < 8; ++i) out[i] = w->w.tstat[i];
  return SLAR_OK;
}

int32_t slar_macro_history(const slar_workspace* w, double* out, int32_t cap) {
  if (!w || (!out && cap > 0) || cap < 0) return -1;
  const int n = std::min(w->w.newton_hist_n, (int)cap);
  for (int i = 0; i < 4 * n; ++i) out[i] = w->w.newton_hist[i];
  return w->w.newton_hist_n;
}

int32_t slar_macro_fallbacks(const slar_workspace* w, int32_t* last) {
  if (!w) return -1;
  if (last) *last = w->w.macro_fell_back ? 1 : 0;
  return w->w.macro_fallbacks;
}

}  // extern "C"
