// Many independent Vlasov--Poisson instances of uneven grid size and rank
// advanced together.
//
// Cross approximation: one persistent launch per phase serves every
// instance.  A fixed grid walks a table of work items (instance, first
// fiber tile, tile count); each instance keeps its own control block and
// partial-sum slots, so the per-tile arithmetic and the pivot decisions are
// those of the one-instance kernels, whatever block runs a tile.  A chunk of
// iterations (row and column launches) plus an active-instance
// count is captured once as a hipGraph and replayed until no instance runs.
//
// The autotuner times whole batched cross approximations on the caller's
// inputs and picks the persistent grid size, the tiles per work item, the
// iterations per graph chunk, and the gather team width per rank bucket.
//
// Truncation, frames and field solves: every step one grouped launch over
// all instances on the caller stream (group.h); the truncation takes the
// rank decisions of all instances after one gathered read of their
// singular values and one of their eigenvalues.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "batch_kernels.h"
#include "fields.h"
#include "group.h"
#include "truncate.h"


using namespace slar;

struct slar_batch {
  int count = 0;
  int device = 0;
  int rmax = 0;
  std::vector<slar_workspace*> ws;
  std::vector<int> nbrow, nbcol, order;   // order: instances by decreasing work
  // device tables
  AcaInst* d_inst = nullptr;
  AcaInst* h_inst = nullptr;       // pinned
  BPrep* d_prep = nullptr;
  BPrep* h_prep = nullptr;         // pinned
  BItem* d_rows = nullptr;
  BItem* d_cols = nullptr;
  int nrow_items = 0, ncol_items = 0;
  int* d_active = nullptr;
  int* h_active = nullptr;         // pinned
  BSummary* d_sum = nullptr;
  BSummary* h_sum = nullptr;       // pinned
  // launch configuration (autotuned)
  int grid = 1024, group = 1, chunk = 8;
  int team[3] = {16, 16, 16};      // rank buckets r <= 16, r <= 32, r > 32
  // captured iteration chunk
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int captured_grid = -1, captured_group = -1, captured_chunk = -1;
  int captures = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double tstat[4] = {0, 0, 0, 0};  // cross ms, chunks, iterations (max over instances), calls
  // grouped truncation and skeleton cores: descriptors and gathered values
  // (device, pinned mirror); both synchronise before they return
  void* d_tg = nullptr;
  void* h_tg = nullptr;
  // grouped field solves (asynchronous): their own staging, reusable once
  // ev_fg (recorded after the upload) has completed
  void* d_fg = nullptr;
  void* h_fg = nullptr;
  size_t fg_bytes = 0;
  hipEvent_t ev_fg = nullptr;
};

static int bucket_of(int r) { return r <= 16 ? 0 : (r <= 32 ? 1 : 2); }

static hipError_t build_items(slar_batch* b) {
  std::vector<BItem> rows, cols;
  for (int q : b->order) {
    for (int t = 0; t < b->nbrow[q]; t += b->group) rows.push_back({q, t, std::min(b->group, b->nbrow[q] - t), 0});
    for (int t = 0; t < b->nbcol[q]; t += b->group) cols.push_back({q, t, std::min(b->group, b->nbcol[q] - t), 0});
  }
  if (b->d_rows) { HIP_CHK(hipFree(b->d_rows)); b->d_rows = nullptr; }
  if (b->d_cols) { HIP_CHK(hipFree(b->d_cols)); b->d_cols = nullptr; }
  HIP_CHK(hipMalloc((void**)&b->d_rows, sizeof(BItem) * rows.size()));
  HIP_CHK(hipMalloc((void**)&b->d_cols, sizeof(BItem) * cols.size()));
  HIP_CHK(hipMemcpy(b->d_rows, rows.data(), sizeof(BItem) * rows.size(), hipMemcpyHostToDevice));
  HIP_CHK(hipMemcpy(b->d_cols, cols.data(), sizeof(BItem) * cols.size(), hipMemcpyHostToDevice));
  b->nrow_items = (int)rows.size();
  b->ncol_items = (int)cols.size();
  return hipSuccess;
}

// Capture `chunk` iterations of the two batched launches plus the count of
// running instances.  Kernel arguments are the batch's own device tables, so
// one capture serves every later call with the same configuration.
static hipError_t capture_chunk(slar_batch* b) {
  if (b->exec) { HIP_CHK(hipGraphExecDestroy(b->exec)); b->exec = nullptr; }
  if (b->graph) { HIP_CHK(hipGraphDestroy(b->graph)); b->graph = nullptr; }
  HIP_CHK(build_items(b));
  HIP_CHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  for (int it = 0; it < b->chunk; ++it) {
    k_batch_row<<<std::min(b->grid, b->nrow_items), FS_THREADS, 0, b->cap>>>(b->d_inst, b->d_rows, b->nrow_items);
    k_batch_col<<<std::min(b->grid, b->ncol_items), FS_THREADS, 0, b->cap>>>(b->d_inst, b->d_cols, b->ncol_items);
  }
  k_batch_status<<<1, 256, 0, b->cap>>>(b->d_inst, b->count, b->d_active, nullptr);
  const hipError_t le = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
  if (le != hipSuccess) return le;
  if (ce != hipSuccess) return ce;
  HIP_CHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->captured_grid = b->grid;
  b->captured_group = b->group;
  b->captured_chunk = b->chunk;
  b->captures += 1;
  return hipSuccess;
}

static slar_status batch_cross(slar_batch* b, const slar_frames* src, const slar_adv* adv, double tol,
                               int kmax, int nprobe, const int32_t* const* probes, slar_lowrank* out,
                               slar_cross_info* info, hipStream_t s) {
  if (b->grid != b->captured_grid || b->group != b->captured_group || b->chunk != b->captured_chunk)
    if (capture_chunk(b) != hipSuccess) return SLAR_E_HIP;
  for (int q = 0; q < b->count; ++q) {
    Workspace& w = b->ws[q]->w;
    const int r = src[q].r, ldt = (r + 3) & ~3;
    const slar_adv& a = adv[q];
    BPrep& p = b->h_prep[q];
    p.X = src[q].X; p.P = src[q].P; p.ldin = src[q].ld; p.r = r; p.ldt = ldt;
    p.nx = w.G.nx; p.nv = w.G.nv; p.dx = w.G.dx;
    p.X32 = w.X32; p.P32 = w.P32;
    p.E0 = a.E[0]; p.E1 = a.E[0] ? a.E[1] : nullptr; p.c0 = a.cE[0]; p.c1 = a.cE[1];
    p.Eeff = w.Eeff; p.used = w.used; p.ctl = (AcaCtl*)w.aca_ctl; p.kmax = kmax; p.tol = tol;
    AcaInst& I = b->h_inst[q];
    I.g = w.G;
    I.a = AdvDev{a.kind, a.order, a.tau, a.cv, w.Eeff, nullptr, 1.0, 0.0, 1};
    I.X = w.X32; I.P = w.P32; I.ld = ldt; I.r = r;
    I.ctl = (AcaCtl*)w.aca_ctl; I.U = out[q].U; I.V = out[q].V; I.used = w.used;
    I.part = w.aca_part; I.nbrow = b->nbrow[q]; I.nbcol = b->nbcol[q];
    I.piv = w.aca_piv;
    I.nprobe = nprobe; I.team = b->team[bucket_of(r)];
    I.probes = nprobe > 0 ? probes[q] : nullptr;
  }
  HIP_TRY(hipMemcpyAsync(b->d_prep, b->h_prep, sizeof(BPrep) * b->count, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->d_inst, b->h_inst, sizeof(AcaInst) * b->count, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(b->ev0, s));
  k_batch_prep<<<dim3(64, b->count), 256, 0, s>>>(b->d_prep);
  HIP_TRY(hipGetLastError());
  const int maxit = kmax + 64;
  int chunks = 0;
  for (int it = 0; it < maxit; it += b->chunk) {
    HIP_TRY(hipGraphLaunch(b->exec, s));
    ++chunks;
    HIP_TRY(hipMemcpyAsync(b->h_active, b->d_active, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*b->h_active == 0) break;
  }
  HIP_TRY(hipEventRecord(b->ev1, s));
  k_batch_status<<<1, 256, 0, s>>>(b->d_inst, b->count, b->d_active, b->d_sum);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(b->h_sum, b->d_sum, sizeof(BSummary) * b->count, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  int maxiters = 0;
  slar_status st = SLAR_OK;
  for (int q = 0; q < b->count; ++q) {
    const BSummary& m = b->h_sum[q];
    out[q].k = m.k;
    maxiters = std::max(maxiters, m.iters);
    if (info) {
      info[q].rank = m.k; info[q].iterations = m.iters; info[q].probe_rounds = m.probe_rounds;
      info[q].converged = m.converged; info[q].samples = m.samples;
    }
    if (!std::isfinite(m.norm2)) st = SLAR_E_NUMERIC;
    else if ((m.capped || m.phase != ACA_DONE) && st == SLAR_OK) st = SLAR_E_RANK_CAP;
  }
  // instances stopped at the term cap: regularised skeleton (as
  // slar_cross_update), their pivot-block SVDs grouped
  if (st != SLAR_E_NUMERIC) {
    std::vector<Workspace*> cws;
    std::vector<slar_lowrank*> cout;
    std::vector<int> cq, ccap;
    for (int q = 0; q < b->count; ++q) {
      const BSummary& m = b->h_sum[q];
      if ((m.capped || m.phase != ACA_DONE) && out[q].k > b->rmax) {
        cws.push_back(&b->ws[q]->w);
        cout.push_back(&out[q]);
        cq.push_back(q);
        ccap.push_back(b->rmax);
      }
    }
    std::vector<slar_status> cst(cq.size(), SLAR_OK);
    const slar_status e = cur_core_group(s, (int)cq.size(), cws.data(), cout.data(), ccap.data(), cst.data(),
                                         b->d_tg, b->h_tg);
    if (e != SLAR_OK) return e;
    for (size_t j = 0; j < cq.size(); ++j) {
      if (cst[j] != SLAR_OK) return cst[j];
      if (info) info[cq[j]].rank = out[cq[j]].k;
    }
  }
  b->tstat[0] += ms; b->tstat[1] += chunks; b->tstat[2] += maxiters; b->tstat[3] += 1;
  return st;
}

static bool batch_frames_ok(const slar_batch* b, const slar_frames* F) {
  for (int q = 0; q < b->count; ++q) {
    const slar_frames& f = F[q];
    if (!f.X || !f.P || f.r < 1 || f.r > SLAR_KMAX || f.ld < f.r) return false;
  }
  return true;
}

// most severe status first; a capped rank is reported but not fatal
static slar_status worst_of(const std::vector<slar_status>& st) {
  static const slar_status sev[] = {SLAR_E_HIP, SLAR_E_NUMERIC, SLAR_E_NOMEM, SLAR_E_INVAL,
                                    SLAR_E_NOCONV, SLAR_E_RANK_CAP};
  for (slar_status c : sev)
    if (std::find(st.begin(), st.end(), c) != st.end()) return c;
  return SLAR_OK;
}


extern "C" {

slar_status slar_batch_destroy(slar_batch* b) {
  if (!b) return SLAR_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_fg) (void)hipEventSynchronize(b->ev_fg);
  for (hipEvent_t e : {b->ev0, b->ev1, b->ev_fg})
    if (e) (void)hipEventDestroy(e);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void* p : {(void*)b->d_inst, (void*)b->d_prep, (void*)b->d_rows, (void*)b->d_cols,
                  (void*)b->d_active, (void*)b->d_sum, b->d_tg, b->d_fg})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)b->h_inst, (void*)b->h_prep, (void*)b->h_active, (void*)b->h_sum, b->h_tg, b->h_fg})
    if (p) (void)hipHostFree(p);
  for (slar_workspace* w : b->ws) slar_workspace_destroy(w);
  delete b;
  return SLAR_OK;
}

slar_status slar_batch_create(int32_t count, const slar_grid* grids, int32_t rmax, slar_batch** out) {
  if (!out || !grids || count < 1 || count > 4096 || rmax < 1 || rmax > 64) return SLAR_E_INVAL;
  *out = nullptr;
  for (int q = 0; q < count; ++q) {
    const slar_grid& g = grids[q];
    if (g.dx != g.dv || (g.dx != 1 && g.dx != 2)) return SLAR_E_INVAL;
  }
  slar_batch* b = new (std::nothrow) slar_batch();
  if (!b) return SLAR_E_NOMEM;
  b->count = count;
  b->rmax = rmax;
  b->ws.assign(count, nullptr);
  auto fail = [&](slar_status st) { slar_batch_destroy(b); return st; };
  if (hipGetDevice(&b->device) != hipSuccess) return fail(SLAR_E_HIP);
  for (int q = 0; q < count; ++q) {
    const slar_status st = slar_workspace_create(&grids[q], rmax, &b->ws[q]);
    if (st != SLAR_OK) return fail(st);
    b->ws[q]->w.fork_aux = false;
    const GridDev& G = b->ws[q]->w.G;
    b->nbrow.push_back((G.nv + ACA_TILE - 1) / ACA_TILE);
    b->nbcol.push_back((G.nx + ACA_TILE - 1) / ACA_TILE);
  }
  // largest sampling work first: stencil rows x fiber lengths
  b->order.resize(count);
  for (int q = 0; q < count; ++q) b->order[q] = q;
  auto work = [&](int q) {
    const GridDev& G = b->ws[q]->w.G;
    return (double)(G.dx == 2 ? 9 : 3) * ((double)G.nx + (double)G.nv);
  };
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return work(a) > work(c); });
  bool ok = true;
  auto dal = [&](void** p, size_t n) { if (ok && hipMalloc(p, std::max(n, (size_t)256)) != hipSuccess) ok = false; };
  auto hal = [&](void** p, size_t n) { if (ok && hipHostMalloc(p, std::max(n, (size_t)256), 0) != hipSuccess) ok = false; };
  dal((void**)&b->d_inst, sizeof(AcaInst) * count);
  dal((void**)&b->d_prep, sizeof(BPrep) * count);
  dal((void**)&b->d_active, sizeof(int));
  dal((void**)&b->d_sum, sizeof(BSummary) * count);
  hal((void**)&b->h_inst, sizeof(AcaInst) * count);
  hal((void**)&b->h_prep, sizeof(BPrep) * count);
  hal((void**)&b->h_active, sizeof(int));
  hal((void**)&b->h_sum, sizeof(BSummary) * count);
  // shared by the grouped truncation and the grouped skeleton cores (never
  // in use at the same time: each returns after synchronising)
  const size_t tg = std::max(truncate_group_bytes(count), cur_core_group_bytes(count));
  dal(&b->d_tg, tg);
  hal(&b->h_tg, tg);
  b->fg_bytes = (size_t)64 * 1024 + (size_t)count * 4096;
  dal(&b->d_fg, b->fg_bytes);
  hal(&b->h_fg, b->fg_bytes);
  if (!ok) return fail(SLAR_E_NOMEM);
  std::memset(b->h_inst, 0, sizeof(AcaInst) * count);
  if (hipMemcpy(b->d_inst, b->h_inst, sizeof(AcaInst) * count, hipMemcpyHostToDevice) != hipSuccess)
    return fail(SLAR_E_HIP);
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return fail(SLAR_E_HIP);
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fg, hipEventDisableTiming) != hipSuccess)
    return fail(SLAR_E_HIP);
  *out = b;
  return SLAR_OK;
}

slar_workspace* slar_batch_workspace(slar_batch* b, int32_t q) {
  if (!b || q < 0 || q >= b->count) return nullptr;
  return b->ws[q];
}

slar_status slar_batch_cross_update(slar_batch* b, const slar_frames* src, const slar_adv* adv,
                                    double tol, int32_t kmax, int32_t nprobe,
                                    const int32_t* const* probes, slar_lowrank* out,
                                    slar_cross_info* info, hipStream_t stream) {
  if (!b || !src || !adv || !out || !batch_frames_ok(b, src)) return SLAR_E_INVAL;
  if (!(tol > 0.0) || kmax < 1 || kmax > SLAR_CROSS_KMAX || nprobe < 0 || nprobe > 1024) return SLAR_E_INVAL;
  if (nprobe > 0 && !probes) return SLAR_E_INVAL;
  for (int q = 0; q < b->count; ++q) {
    const slar_adv& a = adv[q];
    if (a.kind < 0 || a.kind > 2 || a.order != 3 || !std::isfinite(a.tau) || !std::isfinite(a.cv))
      return SLAR_E_INVAL;
    if (a.kind != 0 && a.E[0] == nullptr) return SLAR_E_INVAL;
    if (!out[q].U || !out[q].V) return SLAR_E_INVAL;
    if (nprobe > 0 && !probes[q]) return SLAR_E_INVAL;
  }
  return batch_cross(b, src, adv, tol, kmax, nprobe, probes, out, info, stream);
}

slar_status slar_batch_truncate(slar_batch* b, const slar_lowrank* in, double tol, int32_t rmax,
                                slar_ht* out, slar_frames* frames, int32_t* status,
                                hipStream_t stream) {
  if (!b || !in || !out || !(tol > 0.0) || rmax < 1 || rmax > 64) return SLAR_E_INVAL;
  for (int q = 0; q < b->count; ++q) {
    const Workspace& w = b->ws[q]->w;
    if (!in[q].U || !in[q].V || in[q].k < 1 || in[q].k > SLAR_CROSS_KMAX) return SLAR_E_INVAL;
    const int d = w.G.d;
    if (out[q].d != d) return SLAR_E_INVAL;
    for (int m = 0; m < d; ++m)
      if (!out[q].leaf[m]) return SLAR_E_INVAL;
    if (!out[q].root || (d == 4 && (!out[q].B12 || !out[q].B34))) return SLAR_E_INVAL;
    if (frames && (!frames[q].X || !frames[q].P || frames[q].ld < rmax)) return SLAR_E_INVAL;
  }
  std::vector<TruncJob> jobs(b->count);
  for (int q = 0; q < b->count; ++q) {
    jobs[q].ws = &b->ws[q]->w;
    jobs[q].in = in[q];
    jobs[q].out = &out[q];
    jobs[q].frames = frames ? &frames[q] : nullptr;
  }
  // every step one grouped launch over all instances, on the caller stream
  const slar_status e = truncate_group(stream, jobs, tol, rmax, b->d_tg, b->h_tg);
  if (e != SLAR_OK) return e;
  std::vector<slar_status> st(b->count);
  for (int q = 0; q < b->count; ++q) st[q] = jobs[q].st;
  if (status)
    for (int q = 0; q < b->count; ++q) status[q] = st[q];
  return worst_of(st);
}

slar_status slar_batch_efield(slar_batch* b, const slar_frames* F, const double* n_i,
                              double* const* M, double* const* E, hipStream_t stream) {
  if (!b || !F || !n_i || !M || !E || !batch_frames_ok(b, F)) return SLAR_E_INVAL;
  for (int q = 0; q < b->count; ++q)
    if (!M[q] || !E[q]) return SLAR_E_INVAL;
  // every step one grouped launch over all instances, on the caller stream
  if (hipEventSynchronize(b->ev_fg) != hipSuccess) return SLAR_E_HIP;   // staging free again
  std::vector<Workspace*> ws(b->count);
  for (int q = 0; q < b->count; ++q) ws[q] = &b->ws[q]->w;
  GroupQueue gq(b->d_fg, b->h_fg, b->fg_bytes);
  if (efield_group(gq, b->count, ws.data(), F, n_i, M, E) != hipSuccess) return SLAR_E_HIP;
  if (gq.flush(stream) != hipSuccess) return SLAR_E_HIP;
  if (hipEventRecord(b->ev_fg, stream) != hipSuccess) return SLAR_E_HIP;
  return SLAR_OK;
}

slar_status slar_batch_get_config(const slar_batch* b, int32_t* cfg) {
  if (!b || !cfg) return SLAR_E_INVAL;
  cfg[0] = b->grid; cfg[1] = b->group; cfg[2] = b->chunk;
  cfg[3] = b->team[0]; cfg[4] = b->team[1]; cfg[5] = b->team[2];
  cfg[6] = b->captures; cfg[7] = 0;
  return SLAR_OK;
}

slar_status slar_batch_set_config(slar_batch* b, const int32_t* cfg) {
  if (!b || !cfg) return SLAR_E_INVAL;
  if (cfg[0] < 1 || cfg[0] > 65536 || cfg[1] < 1 || cfg[1] > 16 || cfg[2] < 1 || cfg[2] > 64)
    return SLAR_E_INVAL;
  for (int k = 3; k < 6; ++k)
    if (cfg[k] != 4 && cfg[k] != 8 && cfg[k] != 16) return SLAR_E_INVAL;
  b->grid = cfg[0]; b->group = cfg[1]; b->chunk = cfg[2];
  b->team[0] = cfg[3]; b->team[1] = cfg[4]; b->team[2] = cfg[5];
  return SLAR_OK;
}

slar_status slar_batch_tune(slar_batch* b, const slar_frames* src, const slar_adv* adv, double tol,
                            int32_t kmax, int32_t nprobe, const int32_t* const* probes,
                            slar_lowrank* out, int32_t reps, hipStream_t stream) {
  if (!b || reps < 1 || reps > 100) return SLAR_E_INVAL;
  int32_t best[8];
  slar_batch_get_config(b, best);
  // one candidate: its best wall time over reps full batched cross runs
  auto measure = [&](const int32_t* cfg, double* t) -> slar_status {
    slar_status st = slar_batch_set_config(b, cfg);
    if (st != SLAR_OK) return st;
    *t = 1e30;
    for (int r = 0; r < reps; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      st = slar_batch_cross_update(b, src, adv, tol, kmax, nprobe, probes, out, nullptr, stream);
      if (st != SLAR_OK && st != SLAR_E_RANK_CAP) return st;
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      *t = std::min(*t, dt);
    }
    return SLAR_OK;
  };
  bool used_bucket[3] = {false, false, false};
  for (int q = 0; q < b->count; ++q) used_bucket[bucket_of(src[q].r)] = true;
  double tbest;
  slar_status st = measure(best, &tbest);
  if (st != SLAR_OK) return st;
  auto sweep = [&](int slot, std::initializer_list<int> values) -> slar_status {
    for (int v : values) {
      if (v == best[slot]) continue;
      int32_t cfg[8];
      std::copy(best, best + 8, cfg);
      cfg[slot] = v;
      double t;
      const slar_status s2 = measure(cfg, &t);
      if (s2 != SLAR_OK) return s2;
      if (t < tbest) { tbest = t; best[slot] = v; }
    }
    return SLAR_OK;
  };
  if ((st = sweep(0, {256, 512, 1024, 2048, 4096})) != SLAR_OK) return st;
  if ((st = sweep(1, {1, 2, 4})) != SLAR_OK) return st;
  for (int k = 0; k < 3; ++k)
    if (used_bucket[k] && (st = sweep(3 + k, {4, 8, 16})) != SLAR_OK) return st;
  if ((st = sweep(2, {4, 8, 16})) != SLAR_OK) return st;
  return slar_batch_set_config(b, best);
}

slar_status slar_batch_timing(const slar_batch* b, double* out) {
  if (!b || !out) return SLAR_E_INVAL;
  for (int k = 0; k < 4; ++k) out[k] = b->tstat[k];
  return SLAR_OK;
}

slar_status slar_batch_timing_reset(slar_batch* b) {
  if (!b) return SLAR_E_INVAL;
  for (int k = 0; k < 4; ++k) b->tstat[k] = 0.0;
  return SLAR_OK;
}

}  // extern "C"
