// Nested hierarchical-Tucker cross approximation of the SL-updated tensor
// on the tree {{x1,x2},{v1,v2}} (the cheaper cross sampler that sections 4
// and 5 ask for; nested skeleton after Ballani, Grasedyck and Kluge).
//
// Every leaf and root search is the device-resident cross approximation of
// cross.hip (row and column launches, partial pivoting, tie
// rule, probe restart) in index-table mode: the searched matrix is
// A^(mu)[:, candidates] or A[rows_x, rows_v], and a matrix entry is the grid
// point whose multi-index joins the two table entries.  Between searches
// the host only builds the integer tables (unions of pivot sets, the
// enrichment probes).  The skeleton is then assembled on the device:
//   leaves     W_mu = A^(mu)[:, Q_mu] A^(mu)[R_mu, Q_mu]^-1
//   transfers  B12[a, b, d] = A[R1[a], R2[b], Pv[d]],  B34[p, q, c] = A[Px[c], R3[p], R4[q]]
//   root       A[Px, Pv]^-1
// and checked at the probes against tol ||F||_F / sqrt(Nx Nv).
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include <hip/hip_ext.h>

#include "aca.h"
#include "dense.h"
#include "fields.h"

namespace slar {

hipError_t table_copy(hipStream_t s, int rows, int r, int ldin, const double* in, int ldo,
                      float* o32, double* o64);
hipError_t frame_points(hipStream_t s, const GridDev& G, const AdvDev& A, slar_dtype dt,
                        const void* X, const void* P, int ld, int r, long long n, const int* idx,
                        double* out);
hipError_t ht_sample(hipStream_t st, const GridDev& G, const AdvDev& A, const slar_ht& F,
                     long long n, const int* idx, void* out);
hipError_t frames_from_ht(hipStream_t s, Workspace* ws, const GridDev& G, const slar_ht& F,
                          slar_frames* out);

constexpr int NEST_TAB = FIN_NB * ACA_TILE;   // longest searched row / column
static_assert(NEST_TAB >= 69 * 69, "candidate tables of rank 64 plus enrichment fit");

size_t nest_list_elems() { return (size_t)SLAR_KMAX * SLAR_KMAX * SLAR_KMAX; }

// ------------------------------------------------- small dense inverse
// Minv = M^-1 (r x r, r <= 64, row-major) by Gauss-Jordan elimination with
// partial pivoting (largest |entry| in the column, lowest row on ties), in
// LDS, one block of 256 threads.  *sing is set when a pivot is zero.
__global__ __launch_bounds__(256) void k_gj_inverse(int r, const double* __restrict__ M,
                                                    double* __restrict__ Minv, int* __restrict__ sing) {
  __shared__ double a[64][129];
  __shared__ double s_piv;
  __shared__ int s_p;
  const int t = threadIdx.x;
  for (int e = t; e < r * 2 * r; e += blockDim.x) {
    const int i = e / (2 * r), j = e % (2 * r);
    a[i][j] = j < r ? M[i * r + j] : (j - r == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int c = 0; c < r; ++c) {
    if (t < 64) {
      double m = -1.0;
      int mi = r;
      for (int i = c + t; i < r; i += 64)
        if (fabs(a[i][c]) > m) { m = fabs(a[i][c]); mi = i; }
      for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, 64);
        const int i2 = __shfl_xor(mi, o, 64);
        if (m2 > m || (m2 == m && i2 < mi)) { m = m2; mi = i2; }
      }
      if (t == 0) { s_p = mi; s_piv = a[mi][c]; }
    }
    __syncthreads();
    const int p = s_p;
    const double piv = s_piv;
    if (piv == 0.0) {
      if (t == 0) *sing = 1;
      return;   // uniform: every thread read the same pivot
    }
    if (p != c)
      for (int j = t; j < 2 * r; j += blockDim.x) {
        const double x = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = x;
      }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int j = t; j < 2 * r; j += blockDim.x) a[c][j] *= inv;
    __syncthreads();
    // eliminate column c from the other rows; column c itself holds the
    // multipliers every thread reads, so it is cleared after a barrier
    for (int e = t; e < r * 2 * r; e += blockDim.x) {
      const int i = e / (2 * r), j = e % (2 * r);
      if (i != c && j != c) a[i][j] -= a[i][c] * a[c][j];
    }
    __syncthreads();
    for (int i = t; i < r; i += blockDim.x)
      if (i != c) a[i][c] = 0.0;
    __syncthreads();
  }
  for (int e = t; e < r * r; e += blockDim.x) Minv[e] = a[e / r][r + e % r];
}

// out[0] = number of probes with |approx - truth| > tol ||F|| / sqrt(NxNv),
// out[1] = the first of those with the largest error.  ||F||^2 =
// trace(G_X G_P) with the Gram matrices of the two frames (k x k).
__global__ __launch_bounds__(256) void k_nest_probe(int np, const double* __restrict__ approx,
                                                    const double* __restrict__ truth, int k,
                                                    const double* __restrict__ GX,
                                                    const double* __restrict__ GP, double tol,
                                                    double nxnv, int* __restrict__ out) {
  __shared__ double red[4];
  __shared__ int redi[4];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int e = t; e < k * k; e += blockDim.x) s += GX[e] * GP[(e % k) * k + e / k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  const double norm2 = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  const double thr = tol * sqrt(fmax(norm2, 0.0)) / sqrt(nxnv);
  double m = -1.0;
  int nb = 0;
  for (int e = t; e < np; e += blockDim.x) {
    const double err = fabs(approx[e] - truth[e]);
    if (err > thr) { ++nb; m = fmax(m, err); }
  }
  const double M = block_max(m, red);
  int cnt = nb;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  int best = np;
  if (M > 0.0)
    for (int e = t; e < np; e += blockDim.x) {
      const double err = fabs(approx[e] - truth[e]);
      if (err > thr && err == M) { best = e; break; }
    }
  for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((t & 63) == 0) { redi[t >> 6] = best; red[t >> 6] = (double)cnt; }
  __syncthreads();
  if (t == 0) {
    out[0] = (int)(((red[0] + red[1]) + red[2]) + red[3]);
    out[1] = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  }
}

// -------------------------------------------------------- host driver
using Idx4 = std::array<int, 4>;
using Pair = std::array<int, 2>;

template <typename V>
static void add_unique(std::vector<V>& a, const V& x) {
  if (std::find(a.begin(), a.end(), x) == a.end()) a.push_back(x);
}

struct NestCtx {
  hipStream_t s;
  Workspace* ws;
  const GridDev* G;
  AdvDev A;
  slar_dtype dt;
  const void* X;
  const void* P;
  int ldt, r;
};

// one device-resident cross search in index-table mode; returns the
// accepted pivots (row, col) in order
template <typename T>
static slar_status nest_search(const NestCtx& c, const std::vector<Idx4>& rowtab,
                               const std::vector<Idx4>& coltab, double tol, int kmax, int first_row,
                               const std::vector<Pair>& probes, std::vector<Pair>* piv) {
  Workspace* ws = c.ws;
  const int nrows = (int)rowtab.size(), ncols = (int)coltab.size();
  if (nrows < 1 || ncols < 1 || nrows > NEST_TAB || ncols > NEST_TAB) return SLAR_E_INVAL;
  const int np = (int)std::min<size_t>(probes.size(), 128);
  const hipStream_t s = c.s;
  HIP_TRY(hipMemcpyAsync(ws->nest_rowtab, rowtab.data(), sizeof(Idx4) * nrows, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws->nest_coltab, coltab.data(), sizeof(Idx4) * ncols, hipMemcpyHostToDevice, s));
  if (np > 0)
    HIP_TRY(hipMemcpyAsync(ws->nest_probes, probes.data(), sizeof(Pair) * np, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(ws->nest_used, 0, nrows, s));
  AcaCtl h{};
  h.phase = ACA_RUN; h.k = 0; h.i = first_row; h.j = 0; h.kmax = kmax; h.tol = tol; h.norm2 = 0.0;
  AcaCtl* ctl = (AcaCtl*)ws->aca_ctl;
  AcaCtl* hc = (AcaCtl*)ws->aca_ctl_host;
  *hc = h;
  HIP_TRY(hipMemcpyAsync(ctl, hc, sizeof(AcaCtl), hipMemcpyHostToDevice, s));
  const unsigned bRow = (ncols + ACA_TILE - 1) / ACA_TILE;
  const unsigned bCol = (nrows + ACA_TILE - 1) / ACA_TILE;
  AcaInst I{*c.G, c.A, c.X, c.P, c.ldt, c.r, ctl, ws->nest_U, ws->nest_V, ws->nest_used,
            ws->aca_part, (int)bRow, (int)bCol, np, 16, ws->nest_probes};
  I.nrows = nrows;
  I.ncols = ncols;
  I.rowtab = ws->nest_rowtab;
  I.coltab = ws->nest_coltab;
  I.piv = ws->nest_piv;
  const int maxit = kmax + 64;
  constexpr int CH = 4;
  AcaCtl* ring = hc + 1;
  int it = 0, pending = -1;
  bool stop = false;
  while (it < maxit && !stop) {
    const int ch = it / CH;
    for (const int end = std::min(it + CH, maxit); it < end; ++it) {
      k_aca_row<T, 3, 2, true><<<bRow, FS_THREADS, 0, s>>>(I);
      k_aca_col<T, 3, 2, true><<<bCol, FS_THREADS, 0, s>>>(I);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&ring[ch & 1], ctl, sizeof(AcaCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ws->poll_ev[ch & 1], s));
    if (pending >= 0) {
      HIP_TRY(hipEventSynchronize(ws->poll_ev[pending & 1]));
      stop = ring[pending & 1].phase == ACA_DONE;
    }
    pending = ch;
  }
  HIP_TRY(hipMemcpyAsync(hc, ctl, sizeof(AcaCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!std::isfinite(hc->norm2)) return SLAR_E_NUMERIC;
  const int k = hc->k;
  piv->resize(k);
  if (k > 0) {
    HIP_TRY(hipMemcpy(piv->data(), ws->nest_piv, sizeof(Pair) * k, hipMemcpyDeviceToHost));
    for (const Pair& p : *piv)
      if (p[0] < 0 || p[0] >= nrows || p[1] < 0 || p[1] >= ncols) return SLAR_E_NUMERIC;
  }
  ws->nest_samples += hc->samples;
  return SLAR_OK;
}

static hipError_t sample_list(const NestCtx& c, const std::vector<Idx4>& idx, double* out) {
  if (idx.empty()) return hipSuccess;
  Workspace* ws = c.ws;
  HIP_CHK(hipMemcpyAsync(ws->nest_idx, idx.data(), sizeof(Idx4) * idx.size(), hipMemcpyHostToDevice, c.s));
  HIP_CHK(hipStreamSynchronize(c.s));   // the host list is a temporary
  ws->nest_samples += (long long)idx.size();
  return frame_points(c.s, *c.G, c.A, c.dt, c.X, c.P, c.ldt, c.r, (long long)idx.size(), ws->nest_idx, out);
}

static hipError_t inverse(hipStream_t s, Workspace* ws, int r, const double* M, double* Minv) {
  k_gj_inverse<<<1, 256, 0, s>>>(r, M, Minv, ws->nest_flag);
  return hipGetLastError();
}

static Idx4 leaf_entry(int a, int t, const Idx4& comp) {
  Idx4 g = comp;
  g[a] = t;
  return g;
}

// complements of leaf a (the leaf's own position holds -1)
static std::vector<Idx4> leaf_candidates(int a, const std::vector<int>* R, const std::vector<Pair>& Px,
                                         const std::vector<Pair>& Pv) {
  std::vector<Idx4> c;
  if (a == 0) for (int i2 : R[1]) for (const Pair& v : Pv) c.push_back({-1, i2, v[0], v[1]});
  if (a == 1) for (int i1 : R[0]) for (const Pair& v : Pv) c.push_back({i1, -1, v[0], v[1]});
  if (a == 2) for (const Pair& x : Px) for (int j2 : R[3]) c.push_back({x[0], x[1], -1, j2});
  if (a == 3) for (const Pair& x : Px) for (int j1 : R[2]) c.push_back({x[0], x[1], j1, -1});
  return c;
}

template <typename T>
static slar_status nested_impl(const NestCtx& c, double tol, int kmax, const std::vector<Idx4>& probes,
                               const int* seed, slar_ht* out, slar_nested_info* info) {
  Workspace* ws = c.ws;
  const GridDev& G = *c.G;
  const hipStream_t s = c.s;
  const int n[4] = {G.n[0], G.n[1], G.n[2], G.n[3]};
  const double ntol = tol / 10.0;
  constexpr int ENRICH = 4, MAX_SWEEPS = 12;
  const int m = (int)probes.size();
  std::vector<int> R[4];
  for (int a = 0; a < 4; ++a) R[a] = {seed[a]};
  std::vector<Pair> Px = {{seed[0], seed[1]}}, Pv = {{seed[2], seed[3]}};
  std::vector<Idx4> Q[4];
  std::vector<Idx4> forced;
  ws->nest_samples = 0;
  int sweeps = 0, rounds = 0, converged = 0;
  bool built = false;
  double* vals = ws->nest_vals;
  double* sm = ws->nest_small;   // [6][64*64] small matrices
  for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
    std::vector<Idx4> E;
    for (int t = 0; t < std::min(ENRICH, m); ++t) add_unique(E, probes[(sweep * ENRICH + t) % m]);
    for (const Idx4& f : forced) add_unique(E, f);
    std::vector<int> Ru[4];
    for (int a = 0; a < 4; ++a) {
      Ru[a] = R[a];
      for (const Idx4& e : E) add_unique(Ru[a], e[a]);
    }
    std::vector<Pair> Pxu = Px, Pvu = Pv;
    for (const Idx4& e : E) { add_unique(Pxu, Pair{e[0], e[1]}); add_unique(Pvu, Pair{e[2], e[3]}); }
    bool done[4] = {false, false, false, false};
    for (int a = 0; a < 4; ++a) {
      std::vector<int> Rc[4];
      for (int b = 0; b < 4; ++b) Rc[b] = done[b] ? R[b] : Ru[b];
      const std::vector<Idx4> cands = leaf_candidates(a, Rc, Pxu, Pvu);
      std::vector<Idx4> rows(n[a]);
      for (int t = 0; t < n[a]; ++t) rows[t] = {-1, -1, -1, -1}, rows[t][a] = t;
      std::vector<Pair> pr;
      for (const Idx4& e : E) {
        Idx4 comp = e;
        comp[a] = -1;
        const auto it = std::find(cands.begin(), cands.end(), comp);
        if (it != cands.end()) pr.push_back({e[a], (int)(it - cands.begin())});
      }
      std::vector<Pair> piv;
      slar_status st = nest_search<T>(c, rows, cands, ntol, kmax, R[a][0], pr, &piv);
      if (st != SLAR_OK) return st;
      if (piv.empty()) return SLAR_E_NUMERIC;   // an all-zero update has no skeleton
      R[a].clear();
      Q[a].clear();
      for (const Pair& p : piv) { R[a].push_back(p[0]); Q[a].push_back(cands[p[1]]); }
      done[a] = true;
    }
    // root over the new leaf rows plus the enrichment indices
    std::vector<int> Rr[4];
    for (int a = 0; a < 4; ++a) {
      Rr[a] = R[a];
      for (const Idx4& e : E) add_unique(Rr[a], e[a]);
    }
    std::vector<Idx4> rx, rv;
    for (int i1 : Rr[0]) for (int i2 : Rr[1]) rx.push_back({i1, i2, -1, -1});
    for (int j1 : Rr[2]) for (int j2 : Rr[3]) rv.push_back({-1, -1, j1, j2});
    std::vector<Pair> pr;
    for (const Idx4& e : E) {
      int ix = -1, iv = -1;
      for (size_t q = 0; q < rx.size(); ++q) if (rx[q][0] == e[0] && rx[q][1] == e[1]) { ix = (int)q; break; }
      for (size_t q = 0; q < rv.size(); ++q) if (rv[q][2] == e[2] && rv[q][3] == e[3]) { iv = (int)q; break; }
      if (ix >= 0 && iv >= 0) pr.push_back({ix, iv});
    }
    int first = 0;
    for (size_t q = 0; q < rx.size(); ++q)
      if (rx[q][0] == Px[0][0] && rx[q][1] == Px[0][1]) { first = (int)q; break; }
    std::vector<Pair> piv;
    slar_status st = nest_search<T>(c, rx, rv, ntol, kmax, first, pr, &piv);
    if (st != SLAR_OK) return st;
    if (piv.empty()) return SLAR_E_NUMERIC;
    Px.clear();
    Pv.clear();
    for (const Pair& p : piv) { Px.push_back({rx[p[0]][0], rx[p[0]][1]}); Pv.push_back({rv[p[1]][2], rv[p[1]][3]}); }
    sweeps = sweep + 1;
    // ---- skeleton on the device
    const int k = (int)Px.size();
    int rk[4];
    for (int a = 0; a < 4; ++a) rk[a] = (int)R[a].size();
    if (k > kmax) return SLAR_E_RANK_CAP;
    HIP_TRY(hipMemsetAsync(ws->nest_flag, 0, sizeof(int), s));
    for (int a = 0; a < 4; ++a) {
      // C = A^(a)[:, Q_a] (n_a x r_a), then C[R_a, :]
      std::vector<Idx4> L;
      for (int t = 0; t < n[a]; ++t) for (const Idx4& q : Q[a]) L.push_back(leaf_entry(a, t, q));
      if (sample_list(c, L, vals) != hipSuccess) return SLAR_E_HIP;
      std::vector<Idx4> LR;
      for (int i : R[a]) for (const Idx4& q : Q[a]) LR.push_back(leaf_entry(a, i, q));
      if (sample_list(c, LR, vals + (size_t)n[a] * rk[a]) != hipSuccess) return SLAR_E_HIP;
      if (inverse(s, ws, rk[a], vals + (size_t)n[a] * rk[a], sm) != hipSuccess) return SLAR_E_HIP;
      if (gemm_f64(s, false, false, n[a], rk[a], rk[a], 1.0, vals, rk[a], 0, sm, rk[a], 0, 0.0,
                   (double*)out->leaf[a], rk[a], 0, 1) != hipSuccess)
        return SLAR_E_HIP;
    }
    {
      std::vector<Idx4> L;
      for (int a = 0; a < rk[0]; ++a) for (int b = 0; b < rk[1]; ++b) for (const Pair& v : Pv)
        L.push_back({R[0][a], R[1][b], v[0], v[1]});
      if (sample_list(c, L, (double*)out->B12) != hipSuccess) return SLAR_E_HIP;
      L.clear();
      for (int p = 0; p < rk[2]; ++p) for (int q = 0; q < rk[3]; ++q) for (const Pair& x : Px)
        L.push_back({x[0], x[1], R[2][p], R[3][q]});
      if (sample_list(c, L, (double*)out->B34) != hipSuccess) return SLAR_E_HIP;
      L.clear();
      for (const Pair& x : Px) for (const Pair& v : Pv) L.push_back({x[0], x[1], v[0], v[1]});
      if (sample_list(c, L, vals) != hipSuccess) return SLAR_E_HIP;
      if (inverse(s, ws, k, vals, (double*)out->root) != hipSuccess) return SLAR_E_HIP;
    }
    out->d = 4;
    out->dtype = SLAR_F64;
    for (int a = 0; a < 4; ++a) out->rank[a] = rk[a];
    out->rank[4] = k;
    out->rank[5] = k;
    built = true;
    int sing = 0;
    HIP_TRY(hipMemcpyAsync(&sing, ws->nest_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (sing) return SLAR_E_NUMERIC;
    // ---- probe check: skeleton at the probes (zero-length flow: grid
    // values), the updated entries there, the norm from the frame Grams
    if (m > 0) {
      const AdvDev A0{0, 3, 0.0, 0.0, nullptr, nullptr, 0.0, 0.0, 0};
      if (hipMemcpyAsync(ws->nest_idx, probes.data(), sizeof(Idx4) * m, hipMemcpyHostToDevice, s) != hipSuccess)
        return SLAR_E_HIP;
      if (ht_sample(s, G, A0, *out, m, ws->nest_idx, vals) != hipSuccess) return SLAR_E_HIP;
      if (frame_points(s, G, c.A, c.dt, c.X, c.P, c.ldt, c.r, m, ws->nest_idx, vals + m) != hipSuccess)
        return SLAR_E_HIP;
      ws->nest_samples += m;
      slar_frames fr{0, SLAR_KMAX, ws->nest_fX, ws->nest_fP};
      if (frames_from_ht(s, ws, G, *out, &fr) != hipSuccess) return SLAR_E_HIP;
      double* GX = sm + 64 * 64;
      double* GP = sm + 2 * 64 * 64;
      if (gemm_tn_long(s, ws, k, k, G.nx, fr.X, fr.ld, fr.X, fr.ld, GX, k) != hipSuccess) return SLAR_E_HIP;
      if (gemm_tn_long(s, ws, k, k, G.nv, fr.P, fr.ld, fr.P, fr.ld, GP, k) != hipSuccess) return SLAR_E_HIP;
      k_nest_probe<<<1, 256, 0, s>>>(m, vals, vals + m, k, GX, GP, tol, (double)G.nx * (double)G.nv,
                                     ws->nest_flag + 1);
      int res[2] = {0, 0};
      HIP_TRY(hipMemcpyAsync(res, ws->nest_flag + 1, sizeof(res), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (res[0] == 0 && sweep >= 1) { converged = 1; break; }
      forced.clear();
      if (res[0] > 0 && res[1] >= 0 && res[1] < m) {
        forced.push_back(probes[res[1]]);
        ++rounds;
      }
    } else if (sweep >= 1) {
      converged = 1;
      break;
    }
  }
  if (!built) return SLAR_E_NUMERIC;
  if (info) {
    info->sweeps = sweeps;
    info->probe_rounds = rounds;
    info->converged = converged;
    for (int q = 0; q < 6; ++q) info->rank[q] = out->rank[q];
    info->samples = ws->nest_samples;
  }
  return converged ? SLAR_OK : SLAR_E_NOCONV;
}

slar_status nested_run(hipStream_t s, Workspace* ws, const slar_frames& src, const slar_adv& adv,
                       slar_dtype dt, double tol, int kmax, int nprobe, const int* probes, const int* seed,
                       slar_ht* out, slar_nested_info* info) {
  const GridDev& G = ws->G;
  const int r = src.r;
  const int ldt = (r + 3) & ~3;
  NestCtx c{s, ws, &ws->G, AdvDev{}, dt, nullptr, nullptr, ldt, r};
  if (dt == SLAR_F32) {
    if (table_copy(s, G.nx, r, src.ld, src.X, ldt, ws->X32, nullptr) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(s, G.nv, r, src.ld, src.P, ldt, ws->P32, nullptr) != hipSuccess) return SLAR_E_HIP;
    c.X = ws->X32;
    c.P = ws->P32;
  } else {
    if (table_copy(s, G.nx, r, src.ld, src.X, ldt, nullptr, ws->nest_X64) != hipSuccess) return SLAR_E_HIP;
    if (table_copy(s, G.nv, r, src.ld, src.P, ldt, nullptr, ws->nest_P64) != hipSuccess) return SLAR_E_HIP;
    c.X = ws->nest_X64;
    c.P = ws->nest_P64;
  }
  if (combine_field(s, G, &adv, ws->Eeff) != hipSuccess) return SLAR_E_HIP;
  c.A = AdvDev{adv.kind, adv.order, adv.tau, adv.cv, ws->Eeff, nullptr, 1.0, 0.0, 1};
  std::vector<Idx4> pr(nprobe);
  for (int q = 0; q < nprobe; ++q)
    for (int a = 0; a < 4; ++a) pr[q][a] = probes[4 * q + a];
  if (dt == SLAR_F32) return nested_impl<float>(c, tol, kmax, pr, seed, out, info);
  return nested_impl<double>(c, tol, kmax, pr, seed, out, info);
}

}  // namespace slar
