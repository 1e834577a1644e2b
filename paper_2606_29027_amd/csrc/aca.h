// Device side of the adaptive cross approximation: control block, the
// per-instance argument record and the three per-iteration bodies (row
// fiber, column fiber, bookkeeping).  The bodies take one instance record
// and one fiber tile index, so the same code serves one launch per
// instance and the persistent multi-instance launches.
#pragma once
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
};

constexpr int ACA_MAXBLK = 1024;   // partial slots
// Entries per fiber block (a lane quad per foot in a 256-thread block).  A
// fiber has at most 128^2 entries, i.e. 256 blocks.  Tiles of 32 (two
// blocks per CU) left the sampling launch as long (each block's time is
// the latency of its feet and gathers) and made the bookkeeping launch
// stage twice the candidates, so 64 it is.
constexpr int ACA_TILE = 64;

// Everything one cross approximation reads or writes (one instance).
struct AcaInst {
  GridDev g;
  AdvDev a;
  const void* X;
  const void* P;
  int ld, r;
  AcaCtl* ctl;
  double* U;
  double* V;
  unsigned char* used;
  double* part;
  int nbrow, nbcol, nprobe;
  int team;            // lanes per sample in the fiber gathers (4, 8 or 16)
  const int* probes;
  // index-table mode (nested cross searches): the matrix is nrows x ncols,
  // entry (row, col) is the grid point whose multi-index joins
  // rowtab[4 row ..] and coltab[4 col ..] (entries < 0 unset).  In both
  // modes accepted pivots (row, col) are logged in piv[2 k ..] when piv is
  // set.
  int nrows = 0, ncols = 0;
  const int* rowtab = nullptr;
  const int* coltab = nullptr;
  int* piv = nullptr;
  // host-mapped pinned words that receive, from a bookkeeping launch given
  // them (the last of a chunk of iterations, single-instance driver; null
  // elsewhere), the phase in [0] and then the chunk's sequence number seq
  // in [1]
  int* phase_host = nullptr;
  int seq = 0;
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of x[0..15] over the 64 lanes of a wave by a butterfly
// reduce-scatter (17 exchanges instead of 16 full reductions); lane ln gets
// the total of value 8 b5 + 4 b4 + 2 b3 + b2 (b_i = bit i of ln), which
// the lanes with ln % 4 == 0 hold once each.
__device__ __forceinline__ double wave_sum16_scatter(double* x, int ln) {
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const bool hi = ln & 32;
    const double send = hi ? x[m] : x[m + 8];
    const double keep = hi ? x[m + 8] : x[m];
    x[m] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bool hi = ln & 16;
    const double send = hi ? x[m] : x[m + 4];
    const double keep = hi ? x[m + 4] : x[m];
    x[m] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const bool hi = ln & 8;
    const double send = hi ? x[m] : x[m + 2];
    const double keep = hi ? x[m + 2] : x[m];
    x[m] = keep + __shfl_xor(send, 8, 64);
  }
  {
    const bool hi = ln & 4;
    const double send = hi ? x[0] : x[1];
    const double keep = hi ? x[1] : x[0];
    x[0] = keep + __shfl_xor(send, 4, 64);
  }
  double v = x[0];
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}
__device__ __forceinline__ int scatter_slot(int ln) {
  return ((ln >> 5) & 1) * 8 + ((ln >> 4) & 1) * 4 + ((ln >> 3) & 1) * 2 + ((ln >> 2) & 1);
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

// out[l] = sum_b part[(1 + l) * ACA_MAXBLK + b] for l in [0, cnt), one wave
// per l (l = wave, wave + 4, ...), lanes over b (coalesced), fixed order.
__device__ void block_sum_parts(const double* part, int nb, int cnt, double* out) {
  const int t = threadIdx.x;
  const int wv = t >> 6, ln = t & 63;
  for (int l = wv; l < cnt; l += 4) {
    const double* q = part + (size_t)(1 + l) * ACA_MAXBLK;
    double acc = 0.0;
    for (int b = ln; b < nb; b += 64) acc += q[b];
    acc = wave_sum(acc);
    if (ln == 0) out[l] = acc;
  }
}

template <int DX>
__device__ __forceinline__ void unravel_x(const GridDev& g, int I, int* gi) {
  if (DX == 1) gi[0] = I; else { gi[0] = I / g.n[1]; gi[1] = I % g.n[1]; }
}
template <int DX>
__device__ __forceinline__ void unravel_v(const GridDev& g, int J, int* gi) {
  if (DX == 1) gi[1] = J; else { gi[2] = J / g.n[3]; gi[3] = J % g.n[3]; }
}

// Grid multi-index of matrix entry (row, col): the {x}|{v} matricisation,
// or (TAB) the union of the partial multi-indices of the two tables.
template <int DX, bool TAB>
__device__ __forceinline__ void entry_index(const AcaInst& I, int row, int col, int* gi) {
  if (TAB) {
    const int* rt = I.rowtab + 4 * row;
    const int* ct = I.coltab + 4 * col;
#pragma unroll
    for (int d = 0; d < 4; ++d) gi[d] = rt[d] >= 0 ? rt[d] : ct[d];
  } else {
    unravel_x<DX>(I.g, row, gi);
    unravel_v<DX>(I.g, col, gi);
  }
}

// Partial-sum layout (doubles): part[q * ACA_MAXBLK + b]
//   row kernel: q = 0 block max|r|, q = 1 block candidate index,
//               q = 2 + l  v_l . r  (l <= k < ACA_KC), q = PVAL candidate |r|
//   col kernel: same with base PCOL
//   q = GSUM: sum over row blocks of v_l . r at slot l (written by the
//   column kernel, read by the bookkeeping kernel)
constexpr int ACA_KC = SLAR_CROSS_KMAX;
constexpr int PVAL = ACA_KC + 2;
constexpr int GSUM = ACA_KC + 3;
constexpr int PCOL = ACA_KC + 4;
constexpr int ACA_PART_SLOTS = PCOL + PVAL + 1;
static_assert(ACA_KC <= ACA_MAXBLK, "GSUM holds one slot per cross term");

// Per-block max of |x| (entries with skip() excluded), the lowest index in
// the block whose |x| is within the tie tolerance of that block max, and
// |x| at that index (-1 when the block has no eligible entry).
template <typename Skip>
__device__ void block_candidate(const double* xs, int ns, int base, Skip skip, double* red, int* redi,
                                double* out_max, double* out_idx, double* out_val) {
  const int t = threadIdx.x;
  double v = -1.0;
  if (t < ns && !skip(base + t)) v = fabs(xs[t]);
  const double m = block_max(v, red);
  int cand = 1 << 30;
  if (t < ns && !skip(base + t) && m >= 0.0 && fabs(xs[t]) >= m * (1.0 - 1e-10)) cand = base + t;
  for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o, 64));
  if ((t & 63) == 0) redi[t >> 6] = cand;
  __syncthreads();
  if (t == 0) {
    const int c = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
    *out_max = m;
    *out_idx = (double)c;
    *out_val = (c < base + ns) ? fabs(xs[c - base]) : -1.0;
  }
  __syncthreads();
}

// Global pivot from per-block candidates: lowest index whose |x| is within
// the tie tolerance of the global maximum M (M < 0: nothing eligible).
// pmax / pidx / pval are the per-block maximum, candidate index and
// candidate value; only when the first qualifying block's candidate falls
// below the tolerance is that block's range of x rescanned.
template <typename Skip>
__device__ int pivot_from_parts(const double* x, const double* pmax, const double* pidx,
                                const double* pval, int nb, int n, Skip skip, double* red, int* redi,
                                double* M_out) {
  const int t = threadIdx.x;
  double m = -1.0;
  for (int b = t; b < nb; b += blockDim.x) m = fmax(m, pmax[b]);
  const double M = block_max(m, red);
  *M_out = M;
  if (!(M >= 0.0)) return n;
  const double thr = M * (1.0 - 1e-10);
  int bb = nb;
  for (int b = t; b < nb; b += blockDim.x)
    if (pmax[b] >= thr && b < bb) bb = b;
  for (int o = 32; o > 0; o >>= 1) bb = min(bb, __shfl_xor(bb, o, 64));
  if ((t & 63) == 0) redi[t >> 6] = bb;
  __syncthreads();
  bb = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  __syncthreads();
  if (bb >= nb) return n;
  const int cand = (int)pidx[bb];
  if (cand < n && pval[bb] >= thr) return cand;
  // the block maximum is close to M but below it: rescan that block's range
  int best = n;
  const int e = bb * ACA_TILE + t;
  if (t < ACA_TILE && e < n && !skip(e) && fabs(x[e]) >= thr) best = e;
  for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((t & 63) == 0) redi[t >> 6] = best;
  __syncthreads();
  best = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  __syncthreads();
  return best;
}

struct NoSkip {
  __device__ bool operator()(int) const { return false; }
};
struct SkipUsed {
  const unsigned char* used;
  int also;
  __device__ bool operator()(int e) const { return used[e] != 0 || e == also; }
};

// Earlier cross vectors at this thread's position, cached in registers:
// slot m holds l = wave + 4 m for the first 64 terms; terms 64..127 (when
// the cross runs past 64) are read in a second chunk, l = 64 + wave + 4 m.
constexpr int ACA_LREG = 16;
constexpr int ACA_CHUNK = 4 * ACA_LREG;
static_assert(2 * ACA_CHUNK >= ACA_KC, "two chunks cover every cross term");

template <typename T, int W, int DX, bool TAB = false>
__device__ void aca_row_body(const AcaInst& I, int tile) {
  const GridDev& g = I.g;
  const AdvDev& a = I.a;
  const T* __restrict__ X = (const T*)I.X;
  const T* __restrict__ P = (const T*)I.P;
  const int ld = I.ld, r = I.r;
  AcaCtl* ctl = I.ctl;
  const double* __restrict__ U = I.U;
  double* __restrict__ V = I.V;
  double* __restrict__ part = I.part;
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int s_phase, s_i, s_k;
  __shared__ double acc4[4][FS_SAMPLES];
  __shared__ double rres[FS_SAMPLES];
  const int t = threadIdx.x;
  if (t == 0) { s_phase = ctl->phase; s_i = ctl->i; s_k = ctl->k; }
  __syncthreads();
  if (s_phase != ACA_RUN) return;
  const int i = s_i, k = s_k;
  const int Nx = TAB ? I.nrows : g.nx, Nv = TAB ? I.ncols : g.nv;
  const int J0 = tile * ACA_TILE;
  const int ns = min(ACA_TILE, Nv - J0);
  const int wv = t >> 6, ln = t & 63;
  // earlier row vectors v_l[J] and u_l[i] (loads in flight during the feet)
  double vl[ACA_LREG], ui[ACA_LREG];
#pragma unroll
  for (int m = 0; m < ACA_LREG; ++m) {
    const int l = wv + 4 * m;
    const bool ok = l < k && ln < ns;
    vl[m] = ok ? V[(size_t)l * Nv + J0 + ln] : 0.0;
    ui[m] = ok ? U[(size_t)l * Nx + i] : 0.0;
  }
  {
    const int s = t >> 2;
    if (s < ns) {
      int gi[4];
      entry_index<DX, TAB>(I, i, J0 + s, gi);
      fs_prepare<W, DX, 4>(g, a, gi, L, s, t & 3);
    }
  }
  // residual r_J = A[i, J] - sum_l u_l[i] v_l[J]: the l-sum is split over
  // the four waves (wave w takes l = w, w + 4, ...) and combined in LDS
  {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < ACA_LREG; ++m)
      if (wv + 4 * m < k) acc += ui[m] * vl[m];
    if (k > ACA_CHUNK) {
#pragma unroll 4
      for (int m = 0; m < ACA_LREG; ++m) {
        const int l = ACA_CHUNK + wv + 4 * m;
        if (l < k && ln < ns) acc += U[(size_t)l * Nx + i] * V[(size_t)l * Nv + J0 + ln];
      }
    }
    acc4[wv][ln] = acc;
  }
  __syncthreads();
  fs_evaluate_team<T, W, DX>(I.team, X, P, ld, r, L, ns);
  __syncthreads();
  if (t < 64) {
    double rv = 0.0;
    if (t < ns) {
      rv = L.val[t] - (((acc4[0][t] + acc4[1][t]) + acc4[2][t]) + acc4[3][t]);
      V[(size_t)k * Nv + J0 + t] = rv;
    }
    rres[t] = rv;
  }
  __syncthreads();
  {
    const double r_ = (ln < ns) ? rres[ln] : 0.0;
    double pv[ACA_LREG];
#pragma unroll
    for (int m = 0; m < ACA_LREG; ++m) {
      const int l = wv + 4 * m;
      pv[m] = (l < k ? vl[m] : (l == k ? r_ : 0.0)) * r_;
    }
    const double p = wave_sum16_scatter(pv, ln);
    const int l = wv + 4 * scatter_slot(ln);
    if ((ln & 3) == 0 && l <= k) part[(size_t)(2 + l) * ACA_MAXBLK + tile] = p;
    if (k >= ACA_CHUNK) {
      // second chunk of the dot products, l = 64 + wave + 4 m
#pragma unroll
      for (int m = 0; m < ACA_LREG; ++m) {
        const int l2 = ACA_CHUNK + wv + 4 * m;
        const double v2 = (l2 < k && ln < ns) ? V[(size_t)l2 * Nv + J0 + ln] : (l2 == k ? r_ : 0.0);
        pv[m] = v2 * r_;
      }
      const double p2 = wave_sum16_scatter(pv, ln);
      const int l2 = ACA_CHUNK + wv + 4 * scatter_slot(ln);
      if ((ln & 3) == 0 && l2 <= k) part[(size_t)(2 + l2) * ACA_MAXBLK + tile] = p2;
    }
  }
  block_candidate(rres, ns, J0, NoSkip{}, red, redi, &part[tile], &part[ACA_MAXBLK + tile],
                  &part[(size_t)PVAL * ACA_MAXBLK + tile]);
}

template <typename T, int W, int DX, bool TAB = false>
__device__ void aca_col_body(const AcaInst& I, int tile) {
  const GridDev& g = I.g;
  const AdvDev& a = I.a;
  const T* __restrict__ X = (const T*)I.X;
  const T* __restrict__ P = (const T*)I.P;
  const int ld = I.ld, r = I.r;
  AcaCtl* ctl = I.ctl;
  double* __restrict__ U = I.U;
  const double* __restrict__ V = I.V;
  const unsigned char* __restrict__ used = I.used;
  double* __restrict__ part = I.part;
  const int nbrow = I.nbrow;
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int s_phase, s_i, s_k;
  __shared__ double s_norm2, s_tol;
  __shared__ double acc4[4][FS_SAMPLES];
  __shared__ double ures[FS_SAMPLES];
  const int t = threadIdx.x;
  if (t == 0) { s_phase = ctl->phase; s_i = ctl->i; s_k = ctl->k; s_norm2 = ctl->norm2; s_tol = ctl->tol; }
  __syncthreads();
  if (s_phase != ACA_RUN) return;
  const int i = s_i, k = s_k;
  const int Nx = TAB ? I.nrows : g.nx, Nv = TAB ? I.ncols : g.nv;
  const int I0 = tile * ACA_TILE;
  const int ns = min(ACA_TILE, Nx - I0);
  const int wv = t >> 6, ln = t & 63;
  // earlier column vectors u_l[I] (independent of the pivot: issued first)
  double ul[ACA_LREG];
#pragma unroll
  for (int m = 0; m < ACA_LREG; ++m) {
    const int l = wv + 4 * m;
    ul[m] = (l < k && ln < ns) ? U[(size_t)l * Nx + I0 + ln] : 0.0;
  }
  // column pivot of the row residual (every block computes the same)
  double M;
  const double* vk = V + (size_t)k * Nv;
  const int j = pivot_from_parts(vk, part, part + ACA_MAXBLK, part + (size_t)PVAL * ACA_MAXBLK, nbrow, Nv,
                                 NoSkip{}, red, redi, &M);
  if (tile == 0 && t == 0) { ctl->j = j; ctl->pivot = M; }   // read by the bookkeeping launch
  const double thr = s_tol * sqrt(s_norm2) / sqrt((double)Nx * (double)Nv);
  if (M == 0.0 || M <= thr || j >= Nv) return;   // row already reproduced
  // finish the row-fiber dot products for the bookkeeping launch:
  // gv[l] = sum_b (v_l . r)_b, block `tile` takes l = tile, tile + nbcol, ...
  for (int l = tile; l <= k; l += I.nbcol) {
    const double* q = part + (size_t)(2 + l) * ACA_MAXBLK;
    double acc = 0.0;
    for (int b = t; b < nbrow; b += FS_THREADS) acc += q[b];
    acc = wave_sum(acc);
    if (ln == 0) acc4[wv][0] = acc;
    __syncthreads();
    if (t == 0) part[(size_t)GSUM * ACA_MAXBLK + l] = ((acc4[0][0] + acc4[1][0]) + acc4[2][0]) + acc4[3][0];
    __syncthreads();
  }
  const double piv = vk[j];
  double vj[ACA_LREG];
#pragma unroll
  for (int m = 0; m < ACA_LREG; ++m) {
    const int l = wv + 4 * m;
    vj[m] = (l < k) ? V[(size_t)l * Nv + j] : 0.0;
  }
  {
    const int s = t >> 2;
    if (s < ns) {
      int gi[4];
      entry_index<DX, TAB>(I, I0 + s, j, gi);
      fs_prepare<W, DX, 4>(g, a, gi, L, s, t & 3);
    }
  }
  {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < ACA_LREG; ++m)
      if (wv + 4 * m < k) acc += vj[m] * ul[m];
    if (k > ACA_CHUNK) {
#pragma unroll 4
      for (int m = 0; m < ACA_LREG; ++m) {
        const int l = ACA_CHUNK + wv + 4 * m;
        if (l < k && ln < ns) acc += V[(size_t)l * Nv + j] * U[(size_t)l * Nx + I0 + ln];
      }
    }
    acc4[wv][ln] = acc;
  }
  __syncthreads();
  fs_evaluate_team<T, W, DX>(I.team, X, P, ld, r, L, ns);
  __syncthreads();
  if (t < 64) {
    double u = 0.0;
    if (t < ns) {
      u = (L.val[t] - (((acc4[0][t] + acc4[1][t]) + acc4[2][t]) + acc4[3][t])) / piv;
      U[(size_t)k * Nx + I0 + t] = u;
    }
    ures[t] = u;
  }
  __syncthreads();
  double* pc = part + (size_t)PCOL * ACA_MAXBLK;
  {
    const double u_ = (ln < ns) ? ures[ln] : 0.0;
    double pu[ACA_LREG];
#pragma unroll
    for (int m = 0; m < ACA_LREG; ++m) {
      const int l = wv + 4 * m;
      pu[m] = (l < k ? ul[m] : (l == k ? u_ : 0.0)) * u_;
    }
    const double p = wave_sum16_scatter(pu, ln);
    const int l = wv + 4 * scatter_slot(ln);
    if ((ln & 3) == 0 && l <= k) pc[(size_t)(2 + l) * ACA_MAXBLK + tile] = p;
    if (k >= ACA_CHUNK) {
#pragma unroll
      for (int m = 0; m < ACA_LREG; ++m) {
        const int l2 = ACA_CHUNK + wv + 4 * m;
        const double x2 = (l2 < k && ln < ns) ? U[(size_t)l2 * Nx + I0 + ln] : (l2 == k ? u_ : 0.0);
        pu[m] = x2 * u_;
      }
      const double p2 = wave_sum16_scatter(pu, ln);
      const int l2 = ACA_CHUNK + wv + 4 * scatter_slot(ln);
      if ((ln & 3) == 0 && l2 <= k) pc[(size_t)(2 + l2) * ACA_MAXBLK + tile] = p2;
    }
  }
  block_candidate(ures, ns, I0, SkipUsed{used, i}, red, redi, &pc[tile], &pc[ACA_MAXBLK + tile],
                  &pc[(size_t)PVAL * ACA_MAXBLK + tile]);
}

// One block: bookkeeping of the iteration, stopping test, next row pivot,
// and the random-probe check whenever the approximation wants to stop.
// Every partial the iteration needs (block maxima, candidates and their
// values of both fibers, and the per-block dot products) is loaded in one
// pass of independent loads; the rest works from LDS.
constexpr int FIN_NB = 256;   // blocks per fiber staged in LDS
static_assert(ACA_TILE <= FS_SAMPLES, "a fiber tile fits the sampler's LDS rows");
static_assert(FIN_NB * ACA_TILE >= SLAR_NMAX * SLAR_NMAX && FIN_NB * ACA_TILE >= SLAR_NMAX_1D,
              "every fiber fits the staged partials");

template <typename T, int W, int DX, bool TAB = false>
__device__ void aca_fin_body(const AcaInst& I) {
  const GridDev& g = I.g;
  const AdvDev& a = I.a;
  const T* __restrict__ X = (const T*)I.X;
  const T* __restrict__ P = (const T*)I.P;
  const int ld = I.ld, r = I.r;
  AcaCtl* ctl = I.ctl;
  const double* __restrict__ U = I.U;
  const double* __restrict__ V = I.V;
  unsigned char* __restrict__ used = I.used;
  const double* __restrict__ part = I.part;
  const int nbcol = I.nbcol, nprobe = I.nprobe;
  const int* __restrict__ probes = I.probes;
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ double sgv[ACA_KC + 1], sgu[ACA_KC + 1];
  __shared__ double cmax_[FIN_NB], cidx_[FIN_NB], cval_[FIN_NB];
  __shared__ double res[1024];
  __shared__ int pi[1024];
  __shared__ int s_phase, s_i, s_k, s_stop, s_j;
  __shared__ double s_tol, s_norm2, s_M;
  const int t = threadIdx.x;
  if (t == 0) {
    s_phase = ctl->phase; s_i = ctl->i; s_k = ctl->k; s_tol = ctl->tol; s_norm2 = ctl->norm2;
    s_j = ctl->j; s_M = ctl->pivot;
  }
  const double* pc = part + (size_t)PCOL * ACA_MAXBLK;
  for (int b = t; b < nbcol; b += blockDim.x) {
    cmax_[b] = pc[b]; cidx_[b] = pc[ACA_MAXBLK + b]; cval_[b] = pc[(size_t)PVAL * ACA_MAXBLK + b];
  }
  __syncthreads();
  if (s_phase != ACA_RUN) return;
  const int i = s_i;
  int k = s_k;
  const int Nx = TAB ? I.nrows : g.nx, Nv = TAB ? I.ncols : g.nv;
  // column pivot j of the row residual and its maximum M, as every block
  // of the column launch derived them from the row partials
  const int j = s_j;
  const double M = s_M;
  const double thr = s_tol * sqrt(s_norm2) / sqrt((double)Nx * (double)Nv);
  const bool zero_row = (M == 0.0 || M <= thr || j >= Nv);
  if (t == 0) {
    used[i] = 1;
    ctl->iters += 1;
    ctl->samples += Nv;
  }
  if (!zero_row) {
    // gv[l]: reduced by the column launch; gu[l] = sum_b (u_l . u)_b here:
    // wave w takes l = w + 4 m (m < 16) of each 64-term chunk, lanes run
    // over the blocks, all loads of a chunk are issued before the sums,
    // then a butterfly reduce-scatter leaves the total of value m(lane) in
    // every lane
    {
      const int wv = t >> 6, ln = t & 63;
      for (int c0 = 0; c0 <= k; c0 += ACA_CHUNK) {
        double acc[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int l = min(c0 + wv + 4 * m, ACA_KC - 1);
          const double* q = pc + (size_t)(2 + l) * ACA_MAXBLK;
          double a4 = 0.0;
#pragma unroll
          for (int i4 = 0; i4 < FIN_NB / 64; ++i4) {
            const int b = ln + 64 * i4;
            const double v = q[b];
            a4 += (b < nbcol) ? v : 0.0;
          }
          acc[m] = (c0 + wv + 4 * m <= k) ? a4 : 0.0;
        }
        const double tot = wave_sum16_scatter(acc, ln);
        const int m = scatter_slot(ln);
        const int l = c0 + wv + 4 * m;
        if ((ln & 3) == 0 && l <= k) sgu[l] = tot;
      }
      if (t <= k) sgv[t] = part[(size_t)GSUM * ACA_MAXBLK + t];
    }
    __syncthreads();
    if (t < 64) {
      // cross terms sum_{l<k} (u_l . u_k)(v_l . v_k), k < 128
      double c = (t < k) ? sgu[t] * sgv[t] : 0.0;
      if (t + 64 < k) c += sgu[t + 64] * sgv[t + 64];
      c = wave_sum(c);
      if (t == 0) {
        ctl->samples += Nx;
        if (I.piv) { I.piv[2 * k] = i; I.piv[2 * k + 1] = j; }
        const double nk = sgu[k] * sgv[k];
        const double norm2 = s_norm2 + 2.0 * c + nk;
        ctl->norm2 = norm2;
        ctl->k = k + 1;
        s_norm2 = norm2;
        s_stop = 0;
        if (sqrt(nk) <= s_tol * sqrt(fmax(norm2, 0.0))) s_stop = 1;            // probe
        else if (k + 1 >= ctl->kmax) { ctl->phase = ACA_DONE; ctl->capped = 1; s_stop = 2; }
      }
    }
    __syncthreads();
    k = k + 1;
    if (s_stop == 2) return;
    if (s_stop == 0) {
      // next row pivot: unused row maximising |u_k| (block candidates)
      const double* uk = U + (size_t)(k - 1) * Nx;
      double Mu;
      const int ip = pivot_from_parts(uk, cmax_, cidx_, cval_, nbcol, Nx, SkipUsed{used, i}, red, redi, &Mu);
      if (t == 0) {
        if (!(Mu >= 0.0) || ip >= Nx) ctl->phase = ACA_DONE;
        else ctl->i = ip;
      }
      return;
    }
  }
  // ---- probe check (the approximation wants to stop)
  if (k == 0 || nprobe <= 0) {
    if (t == 0) { ctl->phase = ACA_DONE; ctl->converged = 1; }
    return;
  }
  const double thr2 = s_tol * sqrt(fmax(s_norm2, 0.0)) / sqrt((double)Nx * (double)Nv);
  for (int base = 0; base < nprobe; base += FS_SAMPLES) {
    const int ns = min(FS_SAMPLES, nprobe - base);
    const int s = t >> 2, q = t & 3;
    int pI = 0, pJ = 0;
    if (s < ns) {
      pI = probes[2 * (base + s)];
      pJ = probes[2 * (base + s) + 1];
      int gi[4];
      entry_index<DX, TAB>(I, pI, pJ, gi);
      fs_prepare<W, DX, 4>(g, a, gi, L, s, q);
    }
    // approximation at the probe: the quad splits the l-sum
    double ap = 0.0;
    if (s < ns)
      for (int l = q; l < k; l += 4) ap += U[(size_t)l * Nx + pI] * V[(size_t)l * Nv + pJ];
    ap += __shfl_xor(ap, 1, 4);
    ap += __shfl_xor(ap, 2, 4);
    __syncthreads();
    fs_evaluate_team<T, W, DX>(I.team, X, P, ld, r, L, ns);
    __syncthreads();
    if (s < ns && q == 0) {
      const double v = L.val[s] - ap;
      const bool bad = fabs(v) > thr2 && !used[pI];
      res[base + s] = bad ? fabs(v) : -1.0;
      pi[base + s] = pI;
    }
    __syncthreads();
  }
  double m = -1.0;
  for (int e = t; e < nprobe; e += blockDim.x) m = fmax(m, res[e]);
  m = block_max(m, red);
  int best = nprobe;
  if (m > 0.0) {
    for (int e = t; e < nprobe; e += blockDim.x)
      if (res[e] > 0.0 && res[e] >= m * (1.0 - 1e-10) && e < best) best = e;
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
    }
  }
}

// --------------------------------------------------- single-instance kernels
template <typename T, int W, int DX, bool TAB = false>
__global__ __launch_bounds__(FS_THREADS) void k_aca_row(AcaInst I) { aca_row_body<T, W, DX, TAB>(I, blockIdx.x); }
template <typename T, int W, int DX, bool TAB = false>
__global__ __launch_bounds__(FS_THREADS) void k_aca_col(AcaInst I) { aca_col_body<T, W, DX, TAB>(I, blockIdx.x); }
template <typename T, int W, int DX, bool TAB = false>
__global__ __launch_bounds__(FS_THREADS) void k_aca_fin(AcaInst I) {
  aca_fin_body<T, W, DX, TAB>(I);
  // thread 0 made every change of the phase, so it reads the final value;
  // the host waits for seq, then reads the phase
  if (I.phase_host && threadIdx.x == 0) {
    volatile int* ph = I.phase_host;
    ph[0] = I.ctl->phase;
    __threadfence_system();
    ph[1] = I.seq;
  }
}

}  // namespace slar
