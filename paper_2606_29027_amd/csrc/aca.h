// Device side of the adaptive cross approximation: control block, the
// per-instance argument record and the two per-iteration bodies (row fiber,
// column fiber).  The bodies take one instance record and one fiber tile
// index, so the same code serves one launch per instance and the
// persistent multi-instance launches.
#pragma once
#include <cmath>

#include "slar_internal.h"
#include "frame_sampler.h"

namespace slar {

enum { ACA_RUN = 0, ACA_PROBE = 1, ACA_DONE = 2 };
// What the row launch does before it samples: START (row i), COL (the
// column launch before it sampled term k-1: next row pivot from its
// candidates, and the sums of its dot products), PROBE (the column launch
// before it sampled the probe entries: resolve the probe check).
enum { ACA_NX_START = 0, ACA_NX_COL = 1, ACA_NX_PROBE = 2 };

// Two records per cross approximation: the row launch reads ctl[0] and
// writes ctl[1], the column launch reads ctl[1] and writes ctl[0], so no
// launch writes the record its own blocks read.  Every block takes the
// launch's decision from the same inputs; the block of tile 0 writes it.
struct AcaCtl {
  int phase, k, i, j;
  int iters, probe_rounds, converged, capped;
  int next;    // ACA_NX_* (written by the column launch)
  int rowok;   // the row launch sampled row i (written by the row launch)
  int kmax, pad;
  double pivot, norm2, tol;
  long long samples;
};

constexpr int ACA_MAXBLK = 1024;   // partial slots
// Entries per fiber block (a lane quad per foot in a 256-thread block).  A
// fiber has at most 128^2 entries, i.e. 256 blocks.  Tiles of 32 (two
// blocks per CU) left the sampling launch as long (each block's time is
// the latency of its feet and gathers) and doubled the candidates every
// block of the next launch reduces, so 64 it is.
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
  // host-mapped pinned words that receive, from a column launch given
  // them (the last of a chunk of iterations, single-instance driver; null
  // elsewhere), the phase in [0] and then the chunk's sequence number seq
  // in [1]
  int* phase_host = nullptr;
  int seq = 0;
};

// The thread index through an empty volatile asm.  In the persistent
// multi-instance kernels this keeps the compiler from hoisting every value
// derived from it (lane masks, LDS offsets) out of the work-item loop, where
// they held registers for the whole launch; per item they cost a few ALU
// operations.
__device__ __forceinline__ int aca_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

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
  const int t = aca_tid();
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
  const int t = aca_tid();
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
//   q = GSUM, GSUM1: sum over row blocks of v_l . r at slot l for even /
//   odd term index (written by the column kernel of the term, read by the
//   next column kernel)
//   q = GSU: sum over column blocks of u_l . u at slot l (written by the
//   row kernel after the term's column, read by the next column kernel)
//   q = PRB, PRBI: residual (or -1) and row of each probe entry
constexpr int ACA_KC = SLAR_CROSS_KMAX;
constexpr int PVAL = ACA_KC + 2;
constexpr int GSUM = ACA_KC + 3;
constexpr int PCOL = ACA_KC + 4;
constexpr int GSUM1 = PCOL + PVAL + 1;
constexpr int GSU = GSUM1 + 1;
constexpr int PRB = GSU + 1;
constexpr int PRBI = PRB + 1;
constexpr int ACA_PART_SLOTS = PRBI + 1;
static_assert(ACA_KC <= ACA_MAXBLK, "GSUM holds one slot per cross term");

// Per-block max of |x| (entries with skip() excluded), the lowest index in
// the block whose |x| is within the tie tolerance of that block max, and
// |x| at that index (-1 when the block has no eligible entry).
template <typename Skip>
__device__ void block_candidate(const double* xs, int ns, int base, Skip skip, double* red, int* redi,
                                double* out_max, double* out_idx, double* out_val) {
  const int t = aca_tid();
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


// A fiber has at most FIN_NB blocks, so one thread holds one block's pivot
// candidate.
constexpr int FIN_NB = 256;
static_assert(ACA_TILE <= FS_SAMPLES, "a fiber tile fits the sampler's LDS rows");
static_assert(FIN_NB <= FS_THREADS, "one thread per fiber block");
static_assert(FIN_NB * ACA_TILE >= SLAR_NMAX * SLAR_NMAX && FIN_NB * ACA_TILE >= SLAR_NMAX_1D,
              "every fiber has at most FIN_NB blocks");
static_assert(FS_THREADS * 4 >= 1024 && ACA_MAXBLK >= 1024, "probe slots hold 1024 entries");

// Per-block pivot candidates of one fiber: thread b < nb holds block b's
// maximum, candidate index and candidate value (-1, 0, -1 elsewhere).
struct Cand {
  double m, idx, val;
};
__device__ __forceinline__ Cand load_cand(const double* base, int nb) {
  const int t = aca_tid();
  Cand c{-1.0, 0.0, -1.0};
  if (t < nb) {
    c.m = base[t];
    c.idx = base[ACA_MAXBLK + t];
    c.val = base[(size_t)PVAL * ACA_MAXBLK + t];
  }
  return c;
}

struct PivLds {
  double mx[4], ci[4], cv[4];
  int bb[4], best[4];
};

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Global pivot from candidates held in registers, M the maximum of all
// block maxima (M < 0: nothing eligible): the lowest block whose maximum
// is within the tie tolerance of M gives its candidate; only when that
// candidate falls below the tolerance is the block's range of x rescanned
// (lowest eligible index within the tolerance).
template <typename Skip>
__device__ int pivot_pick(const Cand& c, double M, const double* x, int nb, int n, Skip skip, PivLds& S) {
  const int t = aca_tid(), wv = t >> 6;
  if (!(M >= 0.0)) return n;
  const double thr = M * (1.0 - 1e-10);
  int bb = (t < nb && c.m >= thr) ? t : nb;
  double ci = c.idx, cv = c.val;
  for (int o = 32; o > 0; o >>= 1) {
    const int ob = __shfl_xor(bb, o, 64);
    const double oi = __shfl_xor(ci, o, 64), ov = __shfl_xor(cv, o, 64);
    if (ob < bb) { bb = ob; ci = oi; cv = ov; }
  }
  if ((t & 63) == 0) { S.bb[wv] = bb; S.ci[wv] = ci; S.cv[wv] = cv; }
  __syncthreads();
  int w0 = 0;
#pragma unroll
  for (int w = 1; w < 4; ++w)
    if (S.bb[w] < S.bb[w0]) w0 = w;
  bb = S.bb[w0]; ci = S.ci[w0]; cv = S.cv[w0];
  if (bb >= nb) return n;
  const int cand = (int)ci;
  if (cand < n && cv >= thr) return cand;
  int best = n;
  const int e = bb * ACA_TILE + t;
  if (t < ACA_TILE && e < n && !skip(e) && fabs(x[e]) >= thr) best = e;
  for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((t & 63) == 0) S.best[wv] = best;
  __syncthreads();
  best = min(min(S.best[0], S.best[1]), min(S.best[2], S.best[3]));
  return best;
}

// ------------------------------------------------------------ row launch
// Decision of the row launch, taken alike by every block:
//   START: sample row i;
//   COL:   the next row pivot is the unused row maximising |u_(k-1)| (from
//          the column launch's block candidates); no row when k reached
//          the term cap or no row is eligible.  The row is sampled before
//          the column launch has run the stopping test of term k-1, and is
//          discarded when that test stops the iteration;
//   PROBE: resolve the probe check of the column launch before: largest
//          residual above the threshold among the probes (lowest index
//          within the tie tolerance); none -> converged, term cap ->
//          capped, else sample that probe's row.
// The block given `writer` stores the outcome in ctl[1].
struct RowDec {
  int go, i, k, next;   // next < 0: the cross has stopped
};

template <bool TAB>
__device__ RowDec aca_row_decide(const AcaInst& I, bool writer) {
  __shared__ AcaCtl sc;
  __shared__ PivLds S;
  const int t = aca_tid(), wv = t >> 6;
  const Cand c = load_cand(I.part + (size_t)PCOL * ACA_MAXBLK, I.nbcol);
  if (t == 0) sc = I.ctl[0];
  __syncthreads();
  RowDec d{1, sc.i, sc.k, sc.next};
  if (sc.phase != ACA_RUN) {
    if (writer && t == 0) I.ctl[1] = sc;
    d.go = 0; d.next = -1;
    return d;
  }
  const int k = sc.k;
  const int Nx = TAB ? I.nrows : I.g.nx;
  int phase = ACA_RUN, conv = sc.converged, capd = sc.capped, prounds = sc.probe_rounds;
  if (sc.next == ACA_NX_COL) {
    if (k >= sc.kmax) {
      d.go = 0;
    } else {
      const double mw = wave_max(c.m);
      if ((t & 63) == 0) S.mx[wv] = mw;
      __syncthreads();
      const double M = fmax(fmax(S.mx[0], S.mx[1]), fmax(S.mx[2], S.mx[3]));
      const int ip = pivot_pick(c, M, I.U + (size_t)(k - 1) * Nx, I.nbcol, Nx, SkipUsed{I.used, sc.i}, S);
      if (!(M >= 0.0) || ip >= Nx) d.go = 0;
      else d.i = ip;
    }
  } else if (sc.next == ACA_NX_PROBE) {
    const double* pr = I.part + (size_t)PRB * ACA_MAXBLK;
    const int* pri = (const int*)(I.part + (size_t)PRBI * ACA_MAXBLK);
    const int np = I.nprobe;
    double rv[4];
    double m = -1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + FS_THREADS * q;
      rv[q] = (e < np) ? pr[e] : -1.0;
      m = fmax(m, rv[q]);
    }
    m = wave_max(m);
    if ((t & 63) == 0) S.mx[wv] = m;
    __syncthreads();
    m = fmax(fmax(S.mx[0], S.mx[1]), fmax(S.mx[2], S.mx[3]));
    int best = np;
    if (m > 0.0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + FS_THREADS * q;
        if (e < np && rv[q] > 0.0 && rv[q] >= m * (1.0 - 1e-10) && e < best) best = e;
      }
      for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
      if ((t & 63) == 0) S.best[wv] = best;
      __syncthreads();
      best = min(min(S.best[0], S.best[1]), min(S.best[2], S.best[3]));
    }
    if (m <= 0.0 || best >= np) { phase = ACA_DONE; conv = 1; d.go = 0; }
    else if (k >= sc.kmax) { phase = ACA_DONE; capd = 1; d.go = 0; }
    else { prounds += 1; d.i = pri[best]; }
  }
  if (writer && t == 0) {
    AcaCtl o = sc;
    o.i = d.i; o.rowok = d.go; o.phase = phase;
    o.converged = conv; o.capped = capd; o.probe_rounds = prounds;
    I.ctl[1] = o;
  }
  if (phase != ACA_RUN) d.next = -1;
  return d;
}

// One tile of the row launch: the row fiber A[i, :] through the SL-FD
// evaluator, the residual r = A[i,:] - sum_l u_l[i] v_l stored as V[k],
// per-block partials of v_l . r and a per-block pivot candidate; after a
// COL decision also this tile's share of the sums over the column blocks of
// u_l . u_(k-1) (wave w of tile b takes l = 4 b + w, 4 b + w + 4 nbrow, ...).
template <typename T, int W, int DX, bool TAB = false>
__device__ void aca_row_sample(const AcaInst& I, const RowDec& d, int tile) {
  if (d.next < 0) return;
  const GridDev& g = I.g;
  const AdvDev& a = I.a;
  const T* __restrict__ X = (const T*)I.X;
  const T* __restrict__ P = (const T*)I.P;
  const int ld = I.ld, r = I.r;
  const double* __restrict__ U = I.U;
  double* __restrict__ V = I.V;
  double* __restrict__ part = I.part;
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ double acc4[4][FS_SAMPLES];
  __shared__ double rres[FS_SAMPLES];
  const int t = aca_tid();
  const int k = d.k, i = d.i;
  const int Nx = TAB ? I.nrows : g.nx, Nv = TAB ? I.ncols : g.nv;
  const int J0 = tile * ACA_TILE;
  const int ns = min(ACA_TILE, Nv - J0);
  const int wv = t >> 6, ln = t & 63;
  if (d.go) {
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
  if (d.next == ACA_NX_COL) {
    // gu[l] = sum over the column blocks of (u_l . u_(k-1)), l < k: each
    // lane adds four blocks in order, then a wave butterfly
    const double* pc = part + (size_t)PCOL * ACA_MAXBLK;
    for (int l = 4 * tile + wv; l < k; l += 4 * I.nbrow) {
      const double* q = pc + (size_t)(2 + l) * ACA_MAXBLK;
      double a4 = 0.0;
#pragma unroll
      for (int i4 = 0; i4 < FIN_NB / 64; ++i4) {
        const int b = ln + 64 * i4;
        const double v = q[b];
        a4 += (b < I.nbcol) ? v : 0.0;
      }
      a4 = wave_sum(a4);
      if (ln == 0) part[(size_t)GSU * ACA_MAXBLK + l] = a4;
    }
  }
}

// --------------------------------------------------------- column launch
// Decision of the column launch, taken alike by every block.  First the
// stopping test of term k-1 when the column launch before sampled it
// (COL): ||S||^2 += 2 sum_(l<k-1) (u_l . u)(v_l . v) + |u|^2 |v|^2 from the
// finished sums; |u| |v| <= tol ||S|| -> probe check, term cap -> capped,
// no row from the row launch -> stop.  Otherwise the row i that the row
// launch sampled is accepted: the column pivot j comes from the row
// candidates (lowest index within a relative 1e-10 of the maximum), and a
// row already reproduced (|r_j| below the threshold) leads to the probe
// check.  The block given `writer` stores the outcome in ctl[0].
enum { ACA_A_COL = 0, ACA_A_PROBE = 1, ACA_A_NONE = 2 };
struct ColDec {
  int act, i, j, k;
  double norm2, tol;
  int also;   // row marked used by this launch (excluded from the probes), or -1
};

template <bool TAB>
__device__ ColDec aca_col_decide(const AcaInst& I, bool writer) {
  enum { A_COL = 0, A_PROBE = 1, A_CAP = 2, A_STOP = 3 };
  __shared__ AcaCtl sc;
  __shared__ PivLds S;
  __shared__ double s_norm2;
  __shared__ int s_act;
  const int t = aca_tid(), wv = t >> 6;
  const double* __restrict__ part = I.part;
  const Cand c = load_cand(part, I.nbrow);
  // the finished sums of the stopping test, both parities of v
  double gu0 = 0.0, gu1 = 0.0, ga0 = 0.0, ga1 = 0.0, gb0 = 0.0, gb1 = 0.0;
  if (t < 64) {
    gu0 = part[(size_t)GSU * ACA_MAXBLK + t];
    gu1 = part[(size_t)GSU * ACA_MAXBLK + 64 + t];
    ga0 = part[(size_t)GSUM * ACA_MAXBLK + t];
    ga1 = part[(size_t)GSUM * ACA_MAXBLK + 64 + t];
    gb0 = part[(size_t)GSUM1 * ACA_MAXBLK + t];
    gb1 = part[(size_t)GSUM1 * ACA_MAXBLK + 64 + t];
  }
  if (t == 0) sc = I.ctl[1];
  __syncthreads();
  ColDec d{ACA_A_NONE, sc.i, 0, sc.k, sc.norm2, sc.tol, -1};
  if (sc.phase != ACA_RUN) {
    if (writer && t == 0) I.ctl[0] = sc;
    return d;
  }
  const int k = sc.k;
  const int Nx = TAB ? I.nrows : I.g.nx, Nv = TAB ? I.ncols : I.g.nv;
  const double mw = wave_max(c.m);
  if ((t & 63) == 0) S.mx[wv] = mw;
  if (wv == 0) {
    int act = sc.rowok ? A_COL : A_STOP;
    double norm2 = sc.norm2;
    if (sc.next == ACA_NX_COL) {
      const int kk = k - 1;
      const double gv0 = (kk & 1) ? gb0 : ga0, gv1 = (kk & 1) ? gb1 : ga1;
      double cc = (t < kk) ? gu0 * gv0 : 0.0;
      if (t + 64 < kk) cc += gu1 * gv1;
      cc = wave_sum(cc);
      const double guk = __shfl(kk < 64 ? gu0 : gu1, kk & 63, 64);
      const double gvk = __shfl(kk < 64 ? gv0 : gv1, kk & 63, 64);
      const double nk = guk * gvk;
      norm2 = sc.norm2 + 2.0 * cc + nk;
      if (sqrt(nk) <= sc.tol * sqrt(fmax(norm2, 0.0))) act = A_PROBE;
      else if (k >= sc.kmax) act = A_CAP;
      else act = sc.rowok ? A_COL : A_STOP;
    }
    if (t == 0) { s_norm2 = norm2; s_act = act; }
  }
  __syncthreads();
  const double M = fmax(fmax(S.mx[0], S.mx[1]), fmax(S.mx[2], S.mx[3]));
  const double norm2 = s_norm2;
  const int act = s_act;
  d.norm2 = norm2;
  if (act == A_CAP || act == A_STOP) {
    if (writer && t == 0) {
      AcaCtl o = sc;
      o.norm2 = norm2; o.phase = ACA_DONE;
      if (act == A_CAP) o.capped = 1;
      I.ctl[0] = o;
    }
    return d;
  }
  const int i = sc.i;
  int j = Nv;
  bool zero_row = false;
  if (act == A_COL) {
    j = pivot_pick(c, M, I.V + (size_t)k * Nv, I.nbrow, Nv, NoSkip{}, S);
    const double thr = sc.tol * sqrt(norm2) / sqrt((double)Nx * (double)Nv);
    zero_row = (M == 0.0 || M <= thr || j >= Nv);
  }
  const bool probe = act == A_PROBE || zero_row;
  const bool stop_now = probe && (k == 0 || I.nprobe <= 0);
  if (writer && t == 0) {
    AcaCtl o = sc;
    o.norm2 = norm2;
    if (act == A_COL) {
      I.used[i] = 1;
      o.iters += 1; o.samples += Nv; o.j = j; o.pivot = M;
    }
    if (stop_now) {
      o.phase = ACA_DONE; o.converged = 1;
    } else if (probe) {
      o.next = ACA_NX_PROBE; o.samples += I.nprobe;
    } else {
      o.next = ACA_NX_COL; o.k = k + 1; o.samples += Nx;
      if (I.piv) { I.piv[2 * k] = i; I.piv[2 * k + 1] = j; }
    }
    I.ctl[0] = o;
  }
  d.act = stop_now ? ACA_A_NONE : (probe ? ACA_A_PROBE : ACA_A_COL);
  d.j = j;
  d.also = zero_row ? i : -1;
  return d;
}

// One tile of the column launch.  Probe check: this tile's share of the
// probe entries (base = 64 tile, 64 (tile + nbcol), ...), each residual
// above the threshold in a row not yet used stored as |residual|, else -1.
// Column: the column fiber A[:, j] (Nx entries), its residual scaled by
// 1/r_j stored as U[k], partials of u_l . u and per-block candidates of
// the next row pivot (unused rows), and this tile's share of the sums over
// the row blocks of v_l . v_k for the next stopping test (l = tile,
// tile + nbcol, ...).
template <typename T, int W, int DX, bool TAB = false>
__device__ void aca_col_sample(const AcaInst& I, const ColDec& d, int tile) {
  if (d.act == ACA_A_NONE) return;
  const GridDev& g = I.g;
  const AdvDev& a = I.a;
  const T* __restrict__ X = (const T*)I.X;
  const T* __restrict__ P = (const T*)I.P;
  const int ld = I.ld, r = I.r;
  double* __restrict__ U = I.U;
  const double* __restrict__ V = I.V;
  unsigned char* __restrict__ used = I.used;
  double* __restrict__ part = I.part;
  const int nbrow = I.nbrow;
  __shared__ FsLds<W, DX> L;
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ double acc4[4][FS_SAMPLES];
  __shared__ double ures[FS_SAMPLES];
  const int t = aca_tid();
  const int k = d.k, i = d.i, j = d.j;
  const int Nx = TAB ? I.nrows : g.nx, Nv = TAB ? I.ncols : g.nv;
  const int wv = t >> 6, ln = t & 63;
  if (d.act == ACA_A_PROBE) {
    // the quad of a sample splits the l-sum of the approximation
    const double thr2 = d.tol * sqrt(fmax(d.norm2, 0.0)) / sqrt((double)Nx * (double)Nv);
    double* pr = part + (size_t)PRB * ACA_MAXBLK;
    int* pri = (int*)(part + (size_t)PRBI * ACA_MAXBLK);
    const int* __restrict__ probes = I.probes;
    for (int base = tile * FS_SAMPLES; base < I.nprobe; base += I.nbcol * FS_SAMPLES) {
      const int np = min(FS_SAMPLES, I.nprobe - base);
      const int s = t >> 2, q = t & 3;
      int pI = 0, pJ = 0;
      if (s < np) {
        pI = probes[2 * (base + s)];
        pJ = probes[2 * (base + s) + 1];
        int gi[4];
        entry_index<DX, TAB>(I, pI, pJ, gi);
        fs_prepare<W, DX, 4>(g, a, gi, L, s, q);
      }
      double ap = 0.0;
      if (s < np)
        for (int l = q; l < k; l += 4) ap += U[(size_t)l * Nx + pI] * V[(size_t)l * Nv + pJ];
      ap += __shfl_xor(ap, 1, 4);
      ap += __shfl_xor(ap, 2, 4);
      __syncthreads();
      fs_evaluate_team<T, W, DX>(I.team, X, P, ld, r, L, np);
      __syncthreads();
      if (s < np && q == 0) {
        const double v = L.val[s] - ap;
        const bool bad = fabs(v) > thr2 && !used[pI] && pI != d.also;
        pr[base + s] = bad ? fabs(v) : -1.0;
        pri[base + s] = pI;
      }
      __syncthreads();
    }
    return;
  }
  const int I0 = tile * ACA_TILE;
  const int ns = min(ACA_TILE, Nx - I0);
  // earlier column vectors u_l[I] and v_l[j] (loads in flight during the feet)
  double ul[ACA_LREG], vj[ACA_LREG];
#pragma unroll
  for (int m = 0; m < ACA_LREG; ++m) {
    const int l = wv + 4 * m;
    ul[m] = (l < k && ln < ns) ? U[(size_t)l * Nx + I0 + ln] : 0.0;
    vj[m] = (l < k) ? V[(size_t)l * Nv + j] : 0.0;
  }
  const double piv = V[(size_t)k * Nv + j];
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
  // gv[l] = sum over the row blocks of (v_l . v_k), l <= k
  double* gs = part + (size_t)((k & 1) ? GSUM1 : GSUM) * ACA_MAXBLK;
  for (int l = tile; l <= k; l += I.nbcol) {
    const double* q = part + (size_t)(2 + l) * ACA_MAXBLK;
    double acc = 0.0;
    for (int b = t; b < nbrow; b += FS_THREADS) acc += q[b];
    acc = wave_sum(acc);
    if (ln == 0) acc4[wv][0] = acc;
    __syncthreads();
    if (t == 0) gs[l] = ((acc4[0][0] + acc4[1][0]) + acc4[2][0]) + acc4[3][0];
    __syncthreads();
  }
}

// --------------------------------------------------- single-instance kernels
template <typename T, int W, int DX, bool TAB = false>
__global__ __launch_bounds__(FS_THREADS) void k_aca_row(AcaInst I) {
  const RowDec d = aca_row_decide<TAB>(I, blockIdx.x == 0);
  aca_row_sample<T, W, DX, TAB>(I, d, blockIdx.x);
}
template <typename T, int W, int DX, bool TAB = false>
__global__ __launch_bounds__(FS_THREADS) void k_aca_col(AcaInst I) {
  const ColDec d = aca_col_decide<TAB>(I, blockIdx.x == 0);
  aca_col_sample<T, W, DX, TAB>(I, d, blockIdx.x);
  // thread 0 of block 0 wrote ctl[0] in this launch, so it reads the
  // current phase; the host waits for seq, then reads the phase
  if (I.phase_host && blockIdx.x == 0 && threadIdx.x == 0) {
    volatile int* ph = I.phase_host;
    ph[0] = I.ctl[0].phase;
    __threadfence_system();
    ph[1] = I.seq;
  }
}

}  // namespace slar
