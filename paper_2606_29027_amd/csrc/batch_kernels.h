// Kernels of the batched multi-instance cross approximation: the
// preparation launch (FP32 tables, combined field, cleared marks and control
// blocks of every instance), the persistent row / column launches that walk
// a table of (instance, fiber tile) work items with the one-instance bodies
// of aca.h, and the active-instance count.
#pragma once
#include "aca.h"

namespace slar {

struct BItem {
  int q;    // instance
  int t0;   // first fiber tile (ACA_TILE entries)
  int nt;   // tiles
  int pad;
};

// Per-instance inputs of the preparation kernel.
struct BPrep {
  const double* X;    // source frames, FP64 [rows][ldin]
  const double* P;
  int ldin, r, ldt, nx, nv, dx;
  float* X32;         // FP32 tables [rows][ldt], zero beyond r
  float* P32;
  const double* E0;   // field terms (may be null)
  const double* E1;
  double c0, c1;
  double* Eeff;
  unsigned char* used;
  AcaCtl* ctl;
  int kmax;
  double tol;
};

struct BSummary {
  int k, iters, probe_rounds, converged, capped, phase;
  long long samples;
  double norm2;
};

// -------------------------------------------------------------- kernels
// Block (x, q) strides over instance q: FP32 tables, effective field,
// cleared row marks; block (0, q) initialises the control block.
__global__ __launch_bounds__(256) void k_batch_prep(const BPrep* __restrict__ prep) {
  const BPrep& p = prep[blockIdx.y];
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nX = (long long)p.nx * p.ldt, nP = (long long)p.nv * p.ldt;
  for (long long e = e0; e < nX; e += stride) {
    const int row = (int)(e / p.ldt), c = (int)(e % p.ldt);
    p.X32[e] = (float)((c < p.r) ? p.X[(long long)row * p.ldin + c] : 0.0);
  }
  for (long long e = e0; e < nP; e += stride) {
    const int row = (int)(e / p.ldt), c = (int)(e % p.ldt);
    p.P32[e] = (float)((c < p.r) ? p.P[(long long)row * p.ldin + c] : 0.0);
  }
  // combined field, node-interleaved [Nx][dx] (inputs planar [dx][Nx])
  const long long nE = (long long)p.dx * p.nx;
  for (long long e = e0; e < nE; e += stride) {
    const long long in = (e % p.dx) * p.nx + e / p.dx;
    double v = 0.0;
    if (p.E0 != nullptr) {
      v = p.c0 * p.E0[in];
      if (p.E1 != nullptr) v = v + p.c1 * p.E1[in];
    }
    p.Eeff[e] = v;
  }
  for (long long e = e0; e < p.nx; e += stride) p.used[e] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    AcaCtl* c = p.ctl;
    c->phase = ACA_RUN; c->k = 0; c->i = 0; c->j = 0;
    c->iters = 0; c->probe_rounds = 0; c->converged = 0; c->capped = 0;
    c->next = ACA_NX_START; c->rowok = 0; c->kmax = p.kmax; c->pad = 0;
    c->pivot = 0.0; c->norm2 = 0.0; c->tol = p.tol; c->samples = 0;
  }
}

// Both kernels hold the 1D1V and 2D2V bodies; the column kernel would take
// 260 registers (one wave per SIMD).  Bounded to two waves per SIMD both fit
// 256 VGPRs without spilling, since the bodies read the thread index through
// aca_tid() and nothing derived from it is kept across the item loop.
__global__ __launch_bounds__(FS_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_row(const AcaInst* __restrict__ insts,
                                                           const BItem* __restrict__ items, int nitems) {
  for (int t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BItem w = items[t];
    const AcaInst& I = insts[w.q];
    __syncthreads();
    const RowDec d = aca_row_decide<false>(I, w.t0 == 0);   // once per item
    for (int u = 0; u < w.nt; ++u) {
      __syncthreads();
      if (I.g.dx == 1) aca_row_sample<float, 3, 1>(I, d, w.t0 + u);
      else aca_row_sample<float, 3, 2>(I, d, w.t0 + u);
    }
  }
}

__global__ __launch_bounds__(FS_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_col(const AcaInst* __restrict__ insts,
                                                           const BItem* __restrict__ items, int nitems) {
  for (int t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BItem w = items[t];
    const AcaInst& I = insts[w.q];
    __syncthreads();
    const ColDec d = aca_col_decide<false>(I, w.t0 == 0);   // once per item
    for (int u = 0; u < w.nt; ++u) {
      __syncthreads();
      if (I.g.dx == 1) aca_col_sample<float, 3, 1>(I, d, w.t0 + u);
      else aca_col_sample<float, 3, 2>(I, d, w.t0 + u);
    }
  }
}

// Number of instances still running, and (when sum != null) their summaries.
__global__ __launch_bounds__(256) void k_batch_status(const AcaInst* __restrict__ insts, int count,
                                                      int* __restrict__ active, BSummary* __restrict__ sum) {
  __shared__ int red[4];
  int a = 0;
  for (int q = threadIdx.x; q < count; q += blockDim.x) {
    const AcaCtl* c = insts[q].ctl;
    a += (c->phase != ACA_DONE) ? 1 : 0;
    if (sum) {
      BSummary s;
      s.k = c->k; s.iters = c->iters; s.probe_rounds = c->probe_rounds;
      s.converged = c->converged; s.capped = c->capped; s.phase = c->phase;
      s.samples = c->samples; s.norm2 = c->norm2;
      sum[q] = s;
    }
  }
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) *active = red[0] + red[1] + red[2] + red[3];
}


}  // namespace slar
