// Block-cooperative SL-FD evaluation from node frames.
//
// For a tensor in frame form F[I, J] = sum_c X[I][c] P[J][c] the SL-FD
// update at a grid point is eq. (tp_interp) of F at the foot x*:
//   f(x*) = sum_{x-stencil} W_x X[rows_x] . sum_{v-stencil} W_v P[rows_v],
// i.e. a stencil-weighted gather of w^dx rows of X and w^dv rows of P
// followed by one length-r dot product.  One block of 256 threads evaluates
// 64 samples per round: 64 threads trace the feet (FP64) and write stencil
// rows/weights to LDS, then teams of TEAM lanes (4 columns per lane per
// pass, float4 or 2 x double2 loads) gather the rows and reduce the dot
// product with cross-lane shuffles.  The team width trades idle lanes at
// small rank (r < 4 TEAM) against samples per team; 16 is the default.
#pragma once
#include "slar_internal.h"
#include "dpp.h"

namespace slar {

constexpr int FS_SAMPLES = 64;   // samples per round
constexpr int FS_THREADS = 256;

template <int W, int DX>
struct FsLds {
  static constexpr int RX = (DX == 2) ? W * W : W;
  int xrow[FS_SAMPLES][RX];
  int vrow[FS_SAMPLES][RX];
  double xw[FS_SAMPLES][RX];
  double vw[FS_SAMPLES][RX];
  double val[FS_SAMPLES];
};

// Phase 1 for one sample: grid multi-index -> stencil rows and weights.
// NL = 4: the four lanes of a quad share the foot computation (all pass the
// same sample) and the LDS writes.
template <int W, int DX, int NL = 1>
__device__ __forceinline__ void fs_prepare(const GridDev& g, const AdvDev& a, const int* gidx,
                                           FsLds<W, DX>& L, int s, int lane = 0) {
  double ft[4];
  foot_of<DX, NL>(g, a, gidx, ft, lane);
  int r[4][W];
  double w[4][W];
#pragma unroll
  for (int m = 0; m < 2 * DX; ++m) stencil_of<W>(g, a, m, ft[m], gidx[m], r[m], w[m]);
  if (DX == 1) {
    if (lane != 0) return;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      L.xrow[s][b] = r[0][b]; L.xw[s][b] = w[0][b];
      L.vrow[s][b] = r[1][b]; L.vw[s][b] = w[1][b];
    }
  } else {
    // the W^2 entries are shared out over the lanes of the quad
    const int n1 = g.n[1], n3 = g.n[3];
#pragma unroll
    for (int p = 0; p < W; ++p)
#pragma unroll
      for (int q = 0; q < W; ++q) {
        const int e = p * W + q;
        if (NL == 1 || (e % NL) == lane) {
          L.xrow[s][e] = r[0][p] * n1 + r[1][q];
          L.xw[s][e] = w[0][p] * w[1][q];
          L.vrow[s][e] = r[2][p] * n3 + r[3][q];
          L.vw[s][e] = w[2][p] * w[3][q];
        }
      }
  }
}

static_assert(FS_THREADS == 4 * FS_SAMPLES, "one lane quad per sample in the cooperative prepare");

template <typename T> struct Vec4;
template <> struct Vec4<float> {
  static __device__ __forceinline__ void load(const float* p, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <> struct Vec4<double> {
  static __device__ __forceinline__ void load(const double* p, double* o) {
    const double2 v0 = *reinterpret_cast<const double2*>(p);
    const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
    o[0] = v0.x; o[1] = v0.y; o[2] = v1.x; o[3] = v1.y;
  }
};

// Phase 2: values of the prepared samples [0, ns) into L.val (FP64).
// Tables are [rows][ld] with ld % 4 == 0 and zero columns beyond r.  A team
// takes one sample per pass: all its row loads are issued before the first
// FMA.  (Two samples in flight per team for FP32 tables doubled the
// registers and lost more occupancy than it saved in L2 latency, both in
// the cross approximation's fibers and for scattered requests.)  The
// team's partial dot products are summed with DPP row exchanges.
template <typename T, int W, int DX, int TEAM = 16>
__device__ __forceinline__ void fs_evaluate(const T* __restrict__ X, const T* __restrict__ P,
                                            int ld, int r, FsLds<W, DX>& L, int ns) {
  static_assert(TEAM == 4 || TEAM == 8 || TEAM == 16, "team width");
  constexpr int RX = FsLds<W, DX>::RX;
  constexpr int NT = FS_THREADS / TEAM;
  const int team = threadIdx.x / TEAM;
  const int lane = threadIdx.x % TEAM;
  for (int s = team; s < ns; s += NT) {
    T acc = 0;
    for (int c0 = lane * 4; c0 < r; c0 += 4 * TEAM) {
      T vx[RX][4], vp[RX][4];
#pragma unroll
      for (int b = 0; b < RX; ++b) {
        Vec4<T>::load(X + (size_t)L.xrow[s][b] * ld + c0, vx[b]);
        Vec4<T>::load(P + (size_t)L.vrow[s][b] * ld + c0, vp[b]);
      }
      T y[4] = {0, 0, 0, 0}, z[4] = {0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < RX; ++b) {
        const T wx = (T)L.xw[s][b];
        const T wv = (T)L.vw[s][b];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          y[e] += wx * vx[b][e];
          z[e] += wv * vp[b][e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) acc += y[e] * z[e];
    }
    const T tot = group_sum<TEAM>(acc);
    if (lane == 0) L.val[s] = (double)tot;
  }
}

// Runtime choice of the team width (uniform across the block).
template <typename T, int W, int DX>
__device__ __forceinline__ void fs_evaluate_team(int team, const T* __restrict__ X,
                                                 const T* __restrict__ P, int ld, int r,
                                                 FsLds<W, DX>& L, int ns) {
  if (team == 4) fs_evaluate<T, W, DX, 4>(X, P, ld, r, L, ns);
  else if (team == 8) fs_evaluate<T, W, DX, 8>(X, P, ld, r, L, ns);
  else fs_evaluate<T, W, DX, 16>(X, P, ld, r, L, ns);
}

}  // namespace slar
