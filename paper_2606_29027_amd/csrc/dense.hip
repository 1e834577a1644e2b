// Small dense FP64 linear algebra for the truncation: split-K Gram
// matrices, Cholesky-QR helpers, one-sided
// Jacobi SVD and two-sided Jacobi symmetric eigensolver.  All single-block
// factorizations keep their matrix in LDS (gfx950: 160 KB per CU).
#include <algorithm>

#include "slar_internal.h"
#include "dense.h"
#include "dpp.h"
#include "group.h"

namespace slar {

// ------------------------------------------------------------ Gram
// G = A A^T for A with k <= 128 rows and a long column range, element
// (i, j) read through an addressing functor.  Stage 1: block b takes the
// 32-column chunks b, b + grid, ..., stages each chunk (k x 32) in LDS and
// accumulates its k x k partial in registers (16 x 16 threads, MT x MT
// outputs each); stage 2 sums the partials in block order.  Both triangles
// are computed with the same products in the same order, so G is exactly
// symmetric.
constexpr int GR_C = 32;

struct RowMajor {
  const double* A;
  int lda;
  __device__ double operator()(int i, int j) const { return A[(long long)i * lda + j]; }
};
// mode-2 unfolding of a frame Xs[(i1 * nb + i2) * r + c]: row i2, column
// j = i1 * r + c
struct Mode2 {
  const double* X;
  int nb, r;
  __device__ double operator()(int i, int j) const {
    const int i1 = j / r, c = j - i1 * r;
    return X[((long long)i1 * nb + i) * r + c];
  }
};

// either addressing, chosen per problem (grouped launches)
struct AnyAddr {
  const double* A;
  int lda, nb, r, mode2;
  __device__ double operator()(int i, int j) const {
    if (mode2) {
      const int i1 = j / r, c = j - i1 * r;
      return A[((long long)i1 * nb + i) * r + c];
    }
    return A[(long long)i * lda + j];
  }
};

// block blk of nblk: chunks blk, blk + nblk, ...; partial at part + blk k^2
template <int MT, class Addr>
__device__ __forceinline__ void gram_part_dev(int k, int n, const Addr& A, double* __restrict__ part, int blk,
                                              int nblk) {
  __shared__ double S[16 * MT][GR_C + 1];
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  double acc[MT][MT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = 0.0;
  const int nchunk = (n + GR_C - 1) / GR_C;
  for (int ch = blk; ch < nchunk; ch += nblk) {
    const int j0 = ch * GR_C;
    __syncthreads();
    for (int e = t; e < 16 * MT * GR_C; e += 256) {
      const int i = e / GR_C, c = e - (e / GR_C) * GR_C;
      S[i][c] = (i < k && j0 + c < n) ? A(i, j0 + c) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < GR_C; ++c) {
      double x[MT], y[MT];
#pragma unroll
      for (int a = 0; a < MT; ++a) { x[a] = S[tr + 16 * a][c]; y[a] = S[tc + 16 * a][c]; }
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < MT; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
    }
  }
  double* out = part + (size_t)blk * k * k;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) {
      const int i = tr + 16 * a, j = tc + 16 * b;
      if (i < k && j < k) out[i * k + j] = acc[a][b];
    }
}

template <int MT, class Addr>
__global__ __launch_bounds__(256) void k_gram_part(int k, int n, Addr A, double* __restrict__ part) {
  gram_part_dev<MT>(k, n, A, part, blockIdx.x, gridDim.x);
}

template <int MT>
__global__ __launch_bounds__(256) void k_gram_part_group(const GramDesc* __restrict__ D,
                                                         const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const GramDesc g = D[d];
  const AnyAddr A{g.A, g.lda, g.nb, g.r, g.mode2};
  gram_part_dev<MT>(g.k, g.n, A, g.part, b - first[d], g.nblk);
}

// 64 outputs per block, four waves each summing every fourth partial
// (coalesced over the outputs), combined in a fixed order.
__device__ __forceinline__ void gram_sum_dev(int kk, int nblk, const double* __restrict__ part,
                                             double* __restrict__ G, int blk) {
  __shared__ double q4[4][64];
  const int t = threadIdx.x, ln = t & 63, w = t >> 6;
  const int e = blk * 64 + ln;
  double acc = 0.0;
  if (e < kk) {
#pragma unroll 8
    for (int b = w; b < nblk; b += 4) acc += part[(size_t)b * kk + e];
  }
  q4[w][ln] = acc;
  __syncthreads();
  if (w == 0 && e < kk) G[e] = ((q4[0][ln] + q4[1][ln]) + q4[2][ln]) + q4[3][ln];
}

__global__ __launch_bounds__(256) void k_gram_sum(int kk, int nblk, const double* __restrict__ part,
                                                  double* __restrict__ G) {
  gram_sum_dev(kk, nblk, part, G, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_gram_sum_group(const GramDesc* __restrict__ D,
                                                        const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const GramDesc g = D[d];
  gram_sum_dev(g.k * g.k, g.nblk, g.part, g.G, b - first[d]);
}

hipError_t gram_part_group_launch(hipStream_t s, bool mt8, const GramDesc* d, const int* first, int nd,
                                  int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  if (mt8) k_gram_part_group<8><<<nblocks, 256, 0, s>>>(d, first, nd);
  else k_gram_part_group<4><<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t gram_sum_group_launch(hipStream_t s, const GramDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_gram_sum_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

// part: scratch for the per-block partials, cap doubles (the block count
// shrinks to fit).
template <class Addr>
static hipError_t gram_launch(hipStream_t s, const Scratch& part, int k, int n, Addr A, double* G) {
  if (k < 1 || k > 128 || n < 1) return hipErrorInvalidValue;
  const int nchunk = (n + GR_C - 1) / GR_C;
  int nblk = std::min(nchunk, 128);
  while (nblk > 1 && (size_t)nblk * k * k > part.cap) nblk /= 2;
  if ((size_t)nblk * k * k > part.cap) return hipErrorInvalidValue;
  if (k <= 64) k_gram_part<4><<<nblk, 256, 0, s>>>(k, n, A, part.p);
  else k_gram_part<8><<<nblk, 256, 0, s>>>(k, n, A, part.p);
  k_gram_sum<<<(k * k + 63) / 64, 256, 0, s>>>(k * k, nblk, part.p, G);
  return hipGetLastError();
}

// Gram G = A A^T for A = [k][n] row vectors (long n).
hipError_t gram_rows(hipStream_t s, const Scratch& part, int k, int n, const double* A, int lda,
                     double* G) {
  return gram_launch(s, part, k, n, RowMajor{A, lda}, G);
}

// Gram of the mode-2 unfolding of X[(i1 * nb + i2) * r + c] (i1 < na):
// G[i2][i2'] = sum_{i1, c} X[i1, i2, c] X[i1, i2', c].
hipError_t gram_mode2(hipStream_t s, const Scratch& part, int na, int nb, int r, const double* X,
                      double* G) {
  return gram_launch(s, part, nb, na * r, Mode2{X, nb, r}, G);
}

// --------------------------------------------------- Cholesky-QR helpers

// From Gram G (k x k): column scaling d = sqrt(diag G), Cholesky of
// D^-1 G D^-1 = L L^T.  Writes Linv_scaled = L^-1 D^-1 (k x k, lower) and
// R = L^T D (upper).  A zero column keeps d = 1 and a unit pivot.
__device__ __forceinline__ void chol_inv_dev(int k, const double* __restrict__ G, double* __restrict__ Linv,
                                             double* __restrict__ R, const double* __restrict__ Rprev) {
  __shared__ double L[SLAR_KMAX][SLAR_KMAX + 1];
  __shared__ double Li[SLAR_KMAX][SLAR_KMAX + 1];
  __shared__ double Rp[SLAR_KMAX][SLAR_KMAX + 1];
  __shared__ double d[SLAR_KMAX];
  const int t = threadIdx.x;
  for (int i = t; i < k; i += blockDim.x) {
    const double g = G[i * k + i];
    d[i] = g > 0.0 ? sqrt(g) : 1.0;
  }
  if (Rprev != nullptr)
    for (int e = t; e < k * k; e += blockDim.x) Rp[e / k][e % k] = Rprev[e];
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    L[i][j] = G[e] / (d[i] * d[j]);
  }
  __syncthreads();
  // left-looking (Crout) Cholesky, lower triangle in place: column c takes
  //   t_i = S[i][c] - sum_{m<c} L[i][m] L[c][m]   (i >= c; a quad of lanes
  //   per row, every fourth term, DPP quad sum)
  // then L[c][c] = sqrt(t_c) (1 for a pivot <= 1e-300) and L[i][c] = t_i / L[c][c]
  {
    __shared__ double tcol[SLAR_KMAX];
    const int sub = t & 3;
    for (int c = 0; c < k; ++c) {
      for (int i = c + (t >> 2); i < k; i += blockDim.x >> 2) {
        double s = 0.0;
        for (int m = sub; m < c; m += 4) s += L[i][m] * L[c][m];
        s += dpp_move<0xB1>(s);
        s += dpp_move<0x4E>(s);
        if (sub == 0) tcol[i] = L[i][c] - s;
      }
      __syncthreads();
      const double v = tcol[c];
      const double dc = v > 1e-300 ? sqrt(v) : 1.0;
      for (int i = c + t; i < k; i += blockDim.x) L[i][c] = (i == c) ? dc : tcol[i] / dc;
      __syncthreads();
    }
  }
  // inverse of lower triangular L, column by column (forward substitution):
  //   X[j][j] = 1 / L[j][j],  X[i][j] = -(sum_{j<=m<i} L[i][m] X[m][j]) / L[i][i]
  // A quad of lanes owns column j (every fourth term of each sum, then a
  // DPP quad sum); the recurrence stays inside the quad's wave, whose LDS
  // accesses complete in order, so no block barrier is needed.
  {
    const int sub = t & 3;
    for (int j = t >> 2; j < k; j += blockDim.x >> 2) {
      for (int i = sub; i < j; i += 4) Li[i][j] = 0.0;
      if (sub == 0) Li[j][j] = 1.0 / L[j][j];
      for (int i = j + 1; i < k; ++i) {
        double s = 0.0;
        for (int m = j + sub; m < i; m += 4) s += L[i][m] * Li[m][j];
        s += dpp_move<0xB1>(s);
        s += dpp_move<0x4E>(s);
        if (sub == 0) Li[i][j] = -s / L[i][i];
      }
    }
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    Linv[e] = Li[i][j] / d[j];
    // R = L^T D (upper)
    if (Rprev == nullptr) R[e] = (i <= j) ? L[j][i] * d[j] : 0.0;
  }
  if (Rprev != nullptr) {
    // R_total = (L^T D) Rprev: four adjacent outputs of one row per thread
    // share the loads of (L^T D)[i][m] and keep four independent sums
    const int q4 = (k + 3) / 4;
    for (int w = t; w < k * q4; w += blockDim.x) {
      const int i = w / q4, j0 = 4 * (w % q4);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int m = i; m < k; ++m) {
        const double l = L[m][i] * d[m];
        a0 += l * Rp[m][j0];
        a1 += l * Rp[m][min(j0 + 1, k - 1)];
        a2 += l * Rp[m][min(j0 + 2, k - 1)];
        a3 += l * Rp[m][min(j0 + 3, k - 1)];
      }
      double* r = R + (size_t)i * k + j0;
      r[0] = a0;
      if (j0 + 1 < k) r[1] = a1;
      if (j0 + 2 < k) r[2] = a2;
      if (j0 + 3 < k) r[3] = a3;
    }
  }
}

// The same factorisation for SLAR_KMAX < k <= 128 (cross approximations
// that ran past the HT rank cap) in one LDS array: L in the lower
// triangle, L^-1 transposed in the strict upper triangle (Li[i][j] at
// A[j][i], i > j) with its diagonal in li_d; Rprev is read from global
// memory.  Same arithmetic and summation order as k_chol_inv.
constexpr int CHOL_BIG = SLAR_CROSS_KMAX;
__device__ __forceinline__ void chol_inv_big_dev(int k, const double* __restrict__ G,
                                                 double* __restrict__ Linv, double* __restrict__ R,
                                                 const double* __restrict__ Rprev) {
  __shared__ double A[CHOL_BIG][CHOL_BIG + 1];
  __shared__ double d[CHOL_BIG], tcol[CHOL_BIG], li_d[CHOL_BIG];
  const int t = threadIdx.x;
  for (int i = t; i < k; i += blockDim.x) {
    const double g = G[i * k + i];
    d[i] = g > 0.0 ? sqrt(g) : 1.0;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    if (j <= i) A[i][j] = G[e] / (d[i] * d[j]);
  }
  __syncthreads();
  const int sub = t & 3;
  for (int c = 0; c < k; ++c) {
    for (int i = c + (t >> 2); i < k; i += blockDim.x >> 2) {
      double sm = 0.0;
      for (int m = sub; m < c; m += 4) sm += A[i][m] * A[c][m];
      sm += dpp_move<0xB1>(sm);
      sm += dpp_move<0x4E>(sm);
      if (sub == 0) tcol[i] = A[i][c] - sm;
    }
    __syncthreads();
    const double v = tcol[c];
    const double dc = v > 1e-300 ? sqrt(v) : 1.0;
    for (int i = c + t; i < k; i += blockDim.x) A[i][c] = (i == c) ? dc : tcol[i] / dc;
    __syncthreads();
  }
  // forward substitution per column j (a quad of lanes), into the upper triangle
  for (int j = t >> 2; j < k; j += blockDim.x >> 2) {
    if (sub == 0) li_d[j] = 1.0 / A[j][j];
    for (int i = j + 1; i < k; ++i) {
      double sm = 0.0;
      for (int m = j + sub; m < i; m += 4) sm += A[i][m] * (m == j ? li_d[j] : A[j][m]);
      sm += dpp_move<0xB1>(sm);
      sm += dpp_move<0x4E>(sm);
      if (sub == 0) A[j][i] = -sm / A[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    const double li = (i == j) ? li_d[i] : (i > j ? A[j][i] : 0.0);
    Linv[e] = li / d[j];
    if (Rprev == nullptr) R[e] = (i <= j) ? A[j][i == j ? j : i] * d[j] : 0.0;
  }
  if (Rprev != nullptr) {
    // R_total = (L^T D) Rprev, (L^T D)[i][m] = L[m][i] d[m] for m >= i
    for (int e = t; e < k * k; e += blockDim.x) {
      const int i = e / k, j = e % k;
      double acc = 0.0;
      for (int m = i; m < k; ++m) acc += (m == i ? A[i][i] : A[m][i]) * d[m] * Rprev[(size_t)m * k + j];
      R[e] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_chol_inv(int k, const double* __restrict__ G,
                                                  double* __restrict__ Linv, double* __restrict__ R,
                                                  const double* __restrict__ Rprev) {
  chol_inv_dev(k, G, Linv, R, Rprev);
}
__global__ __launch_bounds__(256) void k_chol_inv_big(int k, const double* __restrict__ G,
                                                      double* __restrict__ Linv, double* __restrict__ R,
                                                      const double* __restrict__ Rprev) {
  chol_inv_big_dev(k, G, Linv, R, Rprev);
}
// one block per descriptor
template <bool BIG>
__global__ __launch_bounds__(256) void k_chol_inv_group(const CholDesc* __restrict__ D) {
  const CholDesc d = D[blockIdx.x];
  if (BIG) chol_inv_big_dev(d.k, d.G, d.Linv, d.R, d.Rprev);
  else chol_inv_dev(d.k, d.G, d.Linv, d.R, d.Rprev);
}

hipError_t chol_inv(hipStream_t s, int k, const double* G, double* Linv, double* R,
                    const double* Rprev) {
  if (k < 1 || k > SLAR_CROSS_KMAX) return hipErrorInvalidValue;
  if (k <= SLAR_KMAX)
    k_chol_inv<<<1, 256, 0, s>>>(k, G, Linv, R, Rprev);
  else
    k_chol_inv_big<<<1, 256, 0, s>>>(k, G, Linv, R, Rprev);
  return hipGetLastError();
}

hipError_t chol_inv_group(hipStream_t s, int count, const CholDesc* d, bool big) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  if (big) k_chol_inv_group<true><<<count, 256, 0, s>>>(d);
  else k_chol_inv_group<false><<<count, 256, 0, s>>>(d);
  return hipGetLastError();
}

// Circle-method round robin on kp (even) players: at step `step` position 0
// holds player 0 and position i >= 1 holds player 1 + (i - 1 + step) mod (kp - 1);
// pair `pid` meets positions pid and kp - 1 - pid.  Every pair meets once
// per kp - 1 steps.
__device__ __forceinline__ int rr_player(int pos, int step, int kp) {
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (kp - 1);
}

// ------------------------------------------- one-sided Jacobi, team form
// Sum over the 16 lanes of a DPP row (every lane gets the total): quad
// exchanges, then the half-row and row mirrors.  Pure VALU data movement,
// so concurrent teams do not queue on the LDS crossbar.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return v;
}

// Reciprocal and reciprocal square root from the hardware estimates with
// two Newton steps each (the estimates carry about half the FP64 mantissa;
// a Jacobi rotation needs c^2 + s^2 = 1 to rounding, not the exact angle).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  const double h = 0.5 * x * r;
  return fma(r, fma(-h, r, 0.5), r);
}

// Columns of C (col-major in LDS, column c at C + c * ldc, n <= 16 RPL
// rows, kp <= 64 columns, kp even) are orthogonalised by cyclic one-sided
// Jacobi rotations in circle-method order; the same rotations are applied
// to V (kv <= 16 VPL rows) when VPL > 0.  512 threads: a team is one
// 16-lane DPP row, team i owns pair i of every step, so a step is one pass
// over registers and one barrier (eight waves keep the SIMDs' issue slots
// for the active teams).
//  * Squared column norms live in nrm2[kp] (LDS): computed exactly at the
//    start of every sweep and updated by each rotation (alpha' = alpha -
//    t gamma, beta' = beta + t gamma), so a step reduces one dot product.
//  * Odd teams visit their register slots shifted by one 16-row block, so
//    the two teams of a half-wave touch disjoint LDS banks whatever their
//    columns (ldc and ldv are multiples of 32 doubles).
// A pair is rotated when |x.y| exceeds the rounding level of its dot
// product (orth |x| |y|) and |x| |y| > floor_abs.  Cyclic Jacobi converges
// quadratically, so a sweep whose rotated pairs all had cosines below
// sqrt(orth) / 8 leaves cosines near orth / 64 for the next one, which then
// rotates nothing: the loop ends there instead of running that sweep.
// s_rot: two LDS flags.  Returns the number of sweeps.
template <int RPL, int VPL>
__device__ int jacobi_cols(double* C, int ldc, int n, int kp, double* V, int ldv, int kv, double orth,
                           double floor_abs, int maxsweep, double* nrm2, int* s_rot) {
  static_assert((RPL & (RPL - 1)) == 0 && (VPL == 0 || (VPL & (VPL - 1)) == 0), "power-of-two slots");
  const int team = threadIdx.x >> 4, lane = threadIdx.x & 15;
  const int odd = team & 1;
  const int nteam = blockDim.x >> 4;
  const int npair = kp / 2;
  const double stop2 = orth / 64.0;   // (sqrt(orth) / 8)^2
  int sweep = 0;
  for (; sweep < maxsweep; ++sweep) {
    if (threadIdx.x == 0) { s_rot[0] = 0; s_rot[1] = 0; }
    for (int c = team; c < kp; c += nteam) {
      const double* cc = C + (size_t)c * ldc;
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = lane + 16 * ((i + odd) & (RPL - 1));
        const double v = (r < n) ? cc[r] : 0.0;
        a += v * v;
      }
      a = row16_sum(a);
      if (lane == 0) nrm2[c] = a;
    }
    __syncthreads();
    bool rotated = false, big = false;
    for (int step = 0; step < kp - 1; ++step) {
      if (team < npair) {
        // rr_player without a division: positions 1 .. kp-1 rotate by step
        int pp = team - 1 + step, qq = kp - 2 - team + step;
        pp -= (pp >= kp - 1) ? kp - 1 : 0;
        qq -= (qq >= kp - 1) ? kp - 1 : 0;
        const int p = (team == 0) ? 0 : 1 + pp;
        const int q = 1 + qq;
        double* cp = C + (size_t)p * ldc;
        double* cq = C + (size_t)q * ldc;
        const double al = nrm2[p], be = nrm2[q];
        double x[RPL], y[RPL];
        double ga = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = lane + 16 * ((i + odd) & (RPL - 1));
          x[i] = (r < n) ? cp[r] : 0.0;
          y[i] = (r < n) ? cq[r] : 0.0;
          ga += x[i] * y[i];
        }
        ga = row16_sum(ga);
        const double ab2 = al * be;
        if (ga * ga > orth * orth * ab2 && ab2 > floor_abs * floor_abs) {
          // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)); 1 / (2 zeta) for
          // huge |zeta|.  t only steers convergence (the rotation stays
          // orthogonal through c below), so it takes the hardware estimates
          // without refinement; c = 1 / sqrt(1 + t^2) is refined.
          const double zeta = (be - al) * __builtin_amdgcn_rcp(2.0 * ga);
          const double az = fabs(zeta);
          double tt;
          if (az < 1e100) {
            const double z2 = fma(zeta, zeta, 1.0);
            tt = __builtin_amdgcn_rcp(az + z2 * __builtin_amdgcn_rsq(z2));
          } else {
            tt = 0.5 * __builtin_amdgcn_rcp(az);
          }
          tt = (zeta >= 0.0) ? tt : -tt;
          const double c = rsq_nr(fma(tt, tt, 1.0)), sn = c * tt;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int r = lane + 16 * ((i + odd) & (RPL - 1));
            if (r < n) {
              cp[r] = c * x[i] - sn * y[i];
              cq[r] = sn * x[i] + c * y[i];
            }
          }
          if (VPL > 0) {
            double* vp = V + (size_t)p * ldv;
            double* vq = V + (size_t)q * ldv;
#pragma unroll
            for (int i = 0; i < (VPL > 0 ? VPL : 1); ++i) {
              const int r = lane + 16 * ((i + odd) & ((VPL > 0 ? VPL : 1) - 1));
              if (r < kv) {
                const double vx = vp[r], vy = vq[r];
                vp[r] = c * vx - sn * vy;
                vq[r] = sn * vx + c * vy;
              }
            }
          }
          if (lane == 0) {
            nrm2[p] = fmax(al - tt * ga, 0.0);
            nrm2[q] = fmax(be + tt * ga, 0.0);
          }
          rotated = true;
          big = big || ga * ga > stop2 * ab2;
        }
      }
      __syncthreads();
    }
    if (rotated && lane == 0) s_rot[0] = 1;
    if (big && lane == 0) s_rot[1] = 1;
    __syncthreads();
    const bool again = s_rot[0] != 0, more = s_rot[1] != 0;
    __syncthreads();   // every wave has read the flags before thread 0 resets them
    if (!again) break;
    if (!more) { ++sweep; break; }
  }
  return sweep;
}

// ---------------------------------------------------- one-sided Jacobi SVD
// M (k x k, row-major, k <= 64) = W diag(s) Z^T, s descending.  Jacobi on
// the columns of M (rotations accumulated in Z); the rotated column norms
// are the singular values.  Outputs W, Z as row-major k x k (columns are
// singular vectors).
constexpr int SVD_KM = 64;

// sv_copy (may be null) receives a second copy of the singular values
__device__ __forceinline__ void svd_jacobi_dev(int k, const double* __restrict__ Min, double* __restrict__ W,
                                               double* __restrict__ sv, double* __restrict__ Z,
                                               double* __restrict__ sv_copy) {
  __shared__ double A[SVD_KM * SVD_KM];   // column c at A + c * SVD_KM
  __shared__ double V[SVD_KM * SVD_KM];
  __shared__ double nrm[SVD_KM];
  __shared__ int order[SVD_KM];
  __shared__ double red[8];
  __shared__ int s_rot[2];
  const int t = threadIdx.x;
  const int kp = (k + 1) & ~1;   // even count (a zero column pads odd k)
  double part = 0.0;
  for (int e = t; e < kp * kp; e += blockDim.x) {
    const int c = e / kp, r = e % kp;
    const double v = (r < k && c < k) ? Min[r * k + c] : 0.0;
    A[c * SVD_KM + r] = v;
    V[c * SVD_KM + r] = (r == c) ? 1.0 : 0.0;
    part += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((t & 63) == 0) red[t >> 6] = part;
  __syncthreads();
  double fro = 0.0;
  for (int w = 0; w < 8; ++w) fro += red[w];
  const double floor_abs = 1e-300 + 1e-22 * fro;   // columns below this are negligible
  const double orth = 4.0 * kp * 2.220446049250313e-16;
  jacobi_cols<4, 4>(A, SVD_KM, kp, kp, V, SVD_KM, kp, orth, floor_abs, 60, nrm, s_rot);
  for (int c = t; c < kp; c += blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < kp; ++r) acc += A[c * SVD_KM + r] * A[c * SVD_KM + r];
    nrm[c] = sqrt(acc);
  }
  __syncthreads();
  // descending order, ties by index
  for (int c = t; c < kp; c += blockDim.x) {
    int rank = 0;
    for (int o = 0; o < kp; ++o)
      if (nrm[o] > nrm[c] || (nrm[o] == nrm[c] && o < c)) ++rank;
    order[rank] = c;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int r = e / k, j = e % k;
    const int c = order[j];
    W[e] = nrm[c] > 0.0 ? A[c * SVD_KM + r] / nrm[c] : (r == j ? 1.0 : 0.0);
    Z[e] = V[c * SVD_KM + r];
  }
  for (int j = t; j < k; j += blockDim.x) {
    sv[j] = nrm[order[j]];
    if (sv_copy) sv_copy[j] = nrm[order[j]];
  }
}

__global__ __launch_bounds__(512) void k_svd_jacobi(int k, const double* __restrict__ Min,
                                                    double* __restrict__ W, double* __restrict__ sv,
                                                    double* __restrict__ Z) {
  svd_jacobi_dev(k, Min, W, sv, Z, nullptr);
}

hipError_t svd_small(hipStream_t s, int k, const double* M, double* W, double* sv, double* Z) {
  if (k < 1 || k > SVD_KM) return hipErrorInvalidValue;
  k_svd_jacobi<<<1, 512, 0, s>>>(k, M, W, sv, Z);
  return hipGetLastError();
}

// Left singular vectors and values of M (k x k, row-major, SVD_KM < k <=
// 128): one-sided Jacobi on the columns of M in LDS (1024 threads, one
// 16-lane team per pair of 128 columns); the rotated columns, normalised
// and sorted by norm (descending, ties by index), are the left singular
// vectors, their norms the singular values.  The right vectors are not
// accumulated: the caller forms the ones it keeps as M^T w / s.
//
// The Jacobi sweeps run on L = P M Q (row-pivoted Householder LQ) instead
// of M: right-multiplying by an orthogonal matrix leaves the left singular
// vectors and the singular values unchanged (the row permutation P is
// undone on output), and the rows of L are graded, so the sweeps converge
// in about a third as many passes as on M itself.
constexpr int SVD_BIG = SLAR_CROSS_KMAX;
constexpr int SVD_BIG_LD = SVD_BIG;   // a multiple of 32 doubles, as the Jacobi teams assume

// In-place Householder LQ with row pivoting of the n x n matrix A (column
// c at A + c * lda, n <= 128, blockDim 1024): on return A holds L = P A Q,
// lower triangular, and perm[r] is the row of the input that row r of L
// came from.  Step i first swaps in the remaining row of largest norm over
// columns i.. (lowest index on ties; the norms are downdated by the entry
// each step leaves in column i, so only the pivot choice depends on their
// rounding), then reflects columns i..n-1 so that row i keeps only its
// diagonal.  Row r's update sums over the columns in eight strided groups
// of 128 threads (one thread per row and group); vrow holds the reflector.
// With the rows ordered by their remaining norm, L's columns come out
// graded and the Jacobi sweeps that follow need fewer passes.
__device__ void lq_lower(double* A, int lda, int n, double* vrow, double (*part)[SVD_BIG], double* s_sc,
                         double* rnorm, int* perm) {
  const int t = threadIdx.x;
  const int row = t & 127, g = t >> 7;
  // squared row norms
  if (row < n) {
    double pr = 0.0;
    for (int c = g; c < n; c += 8) pr += A[c * lda + row] * A[c * lda + row];
    part[g][row] = pr;
  }
  __syncthreads();
  if (t < n) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) a += part[q][t];
    rnorm[t] = a;
    perm[t] = t;
  }
  __syncthreads();
  for (int i = 0; i + 1 < n; ++i) {
    if (t < 64) {
      double m = -1.0;
      int mi = n;
      for (int r = i + t; r < n; r += 64)
        if (rnorm[r] > m) { m = rnorm[r]; mi = r; }
      for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, 64);
        const int i2 = __shfl_xor(mi, o, 64);
        if (m2 > m || (m2 == m && i2 < mi)) { m = m2; mi = i2; }
      }
      if (t == 0) s_sc[2] = (double)mi;
    }
    __syncthreads();
    const int p = (int)s_sc[2];
    if (p != i && p < n) {
      if (t < n) {
        const double a = A[t * lda + i];
        A[t * lda + i] = A[t * lda + p];
        A[t * lda + p] = a;
      }
      if (t == 0) {
        const double a = rnorm[i];
        rnorm[i] = rnorm[p];
        rnorm[p] = a;
        const int q = perm[i];
        perm[i] = perm[p];
        perm[p] = q;
      }
      __syncthreads();
    }
    if (t < 64) {
      double sg = 0.0;
      for (int c = i + 1 + t; c < n; c += 64) {
        const double x = A[c * lda + i];
        vrow[c] = x;
        sg += x * x;
      }
      for (int o = 32; o > 0; o >>= 1) sg += __shfl_xor(sg, o, 64);
      if (t == 0) { s_sc[0] = sg; s_sc[1] = A[i * lda + i]; }
    }
    __syncthreads();
    const double sig = s_sc[0], xi = s_sc[1];
    // x = row i from the diagonal on; H x = alpha e_i with |alpha| = |x|
    // and the sign opposite to x_i, so that v_i = x_i - alpha does not cancel
    const bool act = sig > 0.0;
    const double nx = sqrt(xi * xi + sig);
    const double alpha = (xi >= 0.0) ? -nx : nx;
    const double vi = xi - alpha;
    const double f = act ? 2.0 / (sig + vi * vi) : 0.0;
    if (act && row > i && row < n) {
      double pr = 0.0;
      for (int c = i + g; c < n; c += 8) pr += A[c * lda + row] * (c == i ? vi : vrow[c]);
      part[g][row] = pr;
    }
    __syncthreads();
    if (act && row > i && row < n) {
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) w += part[q][row];
      w *= f;
      for (int c = i + g; c < n; c += 8) A[c * lda + row] -= w * (c == i ? vi : vrow[c]);
    }
    if (act && row == i)
      for (int c = i + g; c < n; c += 8) A[c * lda + i] = (c == i) ? alpha : 0.0;
    __syncthreads();
    // remaining norms over columns i+1.. of the rows below
    if (t > i && t < n) rnorm[t] = fmax(rnorm[t] - A[i * lda + t] * A[i * lda + t], 0.0);
    __syncthreads();
  }
}

__device__ __forceinline__ void svd_left_big_dev(int k, const double* __restrict__ Min, double* __restrict__ W,
                                                 double* __restrict__ sv, double* __restrict__ sv_copy) {
  __shared__ double A[SVD_BIG * SVD_BIG_LD];   // column c at A + c * SVD_BIG_LD
  __shared__ double nrm[SVD_BIG];
  __shared__ int order[SVD_BIG];
  __shared__ double red[16];
  __shared__ int s_rot[2];
  __shared__ double vrow[SVD_BIG];
  __shared__ double lqpart[8][SVD_BIG];
  __shared__ double s_sc[3];
  __shared__ double rnorm[SVD_BIG];
  __shared__ int perm[SVD_BIG];
  const int t = threadIdx.x;
  const int kp = (k + 1) & ~1;
  double part = 0.0;
  for (int e = t; e < kp * kp; e += blockDim.x) {
    const int c = e / kp, r = e % kp;
    const double v = (r < k && c < k) ? Min[r * k + c] : 0.0;
    A[c * SVD_BIG_LD + r] = v;
    part += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((t & 63) == 0) red[t >> 6] = part;
  __syncthreads();
  double fro = 0.0;
  for (int w = 0; w < 16; ++w) fro += red[w];
  const double floor_abs = 1e-300 + 1e-22 * fro;
  const double orth = 4.0 * kp * 2.220446049250313e-16;
  lq_lower(A, SVD_BIG_LD, kp, vrow, lqpart, s_sc, rnorm, perm);
  jacobi_cols<8, 0>(A, SVD_BIG_LD, kp, kp, nullptr, 0, 0, orth, floor_abs, 60, nrm, s_rot);
  for (int c = t; c < kp; c += blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < kp; ++r) acc += A[c * SVD_BIG_LD + r] * A[c * SVD_BIG_LD + r];
    nrm[c] = sqrt(acc);
  }
  __syncthreads();
  for (int c = t; c < kp; c += blockDim.x) {
    int rank = 0;
    for (int o = 0; o < kp; ++o)
      if (nrm[o] > nrm[c] || (nrm[o] == nrm[c] && o < c)) ++rank;
    order[rank] = c;
  }
  __syncthreads();
  // row r of L is row perm[r] of the input; the zero padding row of odd k
  // (perm[r] == k) may have moved, so every row of L is visited and only
  // the input's k rows are written
  for (int e = t; e < kp * k; e += blockDim.x) {
    const int r = e / k, j = e % k;
    const int c = order[j];
    const int ro = perm[r];
    if (ro < k) W[(size_t)ro * k + j] = nrm[c] > 0.0 ? A[c * SVD_BIG_LD + r] / nrm[c] : (ro == j ? 1.0 : 0.0);
  }
  for (int j = t; j < k; j += blockDim.x) {
    sv[j] = nrm[order[j]];
    if (sv_copy) sv_copy[j] = nrm[order[j]];
  }
}

__global__ __launch_bounds__(1024) void k_svd_left_big(int k, const double* __restrict__ Min,
                                                       double* __restrict__ W, double* __restrict__ sv) {
  svd_left_big_dev(k, Min, W, sv, nullptr);
}

hipError_t svd_left_big(hipStream_t s, int k, const double* M, double* W, double* sv) {
  if (k <= SVD_KM || k > SVD_BIG) return hipErrorInvalidValue;
  k_svd_left_big<<<1, 1024, 0, s>>>(k, M, W, sv);
  return hipGetLastError();
}

// one block per descriptor: k <= 64 (full SVD, 512 threads) or 64 < k <=
// 128 (left vectors and values, 1024 threads), as the caller groups them
__global__ __launch_bounds__(512) void k_svd_group_small(const SvdDesc* __restrict__ D) {
  const SvdDesc d = D[blockIdx.x];
  svd_jacobi_dev(d.k, d.M, d.W, d.sv, d.Z, d.sv_copy);
}
__global__ __launch_bounds__(1024) void k_svd_group_big(const SvdDesc* __restrict__ D) {
  const SvdDesc d = D[blockIdx.x];
  svd_left_big_dev(d.k, d.M, d.W, d.sv, d.sv_copy);
}

hipError_t svd_group(hipStream_t s, int count, const SvdDesc* d, bool big) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  if (big) k_svd_group_big<<<count, 1024, 0, s>>>(d);
  else k_svd_group_small<<<count, 512, 0, s>>>(d);
  return hipGetLastError();
}

// Z[:, j] *= 1 / sv[j] (0 where sv[j] == 0), Z row-major k x ld, j < r
__device__ __forceinline__ void scale_cols_inv_dev(int k, int r, double* __restrict__ Z, int ld,
                                                   const double* __restrict__ sv, int e) {
  if (e >= k * r) return;
  const int i = e / r, j = e % r;
  const double s = sv[j];
  Z[(size_t)i * ld + j] = s > 0.0 ? Z[(size_t)i * ld + j] / s : 0.0;
}

__global__ void k_scale_cols_inv(int k, int r, double* __restrict__ Z, int ld, const double* __restrict__ sv) {
  scale_cols_inv_dev(k, r, Z, ld, sv, blockIdx.x * blockDim.x + threadIdx.x);
}

// grouped: scale_cols_inv, or (diag) the r x r root diag(sv[:r]) into Z
__global__ __launch_bounds__(256) void k_scale_group(const ScaleDesc* __restrict__ D, const int* __restrict__ first,
                                                     int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const ScaleDesc g = D[d];
  const int e = (b - first[d]) * 256 + (int)threadIdx.x;
  if (g.diag) {
    if (e < g.r * g.r) g.Z[e] = (e / g.r == e % g.r) ? g.sv[e / g.r] : 0.0;
  } else {
    scale_cols_inv_dev(g.k, g.r, g.Z, g.ld, g.sv, e);
  }
}

hipError_t scale_group_launch(hipStream_t s, const ScaleDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_scale_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t scale_cols_inv(hipStream_t s, int k, int r, double* Z, int ld, const double* sv) {
  k_scale_cols_inv<<<(k * r + 255) / 256, 256, 0, s>>>(k, r, Z, ld, sv);
  return hipGetLastError();
}

// ------------------------------------- symmetric PSD eigendecomposition
// G (n x n, symmetric positive semidefinite, n <= 128) = U diag(lam) U^T,
// lam descending, for the leading eigenpairs.  Two stages in one block:
//  1. pivoted Cholesky G ~ L L^T, L (n x c) built column by column in LDS
//     (pivot = largest remaining diagonal, lowest index on ties), stopping
//     when the remaining diagonal drops below 1e-30 trace or after 64
//     columns; four threads share each row's inner product;
//  2. one-sided Jacobi on the columns of L: the rotated, normalised
//     columns are the eigenvectors of L L^T and their squared norms the
//     eigenvalues.
// Eigenvalues beyond the factor rank are returned as 0 with zero vectors,
// except that lam[c] (c < n) receives the trace left after c columns, so
// that tail sums over lam never undercount.
constexpr int EIG_CM = EIG_COLS;

struct EigBatch {
  int n[4];
  const double* G[4];
  double* lam[4];
  double* U[4];
};

// lam_copy (may be null) receives a second copy of lam
__device__ __forceinline__ void eig_psd_dev(int n, const double* __restrict__ G, double* __restrict__ lam,
                                            double* __restrict__ Uout, double* __restrict__ lam_copy) {
  __shared__ double L[EIG_CM * SLAR_NMAX];   // column c at L + c * SLAR_NMAX
  __shared__ double dres[SLAR_NMAX];
  __shared__ unsigned char taken[SLAR_NMAX];
  __shared__ double nrm[EIG_CM];
  __shared__ int order[EIG_CM];
  __shared__ double s_piv;
  __shared__ int s_p, s_rot[2], s_nc;
  __shared__ double s_trace, s_rest;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += blockDim.x) { dres[i] = fmax(G[(size_t)i * n + i], 0.0); taken[i] = 0; }
  __syncthreads();
  if (t < 64) {
    double a = 0.0;
    for (int i = t; i < n; i += 64) a += dres[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (t == 0) s_trace = a;
  }
  __syncthreads();
  const double trace = s_trace;
  const double stop = 1e-30 * trace + 1e-300;
  // four groups of 128 threads (two waves each) split every inner product
  // over the factor columns; a wave reads 64 consecutive rows of one column
  const int row = t & 127, sub = t >> 7;
  __shared__ double part[4][SLAR_NMAX];
  int c = 0;
  for (; c < EIG_CM && c < n; ++c) {
    // pivot: largest remaining diagonal (lowest index on ties), one wave
    if (t < 64) {
      double m = -1.0;
      int mi = n;
      for (int i = t; i < n; i += 64)
        if (!taken[i] && dres[i] > m) { m = dres[i]; mi = i; }
      for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, 64);
        const int i2 = __shfl_xor(mi, o, 64);
        if (m2 > m || (m2 == m && i2 < mi)) { m = m2; mi = i2; }
      }
      if (t == 0) { s_piv = m; s_p = mi; }
    }
    __syncthreads();
    const double dp = s_piv;
    const int p = s_p;
    if (!(dp > stop) || p >= n) break;
    const double sq = sqrt(dp);
    // the pivot row of G is read before the inner products, so its global
    // load latency overlaps them
    const double gpr = (sub == 0 && row < n) ? G[(size_t)p * n + row] : 0.0;
    if (row < n) {
      double v = 0.0;
      for (int j = sub; j < c; j += 4) v += L[j * SLAR_NMAX + row] * L[j * SLAR_NMAX + p];
      part[sub][row] = v;
    }
    __syncthreads();
    if (sub == 0 && row < n) {
      const double v = (part[0][row] + part[1][row]) + (part[2][row] + part[3][row]);
      double out = 0.0;
      if (row == p) {
        out = sq;
        taken[row] = 1;
        dres[row] = 0.0;
      } else if (!taken[row]) {
        out = (gpr - v) / sq;
        dres[row] = fmax(dres[row] - out * out, 0.0);
      }
      L[c * SLAR_NMAX + row] = out;
    }
    __syncthreads();
  }
  if (t < 64) {
    double a = 0.0;
    for (int i = t; i < n; i += 64) a += taken[i] ? 0.0 : dres[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (t == 0) { s_rest = a; s_nc = c; }
  }
  __syncthreads();
  const int nc = s_nc;
  const int kp = (nc + 1) & ~1;
  if (nc < kp)   // zero padding column
    for (int i = t; i < n; i += blockDim.x) L[nc * SLAR_NMAX + i] = 0.0;
  __syncthreads();
  const double floor_abs = 1e-22 * trace + 1e-300;   // columns below this are negligible
  const double orth = 4.0 * n * 2.220446049250313e-16;
  if (kp >= 2) jacobi_cols<8, 0>(L, SLAR_NMAX, n, kp, nullptr, 0, 0, orth, floor_abs, 40, nrm, s_rot);
  for (int j = t; j < kp; j += blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < n; ++r) acc += L[j * SLAR_NMAX + r] * L[j * SLAR_NMAX + r];
    nrm[j] = acc;
  }
  __syncthreads();
  for (int j = t; j < kp; j += blockDim.x) {
    int rank = 0;
    for (int o = 0; o < kp; ++o)
      if (nrm[o] > nrm[j] || (nrm[o] == nrm[j] && o < j)) ++rank;
    order[rank] = j;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += blockDim.x) {
    const int r = e / n, j = e % n;
    double v = 0.0;
    if (j < nc) {
      const int cidx = order[j];
      const double s = sqrt(nrm[cidx]);
      v = s > 0.0 ? L[cidx * SLAR_NMAX + r] / s : 0.0;
    }
    Uout[e] = v;
  }
  for (int j = t; j < n; j += blockDim.x) {
    const double l = (j < nc) ? nrm[order[j]] : (j == nc ? s_rest : 0.0);
    lam[j] = l;
    if (lam_copy) lam_copy[j] = l;
  }
}

__global__ __launch_bounds__(512) void k_eig_psd(EigBatch B) {
  eig_psd_dev(B.n[blockIdx.x], B.G[blockIdx.x], B.lam[blockIdx.x], B.U[blockIdx.x], nullptr);
}
__global__ __launch_bounds__(512) void k_eig_psd_group(const EigDesc* __restrict__ D) {
  const EigDesc d = D[blockIdx.x];
  eig_psd_dev(d.n, d.G, d.lam, d.U, d.lam_copy);
}

// up to four independent eigenproblems in one launch (one block each)
hipError_t eig_sym_batch(hipStream_t s, int count, const int* n, const double* const* G,
                         double* const* lam, double* const* V) {
  if (count < 1 || count > 4) return hipErrorInvalidValue;
  EigBatch B{};
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > SLAR_NMAX) return hipErrorInvalidValue;
    B.n[i] = n[i]; B.G[i] = G[i]; B.lam[i] = lam[i]; B.U[i] = V[i];
  }
  k_eig_psd<<<count, 512, 0, s>>>(B);
  return hipGetLastError();
}

hipError_t eig_sym_group(hipStream_t s, int count, const EigDesc* d) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  k_eig_psd_group<<<count, 512, 0, s>>>(d);
  return hipGetLastError();
}

// Completion of an orthonormal set to a basis of R^n (n <= 128): E is
// row-major n x n, column j either a unit vector of the set or zero (as the
// eigen kernel leaves the columns past its factor rank).  Each zero column,
// in order, becomes the unit vector e_p with the largest residual
// 1 - sum_c E[p][c]^2 (lowest p on ties), orthogonalised twice against every
// filled column and normalised.  One block per matrix, 512 threads, the
// matrix in LDS column-major.
struct CompleteBatch {
  int n[4];
  double* E[4];
};

__device__ __forceinline__ void complete_basis_dev(int n, double* __restrict__ E) {
  __shared__ double C[SLAR_NMAX * SLAR_NMAX];   // column c at C + c * SLAR_NMAX
  __shared__ double res[SLAR_NMAX], v[SLAR_NMAX], h[SLAR_NMAX], part[4][SLAR_NMAX];
  __shared__ unsigned char filled[SLAR_NMAX];
  __shared__ double red[8];
  __shared__ int redi[8];
  const int t = threadIdx.x;
  for (int e = t; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    C[c * SLAR_NMAX + r] = E[e];
  }
  __syncthreads();
  for (int c = t; c < n; c += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < n; ++r) a += C[c * SLAR_NMAX + r] * C[c * SLAR_NMAX + r];
    filled[c] = a > 0.5;
  }
  __syncthreads();
  for (int r = t; r < n; r += blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < n; ++c)
      if (filled[c]) a += C[c * SLAR_NMAX + r] * C[c * SLAR_NMAX + r];
    res[r] = 1.0 - a;
  }
  __syncthreads();
  const int row = t & 127, grp = t >> 7;   // 4 groups of 128 threads
  for (int z = 0; z < n; ++z) {
    if (filled[z]) continue;   // uniform: filled is in LDS and only changes below
    // pivot: largest residual, lowest index on ties
    double m = -1.0;
    int mi = n;
    for (int r = t; r < n; r += blockDim.x)
      if (res[r] > m) { m = res[r]; mi = r; }
    for (int o = 32; o > 0; o >>= 1) {
      const double m2 = __shfl_xor(m, o, 64);
      const int i2 = __shfl_xor(mi, o, 64);
      if (m2 > m || (m2 == m && i2 < mi)) { m = m2; mi = i2; }
    }
    if ((t & 63) == 0) { red[t >> 6] = m; redi[t >> 6] = mi; }
    __syncthreads();
    int p = redi[0];
    double mp = red[0];
    for (int w = 1; w < 8; ++w)
      if (red[w] > mp || (red[w] == mp && redi[w] < p)) { mp = red[w]; p = redi[w]; }
    for (int r = t; r < n; r += blockDim.x) v[r] = (r == p) ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      // h[c] = C[:, c] . v over the filled columns (one thread per column)
      for (int c = t; c < n; c += blockDim.x) {
        double a = 0.0;
        if (filled[c])
          for (int r = 0; r < n; ++r) a += C[c * SLAR_NMAX + r] * v[r];
        h[c] = a;
      }
      __syncthreads();
      // v[r] -= sum_c C[r][c] h[c]: four column groups per row
      if (row < n) {
        double a = 0.0;
        for (int c = grp; c < n; c += 4) a += C[c * SLAR_NMAX + row] * h[c];
        part[grp][row] = a;
      }
      __syncthreads();
      if (t < n) v[t] -= (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
      __syncthreads();
    }
    double a = 0.0;
    for (int r = t; r < n; r += blockDim.x) a += v[r] * v[r];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((t & 63) == 0) red[t >> 6] = a;
    __syncthreads();
    double nv = 0.0;
    for (int w = 0; w < 8; ++w) nv += red[w];
    const double inv = 1.0 / sqrt(nv);
    for (int r = t; r < n; r += blockDim.x) {
      const double x = v[r] * inv;
      C[z * SLAR_NMAX + r] = x;
      res[r] -= x * x;
    }
    if (t == 0) filled[z] = 1;
    __syncthreads();
  }
  for (int e = t; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    E[e] = C[c * SLAR_NMAX + r];
  }
}

__global__ __launch_bounds__(512) void k_complete_basis(CompleteBatch B) {
  complete_basis_dev(B.n[blockIdx.x], B.E[blockIdx.x]);
}
__global__ __launch_bounds__(512) void k_complete_basis_group(const BasisDesc* __restrict__ D) {
  const BasisDesc d = D[blockIdx.x];
  complete_basis_dev(d.n, d.E);
}

hipError_t complete_basis_group(hipStream_t s, int count, const BasisDesc* d) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  k_complete_basis_group<<<count, 512, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t complete_basis_batch(hipStream_t s, int count, const int* n, double* const* E) {
  if (count < 1 || count > 4) return hipErrorInvalidValue;
  CompleteBatch B{};
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > SLAR_NMAX) return hipErrorInvalidValue;
    B.n[i] = n[i]; B.E[i] = E[i];
  }
  k_complete_basis<<<count, 512, 0, s>>>(B);
  return hipGetLastError();
}

// Sign rule on columns: the entry of largest magnitude (lowest index on
// near-ties within 1e-10) is made positive; the same flip is applied to the
// matching column of B (if given).  A is [rows][lda] (column c), one block
// per column.
__device__ __forceinline__ void sign_fix_dev(int rows, int cols, double* __restrict__ A, int lda,
                                             double* __restrict__ B, int ldb, int rowsB, int c) {
  if (c >= cols) return;
  __shared__ double red[256];
  __shared__ int redi[256];
  const int t = threadIdx.x;
  double m = -1.0;
  for (int r = t; r < rows; r += blockDim.x) m = fmax(m, fabs(A[(long long)r * lda + c]));
  red[t] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] = fmax(red[t], red[t + o]);
    __syncthreads();
  }
  const double top = red[0];
  __syncthreads();
  int best = rows;
  for (int r = t; r < rows; r += blockDim.x)
    if (fabs(A[(long long)r * lda + c]) >= top * (1.0 - 1e-10)) { best = r; break; }
  redi[t] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) redi[t] = min(redi[t], redi[t + o]);
    __syncthreads();
  }
  const int p = redi[0];
  if (p >= rows || top <= 0.0) return;
  if (A[(long long)p * lda + c] < 0.0) {
    for (int r = t; r < rows; r += blockDim.x) A[(long long)r * lda + c] = -A[(long long)r * lda + c];
    if (B != nullptr)
      for (int r = t; r < rowsB; r += blockDim.x) B[(long long)r * ldb + c] = -B[(long long)r * ldb + c];
  }
}

__global__ void k_sign_fix(int rows, int cols, double* __restrict__ A, int lda,
                           double* __restrict__ B, int ldb, int rowsB) {
  sign_fix_dev(rows, cols, A, lda, B, ldb, rowsB, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_sign_fix_group(const SignDesc* __restrict__ D,
                                                        const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const SignDesc g = D[d];
  sign_fix_dev(g.rows, g.cols, g.A, g.lda, g.B, g.ldb, g.rowsB, b - first[d]);
}

hipError_t sign_fix_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_sign_fix_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t sign_fix(hipStream_t s, int rows, int cols, double* A, int lda, double* B, int ldb,
                    int rowsB) {
  if (cols <= 0) return hipSuccess;
  k_sign_fix<<<cols, 256, 0, s>>>(rows, cols, A, lda, B, ldb, rowsB);
  return hipGetLastError();
}

// The same sign rule for tall A (rows >> cols, cols <= 64), in three
// coalesced passes: per-block column maxima; per column the maximum, the
// first block reaching the near-tie threshold and the first such row in
// it (the lowest qualifying index overall); the flips.
constexpr int SF_COLS = 64;

__device__ __forceinline__ void sign_part_dev(int rows, int cols, const double* __restrict__ A, int lda, int rb,
                                              double* __restrict__ part, int blk) {
  __shared__ double red[4][SF_COLS];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int r0 = blk * rb, r1 = min(rows, r0 + rb);
  double m = -1.0;
  if (c < cols)
    for (int r = r0 + rl; r < r1; r += 4) m = fmax(m, fabs(A[(long long)r * lda + c]));
  red[rl][c] = m;
  __syncthreads();
  if (rl == 0 && c < cols)
    part[(size_t)blk * cols + c] = fmax(fmax(red[0][c], red[1][c]), fmax(red[2][c], red[3][c]));
}

__global__ __launch_bounds__(256) void k_sign_part(int rows, int cols, const double* __restrict__ A,
                                                   int lda, int rb, double* __restrict__ part) {
  sign_part_dev(rows, cols, A, lda, rb, part, blockIdx.x);
}

__device__ __forceinline__ void sign_decide_dev(int rows, int cols, const double* __restrict__ A, int lda, int rb,
                                                int nb, const double* __restrict__ part, double* __restrict__ sgn,
                                                int c) {
  __shared__ double redm[256];
  __shared__ int redi[256];
  const int t = threadIdx.x;
  double m = -1.0;
  for (int b = t; b < nb; b += blockDim.x) m = fmax(m, part[(size_t)b * cols + c]);
  redm[t] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) redm[t] = fmax(redm[t], redm[t + o]);
    __syncthreads();
  }
  const double top = redm[0];
  const double thr = top * (1.0 - 1e-10);
  int bb = nb;
  for (int b = t; b < nb; b += blockDim.x)
    if (part[(size_t)b * cols + c] >= thr) { bb = b; break; }
  redi[t] = bb;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) redi[t] = min(redi[t], redi[t + o]);
    __syncthreads();
  }
  const int bstar = redi[0];
  __syncthreads();
  int best = rows;
  if (bstar < nb) {
    const int r1 = min(rows, (bstar + 1) * rb);
    for (int r = bstar * rb + t; r < r1; r += blockDim.x)
      if (fabs(A[(long long)r * lda + c]) >= thr) { best = r; break; }
  }
  redi[t] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) redi[t] = min(redi[t], redi[t + o]);
    __syncthreads();
  }
  if (t == 0) {
    const int p = redi[0];
    sgn[c] = (p < rows && top > 0.0 && A[(long long)p * lda + c] < 0.0) ? -1.0 : 1.0;
  }
}

__global__ __launch_bounds__(256) void k_sign_decide(int rows, int cols, const double* __restrict__ A,
                                                     int lda, int rb, int nb,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ sgn) {
  sign_decide_dev(rows, cols, A, lda, rb, nb, part, sgn, blockIdx.x);
}

__device__ __forceinline__ void sign_apply_dev(long long na, int cols, double* __restrict__ A, int lda,
                                               long long nbe, double* __restrict__ B, int ldb,
                                               const double* __restrict__ sgn, long long e) {
  if (e < na) {
    const int c = (int)(e % cols);
    if (sgn[c] < 0.0) {
      double* a = A + (e / cols) * lda + c;
      *a = -*a;
    }
  } else if (e < na + nbe) {
    const long long f = e - na;
    const int c = (int)(f % cols);
    if (sgn[c] < 0.0) {
      double* b = B + (f / cols) * ldb + c;
      *b = -*b;
    }
  }
}

__global__ void k_sign_apply(long long na, int cols, double* __restrict__ A, int lda, long long nbe,
                             double* __restrict__ B, int ldb, const double* __restrict__ sgn) {
  sign_apply_dev(na, cols, A, lda, nbe, B, ldb, sgn, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// grouped tall form: desc.part holds [nb][cols] partial maxima then [cols] signs
__global__ __launch_bounds__(256) void k_sign_part_group(const SignDesc* __restrict__ D,
                                                         const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const SignDesc g = D[d];
  sign_part_dev(g.rows, g.cols, g.A, g.lda, g.rb, g.part, b - first[d]);
}
__global__ __launch_bounds__(256) void k_sign_decide_group(const SignDesc* __restrict__ D,
                                                           const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const SignDesc g = D[d];
  sign_decide_dev(g.rows, g.cols, g.A, g.lda, g.rb, g.nb, g.part, g.part + (size_t)g.nb * g.cols, b - first[d]);
}
__global__ __launch_bounds__(256) void k_sign_apply_group(const SignDesc* __restrict__ D,
                                                          const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const SignDesc g = D[d];
  const long long na = (long long)g.rows * g.cols, nbe = g.B ? (long long)g.rowsB * g.cols : 0;
  sign_apply_dev(na, g.cols, g.A, g.lda, nbe, g.B, g.ldb, g.part + (size_t)g.nb * g.cols,
                 (long long)(b - first[d]) * 256 + threadIdx.x);
}

hipError_t sign_part_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_sign_part_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}
hipError_t sign_decide_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_sign_decide_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}
hipError_t sign_apply_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_sign_apply_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t sign_fix_tall(hipStream_t s, double* scratch, size_t scratch_elems, int rows, int cols,
                         double* A, int lda, double* B, int ldb, int rowsB) {
  if (cols <= 0) return hipSuccess;
  const int nb = std::min(256, std::max(1, (rows + 63) / 64));
  const int rb = (rows + nb - 1) / nb;
  if (cols > SF_COLS || (size_t)(nb + 1) * cols > scratch_elems)
    return sign_fix(s, rows, cols, A, lda, B, ldb, rowsB);
  double* part = scratch;
  double* sgn = scratch + (size_t)nb * cols;
  k_sign_part<<<nb, 256, 0, s>>>(rows, cols, A, lda, rb, part);
  k_sign_decide<<<cols, 256, 0, s>>>(rows, cols, A, lda, rb, nb, part, sgn);
  const long long na = (long long)rows * cols, nbe = B ? (long long)rowsB * cols : 0;
  k_sign_apply<<<(unsigned)((na + nbe + 255) / 256), 256, 0, s>>>(na, cols, A, lda, nbe, B, ldb, sgn);
  return hipGetLastError();
}

// ------------------------------------------------------------- helpers
__device__ __forceinline__ void copy2d_dev(int rows, int cols, const double* __restrict__ A, int lda,
                                           double* __restrict__ B, int ldb, const double* __restrict__ colscale,
                                           long long e) {
  if (e >= (long long)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  double v = A[(long long)r * lda + c];
  if (colscale) v *= colscale[c];
  B[(long long)r * ldb + c] = v;
}

__global__ void k_copy2d(int rows, int cols, const double* __restrict__ A, int lda,
                         double* __restrict__ B, int ldb, const double* __restrict__ colscale) {
  copy2d_dev(rows, cols, A, lda, B, ldb, colscale, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_copy2d_group(const CopyDesc* __restrict__ D, const int* __restrict__ first,
                                                      int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const CopyDesc g = D[d];
  copy2d_dev(g.rows, g.cols, g.A, g.lda, g.B, g.ldb, g.colscale, (long long)(b - first[d]) * 256 + threadIdx.x);
}

hipError_t copy2d_group_launch(hipStream_t s, const CopyDesc* d, const int* first, int nd, int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  k_copy2d_group<<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

hipError_t copy2d(hipStream_t s, int rows, int cols, const double* A, int lda, double* B, int ldb,
                  const double* colscale) {
  const long long n = (long long)rows * cols;
  if (n <= 0) return hipSuccess;
  k_copy2d<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, cols, A, lda, B, ldb, colscale);
  return hipGetLastError();
}

__global__ void k_fill(double* p, long long n, double v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

hipError_t fill(hipStream_t s, double* p, long long n, double v) {
  if (n <= 0) return hipSuccess;
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace slar
