// FP64 GEMM on the matrix cores for the plain products of the path (the
// truncation's orthogonalisations and projections, the frame builds, the
// moment integrals and the regularised skeleton): row-major
//   C_b = alpha op(A_b) op(B_b) + beta C_b,   b < batch,
// op(A) M x K, op(B) K x N, with element strides lda, ldb, ldc and batch
// strides sA, sB, sC.  beta = 0 never reads C.
//
// A block of 256 threads (four waves) owns a 64 x 64 tile of C; wave w
// owns its 32 x 32 quadrant as 2 x 2 tiles of the 16x16x4 FP64 matrix-core
// step.  K runs in chunks of 16: each chunk of op(A) and op(B) is staged in
// LDS k-major (the operand fragments of a step are 16 consecutive doubles
// per k), while the next chunk's global loads are already in registers.
// Loads are coalesced along the stored row of each operand (k for A, m for
// A^T, n for B, k for B^T) and predicated outside the matrices (zero).
// The summation order is fixed by the tiling, so products are reproducible
// bit for bit.
#include "slar_internal.h"
#include "dense.h"
#include "group.h"

namespace slar {

namespace {

typedef double gm_v4d __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 16;
constexpr int GB_LDA = GB_M + 2;   // k-major rows, padded
constexpr int GB_LDB = GB_N + 2;

// thread t's four elements of a 64 x 16 (A) or 16 x 64 (B) chunk:
// contiguous-in-memory direction first
template <bool ROWK>
__device__ __forceinline__ void chunk_coords(int t, int j, int* outer, int* inner) {
  if (ROWK) {   // memory row = the 64-long dimension, contiguous along k (16)
    *outer = t >> 2;                  // 0..63
    *inner = ((t & 3) << 2) + j;      // k 0..15
  } else {      // memory row = k, contiguous along the 64-long dimension
    *inner = t >> 4;                  // k 0..15
    *outer = ((t & 15) << 2) + j;     // 0..63
  }
}

// the 64 x 64 output tile at (m0, n0) of one batch item (A, B, C already
// offset to it)
template <bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, double alpha, const double* __restrict__ A,
                                          int lda, const double* __restrict__ B, int ldb, double beta,
                                          double* __restrict__ C, int ldc, int m0, int n0) {
  __shared__ double As[GB_K][GB_LDA];   // As[k][m] = op(A)[m0 + m][k0 + k]
  __shared__ double Bs[GB_K][GB_LDB];   // Bs[k][n] = op(B)[k0 + k][n0 + n]
  const int t = threadIdx.x;
  // op(A)[m][k] is A[m * lda + k] (row-major M x K) or A[k * lda + m] (A^T)
  auto ldA = [&](int k0, double* r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int mm, kk;
      chunk_coords<!TA>(t, j, &mm, &kk);
      const int m = m0 + mm, k = k0 + kk;
      const bool ok = m < M && k < K;
      r[j] = ok ? (TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]) : 0.0;
    }
  };
  // op(B)[k][n] is B[k * ldb + n] (row-major K x N) or B[n * ldb + k] (B^T)
  auto ldB = [&](int k0, double* r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int nn, kk;
      chunk_coords<TB>(t, j, &nn, &kk);
      const int n = n0 + nn, k = k0 + kk;
      const bool ok = n < N && k < K;
      r[j] = ok ? (TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n]) : 0.0;
    }
  };
  auto stA = [&](const double* r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int mm, kk;
      chunk_coords<!TA>(t, j, &mm, &kk);
      As[kk][mm] = r[j];
    }
  };
  auto stB = [&](const double* r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int nn, kk;
      chunk_coords<TB>(t, j, &nn, &kk);
      Bs[kk][nn] = r[j];
    }
  };
  const int w = t >> 6, lane = t & 63;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;   // wave quadrant
  const int li = lane & 15, lq = lane >> 4;
  gm_v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gm_v4d{0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  ldA(0, ra);
  ldB(0, rb);
  for (int k0 = 0; k0 < K; k0 += GB_K) {
    stA(ra);
    stB(rb);
    __syncthreads();
    if (k0 + GB_K < K) {   // next chunk in flight during this one's steps
      ldA(k0 + GB_K, ra);
      ldB(k0 + GB_K, rb);
    }
#pragma unroll
    for (int ks = 0; ks < GB_K; ks += 4) {
      // lane holds op(A)[row li][k lq] and op(B)[k lq][col li] of each tile
      double fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = As[ks + lq][wm + 16 * a + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = Bs[ks + lq][wn + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator v of lane l is D[(l / 16) + 4 v][l % 16] of its tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * a + lq + 4 * v;
        const int n = n0 + wn + 16 * b + li;
        if (m < M && n < N) {
          double* c = C + (size_t)m * ldc + n;
          const double x = alpha * acc[a][b][v];
          *c = (beta == 0.0) ? x : x + beta * *c;
        }
      }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda, long long sA,
                                                  const double* __restrict__ B, int ldb, long long sB,
                                                  double beta, double* __restrict__ C, int ldc,
                                                  long long sC) {
  const long long bz = blockIdx.z;
  gemm_tile<TA, TB>(M, N, K, alpha, A + bz * sA, lda, B + bz * sB, ldb, beta, C + bz * sC, ldc,
                    blockIdx.y * GB_M, blockIdx.x * GB_N);
}

// problem d owns tm * tn * batch blocks: batch item, then tile row, then
// tile column, as the one-problem grid (x: tile column, y: tile row, z: item)
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64_group(const GemmDesc* __restrict__ D,
                                                        const int* __restrict__ first, int nd) {
  const int b = blockIdx.x;
  const int d = group_find(first, nd, b);
  const GemmDesc g = D[d];
  const int local = b - first[d];
  const int per = g.tm * g.tn;
  const int bz = local / per, rem = local - bz * per;
  const int mt = rem / g.tn, nt = rem - mt * g.tn;
  gemm_tile<TA, TB>(g.M, g.N, g.K, g.alpha, g.A + (long long)bz * g.sA, g.lda, g.B + (long long)bz * g.sB, g.ldb,
                    g.beta, g.C + (long long)bz * g.sC, g.ldc, mt * GB_M, nt * GB_N);
}

}  // namespace

hipError_t gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                    double beta, double* C, int ldc, long long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (K < 0 || batch > 65535 || (M + GB_M - 1) / GB_M > 65535) return hipErrorInvalidValue;
  const dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, batch);
  if (!ta && !tb)
    k_gemm_f64<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else if (ta && !tb)
    k_gemm_f64<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else if (!ta && tb)
    k_gemm_f64<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else
    k_gemm_f64<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  return hipGetLastError();
}

hipError_t gemm_group_launch(hipStream_t s, bool ta, bool tb, const GemmDesc* d, const int* first, int nd,
                             int nblocks) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  if (!ta && !tb) k_gemm_f64_group<false, false><<<nblocks, 256, 0, s>>>(d, first, nd);
  else if (ta && !tb) k_gemm_f64_group<true, false><<<nblocks, 256, 0, s>>>(d, first, nd);
  else if (!ta && tb) k_gemm_f64_group<false, true><<<nblocks, 256, 0, s>>>(d, first, nd);
  else k_gemm_f64_group<true, true><<<nblocks, 256, 0, s>>>(d, first, nd);
  return hipGetLastError();
}

}  // namespace slar
