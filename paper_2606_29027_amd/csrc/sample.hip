// SL-FD entry evaluation (section 3.1).
//  * k_ht_sample: the paper's contraction on an HT tensor: per sample the
//    leaf interpolations c^(mu) = w(xi_mu) U^(mu)_{J_mu}, then the transfer
//    contractions y12 = (c1 (x) c2) B12, y34 = (c3 (x) c4) B34 and the root
//    bilinear form (O(d r^3) per point).  64 samples per block; the
//    transfer contractions and the root form run on the matrix cores
//    (16x16x4 FP32 / FP64 steps) with B12/B34 streamed from L2.
//  * frame build: X = (U1 (x) U2) B12 and P = ((U3 (x) U4) B34) root^T as
//    two GEMMs per node.
//  * k_frame_points: eq. (tp_interp) from the node frames (frame_sampler.h)
//    for an explicit list of grid points.
#include <vector>

#include "slar_internal.h"
#include "dense.h"
#include "frame_sampler.h"
#include "group.h"

namespace slar {

template <typename T>
struct HtDev {
  int d;
  int r[6];
  const T* U[4];
  const T* B12;
  const T* B34;
  const T* root;
};

// ---------------------------------------------------------------- MFMA
// 16x16x4 matrix-core step, D = A B + C, for one 64-lane wave.  Lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator v = 0..3 of
// lane l is D[row(l / 16, v)][l % 16], with row = 4 (l / 16) + v for the
// FP32 step and (l / 16) + 4 v for the FP64 step.
typedef float hs_v4f __attribute__((ext_vector_type(4)));
typedef double hs_v4d __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc = hs_v4f;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};
template <> struct Mfma<double> {
  using acc = hs_v4d;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};

// A block evaluates HS_S entries with four waves.  Each transfer node is
// the GEMM y[s][c] = sum_(a,b) (c_a[s][a] c_b[s][b]) B[(a,b)][c] with
// M = 64 entries, K = r_a r_b and N = r_parent; the Khatri-Rao operand is
// formed lane by lane from the leaf interpolations in LDS, one product per
// matrix-core step.  The (M, N) plane is 4 x NT tiles of 16 x 16; wave w
// owns column tile w % NT and the row tiles w / NT + k (4 / NT), k < NT,
// so every B fragment it loads feeds NT steps.
constexpr int HS_S = 64;
template <typename T>
struct HsLds {
  static constexpr int LDC = sizeof(T) == 4 ? 68 : 66;   // conflict-free A reads
  int rows[HS_S][12];           // stencil rows, [dim][point] (d W <= 12)
  double wts[HS_S][12];
  T c[2][HS_S][LDC];            // two operand slots, zero beyond the rank
  T part[4][HS_S];              // per column tile partial sums
};

// c[slot][s][a] = sum_w w U^(mu)[row_w][a] for the leaves m0, m0 + 1.
template <typename T, int W>
__device__ __forceinline__ void hs_interp(const HtDev<T>& F, int m0, HsLds<T>& L, int t) {
#pragma unroll 4
  for (int e = t; e < 2 * HS_S * 64; e += 256) {
    const int slot = e / (HS_S * 64), s = (e / 64) % HS_S, col = e % 64;
    const int m = m0 + slot, rm = F.r[m];
    T acc = 0;
    if (col < rm) {
      const T* U = F.U[m];
#pragma unroll
      for (int b = 0; b < W; ++b)
        acc += (T)L.wts[s][m * W + b] * U[(size_t)L.rows[s][m * W + b] * rm + col];
    }
    L.c[slot][s][col] = acc;
  }
}

// One transfer node: acc[k] = tile (w / NT + k (4 / NT), w % NT) of
// (c_a (x) c_b) B, with B [ra rb][rc] row-major.  K steps run a-major; a B
// fragment is fetched four steps ahead of its use.
template <typename T, int NT>
__device__ __forceinline__ void hs_node(const HsLds<T>& L, int ra, int rb, int rc,
                                        const T* __restrict__ B, int w, int lane,
                                        typename Mfma<T>::acc* acc) {
  const int q = lane >> 4, i = lane & 15;
  const int col = 16 * (w % NT) + i;
  const bool colok = col < rc;
  const int nj = (rb + 3) >> 2, nk = ra * nj;
  const float rinv = 1.0f / (float)nj;   // exact floor of (kk + 1/2) / nj for kk < 2^12
  const T(*ca)[HsLds<T>::LDC] = L.c[0];
  const T(*cb)[HsLds<T>::LDC] = L.c[1];
  int mrow[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    mrow[k] = 16 * (w / NT + k * (4 / NT)) + i;
    acc[k] = typename Mfma<T>::acc{0, 0, 0, 0};
  }
  // B fragments are loaded unconditionally from a clamped address (element
  // 0 outside the matrix), so the loads stay in flight across steps: rows
  // past rb meet zero A entries (the slots are zero beyond the rank), and
  // columns past rc are cleared after the loop.
  auto fetch = [&](int kk) -> T {
    const int a = (int)(((float)kk + 0.5f) * rinv);
    const int b = 4 * (kk - a * nj) + q;
    const bool ok = kk < nk && b < rb && colok;
    return B[ok ? (size_t)(a * rb + b) * rc + col : 0];
  };
  int acur = -1;
  T c1[NT];
  // one K step: the Khatri-Rao entries of this lane times the B fragment
  auto step = [&](int kk, T bv) {
    const int a = (int)(((float)kk + 0.5f) * rinv);
    const int b = 4 * (kk - a * nj) + q;
    if (a != acur) {
#pragma unroll
      for (int k = 0; k < NT; ++k) c1[k] = ca[mrow[k]][a];
      acur = a;
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = Mfma<T>::step(c1[k] * cb[mrow[k]][b], bv, acc[k]);
  };
  T ring[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) ring[p] = fetch(p);
  // whole groups of four steps run unguarded, so the fetches stay counted
  // in flight across the loop; a slot is refilled once its steps issue
  const int nk4 = nk & ~3;
  for (int k0 = 0; k0 < nk4; k0 += 4) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      step(k0 + p, ring[p]);
      ring[p] = fetch(k0 + p + 4);
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p)
    if (nk4 + p < nk) step(nk4 + p, ring[p]);
  if (!colok) {
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = typename Mfma<T>::acc{0, 0, 0, 0};
  }
}

// Root form f[s] = sum_c Lop[s][c] sum_e root[c][e] R[s][e], with R in
// slot 1 (K = rk), Lop in slot 0 (N = rn), root [rn][rk].  Ends with the
// per-entry sums in L.part[w % NT][s].
template <typename T, int NT>
__device__ __forceinline__ void hs_root(HsLds<T>& L, int rn, int rk, const T* __restrict__ root,
                                        int w, int lane) {
  const int q = lane >> 4, i = lane & 15;
  const int nt = w % NT, col = 16 * nt + i;
  const bool colok = col < rn;
  typename Mfma<T>::acc z[NT];
  int mrow[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    mrow[k] = 16 * (w / NT + k * (4 / NT));
    z[k] = typename Mfma<T>::acc{0, 0, 0, 0};
  }
  const int nj = (rk + 3) >> 2;
  for (int j = 0; j < nj; ++j) {
    const int e = 4 * j + q;
    const T bv = (colok && e < rk) ? root[(size_t)col * rk + e] : (T)0;
#pragma unroll
    for (int k = 0; k < NT; ++k) z[k] = Mfma<T>::step(L.c[1][mrow[k] + i][e], bv, z[k]);
  }
#pragma unroll
  for (int k = 0; k < NT; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = mrow[k] + Mfma<T>::row(q, v);
      T x = z[k][v] * L.c[0][s][col];
      x += __shfl_xor(x, 8, 16);
      x += __shfl_xor(x, 4, 16);
      x += __shfl_xor(x, 2, 16);
      x += __shfl_xor(x, 1, 16);
      if (i == 0) L.part[nt][s] = x;
    }
}

template <typename T, int W, int DX, int NT>
__global__ __launch_bounds__(256) void k_ht_sample(GridDev g, AdvDev a, HtDev<T> F, long long n,
                                                   const int* __restrict__ idx, T* __restrict__ out) {
  constexpr int d = 2 * DX;
  __shared__ HsLds<T> L;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long long s0 = (long long)blockIdx.x * HS_S;
  {
    // feet: the four lanes of a quad share one entry (entries past n trace
    // grid point 0 and are not stored)
    const int s = t >> 2;
    int gi[4] = {0, 0, 0, 0};
    if (s0 + s < n) {
#pragma unroll
      for (int m = 0; m < d; ++m) gi[m] = idx[(s0 + s) * d + m];
    }
    double ft[4];
    foot_of<DX, 4>(g, a, gi, ft, t & 3);
    int r[4][W];
    double wt[4][W];
#pragma unroll
    for (int m = 0; m < d; ++m) stencil_of<W>(g, a, m, ft[m], gi[m], r[m], wt[m]);
    if ((t & 3) == 0) {
#pragma unroll
      for (int m = 0; m < d; ++m)
#pragma unroll
        for (int b = 0; b < W; ++b) { L.rows[s][m * W + b] = r[m][b]; L.wts[s][m * W + b] = wt[m][b]; }
    }
  }
  __syncthreads();
  hs_interp<T, W>(F, 0, L, t);
  __syncthreads();
  if (d == 4) {
    typename Mfma<T>::acc y12[NT], y34[NT];
    hs_node<T, NT>(L, F.r[0], F.r[1], F.r[4], F.B12, w, lane, y12);
    __syncthreads();
    hs_interp<T, W>(F, 2, L, t);
    __syncthreads();
    hs_node<T, NT>(L, F.r[2], F.r[3], F.r[5], F.B34, w, lane, y34);
    __syncthreads();
    const int q = lane >> 4, i = lane & 15, col = 16 * (w % NT) + i;
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = 16 * (w / NT + k * (4 / NT)) + Mfma<T>::row(q, v);
        L.c[0][s][col] = y12[k][v];
        L.c[1][s][col] = y34[k][v];
      }
    __syncthreads();
    hs_root<T, NT>(L, F.r[4], F.r[5], F.root, w, lane);
  } else {
    hs_root<T, NT>(L, F.r[0], F.r[1], F.root, w, lane);
  }
  __syncthreads();
  if (t < HS_S && s0 + t < n) {
    T f = 0;
#pragma unroll
    for (int k = 0; k < NT; ++k) f += L.part[k][t];
    out[s0 + t] = f;
  }
}

template <typename T, int W, int DX>
static void launch_ht_nt(hipStream_t st, unsigned blocks, int nt, const GridDev& G, const AdvDev& A,
                         const HtDev<T>& H, long long n, const int* idx, T* out) {
  if (nt == 1) k_ht_sample<T, W, DX, 1><<<blocks, 256, 0, st>>>(G, A, H, n, idx, out);
  else if (nt == 2) k_ht_sample<T, W, DX, 2><<<blocks, 256, 0, st>>>(G, A, H, n, idx, out);
  else k_ht_sample<T, W, DX, 4><<<blocks, 256, 0, st>>>(G, A, H, n, idx, out);
}

template <typename T>
static hipError_t launch_ht_sample(hipStream_t st, const GridDev& G, const AdvDev& A,
                                   const slar_ht& F, long long n, const int* idx, void* out) {
  HtDev<T> H{};
  H.d = F.d;
  for (int m = 0; m < 6; ++m) H.r[m] = F.rank[m];
  for (int m = 0; m < F.d; ++m) H.U[m] = (const T*)F.leaf[m];
  H.B12 = (const T*)F.B12; H.B34 = (const T*)F.B34; H.root = (const T*)F.root;
  // column tiles: the widest GEMM output (node ranks, or the x rank of a 2-leaf root)
  const int ncol = F.d == 4 ? (F.rank[4] > F.rank[5] ? F.rank[4] : F.rank[5]) : F.rank[0];
  const int nt = ncol <= 16 ? 1 : (ncol <= 32 ? 2 : 4);
  const unsigned blocks = (unsigned)((n + HS_S - 1) / HS_S);
  if (F.d == 4) launch_ht_nt<T, 3, 2>(st, blocks, nt, G, A, H, n, idx, (T*)out);
  else if (A.order == 5) launch_ht_nt<T, 5, 1>(st, blocks, nt, G, A, H, n, idx, (T*)out);
  else launch_ht_nt<T, 3, 1>(st, blocks, nt, G, A, H, n, idx, (T*)out);
  return hipGetLastError();
}

hipError_t ht_sample(hipStream_t st, const GridDev& G, const AdvDev& A, const slar_ht& F,
                     long long n, const int* idx, void* out) {
  if (n <= 0) return hipSuccess;
  if (F.dtype == SLAR_F32) return launch_ht_sample<float>(st, G, A, F, n, idx, out);
  return launch_ht_sample<double>(st, G, A, F, n, idx, out);
}

// ------------------------------------------------------- frozen field
// Combined frozen field, node-interleaved: out[lin][m] = c0 E0[m][lin] +
// c1 E1[m][lin] (inputs planar [dx][Nx]).
__global__ void k_combine(int nx, int dx, const double* E0, double c0, const double* E1, double c1,
                          double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * dx) return;
  const int lin = e / dx, m = e % dx;
  const size_t in = (size_t)m * nx + lin;
  double v = c0 * E0[in];
  if (E1 != nullptr) v = v + c1 * E1[in];
  out[e] = v;
}

hipError_t combine_field(hipStream_t s, const GridDev& G, const slar_adv* a, double* out) {
  const int count = G.dx * G.nx;
  if (a->E[0] == nullptr) return hipMemsetAsync(out, 0, sizeof(double) * count, s);
  k_combine<<<(count + 255) / 256, 256, 0, s>>>(G.nx, G.dx, a->E[0], a->cE[0], a->E[1], a->cE[1], out);
  return hipGetLastError();
}

// ----------------------------------------------------------- frame build
// X[(i1,i2)][c] = sum_ab U1[i1,a] U2[i2,b] B12[a,b,c]   (x node frame)
// P[(i3,i4)][c] = sum_e ((U3 (x) U4) B34)[(i3,i4)][e] root[c][e]
hipError_t frames_from_ht(hipStream_t s, Workspace* ws, const GridDev& G, const slar_ht& F,
                          slar_frames* out) {
  const int ld = out->ld;
  if (F.d == 2) {
    const int rx = F.rank[0], rv = F.rank[1];
    // X = Ux (n0 x rx); P = Uv root^T (n1 x rx)
    hipError_t e = copy2d(s, G.n[0], rx, (const double*)F.leaf[0], rx, out->X, ld, nullptr);
    if (e != hipSuccess) return e;
    e = gemm_f64(s, false, true, G.n[1], rx, rv, 1.0, (const double*)F.leaf[1], rv, 0,
                 (const double*)F.root, rv, 0, 0.0, out->P, ld, 0, 1);
    out->r = rx;
    return e;
  }
  const int r1 = F.rank[0], r2 = F.rank[1], r3 = F.rank[2], r4 = F.rank[3];
  const int r12 = F.rank[4], r34 = F.rank[5];
  const int n1 = G.n[0], n2 = G.n[1], n3 = G.n[2], n4 = G.n[3];
  double* Z = ws->dwork;   // scratch: max(n1*r2*r12, n3*r4*r34) + n3*n4*r34
  double* V = ws->dwork + (size_t)SLAR_NMAX * SLAR_KMAX * SLAR_KMAX;
  // Z[i1][b*r12 + c] = sum_a U1[i1][a] B12[a][b*r12 + c]
  hipError_t e = gemm_f64(s, false, false, n1, r2 * r12, r1, 1.0, (const double*)F.leaf[0], r1, 0,
                          (const double*)F.B12, r2 * r12, 0, 0.0, Z, r2 * r12, 0, 1);
  if (e != hipSuccess) return e;
  // X[i1][i2][c] = sum_b U2[i2][b] Z[i1][b][c]   (batched over i1)
  e = gemm_f64(s, false, false, n2, r12, r2, 1.0, (const double*)F.leaf[1], r2, 0, Z, r12,
               (long long)r2 * r12, 0.0, out->X, ld, (long long)n2 * ld, n1);
  if (e != hipSuccess) return e;
  e = gemm_f64(s, false, false, n3, r4 * r34, r3, 1.0, (const double*)F.leaf[2], r3, 0,
               (const double*)F.B34, r4 * r34, 0, 0.0, Z, r4 * r34, 0, 1);
  if (e != hipSuccess) return e;
  e = gemm_f64(s, false, false, n4, r34, r4, 1.0, (const double*)F.leaf[3], r4, 0, Z, r34,
               (long long)r4 * r34, 0.0, V, r34, (long long)n4 * r34, n3);
  if (e != hipSuccess) return e;
  // P = V root^T  (Nv x r12)
  e = gemm_f64(s, false, true, n3 * n4, r12, r34, 1.0, V, r34, 0, (const double*)F.root, r34, 0,
               0.0, out->P, ld, 0, 1);
  out->r = r12;
  return e;
}

// The same for n tensors at once, as grouped launches appended to q (one
// per step of the one-tensor call, so each frame is bit-identical to it);
// out[j]->r is set on return.
hipError_t frames_from_ht_group(GroupQueue& q, int n, Workspace* const* ws, const slar_ht* const* F,
                                slar_frames* const* out) {
  std::vector<GemmArgs> g1, g2, g3, g4, g5;
  std::vector<CopyDesc> cp;
  for (int j = 0; j < n; ++j) {
    const GridDev& G = ws[j]->G;
    const slar_ht& H = *F[j];
    slar_frames& o = *out[j];
    const int ld = o.ld;
    if (H.d == 2) {
      const int rx = H.rank[0], rv = H.rank[1];
      cp.push_back(CopyDesc{G.n[0], rx, rx, ld, (const double*)H.leaf[0], o.X, nullptr});
      g5.push_back(GemmArgs{G.n[1], rx, rv, 1.0, (const double*)H.leaf[1], rv, 0, (const double*)H.root, rv, 0,
                            0.0, o.P, ld, 0, 1});
      o.r = rx;
      continue;
    }
    const int r1 = H.rank[0], r2 = H.rank[1], r3 = H.rank[2], r4 = H.rank[3];
    const int r12 = H.rank[4], r34 = H.rank[5];
    const int n1 = G.n[0], n2 = G.n[1], n3 = G.n[2], n4 = G.n[3];
    double* Z = ws[j]->dwork;
    double* V = ws[j]->dwork + (size_t)SLAR_NMAX * SLAR_KMAX * SLAR_KMAX;
    g1.push_back(GemmArgs{n1, r2 * r12, r1, 1.0, (const double*)H.leaf[0], r1, 0, (const double*)H.B12, r2 * r12, 0,
                          0.0, Z, r2 * r12, 0, 1});
    g2.push_back(GemmArgs{n2, r12, r2, 1.0, (const double*)H.leaf[1], r2, 0, Z, r12, (long long)r2 * r12, 0.0, o.X,
                          ld, (long long)n2 * ld, n1});
    g3.push_back(GemmArgs{n3, r4 * r34, r3, 1.0, (const double*)H.leaf[2], r3, 0, (const double*)H.B34, r4 * r34, 0,
                          0.0, Z, r4 * r34, 0, 1});
    g4.push_back(GemmArgs{n4, r34, r4, 1.0, (const double*)H.leaf[3], r4, 0, Z, r34, (long long)r4 * r34, 0.0, V,
                          r34, (long long)n4 * r34, n3});
    g5.push_back(GemmArgs{n3 * n4, r12, r34, 1.0, V, r34, 0, (const double*)H.root, r34, 0, 0.0, o.P, ld, 0, 1});
    o.r = r12;
  }
  // the scratch Z serves the x side, then the v side (as the one-tensor call)
  HIP_CHK(q.copy2d(cp));
  HIP_CHK(q.gemm(false, false, g1));
  HIP_CHK(q.gemm(false, false, g2));
  HIP_CHK(q.gemm(false, false, g3));
  HIP_CHK(q.gemm(false, false, g4));
  return q.gemm(false, true, g5);
}

// ------------------------------------------------ table copies (padded)
__global__ void k_table_copy(int rows, int r, int ldin, const double* __restrict__ in, int ldo,
                             float* __restrict__ o32, double* __restrict__ o64) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * ldo) return;
  const int row = (int)(e / ldo), c = (int)(e % ldo);
  const double v = (c < r) ? in[(long long)row * ldin + c] : 0.0;
  if (o32) o32[e] = (float)v;
  if (o64) o64[e] = v;
}

hipError_t table_copy(hipStream_t s, int rows, int r, int ldin, const double* in, int ldo,
                      float* o32, double* o64) {
  const long long n = (long long)rows * ldo;
  k_table_copy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, r, ldin, in, ldo, o32, o64);
  return hipGetLastError();
}

// ------------------------------------------------- frame points sampler
template <typename T, int W, int DX>
__global__ __launch_bounds__(FS_THREADS) void k_frame_points(GridDev g, AdvDev a,
                                                              const T* __restrict__ X,
                                                              const T* __restrict__ P, int ld,
                                                              int r, long long n,
                                                              const int* __restrict__ idx,
                                                              double* __restrict__ out) {
  __shared__ FsLds<W, DX> L;
  const long long s0 = (long long)blockIdx.x * FS_SAMPLES;
  const int ns = (int)min((long long)FS_SAMPLES, n - s0);
  const int t = threadIdx.x;
  {
    const int s = t >> 2;
    if (s < ns) {
      int gi[4];
      for (int m = 0; m < 2 * DX; ++m) gi[m] = idx[(s0 + s) * (2 * DX) + m];
      fs_prepare<W, DX, 4>(g, a, gi, L, s, t & 3);
    }
  }
  __syncthreads();
  fs_evaluate<T, W, DX>(X, P, ld, r, L, ns);
  __syncthreads();
  if (t < ns) out[s0 + t] = L.val[t];
}

template <typename T>
static hipError_t launch_frame_points(hipStream_t s, const GridDev& G, const AdvDev& A,
                                      const T* X, const T* P, int ld, int r, long long n,
                                      const int* idx, double* out) {
  const unsigned blocks = (unsigned)((n + FS_SAMPLES - 1) / FS_SAMPLES);
  if (G.dx == 1) {
    if (A.order == 5) k_frame_points<T, 5, 1><<<blocks, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, n, idx, out);
    else k_frame_points<T, 3, 1><<<blocks, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, n, idx, out);
  } else {
    k_frame_points<T, 3, 2><<<blocks, FS_THREADS, 0, s>>>(G, A, X, P, ld, r, n, idx, out);
  }
  return hipGetLastError();
}

hipError_t frame_points(hipStream_t s, const GridDev& G, const AdvDev& A, slar_dtype dt,
                        const void* X, const void* P, int ld, int r, long long n, const int* idx,
                        double* out) {
  if (n <= 0) return hipSuccess;
  if (dt == SLAR_F32)
    return launch_frame_points<float>(s, G, A, (const float*)X, (const float*)P, ld, r, n, idx, out);
  return launch_frame_points<double>(s, G, A, (const double*)X, (const double*)P, ld, r, n, idx, out);
}

}  // namespace slar
