// SL-FD entry evaluation (section 3.1).
//  * k_ht_sample: the paper's contraction on an HT tensor: per sample the
//    leaf interpolations c^(mu) = w(xi_mu) U^(mu)_{J_mu}, then the transfer
//    contractions y12 = (c1 (x) c2) B12, y34 = (c3 (x) c4) B34 and the root
//    bilinear form (O(d r^3) per point).  32 samples per block; the
//    contraction loops read B12/B34 with consecutive output ranks on
//    consecutive lanes (coalesced, L2-resident) and c^(mu) from LDS.
//  * frame build: X = (U1 (x) U2) B12 and P = ((U3 (x) U4) B34) root^T as
//    two GEMMs per node.
//  * k_frame_points: eq. (tp_interp) from the node frames (frame_sampler.h)
//    for an explicit list of grid points.
#include "slar_internal.h"
#include "dense.h"
#include "frame_sampler.h"

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

constexpr int HS_TILE = 32;

template <typename T, int W>
__global__ __launch_bounds__(256) void k_ht_sample(GridDev g, AdvDev a, HtDev<T> F, long long n,
                                                   const int* __restrict__ idx, T* __restrict__ out) {
  __shared__ int rows[HS_TILE][4][W];
  __shared__ double wts[HS_TILE][4][W];
  __shared__ T c[4][HS_TILE][SLAR_KMAX];
  __shared__ T y[2][HS_TILE][SLAR_KMAX];
  const int t = threadIdx.x;
  const long long s0 = (long long)blockIdx.x * HS_TILE;
  const int ns = (int)min((long long)HS_TILE, n - s0);
  const int d = F.d;
  if (t < ns) {
    int gi[4];
    for (int m = 0; m < d; ++m) gi[m] = idx[(s0 + t) * d + m];
    double ft[4];
    if (g.dx == 1) foot_of<1>(g, a, gi, ft);
    else foot_of<2>(g, a, gi, ft);
    for (int m = 0; m < d; ++m) stencil_of<W>(g, a, m, ft[m], gi[m], rows[t][m], wts[t][m]);
  }
  __syncthreads();
  // leaf interpolation c^(mu)[s][a] = sum_w w U^(mu)[row_w][a]
  for (int m = 0; m < d; ++m) {
    const int rm = F.r[m];
    const T* U = F.U[m];
    for (int e = t; e < ns * rm; e += blockDim.x) {
      const int s = e / rm, aa = e % rm;
      T acc = 0;
#pragma unroll
      for (int b = 0; b < W; ++b) acc += (T)wts[s][m][b] * U[(size_t)rows[s][m][b] * rm + aa];
      c[m][s][aa] = acc;
    }
  }
  __syncthreads();
  const int wave = t / 64, lane = t % 64;
  if (d == 2) {
    const int rx = F.r[0], rv = F.r[1];
    for (int s = wave; s < ns; s += 4) {
      T p = 0;
      for (int b = lane; b < rv; b += 64) {
        T z = 0;
        for (int aa = 0; aa < rx; ++aa) z += c[0][s][aa] * F.root[aa * rv + b];
        p += z * c[1][s][b];
      }
      for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
      if (lane == 0) out[s0 + s] = p;
    }
    return;
  }
  // transfer contractions of both internal nodes
  for (int node = 0; node < 2; ++node) {
    const int ra = F.r[2 * node], rb = F.r[2 * node + 1], rc = F.r[4 + node];
    const T* B = node == 0 ? F.B12 : F.B34;
    const T(*ca)[SLAR_KMAX] = c[2 * node];
    const T(*cb)[SLAR_KMAX] = c[2 * node + 1];
    for (int e = t; e < ns * rc; e += blockDim.x) {
      const int s = e / rc, cc = e % rc;
      T acc = 0;
      for (int aa = 0; aa < ra; ++aa) {
        T inner = 0;
        const T* Ba = B + (size_t)aa * rb * rc + cc;
        for (int bb = 0; bb < rb; ++bb) inner += cb[s][bb] * Ba[(size_t)bb * rc];
        acc += ca[s][aa] * inner;
      }
      y[node][s][cc] = acc;
    }
  }
  __syncthreads();
  const int r12 = F.r[4], r34 = F.r[5];
  for (int s = wave; s < ns; s += 4) {
    T p = 0;
    for (int e = lane; e < r34; e += 64) {
      T z = 0;
      for (int cc = 0; cc < r12; ++cc) z += y[0][s][cc] * F.root[cc * r34 + e];
      p += z * y[1][s][e];
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if (lane == 0) out[s0 + s] = p;
  }
}

template <typename T>
static hipError_t launch_ht_sample(hipStream_t st, const GridDev& G, const AdvDev& A,
                                   const slar_ht& F, long long n, const int* idx, void* out) {
  HtDev<T> H{};
  H.d = F.d;
  for (int m = 0; m < 6; ++m) H.r[m] = F.rank[m];
  for (int m = 0; m < F.d; ++m) H.U[m] = (const T*)F.leaf[m];
  H.B12 = (const T*)F.B12; H.B34 = (const T*)F.B34; H.root = (const T*)F.root;
  const unsigned blocks = (unsigned)((n + HS_TILE - 1) / HS_TILE);
  if (A.order == 5)
    k_ht_sample<T, 5><<<blocks, 256, 0, st>>>(G, A, H, n, idx, (T*)out);
  else
    k_ht_sample<T, 3><<<blocks, 256, 0, st>>>(G, A, H, n, idx, (T*)out);
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
