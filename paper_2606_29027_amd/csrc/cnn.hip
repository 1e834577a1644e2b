// Learned convolutional preconditioner for the Krylov solve of the
// macroscopic system (an addition to the paper's method, which names
// preconditioning of that solve as future work): FP32 periodic 3x3
// convolutions with tanh between layers, hand-written forward, backward
// (data and weights) and Adam kernels for training, and for use inside the
// solve one fused launch that runs the whole 8 -> 16 -> 16 -> 4 network per
// output tile on the matrix cores (other shapes run layer by layer).
//
// Layout: activations [B][C][H][W]; parameters packed per layer as
// w [Co][Ci][3][3] then b [Co]; out[o,y,x] = b[o] +
// sum_{c,dy,dx} w[o,c,dy,dx] in[c, y+dy-1, x+dx-1] (periodic indices).
//
// Inside the flexible GMRES the network acts on the spectral preconditioner:
//   z = P_spec(v) + rms(v) * CNN([v / rms(v), (U_c - mean U_c) / std U_c]).
#include <cmath>
#include <vector>

#include "slar_internal.h"
#include "fields.h"
#include "lomac.h"

constexpr int CNN_CMAX = 16;
constexpr int CNN_LMAX = 4;

struct slar_cnn {
  int nl = 0;
  int ch[CNN_LMAX + 1] = {};
  int off[CNN_LMAX + 1] = {};   // parameter offsets per layer
  int nparam = 0;
  int maxB = 0, maxHW = 0;
  float* theta = nullptr;
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int step = 0;
  float* act[CNN_LMAX + 1] = {};
  float* d0 = nullptr;
  float* d1 = nullptr;
  float* gpart = nullptr;
  size_t gpart_elems = 0;
  float* lossp = nullptr;
  double* stats = nullptr;
  float* host_loss = nullptr;
  float* bpack = nullptr;   // matrix-core operands of the fused inference (fusable shapes only)
};

namespace slar {

__global__ void k_conv_fwd(int B, int H, int W, int Ci, int Co, const float* __restrict__ in,
                           const float* __restrict__ prm, int act, float* __restrict__ out) {
  __shared__ float w[CNN_CMAX * CNN_CMAX * 9 + CNN_CMAX];
  const int np = Co * Ci * 9 + Co;
  for (int e = threadIdx.x; e < np; e += blockDim.x) w[e] = prm[e];
  __syncthreads();
  const int HW = H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)B * HW) return;
  const int b = (int)(p / HW), pix = (int)(p % HW);
  const int y = pix / W, x = pix % W;
  float acc[CNN_CMAX];
  for (int o = 0; o < Co; ++o) acc[o] = w[Co * Ci * 9 + o];
  for (int c = 0; c < Ci; ++c) {
    const float* ic = in + ((size_t)b * Ci + c) * HW;
    for (int dy = 0; dy < 3; ++dy) {
      const int yy = (y + dy - 1 + H) % H;
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = (x + dx - 1 + W) % W;
        const float vv = ic[yy * W + xx];
        const int t = (c * 3 + dy) * 3 + dx;
        for (int o = 0; o < Co; ++o) acc[o] += w[o * Ci * 9 + t] * vv;
      }
    }
  }
  for (int o = 0; o < Co; ++o) {
    const float z = acc[o];
    out[((size_t)b * Co + o) * HW + pix] = act ? tanhf(z) : z;
  }
}

// dL/d(in) of one layer from dL/dz of its output (transpose correlation)
__global__ void k_conv_bwd_data(int B, int H, int W, int Ci, int Co, const float* __restrict__ dz,
                                const float* __restrict__ prm, float* __restrict__ din) {
  __shared__ float w[CNN_CMAX * CNN_CMAX * 9];
  const int nw = Co * Ci * 9;
  for (int e = threadIdx.x; e < nw; e += blockDim.x) w[e] = prm[e];
  __syncthreads();
  const int HW = H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)B * HW) return;
  const int b = (int)(p / HW), pix = (int)(p % HW);
  const int y = pix / W, x = pix % W;
  float acc[CNN_CMAX];
  for (int c = 0; c < Ci; ++c) acc[c] = 0.f;
  for (int o = 0; o < Co; ++o) {
    const float* go = dz + ((size_t)b * Co + o) * HW;
    for (int dy = 0; dy < 3; ++dy) {
      const int yy = (y - dy + 1 + H) % H;
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = (x - dx + 1 + W) % W;
        const float g = go[yy * W + xx];
        for (int c = 0; c < Ci; ++c) acc[c] += w[o * Ci * 9 + (c * 3 + dy) * 3 + dx] * g;
      }
    }
  }
  for (int c = 0; c < Ci; ++c) din[((size_t)b * Ci + c) * HW + pix] = acc[c];
}

// dz = dL/da * (1 - a^2) for tanh layers
__global__ void k_tanh_bwd(long long n, const float* __restrict__ a, float* __restrict__ d) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] *= (1.f - a[e] * a[e]);
}

// partial weight gradients: part[chunk][e] for e over the layer's parameters
__global__ void k_conv_bwd_w(int B, int H, int W, int Ci, int Co, const float* __restrict__ dz,
                             const float* __restrict__ a_in, int chunk, float* __restrict__ part,
                             int npar) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c0 = blockIdx.y;
  if (e >= npar) return;
  const int HW = H * W;
  const long long P = (long long)B * HW;
  const long long p0 = (long long)c0 * chunk, p1 = min(P, p0 + chunk);
  float acc = 0.f;
  const int nw = Co * Ci * 9;
  if (e < nw) {
    const int o = e / (Ci * 9), rem = e % (Ci * 9), c = rem / 9, t = rem % 9, dy = t / 3, dx = t % 3;
    for (long long p = p0; p < p1; ++p) {
      const int b = (int)(p / HW), pix = (int)(p % HW), y = pix / W, x = pix % W;
      const int yy = (y + dy - 1 + H) % H, xx = (x + dx - 1 + W) % W;
      acc += dz[((size_t)b * Co + o) * HW + pix] * a_in[((size_t)b * Ci + c) * HW + yy * W + xx];
    }
  } else {
    const int o = e - nw;
    for (long long p = p0; p < p1; ++p) {
      const int b = (int)(p / HW), pix = (int)(p % HW);
      acc += dz[((size_t)b * Co + o) * HW + pix];
    }
  }
  part[(size_t)c0 * npar + e] = acc;
}

__global__ void k_sum_part(int npar, int nchunk, const float* __restrict__ part, float* __restrict__ g) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npar) return;
  float acc = 0.f;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * npar + e];
  g[e] = acc;
}

// d = 2 (out - y) / n ; block partial sums of (out - y)^2
__global__ void k_mse(long long n, const float* __restrict__ out, const float* __restrict__ y,
                      float* __restrict__ d, float* __restrict__ lossp) {
  __shared__ float red[256];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float r = 0.f;
  if (e < n) {
    r = out[e] - y[e];
    d[e] = 2.f * r / (float)n;
  }
  red[threadIdx.x] = r * r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0];
}

__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm; v[e] = vv;
  th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// The same layer with the channel counts fixed at compile time: one thread
// per (pixel, group of OG output channels), weights read with uniform
// addresses (scalar loads), accumulators in registers.  Per output channel
// the summation order is that of k_conv_fwd (bias, then c, dy, dx).
template <int CI, int CO, int OG>
__global__ __launch_bounds__(256) void k_conv_fwd_t(int B, int H, int W, const float* __restrict__ in,
                                                    const float* __restrict__ prm, int act,
                                                    float* __restrict__ out) {
  static_assert(CO % OG == 0, "output groups");
  const int HW = H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)B * HW) return;
  const int o0 = blockIdx.y * OG;
  const int b = (int)(p / HW), pix = (int)(p % HW);
  const int y = pix / W, x = pix % W;
  const int rm = (y == 0 ? H - 1 : y - 1) * W, r0 = y * W, rp = (y == H - 1 ? 0 : y + 1) * W;
  const int xm = (x == 0 ? W - 1 : x - 1), xp = (x == W - 1 ? 0 : x + 1);
  float acc[OG];
#pragma unroll
  for (int o = 0; o < OG; ++o) acc[o] = prm[CO * CI * 9 + o0 + o];
#pragma unroll
  for (int c = 0; c < CI; ++c) {
    const float* ic = in + ((size_t)b * CI + c) * HW;
    const float v[9] = {ic[rm + xm], ic[rm + x], ic[rm + xp], ic[r0 + xm], ic[r0 + x],
                        ic[r0 + xp], ic[rp + xm], ic[rp + x], ic[rp + xp]};
#pragma unroll
    for (int o = 0; o < OG; ++o) {
      const float* wo = prm + ((size_t)(o0 + o) * CI + c) * 9;
#pragma unroll
      for (int t = 0; t < 9; ++t) acc[o] += wo[t] * v[t];
    }
  }
#pragma unroll
  for (int o = 0; o < OG; ++o) {
    const float z = acc[o];
    out[((size_t)b * CO + o0 + o) * HW + pix] = act ? tanhf(z) : z;
  }
}

template <int CI, int CO>
static bool conv_fixed(hipStream_t s, int ci, int co, unsigned nb, int B, int H, int W, const float* in,
                       const float* prm, int act, float* out) {
  if (ci != CI || co != CO) return false;
  constexpr int OG = CO < 4 ? CO : 4;
  k_conv_fwd_t<CI, CO, OG><<<dim3(nb, CO / OG), 256, 0, s>>>(B, H, W, in, prm, act, out);
  return true;
}

static hipError_t cnn_forward(hipStream_t s, slar_cnn* c, int B, int H, int W, const float* x) {
  const long long P = (long long)B * H * W;
  const unsigned nb = (unsigned)((P + 255) / 256);
  const float* in = x;
  for (int l = 0; l < c->nl; ++l) {
    const int ci = c->ch[l], co = c->ch[l + 1], act = l < c->nl - 1 ? 1 : 0;
    const float* prm = c->theta + c->off[l];
    float* out = c->act[l + 1];
    const bool fixed = conv_fixed<8, 16>(s, ci, co, nb, B, H, W, in, prm, act, out) ||
                       conv_fixed<16, 16>(s, ci, co, nb, B, H, W, in, prm, act, out) ||
                       conv_fixed<16, 4>(s, ci, co, nb, B, H, W, in, prm, act, out) ||
                       conv_fixed<8, 8>(s, ci, co, nb, B, H, W, in, prm, act, out) ||
                       conv_fixed<8, 4>(s, ci, co, nb, B, H, W, in, prm, act, out);
    if (!fixed) k_conv_fwd<<<nb, 256, 0, s>>>(B, H, W, ci, co, in, prm, act, out);
    in = out;
  }
  return hipGetLastError();
}

// gradient of the MSE loss into c->grad; loss (host) if requested
static hipError_t cnn_backward(hipStream_t s, slar_cnn* c, int B, int H, int W, const float* x,
                               const float* y, float* loss_host) {
  HIP_CHK(cnn_forward(s, c, B, H, W, x));
  const int HW = H * W;
  const long long P = (long long)B * HW;
  const unsigned nb = (unsigned)((P + 255) / 256);
  const int L = c->nl;
  const long long nout = P * c->ch[L];
  const unsigned nbo = (unsigned)((nout + 255) / 256);
  k_mse<<<nbo, 256, 0, s>>>(nout, c->act[L], y, c->d0, c->lossp);
  float* d = c->d0;
  float* dn = c->d1;
  const int chunk = 2048;
  const int nchunk = (int)((P + chunk - 1) / chunk);
  for (int l = L - 1; l >= 0; --l) {
    const int Ci = c->ch[l], Co = c->ch[l + 1];
    if (l < L - 1) k_tanh_bwd<<<(unsigned)((P * Co + 255) / 256), 256, 0, s>>>(P * Co, c->act[l + 1], d);
    const float* a_in = l == 0 ? x : c->act[l];
    const int npar = Co * Ci * 9 + Co;
    if ((size_t)nchunk * npar > c->gpart_elems) return hipErrorInvalidValue;
    k_conv_bwd_w<<<dim3((npar + 255) / 256, nchunk), 256, 0, s>>>(B, H, W, Ci, Co, d, a_in, chunk,
                                                                 c->gpart, npar);
    k_sum_part<<<(npar + 255) / 256, 256, 0, s>>>(npar, nchunk, c->gpart, c->grad + c->off[l]);
    if (l > 0) {
      k_conv_bwd_data<<<nb, 256, 0, s>>>(B, H, W, Ci, Co, d, c->theta + c->off[l], dn);
      float* t = d; d = dn; dn = t;
    }
  }
  HIP_CHK(hipGetLastError());
  if (loss_host) {
    std::vector<float> lp(nbo);
    HIP_CHK(hipMemcpyAsync(lp.data(), c->lossp, sizeof(float) * nbo, hipMemcpyDeviceToHost, s));
    HIP_CHK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (float v : lp) acc += v;
    *loss_host = (float)(acc / (double)nout);
  }
  return hipSuccess;
}

// ---------------------------------------------- use inside the Krylov solve
// Normalisation statistics of one network input, per channel c < K:
// stats[ST_SS + c] = sum v_c^2, stats[ST_MEAN + c] = mean U_c,
// stats[ST_STD + c] = std U_c (three disjoint ranges of ST_STRIDE entries).
constexpr int ST_STRIDE = 16, ST_SS = 0, ST_MEAN = ST_STRIDE, ST_STD = 2 * ST_STRIDE;
constexpr int ST_ELEMS = 3 * CNN_CMAX * 16;   // room for the fused path's partial sums too
static_assert(ST_STRIDE >= CNN_CMAX / 2, "K = input channels / 2 fits one range");

__global__ __launch_bounds__(1024) void k_cnn_stats(int Nx, int K, const double* __restrict__ v,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ stats) {
  __shared__ double r0[1024], r1[1024], r2[1024];
  const int c = blockIdx.x, t = threadIdx.x;
  double a = 0.0, s1 = 0.0, s2 = 0.0;
  for (int e = t; e < Nx; e += 1024) {
    const double x = v[(size_t)c * Nx + e], u = U[(size_t)c * Nx + e];
    a += x * x; s1 += u; s2 += u * u;
  }
  r0[t] = a; r1[t] = s1; r2[t] = s2;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) { r0[t] += r0[t + o]; r1[t] += r1[t + o]; r2[t] += r2[t + o]; }
    __syncthreads();
  }
  if (t == 0) {
    const double mean = r1[0] / Nx;
    const double var = fmax(r2[0] / Nx - mean * mean, 0.0);
    stats[ST_SS + c] = r0[0];
    stats[ST_MEAN + c] = mean;
    stats[ST_STD + c] = sqrt(var) + 1e-12 * fabs(mean) + 1e-300;
  }
}

// rms of v over all K channels
__device__ inline double cnn_rms(const double* __restrict__ stats, int Nx, int K) {
  double ss = 0.0;
  for (int q = 0; q < K; ++q) ss += stats[ST_SS + q];
  return sqrt(ss / (double)(Nx * K));
}

__global__ void k_cnn_features(int Nx, int K, const double* __restrict__ v, const double* __restrict__ U,
                               const double* __restrict__ stats, float* __restrict__ feat) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nx * K) return;
  const int c = e / Nx;
  const double rms = cnn_rms(stats, Nx, K);
  const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
  feat[e] = (float)(v[e] * inv);
  feat[(size_t)K * Nx + e] = (float)((U[e] - stats[ST_MEAN + c]) / stats[ST_STD + c]);
}

__global__ void k_cnn_add(int n, int Nx, int K, const float* __restrict__ out,
                          const double* __restrict__ stats, double* __restrict__ z) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  z[e] += cnn_rms(stats, Nx, K) * (double)out[e];
}

// Partial sums for the statistics, NP chunks per channel: part[(q K + c) NP + b]
// for q = 0 (sum v^2), 1 (sum U), 2 (sum U^2).
constexpr int ST_NP = 16;
static_assert(3 * (CNN_CMAX / 2) * ST_NP <= ST_ELEMS, "partial sums fit the statistics buffer");

__global__ __launch_bounds__(256) void k_cnn_stats_part(int Nx, int K, const double* __restrict__ v,
                                                        const double* __restrict__ U,
                                                        double* __restrict__ part) {
  __shared__ double r0[256], r1[256], r2[256];
  const int c = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const int len = (Nx + ST_NP - 1) / ST_NP, e0 = b * len, e1 = min(Nx, e0 + len);
  double a = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int e = e0 + t; e < e1; e += 256) {
    const double x = v[(size_t)c * Nx + e], u = U[(size_t)c * Nx + e];
    a += x * x; s1 += u; s2 += u * u;
  }
  r0[t] = a; r1[t] = s1; r2[t] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) { r0[t] += r0[t + o]; r1[t] += r1[t + o]; r2[t] += r2[t + o]; }
    __syncthreads();
  }
  if (t == 0) {
    part[(size_t)(0 * K + c) * ST_NP + b] = r0[0];
    part[(size_t)(1 * K + c) * ST_NP + b] = r1[0];
    part[(size_t)(2 * K + c) * ST_NP + b] = r2[0];
  }
}

// ---- fused inference: the convolutions as FP32 matrix-core products.
// A layer on an LDS tile is out[p][o] = b[o] + sum_k X[p][k] W[k][o] with
// k = t CI + c over the taps t = 3 dy + dx and input channels c, X[p][k] =
// in[c][py + dy][px + dx].  One v_mfma_f32_16x16x4f32 step takes 16 pixels
// x 4 values of k: lane l supplies X[16 m + (l & 15)][4 s + (l >> 4)] and
// W[4 s + (l >> 4)][l & 15] and ends with out[16 m + 4 (l >> 4) + i][l & 15],
// i < 4.  With CI a multiple of 4 the tap is the same for the four k of a
// step, so the A operand is an LDS read at a fixed offset from a per-lane
// base.  LDS planes have a channel stride of 16 mod 32 floats, which puts
// the four k rows of a step in disjoint banks.
typedef float cnn_v4f __attribute__((ext_vector_type(4)));

constexpr int cnn_plane(int w) { return ((w * w + 15) / 32) * 32 + 16; }

// B operands of one layer in matrix-core order: row s < CI 9 / 4 holds, at
// lane l, W[k = 4 s + (l >> 4)][o = l & 15] (zero for o >= CO); row
// CI 9 / 4 holds the bias of o = l & 15.  (CI 9 / 4 + 1) x 64 floats.
template <int CI, int CO>
__device__ inline float cnn_b_entry(const float* __restrict__ prm, int s, int l) {
  const int q = l >> 4, o = l & 15;
  if (o >= CO) return 0.f;
  if (s == CI * 9 / 4) return prm[CO * CI * 9 + o];
  const int t = (4 * s) / CI, c = (4 * s) % CI + q;
  return prm[(o * CI + c) * 9 + t];
}

template <int C0, int C1, int C2, int C3>
struct CnnPack {
  static constexpr int R1 = C0 * 9 / 4 + 1, R2 = C1 * 9 / 4 + 1, R3 = C2 * 9 / 4 + 1;
  static constexpr int ELEMS = (R1 + R2 + R3) * 64;
};

template <int C0, int C1, int C2, int C3>
__global__ void k_cnn_pack(const float* __restrict__ theta, int off1, int off2, float* __restrict__ bp) {
  using PK = CnnPack<C0, C1, C2, C3>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= PK::ELEMS) return;
  const int row = e >> 6, l = e & 63;
  float x;
  if (row < PK::R1) x = cnn_b_entry<C0, C1>(theta, row, l);
  else if (row < PK::R1 + PK::R2) x = cnn_b_entry<C1, C2>(theta + off1, row - PK::R1, l);
  else x = cnn_b_entry<C2, C3>(theta + off2, row - PK::R1 - PK::R2, l);
  bp[e] = x;
}

// this lane's B operands and bias of one layer from its packed rows
template <int CI>
__device__ inline void cnn_load_b(const float* __restrict__ rows, float* wb, float& bias) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < CI * 9 / 4; ++s) wb[s] = rows[s * 64 + l];
  bias = rows[(CI * 9 / 4) * 64 + l];
}

// in: [CI] planes of IW x IW (stride cnn_plane(IW)); out: [CO] planes of
// OW x OW, OW = IW - 2, with channel stride OS
template <int CI, int CO, int IW, int OS, bool ACT>
__device__ inline void cnn_layer_mfma(const float* __restrict__ in, float* __restrict__ out,
                                     const float* wb, float bias) {
  static_assert(CI % 4 == 0 && CO <= 16, "four k per step, one column tile");
  constexpr int OW = IW - 2, P = OW * OW, MT = (P + 15) / 16, KS = CI * 9 / 4, IS = cnn_plane(IW);
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
  for (int m = threadIdx.x >> 6; m < MT; m += blockDim.x >> 6) {
    const int pa = min(16 * m + r, P - 1);   // rows past P read a valid pixel and are dropped
    const int py = pa / OW, px = pa - py * OW;
    const float* base = in + q * IS + py * IW + px;
    cnn_v4f acc = {bias, bias, bias, bias};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int t = (4 * s) / CI, c0 = (4 * s) % CI;
      const float a = base[c0 * IS + (t / 3) * IW + t % 3];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, wb[s], acc, 0, 0, 0);
    }
    if (r < CO) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * m + 4 * q + i;
        if (p < P) out[r * OS + p] = ACT ? tanhf(acc[i]) : acc[i];
      }
    }
  }
}

// The whole correction for a three-layer network C0 -> C1 -> C2 -> C3
// (C0 = 2K, C3 = K): one block per TS x TS output tile of the H x W grid.
// Every global load (partial sums, v and U on the tile plus a three-pixel
// periodic halo, the z entries of the tile, this lane's packed weights) is issued
// up front; the statistics are then finished, the normalised input is
// written to LDS, the layers run in LDS and z[c][pixel] += rms(v) out[c] is
// stored.
constexpr int CNN_TS = 8, CNN_NT = 512;

template <int C0, int C1, int C2, int C3>
__global__ __launch_bounds__(CNN_NT) void k_cnn_fused(int H, int W, const double* __restrict__ v,
                                                      const double* __restrict__ U,
                                                      const double* __restrict__ part,
                                                      const float* __restrict__ bp,
                                                      double* __restrict__ z) {
  using PK = CnnPack<C0, C1, C2, C3>;
  constexpr int K = C3, I0 = CNN_TS + 6, I1 = CNN_TS + 4, I2 = CNN_TS + 2;
  constexpr int S0 = cnn_plane(I0), S1 = cnn_plane(I1), S2 = cnn_plane(I2), S3 = CNN_TS * CNN_TS;
  constexpr int NE = K * I0 * I0, NR = (NE + CNN_NT - 1) / CNN_NT, NZ = K * S3;
  static_assert(C0 == 2 * C3, "input channels 2K, output channels K");
  static_assert(NZ <= CNN_NT && 3 * K <= CNN_NT, "one output entry per thread");
  __shared__ float a0[C0 * S0];
  __shared__ float a1[C1 * S1];
  __shared__ float a2[C2 * S2];
  __shared__ float a3[C3 * S3];
  __shared__ double sums[3 * K], s_mean[K], s_sd[K];
  __shared__ double s_rms;
  const int t = threadIdx.x, Nx = H * W;
  const int tx0 = blockIdx.x * CNN_TS, ty0 = blockIdx.y * CNN_TS;
  double acc = 0.0;
  if (t < 3 * K) {
#pragma unroll
    for (int b = 0; b < ST_NP; ++b) acc += part[(size_t)t * ST_NP + b];
  }
  double vv[NR], uu[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = t + r * CNN_NT;
    vv[r] = 0.0; uu[r] = 0.0;
    if (e < NE) {
      const int c = e / (I0 * I0), q = e - c * (I0 * I0), iy = q / I0, ix = q - iy * I0;
      int gy = (ty0 + iy - 3) % H, gx = (tx0 + ix - 3) % W;
      gy += gy < 0 ? H : 0;
      gx += gx < 0 ? W : 0;
      const size_t g = (size_t)c * Nx + (size_t)gy * W + gx;
      vv[r] = v[g];
      uu[r] = U[g];
    }
  }
  long long zi = -1;
  double zz = 0.0;
  if (t < NZ) {
    const int c = t / S3, q = t - c * S3;
    const int y = ty0 + q / CNN_TS, x = tx0 + q % CNN_TS;
    if (y < H && x < W) {
      zi = (long long)c * Nx + (long long)y * W + x;
      zz = z[zi];
    }
  }
  float w1[C0 * 9 / 4], w2[C1 * 9 / 4], w3[C2 * 9 / 4], b1, b2, b3;
  cnn_load_b<C0>(bp, w1, b1);
  cnn_load_b<C1>(bp + PK::R1 * 64, w2, b2);
  cnn_load_b<C2>(bp + (PK::R1 + PK::R2) * 64, w3, b3);
  if (t < 3 * K) sums[t] = acc;
  __syncthreads();
  if (t < K) {
    const double mean = sums[K + t] / Nx;
    const double var = fmax(sums[2 * K + t] / Nx - mean * mean, 0.0);
    s_mean[t] = mean;
    s_sd[t] = sqrt(var) + 1e-12 * fabs(mean) + 1e-300;
  } else if (t == K) {
    double ss = 0.0;
    for (int q = 0; q < K; ++q) ss += sums[q];
    s_rms = sqrt(ss / (double)(Nx * K));
  }
  __syncthreads();
  const double rms = s_rms, inv = rms > 0.0 ? 1.0 / rms : 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = t + r * CNN_NT;
    if (e < NE) {
      const int c = e / (I0 * I0), q = e - c * (I0 * I0);
      a0[c * S0 + q] = (float)(vv[r] * inv);
      a0[(K + c) * S0 + q] = (float)((uu[r] - s_mean[c]) / s_sd[c]);
    }
  }
  __syncthreads();
  cnn_layer_mfma<C0, C1, I0, S1, true>(a0, a1, w1, b1);
  __syncthreads();
  cnn_layer_mfma<C1, C2, I1, S2, true>(a1, a2, w2, b2);
  __syncthreads();
  cnn_layer_mfma<C2, C3, I2, S3, false>(a2, a3, w3, b3);
  __syncthreads();
  if (zi >= 0) z[zi] = zz + rms * (double)a3[t];
}

// the fused inference covers 8 -> 16 -> 16 -> 4 (2D2V moments, 16 hidden)
static bool cnn_fusable(const slar_cnn* c) {
  return c->nl == 3 && c->ch[0] == 8 && c->ch[1] == 16 && c->ch[2] == 16 && c->ch[3] == 4;
}

static constexpr int CNN_PACK_ELEMS = CnnPack<8, 16, 16, 4>::ELEMS;

// refresh the packed operands after the parameters changed (stream order)
static hipError_t cnn_repack(hipStream_t s, slar_cnn* c) {
  if (!c->bpack) return hipSuccess;
  k_cnn_pack<8, 16, 16, 4><<<(CNN_PACK_ELEMS + 255) / 256, 256, 0, s>>>(c->theta, c->off[1], c->off[2],
                                                                       c->bpack);
  return hipGetLastError();
}

hipError_t cnn_apply(hipStream_t s, Workspace* ws, const slar_cnn* net, const double* v,
                     const double* U, double* z) {
  slar_cnn* c = const_cast<slar_cnn*>(net);
  const GridDev& G = ws->G;
  if (G.dx != 2 || c->ch[0] != 2 * (G.dv + 2) || c->ch[c->nl] != G.dv + 2) return hipErrorInvalidValue;
  const int K = G.dv + 2, Nx = G.nx, H = G.n[0], W = G.n[1];
  if (c->bpack) {
    k_cnn_stats_part<<<dim3(ST_NP, K), 256, 0, s>>>(Nx, K, v, U, c->stats);
    const dim3 grid((W + CNN_TS - 1) / CNN_TS, (H + CNN_TS - 1) / CNN_TS);
    k_cnn_fused<8, 16, 16, 4><<<grid, CNN_NT, 0, s>>>(H, W, v, U, c->stats, c->bpack, z);
    return hipGetLastError();
  }
  if (Nx > c->maxHW) return hipErrorInvalidValue;
  k_cnn_stats<<<K, 1024, 0, s>>>(Nx, K, v, U, c->stats);
  k_cnn_features<<<(Nx * K + 255) / 256, 256, 0, s>>>(Nx, K, v, U, c->stats, c->act[0]);
  HIP_CHK(cnn_forward(s, c, 1, H, W, c->act[0]));
  k_cnn_add<<<(Nx * K + 255) / 256, 256, 0, s>>>(Nx * K, Nx, K, c->act[c->nl], c->stats, z);
  return hipGetLastError();
}

// training pair from a flexible-GMRES step: w = J z; features of w and the
// target (z - P_spec(w)) / rms(w)
__global__ void k_record_target(int n, int Nx, int K, const double* __restrict__ z,
                                const double* __restrict__ pw, const double* __restrict__ stats,
                                float* __restrict__ tgt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double rms = cnn_rms(stats, Nx, K);
  tgt[e] = rms > 0.0 ? (float)((z[e] - pw[e]) / rms) : 0.f;
}

hipError_t record_pair(hipStream_t s, Workspace* ws, const double* w, const double* z,
                       const double* U, const double* pw) {
  if (!ws->rec_feat || ws->rec_count >= ws->rec_cap) return hipSuccess;
  const GridDev& G = ws->G;
  const int K = G.dv + 2, Nx = G.nx;
  double* stats = ws->small + 4096;
  float* feat = ws->rec_feat + (size_t)ws->rec_count * 2 * K * Nx;
  float* tgt = ws->rec_targ + (size_t)ws->rec_count * K * Nx;
  k_cnn_stats<<<K, 1024, 0, s>>>(Nx, K, w, U, stats);
  k_cnn_features<<<(Nx * K + 255) / 256, 256, 0, s>>>(Nx, K, w, U, stats, feat);
  k_record_target<<<(Nx * K + 255) / 256, 256, 0, s>>>(Nx * K, Nx, K, z, pw, stats, tgt);
  ws->rec_count += 1;
  return hipGetLastError();
}

}  // namespace slar

using namespace slar;

extern "C" {

slar_status slar_cnn_create(int32_t nlayers, const int32_t* channels, int32_t max_batch,
                            int32_t max_pixels, slar_cnn** out) {
  if (!out || nlayers < 1 || nlayers > CNN_LMAX || !channels || max_batch < 1 || max_pixels < 1)
    return SLAR_E_INVAL;
  for (int l = 0; l <= nlayers; ++l)
    if (channels[l] < 1 || channels[l] > CNN_CMAX) return SLAR_E_INVAL;
  slar_cnn* c = new (std::nothrow) slar_cnn();
  if (!c) return SLAR_E_NOMEM;
  c->nl = nlayers;
  int o = 0, cmax = 0;
  for (int l = 0; l <= nlayers; ++l) { c->ch[l] = channels[l]; cmax = std::max(cmax, channels[l]); }
  for (int l = 0; l < nlayers; ++l) { c->off[l] = o; o += c->ch[l + 1] * c->ch[l] * 9 + c->ch[l + 1]; }
  c->off[nlayers] = o;
  c->nparam = o;
  c->maxB = max_batch;
  c->maxHW = max_pixels;
  const size_t actn = (size_t)max_batch * max_pixels * cmax;
  bool ok = true;
  auto al = [&](void** p, size_t bytes) { if (ok && hipMalloc(p, std::max(bytes, (size_t)256)) != hipSuccess) ok = false; };
  al((void**)&c->theta, sizeof(float) * o);
  al((void**)&c->grad, sizeof(float) * o);
  al((void**)&c->m, sizeof(float) * o);
  al((void**)&c->v, sizeof(float) * o);
  for (int l = 0; l <= nlayers; ++l) al((void**)&c->act[l], sizeof(float) * actn);
  al((void**)&c->d0, sizeof(float) * actn);
  al((void**)&c->d1, sizeof(float) * actn);
  c->gpart_elems = (size_t)((actn / cmax + 2047) / 2048 + 1) * (CNN_CMAX * CNN_CMAX * 9 + CNN_CMAX);
  al((void**)&c->gpart, sizeof(float) * c->gpart_elems);
  al((void**)&c->lossp, sizeof(float) * (actn / 256 + 2));
  al((void**)&c->stats, sizeof(double) * ST_ELEMS);
  if (cnn_fusable(c)) al((void**)&c->bpack, sizeof(float) * CNN_PACK_ELEMS);
  if (ok) {
    if (hipMemset(c->theta, 0, sizeof(float) * o) != hipSuccess || hipMemset(c->m, 0, sizeof(float) * o) != hipSuccess ||
        hipMemset(c->v, 0, sizeof(float) * o) != hipSuccess)
      ok = false;
  }
  if (ok && (cnn_repack(nullptr, c) != hipSuccess || hipDeviceSynchronize() != hipSuccess)) ok = false;
  if (!ok) { slar_cnn_destroy(c); return SLAR_E_NOMEM; }
  *out = c;
  return SLAR_OK;
}

slar_status slar_cnn_destroy(slar_cnn* c) {
  if (!c) return SLAR_OK;
  void* ptrs[] = {c->theta, c->grad, c->m, c->v, c->d0, c->d1, c->gpart, c->lossp, c->stats, c->bpack};
  for (void* p : ptrs) if (p) (void)hipFree(p);
  for (int l = 0; l <= CNN_LMAX; ++l) if (c->act[l]) (void)hipFree(c->act[l]);
  delete c;
  return SLAR_OK;
}

int32_t slar_cnn_nparams(const slar_cnn* c) { return c ? c->nparam : 0; }

slar_status slar_cnn_set_params(slar_cnn* c, const float* host, int32_t n) {
  if (!c || !host || n != c->nparam) return SLAR_E_INVAL;
  HIP_TRY(hipMemcpy(c->theta, host, sizeof(float) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(c->m, 0, sizeof(float) * n));
  HIP_TRY(hipMemset(c->v, 0, sizeof(float) * n));
  HIP_TRY(cnn_repack(nullptr, c));
  HIP_TRY(hipDeviceSynchronize());
  c->step = 0;
  return SLAR_OK;
}

slar_status slar_cnn_get_params(const slar_cnn* c, float* host, int32_t n) {
  if (!c || !host || n != c->nparam) return SLAR_E_INVAL;
  HIP_TRY(hipMemcpy(host, c->theta, sizeof(float) * n, hipMemcpyDeviceToHost));
  return SLAR_OK;
}

static bool cnn_dims_ok(const slar_cnn* c, int B, int H, int W) {
  return c && B >= 1 && B <= c->maxB && H >= 1 && W >= 1 && (long long)H * W <= c->maxHW;
}

slar_status slar_cnn_forward(slar_cnn* c, int32_t B, int32_t H, int32_t W, const float* x, float* y,
                             hipStream_t s) {
  if (!cnn_dims_ok(c, B, H, W) || !x || !y) return SLAR_E_INVAL;
  if (cnn_forward(s, c, B, H, W, x) != hipSuccess) return SLAR_E_HIP;
  HIP_TRY(hipMemcpyAsync(y, c->act[c->nl], sizeof(float) * (size_t)B * H * W * c->ch[c->nl],
                         hipMemcpyDeviceToDevice, s));
  return SLAR_OK;
}

slar_status slar_cnn_grad(slar_cnn* c, int32_t B, int32_t H, int32_t W, const float* x,
                          const float* y, float* grad_host, float* loss_host, hipStream_t s) {
  if (!cnn_dims_ok(c, B, H, W) || !x || !y) return SLAR_E_INVAL;
  if (cnn_backward(s, c, B, H, W, x, y, loss_host) != hipSuccess) return SLAR_E_HIP;
  if (grad_host) {
    HIP_TRY(hipMemcpyAsync(grad_host, c->grad, sizeof(float) * c->nparam, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return SLAR_OK;
}

slar_status slar_cnn_train_step(slar_cnn* c, int32_t B, int32_t H, int32_t W, const float* x,
                                const float* y, float lr, float* loss_host, hipStream_t s) {
  if (!cnn_dims_ok(c, B, H, W) || !x || !y || !(lr > 0.f)) return SLAR_E_INVAL;
  if (cnn_backward(s, c, B, H, W, x, y, loss_host) != hipSuccess) return SLAR_E_HIP;
  c->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
  k_adam<<<(c->nparam + 255) / 256, 256, 0, s>>>(c->nparam, c->theta, c->grad, c->m, c->v, lr, b1, b2,
                                                 1e-8f, c1, c2);
  HIP_TRY(hipGetLastError());
  HIP_TRY(cnn_repack(s, c));
  return SLAR_OK;
}

slar_status slar_record_krylov(slar_workspace* w, float* features, float* targets, int32_t capacity) {
  if (!w || capacity < 0 || (capacity > 0 && (!features || !targets))) return SLAR_E_INVAL;
  w->w.rec_feat = capacity > 0 ? features : nullptr;
  w->w.rec_targ = capacity > 0 ? targets : nullptr;
  w->w.rec_cap = capacity;
  w->w.rec_count = 0;
  return SLAR_OK;
}

int32_t slar_recorded_pairs(const slar_workspace* w) { return w ? w->w.rec_count : 0; }

}  // extern "C"
