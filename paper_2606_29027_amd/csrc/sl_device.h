// Device-side geometry of the semi-Lagrangian update (section 3.1): the
// grid, one linear sub-flow, the feet of the characteristics (RK4 along
// the frozen field, degree-4 periodic field interpolation) and the
// interpolation stencils at the feet.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/slar.h"
#include "dpp.h"

namespace slar {

struct GridDev {
  int dx, dv, d;
  int n[4];
  double lo[4];
  double h[4];
  double ih[4];   // 1 / h
  int nx;   // prod n_x
  int nv;   // prod n_v
};

inline GridDev make_grid(const slar_grid& g) {
  GridDev G{};
  G.dx = g.dx; G.dv = g.dv; G.d = g.dx + g.dv;
  G.nx = 1; G.nv = 1;
  for (int m = 0; m < G.d; ++m) {
    G.n[m] = g.n[m];
    G.lo[m] = g.lo[m];
    G.h[m] = (g.hi[m] - g.lo[m]) / (double)g.n[m];
    G.ih[m] = 1.0 / G.h[m];
    if (m < g.dx) G.nx *= g.n[m]; else G.nv *= g.n[m];
  }
  return G;
}

struct AdvDev {
  int kind;
  int order;
  double tau;
  double cv;
  const double* E;    // frozen field = cE0 * E + cE1 * E1
  const double* E1;   // may be null
  double cE0, cE1;
  int inter;          // layout of E/E1: 0 planar [dx][Nx], 1 node-interleaved [Nx][dx]
};

// Offset of component m at spatial node lin.
__device__ __forceinline__ size_t efield_off(const GridDev& g, const AdvDev& a, int lin, int m) {
  return a.inter ? (size_t)lin * g.dx + m : (size_t)m * g.nx + lin;
}

// Field at node offset off.  TWO says whether E1 is present; it is a
// template argument so that node loads are not split by a branch each.
template <bool TWO>
__device__ __forceinline__ double efield_node(const AdvDev& a, size_t off) {
  double v = a.cE0 * a.E[off];
  if (TWO) v = v + a.cE1 * a.E1[off];
  return v;
}

__device__ __forceinline__ int wrap(int j, int n) {
  // one period away is the common case; the remainder only beyond that
  if (j < 0) j += n;
  else if (j >= n) j -= n;
  if ((unsigned)j >= (unsigned)n) {
    j %= n;
    if (j < 0) j += n;
  }
  return j;
}

// Lagrange weights on nodes -(w/2)..(w/2) evaluated at xi:
// l_m(xi) = prod_{n != m} (xi - n) / (m - n); the constant denominators are
// folded into one reciprocal per weight.
template <int W>
__device__ __forceinline__ void lagrange(double xi, double* w) {
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int m = a - W / 2;
    double p = 1.0;
    double den = 1.0;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int nn = b - W / 2;
      if (nn != m) { p = p * (xi - (double)nn); den *= (double)(m - nn); }
    }
    w[a] = p * (1.0 / den);
  }
}

__device__ __forceinline__ void quad_weights(double xi, double* w) {
  w[0] = 0.5 * xi * (xi - 1.0);
  w[1] = 1.0 - xi * xi;
  w[2] = 0.5 * xi * (xi + 1.0);
}

// Degree-4 periodic tensor-product interpolation of every component of the
// frozen field at the spatial point X (out[0..dx-1]).  The Lagrange weights
// and wrapped node indices are shared by the components.  NL = 4: the four
// lanes of a quad (lane = t & 3) cooperate on one point, lane (h, c) summing
// component c over node rows 3h..3h+2 (2D); every lane of the quad returns
// the same values.  NL = 1: one lane does everything.
template <int DX, int NL, bool TWO>
__device__ __forceinline__ void efield_all(const GridDev& g, const AdvDev& ad, const double* X,
                                           int lane, double* out) {
  if (DX == 1) {
    const double s = (X[0] - g.lo[0]) * g.ih[0];
    const double jf = floor(s);
    double w[5];
    lagrange<5>(s - jf - 0.5, w);
    const int n0 = g.n[0];
    const int base = wrap((int)jf - 2, n0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      int j = base + a;
      j -= (j >= n0) ? n0 : 0;
      acc += w[a] * efield_node<TWO>(ad, j);
    }
    out[0] = acc;
    return;
  }
  const double s0 = (X[0] - g.lo[0]) * g.ih[0];
  const double s1 = (X[1] - g.lo[1]) * g.ih[1];
  const double j0f = floor(s0), j1f = floor(s1);
  double w0[5], w1[5];
  lagrange<5>(s0 - j0f - 0.5, w0);
  lagrange<5>(s1 - j1f - 0.5, w1);
  const int n0 = g.n[0], n1 = g.n[1];
  const int b0 = wrap((int)j0f - 2, n0), b1 = wrap((int)j1f - 2, n1);
  int col[5];
#pragma unroll
  for (int b = 0; b < 5; ++b) col[b] = b1 + b - ((b1 + b >= n1) ? n1 : 0);
  if (NL == 1) {
    double e0 = 0.0, e1 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      int ra = b0 + a;
      ra -= (ra >= n0) ? n0 : 0;
      double r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        r0 += w1[b] * efield_node<TWO>(ad, efield_off(g, ad, ra * n1 + col[b], 0));
        r1 += w1[b] * efield_node<TWO>(ad, efield_off(g, ad, ra * n1 + col[b], 1));
      }
      e0 += w0[a] * r0;
      e1 += w0[a] * r1;
    }
    out[0] = e0;
    out[1] = e1;
    return;
  }
  if (!TWO && ad.inter) {
    // node-interleaved field: lane q reads column q of every node row (and
    // lane 0 column 4 too; the other lanes repeat their column with weight
    // 0), both components per 16-byte load, so the four lanes of a quad
    // touch neighbouring nodes
    const int q = lane;
    const double wq = (q == 0) ? w1[0] : (q == 1) ? w1[1] : (q == 2) ? w1[2] : w1[3];
    const int cq = col[0] + q - ((col[0] + q >= n1) ? n1 : 0);
    const int c2 = (q == 0) ? col[4] : cq;
    const double w2 = (q == 0) ? w1[4] : 0.0;
    const double2* E2 = reinterpret_cast<const double2*>(ad.E);
    double e0 = 0.0, e1 = 0.0, f0 = 0.0, f1 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      int ra = b0 + a;
      ra -= (ra >= n0) ? n0 : 0;
      const double2 u = E2[(size_t)ra * n1 + cq];
      const double2 v = E2[(size_t)ra * n1 + c2];
      e0 += w0[a] * u.x; e1 += w0[a] * u.y;
      f0 += w0[a] * v.x; f1 += w0[a] * v.y;
    }
    double s0 = ad.cE0 * (wq * e0 + w2 * f0), s1 = ad.cE0 * (wq * e1 + w2 * f1);
    s0 = group_sum<4>(s0);
    s1 = group_sum<4>(s1);
    out[0] = s0;
    out[1] = s1;
    return;
  }
  const int c = lane & 1, h = lane >> 1;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // rows 0, 1, 2 (h = 0) or 3, 4 and a zero-weight repeat of 4 (h = 1)
    const double wa = (h == 0) ? w0[i] : (i < 2 ? w0[3 + i] : 0.0);
    int ra = b0 + min(3 * h + i, 4);
    ra -= (ra >= n0) ? n0 : 0;
    double r = 0.0;
#pragma unroll
    for (int b = 0; b < 5; ++b) r += w1[b] * efield_node<TWO>(ad, efield_off(g, ad, ra * n1 + col[b], c));
    acc += wa * r;
  }
  acc += dpp_move<0x4E>(acc);                 // both row halves (a + b == b + a: same in both lanes)
  const double other = dpp_move<0xB1>(acc);   // the other component
  out[0] = (c == 0) ? acc : other;
  out[1] = (c == 0) ? other : acc;
}

// RK4 backwards along the frozen-field flow: d/ds (X, V) = (-c V, +E(X)),
// s in [0, tau], from the grid point (X, V).
// The first stage evaluates the field at the grid node itself, where the
// interpolant equals the nodal value: it is read directly.
template <int DX, int NL, bool TWO>
__device__ __forceinline__ void foot_rk4(const GridDev& g, const AdvDev& a, const double* X,
                                         const double* V, int node, double* out, int lane) {
  constexpr int dx = DX;
  const double t = a.tau, c = a.cv;
  double k1x[2], k1v[2], k2x[2], k2v[2], k3x[2], k3v[2], k4x[2], k4v[2], Y[2];
  for (int m = 0; m < dx; ++m) k1x[m] = -c * V[m];
  for (int m = 0; m < dx; ++m) k1v[m] = efield_node<TWO>(a, efield_off(g, a, node, m));
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + 0.5 * t * k1x[m];
  for (int m = 0; m < dx; ++m) k2x[m] = -c * (V[m] + 0.5 * t * k1v[m]);
  efield_all<DX, NL, TWO>(g, a, Y, lane, k2v);
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + 0.5 * t * k2x[m];
  for (int m = 0; m < dx; ++m) k3x[m] = -c * (V[m] + 0.5 * t * k2v[m]);
  efield_all<DX, NL, TWO>(g, a, Y, lane, k3v);
  for (int m = 0; m < dx; ++m) Y[m] = X[m] + t * k3x[m];
  for (int m = 0; m < dx; ++m) k4x[m] = -c * (V[m] + t * k3v[m]);
  efield_all<DX, NL, TWO>(g, a, Y, lane, k4v);
  for (int m = 0; m < dx; ++m) {
    out[m] = X[m] + (t / 6.0) * (k1x[m] + 2.0 * k2x[m] + 2.0 * k3x[m] + k4x[m]);
    out[dx + m] = V[m] + (t / 6.0) * (k1v[m] + 2.0 * k2v[m] + 2.0 * k3v[m] + k4v[m]);
  }
}

// Foot of the characteristic through grid point idx (section 3.1); DX =
// g.dx.  NL as for efield_all (all four lanes of a quad pass the same idx).
template <int DX, int NL = 1>
__device__ __forceinline__ void foot_of(const GridDev& g, const AdvDev& a, const int* idx,
                                        double* out, int lane = 0) {
  double X[2], V[2];
  constexpr int dx = DX;
  for (int m = 0; m < dx; ++m) {
    X[m] = g.lo[m] + ((double)idx[m] + 0.5) * g.h[m];
    V[m] = g.lo[dx + m] + ((double)idx[dx + m] + 0.5) * g.h[dx + m];
  }
  if (a.kind == 0) {
    for (int m = 0; m < dx; ++m) { out[m] = X[m] - a.cv * a.tau * V[m]; out[dx + m] = V[m]; }
    return;
  }
  if (a.kind == 1) {
    int lin = idx[0];
    if (DX == 2) lin = idx[0] * g.n[1] + idx[1];
    for (int m = 0; m < dx; ++m) {
      const size_t off = efield_off(g, a, lin, m);
      out[m] = X[m];
      out[dx + m] = V[m] + a.tau * (a.E1 != nullptr ? efield_node<true>(a, off) : efield_node<false>(a, off));
    }
    return;
  }
  const int node = (DX == 2) ? idx[0] * g.n[1] + idx[1] : idx[0];
  if (a.E1 != nullptr) foot_rk4<DX, NL, true>(g, a, X, V, node, out, lane);
  else foot_rk4<DX, NL, false>(g, a, X, V, node, out, lane);
}

// Stencil rows (wrapped) and weights of dimension m for a foot coordinate.
template <int W>
__device__ __forceinline__ void stencil_of(const GridDev& g, const AdvDev& a, int m, double xf,
                                           int gidx, int* rows, double* w) {
  const bool moving = (a.kind == 2) || (a.kind == 0 && m < g.dx) || (a.kind == 1 && m >= g.dx);
  int j;
  if (moving) {
    const double s = (xf - g.lo[m]) * g.ih[m];
    const double jf = floor(s);
    const double xi = s - jf - 0.5;
    j = (int)jf;
    if (W == 3) quad_weights(xi, w); else lagrange<W>(xi, w);
  } else {
    j = gidx;
#pragma unroll
    for (int b = 0; b < W; ++b) w[b] = (b == W / 2) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int b = 0; b < W; ++b) rows[b] = wrap(j + b - W / 2, g.n[m]);
}

}  // namespace slar
