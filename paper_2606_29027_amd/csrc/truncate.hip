// HTACA final truncation (Supplement B): from the cross factors
// F ~ sum_l U[l] (x) V[l] to a truncated HT tensor.
//   1. Cholesky-QR2 (with column scaling) of both factor sets:
//      U^T = Qu^T Ru, V^T = Qv^T Rv (Q rows orthonormal);
//   2. one-sided Jacobi SVD of the core Ru Rv^T = W diag(s) Z^T;
//   3. root rank r = smallest with tail ||s[r:]|| <= theta,
//      theta = tol ||s|| / sqrt(2d - 3), capped at rmax; frames
//      X = Qu^T W_r, Y = Qv^T Z_r, sign rule on X (flip Y alike);
//   4. d = 2: leaves X, Y, root diag(s_r);
//      d = 4: per side, Gram matrices of the two mode matricisations of
//      frame * diag(s) (split-K GEMMs), Jacobi eigendecompositions, leaf =
//      leading eigenvectors (same theta on sqrt(eigenvalue) tails, sign
//      rule), transfer tensor = frame projected on the two leaf bases.
#include <cmath>
#include <vector>

#include "slar_internal.h"
#include "dense.h"

namespace slar {

static int tail_rank(const std::vector<double>& s2, double theta, int rmax) {
  // s2 are squared singular values, descending
  const int n = (int)s2.size();
  std::vector<double> tail(n + 1, 0.0);
  for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + std::max(s2[i], 0.0);
  int r = n;
  for (int c = 0; c < n; ++c)
    if (std::sqrt(tail[c]) <= theta) { r = c; break; }
  r = std::max(1, std::min(r, rmax));
  return r;
}

struct Tbuf {
  double *Q1u, *Qu, *Q1v, *Qv, *X, *Y, *Xs, *T;
  double *Gu, *Linv, *R1, *R, *M, *W, *Z, *sv;
  double *G1, *G2, *E1, *E2, *Vw, *lam1, *lam2;
};

static Tbuf carve(Workspace* ws) {
  const GridDev& G = ws->G;
  double* p = ws->small;   // large enough for everything below (see api.hip)
  const size_t K = SLAR_KMAX, NN = (size_t)SLAR_NMAX * SLAR_NMAX;
  Tbuf b;
  b.Q1u = p; p += K * G.nx;
  b.Qu = p; p += K * G.nx;
  b.Q1v = p; p += K * G.nv;
  b.Qv = p; p += K * G.nv;
  b.X = p; p += (size_t)G.nx * K;
  b.Y = p; p += (size_t)G.nv * K;
  b.Xs = p; p += (size_t)std::max(G.nx, G.nv) * K;
  b.T = p; p += K * SLAR_NMAX * K;
  b.Gu = p; p += K * K;
  b.Linv = p; p += K * K;
  b.R1 = p; p += K * K;
  b.R = p; p += K * K * 2;
  b.M = p; p += K * K;
  b.W = p; p += K * K;
  b.Z = p; p += K * K;
  b.sv = p; p += K;
  b.G1 = p; p += NN;
  b.G2 = p; p += NN;
  b.E1 = p; p += NN;
  b.E2 = p; p += NN;
  b.Vw = p; p += NN;
  b.lam1 = p; p += SLAR_NMAX;
  b.lam2 = p; p += SLAR_NMAX;
  return b;
}

size_t truncate_scratch_elems(const GridDev& G) {
  const size_t K = SLAR_KMAX, NN = (size_t)SLAR_NMAX * SLAR_NMAX;
  return 2 * K * G.nx + 2 * K * G.nv + (size_t)G.nx * K + (size_t)G.nv * K +
         (size_t)std::max(G.nx, G.nv) * K + K * SLAR_NMAX * K + 9 * K * K + K + 5 * NN +
         2 * SLAR_NMAX + 64;
}

// Orthonormal rows Q (k x n) and upper R (k x k) with A = R^T Q... i.e.
// A^T = Q^T R, by two Cholesky-QR passes.
static hipError_t cholqr2(hipStream_t s, Workspace* ws, Tbuf& b, int k, int n, const double* A,
                          double* Q1, double* Q, double* Rout) {
  hipError_t e = gram_rows(s, ws, k, n, A, n, b.Gu);
  if (e != hipSuccess) return e;
  e = chol_inv(s, k, b.Gu, b.Linv, b.R1, nullptr);
  if (e != hipSuccess) return e;
  e = gemm_f64(s, false, false, k, n, k, 1.0, b.Linv, k, 0, A, n, 0, 0.0, Q1, n, 0, 1);
  if (e != hipSuccess) return e;
  e = gram_rows(s, ws, k, n, Q1, n, b.Gu);
  if (e != hipSuccess) return e;
  e = chol_inv(s, k, b.Gu, b.Linv, Rout, b.R1);
  if (e != hipSuccess) return e;
  return gemm_f64(s, false, false, k, n, k, 1.0, b.Linv, k, 0, Q1, n, 0, 0.0, Q, n, 0, 1);
}

static slar_status leaf_pair(hipStream_t s, Workspace* ws, Tbuf& b, const double* frame, int na,
                             int nb, int r, const double* sv_dev, double theta, int rmax,
                             double* Ua, double* Ub, double* Bt, int* ra_out, int* rb_out,
                             bool* capped) {
  // Xs = frame * diag(s)
  if (copy2d(s, na * nb, r, frame, r, b.Xs, r, sv_dev) != hipSuccess) return SLAR_E_HIP;
  // G1 = Xs_(na x nb r) Xs^T
  if (gram_rows(s, ws, na, nb * r, b.Xs, nb * r, b.G1) != hipSuccess) return SLAR_E_HIP;
  // G2 = sum_i1 Xs[i1] Xs[i1]^T  (nb x nb)
  if (gemm_f64_sumbatch(s, ws, false, true, nb, nb, r, b.Xs, r, (long long)nb * r, b.Xs, r,
                        (long long)nb * r, b.G2, nb, na) != hipSuccess)
    return SLAR_E_HIP;
  if (eig_sym(s, na, b.G1, b.lam1, b.Vw, b.E1) != hipSuccess) return SLAR_E_HIP;
  if (eig_sym(s, nb, b.G2, b.lam2, b.Vw, b.E2) != hipSuccess) return SLAR_E_HIP;
  std::vector<double> l1(na), l2(nb);
  HIP_TRY(hipMemcpyAsync(l1.data(), b.lam1, sizeof(double) * na, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(l2.data(), b.lam2, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (double v : l1) if (!std::isfinite(v)) return SLAR_E_NUMERIC;
  const int ra = tail_rank(l1, theta, rmax), rb = tail_rank(l2, theta, rmax);
  {
    std::vector<double> t1(l1), t2(l2);
    double tail = 0.0;
    for (int i = ra; i < na; ++i) tail += std::max(t1[i], 0.0);
    if (ra == rmax && std::sqrt(tail) > theta) *capped = true;
    tail = 0.0;
    for (int i = rb; i < nb; ++i) tail += std::max(t2[i], 0.0);
    if (rb == rmax && std::sqrt(tail) > theta) *capped = true;
  }
  if (copy2d(s, na, ra, b.E1, na, Ua, ra, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (copy2d(s, nb, rb, b.E2, nb, Ub, rb, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (sign_fix(s, na, ra, Ua, ra, nullptr, 0, 0) != hipSuccess) return SLAR_E_HIP;
  if (sign_fix(s, nb, rb, Ub, rb, nullptr, 0, 0) != hipSuccess) return SLAR_E_HIP;
  // T[a][(i2, c)] = sum_i1 Ua[i1][a] frame[i1][(i2, c)]
  if (gemm_f64(s, true, false, ra, nb * r, na, 1.0, Ua, ra, 0, frame, nb * r, 0, 0.0, b.T, nb * r,
               0, 1) != hipSuccess)
    return SLAR_E_HIP;
  // Bt[a][b][c] = sum_i2 Ub[i2][b] T[a][i2][c]   (batched over a)
  if (gemm_f64(s, true, false, rb, r, nb, 1.0, Ub, rb, 0, b.T, r, (long long)nb * r, 0.0, Bt, r,
               (long long)rb * r, ra) != hipSuccess)
    return SLAR_E_HIP;
  *ra_out = ra;
  *rb_out = rb;
  return SLAR_OK;
}

__global__ void k_diag(int r, const double* sv, double* root) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  root[e] = (e / r == e % r) ? sv[e / r] : 0.0;
}

slar_status truncate_run(hipStream_t s, Workspace* ws, const slar_lowrank& in, double tol,
                         int rmax, slar_ht* out) {
  const GridDev& G = ws->G;
  Tbuf b = carve(ws);
  const int k = in.k;
  if (cholqr2(s, ws, b, k, G.nx, in.U, b.Q1u, b.Qu, b.R) != hipSuccess) return SLAR_E_HIP;
  double* Rv = b.R + SLAR_KMAX * SLAR_KMAX;
  if (cholqr2(s, ws, b, k, G.nv, in.V, b.Q1v, b.Qv, Rv) != hipSuccess) return SLAR_E_HIP;
  // core M = Ru Rv^T
  if (gemm_f64(s, false, true, k, k, k, 1.0, b.R, k, 0, Rv, k, 0, 0.0, b.M, k, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  if (svd_small(s, k, b.M, b.W, b.sv, b.Z) != hipSuccess) return SLAR_E_HIP;
  std::vector<double> sv(k);
  HIP_TRY(hipMemcpyAsync(sv.data(), b.sv, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double norm2 = 0.0;
  for (double v : sv) {
    if (!std::isfinite(v)) return SLAR_E_NUMERIC;
    norm2 += v * v;
  }
  const int d = G.d;
  const double theta = tol * std::sqrt(norm2) / std::sqrt((double)std::max(2 * d - 3, 1));
  std::vector<double> s2(k);
  for (int i = 0; i < k; ++i) s2[i] = sv[i] * sv[i];
  const int r = tail_rank(s2, theta, rmax);
  bool capped = false;
  {
    double tail = 0.0;
    for (int i = r; i < k; ++i) tail += s2[i];
    if (r == rmax && std::sqrt(tail) > theta) capped = true;
  }
  // frames X = Qu^T W_r (Nx x r), Y = Qv^T Z_r (Nv x r)
  if (gemm_f64(s, true, false, G.nx, r, k, 1.0, b.Qu, G.nx, 0, b.W, k, 0, 0.0, b.X, r, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  if (gemm_f64(s, true, false, G.nv, r, k, 1.0, b.Qv, G.nv, 0, b.Z, k, 0, 0.0, b.Y, r, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  if (sign_fix(s, G.nx, r, b.X, r, b.Y, r, G.nv) != hipSuccess) return SLAR_E_HIP;
  k_diag<<<(r * r + 255) / 256, 256, 0, s>>>(r, b.sv, (double*)out->root);
  if (d == 2) {
    if (copy2d(s, G.nx, r, b.X, r, (double*)out->leaf[0], r, nullptr) != hipSuccess) return SLAR_E_HIP;
    if (copy2d(s, G.nv, r, b.Y, r, (double*)out->leaf[1], r, nullptr) != hipSuccess) return SLAR_E_HIP;
    out->rank[0] = r; out->rank[1] = r;
    for (int m = 2; m < 6; ++m) out->rank[m] = 0;
  } else {
    int r1, r2, r3, r4;
    slar_status st = leaf_pair(s, ws, b, b.X, G.n[0], G.n[1], r, b.sv, theta, rmax,
                               (double*)out->leaf[0], (double*)out->leaf[1], (double*)out->B12,
                               &r1, &r2, &capped);
    if (st != SLAR_OK) return st;
    st = leaf_pair(s, ws, b, b.Y, G.n[2], G.n[3], r, b.sv, theta, rmax, (double*)out->leaf[2],
                   (double*)out->leaf[3], (double*)out->B34, &r3, &r4, &capped);
    if (st != SLAR_OK) return st;
    out->rank[0] = r1; out->rank[1] = r2; out->rank[2] = r3; out->rank[3] = r4;
    out->rank[4] = r; out->rank[5] = r;
  }
  out->dtype = SLAR_F64;
  out->d = d;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return capped ? SLAR_E_RANK_CAP : SLAR_OK;
}

}  // namespace slar
