// HTACA final truncation (Supplement B): from the cross factors
// F ~ sum_l U[l] (x) V[l] (k <= 128 terms) to a truncated HT tensor.
//   1. Cholesky-QR2 (with column scaling) of both factor sets:
//      U^T = Qu^T Ru, V^T = Qv^T Rv (Q rows orthonormal);
//   2. one-sided Jacobi SVD of the core Ru Rv^T = W diag(s) Z^T (for
//      k > 64 only W and s come from the Jacobi sweeps, and the kept
//      right vectors are Z_r = (Ru Rv^T)^T W_r diag(s_r)^-1);
//   3. root rank r = smallest with tail ||s[r:]|| <= theta,
//      theta = tol ||s|| / sqrt(2d - 3), capped at rmax; frames
//      X = Qu^T W_r, Y = Qv^T Z_r, sign rule on X (flip Y alike);
//   4. d = 2: leaves X, Y, root diag(s_r);
//      d = 4: per side, Gram matrices of the two mode matricisations A of
//      frame * diag(s) (split-K GEMMs) and their Jacobi eigendecompositions
//      E; then (unless switched off for the workspace) one refinement pass:
//      E completed to an orthonormal basis of the mode's grid, the rotated
//      matricisation E^T A has a nearly diagonal Gram whose entries carry
//      rounding relative to their own rows, so its eigenvectors V are
//      accurate to the singular-value gaps rather than the squared ones;
//      leaf = leading columns of E V (same theta on sqrt(eigenvalue)
//      tails, sign rule), transfer tensor = frame projected on the two
//      leaf bases.  The completion matters: directions missing from E
//      (past the eigen factor's rank) leave the refined small-eigenvalue
//      vectors no more accurate than the first ones.
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "slar_internal.h"
#include "dense.h"
#include "group.h"
#include "truncate.h"

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

// Scratch of one truncation.  The U and V chains (and the x and v sides of
// the tree) run concurrently on two streams, so each has its own small
// matrices and half of the dense work buffer.
struct Chain {
  double *G, *Linv, *R1;
  Scratch part;
};
struct Tbuf {
  double *Q1u, *Qu, *Q1v, *Qv, *X, *Y, *Xs, *Ys, *T, *T2;
  Chain cu, cv;
  double *R, *M, *W, *Z, *sv;
  double *G1, *G2, *G3, *G4, *E1, *E2, *E3, *E4, *Vw, *lam1, *lam2, *lam3, *lam4;
};

static Tbuf carve(Workspace* ws) {
  const GridDev& G = ws->G;
  double* p = ws->small;   // large enough for everything below (see api.hip)
  const size_t K = SLAR_KMAX, NN = (size_t)SLAR_NMAX * SLAR_NMAX;
  const size_t CK = SLAR_CROSS_KMAX;
  Tbuf b;
  b.Q1u = p; p += CK * G.nx;
  b.Qu = p; p += CK * G.nx;
  b.Q1v = p; p += CK * G.nv;
  b.Qv = p; p += CK * G.nv;
  b.X = p; p += (size_t)G.nx * K;
  b.Y = p; p += (size_t)G.nv * K;
  b.Xs = p; p += (size_t)G.nx * K;
  b.Ys = p; p += (size_t)G.nv * K;
  b.T = p; p += NN * K;
  b.T2 = p; p += NN * K;
  for (Chain* c : {&b.cu, &b.cv}) {
    c->G = p; p += CK * CK;
    c->Linv = p; p += CK * CK;
    c->R1 = p; p += CK * CK;
  }
  const size_t half = ws->dwork_elems / 2;
  b.cu.part = Scratch{ws->dwork, half};
  b.cv.part = Scratch{ws->dwork + half, half};
  b.R = p; p += CK * CK * 2;
  b.M = p; p += CK * CK;
  b.W = p; p += CK * CK;
  b.Z = p; p += CK * CK;
  b.sv = p; p += CK;
  b.G1 = p; p += NN;
  b.G2 = p; p += NN;
  b.G3 = p; p += NN;
  b.G4 = p; p += NN;
  b.E1 = p; p += NN;
  b.E2 = p; p += NN;
  b.E3 = p; p += NN;
  b.E4 = p; p += NN;
  b.Vw = p; p += 4 * NN;
  b.lam1 = p; p += SLAR_NMAX;
  b.lam2 = p; p += SLAR_NMAX;
  b.lam3 = p; p += SLAR_NMAX;
  b.lam4 = p; p += SLAR_NMAX;
  return b;
}

size_t truncate_scratch_elems(const GridDev& G) {
  const size_t K = SLAR_KMAX, NN = (size_t)SLAR_NMAX * SLAR_NMAX, CK = SLAR_CROSS_KMAX;
  return 2 * CK * G.nx + 2 * CK * G.nv + 2 * (size_t)G.nx * K + 2 * (size_t)G.nv * K +
         2 * NN * K + 12 * CK * CK + CK + 12 * NN + 4 * SLAR_NMAX + 64;
}

// Orthonormal rows Q (k x n) and upper R (k x k) with A = R^T Q... i.e.
// A^T = Q^T R, by two Cholesky-QR passes.
static hipError_t cholqr2(hipStream_t s, const Chain& c, int k, int n, const double* A, double* Q1,
                          double* Q, double* Rout) {
  hipError_t e = gram_rows(s, c.part, k, n, A, n, c.G);
  if (e != hipSuccess) return e;
  e = chol_inv(s, k, c.G, c.Linv, c.R1, nullptr);
  if (e != hipSuccess) return e;
  e = gemm_f64(s, false, false, k, n, k, 1.0, c.Linv, k, 0, A, n, 0, 0.0, Q1, n, 0, 1);
  if (e != hipSuccess) return e;
  e = gram_rows(s, c.part, k, n, Q1, n, c.G);
  if (e != hipSuccess) return e;
  e = chol_inv(s, k, c.G, c.Linv, Rout, c.R1);
  if (e != hipSuccess) return e;
  return gemm_f64(s, false, false, k, n, k, 1.0, c.Linv, k, 0, Q1, n, 0, 0.0, Q, n, 0, 1);
}

// Gram matrices of the two mode matricisations of frame * diag(s) for one
// side of the tree (frame: [na*nb][r] packed).  Xs is scratch [na*nb][r].
static hipError_t side_grams(hipStream_t s, const Scratch& part, const double* frame, int na, int nb,
                             int r, const double* sv_dev, double* Xs, double* Ga, double* Gb) {
  HIP_CHK(copy2d(s, na * nb, r, frame, r, Xs, r, sv_dev));
  HIP_CHK(gram_rows(s, part, na, nb * r, Xs, nb * r, Ga));
  return gram_mode2(s, part, na, nb, r, Xs, Gb);
}

// aux waits for the work already on s / s waits for everything on aux
static hipError_t fork(hipStream_t s, Workspace* ws) {
  if (!ws->fork_aux) return hipSuccess;
  HIP_CHK(hipEventRecord(ws->ev_fork, s));
  return hipStreamWaitEvent(ws->aux, ws->ev_fork, 0);
}
static hipError_t join(hipStream_t s, Workspace* ws) {
  if (!ws->fork_aux) return hipSuccess;
  HIP_CHK(hipEventRecord(ws->ev_join, ws->aux));
  return hipStreamWaitEvent(s, ws->ev_join, 0);
}

// Leaf bases (leading eigenvectors, sign rule) and the transfer tensor of
// one side once the eigendecompositions are known.
static slar_status side_finish(hipStream_t s, double* T, const double* frame, int na, int nb, int r,
                               const double* Ea, int lda, const double* Eb, int ldb, int ra, int rb,
                               double* Ua, double* Ub, double* Bt) {
  if (copy2d(s, na, ra, Ea, lda, Ua, ra, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (copy2d(s, nb, rb, Eb, ldb, Ub, rb, nullptr) != hipSuccess) return SLAR_E_HIP;
  if (sign_fix(s, na, ra, Ua, ra, nullptr, 0, 0) != hipSuccess) return SLAR_E_HIP;
  if (sign_fix(s, nb, rb, Ub, rb, nullptr, 0, 0) != hipSuccess) return SLAR_E_HIP;
  // T[a][(i2, c)] = sum_i1 Ua[i1][a] frame[i1][(i2, c)]
  if (gemm_f64(s, true, false, ra, nb * r, na, 1.0, Ua, ra, 0, frame, nb * r, 0, 0.0, T, nb * r,
               0, 1) != hipSuccess)
    return SLAR_E_HIP;
  // Bt[a][b][c] = sum_i2 Ub[i2][b] T[a][i2][c]   (batched over a)
  if (gemm_f64(s, true, false, rb, r, nb, 1.0, Ub, rb, 0, T, r, (long long)nb * r, 0.0, Bt, r,
               (long long)rb * r, ra) != hipSuccess)
    return SLAR_E_HIP;
  return SLAR_OK;
}

// Refinement Grams of one side: with Ea, Eb the eigenvector matrices of
// the two mode Grams (row-major na x na / nb x nb, eigenvector j in column
// j) and c = min(n, 64) leading columns, Ga' = (Ea_c^T A_a)(Ea_c^T A_a)^T
// and Gb' likewise for mode 2 (c x c each).  Xs = frame * diag(s) packed
// [na][nb][r]; T is scratch of c * max(na, nb) * r doubles.
static hipError_t side_refine_grams(hipStream_t s, const Scratch& part, const double* Xs, int na, int nb,
                                    int r, const double* Ea, const double* Eb, int ca, int cb, double* T,
                                    double* Ga, double* Gb) {
  // mode 1: T[a][(i2, c)] = sum_i1 Ea[i1][a] Xs[i1][(i2, c)], a < ca
  HIP_CHK(gemm_f64(s, true, false, ca, nb * r, na, 1.0, Ea, na, 0, Xs, nb * r, 0, 0.0, T, nb * r, 0, 1));
  HIP_CHK(gram_rows(s, part, ca, nb * r, T, nb * r, Ga));
  // mode 2: T[i1][b][c] = sum_i2 Eb[i2][b] Xs[i1][i2][c], b < cb (batched over i1)
  HIP_CHK(gemm_f64(s, true, false, cb, r, nb, 1.0, Eb, nb, 0, Xs, r, (long long)nb * r, 0.0, T, r,
                   (long long)cb * r, na));
  return gram_mode2(s, part, na, cb, r, T, Gb);
}

static int leaf_rank(const std::vector<double>& lam, double theta, int rmax, bool* capped) {
  const int r = tail_rank(lam, theta, rmax);
  double tail = 0.0;
  for (size_t i = r; i < lam.size(); ++i) tail += std::max(lam[i], 0.0);
  if (r == rmax && std::sqrt(tail) > theta) *capped = true;
  return r;
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
  const hipStream_t sa = ws->fork_aux ? ws->aux : s;   // the V-side chain
  double* Rv = b.R + SLAR_CROSS_KMAX * SLAR_CROSS_KMAX;
  // the U and V orthogonalisations are independent: U on s, V on aux
  if (fork(s, ws) != hipSuccess) return SLAR_E_HIP;
  if (cholqr2(s, b.cu, k, G.nx, in.U, b.Q1u, b.Qu, b.R) != hipSuccess) return SLAR_E_HIP;
  if (cholqr2(sa, b.cv, k, G.nv, in.V, b.Q1v, b.Qv, Rv) != hipSuccess) return SLAR_E_HIP;
  if (join(s, ws) != hipSuccess) return SLAR_E_HIP;
  // core M = Ru Rv^T
  if (gemm_f64(s, false, true, k, k, k, 1.0, b.R, k, 0, Rv, k, 0, 0.0, b.M, k, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  const bool big = k > 64;
  if (big) {
    if (svd_left_big(s, k, b.M, b.W, b.sv) != hipSuccess) return SLAR_E_HIP;
  } else if (svd_small(s, k, b.M, b.W, b.sv, b.Z) != hipSuccess) {
    return SLAR_E_HIP;
  }
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
  if (big) {
    // kept right singular vectors Z_r = M^T W_r diag(s_r)^-1 (k x r, ld k)
    if (gemm_f64(s, true, false, k, r, k, 1.0, b.M, k, 0, b.W, k, 0, 0.0, b.Z, k, 0, 1) != hipSuccess)
      return SLAR_E_HIP;
    if (scale_cols_inv(s, k, r, b.Z, k, b.sv) != hipSuccess) return SLAR_E_HIP;
  }
  // frames X = Qu^T W_r (Nx x r), Y = Qv^T Z_r (Nv x r)
  if (fork(s, ws) != hipSuccess) return SLAR_E_HIP;
  if (gemm_f64(s, true, false, G.nx, r, k, 1.0, b.Qu, G.nx, 0, b.W, k, 0, 0.0, b.X, r, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  if (gemm_f64(sa, true, false, G.nv, r, k, 1.0, b.Qv, G.nv, 0, b.Z, k, 0, 0.0, b.Y, r, 0, 1) != hipSuccess)
    return SLAR_E_HIP;
  if (join(s, ws) != hipSuccess) return SLAR_E_HIP;
  // the Cholesky-QR partials in dwork are dead once both chains have joined
  if (sign_fix_tall(s, ws->dwork, ws->dwork_elems, G.nx, r, b.X, r, b.Y, r, G.nv) != hipSuccess)
    return SLAR_E_HIP;
  k_diag<<<(r * r + 255) / 256, 256, 0, s>>>(r, b.sv, (double*)out->root);
  if (d == 2) {
    if (copy2d(s, G.nx, r, b.X, r, (double*)out->leaf[0], r, nullptr) != hipSuccess) return SLAR_E_HIP;
    if (copy2d(s, G.nv, r, b.Y, r, (double*)out->leaf[1], r, nullptr) != hipSuccess) return SLAR_E_HIP;
    out->rank[0] = r; out->rank[1] = r;
    for (int m = 2; m < 6; ++m) out->rank[m] = 0;
  } else {
    // Gram matrices of the four modes, one batched eigen launch, one sync
    if (fork(s, ws) != hipSuccess) return SLAR_E_HIP;
    if (side_grams(s, b.cu.part, b.X, G.n[0], G.n[1], r, b.sv, b.Xs, b.G1, b.G2) != hipSuccess) return SLAR_E_HIP;
    if (side_grams(sa, b.cv.part, b.Y, G.n[2], G.n[3], r, b.sv, b.Ys, b.G3, b.G4) != hipSuccess)
      return SLAR_E_HIP;
    if (join(s, ws) != hipSuccess) return SLAR_E_HIP;
    const int nn[4] = {G.n[0], G.n[1], G.n[2], G.n[3]};
    double* Gw[4] = {b.G1, b.G2, b.G3, b.G4};
    const double* Gs[4] = {b.G1, b.G2, b.G3, b.G4};
    double* lams[4] = {b.lam1, b.lam2, b.lam3, b.lam4};
    double* Es[4] = {b.E1, b.E2, b.E3, b.E4};
    if (eig_sym_batch(s, 4, nn, Gs, lams, Es) != hipSuccess) return SLAR_E_HIP;
    // leaf bases and their leading dimensions: the eigenvectors, or (with
    // the refinement pass) E V, where E is the eigenvector set completed to
    // an orthonormal basis of the mode's grid and V the eigenvectors of the
    // Gram of E^T A, nearly diagonal (into G1..G4, four n x n blocks of Vw)
    const double* Ub[4] = {b.E1, b.E2, b.E3, b.E4};
    int ldu[4] = {nn[0], nn[1], nn[2], nn[3]};
    if (ws->leaf_refine) {
      if (complete_basis_batch(s, 4, nn, Es) != hipSuccess) return SLAR_E_HIP;
      if (fork(s, ws) != hipSuccess) return SLAR_E_HIP;
      if (side_refine_grams(s, b.cu.part, b.Xs, G.n[0], G.n[1], r, b.E1, b.E2, nn[0], nn[1], b.T, b.G1,
                            b.G2) != hipSuccess)
        return SLAR_E_HIP;
      if (side_refine_grams(sa, b.cv.part, b.Ys, G.n[2], G.n[3], r, b.E3, b.E4, nn[2], nn[3], b.T2, b.G3,
                            b.G4) != hipSuccess)
        return SLAR_E_HIP;
      if (join(s, ws) != hipSuccess) return SLAR_E_HIP;
      double* Vs[4];
      for (int m = 0; m < 4; ++m) Vs[m] = b.Vw + (size_t)m * SLAR_NMAX * SLAR_NMAX;
      if (eig_sym_batch(s, 4, nn, Gs, lams, Vs) != hipSuccess) return SLAR_E_HIP;
      for (int m = 0; m < 4; ++m) {
        const int c2 = std::min(nn[m], EIG_COLS);
        if (gemm_f64(s, false, false, nn[m], c2, nn[m], 1.0, Es[m], nn[m], 0, Vs[m], nn[m], 0, 0.0, Gw[m],
                     c2, 0, 1) != hipSuccess)
          return SLAR_E_HIP;
        Ub[m] = Gw[m];
        ldu[m] = c2;
      }
    }
    std::vector<double> lh(4 * SLAR_NMAX);
    for (int m = 0; m < 4; ++m)
      HIP_TRY(hipMemcpyAsync(lh.data() + m * SLAR_NMAX, lams[m], sizeof(double) * nn[m],
                             hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int rk[4];
    for (int m = 0; m < 4; ++m) {
      std::vector<double> l(lh.begin() + m * SLAR_NMAX, lh.begin() + m * SLAR_NMAX + nn[m]);
      for (double v : l) if (!std::isfinite(v)) return SLAR_E_NUMERIC;
      rk[m] = leaf_rank(l, theta, rmax, &capped);
    }
    if (fork(s, ws) != hipSuccess) return SLAR_E_HIP;
    slar_status st = side_finish(s, b.T, b.X, G.n[0], G.n[1], r, Ub[0], ldu[0], Ub[1], ldu[1], rk[0], rk[1],
                                 (double*)out->leaf[0], (double*)out->leaf[1], (double*)out->B12);
    if (st != SLAR_OK) return st;
    st = side_finish(sa, b.T2, b.Y, G.n[2], G.n[3], r, Ub[2], ldu[2], Ub[3], ldu[3], rk[2], rk[3],
                     (double*)out->leaf[2], (double*)out->leaf[3], (double*)out->B34);
    if (st != SLAR_OK) return st;
    if (join(s, ws) != hipSuccess) return SLAR_E_HIP;
    for (int m = 0; m < 4; ++m) out->rank[m] = rk[m];
    out->rank[4] = r; out->rank[5] = r;
  }
  out->dtype = SLAR_F64;
  out->d = d;
  // the ranks are decided; the factors are complete in stream order
  HIP_TRY(hipGetLastError());
  return capped ? SLAR_E_RANK_CAP : SLAR_OK;
}

// ------------------------------------------------------------ grouped form
// The steps of truncate_run, phase by phase over a group of jobs, every
// step one grouped launch for all jobs (group.h): the products, Grams,
// sign rules and copies run the one-problem bodies per job, and the
// single-block factorisations (Cholesky, core SVD, Gram eigenpairs, basis
// completion) one block per job.  The host takes the rank decisions of all
// jobs after one gathered read of the singular values, then of the
// eigenvalues.
namespace {
struct GroupLayout {
  size_t queue, sv, lam, total;
};
GroupLayout group_layout(int n) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  GroupLayout L{};
  L.queue = al((size_t)256 * 1024 + (size_t)n * 32 * 1024);   // descriptors of one call
  L.sv = L.queue;
  L.lam = L.sv + al(sizeof(double) * SLAR_CROSS_KMAX * n);
  L.total = L.lam + al(sizeof(double) * 4 * SLAR_NMAX * n);
  return L;
}

// factorisation descriptors of two size classes (small ones first), staged
// in q and launched with `launch(stream, device descriptors, small, big)`
template <class D, class F>
hipError_t stage_group(GroupQueue& q, const std::vector<D>& sm, const std::vector<D>& bg, F launch) {
  if (sm.empty() && bg.empty()) return hipSuccess;
  std::vector<D> all(sm);
  all.insert(all.end(), bg.begin(), bg.end());
  const D* d = (const D*)q.stage(all.data(), sizeof(D) * all.size());
  if (!d) return hipErrorOutOfMemory;
  const int ns = (int)sm.size(), nb = (int)bg.size();
  q.then([=](hipStream_t s) { return launch(s, d, ns, nb); });
  return hipSuccess;
}
}  // namespace

size_t truncate_group_bytes(int count) { return group_layout(std::max(count, 1)).total; }

slar_status truncate_group(hipStream_t s, std::vector<TruncJob>& jobs, double tol, int rmax, void* dmem,
                           void* hmem) {
  const int n = (int)jobs.size();
  if (n == 0) return SLAR_OK;
  const GroupLayout GL = group_layout(n);
  char* D = (char*)dmem;
  char* H = (char*)hmem;
  GroupQueue q(dmem, hmem, GL.queue);
  const size_t CK = SLAR_CROSS_KMAX;
  std::vector<Tbuf> tb(n);
  for (int j = 0; j < n; ++j) tb[j] = carve(jobs[j].ws);
  auto live = [&](int j) { return jobs[j].st == SLAR_OK; };
  auto Rv_of = [&](int j) { return tb[j].R + CK * CK; };
  // a failure of a grouped launch fails every job of the call
  auto fatal = [&](hipError_t e) {
    if (e == hipSuccess) return false;
    for (TruncJob& J : jobs)
      if (J.st == SLAR_OK) J.st = SLAR_E_HIP;
    return true;
  };
  using GA = GroupQueue::GramArgs;

  // ---- A: Cholesky-QR2 of both factor sets, core M = Ru Rv^T, core SVD
  {
    std::vector<GA> gr;
    for (int j = 0; j < n; ++j) {
      const GridDev& G = jobs[j].ws->G;
      const Tbuf& b = tb[j];
      const int k = jobs[j].in.k;
      gr.push_back(GA{k, G.nx, 0, jobs[j].in.U, G.nx, 0, 0, b.cu.part.p, b.cu.part.cap, b.cu.G});
      gr.push_back(GA{k, G.nv, 0, jobs[j].in.V, G.nv, 0, 0, b.cv.part.p, b.cv.part.cap, b.cv.G});
    }
    if (fatal(q.gram(gr))) return SLAR_E_HIP;
  }
  auto chol = [&](bool second) -> hipError_t {
    std::vector<CholDesc> sm, bg;
    for (int j = 0; j < n; ++j) {
      const Tbuf& b = tb[j];
      const int k = jobs[j].in.k;
      auto& v = (k <= SLAR_KMAX) ? sm : bg;
      if (second) {
        v.push_back(CholDesc{k, b.cu.G, b.cu.Linv, b.R, b.cu.R1});
        v.push_back(CholDesc{k, b.cv.G, b.cv.Linv, Rv_of(j), b.cv.R1});
      } else {
        v.push_back(CholDesc{k, b.cu.G, b.cu.Linv, b.cu.R1, nullptr});
        v.push_back(CholDesc{k, b.cv.G, b.cv.Linv, b.cv.R1, nullptr});
      }
    }
    return stage_group(q, sm, bg, [](hipStream_t st, const CholDesc* d, int ns, int nb) {
      hipError_t e = chol_inv_group(st, ns, d, false);
      return e == hipSuccess ? chol_inv_group(st, nb, d + ns, true) : e;
    });
  };
  if (fatal(chol(false))) return SLAR_E_HIP;
  {
    std::vector<GemmArgs> g;
    std::vector<GA> gr;
    for (int j = 0; j < n; ++j) {
      const GridDev& G = jobs[j].ws->G;
      const Tbuf& b = tb[j];
      const int k = jobs[j].in.k;
      g.push_back(GemmArgs{k, G.nx, k, 1.0, b.cu.Linv, k, 0, jobs[j].in.U, G.nx, 0, 0.0, b.Q1u, G.nx, 0, 1});
      g.push_back(GemmArgs{k, G.nv, k, 1.0, b.cv.Linv, k, 0, jobs[j].in.V, G.nv, 0, 0.0, b.Q1v, G.nv, 0, 1});
      gr.push_back(GA{k, G.nx, 0, b.Q1u, G.nx, 0, 0, b.cu.part.p, b.cu.part.cap, b.cu.G});
      gr.push_back(GA{k, G.nv, 0, b.Q1v, G.nv, 0, 0, b.cv.part.p, b.cv.part.cap, b.cv.G});
    }
    if (fatal(q.gemm(false, false, g)) || fatal(q.gram(gr))) return SLAR_E_HIP;
  }
  if (fatal(chol(true))) return SLAR_E_HIP;
  {
    std::vector<GemmArgs> g, gm;
    std::vector<SvdDesc> sm, bg;
    double* svs = (double*)(D + GL.sv);
    for (int j = 0; j < n; ++j) {
      const GridDev& G = jobs[j].ws->G;
      const Tbuf& b = tb[j];
      const int k = jobs[j].in.k;
      g.push_back(GemmArgs{k, G.nx, k, 1.0, b.cu.Linv, k, 0, b.Q1u, G.nx, 0, 0.0, b.Qu, G.nx, 0, 1});
      g.push_back(GemmArgs{k, G.nv, k, 1.0, b.cv.Linv, k, 0, b.Q1v, G.nv, 0, 0.0, b.Qv, G.nv, 0, 1});
      gm.push_back(GemmArgs{k, k, k, 1.0, b.R, k, 0, Rv_of(j), k, 0, 0.0, b.M, k, 0, 1});
      if (k > 64) bg.push_back(SvdDesc{k, b.M, b.W, b.sv, nullptr, svs + (size_t)j * CK});
      else sm.push_back(SvdDesc{k, b.M, b.W, b.sv, b.Z, svs + (size_t)j * CK});
    }
    if (fatal(q.gemm(false, false, g)) || fatal(q.gemm(false, true, gm))) return SLAR_E_HIP;
    if (fatal(stage_group(q, sm, bg, [](hipStream_t st, const SvdDesc* d, int ns, int nb) {
          hipError_t e = svd_group(st, ns, d, false);
          return e == hipSuccess ? svd_group(st, nb, d + ns, true) : e;
        })))
      return SLAR_E_HIP;
    if (fatal(q.flush(s))) return SLAR_E_HIP;
    HIP_TRY(hipMemcpyAsync(H + GL.sv, D + GL.sv, sizeof(double) * CK * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    q.reset();
  }
  // root ranks (the rule of truncate_run)
  for (int j = 0; j < n; ++j) {
    TruncJob& J = jobs[j];
    const int k = J.in.k;
    const double* sv = (const double*)(H + GL.sv) + (size_t)j * CK;
    double norm2 = 0.0;
    bool finite = true;
    for (int i = 0; i < k; ++i) {
      if (!std::isfinite(sv[i])) finite = false;
      norm2 += sv[i] * sv[i];
    }
    if (!finite) { J.st = SLAR_E_NUMERIC; continue; }
    const int d = J.ws->G.d;
    J.theta = tol * std::sqrt(norm2) / std::sqrt((double)std::max(2 * d - 3, 1));
    std::vector<double> s2(k);
    for (int i = 0; i < k; ++i) s2[i] = sv[i] * sv[i];
    J.r = tail_rank(s2, J.theta, rmax);
    double tail = 0.0;
    for (int i = J.r; i < k; ++i) tail += s2[i];
    J.capped = J.r == rmax && std::sqrt(tail) > J.theta;
  }

  // ---- B: kept right vectors (k > 64), frames, sign rule, root; d = 2
  // leaves; d = 4 mode Grams, eigenpairs (and the refinement pass)
  auto four = [&](int j) { return live(j) && jobs[j].ws->G.d == 4; };
  auto refine = [&](int j) { return four(j) && jobs[j].ws->leaf_refine; };
  double* lst = (double*)(D + GL.lam);
  auto lam_slot = [&](int j, int m) { return lst + ((size_t)j * 4 + m) * SLAR_NMAX; };
  {
    std::vector<GemmArgs> gz, gxy;
    std::vector<ScaleDesc> sz, droot;
    std::vector<GroupQueue::SignArgs> sg;
    std::vector<CopyDesc> cp;
    std::vector<GA> g1, g2;
    for (int j = 0; j < n; ++j) {
      if (!live(j)) continue;
      TruncJob& J = jobs[j];
      Workspace* ws = J.ws;
      const GridDev& G = ws->G;
      const Tbuf& b = tb[j];
      const int k = J.in.k, r = J.r;
      if (k > 64) {
        gz.push_back(GemmArgs{k, r, k, 1.0, b.M, k, 0, b.W, k, 0, 0.0, b.Z, k, 0, 1});
        sz.push_back(ScaleDesc{k, r, k, 0, b.Z, b.sv});
      }
      gxy.push_back(GemmArgs{G.nx, r, k, 1.0, b.Qu, G.nx, 0, b.W, k, 0, 0.0, b.X, r, 0, 1});
      gxy.push_back(GemmArgs{G.nv, r, k, 1.0, b.Qv, G.nv, 0, b.Z, k, 0, 0.0, b.Y, r, 0, 1});
      sg.push_back(GroupQueue::SignArgs{G.nx, r, b.X, r, b.Y, r, G.nv, ws->dwork, ws->dwork_elems});
      droot.push_back(ScaleDesc{0, r, 0, 1, (double*)J.out->root, b.sv});
      if (G.d == 2) {
        cp.push_back(CopyDesc{G.nx, r, r, r, b.X, (double*)J.out->leaf[0], nullptr});
        cp.push_back(CopyDesc{G.nv, r, r, r, b.Y, (double*)J.out->leaf[1], nullptr});
        J.out->rank[0] = r; J.out->rank[1] = r;
        for (int m = 2; m < 6; ++m) J.out->rank[m] = 0;
      } else {
        // side_grams of both sides: frame * diag(s), mode-1 and mode-2 Grams
        // (the mode-2 Gram reuses the side's partial-sum scratch: next launch)
        cp.push_back(CopyDesc{G.n[0] * G.n[1], r, r, r, b.X, b.Xs, b.sv});
        cp.push_back(CopyDesc{G.n[2] * G.n[3], r, r, r, b.Y, b.Ys, b.sv});
        g1.push_back(GA{G.n[0], G.n[1] * r, 0, b.Xs, G.n[1] * r, 0, 0, b.cu.part.p, b.cu.part.cap, b.G1});
        g1.push_back(GA{G.n[2], G.n[3] * r, 0, b.Ys, G.n[3] * r, 0, 0, b.cv.part.p, b.cv.part.cap, b.G3});
        g2.push_back(GA{G.n[1], G.n[0] * r, 1, b.Xs, 0, G.n[1], r, b.cu.part.p, b.cu.part.cap, b.G2});
        g2.push_back(GA{G.n[3], G.n[2] * r, 1, b.Ys, 0, G.n[3], r, b.cv.part.p, b.cv.part.cap, b.G4});
      }
    }
    if (fatal(q.gemm(true, false, gz)) || fatal(q.scale(sz)) || fatal(q.gemm(true, false, gxy)) ||
        fatal(q.sign_fix_tall(sg)) || fatal(q.scale(droot)) || fatal(q.copy2d(cp)) || fatal(q.gram(g1)) ||
        fatal(q.gram(g2)))
      return SLAR_E_HIP;
  }
  bool any4 = false;
  for (int j = 0; j < n; ++j) any4 = any4 || four(j);
  if (any4) {
    std::vector<EigDesc> ed, none;
    std::vector<BasisDesc> bd, noneb;
    for (int j = 0; j < n; ++j) {
      if (!four(j)) continue;
      const Tbuf& b = tb[j];
      const GridDev& G = jobs[j].ws->G;
      const double* Gm[4] = {b.G1, b.G2, b.G3, b.G4};
      double* lm[4] = {b.lam1, b.lam2, b.lam3, b.lam4};
      double* Em[4] = {b.E1, b.E2, b.E3, b.E4};
      for (int m = 0; m < 4; ++m) {
        ed.push_back(EigDesc{G.n[m], Gm[m], lm[m], Em[m], refine(j) ? nullptr : lam_slot(j, m)});
        if (refine(j)) bd.push_back(BasisDesc{G.n[m], Em[m]});
      }
    }
    if (fatal(stage_group(q, ed, none, [](hipStream_t st, const EigDesc* d, int ns, int) {
          return eig_sym_group(st, ns, d);
        })))
      return SLAR_E_HIP;
    if (!bd.empty()) {
      // refinement: completed bases, Grams of the rotated matricisations,
      // their eigenpairs, leaf candidates E V (side_refine_grams)
      if (fatal(stage_group(q, bd, noneb, [](hipStream_t st, const BasisDesc* d, int ns, int) {
            return complete_basis_group(st, ns, d);
          })))
        return SLAR_E_HIP;
      std::vector<GemmArgs> ga, gb, gev;
      std::vector<GA> r1, r2;
      std::vector<EigDesc> ed2;
      for (int j = 0; j < n; ++j) {
        if (!refine(j)) continue;
        const Tbuf& b = tb[j];
        const GridDev& G = jobs[j].ws->G;
        const int r = jobs[j].r;
        const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2], n3 = G.n[3];
        ga.push_back(GemmArgs{n0, n1 * r, n0, 1.0, b.E1, n0, 0, b.Xs, n1 * r, 0, 0.0, b.T, n1 * r, 0, 1});
        ga.push_back(GemmArgs{n2, n3 * r, n2, 1.0, b.E3, n2, 0, b.Ys, n3 * r, 0, 0.0, b.T2, n3 * r, 0, 1});
        r1.push_back(GA{n0, n1 * r, 0, b.T, n1 * r, 0, 0, b.cu.part.p, b.cu.part.cap, b.G1});
        r1.push_back(GA{n2, n3 * r, 0, b.T2, n3 * r, 0, 0, b.cv.part.p, b.cv.part.cap, b.G3});
        gb.push_back(GemmArgs{n1, r, n1, 1.0, b.E2, n1, 0, b.Xs, r, (long long)n1 * r, 0.0, b.T, r,
                              (long long)n1 * r, n0});
        gb.push_back(GemmArgs{n3, r, n3, 1.0, b.E4, n3, 0, b.Ys, r, (long long)n3 * r, 0.0, b.T2, r,
                              (long long)n3 * r, n2});
        r2.push_back(GA{n1, n0 * r, 1, b.T, 0, n1, r, b.cu.part.p, b.cu.part.cap, b.G2});
        r2.push_back(GA{n3, n2 * r, 1, b.T2, 0, n3, r, b.cv.part.p, b.cv.part.cap, b.G4});
        const double* Gm[4] = {b.G1, b.G2, b.G3, b.G4};
        double* lm[4] = {b.lam1, b.lam2, b.lam3, b.lam4};
        double* Em[4] = {b.E1, b.E2, b.E3, b.E4};
        double* Gw[4] = {b.G1, b.G2, b.G3, b.G4};
        for (int m = 0; m < 4; ++m) {
          double* Vm = b.Vw + (size_t)m * SLAR_NMAX * SLAR_NMAX;
          const int nm = G.n[m], c2 = std::min(nm, EIG_COLS);
          ed2.push_back(EigDesc{nm, Gm[m], lm[m], Vm, lam_slot(j, m)});
          gev.push_back(GemmArgs{nm, c2, nm, 1.0, Em[m], nm, 0, Vm, nm, 0, 0.0, Gw[m], c2, 0, 1});
        }
      }
      if (fatal(q.gemm(true, false, ga)) || fatal(q.gram(r1)) || fatal(q.gemm(true, false, gb)) ||
          fatal(q.gram(r2)))
        return SLAR_E_HIP;
      if (fatal(stage_group(q, ed2, none, [](hipStream_t st, const EigDesc* d, int ns, int) {
            return eig_sym_group(st, ns, d);
          })))
        return SLAR_E_HIP;
      if (fatal(q.gemm(false, false, gev))) return SLAR_E_HIP;
    }
  }
  if (fatal(q.flush(s))) return SLAR_E_HIP;
  std::vector<std::array<int, 4>> rk(n);
  if (any4) {
    HIP_TRY(hipMemcpyAsync(H + GL.lam, D + GL.lam, sizeof(double) * 4 * SLAR_NMAX * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    q.reset();
    for (int j = 0; j < n; ++j) {
      if (!four(j)) continue;
      const GridDev& G = jobs[j].ws->G;
      const double* lh = (const double*)(H + GL.lam) + (size_t)j * 4 * SLAR_NMAX;
      for (int m = 0; m < 4 && live(j); ++m) {
        std::vector<double> l(lh + m * SLAR_NMAX, lh + m * SLAR_NMAX + G.n[m]);
        for (double v : l)
          if (!std::isfinite(v)) jobs[j].st = SLAR_E_NUMERIC;
        if (live(j)) rk[j][m] = leaf_rank(l, jobs[j].theta, rmax, &jobs[j].capped);
      }
    }
    // ---- C: leaf bases (sign rule) and transfer tensors (side_finish)
    std::vector<CopyDesc> cp;
    std::vector<GroupQueue::SignArgs> sg;
    std::vector<GemmArgs> gt, gbt;
    for (int j = 0; j < n; ++j) {
      if (!four(j)) continue;
      TruncJob& J = jobs[j];
      const GridDev& G = J.ws->G;
      const Tbuf& b = tb[j];
      const int r = J.r;
      const bool rf = J.ws->leaf_refine;
      const double* Ub[4] = {rf ? b.G1 : b.E1, rf ? b.G2 : b.E2, rf ? b.G3 : b.E3, rf ? b.G4 : b.E4};
      const int* R = rk[j].data();
      double* leaf[4] = {(double*)J.out->leaf[0], (double*)J.out->leaf[1], (double*)J.out->leaf[2],
                         (double*)J.out->leaf[3]};
      for (int m = 0; m < 4; ++m) {
        const int ldu = rf ? std::min(G.n[m], EIG_COLS) : G.n[m];
        cp.push_back(CopyDesc{G.n[m], R[m], ldu, R[m], Ub[m], leaf[m], nullptr});
        sg.push_back(GroupQueue::SignArgs{G.n[m], R[m], leaf[m], R[m], nullptr, 0, 0, nullptr, 0});
      }
      const double* frame[2] = {b.X, b.Y};
      double* T[2] = {b.T, b.T2};
      double* Bt[2] = {(double*)J.out->B12, (double*)J.out->B34};
      for (int sd = 0; sd < 2; ++sd) {
        const int na = G.n[2 * sd], nb = G.n[2 * sd + 1], ra = R[2 * sd], rb = R[2 * sd + 1];
        gt.push_back(GemmArgs{ra, nb * r, na, 1.0, leaf[2 * sd], ra, 0, frame[sd], nb * r, 0, 0.0, T[sd], nb * r,
                              0, 1});
        gbt.push_back(GemmArgs{rb, r, nb, 1.0, leaf[2 * sd + 1], rb, 0, T[sd], r, (long long)nb * r, 0.0, Bt[sd],
                               r, (long long)rb * r, ra});
      }
      for (int m = 0; m < 4; ++m) J.out->rank[m] = R[m];
      J.out->rank[4] = r; J.out->rank[5] = r;
    }
    if (fatal(q.copy2d(cp)) || fatal(q.sign_fix(sg)) || fatal(q.gemm(true, false, gt)) ||
        fatal(q.gemm(true, false, gbt)))
      return SLAR_E_HIP;
  }
  for (TruncJob& J : jobs) {
    if (J.st != SLAR_OK) continue;
    J.out->dtype = SLAR_F64;
    J.out->d = J.ws->G.d;
    if (J.capped) J.st = SLAR_E_RANK_CAP;
  }
  // ---- frames of the new tensors
  {
    std::vector<Workspace*> fw;
    std::vector<const slar_ht*> fh;
    std::vector<slar_frames*> fo;
    for (TruncJob& J : jobs)
      if ((J.st == SLAR_OK || J.st == SLAR_E_RANK_CAP) && J.frames) {
        fw.push_back(J.ws);
        fh.push_back(J.out);
        fo.push_back(J.frames);
      }
    if (!fw.empty() && fatal(frames_from_ht_group(q, (int)fw.size(), fw.data(), fh.data(), fo.data())))
      return SLAR_E_HIP;
  }
  if (fatal(q.flush(s))) return SLAR_E_HIP;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return SLAR_OK;
}

}  // namespace slar
