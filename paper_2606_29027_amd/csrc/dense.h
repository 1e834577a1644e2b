// Dense FP64 helpers shared by the truncation, LoMaC and Krylov code.
#pragma once
#include "slar_internal.h"

namespace slar {
// device scratch region (cap doubles)
struct Scratch {
  double* p;
  size_t cap;
};
hipError_t gram_rows(hipStream_t s, const Scratch& part, int k, int n, const double* A, int lda, double* G);
hipError_t gram_mode2(hipStream_t s, const Scratch& part, int na, int nb, int r, const double* X, double* G);
hipError_t chol_inv(hipStream_t s, int k, const double* G, double* Linv, double* R, const double* Rprev);
hipError_t svd_small(hipStream_t s, int k, const double* M, double* W, double* sv, double* Z);
// left singular vectors / values for 64 < k <= 128 (right vectors not formed)
hipError_t svd_left_big(hipStream_t s, int k, const double* M, double* W, double* sv);
// Z[:, j] /= sv[j] for j < r (Z row-major, k rows, leading dimension ld)
hipError_t scale_cols_inv(hipStream_t s, int k, int r, double* Z, int ld, const double* sv);
// at most EIG_COLS eigenpairs come back nonzero (the factor's column cap)
constexpr int EIG_COLS = 64;
hipError_t eig_sym_batch(hipStream_t s, int count, const int* n, const double* const* G,
                         double* const* lam, double* const* V);
// fill the zero columns of up to four row-major n x n matrices whose other
// columns are orthonormal, so that each becomes an orthonormal basis
hipError_t complete_basis_batch(hipStream_t s, int count, const int* n, double* const* E);
hipError_t sign_fix(hipStream_t s, int rows, int cols, double* A, int lda, double* B, int ldb, int rowsB);
// the same rule for tall A (cols <= 64) in three coalesced passes; scratch
// holds (min(256, rows / 64) + 1) cols doubles (else the one-pass form runs)
hipError_t sign_fix_tall(hipStream_t s, double* scratch, size_t scratch_elems, int rows, int cols,
                         double* A, int lda, double* B, int ldb, int rowsB);
hipError_t copy2d(hipStream_t s, int rows, int cols, const double* A, int lda, double* B, int ldb,
                  const double* colscale);
hipError_t fill(hipStream_t s, double* p, long long n, double v);

// Grouped launches of the single-block factorisations: one block per
// descriptor, the descriptors in device memory, each problem computed
// exactly as by the one-problem call.  *_copy pointers (may be null)
// receive a second copy of the values, for one gathered host read.
struct CholDesc {   // chol_inv
  int k;
  const double* G;
  double* Linv;
  double* R;
  const double* Rprev;
};
struct SvdDesc {    // svd_small (k <= 64) or svd_left_big (64 < k <= 128; Z unused)
  int k;
  const double* M;
  double* W;
  double* sv;
  double* Z;
  double* sv_copy;
};
struct EigDesc {    // eig_sym_batch
  int n;
  const double* G;
  double* lam;
  double* U;
  double* lam_copy;
};
struct BasisDesc {  // complete_basis_batch
  int n;
  double* E;
};
// big: every k in (SLAR_KMAX, SLAR_CROSS_KMAX], else every k <= SLAR_KMAX
hipError_t chol_inv_group(hipStream_t s, int count, const CholDesc* d, bool big);
// big: every k in (64, 128], else every k <= 64
hipError_t svd_group(hipStream_t s, int count, const SvdDesc* d, bool big);
hipError_t eig_sym_group(hipStream_t s, int count, const EigDesc* d);
hipError_t complete_basis_group(hipStream_t s, int count, const BasisDesc* d);
}  // namespace slar
