// Grouped launches: one kernel launch serves a list of independent problems
// of uneven size.  Problem d owns the blocks [first[d], first[d + 1]) of the
// launch (first ascending, first[0] = 0); its descriptor says what to
// compute.  Every grouped kernel runs, per problem, the body of its
// one-problem kernel with the same block-local arguments, so the results
// are bit-identical to the one-problem launches.
//
// GroupQueue collects the descriptors of a sequence of grouped launches in
// pinned host memory, uploads them with one copy and issues the launches in
// order on one stream.  Launches in a sequence may depend on earlier ones
// (stream order); problems within one launch must be independent.
#pragma once
#include <functional>
#include <vector>

#include "slar_internal.h"

namespace slar {

// the problem owning block b: the largest d < nd with first[d] <= b
// (wave-uniform; a ballot over 64 entries per round)
__device__ __forceinline__ int group_find(const int* __restrict__ first, int nd, int b) {
  int d = 0;
  for (int base = 0; base < nd; base += 64) {
    const int i = base + (int)(threadIdx.x & 63);
    const bool le = i < nd && first[i] <= b;
    const unsigned long long m = __ballot(le);
    if (m) d = base + 63 - __clzll((long long)m);
    if (m != ~0ull) break;
  }
  return __builtin_amdgcn_readfirstlane(d);
}

struct GemmDesc {   // gemm_f64 (row-major, batch strides)
  int M, N, K, tm, tn;   // tm x tn output tiles per batch item
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc;
  long long sA, sB, sC;
};
struct GramDesc {   // gram_rows (mode2 = 0) or gram_mode2 (mode2 = 1)
  int k, n, nblk, mode2;
  const double* A;   // RowMajor: A, lda; Mode2: X, nb, r
  int lda, nb, r;
  double* part;
  double* G;
};
struct CopyDesc {   // copy2d
  int rows, cols, lda, ldb;
  const double* A;
  double* B;
  const double* colscale;
};
struct SignDesc {   // sign_fix / sign_fix_tall
  int rows, cols, lda, ldb, rowsB, rb, nb;
  double* A;
  double* B;
  double* part;   // tall form: [nb][cols] partial maxima, then [cols] signs
};
struct LineDesc {   // one batch of line transforms (FFT for 2^logL, else DFT)
  int n0, n1, axis, logL, B;
  double sign;
  const double2* in;
  const double* realin;
  double2* out;
  const double* tw;
};
enum { FIELD_RHO = 0, FIELD_REAL = 1, FIELD_SYMBOL = 2 };
struct FieldDesc {  // pointwise field steps of the spectral solve
  int op, sym, nvec, Nx, n0, n1, dx;
  long long n;      // elements (RHO, REAL)
  double ni, scale, L0, L1;
  const double* rin;
  double* rout;
  const double2* cin;
  double2* cout;
};
struct SumDesc {    // fixed-order sum of batched chunk products (C = sum_b P_b)
  int M, N, batch, ldc;
  const double* P;
  double* C;
};
struct ScaleDesc {  // scale_cols_inv (k x r, ld) or the diagonal root diag(sv[:r])
  int k, r, ld, diag;
  double* Z;
  const double* sv;
};

hipError_t gemm_group_launch(hipStream_t s, bool ta, bool tb, const GemmDesc* d, const int* first, int nd,
                             int nblocks);
hipError_t gram_part_group_launch(hipStream_t s, bool mt8, const GramDesc* d, const int* first, int nd,
                                  int nblocks);
hipError_t gram_sum_group_launch(hipStream_t s, const GramDesc* d, const int* first, int nd, int nblocks);
hipError_t copy2d_group_launch(hipStream_t s, const CopyDesc* d, const int* first, int nd, int nblocks);
hipError_t sign_fix_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks);
hipError_t sign_part_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks);
hipError_t sign_decide_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks);
hipError_t sign_apply_group_launch(hipStream_t s, const SignDesc* d, const int* first, int nd, int nblocks);
hipError_t scale_group_launch(hipStream_t s, const ScaleDesc* d, const int* first, int nd, int nblocks);
hipError_t line_group_launch(hipStream_t s, bool fft, const LineDesc* d, const int* first, int nd, int nblocks);
hipError_t field_group_launch(hipStream_t s, const FieldDesc* d, const int* first, int nd, int nblocks);
hipError_t sum_group_launch(hipStream_t s, const SumDesc* d, const int* first, int nd, int nblocks);

// Arguments of one problem of a grouped operation, as the one-problem calls
// take them.
struct GemmArgs {
  int M, N, K;
  double alpha;
  const double* A;
  int lda;
  long long sA;
  const double* B;
  int ldb;
  long long sB;
  double beta;
  double* C;
  int ldc;
  long long sC;
  int batch;
};

class GroupQueue {
 public:
  // dmem / hmem: device and pinned host staging of cap bytes each
  GroupQueue(void* dmem, void* hmem, size_t cap) : d_((char*)dmem), h_((char*)hmem), cap_(cap) {}
  // one launch each (no launch when the list is empty)
  hipError_t gemm(bool ta, bool tb, const std::vector<GemmArgs>& p);
  // Gram matrices (the one-problem block count rule of gram_rows /
  // gram_mode2 per problem, given its partial-sum scratch)
  struct GramArgs {
    int k, n, mode2;
    const double* A;
    int lda, nb, r;
    double* part;
    size_t part_cap;
    double* G;
  };
  hipError_t gram(const std::vector<GramArgs>& p);
  hipError_t copy2d(const std::vector<CopyDesc>& p);
  struct SignArgs {
    int rows, cols;
    double* A;
    int lda;
    double* B;
    int ldb, rowsB;
    double* scratch;   // tall form only (null: the one-pass form)
    size_t scratch_elems;
  };
  hipError_t sign_fix(const std::vector<SignArgs>& p);        // sign_fix
  hipError_t sign_fix_tall(const std::vector<SignArgs>& p);   // sign_fix_tall
  hipError_t scale(const std::vector<ScaleDesc>& p);
  // line transforms (FFT and DFT problems in two launches)
  hipError_t lines(const std::vector<LineDesc>& p);
  hipError_t field(const std::vector<FieldDesc>& p);
  hipError_t sums(const std::vector<SumDesc>& p);
  // arbitrary launch that reads descriptors staged here: stage() copies
  // bytes into the staging area and returns their device address
  const void* stage(const void* src, size_t bytes);
  void then(std::function<hipError_t(hipStream_t)> fn) { ops_.push_back(std::move(fn)); }
  // upload everything staged, then issue the launches in order
  hipError_t flush(hipStream_t s);
  // staging restarts at 0: only once the stream has passed every earlier
  // upload (after a synchronisation)
  void reset() { used_ = 0; flushed_ = 0; }
  bool overflow() const { return overflow_; }

 private:
  template <class D>
  bool push(const std::vector<D>& descs, const std::vector<int>& first, const D** dd, const int** df);
  char* d_;
  char* h_;
  size_t cap_, used_ = 0, flushed_ = 0;
  bool overflow_ = false;
  std::vector<std::function<hipError_t(hipStream_t)>> ops_;
};

// grouped moments_run + poisson_run (fields.hip): per problem j the moments
// M[j] of frames F[j] and the field E[j] with ion density n_i[j], one
// launch per step of the one-problem calls for all n problems
hipError_t efield_group(GroupQueue& q, int n, Workspace* const* ws, const slar_frames* F, const double* n_i,
                        double* const* M, double* const* E);

// grouped slar_frames_from_ht (sample.hip): one launch per step of the
// one-tensor call for all n tensors; out[j]->r is set on return
hipError_t frames_from_ht_group(GroupQueue& q, int n, Workspace* const* ws, const slar_ht* const* F,
                                slar_frames* const* out);

}  // namespace slar
