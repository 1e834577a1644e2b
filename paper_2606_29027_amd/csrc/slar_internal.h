// Internal declarations of the gfx950 SLAR library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>
#include <vector>

#include "../../include/slar.h"
#include "sl_device.h"

#define SLAR_KMAX 72      // largest frame width (HT rank cap 64 + LoMaC columns)
#define SLAR_CROSS_KMAX 128  // largest number of cross-approximation terms
#define SLAR_NMAX 128     // largest cells per dimension of a 2D2V grid
#define SLAR_NMAX_1D 512  // largest cells per dimension of a 1D1V grid
#define SLAR_NLINE 512    // longest 1D line: FFT lines, 1D velocity bases
#define SLAR_MAXMOM 9     // moments for dv = 2

#define HIP_TRY(expr)                                       \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return SLAR_E_HIP;                \
  } while (0)

// same, for functions returning hipError_t
#define HIP_CHK(expr)                                       \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return e_;                        \
  } while (0)

namespace slar {

// ------------------------------------------------------------------ grid
// ------------------------------------------------------------- workspace
struct Workspace {
  slar_grid grid;
  GridDev G;
  int rmax;
  bool owns_device = true;       // device buffers allocated here (else the caller's work)
  // sampling
  double* Eeff = nullptr;        // [dx][Nx]
  float* X32 = nullptr;          // [Nx][LD32]
  float* P32 = nullptr;          // [Nv][LD32]
  int ld32 = 0;
  // cross approximation
  void* aca_ctl = nullptr;       // AcaCtl
  void* aca_ctl_host = nullptr;  // pinned copies: [0] final, [1], [2] polling ring
  hipEvent_t poll_ev[2] = {nullptr, nullptr};   // completion of the ring copies
  int* phase_host = nullptr;       // host-mapped pinned word: cross phase written by the device
  int* phase_dev = nullptr;        // its device address
  double* aca_part = nullptr;    // partial reductions
  int* aca_piv = nullptr;        // [2 SLAR_CROSS_KMAX] accepted pivots (row, col)
  unsigned char* used = nullptr; // [Nx]
  double* resid = nullptr;       // [max(Nx,Nv)]
  // dense linear algebra scratch
  double* dwork = nullptr;
  size_t dwork_elems = 0;
  double* small = nullptr;       // small matrices (k x k etc.)
  size_t small_elems = 0;
  int* ismall = nullptr;
  void* host_pinned = nullptr;   // pinned host staging
  // spectral
  double* tw[2] = {nullptr, nullptr};   // twiddles per x-dimension [N][2]
  double* cbuf = nullptr;               // complex scratch
  size_t cbuf_elems = 0;
  // moments
  double* psi = nullptr;         // [Nv][nmom]
  // LoMaC closure
  double* lm = nullptr;          // packed closure arrays
  size_t lm_elems = 0;
  double lm_scal[64];            // host copy of 1D scalars
  double n_i = 1.0;
  bool lm_ready = false;
  // macro / Krylov
  double* kry = nullptr;
  size_t kry_elems = 0;
  // history of the last macro solve, one record per Newton iteration:
  // {RMS residual, Krylov iterations, true GMRES residual / ||G||, restarts}
  double newton_hist[4 * 32];
  int newton_hist_n = 0;
  // learned-preconditioner solves that fell back to plain GMRES (count
  // since creation; whether the last solve did)
  int macro_fallbacks = 0;
  bool macro_fell_back = false;
  // second stream (default priority) for independent chains inside a call,
  // joined back before the call returns; fork_aux = false keeps every chain
  // on the caller's stream (batched instances: the pool already overlaps
  // instances, and one more stream per instance would only share the same
  // hardware queues)
  hipStream_t aux = nullptr;
  bool fork_aux = true;
  // refinement pass of the leaf bases in the truncation (accuracy to the
  // singular-value gaps instead of the squared ones); on by default
  bool leaf_refine = true;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional in-stream event timing of the cross-approximation sampling
  // kernels: [0] row ms, [1] row launches, [2] row bytes, [3] col ms,
  // [4] col launches, [5] col bytes
  bool timing = false;
  int timing_every = 1;          // time iterations every-1, 2 every-1, ...
  std::vector<hipEvent_t> events;
  double tstat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // optional recording of (J z, z) pairs for training the preconditioner
  float* rec_feat = nullptr;
  float* rec_targ = nullptr;
  int rec_cap = 0;
  int rec_count = 0;
  // nested HT cross (d = 4 only): search factors and tables, sample lists,
  // small matrices, frames for the norm, FP64 sampling tables
  double* nest_U = nullptr;        // [64][NEST_TAB]
  double* nest_V = nullptr;        // [64][NEST_TAB]
  unsigned char* nest_used = nullptr;
  int* nest_rowtab = nullptr;      // [NEST_TAB][4]
  int* nest_coltab = nullptr;      // [NEST_TAB][4]
  int* nest_probes = nullptr;      // [128][2]
  int* nest_piv = nullptr;         // [2 SLAR_KMAX]
  int* nest_idx = nullptr;         // [nest_list_elems][4]
  double* nest_vals = nullptr;     // [nest_list_elems]
  double* nest_small = nullptr;    // [6][64 * 64]
  int* nest_flag = nullptr;        // [4]
  double* nest_fX = nullptr;       // [Nx][SLAR_KMAX]
  double* nest_fP = nullptr;       // [Nv][SLAR_KMAX]
  double* nest_X64 = nullptr;      // [Nx][SLAR_KMAX]
  double* nest_P64 = nullptr;      // [Nv][SLAR_KMAX]
  long long nest_samples = 0;
};

// launchers implemented across the .hip files
// C_b = alpha op(A_b) op(B_b) + beta C_b (row-major, FP64) on stream s, on
// the matrix cores (gemm.hip); beta = 0 never reads C
hipError_t gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                    double beta, double* C, int ldc, long long sC, int batch);
size_t nest_list_elems();
slar_status nested_run(hipStream_t s, Workspace* ws, const slar_frames& src, const slar_adv& adv,
                       slar_dtype dt, double tol, int kmax, int nprobe, const int* probes, const int* seed,
                       slar_ht* out, slar_nested_info* info);
hipError_t combine_field(hipStream_t s, const GridDev& G, const slar_adv* a, double* out);
// Regularised skeleton of a cross that stopped at its term cap: replaces
// the k terms in out by min(rcap, rank W) terms of C W_r^+ R (synchronises)
slar_status cur_core_run(hipStream_t s, Workspace* ws, slar_lowrank* out, int rcap);
// The same for n crosses at once (the pivot-block SVDs in one grouped
// launch, one host read of all singular values); per-cross statuses in
// st[j].  dmem / hmem: cur_core_group_bytes(n) device / pinned host bytes.
size_t cur_core_group_bytes(int n);
slar_status cur_core_group(hipStream_t s, int n, Workspace* const* ws, slar_lowrank* const* out,
                           const int* rcap, slar_status* st, void* dmem, void* hmem);

}  // namespace slar

struct slar_workspace {
  slar::Workspace w;
};
