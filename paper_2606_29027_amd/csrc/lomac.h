// LoMaC closure, macroscopic solve and projection (internal).
#pragma once
#include "slar_internal.h"

namespace slar {
constexpr int KRY_RESTART = 50;     // GMRES restart length
constexpr int KRY_MAXIT = 500;      // Krylov iterations per Newton step
constexpr int KRY_MAX_NEWTON = 30;
// Krylov iterations per Newton step after which a solve preconditioned by
// the learned network is abandoned for plain GMRES
constexpr int KRY_LEARNED_LIMIT = 100;

struct LmLayout {
  size_t gs, scal, Q, psiQ, Mstar, Cstar, U0, Aflux, total;
};
LmLayout lm_layout(const GridDev& G);
size_t kry_elems_for(int Nx, int K, int m);
slar_status lomac_filter_run(hipStream_t s, Workspace* ws, double* U);
slar_status lomac_prepare_run(hipStream_t s, Workspace* ws, const slar_ht& Fs,
                              const slar_frames& Ff, double delta, double n_i);
hipError_t macro_residual(hipStream_t s, Workspace* ws, const double* U, const double* Uhist,
                          double bdt, double* Gout);
// history of one implicit macroscopic system (DIRK stage or BDF step):
//   G(U) = U - sum_j c_j U_j + sum_j d_j R_j + beta R(U)
struct MacroHist {
  int nh;
  const double* U[3];
  double c[3];
  int nr;
  const double* R[3];
  double d[3];
};
slar_status macro_solve_run(hipStream_t s, Workspace* ws, const MacroHist& hist, double beta,
                            double newton_tol, double krylov_tol, int precond,
                            const slar_cnn* cnn, double* Uout, int* iters);
// R(U) = D.F(U) - S(U) with the prepared closure
hipError_t macro_rhs(hipStream_t s, Workspace* ws, const double* U, double* Rout);
slar_status lomac_project_run(hipStream_t s, Workspace* ws, const slar_frames& Fs,
                              const double* Unew, slar_frames* out);
// training pair recorder (cnn.hip): features of w = J z and the target
// (z - P_spec(w)) / rms(w); pw = P_spec(w)
hipError_t record_pair(hipStream_t s, Workspace* ws, const double* w, const double* z,
                       const double* U, const double* pw);
// learned preconditioner application z = M(v) (cnn.hip)
hipError_t cnn_apply(hipStream_t s, Workspace* ws, const slar_cnn* net, const double* v,
                     const double* U, double* z);
}  // namespace slar
