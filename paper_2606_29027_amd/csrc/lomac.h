// LoMaC closure, macroscopic solve and projection (internal).
#pragma once
#include "slar_internal.h"

namespace slar {
constexpr int KRY_RESTART = 50;     // GMRES restart length
constexpr int KRY_MAXIT = 500;      // Krylov iterations per Newton step
constexpr int KRY_MAX_NEWTON = 30;

struct LmLayout {
  size_t gs, scal, Q, psiQ, Mstar, Cstar, U0, Aflux, total;
};
LmLayout lm_layout(const GridDev& G);
size_t kry_elems_for(int Nx, int K, int m);
slar_status lomac_prepare_run(hipStream_t s, Workspace* ws, const slar_ht& Fs,
                              const slar_frames& Ff, double delta, double n_i);
hipError_t macro_residual(hipStream_t s, Workspace* ws, const double* U, const double* Uhist,
                          double bdt, double* Gout);
slar_status macro_solve_run(hipStream_t s, Workspace* ws, const double* Un, const double* Unm1,
                            double dt, int bdf, double newton_tol, double krylov_tol, int precond,
                            const slar_cnn* cnn, double* Uout, int* iters);
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
