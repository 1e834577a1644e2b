// Field helpers shared by the Poisson, moments, LoMaC and macro code.
#pragma once
#include <vector>

#include "slar_internal.h"

namespace slar {
void host_twiddles(int n, std::vector<double>& tw);
hipError_t dft_forward(hipStream_t s, Workspace* ws, int B, const double* in, double2* out, double2* tmp);
hipError_t dft_inverse(hipStream_t s, Workspace* ws, int B, const double2* in, double* out, double2* tmp);
hipError_t spectral_symbol(hipStream_t s, Workspace* ws, int op, int nvec, const double2* in, double2* out);
// Spectral stage: Bin real fields [Bin][Nx] -> one pointwise map per
// Fourier mode -> Bout real fields [Bout][Nx] (op, Bin -> Bout):
// SPEC_POISSON 1 -> 1 + dx (phi, E), SPEC_DTPHI dx -> dx (grad dt phi),
// SPEC_DIV K dx -> K, SPEC_PRECOND K -> K (Minv [K][K][Nx] complex),
// SPEC_FILTER K -> K (exponential filter sigma(m0) sigma(m1) per mode).
// scr holds 20 Nx complex values.  Power-of-two grids run the axis-1
// forward pass, one fused axis-0 launch and the axis-1 inverse pass.
enum SpecOp { SPEC_POISSON = 0, SPEC_DTPHI = 1, SPEC_DIV = 2, SPEC_PRECOND = 3, SPEC_FILTER = 4 };
hipError_t spectral_stage(hipStream_t s, Workspace* ws, int op, const double* in, double* out,
                          const double2* Minv, double2* scr);
hipError_t poisson_run(hipStream_t s, Workspace* ws, const double* n_e, double n_i, double* phi, double* E);
int nmom_of(int dv);
hipError_t psi_build(hipStream_t s, Workspace* ws);
hipError_t gemm_tn_long(hipStream_t s, Workspace* ws, int rows, int cols, int n, const double* A,
                        int lda, const double* B, int ldb, double* C, int ldc);
hipError_t moments_run(hipStream_t s, Workspace* ws, const slar_frames& F, double* M);
hipError_t conserved_from_moments(hipStream_t s, Workspace* ws, const double* M, double n_i, double* U);

// cbuf layout (in doubles): [0, 80 Nx) complex scratch (40 fields),
// [80 Nx, 96 Nx) real scratch, then 4096 spare.
inline size_t cbuf_elems_for(int Nx) { return (size_t)96 * Nx + 4096; }
}  // namespace slar
