/*
 * slar.h -- C ABI of the MI355X (gfx950) SLAR / LoMaC time-step library.
 *
 * One time step of the conservative semi-Lagrangian adaptive-rank method for
 * Vlasov--Poisson:  SL-FD entry evaluation at the feet of the
 * characteristics (section 3.1, eq. (tp_interp)), cross approximation of the
 * updated tensor and its HT truncation (HTACA; introduction, section 3.1,
 * Supplement B), spectral Poisson solve (section 3.1, eq. (slarvp) and its
 * field solver), and the adaptive-weight LoMaC projection with its implicit
 * macroscopic solve (section 3.2, eqs. (LoMaC_update_discrete),
 * (BE_nonlinear_system)).
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers owned by the caller unless a
 *    comment says "host".  Arrays are dense, row-major, FP64 unless the
 *    descriptor's dtype says FP32.  Nothing is freed or retained by the
 *    library after a call returns, except inside an slar_workspace.
 *  - Phase space is (x_1..x_dx, v_1..v_dv), dx == dv in {1, 2}.  Grids are
 *    uniform, cell-centred (x_i = lo + (i + 1/2)(hi - lo)/n) and periodic in
 *    every coordinate (section 2.1).  Nx = prod n_x, Nv = prod n_v; spatial
 *    and velocity multi-indices are linearised row-major.
 *  - Every call returns an slar_status and never aborts.  Arguments are
 *    validated before anything is enqueued; on SLAR_E_INVAL nothing ran.
 *  - Calls enqueue on the given HIP stream.  Calls whose control flow
 *    depends on device data (slar_cross_update, slar_truncate,
 *    slar_macro_solve) wait on that stream for the data they decide on
 *    (ranks, stopping flags, residuals); work enqueued after the last
 *    decision may still run when they return.  Their outputs are complete
 *    in stream order, and the host-side values they return (ranks, counts,
 *    statuses) are final.
 *  - A workspace may be used by one stream at a time.
 */
#ifndef SLAR_H_
#define SLAR_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLAR_OK = 0,
  SLAR_E_INVAL = 1,     /* bad argument; nothing was enqueued             */
  SLAR_E_NOMEM = 2,     /* device allocation failed / buffer too small     */
  SLAR_E_RANK_CAP = 3,  /* rank cap reached: output valid but truncated    */
  SLAR_E_NOCONV = 4,    /* Newton did not reach its tolerance              */
  SLAR_E_NUMERIC = 5,   /* NaN/Inf met                                     */
  SLAR_E_HIP = 6        /* a HIP runtime call failed                       */
} slar_status;

typedef enum { SLAR_F32 = 0, SLAR_F64 = 1 } slar_dtype;

/* Uniform periodic phase-space grid (section 3.1). */
typedef struct {
  int32_t dx, dv;       /* 1,1 or 2,2                                      */
  int32_t n[4];         /* cells per dimension, x first; 4 <= n <= 128 (2D2V) or 512 (1D1V) */
  double lo[4], hi[4];  /* domain [lo, hi) per dimension                    */
} slar_grid;

/* Hierarchical Tucker tensor on the tree {x}{v} (d = 2, a matrix) or
 * {{x1,x2},{v1,v2}} (d = 4) (section 3.1; section 4.2 rank labels).
 *   leaf[m]  : [n_m][rank[m]]            leaf bases U^(m)
 *   B12, B34 : [rank[0]*rank[1]][rank[4]], [rank[2]*rank[3]][rank[5]]
 *              transfer tensors, index (a*r_right + b)
 *   root     : d = 4: [rank[4]][rank[5]];  d = 2: [rank[0]][rank[1]]
 * F[i1,i2,i3,i4] = sum U1[i1,a] U2[i2,b] B12[a,b,c] root[c,e] U3[i3,p] U4[i4,q] B34[p,q,e]
 * F[i,j]         = sum Ux[i,a] root[a,b] Uv[j,b]                        (d = 2)
 * Ranks are host values.  Element type per dtype.                           */
typedef struct {
  int32_t d;
  int32_t rank[6];
  slar_dtype dtype;
  void* leaf[4];
  void* B12;
  void* B34;
  void* root;
} slar_ht;

/* Frame form of a tensor: F[I, J] = sum_c X[I][c] P[J][c], I spatial, J
 * velocity (linear indices).  X is [Nx][ld], P is [Nv][ld], FP64, columns
 * 0..r-1 used.  This is the {x}|{v} matricisation with the root folded
 * into P; it also holds the LoMaC-corrected tensor exactly (the correction
 * columns are appended, eq. (LoMaC_update_discrete)).                        */
typedef struct {
  int32_t r;
  int32_t ld;
  double* X;
  double* P;
} slar_frames;

/* One linear sub-flow of the SL update (section 3.1 and eq. (slarvp)):
 * characteristics dx/dt = cv * v, dv/dt = -E(x), traced back over tau.
 *   kind 0: split x-shift  x* = x - cv v tau                (exact)
 *   kind 1: split v-shift  v* = v + E(x) tau, E on the grid  (exact)
 *   kind 2: frozen-field flow, one classical RK4 step backwards in time;
 *           E between grid points by periodic degree-4 Lagrange interpolation
 * The frozen field is cE[0]*E[0] + cE[1]*E[1]; E[i] is [dx][Nx] FP64 (E[1]
 * may be NULL).  order is the interpolation stencil width, 3 or 5.          */
typedef struct {
  int32_t kind;
  int32_t order;
  double tau;
  double cv;
  const double* E[2];
  double cE[2];
} slar_adv;

/* Result of the cross approximation: F ~ sum_l U[l][:] (x) V[l][:],
 * U is [kmax][Nx], V is [kmax][Nv] (FP64, caller-owned, written).           */
typedef struct {
  int32_t k;
  double* U;
  double* V;
} slar_lowrank;

typedef struct {
  int32_t rank;          /* cross rank k                                    */
  int32_t iterations;    /* pivot rows visited                              */
  int32_t probe_rounds;  /* continuations forced by the random probes       */
  int32_t converged;
  int64_t samples;       /* SL-FD entries evaluated                         */
} slar_cross_info;

typedef struct slar_workspace slar_workspace;

const char* slar_status_str(slar_status s);

/* Allocates every device buffer the calls below need for grid g and rank
 * cap rmax (<= 64), once.  *ws is written on success.  No call below
 * allocates device memory (the batched, nested and CNN objects have their
 * own create calls).                                                        */
slar_status slar_workspace_create(const slar_grid* g, int32_t rmax, slar_workspace** ws);

/* Device bytes of a workspace for grid g and rank cap rmax: *bytes is
 * written.  Pure host arithmetic (no device call).                         */
slar_status slar_workspace_bytes(const slar_grid* g, int32_t rmax, size_t* bytes);

/* The same workspace with its device buffers carved from the caller's
 * device memory `work` (256-byte aligned, work_bytes >= the size
 * slar_workspace_bytes gives; SLAR_E_NOMEM if smaller, checked before any
 * device call).  The caller keeps `work` alive and unchanged by others
 * until slar_workspace_destroy, which does not free it.  The library still
 * creates its own pinned host words, events and one auxiliary stream.      */
slar_status slar_workspace_create_in(const slar_grid* g, int32_t rmax, void* work, size_t work_bytes,
                                     slar_workspace** ws);
slar_status slar_workspace_destroy(slar_workspace* ws);

/* SL-FD update at requested grid points, evaluated directly on an HT tensor
 * by the leaf interpolation c^(mu) = w(xi_mu) U^(mu)_{J_mu} and the transfer
 * contractions up to the root, O(d r^3) per point (section 3.1, eqs.
 * (1d_quadratic_interp_weight), (tp_interp)).
 *   idx : [n][d] int32 grid multi-indices (0-based) of the points to update
 *   out : [n] values f(x_i, t+tau) = f(x*, t), dtype of F (contractions
 *         in that precision; feet are FP64).
 * Supports order 3 and 5 for d = 2, order 3 for d = 4; ranks <= 64.          */
slar_status slar_ht_sample(const slar_grid* g, const slar_ht* F, const slar_adv* a, int64_t n,
                           const int32_t* idx, void* out, hipStream_t stream);

/* Frame form of an HT tensor (the x node frame (U1 (x) U2) B12 and the v
 * node frame times root^T).  out->X, out->P must have ld >= rank[4]
 * (d = 4) or rank[0] (d = 2) columns; out->r is written.                    */
slar_status slar_frames_from_ht(const slar_grid* g, const slar_ht* F, slar_frames* out,
                                slar_workspace* ws, hipStream_t stream);

/* The same SL-FD update evaluated from the frame form: stencil-weighted
 * gathers of the node frames (mathematically eq. (tp_interp) of the same
 * tensor).  dtype selects FP64 tables or FP32 copies made in ws.            */
slar_status slar_frame_sample(const slar_grid* g, const slar_frames* F, const slar_adv* a,
                              slar_dtype dtype, int64_t n, const int32_t* idx, double* out,
                              slar_workspace* ws, hipStream_t stream);

/* SLAR(F; a, dt, eps_Base) sampling stage (section 3.1; HTACA, introduction):
 * adaptive cross approximation with partial pivoting of the updated tensor
 * in its {x}|{v} matricisation, sampling whole fibers through the SL-FD
 * evaluator.  Pivot rules: first row 0; column pivot = lowest index within a
 * relative 1e-10 of the residual maximum; stop when |u_k||v_k| <= tol
 * ||S_k||_F or k == kmax; on stopping, nprobe host-given random entries
 * probes[nprobe][2] (row, col; device int32) are checked and the
 * approximation continues from the worst one if its residual exceeds
 * tol ||S_k||_F / sqrt(Nx Nv).  dtype is the precision of the sampled
 * tables.  Returns SLAR_E_RANK_CAP when kmax was hit before convergence.  */
slar_status slar_cross_update(const slar_grid* g, const slar_frames* src, const slar_adv* a,
                              slar_dtype dtype, double tol, int32_t kmax, int32_t nprobe,
                              const int32_t* probes, slar_lowrank* out, slar_cross_info* info,
                              slar_workspace* ws, hipStream_t stream);

/* Nested HT cross approximation of the same SL-FD update (d = 4, stencil
 * order 3): the cheaper cross sampler sections 4 and 5 call for, in the
 * nested skeleton form of Ballani, Grasedyck and Kluge (2013).  Leaf pivot
 * rows R_mu and complements Q_mu are searched inside (sibling rows) x
 * (parent complement), the root pivots P_x, P_v inside the products of the
 * leaf rows, each search being the cross approximation of
 * slar_cross_update (same pivot, tie, stopping and probe rules) at
 * tol / 10; the probes (four per sweep in rotation, and the worst failing
 * one) enrich the candidate sets, and after every sweep from the second on
 * they check the skeleton against tol ||F||_F / sqrt(Nx Nv).  Output, a
 * non-orthogonal HT (the skeleton):
 *   leaf[m]  = A^(m)[:, Q_m] A^(m)[R_m, Q_m]^-1            [n_m][rank[m]]
 *   B12      = A[R1, R2, P_v],  B34 = A[P_x, R3, R4]       (slar_ht layout)
 *   root     = A[P_x, P_v]^-1                               [k][k]
 *   probes : host int32 [nprobe][4] grid multi-indices (nprobe <= 1024)
 *   seed   : host int32 [4], the first pivot of every leaf
 *   out    : d = 4, FP64, caller-allocated with capacity leaf[m] n_m*kmax,
 *            B12 and B34 kmax^3, root kmax^2 doubles; ranks are written
 *   kmax   : 1 <= kmax <= 64
 * Synchronises the stream.  SLAR_E_NOCONV: the probes still fail after 12
 * sweeps (out holds the last skeleton); SLAR_E_NUMERIC: an all-zero update
 * or a singular pivot block.                                                  */
typedef struct {
  int32_t sweeps;
  int32_t probe_rounds;
  int32_t converged;
  int32_t rank[6];       /* r1, r2, r3, r4, k, k                            */
  int64_t samples;       /* SL-FD entries evaluated                         */
} slar_nested_info;

slar_status slar_nested_cross(const slar_grid* g, const slar_frames* src, const slar_adv* a,
                              slar_dtype dtype, double tol, int32_t kmax, int32_t nprobe,
                              const int32_t* probes, const int32_t* seed, slar_ht* out,
                              slar_nested_info* info, slar_workspace* ws, hipStream_t stream);

/* HTACA's final truncation (Supplement B): orthogonalise both factor sets,
 * SVD of the small core, root truncation with theta = tol ||F||_F /
 * sqrt(2d-3), then (d = 4) each leaf = leading left singular vectors of its
 * mode matricisation (same theta), transfer tensors by projection.  Column 0
 * of each leaf is the leading left singular vector of its mode.  out must
 * point to FP64 buffers sized for rmax in every rank; out->rank is written.
 * Returns SLAR_E_RANK_CAP if some rank was capped at rmax.                  */
slar_status slar_truncate(const slar_grid* g, const slar_lowrank* in, double tol, int32_t rmax,
                          slar_ht* out, slar_workspace* ws, hipStream_t stream);

/* Velocity moments on the x-grid (eqs. (raw moments), (disc_m0)-(disc_m2) and
 * the flux moments of eq. (macro_sys_comp)): M is [nmom][Nx] with rows
 * 1, v_1..v_dv, |v|^2, v_mu v_nu (mu <= nu), |v|^2 v_mu
 * (nmom = 5 for dv = 1, 9 for dv = 2).                                      */
slar_status slar_moments(const slar_grid* g, const slar_frames* F, double* M,
                         slar_workspace* ws, hipStream_t stream);

/* Spectral Poisson solve (eqs. (Poisson), (Efromphi), (charge_density)):
 * rho = n_i - n_e, -D.D phi = rho on the non-null Fourier modes (phi = 0 on
 * the null ones), E = -D phi, D the spectral derivative with the Nyquist
 * mode set to 0.  n_e, phi are [Nx]; E is [dx][Nx].  phi may be NULL.       */
slar_status slar_poisson(const slar_grid* g, const double* n_e, double n_i, double* phi,
                         double* E, slar_workspace* ws, hipStream_t stream);

/* slar_poisson without a workspace and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * result as slar_poisson.  Its scratch (the transform buffers and twiddle
 * tables, at most 3.2 MB: 2048 + 24 Nx doubles with Nx <= 128^2) is a
 * file-scope device array that every GPU holds until the process ends;
 * the device address is resolved once per device on the first call there.
 * Every call on a device shares that array: calls that overlap in time on
 * one device race and must be serialised by the caller (e.g. one stream).
 * A call writes every scratch element it reads.  Returns SLAR_E_NOMEM if
 * the grid needs more scratch than the array holds, SLAR_E_INVAL on a bad
 * grid or pointer.  Enqueued on stream.                                     */
slar_status slar_poisson_noalloc(const slar_grid* g, const double* n_e, double n_i, double* phi,
                                 double* E, hipStream_t stream);

/* Conserved variables U = (n, m n u, e_k + e_p) of a tensor ([dv+2][Nx]),
 * eq. (macro_sys_comp) with m_e = 1.                                        */
slar_status slar_conserved(const slar_grid* g, const slar_frames* F, double n_i, double* U,
                           slar_workspace* ws, hipStream_t stream);

/* LoMaC closure of F* (Supplement B): the weight omega^(mu) = max(|U^(v_mu)[:,0]|,
 * delta) from column 0 of the velocity leaves of the truncated F*, the
 * weighted Gram--Schmidt basis Q_0, Q_{1,mu}, Q_2 and norms, the moments of
 * F* and its projection coefficients.  Kept in ws for the two calls below.  */
slar_status slar_lomac_prepare(const slar_grid* g, const slar_ht* Fstar,
                               const slar_frames* Fstar_frames, double delta, double n_i,
                               slar_workspace* ws, hipStream_t stream);

/* Implicit macroscopic update (section 3.2.3): solves
 *   G(U) = U - U_hist + b dt (D.F(U) - S(U)) = 0
 * (bdf_order 1: backward Euler, U_hist = U_n, b = 1; 2: BDF2,
 * U_hist = 4/3 U_n - 1/3 U_nm1, b = 2/3) by Jacobian-free Newton--GMRES
 * started from U(F*) (section 4 tolerances: Newton 1e-10 on the RMS
 * residual, Krylov 1e-4 relative).  The flux is closed by the corrected
 * kinetic state of the prepared LoMaC closure.
 *   precond 0: plain GMRES (the paper's solver);
 *           1: flexible GMRES right-preconditioned by the exact per-Fourier-
 *              mode inverse of the linear constant-coefficient part of the
 *              Jacobian (kinetic flux of the closure + linearised Poisson
 *              source);
 *           2: as 1 plus the learned convolutional correction cnn, with
 *              plain GMRES as the fallback (slar_macro_fallbacks).
 * The converged answer is the same Newton root; only the iteration counts
 * change.  iters (host, int32[2]) receives Newton and Krylov counts.
 * Returns SLAR_E_NOCONV if Newton did not reach newton_tol.                 */
typedef struct slar_cnn slar_cnn;
slar_status slar_macro_solve(const slar_grid* g, const double* U_n, const double* U_nm1,
                             double dt, int32_t bdf_order, double newton_tol, double krylov_tol,
                             int32_t precond, const slar_cnn* cnn, double* U_out, int32_t* iters,
                             slar_workspace* ws, hipStream_t stream);

/* General implicit macroscopic system, the form every stage of the
 * section 4 integrators takes (two S-stable DIRK-3 start-up steps, then
 * variable-step BDF-3; section 3.2.3 for the stage structure):
 *   G(U) = U - sum_{j<nhist} c[j] U[j] + sum_{j<nstage} d[j] R[j]
 *          + beta (D.F(U) - S(U)) = 0,
 * solved like slar_macro_solve (same closure, preconditioners, tolerances,
 * status and iteration counts).  U[j] are history states and R[j] right-hand
 * sides of earlier stages (device, [dv+2][Nx] FP64, caller-owned, not
 * U_out); beta > 0 includes the step size.  Weights with sum c = 1 keep the
 * mean of every component exact, hence mass, momentum and energy
 * conserved to round-off.  Backward Euler: nhist 1, c 1, beta dt; a DIRK
 * stage i: U[0] = U_n, c 1, R[j] the earlier stages' right-hand sides with
 * d[j] = dt a_ij, beta = dt a_ii; BDF-k: slar_bdf_weights.                */
typedef struct {
  int32_t nhist;
  const double* U[3];
  double c[3];
  int32_t nstage;
  const double* R[3];
  double d[3];
  double beta;
} slar_macro_system;
slar_status slar_macro_solve_system(const slar_grid* g, const slar_macro_system* S,
                                    double newton_tol, double krylov_tol, int32_t precond,
                                    const slar_cnn* cnn, double* U_out, int32_t* iters,
                                    slar_workspace* ws, hipStream_t stream);

/* Convergence record of the last slar_macro_solve / _system on ws, one
 * record of 4 doubles per Newton iteration (at most 32 records):
 * {RMS residual ||G||_2 / sqrt(n) at the start of the iteration, Krylov
 * iterations of its linear solve, true linear residual ||J d + G|| / ||G||
 * at its end, GMRES restarts}.  The last record holds the final residual
 * (its other fields 0 when Newton converged there).  Copies
 * min(count, cap) records into out (host [cap][4]) and returns count, or
 * -1 on invalid arguments.  Host only; reflects the last solve that ran. */
int32_t slar_macro_history(const slar_workspace* ws, double* out, int32_t cap);

/* Fallback of the learned preconditioner: a solve with precond = 2 whose
 * network-preconditioned attempt fails (a Newton step's linear solve not at
 * krylov_tol within 100 iterations, no Newton convergence, a non-finite
 * residual or a failed launch) is repeated from U(F*) with plain GMRES, and
 * its status is the plain solve's.  Returns the number of solves on ws that
 * fell back since it was created (-1 if ws is NULL); *last (host, may be
 * NULL) is 1 if the last solve did.  Host only.                           */
int32_t slar_macro_fallbacks(const slar_workspace* ws, int32_t* last);

/* Right-hand side R(U) = D.F(U) - S(U) of the moment system U' = -R(U)
 * (eq. (BE_nonlinear_system) without the history), with the closure of the
 * last slar_lomac_prepare on ws (SLAR_E_INVAL if none).  U, R_out device
 * [dv+2][Nx] FP64, distinct.  Enqueued on stream.                          */
slar_status slar_macro_rhs(const slar_grid* g, const double* U, double* R_out,
                           slar_workspace* ws, hipStream_t stream);

/* Butcher tableau of the S-stable three-stage DIRK method (Alexander 1977,
 * Theorem 5) that section 4 uses for start-up: gamma the root in (1/6, 1/2)
 * of 6x^3 - 18x^2 + 9x - 1; c = (gamma, (1 + gamma)/2, 1); A (host,
 * row-major [3][3]) lower triangular with diagonal gamma, a21 = (1-gamma)/2,
 * last row b1 = -(6 gamma^2 - 16 gamma + 1)/4, b2 = (6 gamma^2 - 20 gamma
 * + 5)/4, gamma (= b).  Host only.                                        */
slar_status slar_dirk3_tableau(double* A, double* c);

/* Weights of the classical variable-step BDF-k (Gear 1971), k = 1..3: the
 * derivative at t[0] of the polynomial through (t[j], U_j), j = 0..k (host,
 * t[0] = t_{n+1} > t[1] = t_n > ...), set to -R(U_0), gives
 *   U_0 - sum_{j=1..k} c[j-1] U_j + beta R(U_0) = 0.
 * c (host [k]) and *beta (host) out.  Equal steps h and k = 3 give
 * 18/11, -9/11, 2/11 and 6h/11.  Host only; SLAR_E_INVAL unless the times
 * decrease strictly.                                                       */
slar_status slar_bdf_weights(int32_t k, const double* t, double* c, double* beta);

/* Band-limited LoMaC correction (a stabilisation of this implementation,
 * not in the paper): U <- U(F*) + sigma (U - U(F*)) with U(F*) the
 * conserved variables of the prepared closure and sigma the exponential
 * filter prod_d exp(-36 kappa_d^8) of each x-mode (kappa_d = |m_d| /
 * (n_d / 2), the mode index relative to the Nyquist index; sigma = 1 on
 * the zero mode, 1 - 1e-4 at kappa = 1/5, 0.87 at kappa = 1/2, e^-36 at
 * the Nyquist index).  The macroscopic and kinetic discretisations differ
 * at the upper x-modes (spectral flux divergence against SL
 * interpolation); imposing the macroscopic upper modes on the kinetic
 * state let that mismatch grow from step to step at 128^2 x-cells.  Totals (mass, momentum, energy) are
 * unchanged exactly.  U device [dv+2][Nx] FP64, in place; needs
 * slar_lomac_prepare on ws.  Enqueued on stream.                          */
slar_status slar_lomac_filter(const slar_grid* g, double* U, slar_workspace* ws, hipStream_t stream);

/* LoMaC update eq. (LoMaC_update_discrete):
 *   F^{n+1} = F* - R(U(F*)) + R(U_new) = F* + sum_k dC_k (x) Q_k,
 * returned exactly (no re-truncation) in frame form: out->X = [X* | dC],
 * out->P = [P* | Q]; out->ld >= Fstar_frames->r + dv + 2.                   */
slar_status slar_lomac_project(const slar_grid* g, const slar_frames* Fstar_frames,
                               const double* U_new, slar_frames* out, slar_workspace* ws,
                               hipStream_t stream);

/* ---------------------------------------------------------------------
 * Learned preconditioner (an addition to the paper's solver, whose section 5
 * names preconditioning of the Krylov solve as future work).  A periodic
 * convolutional network, FP32, 3x3 kernels, tanh between layers:
 *   out[o,y,x] = b[o] + sum_{c,dy,dx} w[o,c,dy,dx] in[c, y+dy-1, x+dx-1].
 * Parameters are packed per layer as w [Co][Ci][3][3] then b [Co].  Inside
 * slar_macro_solve (precond = 2) it corrects the spectral preconditioner:
 *   z = P_spec(v) + rms(v) * CNN([v / rms(v), (U_c - mean U_c) / std U_c]),
 * so channels[0] must be 2 (dv + 2) and channels[nlayers] dv + 2.
 * Tensors x, y are device FP32 [B][C][H][W]; host arrays are marked.       */
slar_status slar_cnn_create(int32_t nlayers, const int32_t* channels /* host, nlayers+1 */,
                            int32_t max_batch, int32_t max_pixels, slar_cnn** out);
slar_status slar_cnn_destroy(slar_cnn* cnn);
int32_t slar_cnn_nparams(const slar_cnn* cnn);
slar_status slar_cnn_set_params(slar_cnn* cnn, const float* params_host, int32_t n);
slar_status slar_cnn_get_params(const slar_cnn* cnn, float* params_host, int32_t n);
slar_status slar_cnn_forward(slar_cnn* cnn, int32_t B, int32_t H, int32_t W, const float* x,
                             float* y, hipStream_t stream);
/* gradient of the mean squared error mean((CNN(x) - y)^2) w.r.t. the
 * parameters (grad_host may be NULL; loss_host receives the loss if given) */
slar_status slar_cnn_grad(slar_cnn* cnn, int32_t B, int32_t H, int32_t W, const float* x,
                          const float* y, float* grad_host, float* loss_host, hipStream_t stream);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the same loss             */
slar_status slar_cnn_train_step(slar_cnn* cnn, int32_t B, int32_t H, int32_t W, const float* x,
                                const float* y, float lr, float* loss_host, hipStream_t stream);
/* The learned correction alone, as slar_macro_solve (precond = 2) applies
 * it to the spectral preconditioner's output:
 *   z += rms(v) * CNN([v / rms(v), (U_c - mean U_c) / std U_c]),
 * with rms over all K = dv + 2 components and pixels, the mean and standard
 * deviation per component (std + 1e-12 |mean| + 1e-300, so a constant
 * component maps to zero).  v, U, z device [K][Nx] FP64 on the x grid of g
 * (Nx = n[0] n[1], x1 fastest); z is read and written, distinct from v and
 * U.  Needs dx = 2 and channels 2K -> ... -> K (SLAR_E_INVAL otherwise); a
 * 2K -> 16 -> 16 -> K network of any grid runs fused in one launch after a
 * statistics pass.  Enqueued on stream.  The network object holds the
 * statistics and activation buffers, so calls that share one network
 * (here, in slar_macro_solve or in training) must not overlap in time.     */
slar_status slar_cnn_correct(const slar_grid* g, const slar_cnn* cnn, const double* v,
                             const double* U, double* z, slar_workspace* ws, hipStream_t stream);
/* Records up to `capacity` training pairs from later flexible-GMRES solves
 * of this workspace: features [capacity][2K][Nx] (network input for w = J z)
 * and targets [capacity][K][Nx] ((z - P_spec(w)) / rms(w)), FP32 device
 * buffers owned by the caller.  capacity 0 stops recording.               */
slar_status slar_record_krylov(slar_workspace* ws, float* features, float* targets, int32_t capacity);
int32_t slar_recorded_pairs(const slar_workspace* ws);

/* Leaf bases of slar_truncate (Supplement B, HOSVD of the mode
 * matricisations A): the eigenvectors E of A A^T carry errors of eps s_1^2
 * / (gap of the squared singular values); the refinement pass (on = 1, the
 * default) completes E to an orthonormal basis and re-diagonalises the
 * Gram of E^T A, which brings the leaves to the accuracy of an SVD of A
 * (about eps s_1 / gap).  on = 0 skips it: for FP32 frame tables, whose
 * sampling error is far above either bound.  Returns SLAR_E_INVAL for a
 * null workspace or on outside {0, 1}.                                     */
slar_status slar_leaf_refine(slar_workspace* ws, int32_t on);

/* Timing of the two sampling kernels of slar_cross_update.  on = 0 turns
 * it off; on = n >= 1 times every n-th iteration of each cross
 * approximation (iterations n-1, 2n-1, ...): its row-fiber and
 * column-fiber launches carry start/stop HIP events on their own dispatch
 * (kernel duration, no marker packets in between).  Each timed dispatch
 * costs a few microseconds of pipeline time, so n > 1 keeps the timed
 * program close to the untimed one while the sampled launches still give
 * the average duration.  Enabling clears the counters.  Only iterations
 * that did their work are counted.  slar_timing_read fills host out[8] = {row
 * ms, row launches, row algorithmic bytes, column ms, column launches,
 * column algorithmic bytes, 0, 0}; algorithmic bytes per sampled entry =
 * both stencil gathers of the frame tables + 16 k bytes of previous cross
 * vectors + 8 bytes written.                                               */
slar_status slar_timing_enable(slar_workspace* ws, int32_t on);
slar_status slar_timing_read(const slar_workspace* ws, double* out);

/* ------------------------------------------------------------------------
 * Many independent instances of uneven grid size and rank (each a separate
 * Vlasov--Poisson problem advanced by the same SLAR sub-flows, section 3.1).
 * A batch owns one workspace per instance, the device tables of the
 * persistent multi-instance cross approximation, a captured hipGraph of its
 * iteration chunk, and the staging memory of the grouped launches (one
 * launch per step for all instances) of the truncation, frame builds and
 * field solves; all work runs on the caller's stream.
 * Array arguments below are host arrays of `count` entries, in instance
 * order; the device buffers they point to belong to the caller.  A batch is
 * used from one host thread and one caller stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct slar_batch slar_batch;

/* grids[count]: the instances' grids (each validated as for
 * slar_workspace_create); rmax bounds every rank.  Allocates device memory
 * for count workspaces; synchronises the device.                            */
slar_status slar_batch_create(int32_t count, const slar_grid* grids, int32_t rmax,
                              slar_batch** out);
slar_status slar_batch_destroy(slar_batch* b);

/* The workspace of instance q (owned by the batch; NULL if q is out of
 * range), for the one-instance calls (set-up, moments, diagnostics).        */
slar_workspace* slar_batch_workspace(slar_batch* b, int32_t q);

/* slar_cross_update for every instance at once, FP32 tables, 3-point
 * stencils (order 3 only).  Per instance: src[q], adv[q], probes[q]
 * (device int32 [nprobe][2], may be NULL when nprobe == 0), out[q] (U/V
 * device buffers, k written), info[q] (may be NULL as a whole).  tol, kmax,
 * nprobe are shared.  The pivoting and stopping rules, and with team width
 * 16 every sampled value, are those of slar_cross_update with SLAR_F32.
 * Returns the most severe per-instance status (SLAR_E_RANK_CAP if any
 * instance hit kmax).  Synchronises the stream.                             */
slar_status slar_batch_cross_update(slar_batch* b, const slar_frames* src, const slar_adv* adv,
                                    double tol, int32_t kmax, int32_t nprobe,
                                    const int32_t* const* probes, slar_lowrank* out,
                                    slar_cross_info* info, hipStream_t stream);

/* slar_truncate for every instance (bit-identical results), followed,
 * when frames != NULL, by slar_frames_from_ht into frames[q] (ld >= rmax);
 * every step is one grouped launch over all instances on `stream`, and the
 * host reads the singular values and eigenvalues of all instances in one
 * copy each.  Each workspace's leaf-refinement setting applies to its
 * instance.  status (host int32[count], may be NULL) receives per-instance
 * statuses; the return value is the most severe of them.  Synchronises the
 * stream.                                                                   */
slar_status slar_batch_truncate(slar_batch* b, const slar_lowrank* in, double tol, int32_t rmax,
                                slar_ht* out, slar_frames* frames, int32_t* status,
                                hipStream_t stream);

/* Per instance: moments M[q] ([nmom][Nx], as slar_moments) of F[q] and the
 * spectral Poisson field E[q] ([dx][Nx]) with ion density n_i[q] (host),
 * bit-identical to slar_moments + slar_poisson; every step one grouped
 * launch over all instances, enqueued on `stream` (no synchronisation).     */
slar_status slar_batch_efield(slar_batch* b, const slar_frames* F, const double* n_i,
                              double* const* M, double* const* E, hipStream_t stream);

/* Launch configuration of the batched cross approximation (host int32[8]):
 * {persistent grid blocks, 64-sample tiles per work item, iterations per
 * captured graph chunk, gather team width for source rank <= 16, <= 32,
 * > 32, graph captures so far (read only), 0}.  Team widths are 4, 8 or 16
 * lanes per sample; a width other than 16 changes FP32 rounding order only. */
slar_status slar_batch_get_config(const slar_batch* b, int32_t* cfg);
slar_status slar_batch_set_config(slar_batch* b, const int32_t* cfg);

/* Autotuner: times reps full batched cross approximations of the given
 * inputs per candidate, coordinate-wise over grid size {256..4096}, tiles
 * per item {1,2,4}, team width per occupied rank bucket {4,8,16} and chunk
 * {4,8,16}, and keeps the fastest configuration.  out is overwritten.      */
slar_status slar_batch_tune(slar_batch* b, const slar_frames* src, const slar_adv* adv, double tol,
                            int32_t kmax, int32_t nprobe, const int32_t* const* probes,
                            slar_lowrank* out, int32_t reps, hipStream_t stream);

/* Accumulated batched cross time: host double[4] = {device ms from the
 * first preparation launch to the end of the last graph chunk, graph chunks
 * launched, sum over calls of the largest instance iteration count, calls}. */
slar_status slar_batch_timing(const slar_batch* b, double* out);
slar_status slar_batch_timing_reset(slar_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* SLAR_H_ */
