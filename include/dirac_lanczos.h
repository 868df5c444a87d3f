/*
 * dirac_lanczos.h -- C ABI of the MI355X (gfx950) Lanczos short-time propagator
 * for the two-dimensional Dirac equation.
 *
 * Method: Beerwerth & Bauke, "Krylov subspace methods for the Dirac equation",
 * arXiv:1407.7370.  One time step is psi <- exp(-i A) psi with
 * A = dt * H(t_bar) (Sec. 3, eq. time_evolution_approx, first Magnus term),
 * approximated in an m-dimensional Krylov space built by the Lanczos recurrence
 * (Sec. 2, Fig. 1) as ||psi|| Q exp(-i T) e_1 (Sec. 4, eq. matrix_exp_approx).
 *
 * Hamiltonian (Sec. 3, 2D representation alpha1 = sigma1, alpha2 = sigma2,
 * beta = sigma3):
 *     H = c [sigma1 (p_x - q A_x) + sigma2 (p_y - q A_y)] + m c^2 sigma3 + V
 * with p = -i d/dx realised by central first-derivative differences
 * (f[i+1] - f[i-1]) / (2h) (Sec. 7, first-order finite differences),
 * A = (B/2)(-y, x) + A_L(t) (uniform B_z in the symmetric gauge plus a
 * homogeneous laser field), and V the potential energy q*phi.
 *
 * Conventions shared by every call:
 *   - Grid: x_i = x_min + i*h_x, h_x = (x_max - x_min)/nx, i = 0..nx-1; same
 *     for y.  bc = 0 (Dirichlet): psi = 0 outside the grid; bc = 1: periodic.
 *   - Spinor layout: device array of 2*ny*nx complex128 values (interleaved
 *     re, im doubles), index ((s*ny + j)*nx + i) for component s, row j,
 *     column i -- i.e. a contiguous (2, ny, nx) complex128 tensor.
 *   - Inner product <u,v> = sum over sites and components of conj(u) v;
 *     alpha = Re <q, z>; the norm is Euclidean (no h^2 weight).
 *   - Atomic units: m = 1, c = 137.036, q = -1 for an electron.
 *
 * Ownership: the caller owns every device buffer (psi, the workspace, an
 * optional potential table) and the HIP stream.  The library owns only the
 * opaque host context; it never allocates or frees device memory.
 *
 * Errors: every call returns a dl_status; nothing is thrown across the ABI.
 * dirac_lanczos_last_error() returns a message for the last failing call on a
 * context.  Krylov breakdown (an invariant subspace) is not an error.
 */
#ifndef DIRAC_LANCZOS_H
#define DIRAC_LANCZOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dl_context dl_context;

typedef enum {
    DL_OK = 0,
    DL_ERR_INVALID = 1,     /* invalid parameters or arguments */
    DL_ERR_DEVICE = 2,      /* HIP runtime error (message in last_error) */
    DL_ERR_NONFINITE = 3,   /* a Lanczos reduction became NaN/Inf */
    DL_ERR_WORKSPACE = 4,   /* workspace missing, too small or misaligned */
    DL_ERR_UNSUPPORTED = 5  /* valid request that the library does not provide */
} dl_status;

enum { DL_BC_DIRICHLET = 0, DL_BC_PERIODIC = 1 };
enum { DL_PREC_FP64 = 0, DL_PREC_MIXED = 1 };
enum { DL_POT_NONE = 0, DL_POT_SOFTCORE = 1, DL_POT_PAPER_SOFTCORE = 2 };
enum { DL_PULSE_NONE = 0, DL_PULSE_SIN_SIN2 = 1, DL_PULSE_FOURIER_SIN2 = 2 };
enum { DL_MODE_STEP = 0, DL_MODE_EIGEN = 1, DL_MODE_LOWMEM = 2, DL_MODE_EIGEN_REORTH = 3 };

/*
 * Problem description (Sec. 3 Hamiltonian, Sec. 7 grid).
 *   nx, ny >= 3; x_min < x_max; y_min < y_max.
 *   krylov_dim: m, 1..64 (Lanczos iterations per step, Fig. 1's k).
 *   precision: DL_PREC_FP64 -- every vector and every operation in double;
 *              DL_PREC_MIXED -- Krylov vectors 2..m stored as complex64, all
 *              arithmetic, the state psi, reductions, T, exp(-iT) and the
 *              recombination coefficients in double.
 *   bz: uniform B_z, vector potential (bz/2)(-y, x) about the origin.
 *   pot_kind: DL_POT_SOFTCORE V = -pot_z / sqrt(r^2 + pot_a^2);
 *             DL_POT_PAPER_SOFTCORE V = -(3/2) pot_z / sqrt(r^2 + 3/pot_z^2)
 *             (eq. soft_core_pot).
 *   v_table: optional DEVICE pointer to ny*nx doubles (row-major [j][i])
 *            added to V; must stay valid for the context's lifetime. NULL: none.
 *   pulse_kind: homogeneous laser vector potential A_L(t), zero outside [0, T]:
 *     DL_PULSE_SIN_SIN2: a0 sin(omega t) sin^2(pi t/T) (pulse_e[0], pulse_e[1]);
 *     DL_PULSE_FOURIER_SIN2: sin^2(pi t/T) sum_{k=1}^{n_coef/4}
 *        [(a_k^x sin k w0 t + b_k^x cos k w0 t), (a_k^y sin .. + b_k^y cos ..)]
 *        with w0 = 2 pi / T and coef[4(k-1) + {0,1,2,3}] = {a_k^x, b_k^x,
 *        a_k^y, b_k^y}.  coef is a HOST pointer, copied during init.
 *   t_pulse: T > 0 when pulse_kind != 0.
 *   chirality: +1 (or 0): alpha2 = sigma2 as above; -1: alpha2 = -sigma2, the
 *     other inequivalent 2D representation (Sec. 3: the four-component 2D
 *     equation splits into the two chiralities).  Every sigma2 term changes
 *     sign: the y-derivative and the y components of the vector potential.
 */
typedef struct {
    int32_t nx, ny;
    double x_min, x_max, y_min, y_max;
    int32_t bc_x, bc_y;
    double mass, c, charge;
    int32_t krylov_dim;
    int32_t precision;
    double bz;
    int32_t pot_kind;
    double pot_z, pot_a;
    const double *v_table;
    int32_t pulse_kind;
    double pulse_e[2], a0, omega, t_pulse;
    int32_t n_coef;
    const double *coef;
    int32_t chirality;
} dl_params;

/* Per-step statistics (Sec. 4 eq. matrix_exponential_error and its running
 * sum over the steps of one call, Sec. 6).
 * round_bound (DL_PREC_MIXED; 0 in FP64): a bound, in the units of ||psi||,
 * of the part of the step's error that comes from storing the Krylov vectors
 * u_2..u_k in complex64.  The stored vectors obey the Lanczos relation with a
 * perturbation F whose column j is the rounding of u_{j+1} (norm at most
 * e_j = (2^-24 beta_j + 2^-126 sqrt(4 nx ny)) / (1 - 2^-24)); for Hermitian A
 * the difference between ||psi|| Q exp(-iT) e_1 and exp(-iA) psi is then at
 * most the Krylov term plus int_0^1 ||F s(t)|| dt, s(t) = ||psi|| exp(-itT) e_1,
 * so round_bound = sum_j e_j I_j, j = 1..k-1, with I_j >= int_0^1 |s_j(t)| dt:
 * with R the Gershgorin half-width of T about its centre, I_j = 1.01
 * (int_0^1 |s_j|^2 dt)^(1/2) by Gauss-Legendre quadrature with
 * min(48, ceil(R) + 10) points for R <= 40 (Cauchy-Schwarz), ||psi|| [exp(|T - centre|) e_1]_j for 40 < R <= 70,
 * else ||psi||, each capped at ||psi||.  It holds without orthogonality of
 * the basis; the FP64 arithmetic of both precisions is not included.  Summed
 * over the steps it bounds the distance between a mixed-precision and an FP64
 * run beyond their Krylov and FP64 rounding terms. */
typedef struct {
    int32_t k_eff;       /* Krylov dimension used (< m after breakdown, 0 for psi = 0) */
    double err_est;      /* beta_k ||psi|| |e_k^T exp(-iT) e_1| */
    double cum_bound;    /* sum of err_est over the steps of this call so far */
    double norm2;        /* ||psi||^2 after the step (never renormalised) */
    double round_bound;  /* complex64 storage bound of this step (see above) */
} dl_step_stat;

/*
 * Bytes of caller-provided device workspace a context needs.
 * mode DL_MODE_STEP: for step/apply (the stored Krylov basis, m - 1 vectors);
 * DL_MODE_LOWMEM: for step_lowmem/apply (three Krylov vectors);
 * DL_MODE_EIGEN: additionally for eigen() with up to k_eigen Lanczos
 * iterations; DL_MODE_EIGEN_REORTH: additionally for eigen() with full
 * reorthogonalisation and eigen_vectors() with up to k_eigen iterations
 * (k_eigen stored complex128 vectors, about k_eigen * 32 * nx * ny bytes).
 * init accepts the smaller of the STEP and LOWMEM sizes; every
 * call checks the size it needs (DL_ERR_WORKSPACE).  Returns 0 for invalid
 * parameters.  The workspace must be 256-byte aligned.
 */
size_t dirac_lanczos_workspace_bytes(const dl_params *params, int32_t mode, int32_t k_eigen);

/*
 * Validate params, bind the workspace and stream, and create a context.
 * workspace: DEVICE pointer, ws_bytes >= dirac_lanczos_workspace_bytes(params,
 * mode, k) for every mode used later.  hip_stream: hipStream_t (NULL = the
 * default stream).  On success *out receives the context.  The workspace is
 * initialised on the stream.  Errors: DL_ERR_INVALID, DL_ERR_WORKSPACE,
 * DL_ERR_DEVICE (no gfx950 device / HIP failure).  On error *out is NULL.
 */
dl_status dirac_lanczos_init(const dl_params *params, void *workspace, size_t ws_bytes,
                             void *hip_stream, dl_context **out);

/*
 * y = H(t) x (Sec. 3 Hamiltonian, finite differences of Sec. 7) with the
 * instantaneous laser field A_L(t).  x, y: DEVICE spinors (layout above),
 * must not overlap.  Asynchronous on the context's stream.
 */
dl_status dirac_lanczos_apply(dl_context *ctx, const void *x, void *y, double t);

/*
 * n_steps short-time steps psi(t + dt) = exp(-i dt H(t_bar)) psi(t) starting at
 * time t0 (dt may be negative: backward propagation).  Step n uses the exact
 * average of A_L over [t0 + n dt, t0 + (n+1) dt] (first Magnus term).  Each step
 * runs the m-step Lanczos recurrence of Fig. 1 (in an algebraically equal,
 * single-sweep-per-iteration order), the small exponential exp(-iT) e_1
 * (Sec. 4 leaves the method open: a Chebyshev expansion on the vector while
 * the Gershgorin half-width of T shifted to its centre is below about 190,
 * otherwise an eigendecomposition of T by implicit QR), and recombines the
 * Krylov basis (eq. matrix_exp_approx).  psi (DEVICE) is updated in place and
 * never renormalised.
 * stats != NULL (HOST array of n_steps entries): the call returns after the
 * stream has finished the work.  On DL_ERR_NONFINITE psi holds the state
 * after the last completed step and the stats of the completed steps are
 * filled (later entries have k_eff = -1).
 * stats == NULL: the call only enqueues the work on the context's stream and
 * returns; psi holds the result once the stream reaches that point (a
 * non-finite reduction stops the remaining steps on the device, and psi then
 * holds the state after the last completed step).  dirac_lanczos_wait
 * synchronises and reports the outcome and the statistics; a failure not yet
 * reported by it is reported (DL_ERR_NONFINITE, the call doing nothing else)
 * by the next synchronous call on the context.  The per-step fields of an
 * asynchronous call are staged through pinned host buffers the context
 * allocates on first use.
 */
dl_status dirac_lanczos_step(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps,
                             dl_step_stat *stats);

/*
 * Wait for the work of the context's asynchronous step calls (stats == NULL
 * in dirac_lanczos_step, _step_lowmem, _step_ktol) and report the last one:
 * DL_OK, or DL_ERR_NONFINITE if a reduction became non-finite (psi then holds
 * the state after the last completed step).  steps_done (HOST, may be NULL)
 * receives the number of completed steps of the last call.  stats (HOST,
 * n_stats entries, may be NULL with n_stats = 0) receives the statistics of
 * the last call's steps as dirac_lanczos_step would have returned them, for
 * calls of up to 2048 steps (of the last 2048 steps, cum_bound summed from
 * the first of them, for longer calls); entries beyond them have k_eff = -1.
 */
dl_status dirac_lanczos_wait(dl_context *ctx, dl_step_stat *stats, int32_t n_stats, int32_t *steps_done);

/*
 * Adaptive Krylov dimension (Sec. 4: the estimate eq.
 * matrix_exponential_error can steer k): as dirac_lanczos_step, with each step
 * running k in [k_min, krylov_dim] iterations.  The first step of a call uses
 * krylov_dim; every step then predicts the next step's k on the device from
 * its own tridiagonal T: if its estimate exceeded tol, k grows by two;
 * otherwise k becomes the smallest j >= k_min whose estimate
 * beta_j ||psi|| |e_j^T exp(-iT_j) e_1| for the leading j x j block of T is at
 * most tol / 2 (no host round trip per step).  tol bounds the per-step
 * estimate; a step whose spectrum widened past the prediction may exceed it,
 * which stats reports (err_est, and k_eff = the k used).  tol > 0 finite,
 * 1 <= k_min <= krylov_dim (DL_ERR_INVALID).  Workspace as for step.
 */
dl_status dirac_lanczos_step_ktol(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps, double tol,
                                  int32_t k_min, dl_step_stat *stats);

/*
 * Memory-saving variant of dirac_lanczos_step (Sec. 4: instead of storing
 * the Krylov basis, the Lanczos recurrence is run a second time when Q is
 * multiplied by exp(-iT) e_1).  Same arguments and results as
 * dirac_lanczos_step (to rounding of the recombination order); the
 * workspace holds three Krylov vectors instead of m - 1, at the price of
 * m - 1 more sweeps per step.
 */
dl_status dirac_lanczos_step_lowmem(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps,
                                    dl_step_stat *stats);

/*
 * Adaptive time steps (Sec. 4: the error estimate eq.
 * matrix_exponential_error used to adjust the step size).  Propagates psi
 * (DEVICE, in place) from t0 to t_end > t0 with steps of variable size h, each
 * one step of dirac_lanczos_step.  The step's estimate covers both parts of
 * its error:
 *   - the Krylov error of exp(-i h H), by eq. matrix_exponential_error (an
 *     estimate; it tends to overestimate, Sec. 4);
 *   - the replacement of H(s) by its average over the step (the first
 *     Magnus term, Sec. 3, eq. time_evolution_approx), by the bound
 *     c |q| ||psi|| int_t^{t+h} |a(s) - a_bar| ds of the laser field a(s)
 *     (H_bar - H(s) = -c q (a_bar - a(s)) . alpha has that norm on any
 *     spinor, and the propagation is unitary), taken by quadrature on the
 *     host.  It grows like |da/dt| h^2 per step.
 * A step of size h may spend tol * h / (t_end - t0), so the cumulative
 * estimate stays below tol; a step over its share is rejected (psi untouched)
 * and retried smaller; the next h follows from the ratio
 * (share / estimate)^e, e = 1 where the field part dominates and 1/(k-1)
 * otherwise, within [dt_min, dt_max], and the last step ends at t_end
 * exactly.  dt_taken: HOST array of max_steps doubles receiving the accepted
 * sizes, or NULL.  out (HOST) receives the counts, the time reached, the next
 * dt, the cumulative estimate (cum_bound), its field part (cum_magnus) and
 * ||psi||^2.  Errors: DL_ERR_INVALID (arguments; or max_steps exhausted / tol
 * needing dt < dt_min: psi then holds the state at out->t_reached),
 * DL_ERR_NONFINITE, DL_ERR_DEVICE.  Synchronous.
 */
typedef struct {
    int32_t accepted, rejected;
    double t_reached, dt_next, cum_bound, norm2, cum_magnus;
} dl_adapt_stat;

dl_status dirac_lanczos_step_adaptive(dl_context *ctx, void *psi, double t0, double t_end, double dt_init,
                                      double tol, double dt_min, double dt_max, int32_t max_steps,
                                      double *dt_taken, dl_adapt_stat *out);

/*
 * Eigenvalue mode (Sec. 2 eq. A_approx, eq. error_est; Sec. 5): k_max
 * Lanczos iterations on H (static fields, laser off) from psi0 (DEVICE).
 * Ritz values of T in [e_lo, e_hi] are grouped into clusters of neighbours
 * closer than tol; a cluster whose bound beta_k ||last components of its
 * eigenvectors|| is <= tol is reported as its mean.  Up to n_wanted values go
 * to evals/bounds (HOST arrays of n_wanted doubles), ascending; *n_found
 * receives the count.  reorth == 0: the plain three-term recurrence in the
 * fused sweep order, three rolling vectors, a workspace sized for
 * DL_MODE_EIGEN with k_eigen >= k_max; converged clusters are accumulated
 * over the leading blocks T_k, k = 64, 128, ... and the last k: once
 * orthogonality is lost a converged value acquires copies whose eigenvectors
 * of T mix with its own and its bound can grow again, while the value stays
 * within its earlier bound of an eigenvalue of H (Paige); values closer than
 * tol are one eigenvalue and keep their smallest bound; the call stops at
 * the first checkpoint with n_wanted values and reports the lowest n_wanted.
 * reorth != 0: full
 * reorthogonalisation applied twice (Sec. 2), as classical Gram-Schmidt
 * against all stored vectors (h = Q^H z, z -= Q h, two passes; the first
 * pass also removes the alpha_i q_i and beta_{i-1} q_{i-1} terms of the
 * recurrence, alpha_i = Re h_i of that pass), a workspace sized for
 * DL_MODE_EIGEN_REORTH with k_eigen >= k_max; every 64 iterations the
 * Ritz values of the current T are computed on the host, and the recurrence
 * stops early once n_wanted clusters have converged (the values are then
 * those of that T); otherwise it runs k_max iterations.  A start vector of
 * norm 0 reports nothing; a breakdown (beta_i <= 1e-13 max(|alpha_j|,
 * beta_{j-1})) ends the recurrence at k = i.  DL_ERR_NONFINITE for a
 * non-finite reduction.  Synchronous.
 */
dl_status dirac_lanczos_eigen(dl_context *ctx, const void *psi0, int32_t k_max, int32_t reorth,
                              double e_lo, double e_hi, double tol, int32_t n_wanted,
                              double *evals, double *bounds, int32_t *n_found);

/*
 * The host half of the eigen modes, for a recurrence the caller already has
 * (Sec. 2 eq. error_est): the converged Ritz clusters of the tridiagonal T_k
 * with diagonal alpha[0..k) and off-diagonal beta[0..k-1), bound factor
 * beta[k-1] = beta_k (the norm of the next residual), all HOST arrays.  With
 * check_every > 0 the clusters of the leading blocks T_j, j = check_every,
 * 2 check_every, ... and k, are accumulated as in dirac_lanczos_eigen with
 * reorth = 0; with check_every == 0 only T_k is taken.  Eigenvalues of a block
 * in (e_lo, e_hi] come from bisection on Sturm counts to full precision, the
 * last eigenvector components from inverse iteration, vectors of eigenvalues
 * closer than max(tol, 1e-8 ||T||) kept orthogonal.  Up to n_wanted values
 * (the lowest) go to evals/bounds, ascending; *n_found receives the count.
 * Blocks are solved on up to 16 host threads.  DL_ERR_INVALID for k < 1,
 * check_every < 0, n_wanted < 1, e_hi < e_lo, tol < 0 or null pointers.
 * Needs no device.
 */
dl_status dirac_lanczos_ritz(const double *alpha, const double *beta, int32_t k, double e_lo, double e_hi,
                             double tol, int32_t check_every, int32_t n_wanted, double *evals, double *bounds,
                             int32_t *n_found);

/*
 * Ritz vectors (Sec. 2 eq. eigenvec_approx): dirac_lanczos_eigen with
 * reorth != 0, plus for every reported value the Ritz vector y = Q_k t, t the
 * eigenvector of T_k of the cluster member with the smallest bound
 * |beta_k t_k|.  With the stored vectors orthonormal, ||y|| = 1 and
 * ||H y - theta y|| = |beta_k t_k| (eq. error_est) up to rounding.  The sign
 * of t makes <psi0, y> real and positive (a Ritz vector of a simple value is
 * unique up to that sign).  vecs: DEVICE, n_wanted vectors of 2 * nx * ny
 * complex128 in the state layout, vector i at vecs + i * 32 * nx * ny bytes;
 * only the first *n_found are written.  Workspace as for reorth != 0.
 * Synchronous.
 */
dl_status dirac_lanczos_eigen_vectors(dl_context *ctx, const void *psi0, int32_t k_max, double e_lo,
                                      double e_hi, double tol, int32_t n_wanted, double *evals,
                                      double *bounds, int32_t *n_found, void *vecs);

/*
 * Adjoint (gradient) mode: the derivative of a final observable with respect
 * to the coefficients of the DL_PULSE_FOURIER_SIN2 laser field.  This extends
 * the paper (whose method is the forward propagator of Sec. 4 and the
 * eigenvalue mode of Sec. 5): the forward map is the same chain of short-time
 * steps, each U_n = exp(-i dt H(A_n)) with the step-averaged field A_n
 * (Sec. 3, first Magnus term).
 *
 * Loss: L = sum of the expectation values selected by loss_kind (bit flags
 * DL_LOSS_X, DL_LOSS_Y, DL_LOSS_PX, DL_LOSS_PY) in the final state psi_N,
 * each <psi_N|O|psi_N> / <psi_N|psi_N>, with x, y the grid coordinates and
 * p = -i d/dx by the central differences of the Hamiltonian.
 * Gradient: dL/dcoef_j = sum_n 2 Re <lam_{n+1}| dU_n/dcoef_j |psi_n> with
 * lam_N = (O - L) psi_N / <psi_N|psi_N> and lam_n = U_n^dagger lam_{n+1}
 * (a step with -dt at the same field).  dU_n/dA is the Frechet derivative of
 * the matrix exponential, evaluated in the eigenbases of the two Krylov
 * spaces of step n (the forward one of psi_n and the backward one of
 * lam_{n+1}), with the divided difference of exp(-i .) between their Ritz
 * values.  States psi_n are stored every ckpt_every steps during the forward
 * pass and recomputed segment by segment during the backward pass.  When the
 * forward Krylov bases of one segment (ckpt_every * (krylov_dim - 1)
 * vectors) fit in 32 GiB, the workspace also holds them, and the backward
 * pass uses the bases of the recomputation instead of building them again
 * (the same result, bit for bit; the workspace size reflects the choice).
 *
 * Requirements: precision DL_PREC_FP64, krylov_dim <= 16, pulse_kind
 * DL_PULSE_FOURIER_SIN2, loss_kind in 1..15, n_steps >= 1, ckpt_every >= 1,
 * dt > 0.  adj_ws: DEVICE, 256-byte aligned, adj_bytes >=
 * dirac_lanczos_adjoint_workspace_bytes(params, n_steps, ckpt_every): the
 * checkpoints and, while they fit in 32 GiB, the forward Krylov bases and
 * states of the last segments, which the backward pass then does not
 * recompute (otherwise the context's own workspace holds the forward basis).
 * psi0 (DEVICE) is read only.  loss (HOST, 1 double) receives L, grad (HOST,
 * n_coef doubles) the gradient in the order of params->coef.  Synchronous.
 * Errors: DL_ERR_INVALID, DL_ERR_WORKSPACE, DL_ERR_UNSUPPORTED (other
 * precision/pulse/krylov_dim), DL_ERR_NONFINITE, DL_ERR_DEVICE.
 */
enum { DL_LOSS_X = 1, DL_LOSS_Y = 2, DL_LOSS_PX = 4, DL_LOSS_PY = 8 };

size_t dirac_lanczos_adjoint_workspace_bytes(const dl_params *params, int32_t n_steps,
                                             int32_t ckpt_every);

dl_status dirac_lanczos_adjoint(dl_context *ctx, const void *psi0, double t0, double dt,
                                int32_t n_steps, int32_t ckpt_every, int32_t loss_kind,
                                void *adj_ws, size_t adj_bytes, double *loss, double *grad);

/*
 * Batches of independent packets (hundreds of small
 * grids of different sizes and fields propagated together).  Each packet is
 * described by its own dl_params (grid, box, boundaries, fields, pulse); all
 * packets share krylov_dim, precision and bc_y.  One step of the batch is one
 * launch per Lanczos iteration over all packets (plus the small exponentials
 * and the recombination), with every packet's reductions folded separately
 * in fixed order; the mathematics of each packet is that of
 * dirac_lanczos_step.
 *
 * dirac_lanczos_batch_workspace_bytes: bytes of DEVICE workspace (256-byte
 *   aligned) for the batch; 0 for invalid parameters.
 * dirac_lanczos_batch_init: params is a HOST array of n_packets entries (their
 *   coef arrays are copied; v_table pointers must stay valid).  Errors:
 *   DL_ERR_INVALID, DL_ERR_UNSUPPORTED (packets differ in bc_y),
 *   DL_ERR_WORKSPACE, DL_ERR_DEVICE.
 * dirac_lanczos_batch_step: psi is a HOST array of n_packets DEVICE pointers
 *   (spinor layout above, updated in place); stats is a HOST array of
 *   n_packets * n_steps entries (packet-major) or NULL.  Synchronous.  A
 *   packet whose reduction becomes non-finite stops (its psi holds its last
 *   completed step, later stats have k_eff = -1) while the others continue;
 *   the call then returns DL_ERR_NONFINITE naming the packets.  Calls on one
 *   batch must not overlap (they share its tables and reduction scratch).
 */
typedef struct dl_batch dl_batch;

size_t dirac_lanczos_batch_workspace_bytes(const dl_params *params, int32_t n_packets);
dl_status dirac_lanczos_batch_init(const dl_params *params, int32_t n_packets, void *workspace,
                                   size_t ws_bytes, void *hip_stream, dl_batch **out);
dl_status dirac_lanczos_batch_step(dl_batch *batch, void *const *psi, double t0, double dt,
                                   int32_t n_steps, dl_step_stat *stats);
dl_status dirac_lanczos_batch_destroy(dl_batch *batch);
/* Message of the last failing call on batch, or of the last failing
 * batch_init on this thread when batch is NULL. */
const char *dirac_lanczos_batch_last_error(const dl_batch *batch);

/*
 * Hermite pseudospectral discretisation (Sec. 5): each spinor component is
 * represented by its values at the n x n collocation points (x_i, y_j),
 * x_i = scale * xi_i with xi_i the roots of the n-th Hermite polynomial (the
 * span of the products of the first n Hermite functions; the wave function
 * vanishes at infinity), and the derivatives by dense n x n matrices.
 * Spinors are DEVICE arrays of 2 n^2 complex128 in the layout (2, n, n), x
 * fastest, of the variables phi_ij = sqrt(w_i w_j) psi(x_i, y_j) with w the
 * weights of dirac_lanczos_hermite_nodes, so that the Euclidean norm is the
 * L^2 norm; in them the derivative D~_ij = (-1)^(i+j) / (x_i - x_j) (i != j,
 * zero diagonal) is antisymmetric and H = c [sigma1 (p_x - q A_x) +
 * chi sigma2 (p_y - q A_y)] + sigma3 m c^2 + V, p = -i D~ along each axis,
 * A = (B/2)(-y, x), is Hermitian.  V as in dl_params (pot_kind 0, 1 or 2).
 * n is 16, 32, 48 or 64.  The matrix products run on the FP64 matrix cores.
 */
typedef struct {
    int32_t n;          /* collocation points per axis */
    double scale;       /* length scale of the Hermite functions */
    double mass, c, charge;
    double bz;          /* uniform B_z, symmetric gauge about the origin */
    int32_t pot_kind;
    double pot_z, pot_a;
    int32_t chirality;  /* as dl_params */
} dl_hermite_params;

/* HOST: the n collocation points x (ascending, times scale) and weights w
 * (Christoffel numbers of the Hermite functions, times scale: sum_i w_i f(x_i)
 * integrates f exactly on products of the first n Hermite functions). */
dl_status dirac_lanczos_hermite_nodes(int32_t n, double scale, double *x, double *w);

/* Bytes of DEVICE workspace (256-byte aligned) for n_problems problems and up
 * to k_max Lanczos iterations (0 for invalid parameters). */
size_t dirac_lanczos_hermite_workspace_bytes(const dl_hermite_params *params, int32_t n_problems, int32_t k_max);

/* y = H x for one problem (x, y DEVICE spinors, distinct); the workspace is
 * sized for (params, 1, 1).  Synchronous on hip_stream. */
dl_status dirac_lanczos_hermite_apply(const dl_hermite_params *params, const void *x, void *y, void *workspace,
                                      size_t ws_bytes, void *hip_stream);

/* Eigenvalue mode for a batch of problems (Sec. 2, Sec. 5): k_max
 * iterations of the plain Lanczos recurrence of Fig. 1 from psi0[i] (HOST
 * array of DEVICE start vectors), one workgroup per problem and all
 * iterations in one launch; then, per problem, the converged Ritz clusters
 * of the leading blocks T_k, k = 64, 128, ... and k_max, in [e_lo[i],
 * e_hi[i]] with bound <= tol, accumulated as in dirac_lanczos_eigen with
 * reorth = 0.  evals/bounds: HOST arrays of n_problems * n_wanted (problem i
 * at offset i * n_wanted, ascending), n_found: HOST array of n_problems.  A
 * start vector of norm 0 reports nothing.  Errors: DL_ERR_INVALID,
 * DL_ERR_WORKSPACE, DL_ERR_NONFINITE (a reduction of some problem became
 * non-finite; the others are reported), DL_ERR_DEVICE.  Synchronous. */
dl_status dirac_lanczos_hermite_eigen(const dl_hermite_params *params, int32_t n_problems, const void *const *psi0,
                                      int32_t k_max, const double *e_lo, const double *e_hi, double tol,
                                      int32_t n_wanted, void *workspace, size_t ws_bytes, void *hip_stream,
                                      double *evals, double *bounds, int32_t *n_found);

/* Message of the last failing Hermite call on this thread ("" if none). */
const char *dirac_lanczos_hermite_last_error(void);

/*
 * Launch shape (tuning; results are equal to rounding for every shape).
 * dirac_lanczos_set_launch: at most sweep_waves_per_cu waves per compute unit
 *   in the Lanczos sweeps (0: the built-in default, floor(strips * ny /
 *   (24 * compute units)) within 2..8, i.e. row chunks of at least 24 rows
 *   where the grid allows); the row chunks are re-planned for one resident
 *   round of waves.  *waves_out (HOST, may
 *   be NULL) receives the value in use (capped by occupancy).
 * dirac_lanczos_batch_set_launch: rows per chunk of the batched sweeps
 *   (>= 4; 0: the default choice, the smallest power of two giving at most
 *   one resident round of waves).  *rows_out (HOST, may be NULL) receives it.
 * The autotuner of the Python package times candidates and caches the best.
 */
dl_status dirac_lanczos_set_launch(dl_context *ctx, int32_t sweep_waves_per_cu, int32_t *waves_out);
dl_status dirac_lanczos_batch_set_launch(dl_batch *batch, int32_t rows_per_chunk, int32_t *rows_out);

/*
 * Kernel timing with HIP events recorded on the context's stream around every
 * launch of dirac_lanczos_step (a diagnostic for roofline measurements).
 * Classes: 0 first Lanczos iteration; 1 recurrence sweeps whose operands are
 * all Krylov vectors (iterations >= 4, each reads u_{p-1}, u_{p-2} and writes
 * u_p); 2 recurrence sweeps that read psi (iterations 2 and 3); 3 tridiagonal
 * exponential; 4 recombination.
 * enable = 1 clears the accumulators and starts recording, enable = 0 stops.
 * out (HOST, may be NULL) receives the accumulated counts and milliseconds;
 * reading them waits for the recorded events.
 */
typedef struct {
    int64_t launches[5];
    double total_ms[5];
} dl_timing;

dl_status dirac_lanczos_timing(dl_context *ctx, int32_t enable, dl_timing *out);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): n_steps steps of
 * dirac_lanczos_step for the problem `params`, on hip_stream (NULL: the
 * default stream), without a context or a caller workspace.  The workspace of
 * the step lives in a static device array of 64 MiB that every GPU the
 * library runs on holds until the process ends; the problem must fit it
 * (dirac_lanczos_workspace_bytes(params, DL_MODE_STEP, 0) <= 64 MiB: about
 * 350^2 sites in FP64 or 490^2 in mixed precision at m = 16), otherwise
 * DL_ERR_WORKSPACE before any device work.  The call allocates nothing on the
 * device or the host.  Calls on one GPU share that array: calls that overlap
 * in time on a GPU (from several threads or streams) race; sequential calls
 * are independent (each starts from zeroed scalars).  params->coef is read
 * during the call only.  psi (DEVICE) as for dirac_lanczos_step.
 * stats != NULL (HOST, n_steps entries): synchronous, statistics and
 * DL_ERR_NONFINITE as for dirac_lanczos_step.  stats == NULL: the work is only
 * enqueued (kernels only, no host copies), and a non-finite reduction is not
 * reported.  Errors: DL_ERR_INVALID, DL_ERR_WORKSPACE, DL_ERR_DEVICE (no
 * gfx950 device, or a HIP failure); no message is kept.
 */
dl_status dirac_lanczos_step_noalloc(const dl_params *params, void *psi, double t0, double dt, int32_t n_steps,
                                     void *hip_stream, dl_step_stat *stats);

/* Free the host context (the caller frees its own device buffers). */
dl_status dirac_lanczos_destroy(dl_context *ctx);

/* Message of the last failing call on ctx (never NULL; "" if none). */
const char *dirac_lanczos_last_error(const dl_context *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DIRAC_LANCZOS_H */
