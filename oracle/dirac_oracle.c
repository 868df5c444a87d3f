/*
 * dirac_oracle.c -- plain CPU FP64 reference of the Lanczos short-time
 * propagator for the two-dimensional Dirac equation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the GPU library and must never be called from the product path.
 *
 * Everything is double precision, plain loops, no blocking or fusion, built
 * with -O2 -ffp-contract=off.  Each function names the passage of Beerwerth &
 * Bauke, "Krylov subspace methods for the Dirac equation" (arXiv:1407.7370)
 * that it follows:
 *
 *   orc_apply_h       Sec. 3, Dirac Hamiltonian H(t) with the 2D Pauli
 *                     representation alpha1=sigma1, alpha2=sigma2, beta=sigma3
 *                     (or alpha2=-sigma2: the other chirality, Sec. 3);
 *                     Sec. 7, derivatives by first-order (central) finite
 *                     differences on a rectangular grid.
 *   orc_field_average Sec. 3, eq. time_evolution_approx: first Magnus term,
 *                     i.e. the time integral of H over one step.
 *   orc_lanczos       Sec. 2, Fig. 1 (Lanczos in Paige's modified
 *                     Gram-Schmidt order), plus full reorthogonalisation
 *                     applied twice (Sec. 2) for the eigenvalue mode.
 *   orc_tridiag_eig   Sec. 4: exp(-iT) via an eigendecomposition of the
 *                     tridiagonal T (here: cyclic Jacobi).
 *   orc_expm_e1       Sec. 4, eq. matrix_exp_approx.
 *   orc_propagate     Sec. 4, eq. matrix_exp_approx, error estimate
 *                     eq. matrix_exponential_error and its cumulative sum
 *                     (Sec. 6).
 *   orc_lanczos_plain Sec. 2, the same recurrence with three stored vectors
 *                     (no reorthogonalisation; eigenvalue mode at scale).
 *   orc_eigen         Sec. 2, Ritz values and bound eq. error_est; Sec. 5.
 *   orc_eigen_vectors Sec. 2 eq. eigenvec_approx (Ritz vectors, full reorth).
 *   orc_hermite_*     Sec. 5, Hermite pseudospectral discretisation: collocation
 *                     at the roots of the N-th Hermite polynomial, dense
 *                     differentiation matrices.
 *
 * Readings where the paper is silent (shared with the GPU library only as
 * written conventions, never as code):
 *   - first-order finite differences (Sec. 7) = central first-derivative
 *     differences (f[j+1]-f[j-1])/(2h), the 3-point form that keeps -iD
 *     Hermitian (Hermiticity is required in Sec. 4 and Sec. 8).
 *   - grid x_i = x_min + i*h, h = (x_max-x_min)/n; Dirichlet boundaries mean
 *     psi = 0 outside the grid, periodic boundaries wrap.
 *   - vector potential couples pointwise: A(x) multiplies the spinor.
 *     Uniform B_z enters in the symmetric gauge A = (B/2)(-y, x).
 *   - the potential term of H is the potential energy V = q*phi.
 *   - alpha_i = Re(q_i . z) (the imaginary part is rounding only).
 *   - beta_k = ||z - alpha_k q_k|| after the loop (error estimate input).
 *   - breakdown: if beta_i <= 1e-13 * max_{j<=i}(|alpha_j|, beta_{j-1})
 *     the recurrence stops with k_eff = i (the subspace is invariant).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Physical problem; mirrored field by field by oracle/__init__.py. */
typedef struct {
    int32_t nx, ny;
    double x_min, x_max, y_min, y_max;
    int32_t bc_x, bc_y;          /* 0 Dirichlet, 1 periodic */
    double mass, c, charge;
    double bz;                   /* uniform magnetic field, symmetric gauge */
    int32_t pot_kind;            /* 0 none, 1 -Z/sqrt(r^2+a^2), 2 soft-core of eq. soft_core_pot */
    double pot_z, pot_a;
    const double *v_table;       /* optional [ny][nx] potential energy (host) */
    int32_t pulse_kind;          /* 0 none, 1 A0 sin(wt) sin^2(pi t/T) e, 2 Fourier series * sin^2 */
    double pulse_e[2], a0, omega, t_pulse;
    int32_t n_coef;
    const double *coef;          /* kind 2: for k=1..n/4: a_k^x, b_k^x, a_k^y, b_k^y */
    int32_t chirality;           /* -1: alpha2 = -sigma2 (the other 2D representation); else +sigma2 */
} orc_params;

typedef struct {
    int32_t k_eff;
    double err_est, cum_bound, norm2;
} orc_stat;

/* ------------------------------------------------------------------------ */
/* Pauli matrices: the 2D representation alpha1 = sigma1, alpha2 = sigma2,   */
/* beta = sigma3 (Sec. 3).                                                   */
/* ------------------------------------------------------------------------ */
static void pauli(int which, cplx s[2][2])
{
    if (which == 1) {
        s[0][0] = 0; s[0][1] = 1; s[1][0] = 1; s[1][1] = 0;
    } else if (which == 2) {
        s[0][0] = 0; s[0][1] = -I; s[1][0] = I; s[1][1] = 0;
    } else {
        s[0][0] = 1; s[0][1] = 0; s[1][0] = 0; s[1][1] = -1;
    }
}

/* Exposed so a test can check the Dirac algebra of eq.
 * dirac_matrices_conditions on the matrices the oracle actually uses.
 * out = 8 doubles (re, im of s00, s01, s10, s11). */
void orc_pauli(int which, double *out)
{
    cplx s[2][2];
    pauli(which, s);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            out[2 * (2 * a + b)] = creal(s[a][b]);
            out[2 * (2 * a + b) + 1] = cimag(s[a][b]);
        }
}

static double grid_h(double lo, double hi, int n) { return (hi - lo) / n; }

/* Potential energy V(x, y) at grid site (i, j). */
static double potential(const orc_params *p, int i, int j, double x, double y)
{
    double v = 0.0;
    if (p->pot_kind == 1) {
        v = -p->pot_z / sqrt(x * x + y * y + p->pot_a * p->pot_a);
    } else if (p->pot_kind == 2) {
        /* eq. soft_core_pot in atomic units: -(3/2) Z / sqrt(r^2 + 3/Z^2) */
        v = -1.5 * p->pot_z / sqrt(x * x + y * y + 3.0 / (p->pot_z * p->pot_z));
    }
    if (p->v_table) v += p->v_table[(size_t)j * p->nx + i];
    return v;
}

/* Spinor component s at grid site (i, j), honouring the boundary reading. */
static cplx site(const orc_params *p, const cplx *v, int s, int i, int j)
{
    if (i < 0 || i >= p->nx) {
        if (!p->bc_x) return 0;
        i = ((i % p->nx) + p->nx) % p->nx;
    }
    if (j < 0 || j >= p->ny) {
        if (!p->bc_y) return 0;
        j = ((j % p->ny) + p->ny) % p->ny;
    }
    return v[((size_t)s * p->ny + j) * p->nx + i];
}

/*
 * out = H in, with the vector potential A = A_B(x, y) + a_hom and the static
 * scalar potential (Sec. 3, Hamiltonian H(t); Sec. 7, finite differences):
 *   H = c [sigma1 (p_x - q A_x) + sigma2 (p_y - q A_y)] + sigma3 m c^2 + V,
 *   p_x = -i d/dx realised as -i (f[i+1] - f[i-1]) / (2 h_x).
 */
void orc_apply_h(const orc_params *p, const double *a_hom, const double *in_d, double *out_d)
{
    const cplx *in = (const cplx *)in_d;
    cplx *out = (cplx *)out_d;
    const double hx = grid_h(p->x_min, p->x_max, p->nx);
    const double hy = grid_h(p->y_min, p->y_max, p->ny);
    const double mc2 = p->mass * p->c * p->c;
    cplx s1[2][2], s2[2][2], s3[2][2];
    pauli(1, s1);
    pauli(2, s2);
    pauli(3, s3);
    /* alpha2 = chi sigma2 */
    const double chi = p->chirality < 0 ? -1.0 : 1.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s2[a][b] *= chi;
    for (int j = 0; j < p->ny; ++j) {
        const double y = p->y_min + j * hy;
        for (int i = 0; i < p->nx; ++i) {
            const double x = p->x_min + i * hx;
            const double v = potential(p, i, j, x, y);
            const double ax = -0.5 * p->bz * y + a_hom[0];
            const double ay = 0.5 * p->bz * x + a_hom[1];
            cplx psi[2], pix[2], piy[2];
            for (int s = 0; s < 2; ++s) {
                psi[s] = site(p, in, s, i, j);
                const cplx dx = (site(p, in, s, i + 1, j) - site(p, in, s, i - 1, j)) / (2.0 * hx);
                const cplx dy = (site(p, in, s, i, j + 1) - site(p, in, s, i, j - 1)) / (2.0 * hy);
                pix[s] = -I * dx - p->charge * ax * psi[s];
                piy[s] = -I * dy - p->charge * ay * psi[s];
            }
            for (int a = 0; a < 2; ++a) {
                cplx acc = v * psi[a];
                for (int b = 0; b < 2; ++b)
                    acc += p->c * (s1[a][b] * pix[b] + s2[a][b] * piy[b]) + mc2 * s3[a][b] * psi[b];
                out[((size_t)a * p->ny + j) * p->nx + i] = acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Homogeneous laser vector potential A_L(t) and its step average.           */
/* ------------------------------------------------------------------------ */
void orc_pulse(const orc_params *p, double t, double *a)
{
    a[0] = a[1] = 0.0;
    if (p->pulse_kind == 0 || t < 0.0 || t > p->t_pulse) return;
    const double env = sin(M_PI * t / p->t_pulse);
    const double env2 = env * env;
    if (p->pulse_kind == 1) {
        const double f = p->a0 * sin(p->omega * t) * env2;
        a[0] = f * p->pulse_e[0];
        a[1] = f * p->pulse_e[1];
    } else if (p->pulse_kind == 2) {
        const double w0 = 2.0 * M_PI / p->t_pulse;
        for (int k = 1; 4 * k <= p->n_coef; ++k) {
            const double sk = sin(k * w0 * t), ck = cos(k * w0 * t);
            a[0] += p->coef[4 * (k - 1) + 0] * sk + p->coef[4 * (k - 1) + 1] * ck;
            a[1] += p->coef[4 * (k - 1) + 2] * sk + p->coef[4 * (k - 1) + 3] * ck;
        }
        a[0] *= env2;
        a[1] *= env2;
    }
}

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n. */
#define ORC_GL 12
static void gauss_legendre(double *x, double *w)
{
    for (int k = 0; k < ORC_GL; ++k) {
        double z = cos(M_PI * (k + 0.75) / (ORC_GL + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int n = 1; n <= ORC_GL; ++n) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p2) / n;
            }
            dp = ORC_GL * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/*
 * Step average (1/dt) * integral_{t0}^{t0+dt} A_L(t) dt, the first Magnus
 * term of eq. time_evolution_approx restricted to the (only) time-dependent
 * part of H.  The integral is evaluated by Gauss-Legendre quadrature on the
 * part of the step where the pulse is on.
 */
void orc_field_average(const orc_params *p, double t0, double dt, double *a)
{
    a[0] = a[1] = 0.0;
    if (p->pulse_kind == 0) return;
    double lo = t0 < t0 + dt ? t0 : t0 + dt;
    double hi = t0 < t0 + dt ? t0 + dt : t0;
    if (lo < 0.0) lo = 0.0;
    if (hi > p->t_pulse) hi = p->t_pulse;
    if (hi <= lo) return;
    double x[ORC_GL], w[ORC_GL];
    gauss_legendre(x, w);
    const double mid = 0.5 * (hi + lo), half = 0.5 * (hi - lo);
    for (int k = 0; k < ORC_GL; ++k) {
        double ak[2];
        orc_pulse(p, mid + half * x[k], ak);
        a[0] += w[k] * half * ak[0];
        a[1] += w[k] * half * ak[1];
    }
    a[0] /= fabs(dt);
    a[1] /= fabs(dt);
}

/* ------------------------------------------------------------------------ */
/* Vector helpers (N complex entries).                                        */
/* ------------------------------------------------------------------------ */
static cplx vdot(size_t n, const cplx *u, const cplx *v)
{
    cplx s = 0;
    for (size_t k = 0; k < n; ++k) s += conj(u[k]) * v[k];
    return s;
}

static double vnorm(size_t n, const cplx *u) { return sqrt(creal(vdot(n, u, u))); }

/* out = dt * H in  (the Hermitian matrix A of Sec. 4). */
static void apply_a(const orc_params *p, const double *a_hom, double dt, const cplx *in, cplx *out)
{
    orc_apply_h(p, a_hom, (const double *)in, (double *)out);
    const size_t n = (size_t)2 * p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) out[k] *= dt;
}

/*
 * Lanczos algorithm of Fig. 1 on A = dt * H(a_hom), start vector b:
 *   q1 = b/||b||; z = A q1
 *   for i = 1..k-1:  alpha_i = q_i.z;  z -= alpha_i q_i;  beta_i = ||z||;
 *                    q_{i+1} = z / beta_i;  z = A q_{i+1} - beta_i q_i
 *   alpha_k = q_k.z
 * followed by beta_k = ||z - alpha_k q_k|| for the error estimate.
 * reorth != 0 additionally orthogonalises z against all previous q, twice
 * (full reorthogonalisation, Sec. 2).
 * Q receives k vectors of n = 2*nx*ny complex values.  Returns k_eff
 * (0 for b = 0).  alpha[0..k_eff-1], beta[0..k_eff-1].
 */
int orc_lanczos(const orc_params *p, const double *a_hom, double dt, const double *b_d, int k,
                int reorth, double *q_d, double *alpha, double *beta)
{
    const size_t n = (size_t)2 * p->nx * p->ny;
    const cplx *b = (const cplx *)b_d;
    cplx *Q = (cplx *)q_d;
    const double nb = vnorm(n, b);
    if (nb == 0.0) return 0;
    cplx *z = (cplx *)malloc(n * sizeof(cplx));
    for (size_t t = 0; t < n; ++t) Q[t] = b[t] / nb;
    apply_a(p, a_hom, dt, Q, z);
    double scale = 0.0;
    int keff = k;
    for (int i = 1; i <= k; ++i) {
        cplx *qi = Q + (size_t)(i - 1) * n;
        alpha[i - 1] = creal(vdot(n, qi, z));
        for (size_t t = 0; t < n; ++t) z[t] -= alpha[i - 1] * qi[t];
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 1; j <= i; ++j) {
                    const cplx *qj = Q + (size_t)(j - 1) * n;
                    const cplx h = vdot(n, qj, z);
                    for (size_t t = 0; t < n; ++t) z[t] -= h * qj[t];
                }
        }
        beta[i - 1] = vnorm(n, z);
        if (fabs(alpha[i - 1]) > scale) scale = fabs(alpha[i - 1]);
        if (i > 1 && beta[i - 2] > scale) scale = beta[i - 2];
        if (i == k) break;
        if (beta[i - 1] <= 1e-13 * scale) {
            keff = i;
            break;
        }
        cplx *qn = Q + (size_t)i * n;
        for (size_t t = 0; t < n; ++t) qn[t] = z[t] / beta[i - 1];
        apply_a(p, a_hom, dt, qn, z);
        for (size_t t = 0; t < n; ++t) z[t] -= beta[i - 1] * qi[t];
    }
    free(z);
    return keff;
}

/* An operator out = Op in on vectors of n complex entries. */
typedef void (*orc_op)(const void *ctx, const cplx *in, cplx *out);

/*
 * Plain Lanczos recurrence with three stored vectors (Sec. 2: without
 * reorthogonalisation only q_{i-1}, q_i and z are needed; the Ritz values
 * follow from alpha and beta alone).  The loop is the one of orc_lanczos with
 * reorth = 0 -- the same operations in the same order -- so alpha and beta
 * agree with it bit for bit; only the storage differs.  Returns k_eff (0 for
 * b = 0); alpha[0..k_eff-1], beta[0..k_eff-1] (beta[k_eff-1] is
 * ||z - alpha_k q_k|| after the last iteration, the input of eq. error_est).
 */
static int lanczos3(size_t n, orc_op op, const void *ctx, const cplx *b, int k, double *alpha, double *beta)
{
    const double nb = vnorm(n, b);
    if (nb == 0.0) return 0;
    cplx *qprev = (cplx *)malloc(n * sizeof(cplx));
    cplx *qcur = (cplx *)malloc(n * sizeof(cplx));
    cplx *z = (cplx *)malloc(n * sizeof(cplx));
    for (size_t t = 0; t < n; ++t) qcur[t] = b[t] / nb;
    op(ctx, qcur, z);
    double scale = 0.0;
    int keff = k;
    for (int i = 1; i <= k; ++i) {
        alpha[i - 1] = creal(vdot(n, qcur, z));
        for (size_t t = 0; t < n; ++t) z[t] -= alpha[i - 1] * qcur[t];
        beta[i - 1] = vnorm(n, z);
        if (fabs(alpha[i - 1]) > scale) scale = fabs(alpha[i - 1]);
        if (i > 1 && beta[i - 2] > scale) scale = beta[i - 2];
        if (i == k) break;
        if (beta[i - 1] <= 1e-13 * scale) {
            keff = i;
            break;
        }
        /* q_{i+1} = z / beta_i replaces q_{i-1}; z = A q_{i+1} - beta_i q_i */
        cplx *qn = qprev;
        for (size_t t = 0; t < n; ++t) qn[t] = z[t] / beta[i - 1];
        op(ctx, qn, z);
        for (size_t t = 0; t < n; ++t) z[t] -= beta[i - 1] * qcur[t];
        qprev = qcur;
        qcur = qn;
    }
    free(qprev);
    free(qcur);
    free(z);
    return keff;
}

typedef struct {
    const orc_params *p;
    const double *a_hom;
    double dt;
} fd_op_ctx;

static void fd_op(const void *ctx, const cplx *in, cplx *out)
{
    const fd_op_ctx *c = (const fd_op_ctx *)ctx;
    apply_a(c->p, c->a_hom, c->dt, in, out);
}

/* The finite-difference A = dt H of orc_lanczos with three stored vectors. */
int orc_lanczos_plain(const orc_params *p, const double *a_hom, double dt, const double *b_d, int k,
                      double *alpha, double *beta)
{
    const fd_op_ctx ctx = {p, a_hom, dt};
    return lanczos3((size_t)2 * p->nx * p->ny, fd_op, &ctx, (const cplx *)b_d, k, alpha, beta);
}

/*
 * Eigendecomposition of the symmetric tridiagonal T (diag alpha, off-diagonal
 * beta) by the cyclic Jacobi method: evals[k], evecs[k*k] row-major with
 * column l the eigenvector of evals[l].
 */
void orc_tridiag_eig(int k, const double *alpha, const double *beta, double *evals, double *evecs)
{
    /* a is the full symmetric matrix; only rows are touched in the rotation
     * loops and symmetry is restored by copying row entries to the columns. */
    double *a = (double *)calloc((size_t)k * k, sizeof(double));
    /* vt holds the transpose of the eigenvector matrix: row l = vector l */
    double *vt = (double *)calloc((size_t)k * k, sizeof(double));
    for (int i = 0; i < k; ++i) {
        a[i * k + i] = alpha[i];
        if (i + 1 < k) a[i * k + i + 1] = a[(i + 1) * k + i] = beta[i];
        vt[i * k + i] = 1.0;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < k; ++r)
            for (int s = 0; s < k; ++s) {
                tot += a[r * k + s] * a[r * k + s];
                if (r != s) off += a[r * k + s] * a[r * k + s];
            }
        if (off <= 1e-36 * tot || off == 0.0) break;
        for (int r = 0; r < k - 1; ++r)
            for (int s = r + 1; s < k; ++s) {
                const double apq = a[r * k + s];
                if (apq == 0.0) continue;
                /* plane rotation J(r, s) with J^T A J zeroing a[r][s] */
                const double theta = (a[s * k + s] - a[r * k + r]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                const double arr = a[r * k + r], ass = a[s * k + s];
                /* rows r and s of A J (off the 2x2 block); columns follow by symmetry */
                for (int u = 0; u < k; ++u) {
                    if (u == r || u == s) continue;
                    const double aru = a[r * k + u], asu = a[s * k + u];
                    a[r * k + u] = a[u * k + r] = cs * aru - sn * asu;
                    a[s * k + u] = a[u * k + s] = sn * aru + cs * asu;
                }
                a[r * k + r] = arr - t * apq;
                a[s * k + s] = ass + t * apq;
                a[r * k + s] = a[s * k + r] = 0.0;
                for (int u = 0; u < k; ++u) {
                    const double vr = vt[r * k + u], vs = vt[s * k + u];
                    vt[r * k + u] = cs * vr - sn * vs;
                    vt[s * k + u] = sn * vr + cs * vs;
                }
            }
    }
    for (int i = 0; i < k; ++i) evals[i] = a[i * k + i];
    for (int l = 0; l < k; ++l)
        for (int u = 0; u < k; ++u) evecs[u * k + l] = vt[l * k + u];
    free(a);
    free(vt);
}

/* coef = nrm * exp(-i T) e_1 via the eigendecomposition (eq. matrix_exp_approx).
 * coef: k complex (2k doubles). */
void orc_expm_e1(int k, const double *alpha, const double *beta, double nrm, double *coef_d)
{
    cplx *coef = (cplx *)coef_d;
    double *ev = (double *)malloc(sizeof(double) * k);
    double *V = (double *)malloc(sizeof(double) * k * k);
    orc_tridiag_eig(k, alpha, beta, ev, V);
    for (int j = 0; j < k; ++j) {
        cplx s = 0;
        for (int l = 0; l < k; ++l) s += V[j * k + l] * cexp(-I * ev[l]) * V[0 * k + l];
        coef[j] = nrm * s;
    }
    free(ev);
    free(V);
}

/*
 * n_steps short-time steps psi <- exp(-i A_n) psi, A_n = dt H(t_n averaged),
 * each by an m-dimensional Krylov space (eq. matrix_exp_approx).  psi is
 * updated in place; the norm is never renormalised.  stats may be NULL.
 */
int orc_propagate(const orc_params *p, double *psi_d, double t0, double dt, int n_steps, int m,
                  orc_stat *stats)
{
    const size_t n = (size_t)2 * p->nx * p->ny;
    cplx *psi = (cplx *)psi_d;
    cplx *Q = (cplx *)malloc(n * m * sizeof(cplx));
    double *alpha = (double *)malloc(sizeof(double) * m), *beta = (double *)malloc(sizeof(double) * m);
    cplx *coef = (cplx *)malloc(sizeof(cplx) * m);
    double cum = 0.0;
    for (int step = 0; step < n_steps; ++step) {
        double a_hom[2];
        orc_field_average(p, t0 + step * dt, dt, a_hom);
        const double nrm = vnorm(n, psi);
        const int keff = orc_lanczos(p, a_hom, dt, (const double *)psi, m, 0, (double *)Q, alpha, beta);
        double err = 0.0;
        if (keff > 0) {
            orc_expm_e1(keff, alpha, beta, nrm, (double *)coef);
            for (size_t t = 0; t < n; ++t) psi[t] = 0;
            for (int j = 0; j < keff; ++j) {
                const cplx *qj = Q + (size_t)j * n;
                for (size_t t = 0; t < n; ++t) psi[t] += coef[j] * qj[t];
            }
            /* eq. matrix_exponential_error: beta_k ||psi|| |e_k^T exp(-iT) e_1| */
            err = beta[keff - 1] * cabs(coef[keff - 1]);
        }
        cum += err;
        if (stats) {
            stats[step].k_eff = keff;
            stats[step].err_est = err;
            stats[step].cum_bound = cum;
            stats[step].norm2 = creal(vdot(n, psi, psi));
        }
    }
    free(Q);
    free(alpha);
    free(beta);
    free(coef);
    return 0;
}

/*
 * Ritz vector y = sum_j t_j q_j (Sec. 2 eq. eigenvec_approx) of the
 * eigenvector t = column l of V (keff x keff, row-major).  The sign of t is
 * fixed so that t_1 = <q_1, y> > 0 (the overlap with the start vector is real
 * and positive); a zero t_1 takes the sign of the component of largest
 * magnitude instead.  A Ritz vector of a simple Ritz value is unique up to
 * that sign.
 */
static void ritz_vector(size_t n, int keff, const double *Q_d, const double *V, int l, cplx *y)
{
    const cplx *Q = (const cplx *)Q_d;
    int lead = 0;
    for (int j = 1; j < keff; ++j)
        if (fabs(V[j * keff + l]) > fabs(V[lead * keff + l])) lead = j;
    const double piv = V[l] != 0.0 ? V[l] : V[lead * keff + l];
    const double sgn = piv < 0.0 ? -1.0 : 1.0;
    for (size_t t = 0; t < n; ++t) y[t] = 0.0;
    for (int j = 0; j < keff; ++j) {
        const double tj = sgn * V[j * keff + l];
        const cplx *qj = Q + (size_t)j * n;
        for (size_t t = 0; t < n; ++t) y[t] += tj * qj[t];
    }
}

/*
 * Eigenvalue mode (Sec. 2 eq. A_approx / error_est, Sec. 5): k Lanczos
 * iterations on H (dt = 1, fields at t = 0) from psi0, optionally with full
 * reorthogonalisation applied twice.  The Ritz values of T_k in [e_lo, e_hi]
 * are sorted and grouped into clusters whose neighbours lie within tol (a
 * converged eigenvalue reappears as several copies once orthogonality is lost,
 * Sec. 2 and Sec. 5).  A cluster's bound is beta_k times the norm of the last
 * components of its eigenvectors (eq. error_est, taken over the cluster so that
 * the split of nearly equal Ritz vectors does not matter).  Clusters with bound
 * <= tol are reported, ascending, as their mean value.  Returns k_eff; the
 * number reported (at most max_out) goes to n_found.
 */
static int eigen_core(const orc_params *p, const double *psi0, int k, int reorth, double e_lo, double e_hi,
                      double tol, int max_out, double *evals_out, double *bounds_out, int *n_found,
                      double *vecs_out)
{
    const size_t n = (size_t)2 * p->nx * p->ny;
    double *Q = (double *)malloc(n * (size_t)k * sizeof(cplx));
    double *alpha = (double *)malloc(sizeof(double) * k), *beta = (double *)malloc(sizeof(double) * k);
    const double zero[2] = {0.0, 0.0};
    const int keff = orc_lanczos(p, zero, 1.0, psi0, k, reorth, Q, alpha, beta);
    *n_found = 0;
    if (keff == 0) {
        free(Q);
        free(alpha);
        free(beta);
        return 0;
    }
    double *ev = (double *)malloc(sizeof(double) * keff);
    double *V = (double *)malloc(sizeof(double) * keff * keff);
    orc_tridiag_eig(keff, alpha, beta, ev, V);
    /* candidates in the window, with their last eigenvector components */
    int nc = 0;
    double *cv = (double *)malloc(sizeof(double) * keff), *ct = (double *)malloc(sizeof(double) * keff);
    int *cl = (int *)malloc(sizeof(int) * keff);
    for (int l = 0; l < keff; ++l) {
        if (ev[l] >= e_lo && ev[l] <= e_hi) {
            cv[nc] = ev[l];
            ct[nc] = V[(keff - 1) * keff + l];
            cl[nc] = l;
            ++nc;
        }
    }
    /* sort ascending (insertion sort) */
    for (int a = 1; a < nc; ++a) {
        const double v = cv[a], t = ct[a];
        const int li = cl[a];
        int c = a - 1;
        while (c >= 0 && cv[c] > v) {
            cv[c + 1] = cv[c];
            ct[c + 1] = ct[c];
            cl[c + 1] = cl[c];
            --c;
        }
        cv[c + 1] = v;
        ct[c + 1] = t;
        cl[c + 1] = li;
    }
    int nf = 0;
    for (int a = 0; a < nc;) {
        int b = a + 1;
        while (b < nc && cv[b] - cv[b - 1] <= tol) ++b;
        double sum = 0.0, t2 = 0.0;
        int rep = a;
        for (int c = a; c < b; ++c) {
            sum += cv[c];
            t2 += ct[c] * ct[c];
            if (fabs(ct[c]) < fabs(ct[rep])) rep = c;
        }
        const double bound = fabs(beta[keff - 1]) * sqrt(t2);
        if (bound <= tol && nf < max_out) {
            evals_out[nf] = sum / (b - a);
            bounds_out[nf] = bound;
            if (vecs_out) ritz_vector(n, keff, Q, V, cl[rep], (cplx *)vecs_out + (size_t)nf * n);
            ++nf;
        }
        a = b;
    }
    *n_found = nf;
    free(cl);
    free(cv);
    free(ct);
    free(ev);
    free(V);
    free(Q);
    free(alpha);
    free(beta);
    return keff;
}

int orc_eigen(const orc_params *p, const double *psi0, int k, int reorth, double e_lo, double e_hi,
              double tol, int max_out, double *evals_out, double *bounds_out, int *n_found)
{
    return eigen_core(p, psi0, k, reorth, e_lo, e_hi, tol, max_out, evals_out, bounds_out, n_found, NULL);
}

/*
 * Ritz vectors (Sec. 2 eq. eigenvec_approx) of the values orc_eigen reports,
 * with full reorthogonalisation (the stored q_j are then orthonormal and
 * y = Q_k t is a unit vector).  vecs_out receives max_out vectors of
 * n = 2*nx*ny complex values.
 */
int orc_eigen_vectors(const orc_params *p, const double *psi0, int k, double e_lo, double e_hi, double tol,
                      int max_out, double *evals_out, double *bounds_out, int *n_found, double *vecs_out)
{
    return eigen_core(p, psi0, k, 1, e_lo, e_hi, tol, max_out, evals_out, bounds_out, n_found, vecs_out);
}

/*
 * Expectation values at the final time for the differentiable observable of
 * the adjoint check: out = {<psi|psi>, <x>, <y>, <p_x>, <p_y>} with
 * <O> = <psi|O|psi>/<psi|psi>, x, y the grid coordinates and p = -i D the
 * same central difference as the Hamiltonian (Sec. 3 momentum operator).
 */
void orc_expectations(const orc_params *p, const double *psi_d, double *out)
{
    const cplx *psi = (const cplx *)psi_d;
    const double hx = grid_h(p->x_min, p->x_max, p->nx);
    const double hy = grid_h(p->y_min, p->y_max, p->ny);
    double n = 0.0, sx = 0.0, sy = 0.0;
    cplx spx = 0, spy = 0;
    for (int s = 0; s < 2; ++s)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                const cplx v = site(p, psi, s, i, j);
                const double w = creal(conj(v) * v);
                n += w;
                sx += (p->x_min + i * hx) * w;
                sy += (p->y_min + j * hy) * w;
                const cplx dx = (site(p, psi, s, i + 1, j) - site(p, psi, s, i - 1, j)) / (2.0 * hx);
                const cplx dy = (site(p, psi, s, i, j + 1) - site(p, psi, s, i, j - 1)) / (2.0 * hy);
                spx += conj(v) * (-I * dx);
                spy += conj(v) * (-I * dy);
            }
    out[0] = n;
    out[1] = n > 0 ? sx / n : 0.0;
    out[2] = n > 0 ? sy / n : 0.0;
    out[3] = n > 0 ? creal(spx) / n : 0.0;
    out[4] = n > 0 ? creal(spy) / n : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Hermite pseudospectral discretisation (Sec. 5).  Each spinor component is */
/* represented by its values at the N x N collocation points (x_i, y_j),     */
/* x_i = scale * xi_i with xi_i the roots of the N-th Hermite polynomial,    */
/* i.e. in the span of the tensor products of the first N Hermite functions. */
/* The variables are phi_ij = sqrt(lambda_i lambda_j) psi(x_i, y_j) with the  */
/* Christoffel numbers lambda (scaled), so that sum |phi|^2 is the L^2 norm   */
/* of the interpolant and the derivative is an antisymmetric matrix D~:      */
/* H is Hermitian in the Euclidean inner product, as in the finite-difference */
/* discretisation.                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;              /* collocation points per axis */
    double scale;           /* x = scale * xi */
    double mass, c, charge;
    double bz;              /* uniform magnetic field, symmetric gauge */
    int32_t pot_kind;       /* as orc_params */
    double pot_z, pot_a;
    int32_t chirality;
} orc_hparams;

/* Orthonormal Hermite functions h_0..h_nmax at x (three-term recurrence). */
static void hermite_functions(int nmax, double x, double *h)
{
    h[0] = pow(M_PI, -0.25) * exp(-0.5 * x * x);
    if (nmax >= 1) h[1] = sqrt(2.0) * x * h[0];
    for (int n = 1; n < nmax; ++n) h[n + 1] = sqrt(2.0 / (n + 1)) * x * h[n] - sqrt((double)n / (n + 1)) * h[n - 1];
}

/*
 * Roots xi_0 < ... < xi_{N-1} of the N-th Hermite polynomial (the eigenvalues
 * of its Jacobi matrix: zero diagonal, off-diagonal sqrt(k/2), k = 1..N-1, by
 * the oracle's cyclic Jacobi, then Newton on h_N) and the Christoffel numbers
 * lambda_i = 1 / sum_{n<N} h_n(xi_i)^2 (the quadrature sum_i lambda_i
 * f(xi_i) integrates h_a h_b exactly for a, b < N).
 */
void orc_hermite_nodes(int N, double *xi, double *lambda)
{
    double *al = (double *)calloc(N, sizeof(double)), *be = (double *)calloc(N, sizeof(double));
    double *V = (double *)malloc(sizeof(double) * N * N), *h = (double *)malloc(sizeof(double) * (N + 2));
    for (int k = 1; k < N; ++k) be[k - 1] = sqrt(0.5 * k);
    orc_tridiag_eig(N, al, be, xi, V);
    /* ascending (insertion sort) */
    for (int a = 1; a < N; ++a) {
        const double v = xi[a];
        int b = a - 1;
        while (b >= 0 && xi[b] > v) {
            xi[b + 1] = xi[b];
            --b;
        }
        xi[b + 1] = v;
    }
    for (int i = 0; i < N; ++i) {
        double x = xi[i];
        for (int it = 0; it < 20; ++it) {
            hermite_functions(N, x, h);
            /* h_N' = sqrt(2N) h_{N-1} - x h_N */
            const double d = sqrt(2.0 * N) * h[N - 1] - x * h[N];
            const double dx = h[N] / d;
            x -= dx;
            if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) break;
        }
        xi[i] = x;
        hermite_functions(N, x, h);
        double s2 = 0.0;
        for (int n = 0; n < N; ++n) s2 += h[n] * h[n];
        lambda[i] = 1.0 / s2;
    }
    free(al);
    free(be);
    free(V);
    free(h);
}

/*
 * D~ (N x N, row-major, unit scale): the derivative of the interpolant in
 * span{h_0..h_{N-1}} in the variables phi_i = sqrt(lambda_i) f(xi_i), built
 * from the basis: with E_in = sqrt(lambda_i) h_n(xi_i) (orthogonal: E^T E =
 * I by the exact quadrature) and E'_in = sqrt(lambda_i) h_n'(xi_i),
 * h_n' = sqrt(n/2) h_{n-1} - sqrt((n+1)/2) h_{n+1}, D~ = E' E^T.
 */
void orc_hermite_dmat(int N, const double *xi, const double *lambda, double *dmat)
{
    double *E = (double *)malloc(sizeof(double) * N * N), *Ed = (double *)malloc(sizeof(double) * N * N);
    double *h = (double *)malloc(sizeof(double) * (N + 2));
    for (int i = 0; i < N; ++i) {
        hermite_functions(N, xi[i], h);
        const double w = sqrt(lambda[i]);
        for (int n = 0; n < N; ++n) {
            E[i * N + n] = w * h[n];
            const double dn = (n > 0 ? sqrt(0.5 * n) * h[n - 1] : 0.0) - sqrt(0.5 * (n + 1)) * h[n + 1];
            Ed[i * N + n] = w * dn;
        }
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int n = 0; n < N; ++n) acc += Ed[i * N + n] * E[j * N + n];
            dmat[i * N + j] = acc;
        }
    free(E);
    free(Ed);
    free(h);
}

typedef struct {
    const orc_hparams *p;
    double *x;   /* scaled nodes */
    double *D;   /* D~ / scale */
} herm_op_ctx;

static void herm_setup(const orc_hparams *p, herm_op_ctx *c)
{
    const int N = p->n;
    double *lam = (double *)malloc(sizeof(double) * N);
    c->p = p;
    c->x = (double *)malloc(sizeof(double) * N);
    c->D = (double *)malloc(sizeof(double) * N * N);
    orc_hermite_nodes(N, c->x, lam);
    orc_hermite_dmat(N, c->x, lam, c->D);
    for (int i = 0; i < N; ++i) c->x[i] *= p->scale;
    for (int i = 0; i < N * N; ++i) c->D[i] /= p->scale;
    free(lam);
}

static void herm_free(herm_op_ctx *c)
{
    free(c->x);
    free(c->D);
}

static double herm_potential(const orc_hparams *p, double x, double y)
{
    if (p->pot_kind == 1) return -p->pot_z / sqrt(x * x + y * y + p->pot_a * p->pot_a);
    if (p->pot_kind == 2) return -1.5 * p->pot_z / sqrt(x * x + y * y + 3.0 / (p->pot_z * p->pot_z));
    return 0.0;
}

/*
 * out = H in for the Hermite collocation variables (layout (2, N, N), x
 * fastest): H = c [sigma1 (p_x - q A_x) + chi sigma2 (p_y - q A_y)] +
 * sigma3 m c^2 + V with p = -i D~ along each axis and A = (B/2)(-y, x)
 * (Sec. 3 Hamiltonian, Sec. 5 discretisation).
 */
static void herm_op(const void *ctx, const cplx *in, cplx *out)
{
    const herm_op_ctx *c = (const herm_op_ctx *)ctx;
    const orc_hparams *p = c->p;
    const int N = p->n;
    const double mc2 = p->mass * p->c * p->c;
    cplx s1[2][2], s2[2][2], s3[2][2];
    pauli(1, s1);
    pauli(2, s2);
    pauli(3, s3);
    const double chi = p->chirality < 0 ? -1.0 : 1.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s2[a][b] *= chi;
    for (int j = 0; j < N; ++j) {
        const double y = c->x[j];
        for (int i = 0; i < N; ++i) {
            const double x = c->x[i];
            const double v = herm_potential(p, x, y);
            const double ax = -0.5 * p->bz * y, ay = 0.5 * p->bz * x;
            cplx psi[2], pix[2], piy[2];
            for (int s = 0; s < 2; ++s) {
                const cplx *f = in + (size_t)s * N * N;
                psi[s] = f[j * N + i];
                cplx dx = 0, dy = 0;
                for (int k = 0; k < N; ++k) {
                    dx += c->D[i * N + k] * f[j * N + k];
                    dy += c->D[j * N + k] * f[k * N + i];
                }
                pix[s] = -I * dx - p->charge * ax * psi[s];
                piy[s] = -I * dy - p->charge * ay * psi[s];
            }
            for (int a = 0; a < 2; ++a) {
                cplx acc = v * psi[a];
                for (int b = 0; b < 2; ++b)
                    acc += p->c * (s1[a][b] * pix[b] + s2[a][b] * piy[b]) + mc2 * s3[a][b] * psi[b];
                out[(size_t)a * N * N + j * N + i] = acc;
            }
        }
    }
}

/* Scaled nodes x_i and D~ / scale of the problem (x: N, dmat: N*N). */
void orc_hermite_operator(const orc_hparams *p, double *x, double *dmat)
{
    herm_op_ctx c;
    herm_setup(p, &c);
    memcpy(x, c.x, sizeof(double) * p->n);
    memcpy(dmat, c.D, sizeof(double) * p->n * p->n);
    herm_free(&c);
}

void orc_apply_h_hermite(const orc_hparams *p, const double *in_d, double *out_d)
{
    herm_op_ctx c;
    herm_setup(p, &c);
    herm_op(&c, (const cplx *)in_d, (cplx *)out_d);
    herm_free(&c);
}

/* The three-vector recurrence (Sec. 2) on the Hermite H (eigenvalue mode). */
int orc_lanczos_plain_hermite(const orc_hparams *p, const double *b_d, int k, double *alpha, double *beta)
{
    herm_op_ctx c;
    herm_setup(p, &c);
    const int keff = lanczos3((size_t)2 * p->n * p->n, herm_op, &c, (const cplx *)b_d, k, alpha, beta);
    herm_free(&c);
    return keff;
}
