// Internal interface between the host runtime (host.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dl {

constexpr int kMaxM = 64;         // largest Krylov dimension of a time step
constexpr int kBlock = 256;       // threads per workgroup (four wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 8192;  // capacity of the per-workgroup partial-sum table
constexpr int kPartialStride = 8; // doubles per workgroup in the partial-sum table
constexpr int kChunk = 2048;      // time steps whose fields/stats are staged per batch
// Extra bytes between consecutive Krylov vectors so that the vectors a sweep
// streams concurrently do not sit a power of two apart in HBM.
constexpr size_t kVecPad = 4096 + 768;

// Device-resident scalars of the running Lanczos step.  Written only by the
// last workgroup of a sweep (deterministic fixed-order reductions) and by the
// single-wave tridiagonal kernel; read by every later kernel on the stream.
struct Scalars {
    double coef[2 * (kMaxM + 2)];  // c_j / gamma_j (re, im) for the recombination, j = 1..k
    double scale;                  // running max of |alpha_j|, beta_j (breakdown test)
    double cabs_k;                 // |c_k|, input of the error estimate
    double beta_k;                 // beta_k of the step (error estimate)
    double sigma;                  // spectral shift of the sweeps: they run on A - sigma I
    int kstop;                     // sweeps with index > kstop do nothing this step
    int keff;                      // Krylov dimension in use (set at the end of the recurrence)
    int status;                    // 0 ok, 3 non-finite (whole call aborted)
    int steps_done;                // completed steps of the current call
    unsigned int ticket;           // last-workgroup-done counter (self-resetting)
    // adaptive Krylov dimension (ktol > 0): each step runs knext iterations
    // (0: m), and the small exponential predicts knext for the next step
    int kmin, kmax, knext;
    double ktol;                   // per-step bound on the error estimate (0: off)
};

struct StepStat {
    double err_est;
    double norm2;
    int keff;
    int pad;
    double round_bound;  // a-priori bound of the step's error from complex64 storage (0 in FP64)
};

// Rounding of the complex64 Krylov storage (mixed precision): each real
// component of a stored vector is rounded to nearest with relative error at
// most 2^-24; a component below the normal range adds at most 2^-126.
constexpr double kStoreEps32 = 5.9604644775390625e-8;    // 2^-24
constexpr double kStoreTiny32 = 1.1754943508222875e-38;  // 2^-126

// Coefficients of the operator A = s * H applied by the sweeps, s = dt for a
// time step and s = 1 for the plain Hamiltonian.
struct Op {
    int nx, ny, bcx, bcy;
    double xmin, ymin, hx, hy;
    double kx, ky;        // s c / (2 h_x), chir s c / (2 h_y) (chir = +-1: alpha2 = chir sigma2)
    double mc2;           // s m c^2
    double bq;            // s c q B / 2: gx = gx_hom + bq y
    double bqy;           // chir bq: gy = gy_hom - bqy x (gy_hom carries chir as well)
    int pot_kind;         // 0 none, 1 s*(-zc / sqrt(r^2 + a2))
    int has_table;
    double vz, va2;       // s*zc, a2
    const double *vtab;   // optional potential table (device), multiplied by s
    double vscale;
};

// Site-dependent terms of the operator (compile-time specialisations of the
// sweeps): the potential (or potential table) and the magnetic field.
constexpr int kTermPot = 1;
constexpr int kTermB = 2;

// Wave-to-tile mapping of one sweep: every wave owns `own` consecutive columns
// of one strip and `rows` consecutive rows of it (its chunk).
struct Tiles {
    int halo, own, nstrips, nchunks, rows, nblocks;
};

// Vector layouts.  The state psi (and its ping-pong partner) uses the caller's
// layout: two planes of nx*ny complex128 values.  Krylov vectors u_2.. hold
// both components of a site next to each other ([site][component]), complex64
// in mixed precision or complex128 in FP64.

// Arguments of a recurrence sweep (Lanczos iteration p >= 2).
struct PassArgs {
    Op op;
    Tiles t;
    const void *u1;      // u_{p-1} (psi layout when p == 2)
    const void *u2;      // u_{p-2} (psi layout when p == 3; unused when p == 2)
    void *uo;            // u_p (written)
    const double *field; // (gx_hom, gy_hom) of this step
    double *alpha;       // alpha[1..]
    double *gamma;       // gamma[1..]: gamma_1 = ||psi||, gamma_p = beta_{p-1}
    Scalars *sc;
    double *partials;
    int pass;
    int m;
    int replay;          // 1: recompute u_p only (second Lanczos run), no reductions or scalar updates
    // 1: this iteration's partials are folded by the next kernel, and (p >= 3)
    // this kernel folds those of iteration p-1 from prev_partials (prev_nblk
    // workgroups) before its march
    int defer;
    const double *prev_partials;
    int prev_nblk;
};

// The last iteration's partials, folded by the small exponential's kernel
// (pass 0: nothing to fold).
struct TailFold {
    const double *partials;
    int nblk;
    int pass;
};

// Arguments of the recombination psi_new = sum_j coef_j u_j (flat streaming).
struct CombArgs {
    const double2 *psi;  // u_1 (psi layout)
    const void *basis;   // u_2..u_m
    size_t vec_bytes;    // byte stride between consecutive Krylov vectors
    size_t sites;        // nx*ny
    double2 *out;        // new state (psi layout)
    Scalars *sc;
    double *partials;
    StepStat *stat;      // entry of this step
    // keep != NULL: workgroup 0 also copies the step's scalars (raw words) to
    // keep, alpha[0..keep_nab) to keep + keep_alpha and gamma[0..keep_nab) to
    // keep + keep_gamma (what a later pass reads of this step)
    const double *alpha, *gamma;
    char *keep;
    size_t keep_alpha, keep_gamma;
    int keep_nab;
};

// One term of the recombination during a second Lanczos run (the basis is not
// stored): out = c_1 psi for p = 1, out += c_p u_p for p = 2..k_eff; the
// launch with p = k_eff also reduces ||out||^2 into the step statistics.
// Recombination terms p0 .. p0 + nv - 1 (nv <= kAccumTerms) of the second
// Lanczos run, added to the new state in term order; p0 = 1 starts the sum
// with c_1 psi instead of reading the state.
constexpr int kAccumTerms = 3;
struct AccumArgs {
    const double2 *psi;           // u_1 (psi layout)
    const void *u[kAccumTerms];   // u_{p0+v} (paired layout); unused for term 1
    size_t sites;
    double2 *out;                 // new state (psi layout)
    Scalars *sc;
    double *partials;
    StepStat *stat;
    int p0, nv;
};
void launch_accum(const AccumArgs &a, bool mixed, int nblocks, hipStream_t st);

// Observables <x>, <y>, <p_x>, <p_y> of a state and the adjoint seed.
// obs (device, 8 doubles): N = <psi|psi>, <x>, <y>, <p_x>, <p_y>, loss = sum of
// the expectations selected by the loss flags (1 x, 2 y, 4 p_x, 8 p_y).
void launch_observe(const Op &op, const double2 *psi, int loss_kind, Scalars *sc, double *partials,
                    double *obs, int nblocks, hipStream_t st);
// lam = (O psi - loss psi) / N with O the sum of the selected observables.
void launch_adjoint_seed(const Op &op, const double2 *psi, int loss_kind, const double *obs,
                         double2 *lam, hipStream_t st);

// Contraction of two Krylov bases for the adjoint: for a < k_lam, b < k_psi
//   S01[a][b] = sum_sites conj(ul_a,0) up_b,1,  S10[a][b] = sum_sites conj(ul_a,1) up_b,0
// with ul_1 = lam (psi layout), ul_j the lam basis; likewise for psi.
constexpr int kContractM = 16;  // largest Krylov dimension of the adjoint
// Per-step record of the adjoint (doubles): the contraction, then both
// tridiagonal chains and the scalars needed to rebuild T and the basis norms.
constexpr int kRecS = 0;                                // 256 pairs x (S01 re, im, S10 re, im)
constexpr int kRecAlphaL = kRecS + 4 * kContractM * kContractM;
constexpr int kRecGammaL = kRecAlphaL + kContractM + 2;  // index 0..kContractM+1 as on the device
constexpr int kRecAlphaP = kRecGammaL + kContractM + 2;
constexpr int kRecGammaP = kRecAlphaP + kContractM + 2;
constexpr int kRecMeta = kRecGammaP + kContractM + 2;    // sigma_l, sigma_p, keff_l, keff_p, status_l, status_p
constexpr int kRecLen = 1120;                            // padded: 8960 bytes per record
static_assert(kRecMeta + 6 <= kRecLen, "adjoint record overflow");
struct ContractArgs {
    const double2 *lam1;
    const char *lam_basis;
    const double2 *psi1;
    const char *psi_basis;
    size_t vec_bytes;
    size_t sites;
    const Scalars *sc_lam;
    const Scalars *sc_psi;
    const double *alpha_lam, *gamma_lam, *alpha_psi, *gamma_psi;
    double *partials;  // this step's partial table: 4 kBlock outputs x nblocks
    double *rec;       // record of this step (kRecLen doubles); the contraction writes the chains and scalars
};
void launch_contract(const ContractArgs &a, int nblocks, hipStream_t st);
// The contraction sums of steps i0 .. i0 + nsteps - 1 into their records (rec
// + step * kRecLen); step s's partials are in slot s % nslot of `partials`.
void launch_contract_fold(const double *partials, int nslot, int nblocks, double *rec, int i0, int nsteps,
                          hipStream_t st);

void launch_first(const Op &op, const Tiles &t, const double2 *psi, const double *field,
                  double *alpha, double *gamma, Scalars *sc, double *partials, int m,
                  int shift, hipStream_t st);
void launch_recur(const PassArgs &a, bool mixed, hipStream_t st);
// reps, rabs: relative and absolute rounding of one stored Krylov vector
// (kStoreEps32 and kStoreTiny32 * sqrt(4 * sites) in mixed precision, 0 in FP64)
void launch_tridiag(double *alpha, double *gamma, Scalars *sc, StepStat *stat, double reps, double rabs,
                    const TailFold &fold, hipStream_t st);
// the last iteration's scalar update from the partials it left (TailFold)
void launch_fold_tail(double *alpha, double *gamma, Scalars *sc, const TailFold &fold, hipStream_t st);
// wide: the complex64 form with 16 sites per thread (see combine_wide)
void launch_combine(const CombArgs &a, bool mixed, bool wide, int nblocks, hipStream_t st);
void launch_apply(const Op &op, const Tiles &t, const double2 *x, double2 *y, double gxh,
                  double gyh, hipStream_t st);
void launch_reset(Scalars *sc, hipStream_t st);
// Reset at the start of a step call (see k_reset): keep_status for
// asynchronous calls, the adaptive-dimension parameters (ktol = 0: off).
void launch_reset_call(Scalars *sc, int keep_status, int kmin, int kmax, double ktol, hipStream_t st);
// psi <- state (n complex128 values) when sc->steps_done is odd.
void launch_finish_copy(const Scalars *sc, const double2 *state, double2 *psi, size_t n, int cus, hipStream_t st);

// ---------------------------------------------------------------------------
// Batches of independent packets (grids of different sizes and fields, one
// Krylov dimension and precision): every kernel of a step is one launch over
// all packets.  Workgroups of a launch are grouped by packet (the four waves
// of a workgroup belong to one packet), so each packet's reductions are a
// segment of the workgroups, folded in fixed order by the segment's last
// workgroup with the packet's own ticket.
// ---------------------------------------------------------------------------
enum { kGridSweep = 0, kGridFirst = 1, kGridCombine = 2, kGridKinds = 3 };

struct BatchPacket {
    Op op;             // A = dt H of the packet (static part; the laser term per step in `fields`)
    Tiles tiles[2];    // strip geometry of the sweeps (halo 2) and of iteration 1 (halo 1)
    double2 *psi;      // caller's state
    double2 *state;    // ping-pong partner (workspace)
    char *basis;       // u_2 .. u_m
    size_t vstride;    // bytes between consecutive Krylov vectors
    size_t sites;      // nx * ny
    double *alpha, *gamma;
    Scalars *sc;
    StepStat *stats;   // kChunk entries
    double *fields;    // (gx_hom, gy_hom) per step of the chunk
    double reps, rabs; // rounding of one stored Krylov vector (see launch_tridiag)
};

struct BatchBlock {    // one workgroup of a batched launch
    int packet;        // packet of the workgroup
    int local;         // index of the workgroup within its packet's segment
    int nblk;          // workgroups of the segment
    int first;         // first workgroup of the segment (partials offset)
};

struct BatchTask {     // one wave of a batched sweep (inactive when y0 >= y1)
    int strip, y0, y1, pad;
};

struct BatchArgs {
    const BatchPacket *pk;
    const BatchBlock *blocks;  // of this launch's grid kind
    const BatchTask *tasks;    // kWaves per workgroup (sweeps and iteration 1)
    const int *wg_first;       // resident workgroup g runs entries wg_first[g] .. wg_first[g + 1] - 1
    double *partials;          // kPartialStride doubles per workgroup
    int pass, m, step, parity; // step: index in the chunk tables; parity 1: the input is `state`
    int ntasks;                // block entries of the launch (spread over the resident workgroups)
};
// Resident workgroups per compute unit of the batched sweeps (measured on the
// 256-packet batch with balanced entry lists, ms per step: 2 per CU 5.54-5.58
// for R = 32..64, 3 per CU 5.63-5.91, 1 per CU 5.73-5.82).
#ifndef DL_BATCH_WGS_PER_CU
#define DL_BATCH_WGS_PER_CU 2
#endif
constexpr int kBatchWgsPerCu = DL_BATCH_WGS_PER_CU;

void launch_first_batch(const BatchArgs &b, int nblocks, bool py, int terms, hipStream_t st);
void launch_recur_batch(const BatchArgs &b, int nblocks, bool mixed, bool py, int terms, hipStream_t st);
void launch_tridiag_batch(const BatchArgs &b, int npackets, hipStream_t st);
void launch_reset_batch(const BatchPacket *pk, int n, hipStream_t st);
void launch_combine_batch(const BatchArgs &b, int nblocks, bool mixed, hipStream_t st);
// Resident waves per compute unit of the batched kernels (0 first, 1 sweeps).
// Sites per recombination tile.
int combine_tile_sites(bool mixed);

Tiles make_tiles(int nx, int ny, int halo, int target_waves);
// Whether the recombination of `sites` sites uses the wide complex64 form
// (at least one wide tile per compute unit).
bool combine_wide(size_t sites, bool mixed, int cus);
// Workgroups of the recombination for `sites` sites (<= kMaxBlocks); wide as
// above (the second Lanczos run's accumulation uses the narrow form).
int combine_grid(size_t sites, bool mixed, int cus, bool wide);
// Resident waves per compute unit of a kernel family: 0 first iteration,
// 1 recurrence sweep p >= 4, 2 sweep p = 2, 3 sweep p = 3, 4 apply; py:
// periodic in y, terms: site-dependent terms (sweep_terms).
int sweep_waves_per_cu(int which, bool mixed, bool py, int terms);
int sweep_terms(const Op &op);

// Hermite pseudospectral problems (hermite_kernels.hip): n x n collocation
// points, n a multiple of 16 up to 64.
struct HermOp {
    int n;
    int pot_kind;        // 0 none, 1 -vz / sqrt(r^2 + va2)
    double c, chi;       // speed of light, alpha2 = chi sigma2
    double mc2;          // m c^2
    double bq;           // c q B / 2 (symmetric gauge)
    double vz, va2;
    const double *dmat;  // D~ / scale, n x n row-major (device)
    const double *x;     // scaled nodes (device)
};
struct HermRun {
    const double2 *b;    // start vector (device, layout (2, n, n))
    double *alpha, *beta;
    int keff;            // iterations done; 0 for b = 0, -1 for a non-finite reduction
    int pad;
};
void launch_herm_apply(const HermOp *ops, const double2 *const *x, double2 *const *y, int n, hipStream_t st);
void launch_herm_lanczos(const HermOp *ops, HermRun *runs, int n, int k_max, hipStream_t st);

// Eigen mode with full reorthogonalisation (eigen_kernels.hip).  Stored
// complex128 vectors q_1..q_K at q + (j-1) * vstride; the projection partial
// table holds 2 * proj_tiles(n) doubles per vector.
constexpr int kProjTiles = 1024;  // workgroups per vector chunk of a projection (cap)
constexpr int kRitzVecs = 16;     // Ritz vectors formed per pass over the basis
inline int proj_tiles(size_t nelem)
{
    const size_t t = (nelem + kBlock - 1) / kBlock;
    return (int)(t < (size_t)kProjTiles ? (t < 1 ? 1 : t) : (size_t)kProjTiles);
}
// h = Q[0..nvec)^H z (complex, fixed-order reduction).
void launch_proj(const char *q, size_t vstride, int nvec, const double2 *z, size_t nelem, double *pproj,
                 double *h, hipStream_t st);
// z -= Q[0..nvec) h.
void launch_sub_q(const char *q, size_t vstride, int nvec, const double *h, double2 *z, size_t nelem,
                  int nblocks, hipStream_t st);
// beta_0 = ||psi||, q_1 = psi / beta_0 (kstop = 0 when psi = 0).
void launch_first_q(const double2 *psi, size_t nelem, double2 *q1, Scalars *sc, double *beta, double *partials,
                    int nblocks, hipStream_t st);
// beta_i = ||z||, alpha_i = Re h1_i, breakdown test; then q_{i+1} = z / beta_i
// when i < k and the recurrence goes on.
void launch_norm_next(const double2 *z, size_t nelem, const double *h1, int i, int k, double *alpha, double *beta,
                      Scalars *sc, double *partials, double2 *qn, int nblocks, hipStream_t st);
// Y[:, v] = Q[0..nvec) t[:, v] for v < r <= kRitzVecs (t: nvec x kRitzVecs
// row-major, real), y_v at y + v * nelem.
void launch_ritz(const char *q, size_t vstride, int nvec, const double *t, int r, double2 *y, size_t nelem,
                 int nblocks, hipStream_t st);

}  // namespace dl
