// Host runtime of the C ABI declared in include/dirac_lanczos.h: parameter
// validation, workspace planning, the per-step field averages (first Magnus
// term, Sec. 3 eq. time_evolution_approx), the launch sequence of a time step
// (Sec. 4 eq. matrix_exp_approx) and the Ritz-value extraction of the
// eigenvalue mode (Sec. 2 eq. error_est).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

using dl::kChunk;
using dl::kMaxBlocks;
using dl::kMaxM;

namespace dlh {

// Workspace plan.  Vector region: step mode holds the second state buffer
// (complex128) and the Krylov vectors u_2..u_m (complex128, or complex64 in
// mixed precision); eigen mode needs three rolling complex128 vectors.
Layout plan(const dl_params &p, int mode, int k_eigen)
{
    Layout L;
    const int m = p.krylov_dim;
    const bool eig = mode == DL_MODE_EIGEN || mode == DL_MODE_EIGEN_REORTH;
    L.ab_len = std::max(m, eig ? k_eigen + 1 : 0) + 3;
    size_t off = 0;
    L.sc = off;
    off = align256(off + sizeof(dl::Scalars));
    L.alpha = off;
    off = align256(off + sizeof(double) * L.ab_len);
    L.gamma = off;
    off = align256(off + sizeof(double) * L.ab_len);
    L.partials = off;
    off = align256(off + sizeof(double) * dl::kPartialStride * kMaxBlocks);
    L.fields = off;
    off = align256(off + sizeof(double) * 2 * kChunk);
    L.stats = off;
    off = align256(off + sizeof(dl::StepStat) * kChunk);
    L.vecs = off;
    const size_t n = vec_elems(p);
    const size_t basis_elem = p.precision == DL_PREC_MIXED ? 8 : 16;
    // the second state buffer, then the Krylov basis u_2..u_m (stored basis) or
    // three rolling vectors (second Lanczos run)
    const size_t nbasis = mode == DL_MODE_LOWMEM ? (size_t)std::min(m - 1, 3) : (size_t)(m - 1);
    size_t step_region = align256(n * 16) + nbasis * vec_stride(n, basis_elem);
    size_t eig_region = mode == DL_MODE_EIGEN ? 3 * vec_stride(n, 16) : 0;
    if (mode == DL_MODE_EIGEN_REORTH) eig_region = reorth_layout(n, k_eigen).total;
    off += std::max(step_region, eig_region);
    L.total = off;
    return L;
}

const char *validate(const dl_params *p)
{
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
    if ((double)p->nx * (double)p->ny > 2.0e9) return "grid too large (nx*ny > 2e9)";
    if (!(p->x_max > p->x_min) || !(p->y_max > p->y_min)) return "empty box (x_max <= x_min or y_max <= y_min)";
    if (!std::isfinite(p->x_min) || !std::isfinite(p->x_max) || !std::isfinite(p->y_min) ||
        !std::isfinite(p->y_max))
        return "box bounds must be finite";
    if ((p->bc_x != 0 && p->bc_x != 1) || (p->bc_y != 0 && p->bc_y != 1)) return "bc must be 0 or 1";
    if (p->chirality < -1 || p->chirality > 1) return "chirality must be -1, 0 or +1";
    if (!(p->c > 0.0) || !std::isfinite(p->c)) return "c must be positive";
    if (!(p->mass >= 0.0) || !std::isfinite(p->mass)) return "mass must be >= 0";
    if (!std::isfinite(p->charge) || !std::isfinite(p->bz)) return "charge and bz must be finite";
    if (p->krylov_dim < 1 || p->krylov_dim > kMaxM) return "krylov_dim must be in 1..64";
    if (p->precision != DL_PREC_FP64 && p->precision != DL_PREC_MIXED) return "unknown precision";
    if (p->pot_kind < 0 || p->pot_kind > 2) return "unknown pot_kind";
    if (p->pot_kind == 1 && !(p->pot_a != 0.0 && std::isfinite(p->pot_a) && std::isfinite(p->pot_z)))
        return "soft-core potential needs pot_a != 0";
    if (p->pot_kind == 2 && !(p->pot_z != 0.0 && std::isfinite(p->pot_z)))
        return "paper soft-core potential needs pot_z != 0";
    if (p->pulse_kind < 0 || p->pulse_kind > 2) return "unknown pulse_kind";
    if (p->pulse_kind != 0 && !(p->t_pulse > 0.0 && std::isfinite(p->t_pulse))) return "t_pulse must be > 0";
    if (p->pulse_kind == 1 && !(std::isfinite(p->a0) && std::isfinite(p->omega) &&
                                std::isfinite(p->pulse_e[0]) && std::isfinite(p->pulse_e[1])))
        return "pulse parameters must be finite";
    if (p->pulse_kind == 2) {
        if (p->n_coef <= 0 || p->n_coef % 4 != 0 || p->n_coef > 1024 || !p->coef)
            return "Fourier pulse needs coef with n_coef a positive multiple of 4 (<= 1024)";
        for (int i = 0; i < p->n_coef; ++i)
            if (!std::isfinite(p->coef[i])) return "Fourier coefficients must be finite";
    }
    return nullptr;
}

// --- homogeneous laser field --------------------------------------------------
const double kPi = 3.14159265358979323846;

void pulse_now(const dl_params &p, CoefView coef, double t, double *a)
{
    a[0] = a[1] = 0.0;
    if (p.pulse_kind == 0 || t < 0.0 || t > p.t_pulse) return;
    const double s = std::sin(kPi * t / p.t_pulse), env = s * s;
    if (p.pulse_kind == 1) {
        const double f = p.a0 * std::sin(p.omega * t) * env;
        a[0] = f * p.pulse_e[0];
        a[1] = f * p.pulse_e[1];
        return;
    }
    const double w0 = 2.0 * kPi / p.t_pulse;
    for (size_t k = 1; 4 * k <= coef.size(); ++k) {
        const double sk = std::sin(k * w0 * t), ck = std::cos(k * w0 * t);
        a[0] += coef[4 * (k - 1)] * sk + coef[4 * (k - 1) + 1] * ck;
        a[1] += coef[4 * (k - 1) + 2] * sk + coef[4 * (k - 1) + 3] * ck;
    }
    a[0] *= env;
    a[1] *= env;
}

// Exact integrals over [lo, hi] written without cancellation:
//   int sin(nu t) = (2/nu) sin(nu tm) sin(nu h2), int cos(nu t) = (2/nu) cos(nu tm) sin(nu h2)
// with tm the midpoint and h2 the half width.
double int_sin(double nu, double tm, double h2)
{
    if (nu == 0.0) return 0.0;
    return 2.0 / nu * std::sin(nu * tm) * std::sin(nu * h2);
}

double int_cos(double nu, double tm, double h2)
{
    if (nu == 0.0) return 2.0 * h2;
    return 2.0 / nu * std::cos(nu * tm) * std::sin(nu * h2);
}

double basis_average(const dl_params &p, int k, bool cosine, double t0, double dt)
{
    double lo = std::min(t0, t0 + dt), hi = std::max(t0, t0 + dt);
    lo = std::max(lo, 0.0);
    hi = std::min(hi, p.t_pulse);
    if (!(hi > lo)) return 0.0;
    const double tm = 0.5 * (lo + hi), h2 = 0.5 * (hi - lo);
    const double W = 2.0 * kPi / p.t_pulse, nu = k * W;
    double v;
    if (cosine)
        v = 0.5 * int_cos(nu, tm, h2) - 0.25 * (int_cos(nu + W, tm, h2) + int_cos(nu - W, tm, h2));
    else
        v = 0.5 * int_sin(nu, tm, h2) - 0.25 * (int_sin(nu + W, tm, h2) + int_sin(nu - W, tm, h2));
    return v / std::fabs(dt);
}

// (1/|dt|) integral of A_L over the step [t0, t0 + dt]; the envelope
// sin^2(pi t/T) = (1 - cos(W t))/2 (W = 2 pi/T) turns every term into single
// sines and cosines whose integrals are closed forms.
void pulse_average(const dl_params &p, CoefView coef, double t0, double dt, double *a)
{
    a[0] = a[1] = 0.0;
    if (p.pulse_kind == 0) return;
    double lo = std::min(t0, t0 + dt), hi = std::max(t0, t0 + dt);
    lo = std::max(lo, 0.0);
    hi = std::min(hi, p.t_pulse);
    if (!(hi > lo)) return;
    const double tm = 0.5 * (lo + hi), h2 = 0.5 * (hi - lo);
    const double W = 2.0 * kPi / p.t_pulse;
    if (p.pulse_kind == 1) {
        const double w = p.omega;
        const double v = 0.5 * int_sin(w, tm, h2) - 0.25 * (int_sin(w + W, tm, h2) + int_sin(w - W, tm, h2));
        a[0] = p.a0 * v * p.pulse_e[0];
        a[1] = p.a0 * v * p.pulse_e[1];
    } else {
        for (size_t k = 1; 4 * k <= coef.size(); ++k) {
            const double is = basis_average(p, (int)k, false, t0, dt) * std::fabs(dt);
            const double ic = basis_average(p, (int)k, true, t0, dt) * std::fabs(dt);
            a[0] += coef[4 * (k - 1)] * is + coef[4 * (k - 1) + 1] * ic;
            a[1] += coef[4 * (k - 1) + 2] * is + coef[4 * (k - 1) + 3] * ic;
        }
    }
    a[0] /= std::fabs(dt);
    a[1] /= std::fabs(dt);
}

namespace {
// The sweeps of a step alternate between the two halves of the partials table:
// iteration p writes half p mod 2 while the next kernel folds it.
double *partials_half(double *partials, int p)
{
    return partials + (size_t)(p & 1) * (size_t)(kMaxBlocks / 2) * dl::kPartialStride;
}
}  // namespace

dl_status run_build(dl_context *ctx, const Engine &e, const dl::Op &op, const double2 *in,
                    const double *field, double *partials, int shift, bool complete)
{
    hipStream_t st = ctx->stream;
    DL_HIP(ctx, ctx->timed(0, [&] {
        dl::launch_first(op, ctx->tiles_first, in, field, e.alpha, e.gamma, e.sc, partials, e.m, shift, st);
    }));
    // each half of the partials table holds one iteration's workgroups
    for (int pp = 2; pp <= e.m; ++pp)
        if (ctx->tiles_pass(pp).nblocks > kMaxBlocks / 2)
            return ctx->fail(DL_ERR_WORKSPACE, "sweep grid exceeds half of the partials table");
    auto launch = [&](int pp) {
        dl::PassArgs a{};
        a.op = op;
        a.t = ctx->tiles_pass(pp);
        a.u1 = (pp - 1 == 1) ? static_cast<const void *>(in) : e.bvec(pp - 1);
        a.u2 = (pp - 2 == 1) ? static_cast<const void *>(in) : (pp - 2 >= 2 ? e.bvec(pp - 2) : nullptr);
        a.uo = e.bvec(pp);
        a.field = field;
        a.alpha = e.alpha;
        a.gamma = e.gamma;
        a.sc = e.sc;
        a.partials = partials_half(partials, pp);
        a.pass = pp;
        a.m = e.m;
        a.defer = 1;
        if (pp >= 3) {
            a.prev_partials = partials_half(partials, pp - 1);
            a.prev_nblk = ctx->tiles_pass(pp - 1).nblocks;
        }
        dl::launch_recur(a, e.mixed, st);
    };
    for (int pp = 2; pp <= std::min(e.m, 3); ++pp) DL_HIP(ctx, ctx->timed(2, [&] { launch(pp); }));
    // iterations 4..m back to back, timed as one block (an event pair per
    // launch would sit between the kernels)
    if (e.m >= 4)
        DL_HIP(ctx, ctx->timed(1, [&] {
            for (int pp = 4; pp <= e.m; ++pp) launch(pp);
        }, e.m - 3));
    if (complete && e.m >= 2)
        dl::launch_fold_tail(e.alpha, e.gamma, e.sc,
                             dl::TailFold{partials_half(partials, e.m), ctx->tiles_pass(e.m).nblocks, e.m}, st);
    return DL_OK;
}

// One step by the second Lanczos run (the basis is not stored): iterations
// 1..m with three rolling vectors give T, exp(-iT) gives the coefficients,
// then iterations 2..m are replayed bitwise identically (same inputs, no
// scalar updates) and each u_p is added to the new state as it reappears.
dl_status run_twice(dl_context *ctx, const Engine &e, const dl::Op &op, const double2 *in, double2 *out,
                    const double *field, dl::StepStat *stat, double *partials)
{
    hipStream_t st = ctx->stream;
    auto rb = [&](int j) -> void * { return e.basis + (size_t)(j % 3) * e.vstride; };
    auto pass = [&](int pp, int replay) {
        dl::PassArgs a{};
        a.op = op;
        a.t = ctx->tiles_pass(pp);
        a.u1 = (pp - 1 == 1) ? static_cast<const void *>(in) : rb(pp - 1);
        a.u2 = (pp - 2 == 1) ? static_cast<const void *>(in) : (pp - 2 >= 2 ? rb(pp - 2) : nullptr);
        a.uo = rb(pp);
        a.field = field;
        a.alpha = e.alpha;
        a.gamma = e.gamma;
        a.sc = e.sc;
        a.partials = partials;
        a.pass = pp;
        a.m = e.m;
        a.replay = replay;
        return ctx->timed(pp >= 4 ? 1 : 2, [&] { dl::launch_recur(a, e.mixed, st); });
    };
    DL_HIP(ctx, ctx->timed(0, [&] {
        dl::launch_first(op, ctx->tiles_first, in, field, e.alpha, e.gamma, e.sc, partials, e.m, 1, st);
    }));
    for (int pp = 2; pp <= e.m; ++pp) DL_HIP(ctx, pass(pp, 0));
    double reps, rabs;
    store_rounding(ctx->p, reps, rabs);
    DL_HIP(ctx, ctx->timed(3, [&] {
        dl::launch_tridiag(e.alpha, e.gamma, e.sc, stat, reps, rabs, dl::TailFold{nullptr, 0, 0}, st);
    }));
    dl::AccumArgs c{};
    c.psi = in;
    c.sites = vec_elems(ctx->p) / 2;
    c.out = out;
    c.sc = e.sc;
    c.partials = partials;
    c.stat = stat;
    // terms next..pp go into the state together once kAccumTerms of them are
    // regenerated (the three rolling vectors hold u_{pp-2}, u_{pp-1}, u_pp)
    auto accum = [&](int p0, int p1) {
        c.p0 = p0;
        c.nv = p1 - p0 + 1;
        for (int v = 0; v < dl::kAccumTerms; ++v) c.u[v] = (p0 + v >= 2 && p0 + v <= p1) ? rb(p0 + v) : nullptr;
        return ctx->timed(4, [&] { dl::launch_accum(c, e.mixed, ctx->combine_blocks, st); });
    };
    if (e.m == 1) {
        DL_HIP(ctx, accum(1, 1));
        return DL_OK;
    }
    int next = 1;
    for (int pp = 2; pp <= e.m; ++pp) {
        DL_HIP(ctx, pass(pp, 1));
        if (pp - next + 1 == dl::kAccumTerms || pp == e.m) {
            DL_HIP(ctx, accum(next, pp));
            next = pp + 1;
        }
    }
    return DL_OK;
}

dl_status run_finish(dl_context *ctx, const Engine &e, const double2 *in, double2 *out,
                     dl::StepStat *stat, double *partials, bool folded, const KeepDst &keep)
{
    hipStream_t st = ctx->stream;
    double reps, rabs;
    store_rounding(ctx->p, reps, rabs);
    // the last iteration's partials (run_build leaves them for this kernel)
    const dl::TailFold fold{partials_half(partials, e.m), ctx->tiles_pass(e.m).nblocks,
                            (e.m >= 2 && !folded) ? e.m : 0};
    DL_HIP(ctx, ctx->timed(3, [&] { dl::launch_tridiag(e.alpha, e.gamma, e.sc, stat, reps, rabs, fold, st); }));
    dl::CombArgs r{};
    r.psi = in;
    r.basis = e.basis;
    r.vec_bytes = e.vstride;
    r.sites = vec_elems(ctx->p) / 2;
    r.out = out;
    r.sc = e.sc;
    r.partials = partials;
    r.stat = stat;
    r.alpha = e.alpha;
    r.gamma = e.gamma;
    r.keep = keep.dst;
    r.keep_alpha = keep.off_alpha;
    r.keep_gamma = keep.off_gamma;
    r.keep_nab = keep.nab;
    DL_HIP(ctx, ctx->timed(4, [&] {
        dl::launch_combine(r, e.mixed, ctx->combine_wide, ctx->combine_blocks_wide, st);
    }));
    return DL_OK;
}

// A failure of an earlier asynchronous call that dirac_lanczos_wait has not
// reported yet: synchronise, read the scalars, and report and clear it.
dl_status take_async_failure(dl_context *ctx)
{
    if (!ctx->async_pending) return DL_OK;
    ctx->async_pending = false;
    DL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    dl::Scalars hs;
    DL_HIP(ctx, hipMemcpy(&hs, ctx->sc(), sizeof(hs), hipMemcpyDeviceToHost));
    if (hs.status == 0) return DL_OK;
    dl::launch_reset(ctx->sc(), ctx->stream);
    DL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in an asynchronous call after " +
                                           std::to_string(hs.steps_done) + " of its steps");
}

}  // namespace dlh

namespace {
thread_local std::string g_init_error;
}  // namespace

using namespace dlh;

// Rounds of resident waves per recurrence sweep, and a cap on the waves per
// compute unit of a sweep (0: as many as fit).  Build-time tuning parameters;
// eight waves per compute unit (two per SIMD) measured best on the 4096^2
// workload: more concurrent row streams lower the DRAM efficiency.
#ifndef DL_RECUR_ROUNDS
#define DL_RECUR_ROUNDS 1
#endif
#ifndef DL_RECUR_WAVES_PER_CU
#define DL_RECUR_WAVES_PER_CU 4
#endif

namespace {

// Launch shapes of the sweeps: one resident round of waves per sweep (each
// wave marches its row chunk), with at most `cap` waves per compute unit
// (0: the default).  The default keeps row chunks at 24 rows or more where
// the grid allows, between 2 and DL_RECUR_WAVES_PER_CU waves per compute unit:
// on small grids short chunks spend their time in the march prologue
// (measured per step, FP64: 512^2 m = 12 278 -> 222 us, 1024^2 m = 20
// 1034 -> 769 us).  Four waves (one per SIMD, one workgroup per compute
// unit) is the cap: with the FIFO of loads really in flight, fewer and
// longer row streams use the DRAM better (dominant sweep, 4096^2 mixed:
// 4 waves 154 us, 8 waves 167 us; 2048^2 52 vs 67 us; FP64 alike).
int default_sweep_waves(const dl_params &p, int cus)
{
    const long strips = (p.nx + 59) / 60;
    const long w = strips * (long)p.ny / (24L * cus);
    return (int)std::max(2L, std::min<long>(w, DL_RECUR_WAVES_PER_CU));
}

void set_tiles(dl_context *ctx, int cap)
{
    const dl_params &p = ctx->p;
    const int lim = cap > 0 ? cap : default_sweep_waves(p, ctx->cus);
    auto capw = [&](int w) { return lim > 0 ? std::max(1, std::min(w, lim)) : w; };
    const bool mixed = p.precision == DL_PREC_MIXED;
    const bool py = p.bc_y != 0;
    const int site = dl::sweep_terms(ctx->op(1.0));
    const int wf = capw(dl::sweep_waves_per_cu(0, mixed, py, site));
    const int wr = capw(dl::sweep_waves_per_cu(1, mixed, py, site));
    const int wa = dl::sweep_waves_per_cu(4, mixed, py, site);
    const int w2 = capw(dl::sweep_waves_per_cu(2, mixed, py, site));
    const int w3 = capw(dl::sweep_waves_per_cu(3, mixed, py, site));
    ctx->sweep_waves = wr;
    ctx->tiles_first = dl::make_tiles(p.nx, p.ny, 1, wf * ctx->cus);
    ctx->tiles_recur = dl::make_tiles(p.nx, p.ny, 2, wr * ctx->cus * DL_RECUR_ROUNDS);
    ctx->tiles_p2 = dl::make_tiles(p.nx, p.ny, 2, w2 * ctx->cus * DL_RECUR_ROUNDS);
    ctx->tiles_p3 = dl::make_tiles(p.nx, p.ny, 2, w3 * ctx->cus * DL_RECUR_ROUNDS);
    ctx->tiles_apply = dl::make_tiles(p.nx, p.ny, 1, wa * ctx->cus);
    // the accumulation of the second run takes the narrow complex64 form and
    // the 8-site FP64 form
    ctx->combine_blocks = dl::combine_grid(vec_elems(p) / 2, mixed, ctx->cus, !mixed);
    ctx->combine_wide = dl::combine_wide(vec_elems(p) / 2, mixed, ctx->cus);
    ctx->combine_blocks_wide = dl::combine_grid(vec_elems(p) / 2, mixed, ctx->cus, ctx->combine_wide);
}

}  // namespace

void dlh::configure_launch(dl_context *ctx) { set_tiles(ctx, 0); }

extern "C" {

size_t dirac_lanczos_workspace_bytes(const dl_params *params, int32_t mode, int32_t k_eigen)
{
    if (validate(params)) return 0;
    if (mode != DL_MODE_STEP && mode != DL_MODE_EIGEN && mode != DL_MODE_LOWMEM && mode != DL_MODE_EIGEN_REORTH)
        return 0;
    const bool eig = mode == DL_MODE_EIGEN || mode == DL_MODE_EIGEN_REORTH;
    if (eig && (k_eigen < 1 || k_eigen > 1000000)) return 0;
    return plan(*params, mode, eig ? k_eigen : 0).total;
}

dl_status dirac_lanczos_init(const dl_params *params, void *workspace, size_t ws_bytes,
                             void *hip_stream, dl_context **out)
{
    if (!out) {
        g_init_error = "out is NULL";
        return DL_ERR_INVALID;
    }
    *out = nullptr;
    if (const char *msg = validate(params)) {
        g_init_error = msg;
        return DL_ERR_INVALID;
    }
    // the smaller of the stored-basis and the second-run layouts; step() and
    // step_lowmem() check their own need
    Layout L = plan(*params, DL_MODE_STEP, 0);
    const Layout Lm = plan(*params, DL_MODE_LOWMEM, 0);
    if (Lm.total < L.total) L = Lm;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) {
        g_init_error = "workspace must be a non-NULL, 256-byte aligned device pointer";
        return DL_ERR_WORKSPACE;
    }
    if (ws_bytes < L.total) {
        g_init_error = "workspace too small: need " + std::to_string(L.total) + " bytes";
        return DL_ERR_WORKSPACE;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        g_init_error = "no HIP device";
        return DL_ERR_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_init_error = std::string("built for gfx950 only, device is ") + prop.gcnArchName;
        return DL_ERR_DEVICE;
    }
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        g_init_error = "workspace is not device memory";
        return DL_ERR_WORKSPACE;
    }
    dl_context *ctx = new dl_context();
    ctx->p = *params;
    if (params->pulse_kind == 2) ctx->coef.assign(params->coef, params->coef + params->n_coef);
    ctx->p.coef = nullptr;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->ws = static_cast<char *>(workspace);
    ctx->ws_bytes = ws_bytes;
    ctx->L = L;
    ctx->cus = prop.multiProcessorCount;
    set_tiles(ctx, 0);
    dl::launch_reset(ctx->sc(), ctx->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_init_error = std::string("kernel launch failed: ") + hipGetErrorString(e);
        delete ctx;
        return DL_ERR_DEVICE;
    }
    *out = ctx;
    return DL_OK;
}

dl_status dirac_lanczos_apply(dl_context *ctx, const void *x, void *y, double t)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!x || !y || x == y) return ctx->fail(DL_ERR_INVALID, "apply needs distinct non-NULL x and y");
    if (!std::isfinite(t)) return ctx->fail(DL_ERR_INVALID, "t must be finite");
    const dl::Op op = ctx->op(1.0);
    double a[2];
    pulse_now(ctx->p, ctx->coef, t, a);
    const double k = -ctx->p.c * ctx->p.charge;
    dl::launch_apply(op, ctx->tiles_apply, static_cast<const double2 *>(x), static_cast<double2 *>(y), k * a[0],
                     k * chir(ctx->p) * a[1], ctx->stream);
    DL_HIP(ctx, hipGetLastError());
    return DL_OK;
}

// Stage the per-step fields of steps s0 .. s0+nc-1 into a pinned buffer (for
// an asynchronous upload) or the context's pageable one.
static dl_status stage_fields(dl_context *ctx, bool async, double t0, double dt, int s0, int nc, double *dev)
{
    const dl_params &p = ctx->p;
    const double kf = -dt * p.c * p.charge;
    double *h;
    if (async) {
        const int b = ctx->pin_next;
        ctx->pin_next ^= 1;
        if (!ctx->pin_fields[b]) {
            DL_HIP(ctx, hipHostMalloc(reinterpret_cast<void **>(&ctx->pin_fields[b]), sizeof(double) * 2 * kChunk,
                                      hipHostMallocDefault));
            DL_HIP(ctx, hipEventCreateWithFlags(&ctx->pin_ev[b], hipEventDisableTiming));
        } else {
            DL_HIP(ctx, hipEventSynchronize(ctx->pin_ev[b]));  // its previous upload has been consumed
        }
        h = ctx->pin_fields[b];
        for (int i = 0; i < nc; ++i) {
            double a[2];
            pulse_average(p, ctx->coef, t0 + (double)(s0 + i) * dt, dt, a);
            h[2 * i] = kf * a[0];
            h[2 * i + 1] = kf * chir(p) * a[1];
        }
        DL_HIP(ctx, hipMemcpyAsync(dev, h, sizeof(double) * 2 * nc, hipMemcpyHostToDevice, ctx->stream));
        DL_HIP(ctx, hipEventRecord(ctx->pin_ev[b], ctx->stream));
        return DL_OK;
    }
    ctx->host_fields.resize(2 * kChunk);
    h = ctx->host_fields.data();
    for (int i = 0; i < nc; ++i) {
        double a[2];
        pulse_average(p, ctx->coef, t0 + (double)(s0 + i) * dt, dt, a);
        h[2 * i] = kf * a[0];
        h[2 * i + 1] = kf * chir(p) * a[1];
    }
    DL_HIP(ctx, hipMemcpyAsync(dev, h, sizeof(double) * 2 * nc, hipMemcpyHostToDevice, ctx->stream));
    return DL_OK;
}

static dl_status run_steps(dl_context *ctx, void *psi_v, double t0, double dt, int32_t n_steps,
                           dl_step_stat *stats, bool lowmem, double ktol = 0.0, int kmin = 0)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!psi_v) return ctx->fail(DL_ERR_INVALID, "psi is NULL");
    if (n_steps < 0) return ctx->fail(DL_ERR_INVALID, "n_steps must be >= 0");
    if (!(dt != 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
        return ctx->fail(DL_ERR_INVALID, "dt must be finite and non-zero, t0 finite");
    const bool async = stats == nullptr;
    if (!async) {
        const dl_status pend = take_async_failure(ctx);
        if (pend != DL_OK) return pend;
    }
    if (n_steps == 0) return DL_OK;
    const dl_params &p = ctx->p;
    const size_t need = plan(p, lowmem ? DL_MODE_LOWMEM : DL_MODE_STEP, 0).total;
    if (ctx->ws_bytes < need)
        return ctx->fail(DL_ERR_WORKSPACE, std::string("workspace too small for ") +
                                               (lowmem ? "the second-run mode" : "the stored Krylov basis") +
                                               ": need " + std::to_string(need) + " bytes");
    const int m = p.krylov_dim;
    const bool mixed = p.precision == DL_PREC_MIXED;
    const size_t n = vec_elems(p);
    const size_t belem = mixed ? 8 : 16;
    char *ws = ctx->ws;
    const Layout &L = ctx->L;
    dl::Scalars *sc = ctx->sc();
    double *alpha = reinterpret_cast<double *>(ws + L.alpha);
    double *gamma = reinterpret_cast<double *>(ws + L.gamma);
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    double *fields = reinterpret_cast<double *>(ws + L.fields);
    dl::StepStat *dstats = reinterpret_cast<dl::StepStat *>(ws + L.stats);
    double2 *psi = static_cast<double2 *>(psi_v);
    double2 *state = reinterpret_cast<double2 *>(ws + L.vecs);
    char *basis = ws + L.vecs + align256(n * 16);
    const size_t vstride = vec_stride(n, belem);
    const Engine eng{sc, alpha, gamma, basis, vstride, m, mixed};

    const dl::Op op = ctx->op(dt);
    hipStream_t st = ctx->stream;

    // adaptive dimension (ktol > 0): the first step runs m iterations, later
    // ones the dimension the previous step predicted
    dl::launch_reset_call(sc, async ? 1 : 0, ktol > 0.0 ? kmin : 0, ktol > 0.0 ? m : 0, ktol > 0.0 ? ktol : 0.0,
                          st);
    DL_HIP(ctx, hipGetLastError());
    double cum = 0.0;
    int completed = 0;
    bool aborted = false;
    ctx->host_stats.resize(kChunk);
    for (int s0 = 0; s0 < n_steps && !aborted; s0 += kChunk) {
        const int nc = std::min(kChunk, n_steps - s0);
        const dl_status sf = stage_fields(ctx, async, t0, dt, s0, nc, fields);
        if (sf != DL_OK) return sf;
        for (int i = 0; i < nc; ++i) {
            const int g = s0 + i;
            double2 *in = (g % 2 == 0) ? psi : state;
            double2 *out = (g % 2 == 0) ? state : psi;
            const double *fp = fields + 2 * i;
            const dl_status sb = lowmem ? run_twice(ctx, eng, op, in, out, fp, dstats + i, partials)
                                        : run_build(ctx, eng, op, in, fp, partials, 1);
            if (sb != DL_OK) return sb;
            if (!lowmem) {
                const dl_status sr = run_finish(ctx, eng, in, out, dstats + i, partials);
                if (sr != DL_OK) return sr;
            }
        }
        DL_HIP(ctx, hipGetLastError());
        if (async) {
            ctx->async_s0 = s0;
            ctx->async_nc = nc;
            continue;
        }
        dl::Scalars hs;
        DL_HIP(ctx, hipMemcpyAsync(ctx->host_stats.data(), dstats, sizeof(dl::StepStat) * nc,
                                   hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        const int done_here = hs.steps_done - completed;
        for (int i = 0; i < nc; ++i) {
            dl_step_stat &o = stats[s0 + i];
            if (i < done_here) {
                cum += ctx->host_stats[i].err_est;
                o.k_eff = ctx->host_stats[i].keff;
                o.err_est = ctx->host_stats[i].err_est;
                o.cum_bound = cum;
                o.norm2 = ctx->host_stats[i].norm2;
                o.round_bound = ctx->host_stats[i].round_bound;
            } else {
                o.k_eff = -1;
                o.err_est = o.cum_bound = o.norm2 = o.round_bound = 0.0;
            }
        }
        completed = hs.steps_done;
        if (hs.status != 0) aborted = true;
    }
    if (async) {
        // the state after the completed steps is copied to psi on the device
        dl::launch_finish_copy(sc, state, psi, n, ctx->cus, st);
        DL_HIP(ctx, hipGetLastError());
        ctx->async_pending = true;
        return DL_OK;
    }
    if (aborted)
        for (int i = completed; i < n_steps; ++i) {
            stats[i].k_eff = -1;
            stats[i].err_est = stats[i].cum_bound = stats[i].norm2 = stats[i].round_bound = 0.0;
        }
    // the state after `completed` steps sits in psi (even) or in the workspace (odd)
    if (completed % 2 == 1) {
        DL_HIP(ctx, hipMemcpyAsync(psi, state, n * 16, hipMemcpyDeviceToDevice, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
    }
    if (aborted)
        return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction after " +
                                               std::to_string(completed) + " completed steps");
    return DL_OK;
}

dl_status dirac_lanczos_step(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps,
                             dl_step_stat *stats)
{
    return run_steps(ctx, psi, t0, dt, n_steps, stats, false);
}

dl_status dirac_lanczos_step_lowmem(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps,
                                    dl_step_stat *stats)
{
    return run_steps(ctx, psi, t0, dt, n_steps, stats, true);
}

dl_status dirac_lanczos_step_ktol(dl_context *ctx, void *psi, double t0, double dt, int32_t n_steps, double tol,
                                  int32_t k_min, dl_step_stat *stats)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!(tol > 0.0) || !std::isfinite(tol)) return ctx->fail(DL_ERR_INVALID, "tol must be finite and > 0");
    if (k_min < 1 || k_min > ctx->p.krylov_dim)
        return ctx->fail(DL_ERR_INVALID, "k_min must be in 1..krylov_dim");
    return run_steps(ctx, psi, t0, dt, n_steps, stats, false, tol, k_min);
}

dl_status dirac_lanczos_eigen(dl_context *ctx, const void *psi0, int32_t k_max, int32_t reorth,
                              double e_lo, double e_hi, double tol, int32_t n_wanted, double *evals,
                              double *bounds, int32_t *n_found)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!psi0 || !evals || !bounds || !n_found || n_wanted < 1 || k_max < 1 || !(tol >= 0.0) ||
        !(e_hi >= e_lo))
        return ctx->fail(DL_ERR_INVALID, "invalid eigen arguments");
    *n_found = 0;
    const dl_status pend = take_async_failure(ctx);
    if (pend != DL_OK) return pend;
    if (reorth) return eigen_reorth(ctx, psi0, k_max, e_lo, e_hi, tol, n_wanted, evals, bounds, n_found, nullptr);
    const dl_params &p = ctx->p;
    const Layout E = plan(p, DL_MODE_EIGEN, k_max);
    if (ctx->ws_bytes < E.total)
        return ctx->fail(DL_ERR_WORKSPACE, "workspace too small for eigen mode: need " +
                                               std::to_string(E.total) + " bytes");
    const size_t n = vec_elems(p);
    char *ws = ctx->ws;
    dl::Scalars *sc = ctx->sc();
    double *alpha = reinterpret_cast<double *>(ws + E.alpha);
    double *gamma = reinterpret_cast<double *>(ws + E.gamma);
    double *partials = reinterpret_cast<double *>(ws + E.partials);
    double *fields = reinterpret_cast<double *>(ws + E.fields);
    double2 *v[3];
    for (int i = 0; i < 3; ++i) v[i] = reinterpret_cast<double2 *>(ws + E.vecs + i * vec_stride(n, 16));
    hipStream_t st = ctx->stream;
    const dl::Op op = ctx->op(1.0);
    const dl::Tiles &t1 = ctx->tiles_first;
    // the eigen sweeps run the complex128 kernels whatever the context precision
    dl::Tiles tp[3];
    for (int kind = 0; kind < 3; ++kind)
        tp[kind] = dl::make_tiles(
            p.nx, p.ny, 2,
            std::min(default_sweep_waves(p, ctx->cus),
                     dl::sweep_waves_per_cu(kind == 2 ? 1 : kind + 2, false, p.bc_y != 0, dl::sweep_terms(op))) *
                ctx->cus);
    const double zero[2] = {0.0, 0.0};
    DL_HIP(ctx, hipMemcpyAsync(fields, zero, sizeof(zero), hipMemcpyHostToDevice, st));
    DL_HIP(ctx, hipMemcpyAsync(v[1], psi0, n * 16, hipMemcpyDeviceToDevice, st));
    dl::launch_reset(sc, st);
    const int K1 = k_max + 1;  // the extra iteration yields beta_k for the bounds
    dl::launch_first(op, t1, v[1], fields, alpha, gamma, sc, partials, K1, 0, st);
    std::vector<double> ha(K1 + 1), hg(K1 + 1);
    dl::Scalars hs;
    auto fetch = [&]() -> dl_status {
        DL_HIP(ctx, hipMemcpyAsync(ha.data(), alpha, sizeof(double) * (K1 + 1), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipMemcpyAsync(hg.data(), gamma, sizeof(double) * (K1 + 1), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        if (hs.status != 0) return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in eigen mode");
        return DL_OK;
    };
    // T_k after pass p: alpha_1..alpha_k in ha[1..], beta_1..beta_k in hg[2..]
    // (gamma_{j+1} = beta_j), so k = p - 1 is complete after pass p.  Converged
    // clusters are accumulated over the checkpoints k = 64, 128, ... and the
    // final k (merge_converged).
    std::vector<std::pair<double, double>> found;
    std::vector<double> ev((size_t)k_max + 1), bd(ev.size());  // at most k Ritz values per T_k
    auto harvest = [&](int k) {
        const int nf = ritz_chain(ha.data() + 1, hg.data() + 2, k, e_lo, e_hi, tol, (int)ev.size(), ev.data(),
                                  bd.data(), nullptr, nullptr);
        merge_converged(found, ev.data(), bd.data(), nf, tol);
    };
    int pending = 0;  // checkpoint fetched but not yet solved
    for (int pp = 2; pp <= K1; ++pp) {
        dl::PassArgs a{};
        a.op = op;
        a.t = tp[pp == 2 ? 0 : (pp == 3 ? 1 : 2)];
        a.u1 = v[(pp - 1) % 3];
        a.u2 = pp >= 3 ? v[(pp - 2) % 3] : nullptr;
        a.uo = v[pp % 3];
        a.field = fields;
        a.alpha = alpha;
        a.gamma = gamma;
        a.sc = sc;
        a.partials = partials;
        a.pass = pp;
        a.m = K1;
        dl::launch_recur(a, false, st);
        if ((pp - 1) % kEigenCheckEvery == 0 && pp < K1) {
            DL_HIP(ctx, hipGetLastError());
            // the previous checkpoint is solved while the device runs the
            // passes since then; the decision to stop is the same, only the
            // passes queued meanwhile are extra work
            if (pending > 0) {
                harvest(pending);
                pending = 0;
                if ((int)found.size() >= n_wanted) break;
            }
            const dl_status s = fetch();
            if (s != DL_OK) return s;
            if (hs.kstop < pp) break;  // breakdown: the recurrence is over
            pending = pp - 1;
        }
    }
    DL_HIP(ctx, hipGetLastError());
    const dl_status s = fetch();
    if (s != DL_OK) return s;
    if (pending > 0) harvest(pending);
    if ((int)found.size() < n_wanted) {
        const int k = std::min(hs.keff, k_max);
        if (k > 0) harvest(k);
    }
    const int nf = std::min((int)found.size(), n_wanted);
    for (int i = 0; i < nf; ++i) {
        evals[i] = found[i].first;
        bounds[i] = found[i].second;
    }
    *n_found = nf;
    return DL_OK;
}

dl_status dirac_lanczos_wait(dl_context *ctx, dl_step_stat *stats, int32_t n_stats, int32_t *steps_done)
{
    if (!ctx) return DL_ERR_INVALID;
    if (n_stats < 0 || (n_stats > 0 && !stats)) return ctx->fail(DL_ERR_INVALID, "stats must hold n_stats entries");
    DL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    dl::Scalars hs;
    DL_HIP(ctx, hipMemcpy(&hs, ctx->sc(), sizeof(hs), hipMemcpyDeviceToHost));
    if (steps_done) *steps_done = hs.steps_done;
    const int nc = ctx->async_pending ? ctx->async_nc : 0;
    const int nfill = std::min(n_stats, nc);
    if (nfill > 0) {
        ctx->host_stats.resize(kChunk);
        DL_HIP(ctx, hipMemcpy(ctx->host_stats.data(), ctx->ws + ctx->L.stats, sizeof(dl::StepStat) * nc,
                              hipMemcpyDeviceToHost));
        const int done_here = hs.steps_done - ctx->async_s0;
        double cum = 0.0;
        for (int i = 0; i < nfill; ++i) {
            dl_step_stat &o = stats[i];
            if (i < done_here) {
                cum += ctx->host_stats[i].err_est;
                o.k_eff = ctx->host_stats[i].keff;
                o.err_est = ctx->host_stats[i].err_est;
                o.cum_bound = cum;
                o.norm2 = ctx->host_stats[i].norm2;
                o.round_bound = ctx->host_stats[i].round_bound;
            } else {
                o.k_eff = -1;
                o.err_est = o.cum_bound = o.norm2 = o.round_bound = 0.0;
            }
        }
    }
    for (int i = nfill; i < n_stats; ++i) {
        stats[i].k_eff = -1;
        stats[i].err_est = stats[i].cum_bound = stats[i].norm2 = stats[i].round_bound = 0.0;
    }
    ctx->async_pending = false;
    if (hs.status != 0) {
        dl::launch_reset(ctx->sc(), ctx->stream);
        DL_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction after " + std::to_string(hs.steps_done) +
                                               " completed steps of the last call");
    }
    return DL_OK;
}

dl_status dirac_lanczos_set_launch(dl_context *ctx, int32_t sweep_waves_per_cu, int32_t *waves_out)
{
    if (!ctx) return DL_ERR_INVALID;
    if (sweep_waves_per_cu < 0 || sweep_waves_per_cu > 64)
        return ctx->fail(DL_ERR_INVALID, "sweep_waves_per_cu must be in 0..64");
    set_tiles(ctx, sweep_waves_per_cu);
    if (waves_out) *waves_out = ctx->sweep_waves;
    return DL_OK;
}

dl_status dirac_lanczos_timing(dl_context *ctx, int32_t enable, dl_timing *out)
{
    if (!ctx) return DL_ERR_INVALID;
    DL_HIP(ctx, ctx->harvest());
    if (out) {
        for (int i = 0; i < 5; ++i) {
            out->launches[i] = ctx->t_launches[i];
            out->total_ms[i] = ctx->t_ms[i];
        }
    }
    if (enable) {
        if (ctx->ev0.empty()) {
            const size_t n = 512;
            ctx->ev0.resize(n);
            ctx->ev1.resize(n);
            ctx->ev_cls.resize(n);
            ctx->ev_cnt.resize(n);
            for (size_t i = 0; i < n; ++i) {
                DL_HIP(ctx, hipEventCreate(&ctx->ev0[i]));
                DL_HIP(ctx, hipEventCreate(&ctx->ev1[i]));
            }
        }
        for (int i = 0; i < 5; ++i) {
            ctx->t_launches[i] = 0;
            ctx->t_ms[i] = 0.0;
        }
        ctx->timing = true;
    } else {
        ctx->timing = false;
    }
    return DL_OK;
}

dl_status dirac_lanczos_destroy(dl_context *ctx)
{
    delete ctx;
    return DL_OK;
}

const char *dirac_lanczos_last_error(const dl_context *ctx)
{
    if (!ctx) return g_init_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"
