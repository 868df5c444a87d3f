// Adaptive time steps (C ABI dirac_lanczos_step_adaptive).
//
// Two errors enter a step of size h from t.  The Krylov error of
// exp(-i h H) (Sec. 4, eq. matrix_exponential_error, which the paper notes
// can steer the step size) behaves like h^k.  With a time-dependent field the
// step also replaces H(s) by its average over the step (the first Magnus
// term, Sec. 3, eq. time_evolution_approx).  That part is bounded exactly:
// with psi_a the piecewise propagation and psi_e the exact one,
// i (psi_a - psi_e)' = H(s) (psi_a - psi_e) + (H_bar - H(s)) psi_a, and
// H_bar - H(s) = -c q (a_bar - a(s)) . (sigma1, chi sigma2) has norm
// c |q| |a_bar - a(s)| on any spinor, so the step adds at most
// c |q| ||psi|| int_t^{t+h} |a(s) - a_bar| ds (unitary propagation keeps it).
// The integral is taken by composite Gauss-Legendre quadrature (64 panels of
// three nodes; the integrand is Lipschitz with a kink where a(s) = a_bar, so a
// 1% margin keeps the quadrature on the safe side).  The step's estimate is
// the Krylov estimate plus this bound.  Reading used here: the cumulative
// estimate over [t0, t_end] is to stay below tol, so a step of size h may
// spend tol * h / (t_end - t0).  A step over its share is rejected (the state
// is untouched: a step writes into the ping-pong partner) and retried
// smaller; after every step h is rescaled by 0.9 (share / estimate)^e with
// e = 1 where the field part dominates (it grows like h^2 against the share's
// h) and 1/(k-1) otherwise, at most x2 and at least x1/4, within
// [dt_min, dt_max], and the last step lands on t_end exactly.
#include <algorithm>
#include <cmath>
#include <string>

#include "context.h"

using namespace dlh;

namespace {

// int_t^{t+h} |a(s) - a_bar| ds for the homogeneous laser field (h > 0).
double field_deviation(const dl_params &p, CoefView coef, double t, double h)
{
    if (p.pulse_kind == 0 || t >= p.t_pulse || t + h <= 0.0) return 0.0;
    static const double gx[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
    static const double gw[3] = {0.5555555555555556, 0.8888888888888888, 0.5555555555555556};
    constexpr int kPanels = 64;
    double abar[2];
    pulse_average(p, coef, t, h, abar);
    const double ph = h / kPanels;
    double tot = 0.0;
    for (int k = 0; k < kPanels; ++k) {
        const double mid = t + (k + 0.5) * ph;
        for (int q = 0; q < 3; ++q) {
            double a[2];
            pulse_now(p, coef, mid + 0.5 * ph * gx[q], a);
            tot += 0.5 * ph * gw[q] * std::hypot(a[0] - abar[0], a[1] - abar[1]);
        }
    }
    return 1.01 * tot;
}

}  // namespace

extern "C" {

dl_status dirac_lanczos_step_adaptive(dl_context *ctx, void *psi_v, double t0, double t_end, double dt_init,
                                      double tol, double dt_min, double dt_max, int32_t max_steps,
                                      double *dt_taken, dl_adapt_stat *out)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!psi_v || !out) return ctx->fail(DL_ERR_INVALID, "psi and out must be non-NULL");
    if (!std::isfinite(t0) || !std::isfinite(t_end) || !(t_end > t0))
        return ctx->fail(DL_ERR_INVALID, "need finite t0 < t_end");
    if (!(tol > 0.0) || !(dt_min > 0.0) || !(dt_max >= dt_min) || !(dt_init > 0.0) || !std::isfinite(dt_max))
        return ctx->fail(DL_ERR_INVALID, "need tol > 0 and 0 < dt_min <= dt_max, dt_init > 0");
    if (max_steps < 1) return ctx->fail(DL_ERR_INVALID, "max_steps must be >= 1");
    const dl_params &p = ctx->p;
    const int m = p.krylov_dim;
    if (ctx->ws_bytes < plan(ctx->p, DL_MODE_STEP, 0).total)
        return ctx->fail(DL_ERR_WORKSPACE, "context workspace too small for the stored Krylov basis (DL_MODE_STEP)");
    const bool mixed = p.precision == DL_PREC_MIXED;
    const size_t n = vec_elems(p);
    char *ws = ctx->ws;
    const Layout &L = ctx->L;
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    double *fields = reinterpret_cast<double *>(ws + L.fields);
    dl::StepStat *dstat = reinterpret_cast<dl::StepStat *>(ws + L.stats);
    double2 *psi = static_cast<double2 *>(psi_v);
    double2 *state = reinterpret_cast<double2 *>(ws + L.vecs);
    const Engine eng{ctx->sc(), reinterpret_cast<double *>(ws + L.alpha), reinterpret_cast<double *>(ws + L.gamma),
                     ws + L.vecs + align256(n * 16), vec_stride(n, mixed ? 8 : 16), m, mixed};
    hipStream_t st = ctx->stream;
    const double span = t_end - t0;
    const double expo_k = 1.0 / std::max(1, m - 1);
    const double cq = p.c * std::fabs(p.charge);

    *out = dl_adapt_stat{};
    out->t_reached = t0;
    double t = t0, dt = std::min(std::max(dt_init, dt_min), dt_max), cum = 0.0, cum_mag = 0.0;
    double2 *cur = psi, *nxt = state;
    const dl_status pend = take_async_failure(ctx);
    if (pend != DL_OK) return pend;
    dl::launch_reset(eng.sc, st);
    DL_HIP(ctx, hipGetLastError());
    dl_status result = DL_OK;
    std::string why;
    while (t < t_end) {
        if (out->accepted + out->rejected >= max_steps) {
            result = DL_ERR_INVALID;
            why = "max_steps reached before t_end";
            break;
        }
        const bool last = t_end - t <= dt * (1.0 + 1e-12);
        const double h = last ? t_end - t : dt;
        double a[2], f[2];
        pulse_average(p, ctx->coef, t, h, a);
        f[0] = -h * p.c * p.charge * a[0];
        f[1] = -h * p.c * p.charge * chir(p) * a[1];
        DL_HIP(ctx, hipMemcpyAsync(fields, f, sizeof(f), hipMemcpyHostToDevice, st));
        const dl::Op op = ctx->op(h);
        dl_status s = run_build(ctx, eng, op, cur, fields, partials, 1);
        if (s != DL_OK) return s;
        s = run_finish(ctx, eng, cur, nxt, dstat, partials);
        if (s != DL_OK) return s;
        dl::StepStat hs;
        int status = 0;
        DL_HIP(ctx, hipMemcpyAsync(&hs, dstat, sizeof(hs), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipMemcpyAsync(&status, &eng.sc->status, sizeof(int), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        if (status != 0) {
            result = DL_ERR_NONFINITE;
            why = "non-finite Lanczos reduction";
            break;
        }
        const double share = tol * h / span;
        // ||psi|| before the step: the norm is conserved up to the estimate
        const double est_m = cq * std::sqrt(hs.norm2) * field_deviation(p, ctx->coef, t, h);
        const double est = hs.err_est + est_m;
        const double expo = est_m > hs.err_est ? 1.0 : expo_k;
        const double factor = est > 0.0 ? std::min(2.0, std::max(0.25, 0.9 * std::pow(share / est, expo))) : 2.0;
        if (est <= share) {
            if (dt_taken) dt_taken[out->accepted] = h;
            out->accepted += 1;
            cum += est;
            cum_mag += est_m;
            t = last ? t_end : t + h;
            out->norm2 = hs.norm2;
            std::swap(cur, nxt);
            if (!last) dt = std::min(dt_max, std::max(dt_min, h * factor));
        } else {
            out->rejected += 1;
            if (h <= dt_min) {
                result = DL_ERR_INVALID;
                why = "the tolerance needs a step below dt_min";
                break;
            }
            dt = std::max(dt_min, h * std::min(factor, 0.5));
        }
    }
    out->t_reached = t;
    out->cum_bound = cum;
    out->cum_magnus = cum_mag;
    out->dt_next = dt;
    if (cur != psi) {
        DL_HIP(ctx, hipMemcpyAsync(psi, cur, n * 16, hipMemcpyDeviceToDevice, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
    }
    if (result != DL_OK) return ctx->fail(result, why + " (state at t = " + std::to_string(t) + ")");
    return DL_OK;
}

}  // extern "C"
