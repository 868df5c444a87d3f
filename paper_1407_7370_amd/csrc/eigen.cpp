// Eigenvalue mode with full reorthogonalisation and Ritz vectors (C ABI
// dirac_lanczos_eigen with reorth != 0, dirac_lanczos_eigen_vectors).
//
// Sec. 2: the Lanczos vectors lose orthogonality once Ritz values converge,
// which shows up as copies of converged values; orthogonalising every new
// vector against all stored ones, twice, prevents it.  Iteration i:
//   z = H q_i
//   h1 = Q_i^H z;  z -= Q_i h1      (first pass; removes alpha_i q_i and
//   h2 = Q_i^H z;  z -= Q_i h2       beta_{i-1} q_{i-1} as well)
//   alpha_i = Re h1_i,  beta_i = ||z||,  q_{i+1} = z / beta_i
// Ritz values and bounds follow eq. A_approx and eq. error_est (as in the
// plain mode); the Ritz vectors are y = Q_k t (eq. eigenvec_approx).
//
// Everything between the start vector and the Ritz vectors stays on the
// device: the scalars of the recurrence are updated by the last workgroup of
// the norm reduction, and the host reads the breakdown flag every
// kPollEvery iterations only (iterations past a breakdown are skipped by the
// kernels: their scalar updates are masked).  Every kEigenCheckEvery
// iterations the host also computes the Ritz values of T and stops once
// n_wanted clusters have converged.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "context.h"

namespace dlh {

namespace {
constexpr int kPollEvery = 16;
}

dl_status eigen_reorth(dl_context *ctx, const void *psi0, int k_max, double e_lo, double e_hi, double tol,
                       int n_wanted, double *evals, double *bounds, int32_t *n_found, void *vecs)
{
    const dl_params &p = ctx->p;
    const Layout E = plan(p, DL_MODE_EIGEN_REORTH, k_max);
    if (ctx->ws_bytes < E.total)
        return ctx->fail(DL_ERR_WORKSPACE, "workspace too small for eigen mode with full reorthogonalisation "
                                           "(DL_MODE_EIGEN_REORTH): need " +
                                               std::to_string(E.total) + " bytes");
    const size_t n = vec_elems(p);
    const size_t vs = vec_stride(n, 16);
    const ReorthLayout R = reorth_layout(n, k_max);
    char *ws = ctx->ws;
    char *vreg = ws + E.vecs;
    dl::Scalars *sc = ctx->sc();
    double *alpha = reinterpret_cast<double *>(ws + E.alpha);
    double *beta = reinterpret_cast<double *>(ws + E.gamma);
    double *partials = reinterpret_cast<double *>(ws + E.partials);
    double2 *z = reinterpret_cast<double2 *>(vreg + R.z);
    char *Q = vreg + R.q;
    auto qv = [&](int j) { return reinterpret_cast<double2 *>(Q + (size_t)(j - 1) * vs); };  // q_j, 1-based
    double *h1 = reinterpret_cast<double *>(vreg + R.h1);
    double *h2 = reinterpret_cast<double *>(vreg + R.h2);
    double *pproj = reinterpret_cast<double *>(vreg + R.pproj);
    double *tsel = reinterpret_cast<double *>(vreg + R.tsel);
    hipStream_t st = ctx->stream;
    const dl::Op op = ctx->op(1.0);
    // streaming kernels: a few workgroups per compute unit, never more than tiles
    const size_t tiles = (n + dl::kBlock - 1) / dl::kBlock;
    const int nb = (int)std::max<size_t>(1, std::min<size_t>(tiles, (size_t)8 * ctx->cus));

    const dl_status pend = take_async_failure(ctx);
    if (pend != DL_OK) return pend;
    dl::launch_reset(sc, st);
    dl::launch_first_q(static_cast<const double2 *>(psi0), n, qv(1), sc, beta, partials, nb, st);
    DL_HIP(ctx, hipGetLastError());
    std::vector<double> ha(k_max + 1), hb(k_max + 1);
    dl::Scalars hs;
    auto fetch = [&](bool chain) -> dl_status {
        if (chain) {
            DL_HIP(ctx, hipMemcpyAsync(ha.data(), alpha, sizeof(double) * (k_max + 1), hipMemcpyDeviceToHost, st));
            DL_HIP(ctx, hipMemcpyAsync(hb.data(), beta, sizeof(double) * (k_max + 1), hipMemcpyDeviceToHost, st));
        }
        DL_HIP(ctx, hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        return DL_OK;
    };
    // T_k after iteration k: alpha_1..alpha_k in ha[1..], beta_1..beta_k in hb[1..]
    int k_early = 0;
    for (int i = 1; i <= k_max; ++i) {
        if ((i - 1) % kPollEvery == 0) {
            const bool check = i > 1 && (i - 1) % kEigenCheckEvery == 0;
            const dl_status s = fetch(check);
            if (s != DL_OK) return s;
            if (hs.status != 0 || hs.kstop < i) break;
            if (check) {
                std::vector<double> ev(n_wanted), bd(n_wanted);
                if (ritz_chain(ha.data() + 1, hb.data() + 1, i - 1, e_lo, e_hi, tol, n_wanted, ev.data(), bd.data(),
                               nullptr, nullptr) >= n_wanted) {
                    k_early = i - 1;
                    break;
                }
            }
        }
        dl::launch_apply(op, ctx->tiles_apply, qv(i), z, 0.0, 0.0, st);
        dl::launch_proj(Q, vs, i, z, n, pproj, h1, st);
        dl::launch_sub_q(Q, vs, i, h1, z, n, nb, st);
        dl::launch_proj(Q, vs, i, z, n, pproj, h2, st);
        dl::launch_sub_q(Q, vs, i, h2, z, n, nb, st);
        dl::launch_norm_next(z, n, h1, i, k_max, alpha, beta, sc, partials, i < k_max ? qv(i + 1) : nullptr, nb,
                             st);
        DL_HIP(ctx, hipGetLastError());
    }
    {
        const dl_status s = fetch(true);
        if (s != DL_OK) return s;
    }
    if (hs.status != 0) return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in eigen mode");
    const int k = k_early > 0 ? k_early : std::min(hs.keff, k_max);
    if (k <= 0) return DL_OK;
    std::vector<double> V;
    std::vector<int> rep;
    const int nf = ritz_chain(ha.data() + 1, hb.data() + 1, k, e_lo, e_hi, tol, n_wanted, evals, bounds,
                              vecs ? &rep : nullptr, vecs ? &V : nullptr);
    *n_found = nf;
    if (!vecs || nf == 0) return DL_OK;
    // columns of the selected eigenvectors, kRitzVecs at a time, signed so that
    // t_1 > 0 (else the component of largest magnitude > 0)
    const int chunks = (nf + dl::kRitzVecs - 1) / dl::kRitzVecs;
    std::vector<double> tall((size_t)chunks * k * dl::kRitzVecs, 0.0);
    for (int c = 0; c < chunks; ++c) {
        const int r = std::min(dl::kRitzVecs, nf - c * dl::kRitzVecs);
        double *tc = tall.data() + (size_t)c * k * dl::kRitzVecs;
        for (int v = 0; v < r; ++v) {
            const int l = rep[c * dl::kRitzVecs + v];
            int lead = 0;
            for (int j = 1; j < k; ++j)
                if (std::fabs(V[(size_t)j * k + l]) > std::fabs(V[(size_t)lead * k + l])) lead = j;
            const double piv = V[l] != 0.0 ? V[l] : V[(size_t)lead * k + l];
            const double sgn = piv < 0.0 ? -1.0 : 1.0;
            for (int j = 0; j < k; ++j) tc[(size_t)j * dl::kRitzVecs + v] = sgn * V[(size_t)j * k + l];
        }
        DL_HIP(ctx, hipMemcpyAsync(tsel, tc, sizeof(double) * k * dl::kRitzVecs, hipMemcpyHostToDevice, st));
        dl::launch_ritz(Q, vs, k, tsel, r, static_cast<double2 *>(vecs) + (size_t)c * dl::kRitzVecs * n, n, nb,
                        st);
        DL_HIP(ctx, hipGetLastError());
    }
    DL_HIP(ctx, hipStreamSynchronize(st));
    return DL_OK;
}

}  // namespace dlh

using namespace dlh;

extern "C" {

dl_status dirac_lanczos_eigen_vectors(dl_context *ctx, const void *psi0, int32_t k_max, double e_lo, double e_hi,
                                      double tol, int32_t n_wanted, double *evals, double *bounds,
                                      int32_t *n_found, void *vecs)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!psi0 || !evals || !bounds || !n_found || !vecs || n_wanted < 1 || k_max < 1 || !(tol >= 0.0) ||
        !(e_hi >= e_lo))
        return ctx->fail(DL_ERR_INVALID, "invalid eigen_vectors arguments");
    *n_found = 0;
    return eigen_reorth(ctx, psi0, k_max, e_lo, e_hi, tol, n_wanted, evals, bounds, n_found, vecs);
}

}  // extern "C"
