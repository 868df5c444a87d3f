// Adjoint mode of the C ABI: gradient of a final observable with respect to
// the Fourier coefficients of the laser field.
//
// Forward map: psi_{n+1} = U_n psi_n, U_n = exp(-i A_n), A_n = dt H(Abar_n)
// with the step-averaged field Abar_n (first Magnus term, Sec. 3), each U_n
// applied by the Lanczos propagator of Sec. 4.  Abar_n is linear in the
// coefficients: Abar_n = sum_j coef_j w_nj with w_nj the step average of the
// j-th basis function of the sin^2-enveloped Fourier pulse.
//
// Backward pass: lam_N = (O - L) psi_N / N and lam_n = U_n^dagger lam_{n+1};
// U_n^dagger = exp(+i A_n) is one propagator step with -dt at the same field,
// so it reuses the forward kernels.  The derivative of step n is
//   <lam_{n+1}| dU_n |psi_n> = int_0^1 <lam| e^{-i s A} (-i dA) e^{-i (1-s) A} |psi> ds.
// Both half-propagations are taken in their own Krylov spaces (the backward
// one of lam_{n+1} with operator -A, the forward one of psi_n with A): with
// eigenpairs (tau_a, W) and (mu_b, V) of the two tridiagonal matrices and
// nu_a = -tau_a the s-integral becomes the divided difference
//   phi(nu, mu) = (e^{-i nu} - e^{-i mu}) / (-i (nu - mu))
//               = e^{-i (nu + mu)/2} sin(d/2) / (d/2),  d = nu - mu,
// and the matrix element needs only the basis contraction
// M_ij = <q^lam_i| sigma |q^psi_j> (kernel k_contract).  The laser enters H as
// -c q (sigma1 A_x + sigma2 A_y), so dA/dAbar_x = -dt c q sigma1 and
// dL/dAbar_x,n = 2 Re(i dt c q F_sigma1), F = ||lam|| ||psi|| sum_ab
// W_0a (W^T M V)_ab phi(nu_a, mu_b) V_0b.
//
// Memory: psi_n is stored every ckpt_every steps in the forward pass; the
// backward pass recomputes one segment of states at a time (the last segment
// is still resident from the forward pass).  Per-step records (contraction,
// both tridiagonal chains, shifts, k_eff) are written by the device and read
// once per segment, so the host never waits inside a segment.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

using namespace dlh;

namespace {

// workgroups of the contraction (its partials: 8 KiB each)
#ifndef DL_CONTRACT_BLOCKS
#define DL_CONTRACT_BLOCKS 1024
#endif
constexpr int kContractBlocks = DL_CONTRACT_BLOCKS;
// backward steps whose contraction partials are folded by one launch
constexpr int kFoldSteps = 64;
constexpr int kObserveBlocks = 1024;

// Largest store of kept forward segments (Krylov bases and states; see
// AdjLayout::keep).
#ifndef DL_ADJ_KEEP_GIB
#define DL_ADJ_KEEP_GIB 32
#endif
constexpr size_t kKeepBasesBytes = size_t(DL_ADJ_KEEP_GIB) << 30;

struct AdjLayout {
    size_t sc = 0, alpha = 0, gamma = 0, obs = 0, fields = 0, cpart = 0, rec = 0, basis = 0, lam = 0,
           seg = 0, ckpt = 0, kbasis = 0, kscal = 0, total = 0;
    int seglen = 0, nseg = 0;
    // keep: the forward sweep of a segment leaves every step's Krylov basis
    // (kbasis, kb_stride apart) and its scalars, alpha and gamma (kscal,
    // ks_stride apart) in place, so the backward pass does not build them
    // again; only when one segment's bases fit in kKeepBasesBytes.  nslot
    // segments (bases, scalars and states) are held at once, segment g in
    // slot g mod nslot, as many as fit in kKeepBasesBytes: the last nslot
    // segments of the forward pass are still there when the backward pass
    // reaches them and are not run again.
    bool keep = false;
    int nslot = 1;
    size_t kb_stride = 0, ks_stride = 0, ks_alpha = 0, ks_gamma = 0;
    size_t seg_slot = 0, kb_slot = 0, ks_slot = 0;  // bytes per slot
    int nfold = 1;  // contraction partial tables (one per backward step until the fold)
};

AdjLayout adj_plan(const dl_params &p, int n_steps, int ckpt_every)
{
    AdjLayout A;
    const size_t n = vec_elems(p);
    const size_t vb = align256(n * 16);
    const int m = p.krylov_dim;
    A.seglen = std::min(ckpt_every, n_steps);
    A.nseg = (n_steps + A.seglen - 1) / A.seglen;
    size_t off = 0;
    A.sc = off;
    off = align256(off + sizeof(dl::Scalars));
    A.alpha = off;
    off = align256(off + sizeof(double) * (dl::kContractM + 3));
    A.gamma = off;
    off = align256(off + sizeof(double) * (dl::kContractM + 3));
    A.obs = off;
    off = align256(off + sizeof(double) * 8);
    A.fields = off;
    off = align256(off + sizeof(double) * 4 * (size_t)n_steps);
    A.nfold = std::min(kFoldSteps, A.seglen);
    A.cpart = off;
    off = align256(off + sizeof(double) * 4 * dl::kBlock * (size_t)kContractBlocks * (size_t)A.nfold);
    A.rec = off;
    off = align256(off + sizeof(double) * dl::kRecLen * (size_t)A.seglen);
    A.basis = off;
    off += (size_t)(m - 1) * vec_stride(n, 16);
    A.lam = off;
    off += 2 * vb;
    A.kb_stride = (size_t)(m - 1) * vec_stride(n, 16);
    A.keep = A.kb_stride * (size_t)A.seglen <= kKeepBasesBytes;
    A.seg_slot = (size_t)(A.seglen + 1) * vb;
    if (A.keep) {
        A.ks_alpha = align256(sizeof(dl::Scalars));
        A.ks_gamma = A.ks_alpha + align256(sizeof(double) * (m + 3));
        A.ks_stride = A.ks_gamma + align256(sizeof(double) * (m + 3));
        A.kb_slot = A.kb_stride * (size_t)A.seglen;
        A.ks_slot = A.ks_stride * (size_t)A.seglen;
        const size_t per = A.kb_slot + A.ks_slot + A.seg_slot;
        A.nslot = (int)std::min<size_t>((size_t)A.nseg, std::max<size_t>(1, kKeepBasesBytes / per));
    }
    A.seg = off;
    off += (size_t)A.nslot * A.seg_slot;
    A.ckpt = off;
    off += (size_t)(A.nseg - 1) * vb;  // starts of segments 1 .. nseg-1 (segment 0 starts at psi0)
    if (A.keep) {
        off = align256(off);
        A.kbasis = off;
        off += (size_t)A.nslot * A.kb_slot;
        A.kscal = off;
        off += (size_t)A.nslot * A.ks_slot;
    }
    A.total = off;
    return A;
}

const char *adj_check(const dl_params &p, int n_steps, int ckpt_every)
{
    if (n_steps < 1 || n_steps > 10000000) return "n_steps must be in 1..1e7";
    if (ckpt_every < 1) return "ckpt_every must be >= 1";
    (void)p;
    return nullptr;
}

// exp(-i nu) and exp(-i mu) divided difference (the s-integral of one pair).
std::complex<double> divdiff_exp(double nu, double mu)
{
    const double h = 0.5 * (nu - mu);
    const double sinc = std::fabs(h) < 1e-4 ? 1.0 - h * h / 6.0 : std::sin(h) / h;
    const double ph = -0.5 * (nu + mu);
    return std::complex<double>(std::cos(ph) * sinc, std::sin(ph) * sinc);
}

// Derivatives of the loss with respect to Abar_x and Abar_y of one step.
void step_gradient(const double *rec, double dt, double cq, double *gx, double *gy)
{
    using cd = std::complex<double>;
    *gx = *gy = 0.0;
    const int kl = (int)rec[dl::kRecMeta + 2], kp = (int)rec[dl::kRecMeta + 3];
    if (kl <= 0 || kp <= 0) return;
    const double sl = rec[dl::kRecMeta + 0], sp = rec[dl::kRecMeta + 1];
    std::vector<double> dlv(kl), elv(kl > 1 ? kl - 1 : 0), dpv(kp), epv(kp > 1 ? kp - 1 : 0);
    for (int i = 0; i < kl; ++i) dlv[i] = rec[dl::kRecAlphaL + 1 + i] + sl;
    for (int i = 0; i + 1 < kl; ++i) elv[i] = rec[dl::kRecGammaL + 2 + i];
    for (int i = 0; i < kp; ++i) dpv[i] = rec[dl::kRecAlphaP + 1 + i] + sp;
    for (int i = 0; i + 1 < kp; ++i) epv[i] = rec[dl::kRecGammaP + 2 + i];
    std::vector<double> tau, W, mu, V;
    tridiag_full(dlv, elv, tau, W);
    tridiag_full(dpv, epv, mu, V);
    // basis contraction, normalised: u_j = gamma_j q_j
    std::vector<cd> m1((size_t)kl * kp), m2((size_t)kl * kp);
    for (int i = 0; i < kl; ++i)
        for (int j = 0; j < kp; ++j) {
            const double *s = rec + dl::kRecS + 4 * (i * dl::kContractM + j);
            const cd s01(s[0], s[1]), s10(s[2], s[3]);
            const double nrm = rec[dl::kRecGammaL + 1 + i] * rec[dl::kRecGammaP + 1 + j];
            m1[(size_t)i * kp + j] = (s01 + s10) / nrm;
            m2[(size_t)i * kp + j] = cd(0.0, 1.0) * (s10 - s01) / nrm;
        }
    // MV = M V  (kl x kp), then F = sum_ab W_0a (W^T MV)_ab phi_ab V_0b
    std::vector<cd> mv1((size_t)kl * kp), mv2((size_t)kl * kp);
    for (int i = 0; i < kl; ++i)
        for (int b = 0; b < kp; ++b) {
            cd a1 = 0.0, a2 = 0.0;
            for (int j = 0; j < kp; ++j) {
                a1 += m1[(size_t)i * kp + j] * V[(size_t)j * kp + b];
                a2 += m2[(size_t)i * kp + j] * V[(size_t)j * kp + b];
            }
            mv1[(size_t)i * kp + b] = a1;
            mv2[(size_t)i * kp + b] = a2;
        }
    cd f1 = 0.0, f2 = 0.0;
    for (int a = 0; a < kl; ++a)
        for (int b = 0; b < kp; ++b) {
            cd h1 = 0.0, h2 = 0.0;
            for (int i = 0; i < kl; ++i) {
                h1 += W[(size_t)i * kl + a] * mv1[(size_t)i * kp + b];
                h2 += W[(size_t)i * kl + a] * mv2[(size_t)i * kp + b];
            }
            const cd w = W[a] * V[b] * divdiff_exp(-tau[a], mu[b]);  // row 0 of W and V
            f1 += w * h1;
            f2 += w * h2;
        }
    const double scale = rec[dl::kRecGammaL + 1] * rec[dl::kRecGammaP + 1];
    f1 *= scale;
    f2 *= scale;
    // 2 Re(i dt c q F) = -2 dt c q Im F
    *gx = -2.0 * dt * cq * f1.imag();
    *gy = -2.0 * dt * cq * f2.imag();
}

}  // namespace

size_t dirac_lanczos_adjoint_workspace_bytes(const dl_params *params, int32_t n_steps, int32_t ckpt_every)
{
    if (validate(params)) return 0;
    if (adj_check(*params, n_steps, ckpt_every)) return 0;
    return adj_plan(*params, n_steps, ckpt_every).total;
}

dl_status dirac_lanczos_adjoint(dl_context *ctx, const void *psi0_v, double t0, double dt, int32_t n_steps,
                                int32_t ckpt_every, int32_t loss_kind, void *adj_ws, size_t adj_bytes,
                                double *loss, double *grad)
{
    if (!ctx) return DL_ERR_INVALID;
    if (!psi0_v || !loss || !grad) return ctx->fail(DL_ERR_INVALID, "psi0, loss and grad must be non-NULL");
    if (loss_kind < 1 || loss_kind > 15) return ctx->fail(DL_ERR_INVALID, "loss_kind must be in 1..15");
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
        return ctx->fail(DL_ERR_INVALID, "dt must be finite and positive, t0 finite");
    const dl_params &p = ctx->p;
    if (const char *msg = adj_check(p, n_steps, ckpt_every)) return ctx->fail(DL_ERR_INVALID, msg);
    if (p.precision != DL_PREC_FP64)
        return ctx->fail(DL_ERR_UNSUPPORTED, "the adjoint needs a DL_PREC_FP64 context");
    if (p.pulse_kind != DL_PULSE_FOURIER_SIN2 || ctx->coef.size() < 4)
        return ctx->fail(DL_ERR_UNSUPPORTED, "the adjoint differentiates DL_PULSE_FOURIER_SIN2 coefficients");
    const int m = p.krylov_dim;
    if (m > dl::kContractM)
        return ctx->fail(DL_ERR_UNSUPPORTED, "the adjoint supports krylov_dim <= 16");
    const AdjLayout A = adj_plan(p, n_steps, ckpt_every);
    if (ctx->ws_bytes < plan(ctx->p, DL_MODE_STEP, 0).total)
        return ctx->fail(DL_ERR_WORKSPACE, "context workspace too small for the stored Krylov basis (DL_MODE_STEP)");
    if (!adj_ws || ((uintptr_t)adj_ws & 255u) != 0)
        return ctx->fail(DL_ERR_WORKSPACE, "adjoint workspace must be a non-NULL, 256-byte aligned device pointer");
    if (adj_bytes < A.total)
        return ctx->fail(DL_ERR_WORKSPACE, "adjoint workspace too small: need " + std::to_string(A.total) + " bytes");

    hipStream_t st = ctx->stream;
    const size_t n = vec_elems(p);
    const size_t sites = n / 2;
    const size_t vb = align256(n * 16);
    const size_t vstride = vec_stride(n, 16);
    char *ws = ctx->ws;
    char *aw = static_cast<char *>(adj_ws);
    const Layout &L = ctx->L;
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    dl::StepStat *dstat = reinterpret_cast<dl::StepStat *>(ws + L.stats);
    const Engine ep{ctx->sc(), reinterpret_cast<double *>(ws + L.alpha), reinterpret_cast<double *>(ws + L.gamma),
                    ws + L.vecs + align256(n * 16), vstride, m, false};
    const Engine el{reinterpret_cast<dl::Scalars *>(aw + A.sc), reinterpret_cast<double *>(aw + A.alpha),
                    reinterpret_cast<double *>(aw + A.gamma), aw + A.basis, vstride, m, false};
    double *obs = reinterpret_cast<double *>(aw + A.obs);
    double *fields = reinterpret_cast<double *>(aw + A.fields);
    double *cpart = reinterpret_cast<double *>(aw + A.cpart);
    double *rec = reinterpret_cast<double *>(aw + A.rec);
    const double2 *psi0 = static_cast<const double2 *>(psi0_v);
    auto lam = [&](int i) { return reinterpret_cast<double2 *>(aw + A.lam + (size_t)i * vb); };
    // state i of segment g (its slot)
    auto seg = [&](int g, int i) {
        return reinterpret_cast<double2 *>(aw + A.seg + (size_t)(g % A.nslot) * A.seg_slot + (size_t)i * vb);
    };
    auto ckpt = [&](int g) -> const double2 * {
        return g == 0 ? psi0 : reinterpret_cast<const double2 *>(aw + A.ckpt + (size_t)(g - 1) * vb);
    };

    // fields of every step: forward (A = dt H) then backward (A = -dt H)
    const double cq = p.c * p.charge;
    const double kf = -dt * cq;
    std::vector<double> hf(4 * (size_t)n_steps);
    for (int i = 0; i < n_steps; ++i) {
        double a[2];
        pulse_average(p, ctx->coef, t0 + (double)i * dt, dt, a);
        hf[4 * (size_t)i + 0] = kf * a[0];
        hf[4 * (size_t)i + 1] = kf * chir(p) * a[1];
        hf[4 * (size_t)i + 2] = -kf * a[0];
        hf[4 * (size_t)i + 3] = -kf * chir(p) * a[1];
    }
    DL_HIP(ctx, hipMemcpyAsync(fields, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice, st));
    const dl::Op opf = ctx->op(dt), opb = ctx->op(-dt), op1 = ctx->op(1.0);
    const dl_status pend = take_async_failure(ctx);
    if (pend != DL_OK) return pend;
    dl::launch_reset(ep.sc, st);
    dl::launch_reset(el.sc, st);
    DL_HIP(ctx, hipGetLastError());

    const int C = A.seglen, G = A.nseg;
    auto seg_len = [&](int g) { return std::min(C, n_steps - g * C); };
    // forward states of segment g into seg(g, 0..len)
    // step i of a segment: its own basis when the bases are kept, else the context's
    auto step_engine = [&](int g, int i) {
        Engine e = ep;
        if (A.keep) e.basis = aw + A.kbasis + (size_t)(g % A.nslot) * A.kb_slot + (size_t)i * A.kb_stride;
        return e;
    };
    auto kept_scal = [&](int g, int i) {
        return aw + A.kscal + (size_t)(g % A.nslot) * A.ks_slot + (size_t)i * A.ks_stride;
    };
    auto run_segment = [&](int g) -> dl_status {
        const int len = seg_len(g);
        DL_HIP(ctx, hipMemcpyAsync(seg(g, 0), ckpt(g), n * 16, hipMemcpyDeviceToDevice, st));
        for (int i = 0; i < len; ++i) {
            const double *fp = fields + 4 * (size_t)(g * C + i);
            const Engine ei = step_engine(g, i);
            const dl_status sb = run_build(ctx, ei, opf, seg(g, i), fp, partials, 1);
            if (sb != DL_OK) return sb;
            // what the backward contraction reads of this step (k_eff, shift,
            // status, alpha and gamma, whole once the small exponential has
            // folded the last iteration) is copied by the recombination
            KeepDst keep;
            if (A.keep) keep = KeepDst{kept_scal(g, i), A.ks_alpha, A.ks_gamma, m + 3};
            const dl_status sf = run_finish(ctx, ei, seg(g, i), seg(g, i + 1), dstat, partials, false, keep);
            if (sf != DL_OK) return sf;
        }
        DL_HIP(ctx, hipGetLastError());
        return DL_OK;
    };
    auto check_status = [&](const dl::Scalars *sc, const char *what) -> dl_status {
        int status = 0;
        DL_HIP(ctx, hipMemcpyAsync(&status, &sc->status, sizeof(int), hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        if (status != 0) return ctx->fail(DL_ERR_NONFINITE, std::string("non-finite Lanczos reduction in the ") + what);
        return DL_OK;
    };

    // forward pass with checkpoints
    for (int g = 0; g < G; ++g) {
        const dl_status s = run_segment(g);
        if (s != DL_OK) return s;
        if (g + 1 < G)
            DL_HIP(ctx, hipMemcpyAsync(const_cast<double2 *>(ckpt(g + 1)), seg(g, seg_len(g)), n * 16,
                                       hipMemcpyDeviceToDevice, st));
    }
    {
        const dl_status s = check_status(ep.sc, "forward pass");
        if (s != DL_OK) return s;
    }
    // loss and adjoint seed from psi_N (the end of the last segment, still in seg)
    const double2 *psin = seg(G - 1, seg_len(G - 1));
    const int nbo = (int)std::max<size_t>(1, std::min<size_t>(kObserveBlocks, (sites + dl::kBlock - 1) / dl::kBlock));
    dl::launch_observe(op1, psin, loss_kind, el.sc, partials, obs, nbo, st);
    dl::launch_adjoint_seed(op1, psin, loss_kind, obs, lam(0), st);
    DL_HIP(ctx, hipGetLastError());
    double hobs[8];
    DL_HIP(ctx, hipMemcpyAsync(hobs, obs, sizeof(hobs), hipMemcpyDeviceToHost, st));
    DL_HIP(ctx, hipStreamSynchronize(st));
    if (!std::isfinite(hobs[5]) || !(hobs[0] > 0.0))
        return ctx->fail(DL_ERR_NONFINITE, "final state has zero or non-finite norm");

    // backward pass
    const size_t ncoef = ctx->coef.size();
    std::vector<double> gsum(ncoef, 0.0);
    std::vector<double> gstep(2 * (size_t)n_steps, 0.0);  // dL/dAbar_x, dL/dAbar_y per step
    std::vector<double> hrec((size_t)dl::kRecLen * C);
    const int ncb = (int)std::max<size_t>(
        1, std::min<size_t>(kContractBlocks, (sites + 31) / 32));  // one 32-site tile per block and round
    int cur = 0, pending = 0;
    for (int g = G - 1; g >= 0; --g) {
        const int len = seg_len(g);
        if (g < G - A.nslot) {  // the last nslot segments are still in their slots
            const dl_status s = run_segment(g);
            if (s != DL_OK) return s;
        }
        for (int i = len - 1; i >= 0; --i) {
            const size_t ns = (size_t)g * C + i;
            dl_status s = DL_OK;
            const Engine ei = step_engine(g, i);
            if (!A.keep) {
                s = run_build(ctx, ei, opf, seg(g, i), fields + 4 * ns, partials, 1, true);
                if (s != DL_OK) return s;
            }
            // the backward step first: its small exponential completes T of the
            // lambda basis, and the recombination leaves the basis and lam(cur)
            // for the contraction below
            s = run_build(ctx, el, opb, lam(cur), fields + 4 * ns + 2, partials, 1);
            if (s != DL_OK) return s;
            s = run_finish(ctx, el, lam(cur), lam(1 - cur), dstat, partials);
            if (s != DL_OK) return s;
            dl::ContractArgs ca{};
            ca.lam1 = lam(cur);
            ca.lam_basis = el.basis;
            ca.psi1 = seg(g, i);
            ca.psi_basis = ei.basis;
            ca.vec_bytes = vstride;
            ca.sites = sites;
            ca.sc_lam = el.sc;
            ca.alpha_lam = el.alpha;
            ca.gamma_lam = el.gamma;
            if (A.keep) {
                char *ks = kept_scal(g, i);
                ca.sc_psi = reinterpret_cast<const dl::Scalars *>(ks);
                ca.alpha_psi = reinterpret_cast<const double *>(ks + A.ks_alpha);
                ca.gamma_psi = reinterpret_cast<const double *>(ks + A.ks_gamma);
            } else {
                ca.sc_psi = ep.sc;
                ca.alpha_psi = ep.alpha;
                ca.gamma_psi = ep.gamma;
            }
            ca.partials = cpart + (size_t)(i % A.nfold) * 4 * dl::kBlock * (size_t)ncb;
            ca.rec = rec + (size_t)i * dl::kRecLen;
            dl::launch_contract(ca, ncb, st);
            // the sums of the pending steps i .. i + pending - 1 (distinct
            // partial tables) are folded together
            if (++pending == A.nfold || i == 0) {
                dl::launch_contract_fold(cpart, A.nfold, ncb, rec, i, pending, st);
                pending = 0;
            }
            cur = 1 - cur;
        }
        DL_HIP(ctx, hipGetLastError());
        DL_HIP(ctx, hipMemcpyAsync(hrec.data(), rec, sizeof(double) * dl::kRecLen * len, hipMemcpyDeviceToHost, st));
        DL_HIP(ctx, hipStreamSynchronize(st));
        for (int i = 0; i < len; ++i) {
            const double *r = hrec.data() + (size_t)i * dl::kRecLen;
            if (r[dl::kRecMeta + 4] != 0.0 || r[dl::kRecMeta + 5] != 0.0)
                return ctx->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in the backward pass");
            double gx, gy;
            step_gradient(r, dt, cq, &gx, &gy);
            gy *= chir(p);  // dA/dAbar_y = -dt c q chir sigma2
            if (!std::isfinite(gx) || !std::isfinite(gy))
                return ctx->fail(DL_ERR_NONFINITE, "non-finite gradient contribution");
            gstep[2 * ((size_t)g * C + i)] = gx;
            gstep[2 * ((size_t)g * C + i) + 1] = gy;
        }
    }
    // chain rule through the step averages, summed in step order (the result
    // does not depend on the checkpoint interval)
    for (int s = 0; s < n_steps; ++s) {
        const double tn = t0 + (double)s * dt;
        const double gx = gstep[2 * (size_t)s], gy = gstep[2 * (size_t)s + 1];
        for (size_t k = 1; 4 * k <= ncoef; ++k) {
            const double ws_ = basis_average(p, (int)k, false, tn, dt);
            const double wc_ = basis_average(p, (int)k, true, tn, dt);
            gsum[4 * (k - 1) + 0] += ws_ * gx;
            gsum[4 * (k - 1) + 1] += wc_ * gx;
            gsum[4 * (k - 1) + 2] += ws_ * gy;
            gsum[4 * (k - 1) + 3] += wc_ * gy;
        }
    }
    *loss = hobs[5];
    std::copy(gsum.begin(), gsum.end(), grad);
    return DL_OK;
}
