// Host-side context of the C ABI, shared by host.cpp (init/step/eigen) and
// adjoint.cpp.  Internal; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "dirac_lanczos.h"
#include "dl_internal.h"
#include "ritz.h"

namespace dlh {

struct Layout {
    size_t sc = 0, alpha = 0, gamma = 0, partials = 0, fields = 0, stats = 0, vecs = 0, total = 0;
    int ab_len = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline size_t vec_elems(const dl_params &p) { return (size_t)2 * (size_t)p.nx * (size_t)p.ny; }
// Byte stride between workspace vectors: padded so that vectors streamed
// together are not a power of two apart.
inline size_t vec_stride(size_t n, size_t elem) { return align256(n * elem) + dl::kVecPad; }

Layout plan(const dl_params &p, int mode, int k_eigen);

// Vector region of the eigen mode with full reorthogonalisation (offsets from
// Layout::vecs): z, the k stored complex128 basis vectors, the two projection
// coefficient arrays (k complex each), the projection partial table and the
// staged eigenvector columns of the Ritz vectors.
struct ReorthLayout {
    size_t z = 0, q = 0, h1 = 0, h2 = 0, pproj = 0, tsel = 0, total = 0;
};
inline ReorthLayout reorth_layout(size_t n, int k)
{
    ReorthLayout R;
    const size_t vs = vec_stride(n, 16);
    size_t off = 0;
    R.z = off;
    off += vs;
    R.q = off;
    off += (size_t)k * vs;
    R.h1 = off;
    off += align256(sizeof(double) * 2 * (size_t)k);
    R.h2 = off;
    off += align256(sizeof(double) * 2 * (size_t)k);
    R.pproj = off;
    off += align256(sizeof(double) * 2 * (size_t)dl::proj_tiles(n) * (size_t)k);
    R.tsel = off;
    off += align256(sizeof(double) * (size_t)dl::kRitzVecs * (size_t)k);
    R.total = off;
    return R;
}
const char *validate(const dl_params *p);
// Fourier coefficients of the laser field (a context's copy, or a caller's
// array for the duration of one call).
struct CoefView {
    const double *c = nullptr;
    size_t n = 0;
    CoefView() = default;
    CoefView(const std::vector<double> &v) : c(v.data()), n(v.size()) {}
    CoefView(const double *p, size_t k) : c(p), n(p ? k : 0) {}
    size_t size() const { return n; }
    double operator[](size_t i) const { return c[i]; }
};
void pulse_now(const dl_params &p, CoefView coef, double t, double *a);
void pulse_average(const dl_params &p, CoefView coef, double t0, double dt, double *a);
// Step average of one Fourier basis function of the sin^2-enveloped pulse:
// harmonic k, sine (cosine = false) or cosine (cosine = true).
double basis_average(const dl_params &p, int k, bool cosine, double t0, double dt);

// Rounding of one stored Krylov vector of nx*ny sites (mixed precision:
// complex64 storage, see dl::kStoreEps32), or zero in FP64.
inline void store_rounding(const dl_params &p, double &reps, double &rabs)
{
    reps = rabs = 0.0;
    if (p.precision != DL_PREC_MIXED) return;
    reps = dl::kStoreEps32;
    rabs = dl::kStoreTiny32 * std::sqrt(4.0 * (double)p.nx * (double)p.ny);
}

// Sign of the sigma2 terms: alpha2 = chir * sigma2.
inline double chir(const dl_params &p) { return p.chirality < 0 ? -1.0 : 1.0; }

// A = s H with the geometry and static fields of the problem (the homogeneous
// laser term is passed to the kernels per step, its y component times chir).
inline dl::Op make_op(const dl_params &p, double s)
{
    dl::Op o{};
    o.nx = p.nx;
    o.ny = p.ny;
    o.bcx = p.bc_x;
    o.bcy = p.bc_y;
    o.hx = (p.x_max - p.x_min) / p.nx;
    o.hy = (p.y_max - p.y_min) / p.ny;
    o.xmin = p.x_min;
    o.ymin = p.y_min;
    o.kx = s * p.c / (2.0 * o.hx);
    o.ky = chir(p) * s * p.c / (2.0 * o.hy);
    o.mc2 = s * p.mass * p.c * p.c;
    o.bq = s * p.c * p.charge * p.bz * 0.5;
    o.bqy = chir(p) * o.bq;
    o.pot_kind = p.pot_kind ? 1 : 0;
    if (p.pot_kind == 1) {
        o.vz = s * p.pot_z;
        o.va2 = p.pot_a * p.pot_a;
    } else if (p.pot_kind == 2) {
        o.vz = s * 1.5 * p.pot_z;
        o.va2 = 3.0 / (p.pot_z * p.pot_z);
    }
    o.has_table = p.v_table ? 1 : 0;
    o.vtab = p.v_table;
    o.vscale = s;
    return o;
}

}  // namespace dlh

struct dl_context {
    dl_params p{};
    std::vector<double> coef;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    dlh::Layout L;
    int cus = 256;
    dl::Tiles tiles_first{}, tiles_recur{}, tiles_p2{}, tiles_p3{}, tiles_apply{};
    // tiles of recurrence sweep p (each sweep kind has its own occupancy)
    const dl::Tiles &tiles_pass(int p) const { return p == 2 ? tiles_p2 : (p == 3 ? tiles_p3 : tiles_recur); }
    int combine_blocks = 1024;       // recombination (narrow form) and second-run accumulation
    bool combine_wide = false;       // recombination in the wide form (more sites per thread)
    int combine_blocks_wide = 1024;  // its workgroups
    int sweep_waves = 8;  // waves per compute unit of the sweeps (launch shape)
    std::vector<double> host_fields;
    std::vector<dl::StepStat> host_stats;
    std::string err;
    // event timing (dirac_lanczos_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<int> ev_cls, ev_cnt;  // class and number of launches of each event pair
    size_t ev_used = 0;
    int64_t t_launches[5] = {0, 0, 0, 0, 0};
    double t_ms[5] = {0, 0, 0, 0, 0};
    // asynchronous steps (stats == NULL): two pinned host buffers stage the
    // per-step fields of a chunk; an event after each upload guards the
    // buffer's reuse.  The statistics of the last chunk stay on the device
    // until dirac_lanczos_wait.
    double *pin_fields[2] = {nullptr, nullptr};
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    int pin_next = 0;
    bool async_pending = false;
    int async_s0 = 0, async_nc = 0;

    ~dl_context()
    {
        for (hipEvent_t e : ev0) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev1) (void)hipEventDestroy(e);
        for (int i = 0; i < 2; ++i) {
            if (pin_ev[i]) (void)hipEventSynchronize(pin_ev[i]);
            if (pin_ev[i]) (void)hipEventDestroy(pin_ev[i]);
            if (pin_fields[i]) (void)hipHostFree(pin_fields[i]);
        }
    }

    // Fold the recorded event pairs into the per-class totals.
    hipError_t harvest()
    {
        if (ev_used == 0) return hipSuccess;
        hipError_t e = hipEventSynchronize(ev1[ev_used - 1]);
        if (e != hipSuccess) return e;
        for (size_t i = 0; i < ev_used; ++i) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev0[i], ev1[i]);
            if (e != hipSuccess) return e;
            t_ms[ev_cls[i]] += ms;
            t_launches[ev_cls[i]] += ev_cnt[i];
        }
        ev_used = 0;
        return hipSuccess;
    }

    // Launch `fn` (`count` launches of class cls, back to back) bracketed by
    // an event pair when timing is on.
    template <class F>
    hipError_t timed(int cls, F &&fn, int count = 1)
    {
        if (!timing) {
            fn();
            return hipSuccess;
        }
        if (ev_used == ev0.size()) {
            hipError_t e = harvest();
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipEventRecord(ev0[ev_used], stream);
        if (e != hipSuccess) return e;
        fn();
        e = hipEventRecord(ev1[ev_used], stream);
        if (e != hipSuccess) return e;
        ev_cls[ev_used] = cls;
        ev_cnt[ev_used++] = count;
        return hipSuccess;
    }

    dl_status fail(dl_status s, const std::string &msg)
    {
        err = msg;
        return s;
    }
    dl_status hip_fail(hipError_t e, const char *what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return DL_ERR_DEVICE;
    }
    dl::Scalars *sc() const { return reinterpret_cast<dl::Scalars *>(ws + L.sc); }

    // A = s H with the geometry and static fields of the problem.
    dl::Op op(double s) const { return dlh::make_op(p, s); }
};

#define DL_HIP(ctx, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #call); \
    } while (0)


namespace dlh {

// One Lanczos engine: scalars, alpha/gamma chains and Krylov vectors u_2..u_m.
struct Engine {
    dl::Scalars *sc;
    double *alpha;
    double *gamma;
    char *basis;
    size_t vstride;
    int m;
    bool mixed;
    void *bvec(int j) const { return basis + (size_t)(j - 2) * vstride; }
};

// Iterations 1..m on `in` (sweeps; shift: run on A - alpha_1 I after iteration 1).
// The last iteration's scalar update is left to run_finish unless `complete`
// (then T is whole on return, and run_finish must be told it is).
dl_status run_build(dl_context *ctx, const Engine &e, const dl::Op &op, const double2 *in,
                    const double *field, double *partials, int shift, bool complete = false);
// One whole step by the second Lanczos run (three rolling Krylov vectors).
dl_status run_twice(dl_context *ctx, const Engine &e, const dl::Op &op, const double2 *in, double2 *out,
                    const double *field, dl::StepStat *stat, double *partials);
// Where the recombination also copies the step's scalars, alpha and gamma
// (dst == NULL: nowhere); see dl::CombArgs::keep.
struct KeepDst {
    char *dst = nullptr;
    size_t off_alpha = 0, off_gamma = 0;
    int nab = 0;
};
// exp(-iT) and the recombination into `out` (stat receives k_eff, estimate, norm).
dl_status run_finish(dl_context *ctx, const Engine &e, const double2 *in, double2 *out,
                     dl::StepStat *stat, double *partials, bool folded = false, const KeepDst &keep = KeepDst{});

// Default launch shapes of a context's sweeps and recombination (ctx->p and
// ctx->cus set).
void configure_launch(dl_context *ctx);

// Report (DL_ERR_NONFINITE) and clear a failure of an earlier asynchronous
// step call that dirac_lanczos_wait has not reported; DL_OK otherwise.  Every
// synchronous entry point that resets the scalars calls it first.
dl_status take_async_failure(dl_context *ctx);

// Eigen mode with full reorthogonalisation (eigen.cpp); vecs (device, may be
// NULL) receives the Ritz vectors of the reported values.
dl_status eigen_reorth(dl_context *ctx, const void *psi0, int k_max, double e_lo, double e_hi, double tol,
                       int n_wanted, double *evals, double *bounds, int32_t *n_found, void *vecs);

}  // namespace dlh
