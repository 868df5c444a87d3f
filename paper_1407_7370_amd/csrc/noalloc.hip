// dirac_lanczos_step_noalloc: the time step of dirac_lanczos_step for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid allocation).  The whole workspace of the step -- the
// scalars, the reduction partials, the per-step fields and statistics, the
// ping-pong state and the Krylov basis -- lives in `scratch`, a file-scope
// device array of kScratchBytes that every GPU the library runs on holds until
// the process ends.  The call allocates nothing, on the device or the host:
// the per-step fields reach the device as kernel arguments, and the host
// staging of the statistics uses buffers on the stack.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "context.h"

using namespace dlh;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

// Per-device address of `scratch` (the array's name is a host-side stand-in,
// not a device address) and compute-unit count, set on the first call on the
// device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch[kMaxDevices];
int g_cus[kMaxDevices];

// Steps staged per round trip: fields through one kernel argument block.
constexpr int kRound = 64;
struct FieldBlock {
    double f[2 * kRound];
};

__global__ void k_put_fields(double *dst, FieldBlock fb, int n)
{
    const int i = threadIdx.x;
    if (i < 2 * n) dst[i] = fb.f[i];
}

}  // namespace

extern "C" dl_status dirac_lanczos_step_noalloc(const dl_params *params, void *psi_v, double t0, double dt,
                                                int32_t n_steps, void *hip_stream, dl_step_stat *stats)
{
    if (validate(params)) return DL_ERR_INVALID;
    if (!psi_v || n_steps < 0 || !(dt != 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return DL_ERR_INVALID;
    if (params->pulse_kind == DL_PULSE_FOURIER_SIN2 && !params->coef) return DL_ERR_INVALID;
    const Layout L = plan(*params, DL_MODE_STEP, 0);
    if (L.total > kScratchBytes) return DL_ERR_WORKSPACE;  // beyond the static scratch
    if (n_steps == 0) return DL_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DL_ERR_DEVICE;
    void *ws;
    int cus;
    {
        std::lock_guard<std::mutex> guard(g_lock);
        if (!g_scratch[dev]) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DL_ERR_DEVICE;
            if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DL_ERR_DEVICE;
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DL_ERR_DEVICE;
            g_cus[dev] = prop.multiProcessorCount;
            g_scratch[dev] = ptr;
        }
        ws = g_scratch[dev];
        cus = g_cus[dev];
    }
    const dl_params &p = *params;
    const int m = p.krylov_dim;
    const bool mixed = p.precision == DL_PREC_MIXED;
    const size_t n = vec_elems(p);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // a context on the stack over the scratch (its containers stay empty)
    dl_context ctx;
    ctx.p = p;
    ctx.stream = st;
    ctx.ws = static_cast<char *>(ws);
    ctx.ws_bytes = kScratchBytes;
    ctx.L = L;
    ctx.cus = cus;
    configure_launch(&ctx);
    char *w = ctx.ws;
    dl::Scalars *sc = ctx.sc();
    double *partials = reinterpret_cast<double *>(w + L.partials);
    double *fields = reinterpret_cast<double *>(w + L.fields);
    dl::StepStat *dstats = reinterpret_cast<dl::StepStat *>(w + L.stats);
    double2 *psi = static_cast<double2 *>(psi_v);
    double2 *state = reinterpret_cast<double2 *>(w + L.vecs);
    const size_t belem = mixed ? 8 : 16;
    const Engine eng{sc, reinterpret_cast<double *>(w + L.alpha), reinterpret_cast<double *>(w + L.gamma),
                     w + L.vecs + align256(n * 16), vec_stride(n, belem), m, mixed};
    const dl::Op op = ctx.op(dt);
    const CoefView coef(p.coef, p.pulse_kind == DL_PULSE_FOURIER_SIN2 ? (size_t)p.n_coef : 0);
    const double kf = -dt * p.c * p.charge;

    // every call starts from zeroed scalars and reduction ticket
    dl::launch_reset(sc, st);
    if (hipGetLastError() != hipSuccess) return DL_ERR_DEVICE;
    double cum = 0.0;
    int completed = 0;
    bool aborted = false;
    for (int s0 = 0; s0 < n_steps && !aborted; s0 += kRound) {
        const int nc = std::min(kRound, n_steps - s0);
        FieldBlock fb;
        for (int i = 0; i < nc; ++i) {
            double a[2];
            pulse_average(p, coef, t0 + (double)(s0 + i) * dt, dt, a);
            fb.f[2 * i] = kf * a[0];
            fb.f[2 * i + 1] = kf * chir(p) * a[1];
        }
        hipLaunchKernelGGL(k_put_fields, dim3(1), dim3(2 * kRound), 0, st, fields, fb, nc);
        for (int i = 0; i < nc; ++i) {
            const int g = s0 + i;
            double2 *in = (g % 2 == 0) ? psi : state;
            double2 *out = (g % 2 == 0) ? state : psi;
            if (run_build(&ctx, eng, op, in, fields + 2 * i, partials, 1) != DL_OK) return DL_ERR_DEVICE;
            if (run_finish(&ctx, eng, in, out, dstats + i, partials) != DL_OK) return DL_ERR_DEVICE;
        }
        if (hipGetLastError() != hipSuccess) return DL_ERR_DEVICE;
        if (!stats) continue;
        dl::StepStat hs[kRound];
        dl::Scalars hsc;
        if (hipMemcpyAsync(hs, dstats, sizeof(dl::StepStat) * nc, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&hsc, sc, sizeof(hsc), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return DL_ERR_DEVICE;
        const int done_here = hsc.steps_done - completed;
        for (int i = 0; i < nc; ++i) {
            dl_step_stat &o = stats[s0 + i];
            if (i < done_here) {
                cum += hs[i].err_est;
                o.k_eff = hs[i].keff;
                o.err_est = hs[i].err_est;
                o.cum_bound = cum;
                o.norm2 = hs[i].norm2;
                o.round_bound = hs[i].round_bound;
            } else {
                o.k_eff = -1;
                o.err_est = o.cum_bound = o.norm2 = o.round_bound = 0.0;
            }
        }
        completed = hsc.steps_done;
        aborted = hsc.status != 0;
    }
    if (stats && aborted)
        for (int i = completed; i < n_steps; ++i) {
            stats[i].k_eff = -1;
            stats[i].err_est = stats[i].cum_bound = stats[i].norm2 = stats[i].round_bound = 0.0;
        }
    // the state after the completed steps is moved to psi on the device
    dl::launch_finish_copy(sc, state, psi, n, cus, st);
    if (hipGetLastError() != hipSuccess) return DL_ERR_DEVICE;
    if (stats && hipStreamSynchronize(st) != hipSuccess) return DL_ERR_DEVICE;
    return aborted ? DL_ERR_NONFINITE : DL_OK;
}
