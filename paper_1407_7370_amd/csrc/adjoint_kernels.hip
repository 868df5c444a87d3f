// gfx950 kernels of the adjoint (gradient) mode: observables of the final
// state, the adjoint seed, and the contraction of the two Krylov bases of a
// backward step.  One thread per site with direct neighbour reads: these run
// once per call (observables, seed) or once per step beside 2m sweeps
// (contraction), so they are not on the bandwidth-critical path.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_reduce.h"
#include "dl_internal.h"

namespace dl {
namespace {

// Both components of one site (16-byte aligned pairs).
struct Site {
    double2 a, b;
};

__device__ __forceinline__ double2 site_val(const double2 *psi, const Op &op, int comp, int i, int j)
{
    if (i < 0 || i >= op.nx) {
        if (!op.bcx) return make_double2(0.0, 0.0);
        i = i < 0 ? i + op.nx : i - op.nx;
    }
    if (j < 0 || j >= op.ny) {
        if (!op.bcy) return make_double2(0.0, 0.0);
        j = j < 0 ? j + op.ny : j - op.ny;
    }
    return psi[((size_t)comp * op.ny + j) * op.nx + i];
}

__global__ __launch_bounds__(kBlock) void k_observe(Op op, const double2 *__restrict__ psi, int loss_kind,
                                                    Scalars *sc, double *partials, double *obs)
{
    const size_t sites = (size_t)op.nx * op.ny;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (size_t s = (size_t)blockIdx.x * kBlock + threadIdx.x; s < sites; s += (size_t)gridDim.x * kBlock) {
        const int i = (int)(s % op.nx), j = (int)(s / op.nx);
        const double x = op.xmin + i * op.hx, y = op.ymin + j * op.hy;
        for (int c = 0; c < 2; ++c) {
            const double2 v = psi[(size_t)c * sites + s];
            const double w = v.x * v.x + v.y * v.y;
            const double2 xr = site_val(psi, op, c, i + 1, j), xl = site_val(psi, op, c, i - 1, j);
            const double2 yu = site_val(psi, op, c, i, j + 1), yd = site_val(psi, op, c, i, j - 1);
            const double dxr = (xr.x - xl.x) / (2.0 * op.hx), dxi = (xr.y - xl.y) / (2.0 * op.hx);
            const double dyr = (yu.x - yd.x) / (2.0 * op.hy), dyi = (yu.y - yd.y) / (2.0 * op.hy);
            acc[0] += w;
            acc[1] += x * w;
            acc[2] += y * w;
            acc[3] += v.x * dxi - v.y * dxr;  // Re conj(v) (-i d)
            acc[4] += v.x * dyi - v.y * dyr;
        }
    }
    double tot[5];
    if (!grid_reduce(acc, partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        const double n = tot[0];
        double l = 0.0;
        obs[0] = n;
        for (int b = 0; b < 4; ++b) {
            const double e = n > 0.0 ? tot[1 + b] / n : 0.0;
            obs[1 + b] = e;
            if (loss_kind & (1 << b)) l += e;
        }
        obs[5] = l;
    }
}

__global__ __launch_bounds__(kBlock) void k_adjoint_seed(Op op, const double2 *__restrict__ psi, int loss_kind,
                                                         const double *__restrict__ obs, double2 *__restrict__ lam)
{
    const size_t sites = (size_t)op.nx * op.ny;
    const double n = obs[0], l = obs[5];
    const double inv = n > 0.0 ? 1.0 / n : 0.0;
    const double wx = (loss_kind & 1) ? 1.0 : 0.0, wy = (loss_kind & 2) ? 1.0 : 0.0;
    const double wpx = (loss_kind & 4) ? 1.0 : 0.0, wpy = (loss_kind & 8) ? 1.0 : 0.0;
    for (size_t s = (size_t)blockIdx.x * kBlock + threadIdx.x; s < sites; s += (size_t)gridDim.x * kBlock) {
        const int i = (int)(s % op.nx), j = (int)(s / op.nx);
        const double x = op.xmin + i * op.hx, y = op.ymin + j * op.hy;
        const double diag = wx * x + wy * y - l;
        for (int c = 0; c < 2; ++c) {
            const double2 v = psi[(size_t)c * sites + s];
            const double2 xr = site_val(psi, op, c, i + 1, j), xl = site_val(psi, op, c, i - 1, j);
            const double2 yu = site_val(psi, op, c, i, j + 1), yd = site_val(psi, op, c, i, j - 1);
            const double dxr = (xr.x - xl.x) / (2.0 * op.hx), dxi = (xr.y - xl.y) / (2.0 * op.hx);
            const double dyr = (yu.x - yd.x) / (2.0 * op.hy), dyi = (yu.y - yd.y) / (2.0 * op.hy);
            // (-i d) = (d.im, -d.re)
            const double re = diag * v.x + wpx * dxi + wpy * dyi;
            const double im = diag * v.y - wpx * dxr - wpy * dyr;
            lam[(size_t)c * sites + s] = make_double2(re * inv, im * inv);
        }
    }
}

// ---------------------------------------------------------------------------
// Contraction of the two Krylov bases of one adjoint step (see ContractArgs):
// S01 = L0^H P1 and S10 = L1^H P0 (16 x 16 complex; L, P the lambda and psi
// bases, 0/1 the spinor components) are dense products over the sites, so
// they run on the FP64 matrix cores: v_mfma_f64_16x16x4f64 multiplies a
// 16 x 4 block A by a 4 x 16 block B, with lane l holding A[l % 16][l / 16],
// B[l / 16][l % 16] and D[4 r + l / 16][l % 16] in its register r (the
// layout checked on the device before use).  Per step of four sites lane l
// loads site s0 + l / 16 of basis vector l % 16 of both bases, and the eight
// real products of the two complex contractions accumulate in four 16 x 16
// blocks.  Waves stride over the four-site groups; a workgroup sums its four
// waves in order and writes its partials for k_contract_fold.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Site basis_site(const double2 *u1, const char *basis, size_t vec_bytes,
                                                   size_t sites, int v, size_t site)
{
    if (v == 0) return Site{u1[site], u1[sites + site]};
    return *reinterpret_cast<const Site *>(basis + (size_t)(v - 1) * vec_bytes + site * 32);
}

__device__ __forceinline__ v4d mfma(double x, double y, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

__global__ __launch_bounds__(kBlock) void k_contract(ContractArgs a)
{
    static_assert(kContractM == 16, "one 16 x 16 block per contraction");
    __shared__ double red[kWaves][4][64][4];
    const int kl = a.sc_lam->keff, kp = a.sc_psi->keff;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int v = lane & 15, ks = lane >> 4;
    v4d s01r = {0.0, 0.0, 0.0, 0.0}, s01i = s01r, s10r = s01r, s10i = s01r;
    const size_t groups = (a.sites + 3) / 4;
    for (size_t g = (size_t)blockIdx.x * kWaves + w; g < groups; g += (size_t)gridDim.x * kWaves) {
        const size_t site = g * 4 + ks;
        Site x = Site{make_double2(0.0, 0.0), make_double2(0.0, 0.0)}, y = x;
        if (site < a.sites) {
            if (v < kl) x = basis_site(a.lam1, a.lam_basis, a.vec_bytes, a.sites, v, site);
            if (v < kp) y = basis_site(a.psi1, a.psi_basis, a.vec_bytes, a.sites, v, site);
        }
        // conj(l0) p1 and conj(l1) p0, real and imaginary parts
        s01r = mfma(x.a.x, y.b.x, s01r);
        s01r = mfma(x.a.y, y.b.y, s01r);
        s01i = mfma(x.a.x, y.b.y, s01i);
        s01i = mfma(-x.a.y, y.b.x, s01i);
        s10r = mfma(x.b.x, y.a.x, s10r);
        s10r = mfma(x.b.y, y.a.y, s10r);
        s10i = mfma(x.b.x, y.a.y, s10i);
        s10i = mfma(-x.b.y, y.a.x, s10i);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        red[w][0][lane][r] = s01r[r];
        red[w][1][lane][r] = s01i[r];
        red[w][2][lane][r] = s10r[r];
        red[w][3][lane][r] = s10i[r];
    }
    __syncthreads();
    // thread t = 16 a + b owns pair (a, b), held by lane b + 16 (a % 4), register a / 4;
    // output o = 4 t + c at partials[o * nblocks + block]: the fold reads each
    // output's partials contiguously
    const int t = threadIdx.x, pa = t >> 4, pb = t & 15;
    const int src = pb + 16 * (pa & 3), reg = pa >> 2;
    const size_t nb = gridDim.x, b = blockIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double acc = red[0][c][src][reg];
        for (int i = 1; i < kWaves; ++i) acc += red[i][c][src][reg];
        a.partials[(size_t)(4 * t + c) * nb + b] = acc;
    }
    if (blockIdx.x != 0) return;
    // the step's chains and scalars into its record (the fold of the sums
    // runs later, for several steps at once)
    if (t < kContractM + 2) {
        // entries 0..k+1 of each chain exist (the chains hold m + 3 >= k + 3 values)
        const bool inl = t <= kl + 1, inp = t <= kp + 1;
        a.rec[kRecAlphaL + t] = inl ? a.alpha_lam[t] : 0.0;
        a.rec[kRecGammaL + t] = inl ? a.gamma_lam[t] : 0.0;
        a.rec[kRecAlphaP + t] = inp ? a.alpha_psi[t] : 0.0;
        a.rec[kRecGammaP + t] = inp ? a.gamma_psi[t] : 0.0;
    }
    if (t == 0) {
        a.rec[kRecMeta + 0] = a.sc_lam->sigma;
        a.rec[kRecMeta + 1] = a.sc_psi->sigma;
        a.rec[kRecMeta + 2] = (double)kl;
        a.rec[kRecMeta + 3] = (double)kp;
        a.rec[kRecMeta + 4] = (double)a.sc_lam->status;
        a.rec[kRecMeta + 5] = (double)a.sc_psi->status;
    }
}

// One wave per output (4 kBlock outputs of each of nsteps steps, kWaves per
// workgroup): lane l sums partials l, l + 64, ... of its output in order,
// then a butterfly; the order is fixed by nblocks, so the result is bitwise
// reproducible.  Step i0 + j (j < nsteps) reads its partials from slot
// (i0 + j) % nslot of the partial table (slot stride 4 kBlock nblocks) and
// writes its record rec + (i0 + j) kRecLen.
__global__ __launch_bounds__(kBlock) void k_contract_fold(const double *partials, int nslot, int nblocks,
                                                          double *rec, int i0)
{
    constexpr int kPerStep = 4 * kBlock / kWaves;  // workgroups per step
    const int t = threadIdx.x, lane = t & 63;
    const int step = i0 + (int)blockIdx.x / kPerStep;
    const int o = ((int)blockIdx.x % kPerStep) * kWaves + (t >> 6);
    double v[1] = {0.0};
    const double *src =
        partials + ((size_t)(step % nslot) * 4 * kBlock + (size_t)o) * (size_t)nblocks;
    for (int b = lane; b < nblocks; b += 64) v[0] += src[b];
    wave_sum(v);
    if (lane == 0) rec[(size_t)step * kRecLen + kRecS + o] = v[0];
}

}  // namespace

void launch_observe(const Op &op, const double2 *psi, int loss_kind, Scalars *sc, double *partials,
                    double *obs, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_observe, dim3(nblocks), dim3(kBlock), 0, st, op, psi, loss_kind, sc, partials, obs);
}

void launch_adjoint_seed(const Op &op, const double2 *psi, int loss_kind, const double *obs, double2 *lam,
                         hipStream_t st)
{
    const size_t sites = (size_t)op.nx * op.ny;
    const int nb = (int)std::min<size_t>((sites + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_adjoint_seed, dim3(nb), dim3(kBlock), 0, st, op, psi, loss_kind, obs, lam);
}

void launch_contract(const ContractArgs &a, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_contract, dim3(nblocks), dim3(kBlock), 0, st, a);
}

void launch_contract_fold(const double *partials, int nslot, int nblocks, double *rec, int i0, int nsteps,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_contract_fold, dim3(nsteps * (4 * kBlock / kWaves)), dim3(kBlock), 0, st, partials, nslot,
                       nblocks, rec, i0);
}

}  // namespace dl
