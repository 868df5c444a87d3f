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
// Contraction of the two Krylov bases of one adjoint step (see ContractArgs).
// A workgroup stages a tile of sites of every basis vector in LDS; thread
// t = 16 a + b accumulates pair (a, b); per-workgroup partials are folded in
// fixed order by k_contract_fold.
// ---------------------------------------------------------------------------
constexpr int kTileSites = 32;

__device__ __forceinline__ Site basis_site(const double2 *u1, const char *basis, size_t vec_bytes,
                                                   size_t sites, int v, size_t site)
{
    if (v == 0) return Site{u1[site], u1[sites + site]};
    return *reinterpret_cast<const Site *>(basis + (size_t)(v - 1) * vec_bytes + site * 32);
}

__global__ __launch_bounds__(kBlock) void k_contract(ContractArgs a)
{
    __shared__ double ls[kContractM][kTileSites][4];
    __shared__ double ps[kContractM][kTileSites][4];
    const int kl = a.sc_lam->keff, kp = a.sc_psi->keff;
    const int t = threadIdx.x, pa = t >> 4, pb = t & 15;
    const bool act = pa < kl && pb < kp;
    double s01r = 0.0, s01i = 0.0, s10r = 0.0, s10i = 0.0;
    for (size_t s0 = (size_t)blockIdx.x * kTileSites; s0 < a.sites; s0 += (size_t)gridDim.x * kTileSites) {
        for (int idx = t; idx < kContractM * kTileSites; idx += kBlock) {
            const int v = idx / kTileSites, s = idx % kTileSites;
            const size_t site = s0 + s;
            Site x = Site{make_double2(0.0, 0.0), make_double2(0.0, 0.0)}, y = Site{make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
            if (site < a.sites) {
                if (v < kl) x = basis_site(a.lam1, a.lam_basis, a.vec_bytes, a.sites, v, site);
                if (v < kp) y = basis_site(a.psi1, a.psi_basis, a.vec_bytes, a.sites, v, site);
            }
            ls[v][s][0] = x.a.x;
            ls[v][s][1] = x.a.y;
            ls[v][s][2] = x.b.x;
            ls[v][s][3] = x.b.y;
            ps[v][s][0] = y.a.x;
            ps[v][s][1] = y.a.y;
            ps[v][s][2] = y.b.x;
            ps[v][s][3] = y.b.y;
        }
        __syncthreads();
        if (act) {
            for (int s = 0; s < kTileSites; ++s) {
                const double l0r = ls[pa][s][0], l0i = ls[pa][s][1], l1r = ls[pa][s][2], l1i = ls[pa][s][3];
                const double p0r = ps[pb][s][0], p0i = ps[pb][s][1], p1r = ps[pb][s][2], p1i = ps[pb][s][3];
                // conj(l0) p1 and conj(l1) p0
                s01r += l0r * p1r + l0i * p1i;
                s01i += l0r * p1i - l0i * p1r;
                s10r += l1r * p0r + l1i * p0i;
                s10i += l1r * p0i - l1i * p0r;
            }
        }
        __syncthreads();
    }
    // output o = 4 t + c of this workgroup at partials[o * nblocks + block]:
    // the fold then reads each output's partials contiguously
    const size_t nb = gridDim.x, b = blockIdx.x;
    a.partials[(size_t)(4 * t + 0) * nb + b] = s01r;
    a.partials[(size_t)(4 * t + 1) * nb + b] = s01i;
    a.partials[(size_t)(4 * t + 2) * nb + b] = s10r;
    a.partials[(size_t)(4 * t + 3) * nb + b] = s10i;
}

// One wave per output (4 kBlock outputs, kWaves per workgroup): lane l sums
// partials l, l + 64, ... of its output in order, then a butterfly; the
// order is fixed by nblocks, so the result is bitwise reproducible.  The
// first workgroup also copies the chains and scalars into the record.
__global__ __launch_bounds__(kBlock) void k_contract_fold(ContractArgs a, int nblocks)
{
    const int t = threadIdx.x, lane = t & 63;
    const int o = blockIdx.x * kWaves + (t >> 6);
    double v[1] = {0.0};
    const double *src = a.partials + (size_t)o * nblocks;
    for (int b = lane; b < nblocks; b += 64) v[0] += src[b];
    wave_sum(v);
    if (lane == 0) a.rec[kRecS + o] = v[0];
    if (blockIdx.x != 0) return;
    if (t < kContractM + 2) {
        // entries 0..k+1 of each chain exist (the chains hold m + 3 >= k + 3 values)
        const bool inl = t <= a.sc_lam->keff + 1, inp = t <= a.sc_psi->keff + 1;
        a.rec[kRecAlphaL + t] = inl ? a.alpha_lam[t] : 0.0;
        a.rec[kRecGammaL + t] = inl ? a.gamma_lam[t] : 0.0;
        a.rec[kRecAlphaP + t] = inp ? a.alpha_psi[t] : 0.0;
        a.rec[kRecGammaP + t] = inp ? a.gamma_psi[t] : 0.0;
    }
    if (t == 0) {
        a.rec[kRecMeta + 0] = a.sc_lam->sigma;
        a.rec[kRecMeta + 1] = a.sc_psi->sigma;
        a.rec[kRecMeta + 2] = (double)a.sc_lam->keff;
        a.rec[kRecMeta + 3] = (double)a.sc_psi->keff;
        a.rec[kRecMeta + 4] = (double)a.sc_lam->status;
        a.rec[kRecMeta + 5] = (double)a.sc_psi->status;
    }
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
    hipLaunchKernelGGL(k_contract_fold, dim3(4 * kBlock / kWaves), dim3(kBlock), 0, st, a, nblocks);
}

}  // namespace dl
