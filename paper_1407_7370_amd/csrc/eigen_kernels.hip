// gfx950 kernels of the eigenvalue mode with full reorthogonalisation
// (Sec. 2: the Lanczos vectors are kept and every new vector is
// orthogonalised against all of them, twice) and of the Ritz vectors
// (Sec. 2 eq. eigenvec_approx).
//
// Classical Gram-Schmidt in two passes (CGS2): h = Q^H z, z -= Q h, twice.
// The projections of a pass all use the same z, so one pass is a
// tall-skinny product that streams the stored basis once; the modified form
// would stream it once per vector.  Every kernel here is bound by HBM
// bandwidth: per pass, the projection reads the i stored vectors and z, the
// update reads them again and rewrites z.  Reductions are per-workgroup
// partials folded in a fixed order, so results are bitwise reproducible.
//
// Vectors use the state layout (complex128, both spinor planes), vector j
// (0-based) of the basis at q + j * vstride bytes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_reduce.h"
#include "dl_internal.h"

namespace dl {
namespace {

#ifndef DL_DOT_VECS
#define DL_DOT_VECS 16
#endif
#ifndef DL_PROJ_WORKGROUPS
#define DL_PROJ_WORKGROUPS 8192
#endif
constexpr int kDotVecs = DL_DOT_VECS;  // basis vectors per workgroup of a projection
// workgroups of a projection launch (at most kProjTiles per vector chunk);
// measured on 1024^2 with K = 500: 2048 -> 3.30 s, 4096 -> 3.26 s, 8192 -> 3.21 s
constexpr int kProjWorkgroups = DL_PROJ_WORKGROUPS;
constexpr int kSubChunk = 256;  // coefficients staged in LDS per chunk of the update
static_assert(kSubChunk % kDotVecs == 0, "the update pads a chunk to whole groups of kDotVecs");
constexpr int kRitzChunk = 64;  // basis rows of t staged in LDS per chunk

__device__ __forceinline__ const double2 *qvec(const char *q, size_t vstride, int j)
{
    return reinterpret_cast<const double2 *>(q + (size_t)j * vstride);
}

// Partial projections.  Workgroup (t, c) accumulates conj(q_j) . z over the
// elements t*256 + tid + r * ntiles*256 for the 16 vectors j = 16c .. 16c+15
// (< nvec) and writes them to pproj[(j * ntiles + t) * 2 + {re, im}].
__global__ __launch_bounds__(kBlock) void k_proj(const char *__restrict__ q, size_t vstride, int nvec,
                                                 const double2 *__restrict__ z, size_t nelem,
                                                 double *__restrict__ pproj, int ntiles)
{
    __shared__ double red[kWaves][2 * kDotVecs];
    const int t = blockIdx.x, j0 = blockIdx.y * kDotVecs;
    const int nj = min(kDotVecs, nvec - j0);
    double re[kDotVecs], im[kDotVecs];
#pragma unroll
    for (int jj = 0; jj < kDotVecs; ++jj) re[jj] = im[jj] = 0.0;
    for (size_t e = (size_t)t * kBlock + threadIdx.x; e < nelem; e += (size_t)ntiles * kBlock) {
        const double2 zv = z[e];
        // every load unconditional (a short last chunk re-reads its last
        // vector into accumulators that are never written out), so the 16
        // loads of a site are in flight together
#pragma unroll
        for (int jj = 0; jj < kDotVecs; ++jj) {
            const double2 qv = qvec(q, vstride, j0 + min(jj, nj - 1))[e];
            re[jj] += qv.x * zv.x + qv.y * zv.y;
            im[jj] += qv.x * zv.y - qv.y * zv.x;
        }
    }
    wave_sum(re);
    wave_sum(im);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int jj = 0; jj < kDotVecs; ++jj) {
            red[w][2 * jj] = re[jj];
            red[w][2 * jj + 1] = im[jj];
        }
    __syncthreads();
    if (threadIdx.x < 2 * nj) {
        double a = red[0][threadIdx.x];
        for (int i = 1; i < kWaves; ++i) a += red[i][threadIdx.x];
        const int jj = threadIdx.x >> 1, part = threadIdx.x & 1;
        pproj[((size_t)(j0 + jj) * ntiles + t) * 2 + part] = a;
    }
}

// h_j = sum of the ntiles partials of vector j (workgroup j; fixed order).
__global__ __launch_bounds__(kBlock) void k_proj_fold(const double *__restrict__ pproj, int ntiles, double *h)
{
    __shared__ double red[kWaves][2];
    const int j = blockIdx.x;
    double s[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < ntiles; t += kBlock) {
        s[0] += pproj[((size_t)j * ntiles + t) * 2];
        s[1] += pproj[((size_t)j * ntiles + t) * 2 + 1];
    }
    wave_sum(s);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[w][0] = s[0];
        red[w][1] = s[1];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = red[0][threadIdx.x];
        for (int i = 1; i < kWaves; ++i) a += red[i][threadIdx.x];
        h[2 * j + threadIdx.x] = a;
    }
}

// z -= sum_j h_j q_j.  The loop over element tiles has a workgroup-uniform
// trip count (the LDS staging of h needs every thread at the barriers).
__global__ __launch_bounds__(kBlock) void k_sub_q(const char *__restrict__ q, size_t vstride, int nvec,
                                                  const double *__restrict__ h, double2 *__restrict__ z,
                                                  size_t nelem)
{
    __shared__ double hs[2 * kSubChunk];
    const size_t step = (size_t)gridDim.x * kBlock;
    for (size_t base = (size_t)blockIdx.x * kBlock; base < nelem; base += step) {
        const size_t e = base + threadIdx.x;
        const bool live = e < nelem;
        double ar = 0.0, ai = 0.0;
        for (int j0 = 0; j0 < nvec; j0 += kSubChunk) {
            const int nj = min(kSubChunk, nvec - j0);
            // coefficients padded with zeros to whole groups of kDotVecs, so
            // each group issues all its loads before the first use
            const int njp = (nj + kDotVecs - 1) / kDotVecs * kDotVecs;
            __syncthreads();
            for (int i = threadIdx.x; i < 2 * njp; i += kBlock) hs[i] = i < 2 * nj ? h[2 * (size_t)j0 + i] : 0.0;
            __syncthreads();
            if (live) {
                for (int jb = 0; jb < njp; jb += kDotVecs) {
                    double2 qv[kDotVecs];
#pragma unroll
                    for (int u = 0; u < kDotVecs; ++u) qv[u] = qvec(q, vstride, j0 + min(jb + u, nj - 1))[e];
                    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the arithmetic
#pragma unroll
                    for (int u = 0; u < kDotVecs; ++u) {
                        const double hr = hs[2 * (jb + u)], hi = hs[2 * (jb + u) + 1];
                        ar += hr * qv[u].x - hi * qv[u].y;
                        ai += hr * qv[u].y + hi * qv[u].x;
                    }
                }
            }
        }
        if (live) {
            const double2 zv = z[e];
            z[e] = make_double2(zv.x - ar, zv.y - ai);
        }
    }
}

// beta_0 = ||psi|| (grid-wide fixed-order reduction); kstop = 0 for psi = 0,
// status 3 when the norm is not finite.
__global__ __launch_bounds__(kBlock) void k_first_norm(const double2 *__restrict__ psi, size_t nelem,
                                                       Scalars *sc, double *beta, double *partials)
{
    double s[1] = {0.0};
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < nelem; e += (size_t)gridDim.x * kBlock) {
        const double2 v = psi[e];
        s[0] += v.x * v.x + v.y * v.y;
    }
    double tot[1];
    if (!grid_reduce(s, partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        const double b = sqrt(tot[0]);
        beta[0] = b;
        sc->scale = 0.0;
        sc->keff = 0;
        if (!isfinite(b)) {
            sc->status = 3;
            sc->kstop = -1;
        } else {
            sc->kstop = b > 0.0 ? 0x40000000 : 0;
        }
    }
}

// out = in / beta[idx] while the recurrence goes on past iteration idx.
__global__ __launch_bounds__(kBlock) void k_scale_q(const double2 *__restrict__ in, size_t nelem,
                                                    double2 *__restrict__ out, const double *beta, int idx,
                                                    const Scalars *sc)
{
    if (sc->kstop <= idx) return;
    const double ib = 1.0 / beta[idx];
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < nelem; e += (size_t)gridDim.x * kBlock) {
        const double2 v = in[e];
        out[e] = make_double2(v.x * ib, v.y * ib);
    }
}

// Scalar update of iteration i from ||z||^2: alpha_i = Re h1_i (first
// projection pass), beta_i = ||z||, the running scale max(|alpha_j|,
// beta_{j-1}) and the breakdown test beta_i <= 1e-13 scale, which stops the
// recurrence with k_eff = i (the Krylov space is invariant).
__global__ __launch_bounds__(kBlock) void k_norm_update(const double2 *__restrict__ z, size_t nelem,
                                                        const double *__restrict__ h1, int i, double *alpha,
                                                        double *beta, Scalars *sc, double *partials)
{
    double s[1] = {0.0};
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < nelem; e += (size_t)gridDim.x * kBlock) {
        const double2 v = z[e];
        s[0] += v.x * v.x + v.y * v.y;
    }
    double tot[1];
    if (!grid_reduce(s, partials, &sc->ticket, tot)) return;
    if (threadIdx.x != 0 || sc->kstop < i) return;
    const double al = h1[2 * (i - 1)];
    const double b = sqrt(tot[0]);
    if (!isfinite(b) || !isfinite(al)) {
        sc->status = 3;
        sc->kstop = -1;
        return;
    }
    alpha[i] = al;
    beta[i] = b;
    double scale = fmax(sc->scale, fabs(al));
    if (i > 1) scale = fmax(scale, beta[i - 1]);
    sc->scale = scale;
    sc->keff = i;
    if (b <= 1e-13 * scale) sc->kstop = i;
}

// Y[:, v] = sum_j t[j][v] q_j for v < r: the basis is streamed once for up to
// kRitzVecs vectors; rows of t are staged in LDS.
__global__ __launch_bounds__(kBlock) void k_ritz(const char *__restrict__ q, size_t vstride, int nvec,
                                                 const double *__restrict__ t, int r, double2 *__restrict__ y,
                                                 size_t nelem)
{
    __shared__ double ts[kRitzChunk][kRitzVecs];
    const size_t step = (size_t)gridDim.x * kBlock;
    for (size_t base = (size_t)blockIdx.x * kBlock; base < nelem; base += step) {
        const size_t e = base + threadIdx.x;
        const bool live = e < nelem;
        double ar[kRitzVecs], ai[kRitzVecs];
#pragma unroll
        for (int v = 0; v < kRitzVecs; ++v) ar[v] = ai[v] = 0.0;
        for (int j0 = 0; j0 < nvec; j0 += kRitzChunk) {
            const int nj = min(kRitzChunk, nvec - j0);
            __syncthreads();
            for (int i = threadIdx.x; i < nj * kRitzVecs; i += kBlock)
                ts[i / kRitzVecs][i % kRitzVecs] = t[(size_t)j0 * kRitzVecs + i];
            __syncthreads();
            if (live)
                for (int jj = 0; jj < nj; ++jj) {
                    const double2 qv = qvec(q, vstride, j0 + jj)[e];
#pragma unroll
                    for (int v = 0; v < kRitzVecs; ++v) {
                        ar[v] += ts[jj][v] * qv.x;
                        ai[v] += ts[jj][v] * qv.y;
                    }
                }
        }
        if (live)
#pragma unroll
            for (int v = 0; v < kRitzVecs; ++v)
                if (v < r) y[(size_t)v * nelem + e] = make_double2(ar[v], ai[v]);
    }
}

}  // namespace

void launch_proj(const char *q, size_t vstride, int nvec, const double2 *z, size_t nelem, double *pproj,
                 double *h, hipStream_t st)
{
    const int nchunk = (nvec + kDotVecs - 1) / kDotVecs;
    const int ntiles = std::max(1, std::min(proj_tiles(nelem), kProjWorkgroups / nchunk));
    hipLaunchKernelGGL(k_proj, dim3(ntiles, nchunk), dim3(kBlock), 0, st, q, vstride, nvec, z, nelem, pproj,
                       ntiles);
    hipLaunchKernelGGL(k_proj_fold, dim3(nvec), dim3(kBlock), 0, st, pproj, ntiles, h);
}

void launch_sub_q(const char *q, size_t vstride, int nvec, const double *h, double2 *z, size_t nelem, int nblocks,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_sub_q, dim3(nblocks), dim3(kBlock), 0, st, q, vstride, nvec, h, z, nelem);
}

void launch_first_q(const double2 *psi, size_t nelem, double2 *q1, Scalars *sc, double *beta, double *partials,
                    int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_first_norm, dim3(nblocks), dim3(kBlock), 0, st, psi, nelem, sc, beta, partials);
    hipLaunchKernelGGL(k_scale_q, dim3(nblocks), dim3(kBlock), 0, st, psi, nelem, q1, beta, 0, sc);
}

void launch_norm_next(const double2 *z, size_t nelem, const double *h1, int i, int k, double *alpha, double *beta,
                      Scalars *sc, double *partials, double2 *qn, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_update, dim3(nblocks), dim3(kBlock), 0, st, z, nelem, h1, i, alpha, beta, sc,
                       partials);
    if (i < k) hipLaunchKernelGGL(k_scale_q, dim3(nblocks), dim3(kBlock), 0, st, z, nelem, qn, beta, i, sc);
}

void launch_ritz(const char *q, size_t vstride, int nvec, const double *t, int r, double2 *y, size_t nelem,
                 int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_ritz, dim3(nblocks), dim3(kBlock), 0, st, q, vstride, nvec, t, r, y, nelem);
}

}  // namespace dl
