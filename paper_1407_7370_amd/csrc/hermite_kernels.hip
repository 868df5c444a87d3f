// Hermite pseudospectral discretisation (Sec. 5 of Beerwerth & Bauke,
// arXiv:1407.7370) on gfx950: each spinor component is held at the n x n
// collocation points (x_i, y_j) in the variables phi = sqrt(w_i w_j) psi, and
// the derivatives are dense n x n matrices, so H phi is a set of dense
// contractions -- the one matrix-shaped workload of the method.  They run on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup (four wave64) owns one problem and runs the whole Lanczos
// recurrence of the eigenvalue mode (Sec. 2, Fig. 1 order, three vectors in
// global memory) in a single launch; a batch of problems (other Z, fields,
// chirality) runs on as many compute units.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dl_internal.h"

namespace dl {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kHermMaxN = 64;
constexpr int kTilesPerWave = 4;  // (64/16)^2 tiles over four waves

__device__ __forceinline__ double herm_potential(const HermOp &op, double x, double y)
{
    if (op.pot_kind == 1) return -op.vz / sqrt(x * x + y * y + op.va2);
    return 0.0;
}

// Block-wide sum (fixed order: butterfly in the wave, then waves 0..3).
__device__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// z = H phi on the tiles of this wave, in the matrix-core output layout: tile
// t of the wave covers rows (y) 16 ti .. and columns (x) 16 tj ..; element
// (i, j) of a tile sits in lane j + 16 (i mod 4), register i / 4.  acc[t][c]:
// plane c = 0 Re z_0, 1 Im z_0, 2 Re z_1, 3 Im z_1.  x-derivative
// (D phi^T)^T = phi D^T, y-derivative D phi, both with D = D~ / scale:
//   z_0 = (mc2 + V) phi_0 + c [-i D_x phi_1 - chi D_y phi_1] - q c (A_x - i chi A_y) phi_1
//   z_1 = (V - mc2) phi_1 + c [-i D_x phi_0 + chi D_y phi_0] - q c (A_x + i chi A_y) phi_0
// cur holds a vector q at the same elements on entry: z -= bsub q is folded
// in (the recurrence's - beta_i q_i), and cur then receives phi there.
__device__ void herm_matvec(const HermOp &op, const double *__restrict__ dsh, const double *__restrict__ xsh,
                            const double2 *__restrict__ phi, v4d (&acc)[kTilesPerWave][4],
                            v4d (&cur)[kTilesPerWave][4], double bsub)
{
    const int n = op.n, nt = n / 16, ntiles = nt * nt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const size_t plane = (size_t)n * n;
    const double c = op.c, cchi = op.c * op.chi;
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int t = w + 4 * tt;
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
        if (t >= ntiles) continue;
        const int r0 = 16 * (t / nt), c0 = 16 * (t % nt);
        for (int kb = 0; kb < n / 4; ++kb) {
            const int k = 4 * kb + lk;
            // x-derivative: A = phi[r0 + lr][k], B = D[c0 + lr][k]
            const double2 q0 = phi[(size_t)(r0 + lr) * n + k];
            const double2 q1 = phi[plane + (size_t)(r0 + lr) * n + k];
            const double dx = dsh[(c0 + lr) * kHermMaxN + k];
            acc[tt][0] = mfma(c * q1.y, dx, acc[tt][0]);
            acc[tt][1] = mfma(-c * q1.x, dx, acc[tt][1]);
            acc[tt][2] = mfma(c * q0.y, dx, acc[tt][2]);
            acc[tt][3] = mfma(-c * q0.x, dx, acc[tt][3]);
            // y-derivative: A = D[r0 + lr][k], B = phi[k][c0 + lr]
            const double dy = dsh[(r0 + lr) * kHermMaxN + k];
            const double2 p0 = phi[(size_t)k * n + c0 + lr];
            const double2 p1 = phi[plane + (size_t)k * n + c0 + lr];
            acc[tt][0] = mfma(dy, -cchi * p1.x, acc[tt][0]);
            acc[tt][1] = mfma(dy, -cchi * p1.y, acc[tt][1]);
            acc[tt][2] = mfma(dy, cchi * p0.x, acc[tt][2]);
            acc[tt][3] = mfma(dy, cchi * p0.y, acc[tt][3]);
        }
        // site terms
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int iy = r0 + 4 * r + lk, ix = c0 + lr;
            const double x = xsh[ix], y = xsh[iy];
            const double2 f0 = phi[(size_t)iy * n + ix], f1 = phi[plane + (size_t)iy * n + ix];
            const double v = herm_potential(op, x, y);
            const double d0 = op.mc2 + v, d1 = v - op.mc2;
            // g = -q c A with A = (B/2)(-y, x): gx = bq y, chi gy = -chi bq x
            // (bq = c q B / 2); coupling (gx -+ i chi gy) to the other component
            const double gx = op.bq * y, gy = -op.bq * x * op.chi;
            acc[tt][0][r] += d0 * f0.x + gx * f1.x + gy * f1.y - bsub * cur[tt][0][r];
            acc[tt][1][r] += d0 * f0.y + gx * f1.y - gy * f1.x - bsub * cur[tt][1][r];
            acc[tt][2][r] += d1 * f1.x + gx * f0.x - gy * f0.y - bsub * cur[tt][2][r];
            acc[tt][3][r] += d1 * f1.y + gx * f0.y + gy * f0.x - bsub * cur[tt][3][r];
            cur[tt][0][r] = f0.x;
            cur[tt][1][r] = f0.y;
            cur[tt][2][r] = f1.x;
            cur[tt][3][r] = f1.y;
        }
    }
}

// Stage D~ / scale and the scaled nodes of a problem in LDS.
__device__ void herm_stage(const HermOp &op, double *dsh, double *xsh)
{
    const int n = op.n;
    for (int i = threadIdx.x; i < n * n; i += kBlock) dsh[(i / n) * kHermMaxN + (i % n)] = op.dmat[i];
    for (int i = threadIdx.x; i < n; i += kBlock) xsh[i] = op.x[i];
    __syncthreads();
}

// Visit every element of the wave's tiles: f(tt, plane, r, site index of the plane).
template <class F>
__device__ __forceinline__ void herm_tiles(const HermOp &op, F &&f)
{
    const int n = op.n, nt = n / 16, ntiles = nt * nt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int t = w + 4 * tt;
        if (t >= ntiles) continue;
        const int r0 = 16 * (t / nt), c0 = 16 * (t % nt);
#pragma unroll
        for (int r = 0; r < 4; ++r) f(tt, r, (size_t)(r0 + 4 * r + (lane >> 4)) * n + c0 + (lane & 15));
    }
}

__global__ __launch_bounds__(kBlock) void k_herm_apply(const HermOp *ops, const double2 *const *x,
                                                       double2 *const *y)
{
    __shared__ double dsh[kHermMaxN * kHermMaxN];
    __shared__ double xsh[kHermMaxN];
    const HermOp op = ops[blockIdx.x];
    herm_stage(op, dsh, xsh);
    v4d acc[kTilesPerWave][4], cur[kTilesPerWave][4];
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
        for (int p = 0; p < 4; ++p) cur[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
    herm_matvec(op, dsh, xsh, x[blockIdx.x], acc, cur, 0.0);
    double2 *out = y[blockIdx.x];
    const size_t plane = (size_t)op.n * op.n;
    herm_tiles(op, [&](int tt, int r, size_t s) {
        out[s] = make_double2(acc[tt][0][r], acc[tt][1][r]);
        out[plane + s] = make_double2(acc[tt][2][r], acc[tt][3][r]);
    });
}

// The Lanczos recurrence of Fig. 1 (three vectors, no reorthogonalisation)
// on one problem per workgroup:
//   q_1 = b / ||b||; z = H q_1;
//   i = 1..k: alpha_i = Re <q_i, z>; z -= alpha_i q_i; beta_i = ||z||;
//             stop at k or on breakdown (beta_i <= 1e-13 max_j(|alpha_j|, beta_{j-1}));
//             q_{i+1} = z / beta_i; z = H q_{i+1} - beta_i q_i.
// z lives in registers (the tiles' output layout); q_i and q_{i-1} in two
// global buffers per problem.
__global__ __launch_bounds__(kBlock) void k_herm_lanczos(const HermOp *ops, HermRun *runs, int k_max)
{
    __shared__ double dsh[kHermMaxN * kHermMaxN];
    __shared__ double xsh[kHermMaxN];
    __shared__ double red[4];
    const HermOp op = ops[blockIdx.x];
    HermRun &run = runs[blockIdx.x];
    herm_stage(op, dsh, xsh);
    const size_t plane = (size_t)op.n * op.n, nel = 2 * plane;
    double2 *qa = run.q[0], *qb = run.q[1];
    // q_1 = b / ||b||
    double s = 0.0;
    for (size_t i = threadIdx.x; i < nel; i += kBlock) {
        const double2 v = run.b[i];
        s += v.x * v.x + v.y * v.y;
    }
    const double nb2 = block_sum(s, red);
    if (!(nb2 > 0.0) || !isfinite(nb2)) {
        if (threadIdx.x == 0) run.keff = isfinite(nb2) ? 0 : -1;
        return;
    }
    const double inb = 1.0 / sqrt(nb2);
    for (size_t i = threadIdx.x; i < nel; i += kBlock) {
        const double2 v = run.b[i];
        qa[i] = make_double2(v.x * inb, v.y * inb);
    }
    __threadfence();
    __syncthreads();
    v4d z[kTilesPerWave][4], qc[kTilesPerWave][4];
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
        for (int p = 0; p < 4; ++p) qc[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
    herm_matvec(op, dsh, xsh, qa, z, qc, 0.0);
    double scale = 0.0, beta_prev = 0.0;
    int keff = k_max;
    for (int i = 1; i <= k_max; ++i) {
        double pa = 0.0;
        herm_tiles(op, [&](int tt, int r, size_t) {
#pragma unroll
            for (int p = 0; p < 4; ++p) pa += qc[tt][p][r] * z[tt][p][r];
        });
        const double alpha = block_sum(pa, red);
        double pn = 0.0;
        herm_tiles(op, [&](int tt, int r, size_t) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                z[tt][p][r] -= alpha * qc[tt][p][r];
                pn += z[tt][p][r] * z[tt][p][r];
            }
        });
        const double beta = sqrt(block_sum(pn, red));
        if (threadIdx.x == 0) {
            run.alpha[i - 1] = alpha;
            run.beta[i - 1] = beta;
        }
        if (!isfinite(alpha) || !isfinite(beta)) {
            keff = -1;
            break;
        }
        scale = fmax(scale, fabs(alpha));
        if (i > 1) scale = fmax(scale, beta_prev);
        if (i == k_max) break;
        if (beta <= 1e-13 * scale) {
            keff = i;
            break;
        }
        // q_{i+1} = z / beta_i into the older buffer; z = H q_{i+1} - beta_i q_i
        const double ib = 1.0 / beta;
        herm_tiles(op, [&](int tt, int r, size_t st) {
            qb[st] = make_double2(z[tt][0][r] * ib, z[tt][1][r] * ib);
            qb[plane + st] = make_double2(z[tt][2][r] * ib, z[tt][3][r] * ib);
        });
        __threadfence();
        __syncthreads();
        herm_matvec(op, dsh, xsh, qb, z, qc, beta);
        double2 *tmp = qa;
        qa = qb;
        qb = tmp;
        beta_prev = beta;
        __syncthreads();  // every wave has read q_{i-1} (now qb) before it is overwritten
    }
    if (threadIdx.x == 0) run.keff = keff;
}

}  // namespace

void launch_herm_apply(const HermOp *ops, const double2 *const *x, double2 *const *y, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_herm_apply, dim3(n), dim3(kBlock), 0, st, ops, x, y);
}

void launch_herm_lanczos(const HermOp *ops, HermRun *runs, int n, int k_max, hipStream_t st)
{
    hipLaunchKernelGGL(k_herm_lanczos, dim3(n), dim3(kBlock), 0, st, ops, runs, k_max);
}

}  // namespace dl
