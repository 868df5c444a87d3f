// Hermite pseudospectral discretisation (Sec. 5 of Beerwerth & Bauke,
// arXiv:1407.7370) on gfx950: each spinor component is held at the n x n
// collocation points (x_i, y_j) in the variables phi = sqrt(w_i w_j) psi, and
// the derivatives are dense n x n matrices, so H phi is a set of dense
// contractions -- the one matrix-shaped workload of the method.  They run on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup (eight wave64, two per SIMD) owns one problem and runs the
// whole Lanczos recurrence of the eigenvalue mode (Sec. 2, Fig. 1 order) in a
// single launch.  The Lanczos vectors never leave the compute unit: z and q
// live in registers in the matrix-core output layout (each wave owns two
// 16 x 16 tiles of the n x n planes), and the matrix products read D and one
// component of q at a time from LDS.  A batch of problems (other Z, fields,
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
constexpr int kHermWaves = 8;
constexpr int kHermBlock = 64 * kHermWaves;
constexpr int kTilesPerWave = 16 / kHermWaves;  // (64/16)^2 tiles over the waves
// LDS row strides: lane (r, k) of an operand read hits bank group 4r + 2k
// (D, doubles) or r (a staged component, 16-byte values), so the 16 rows of
// a read are on distinct banks.
constexpr int kDStride = 66;
constexpr int kPStride = 65;

struct HermLds {
    double d[kHermMaxN * kDStride];    // D~ / scale
    double2 p[kHermMaxN * kPStride];   // one component of the vector being multiplied
    double x[kHermMaxN];               // scaled nodes
    double red[kHermWaves];
};

typedef v4d Tiles[kTilesPerWave][4];  // planes: Re phi_0, Im phi_0, Re phi_1, Im phi_1

__device__ __forceinline__ double herm_potential(const HermOp &op, double x, double y)
{
    if (op.pot_kind == 1) return -op.vz / sqrt(x * x + y * y + op.va2);
    return 0.0;
}

// Block-wide sum (fixed order: butterfly in the wave, then waves in order).
__device__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kHermWaves; ++i) t += red[i];
    return t;
}

// Visit every element of the wave's tiles: f(tt, r, row, col).  Tile t of
// wave w (t = w + kHermWaves tt) covers rows (y) 16 (t / nt) .. and columns (x)
// 16 (t mod nt) ..; element (i, j) of a tile sits in lane j + 16 (i mod 4),
// register i / 4 of the matrix-core output.
template <class F>
__device__ __forceinline__ void herm_tiles(const HermOp &op, F &&f)
{
    const int nt = op.n / 16, ntiles = nt * nt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int t = w + kHermWaves * tt;
        if (t >= ntiles) continue;
        const int r0 = 16 * (t / nt), c0 = 16 * (t % nt);
#pragma unroll
        for (int r = 0; r < 4; ++r) f(tt, r, r0 + 4 * r + (lane >> 4), c0 + (lane & 15));
    }
}

// Component s of the tiles' vector into the LDS staging plane.
__device__ __forceinline__ void herm_put(const HermOp &op, HermLds &L, const Tiles &q, int s)
{
    herm_tiles(op, [&](int tt, int r, int row, int col) {
        L.p[row * kPStride + col] = make_double2(q[tt][2 * s][r], q[tt][2 * s + 1][r]);
    });
}

// Derivative terms of the staged component into planes P, P + 1 of acc:
// c (-i) D_x phi (the x-derivative, phi D^T along rows) plus sy D_y phi (the
// y-derivative, D phi along columns), both with D = D~ / scale:
//   acc_P   += c Im(phi) D_x^T + sy D_y Re(phi)
//   acc_P+1 -= c Re(phi) D_x^T - sy D_y Im(phi)
template <int P>
__device__ __forceinline__ void herm_deriv(const HermOp &op, const HermLds &L, Tiles &acc, double sy)
{
    const int n = op.n, nt = n / 16, ntiles = nt * nt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const double c = op.c;
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int t = w + kHermWaves * tt;
        if (t >= ntiles) continue;
        const int r0 = 16 * (t / nt), c0 = 16 * (t % nt);
        const double2 *pa = L.p + (r0 + lr) * kPStride + lk;   // A of the x-product: phi[r0 + lr][k]
        const double2 *pb = L.p + lk * kPStride + c0 + lr;     // B of the y-product: phi[k][c0 + lr]
        const double *dx = L.d + (c0 + lr) * kDStride + lk;    // B of the x-product: D[c0 + lr][k]
        const double *dy = L.d + (r0 + lr) * kDStride + lk;    // A of the y-product: D[r0 + lr][k]
        v4d a0 = acc[tt][P], a1 = acc[tt][P + 1];
        for (int kb = 0; kb < n / 4; ++kb) {
            const double2 fa = pa[4 * kb];
            const double2 fb = pb[4 * kb * kPStride];
            const double ex = dx[4 * kb], ey = dy[4 * kb];
            a0 = mfma(c * fa.y, ex, a0);
            a1 = mfma(-c * fa.x, ex, a1);
            a0 = mfma(ey, sy * fb.x, a0);
            a1 = mfma(ey, sy * fb.y, a1);
        }
        acc[tt][P] = a0;
        acc[tt][P + 1] = a1;
    }
}

// z += H q on the wave's tiles (q and z in the output layout):
//   (H q)_0 = (mc2 + V) q_0 + c [-i D_x q_1 - chi D_y q_1] - q c (A_x - i chi A_y) q_1
//   (H q)_1 = (V - mc2) q_1 + c [-i D_x q_0 + chi D_y q_0] - q c (A_x + i chi A_y) q_0
__device__ void herm_matvec(const HermOp &op, HermLds &L, const Tiles &q, Tiles &z)
{
    const double cchi = op.c * op.chi;
    __syncthreads();  // the staging plane is free
    herm_put(op, L, q, 1);
    __syncthreads();
    herm_deriv<0>(op, L, z, -cchi);
    __syncthreads();
    herm_put(op, L, q, 0);
    __syncthreads();
    herm_deriv<2>(op, L, z, cchi);
    // site terms
    herm_tiles(op, [&](int tt, int r, int row, int col) {
        const double x = L.x[col], y = L.x[row];
        const double v = herm_potential(op, x, y);
        const double d0 = op.mc2 + v, d1 = v - op.mc2;
        // g = -q c A with A = (B/2)(-y, x): gx = bq y, chi gy = -chi bq x
        // (bq = c q B / 2); coupling (gx -+ i chi gy) to the other component
        const double gx = op.bq * y, gy = -op.bq * x * op.chi;
        const double f0x = q[tt][0][r], f0y = q[tt][1][r], f1x = q[tt][2][r], f1y = q[tt][3][r];
        z[tt][0][r] += d0 * f0x + gx * f1x + gy * f1y;
        z[tt][1][r] += d0 * f0y + gx * f1y - gy * f1x;
        z[tt][2][r] += d1 * f1x + gx * f0x - gy * f0y;
        z[tt][3][r] += d1 * f1y + gx * f0y + gy * f0x;
    });
}

// Stage D~ / scale and the scaled nodes of a problem in LDS.
__device__ void herm_stage(const HermOp &op, HermLds &L)
{
    const int n = op.n;
    for (int i = threadIdx.x; i < n * n; i += kHermBlock) L.d[(i / n) * kDStride + (i % n)] = op.dmat[i];
    for (int i = threadIdx.x; i < n; i += kHermBlock) L.x[i] = op.x[i];
    __syncthreads();
}

// A global spinor (layout (2, n, n)) at the wave's tile elements.
__device__ void herm_load(const HermOp &op, const double2 *__restrict__ v, Tiles &q)
{
    const size_t plane = (size_t)op.n * op.n;
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
        for (int p = 0; p < 4; ++p) q[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
    herm_tiles(op, [&](int tt, int r, int row, int col) {
        const size_t s = (size_t)row * op.n + col;
        const double2 a = v[s], b = v[plane + s];
        q[tt][0][r] = a.x;
        q[tt][1][r] = a.y;
        q[tt][2][r] = b.x;
        q[tt][3][r] = b.y;
    });
}

__global__ __launch_bounds__(kHermBlock) void k_herm_apply(const HermOp *ops, const double2 *const *x,
                                                           double2 *const *y)
{
    __shared__ HermLds L;
    const HermOp op = ops[blockIdx.x];
    herm_stage(op, L);
    Tiles q, z;
    herm_load(op, x[blockIdx.x], q);
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
        for (int p = 0; p < 4; ++p) z[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
    herm_matvec(op, L, q, z);
    double2 *out = y[blockIdx.x];
    const size_t plane = (size_t)op.n * op.n;
    herm_tiles(op, [&](int tt, int r, int row, int col) {
        const size_t s = (size_t)row * op.n + col;
        out[s] = make_double2(z[tt][0][r], z[tt][1][r]);
        out[plane + s] = make_double2(z[tt][2][r], z[tt][3][r]);
    });
}

// The Lanczos recurrence of Fig. 1 (three vectors, no reorthogonalisation)
// on one problem per workgroup:
//   q_1 = b / ||b||; z = H q_1;
//   i = 1..k: alpha_i = Re <q_i, z>; z -= alpha_i q_i; beta_i = ||z||;
//             stop at k or on breakdown (beta_i <= 1e-13 max_j(|alpha_j|, beta_{j-1}));
//             q_{i+1} = z / beta_i; z = H q_{i+1} - beta_i q_i.
// Every element of the n x n planes belongs to exactly one lane and register
// of one wave, so the inner products are sums over the tiles.  Two vectors
// are live: q (q_i, then q_{i+1}) and z, which starts a product as -beta_i q_i.
__global__ __launch_bounds__(kHermBlock) void k_herm_lanczos(const HermOp *ops, HermRun *runs, int k_max)
{
    __shared__ HermLds L;
    const HermOp op = ops[blockIdx.x];
    HermRun &run = runs[blockIdx.x];
    herm_stage(op, L);
    Tiles qn, z;
    herm_load(op, run.b, qn);
    double s = 0.0;
    herm_tiles(op, [&](int tt, int r, int, int) {
#pragma unroll
        for (int p = 0; p < 4; ++p) s += qn[tt][p][r] * qn[tt][p][r];
    });
    const double nb2 = block_sum(s, L.red);
    if (!(nb2 > 0.0) || !isfinite(nb2)) {
        if (threadIdx.x == 0) run.keff = isfinite(nb2) ? 0 : -1;
        return;
    }
    const double inb = 1.0 / sqrt(nb2);
#pragma unroll
    for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            qn[tt][p] *= inb;
            z[tt][p] = v4d{0.0, 0.0, 0.0, 0.0};
        }
    herm_matvec(op, L, qn, z);
    double scale = 0.0, beta_prev = 0.0;
    int keff = k_max;
    for (int i = 1; i <= k_max; ++i) {
        double pa = 0.0;
        herm_tiles(op, [&](int tt, int r, int, int) {
#pragma unroll
            for (int p = 0; p < 4; ++p) pa += qn[tt][p][r] * z[tt][p][r];
        });
        const double alpha = block_sum(pa, L.red);
        double pn = 0.0;
        herm_tiles(op, [&](int tt, int r, int, int) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                z[tt][p][r] -= alpha * qn[tt][p][r];
                pn += z[tt][p][r] * z[tt][p][r];
            }
        });
        const double beta = sqrt(block_sum(pn, L.red));
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
        // q_{i+1} = z / beta_i; z = H q_{i+1} - beta_i q_i
        const double ib = 1.0 / beta;
#pragma unroll
        for (int tt = 0; tt < kTilesPerWave; ++tt)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const v4d next = z[tt][p] * ib;
                z[tt][p] = -beta * qn[tt][p];
                qn[tt][p] = next;
            }
        herm_matvec(op, L, qn, z);
        beta_prev = beta;
    }
    if (threadIdx.x == 0) run.keff = keff;
}

}  // namespace

void launch_herm_apply(const HermOp *ops, const double2 *const *x, double2 *const *y, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_herm_apply, dim3(n), dim3(kHermBlock), 0, st, ops, x, y);
}

void launch_herm_lanczos(const HermOp *ops, HermRun *runs, int n, int k_max, hipStream_t st)
{
    hipLaunchKernelGGL(k_herm_lanczos, dim3(n), dim3(kHermBlock), 0, st, ops, runs, k_max);
}

}  // namespace dl
