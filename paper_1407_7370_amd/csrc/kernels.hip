// gfx950 kernels of the Lanczos short-time propagator for the 2D Dirac
// equation (Beerwerth & Bauke, arXiv:1407.7370).
//
// Layout: a spinor is two planes (components) of ny rows of nx complex values,
// x fastest.  Every sweep kernel maps one wave64 to a strip of columns and a
// chunk of rows and marches down the rows: lane l holds column
// strip*own - halo + l, neighbours in x come from the adjacent lanes through
// DPP wave rotations, neighbours in y from a three-row register ring.  No LDS
// tile and no barrier is needed inside the march; the `halo` edge lanes of a
// wave only feed their neighbours.  Reductions are per-lane FP64 sums folded
// by a fixed butterfly, per workgroup, and finally by the last workgroup to
// finish in fixed order, so results are bitwise reproducible.
//
// A sweep p >= 2 fuses one whole Lanczos iteration of Fig. 1 (Sec. 2) into one
// pass over memory: with u_i = gamma_i q_i (gamma_i = ||u_i|| = beta_{i-1})
//   u_p = (A u_{p-1} - alpha_{p-1} u_{p-1}) / gamma_{p-1}
//         - (gamma_{p-1} / gamma_{p-2}) u_{p-2}                  (eq. lanczos_base)
// is formed on the tile plus a one-site rim (A u_{p-1} is recomputed there
// from u_{p-1} with a two-site rim), stored, and A u_p is applied on the tile
// to reduce ||u_p||^2, Re<u_p, A u_p> and Re<u_p, u_{p-1}>.  From these the
// last workgroup forms gamma_p and alpha_p = Re<q_p, A q_p> - beta_{p-1}
// Re<q_p, q_{p-1}>, the modified Gram-Schmidt form of Fig. 1.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dl_internal.h"

namespace dl {
namespace {

struct Sp {
    double r0, i0, r1, i1;  // component 0 (re, im), component 1 (re, im)
};

__device__ __forceinline__ Sp sp_zero() { return Sp{0.0, 0.0, 0.0, 0.0}; }

// DPP wave rotations: wave_ror:1 delivers the value of lane l-1 to lane l,
// wave_rol:1 the value of lane l+1.  Lanes 0 and 63 receive wrapped values
// that only feed rim lanes whose results are discarded.
__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x13C, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x13C, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x134, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ Sp sp_left(const Sp &s)
{
    return Sp{from_left(s.r0), from_left(s.i0), from_left(s.r1), from_left(s.i1)};
}

__device__ __forceinline__ Sp sp_right(const Sp &s)
{
    return Sp{from_right(s.r0), from_right(s.i0), from_right(s.r1), from_right(s.i1)};
}

template <class T>
struct Vec;

template <>
struct Vec<double2> {
    static __device__ __forceinline__ Sp load(const double2 *b, size_t plane, size_t off)
    {
        const double2 a = b[off];
        const double2 c = b[plane + off];
        return Sp{a.x, a.y, c.x, c.y};
    }
    static __device__ __forceinline__ void store(double2 *b, size_t plane, size_t off, const Sp &s)
    {
        b[off] = make_double2(s.r0, s.i0);
        b[plane + off] = make_double2(s.r1, s.i1);
    }
    static __device__ __forceinline__ Sp round(const Sp &s) { return s; }
};

template <>
struct Vec<float2> {
    static __device__ __forceinline__ Sp load(const float2 *b, size_t plane, size_t off)
    {
        const float2 a = b[off];
        const float2 c = b[plane + off];
        return Sp{(double)a.x, (double)a.y, (double)c.x, (double)c.y};
    }
    static __device__ __forceinline__ void store(float2 *b, size_t plane, size_t off, const Sp &s)
    {
        b[off] = make_float2((float)s.r0, (float)s.i0);
        b[plane + off] = make_float2((float)s.r1, (float)s.i1);
    }
    // The value that a later sweep will read back from storage.
    static __device__ __forceinline__ Sp round(const Sp &s)
    {
        return Sp{(double)(float)s.r0, (double)(float)s.i0, (double)(float)s.r1,
                  (double)(float)s.i1};
    }
};

struct LaneGeo {
    int colw;   // column index used for memory (wrapped when periodic)
    bool inx;   // column exists (inside, or periodic image)
    bool own;   // lane writes and reduces its column
    double x;   // coordinate of colw
};

__device__ __forceinline__ LaneGeo lane_geo(const Op &op, const Tiles &t, int strip, int lane)
{
    LaneGeo g;
    const int col = strip * t.own - t.halo + lane;
    const bool inside = col >= 0 && col < op.nx;
    int colw = col;
    if (!inside) colw = op.bcx ? ((col % op.nx) + op.nx) % op.nx : 0;
    g.colw = colw;
    g.inx = inside || op.bcx;
    g.own = inside && lane >= t.halo && lane < 64 - t.halo;
    g.x = op.xmin + colw * op.hx;
    return g;
}

struct RowGeo {
    int jw;
    bool iny;
    double y;
};

__device__ __forceinline__ RowGeo row_geo(const Op &op, int r)
{
    RowGeo g;
    const bool inside = r >= 0 && r < op.ny;
    int jw = r;
    if (!inside) jw = op.bcy ? ((r % op.ny) + op.ny) % op.ny : 0;
    g.jw = jw;
    g.iny = inside || op.bcy;
    g.y = op.ymin + jw * op.hy;
    return g;
}

template <class T>
__device__ __forceinline__ Sp load_site(const T *b, const Op &op, const LaneGeo &lg, const RowGeo &rg)
{
    if (!(lg.inx && rg.iny)) return sp_zero();
    const size_t plane = (size_t)op.nx * op.ny;
    return Vec<T>::load(b, plane, (size_t)rg.jw * op.nx + lg.colw);
}

// Potential energy (times the operator scale) at a site.
__device__ __forceinline__ double site_pot(const Op &op, const LaneGeo &lg, const RowGeo &rg)
{
    double v = 0.0;
    if (op.pot_kind) v = -op.vz / sqrt(lg.x * lg.x + rg.y * rg.y + op.va2);
    if (op.has_table && lg.inx && rg.iny) v += op.vscale * op.vtab[(size_t)rg.jw * op.nx + lg.colw];
    return v;
}

// (A psi) at one site from the site value c, its x neighbours l, r and its y
// neighbours d (row below), u (row above):
//   (A psi)_0 = (mc2 + V) psi_0 + kx (-i)(psi_1[x+1] - psi_1[x-1])
//               - ky (psi_1[y+1] - psi_1[y-1]) + (gx - i gy) psi_1
//   (A psi)_1 = (V - mc2) psi_1 + kx (-i)(psi_0[x+1] - psi_0[x-1])
//               + ky (psi_0[y+1] - psi_0[y-1]) + (gx + i gy) psi_0
// i.e. c[sigma1 (p_x - qA_x) + sigma2 (p_y - qA_y)] + sigma3 m c^2 + V scaled
// by s, with gx = -s c q A_x and gy = -s c q A_y (Sec. 3 Hamiltonian).
__device__ __forceinline__ Sp hop(const Op &op, const Sp &c, const Sp &l, const Sp &r, const Sp &d,
                                  const Sp &u, double v, double gx, double gy)
{
    const double d0 = op.mc2 + v, d1 = v - op.mc2;
    const double x0r = r.r0 - l.r0, x0i = r.i0 - l.i0, x1r = r.r1 - l.r1, x1i = r.i1 - l.i1;
    const double y0r = u.r0 - d.r0, y0i = u.i0 - d.i0, y1r = u.r1 - d.r1, y1i = u.i1 - d.i1;
    Sp o;
    o.r0 = d0 * c.r0 + op.kx * x1i - op.ky * y1r + gx * c.r1 + gy * c.i1;
    o.i0 = d0 * c.i0 - op.kx * x1r - op.ky * y1i + gx * c.i1 - gy * c.r1;
    o.r1 = d1 * c.r1 + op.kx * x0i + op.ky * y0r + gx * c.r0 - gy * c.i0;
    o.i1 = d1 * c.i1 - op.kx * x0r + op.ky * y0i + gx * c.i0 + gy * c.r0;
    return o;
}

__device__ __forceinline__ double sp_norm2(const Sp &a)
{
    return a.r0 * a.r0 + a.i0 * a.i0 + a.r1 * a.r1 + a.i1 * a.i1;
}

// Re <a, b> at one site.
__device__ __forceinline__ double sp_redot(const Sp &a, const Sp &b)
{
    return a.r0 * b.r0 + a.i0 * b.i0 + a.r1 * b.r1 + a.i1 * b.i1;
}

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV])
{
    // Butterfly: after each stage partner lanes hold bitwise equal sums.
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], s, 64);
}

// Fold the per-lane sums of the whole grid in a fixed order.  Returns true in
// the last workgroup to finish, where every thread then holds the totals.
template <int NV>
__device__ bool grid_reduce(double (&v)[NV], double *partials, unsigned int *ticket, double (&tot)[NV])
{
    __shared__ double red[kWaves][NV];
    __shared__ int last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    wave_sum(v);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = red[0][k];
            for (int i = 1; i < kWaves; ++i) s += red[i][k];
            partials[(size_t)blockIdx.x * NV + k] = s;
        }
        __threadfence();
        const unsigned int t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += __builtin_nontemporal_load(&partials[(size_t)b * NV + k]);
    wave_sum(s);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[w][k] = s[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = red[0][k];
        for (int i = 1; i < kWaves; ++i) a += red[i][k];
        tot[k] = a;
    }
    if (threadIdx.x == 0) *ticket = 0u;
    return true;
}

struct WaveTask {
    bool active;
    int strip, y0, y1;
};

__device__ __forceinline__ WaveTask wave_task(const Op &op, const Tiles &t)
{
    WaveTask w;
    const int task = blockIdx.x * kWaves + (threadIdx.x >> 6);
    w.active = task < t.nstrips * t.nchunks;
    w.strip = task % t.nstrips;
    const int chunk = task / t.nstrips;
    w.y0 = chunk * t.rows;
    w.y1 = min(w.y0 + t.rows, op.ny);
    if (w.y0 >= op.ny) w.active = false;
    return w;
}

// ---------------------------------------------------------------------------
// Lanczos iteration 1: gamma_1 = ||psi||, alpha_1 = Re<psi, A psi>/||psi||^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_first(Op op, Tiles t, const double2 *__restrict__ psi,
                                                  const double *__restrict__ field, double *alpha,
                                                  double *gamma, Scalars *sc, double *partials, int m)
{
    if (sc->status != 0) return;
    const int lane = threadIdx.x & 63;
    const WaveTask wt = wave_task(op, t);
    const double gxh = field[0], gyh = field[1];
    double acc[2] = {0.0, 0.0};
    if (wt.active) {
        const LaneGeo lg = lane_geo(op, t, wt.strip, lane);
        const double gy = gyh - op.bq * lg.x;
        Sp p0 = sp_zero(), p1 = sp_zero();
        Sp p2 = load_site(psi, op, lg, row_geo(op, wt.y0 - 1));
        for (int R = wt.y0; R <= wt.y1; ++R) {
            p0 = p1;
            p1 = p2;
            p2 = load_site(psi, op, lg, row_geo(op, R));
            if (R - 1 < wt.y0) continue;  // rows y0-1 and y0 are still filling the ring
            const RowGeo rg = row_geo(op, R - 1);
            const Sp y = hop(op, p1, sp_left(p1), sp_right(p1), p0, p2, site_pot(op, lg, rg),
                             gxh + op.bq * rg.y, gy);
            if (lg.own) {
                acc[0] += sp_norm2(p1);
                acc[1] += sp_redot(p1, y);
            }
        }
    }
    double tot[2];
    if (!grid_reduce(acc, partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        const double n = tot[0], a = tot[1];
        if (!isfinite(n) || !isfinite(a)) {
            sc->status = 3;
            sc->kstop = -1;
            return;
        }
        if (n == 0.0) {
            gamma[1] = 0.0;
            alpha[1] = 0.0;
            sc->keff = 0;
            sc->kstop = 0;
            return;
        }
        gamma[1] = sqrt(n);
        alpha[1] = a / n;
        sc->scale = fabs(alpha[1]);
        sc->keff = m;
        sc->kstop = m;
    }
}

// ---------------------------------------------------------------------------
// Lanczos iteration p >= 2 (see the file comment).  T1, T2, TO: storage types
// of u_{p-1}, u_{p-2}, u_p.
// ---------------------------------------------------------------------------
template <class T1, class T2, class TO, bool HAS2>
__global__ __launch_bounds__(kBlock) void k_recur(PassArgs a)
{
    Scalars *sc = a.sc;
    const int p = a.pass;
    if (sc->kstop < p) return;
    const Op &op = a.op;
    const int lane = threadIdx.x & 63;
    const WaveTask wt = wave_task(op, a.t);
    const double g1 = a.gamma[p - 1];
    const double inv_g1 = 1.0 / g1;
    const double ca = a.alpha[p - 1] * inv_g1;
    const double cb = HAS2 ? g1 / a.gamma[p - 2] : 0.0;
    const double gxh = a.field[0], gyh = a.field[1];
    const T1 *__restrict__ u1 = static_cast<const T1 *>(a.u1);
    const T2 *__restrict__ u2 = static_cast<const T2 *>(a.u2);
    TO *__restrict__ uo = static_cast<TO *>(a.uo);
    const size_t plane = (size_t)op.nx * op.ny;
    double acc[3] = {0.0, 0.0, 0.0};
    if (wt.active) {
        const LaneGeo lg = lane_geo(op, a.t, wt.strip, lane);
        const double gy = gyh - op.bq * lg.x;
        // ring of u_{p-1}: rows R-2, R-1, R; ring of u_p: rows R-3, R-2, R-1
        Sp p0 = sp_zero(), p1 = sp_zero(), p2 = sp_zero();
        Sp q0 = sp_zero(), q1 = sp_zero(), q2 = sp_zero();
        double v_prev = 0.0, v_cur = 0.0;
        p2 = load_site(u1, op, lg, row_geo(op, wt.y0 - 2));
        for (int R = wt.y0 - 1; R <= wt.y1 + 1; ++R) {
            p0 = p1;
            p1 = p2;
            p2 = load_site(u1, op, lg, row_geo(op, R));
            q0 = q1;
            q1 = q2;
            v_prev = v_cur;
            // u_p at row R-1 (rows y0-1 .. y1)
            if (R >= wt.y0) {
                const RowGeo rg = row_geo(op, R - 1);
                v_cur = site_pot(op, lg, rg);
                const Sp w = hop(op, p1, sp_left(p1), sp_right(p1), p0, p2, v_cur,
                                 gxh + op.bq * rg.y, gy);
                Sp o = HAS2 ? load_site(u2, op, lg, rg) : sp_zero();
                Sp u;
                u.r0 = inv_g1 * w.r0 - ca * p1.r0 - cb * o.r0;
                u.i0 = inv_g1 * w.i0 - ca * p1.i0 - cb * o.i0;
                u.r1 = inv_g1 * w.r1 - ca * p1.r1 - cb * o.r1;
                u.i1 = inv_g1 * w.i1 - ca * p1.i1 - cb * o.i1;
                if (!(lg.inx && rg.iny)) u = sp_zero();
                u = Vec<TO>::round(u);
                q2 = u;
                if (lg.own && R - 1 >= wt.y0 && R - 1 < wt.y1)
                    Vec<TO>::store(uo, plane, (size_t)(R - 1) * op.nx + lg.colw, u);
            }
            // A u_p at row R-2 (rows y0 .. y1-1) and the three reductions
            if (R >= wt.y0 + 2) {
                const RowGeo rg = row_geo(op, R - 2);
                const Sp y = hop(op, q1, sp_left(q1), sp_right(q1), q0, q2, v_prev,
                                 gxh + op.bq * rg.y, gy);
                if (lg.own) {
                    acc[0] += sp_norm2(q1);
                    acc[1] += sp_redot(q1, y);
                    acc[2] += sp_redot(q1, p0);
                }
            }
        }
    }
    double tot[3];
    if (!grid_reduce(acc, a.partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        const double n = tot[0], an = tot[1], o = tot[2];
        if (!isfinite(n) || !isfinite(an) || !isfinite(o)) {
            sc->status = 3;
            sc->kstop = -1;
            return;
        }
        const double gp = sqrt(n);  // beta_{p-1}
        const double scale = fmax(sc->scale, fabs(a.alpha[p - 1]));
        a.gamma[p] = gp;
        if (gp <= 1e-13 * scale) {
            // invariant Krylov subspace: stop with k_eff = p - 1
            sc->keff = p - 1;
            sc->kstop = p - 1;
            return;
        }
        sc->scale = fmax(scale, gp);
        a.alpha[p] = an / n - o / g1;
    }
}

// ---------------------------------------------------------------------------
// exp(-iT) e_1 through the eigendecomposition of the k x k tridiagonal T
// (Sec. 4): implicit symmetric QR steps with Wilkinson shift, eigenvectors
// accumulated row-wise (lane j owns row j).  Every lane runs the same scalar
// bulge chase on its own private copy of the diagonals (lane-interleaved LDS
// columns), so no lane reads another lane's data until the final sum.
// Output: coef[j] = c_j / gamma_j with c = ||psi|| V exp(-i Lambda) V^T e_1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_tridiag(const double *alpha, const double *gamma, Scalars *sc)
{
    __shared__ double dpr[kMaxM * 64];
    __shared__ double epr[kMaxM * 64];
    __shared__ double zpr[kMaxM * 64];
    const int lane = threadIdx.x;
    if (sc->status != 0) return;
    const int k = sc->keff;
    if (k <= 0) {
        for (int j = lane; j < 2 * (kMaxM + 2); j += 64) sc->coef[j] = 0.0;
        if (lane == 0) sc->cabs_k = 0.0;
        return;
    }
#define DD(i) dpr[(i) * 64 + lane]
#define EE(i) epr[(i) * 64 + lane]
#define ZZ(i) zpr[(i) * 64 + lane]
    for (int i = 0; i < k; ++i) {
        DD(i) = alpha[i + 1];
        EE(i) = (i + 1 < k) ? gamma[i + 2] : 0.0;
        ZZ(i) = (i == lane) ? 1.0 : 0.0;
    }
    const double eps = 2.220446049250313e-16;
    int h = k - 1, iter = 0;
    while (h > 0) {
        if (fabs(EE(h - 1)) <= eps * (fabs(DD(h - 1)) + fabs(DD(h)))) {
            EE(h - 1) = 0.0;
            --h;
            iter = 0;
            continue;
        }
        if (++iter > 100) break;
        int l = h - 1;
        while (l > 0 && fabs(EE(l - 1)) > eps * (fabs(DD(l - 1)) + fabs(DD(l)))) --l;
        // Wilkinson shift from the trailing 2x2 block
        const double delta = 0.5 * (DD(h - 1) - DD(h));
        const double b2 = EE(h - 1) * EE(h - 1);
        const double mu = DD(h) - b2 / (delta + copysign(sqrt(delta * delta + b2), delta));
        double x = DD(l) - mu, z = EE(l);
        for (int q = l; q < h; ++q) {
            const double r = hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                const double ir = 1.0 / r;
                c = x * ir;
                s = -z * ir;
            }
            if (q > l) EE(q - 1) = r;
            const double aq = DD(q), aq1 = DD(q + 1), bq = EE(q);
            const double cc = c * c, ss = s * s, cs = c * s;
            DD(q) = cc * aq - 2.0 * cs * bq + ss * aq1;
            DD(q + 1) = ss * aq + 2.0 * cs * bq + cc * aq1;
            EE(q) = cs * (aq - aq1) + (cc - ss) * bq;
            if (q + 1 < h) {
                const double bq1 = EE(q + 1);
                x = EE(q);
                z = -s * bq1;
                EE(q + 1) = c * bq1;
            }
            const double zq = ZZ(q), zq1 = ZZ(q + 1);
            ZZ(q) = c * zq - s * zq1;
            ZZ(q + 1) = s * zq + c * zq1;
        }
    }
    __syncthreads();
    // c_j = gamma_1 sum_i Z[j][i] exp(-i lambda_i) Z[0][i]; row 0 belongs to lane 0
    const double g1 = gamma[1];
    if (lane < k) {
        double cr = 0.0, ci = 0.0;
        for (int i = 0; i < k; ++i) {
            double sn, cs;
            sincos(DD(i), &sn, &cs);
            const double w = zpr[i * 64 + 0] * ZZ(i);
            cr += w * cs;
            ci -= w * sn;
        }
        cr *= g1;
        ci *= g1;
        const double ig = 1.0 / gamma[lane + 1];
        sc->coef[2 * (lane + 1)] = cr * ig;
        sc->coef[2 * (lane + 1) + 1] = ci * ig;
        if (lane == k - 1) sc->cabs_k = sqrt(cr * cr + ci * ci);
    }
#undef DD
#undef EE
#undef ZZ
}

// ---------------------------------------------------------------------------
// Recombination psi_new = sum_j c_j q_j = sum_j (c_j / gamma_j) u_j
// (eq. matrix_exp_approx), plus u_{k+1} = (A u_k - alpha_k u_k)/gamma_k
// - (gamma_k/gamma_{k-1}) u_{k-1} for beta_k = ||u_{k+1}|| of the error
// estimate eq. matrix_exponential_error, and ||psi_new||^2.
// ---------------------------------------------------------------------------
template <class TB>
__device__ __forceinline__ Sp load_u(const RecArgs &a, const Op &op, const LaneGeo &lg,
                                     const RowGeo &rg, int j)
{
    if (j == 1) return load_site(a.psi, op, lg, rg);
    return load_site(static_cast<const TB *>(a.basis) + (size_t)(j - 2) * a.vec_elems, op, lg, rg);
}

template <class TB>
__global__ __launch_bounds__(kBlock) void k_recombine(RecArgs a)
{
    Scalars *sc = a.sc;
    if (sc->status != 0) return;
    const Op &op = a.op;
    const int k = sc->keff;
    const int lane = threadIdx.x & 63;
    const WaveTask wt = wave_task(op, a.t);
    const size_t plane = (size_t)op.nx * op.ny;
    const double gxh = a.field[0], gyh = a.field[1];
    double inv_gk = 0.0, ca = 0.0, cb = 0.0;
    if (k >= 1) {
        inv_gk = 1.0 / a.gamma[k];
        ca = a.alpha[k] * inv_gk;
        if (k >= 2) cb = a.gamma[k] / a.gamma[k - 1];
    }
    double acc[2] = {0.0, 0.0};
    if (wt.active) {
        const LaneGeo lg = lane_geo(op, a.t, wt.strip, lane);
        const double gy = gyh - op.bq * lg.x;
        Sp p0 = sp_zero(), p1 = sp_zero(), p2 = sp_zero();
        if (k >= 1) p2 = load_u<TB>(a, op, lg, row_geo(op, wt.y0 - 1), k);
        for (int R = wt.y0; R <= wt.y1; ++R) {
            const int rr = R - 1;
            p0 = p1;
            p1 = p2;
            if (k >= 1) p2 = load_u<TB>(a, op, lg, row_geo(op, R), k);
            if (rr < wt.y0) continue;
            const RowGeo rg = row_geo(op, rr);
            Sp s = sp_zero();
            if (k >= 1) {
                const Sp w = hop(op, p1, sp_left(p1), sp_right(p1), p0, p2, site_pot(op, lg, rg),
                                 gxh + op.bq * rg.y, gy);
                const Sp um = (k >= 2) ? load_u<TB>(a, op, lg, rg, k - 1) : sp_zero();
                Sp res;
                res.r0 = inv_gk * w.r0 - ca * p1.r0 - cb * um.r0;
                res.i0 = inv_gk * w.i0 - ca * p1.i0 - cb * um.i0;
                res.r1 = inv_gk * w.r1 - ca * p1.r1 - cb * um.r1;
                res.i1 = inv_gk * w.i1 - ca * p1.i1 - cb * um.i1;
                if (lg.own) acc[0] += sp_norm2(res);
                // sum over the basis, four loads in flight at a time
                for (int jb = 1; jb <= k; jb += 4) {
                    Sp v[4];
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) {
                        const int j = jb + t2;
                        if (j == k) v[t2] = p1;
                        else if (j == k - 1) v[t2] = um;
                        else if (j < k) v[t2] = load_u<TB>(a, op, lg, rg, j);
                        else v[t2] = sp_zero();
                    }
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) {
                        const int j = jb + t2;
                        if (j <= k) {
                            const double cr = sc->coef[2 * j], ci = sc->coef[2 * j + 1];
                            s.r0 += cr * v[t2].r0 - ci * v[t2].i0;
                            s.i0 += cr * v[t2].i0 + ci * v[t2].r0;
                            s.r1 += cr * v[t2].r1 - ci * v[t2].i1;
                            s.i1 += cr * v[t2].i1 + ci * v[t2].r1;
                        }
                    }
                }
            }
            if (lg.own) {
                Vec<double2>::store(a.out, plane, (size_t)rr * op.nx + lg.colw, s);
                acc[1] += sp_norm2(s);
            }
        }
    }
    double tot[2];
    if (!grid_reduce(acc, a.partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        const double beta_k = sqrt(tot[0]);
        a.stat->err_est = (k >= 1) ? beta_k * sc->cabs_k : 0.0;
        a.stat->norm2 = tot[1];
        a.stat->keff = k;
        if (!isfinite(tot[0]) || !isfinite(tot[1])) {
            sc->status = 3;
            sc->kstop = -1;
            return;
        }
        sc->steps_done += 1;
    }
}

// ---------------------------------------------------------------------------
// y = H x (test hook; operator scale 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_apply(Op op, Tiles t, const double2 *__restrict__ x,
                                                  double2 *__restrict__ y, double gxh, double gyh)
{
    const int lane = threadIdx.x & 63;
    const WaveTask wt = wave_task(op, t);
    if (!wt.active) return;
    const size_t plane = (size_t)op.nx * op.ny;
    const LaneGeo lg = lane_geo(op, t, wt.strip, lane);
    const double gy = gyh - op.bq * lg.x;
    Sp p0 = sp_zero(), p1 = sp_zero();
    Sp p2 = load_site(x, op, lg, row_geo(op, wt.y0 - 1));
    for (int R = wt.y0; R <= wt.y1; ++R) {
        p0 = p1;
        p1 = p2;
        p2 = load_site(x, op, lg, row_geo(op, R));
        if (R - 1 < wt.y0) continue;
        const RowGeo rg = row_geo(op, R - 1);
        const Sp o = hop(op, p1, sp_left(p1), sp_right(p1), p0, p2, site_pot(op, lg, rg),
                         gxh + op.bq * rg.y, gy);
        if (lg.own) Vec<double2>::store(y, plane, (size_t)(R - 1) * op.nx + lg.colw, o);
    }
}

__global__ void k_reset(Scalars *sc)
{
    if (threadIdx.x == 0) {
        sc->status = 0;
        sc->steps_done = 0;
        sc->ticket = 0u;
        sc->kstop = 0;
        sc->keff = 0;
        sc->scale = 0.0;
        sc->cabs_k = 0.0;
    }
}

}  // namespace

Tiles make_tiles(int nx, int ny, int halo, int target_waves)
{
    Tiles t;
    t.halo = halo;
    t.own = 64 - 2 * halo;
    t.nstrips = (nx + t.own - 1) / t.own;
    int nchunks = target_waves / t.nstrips;
    if (nchunks < 1) nchunks = 1;
    const int max_chunks = (ny + 3) / 4;  // at least four rows per chunk
    if (nchunks > max_chunks) nchunks = max_chunks;
    t.rows = (ny + nchunks - 1) / nchunks;
    for (;;) {
        t.nchunks = (ny + t.rows - 1) / t.rows;
        t.nblocks = (t.nstrips * t.nchunks + kWaves - 1) / kWaves;
        if (t.nblocks <= kMaxBlocks) break;
        t.rows *= 2;
    }
    return t;
}

void launch_first(const Op &op, const Tiles &t, const double2 *psi, const double *field,
                  double *alpha, double *gamma, Scalars *sc, double *partials, int m, hipStream_t st)
{
    hipLaunchKernelGGL(k_first, dim3(t.nblocks), dim3(kBlock), 0, st, op, t, psi, field, alpha,
                       gamma, sc, partials, m);
}

void launch_recur(const PassArgs &a, bool mixed, hipStream_t st)
{
    const dim3 g(a.t.nblocks), b(kBlock);
    if (!mixed) {
        if (a.pass == 2)
            hipLaunchKernelGGL((k_recur<double2, double2, double2, false>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((k_recur<double2, double2, double2, true>), g, b, 0, st, a);
    } else {
        if (a.pass == 2)
            hipLaunchKernelGGL((k_recur<double2, double2, float2, false>), g, b, 0, st, a);
        else if (a.pass == 3)
            hipLaunchKernelGGL((k_recur<float2, double2, float2, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((k_recur<float2, float2, float2, true>), g, b, 0, st, a);
    }
}

void launch_tridiag(const double *alpha, const double *gamma, Scalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(64), 0, st, alpha, gamma, sc);
}

void launch_recombine(const RecArgs &a, bool mixed, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL(k_recombine<float2>, dim3(a.t.nblocks), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_recombine<double2>, dim3(a.t.nblocks), dim3(kBlock), 0, st, a);
}

void launch_apply(const Op &op, const Tiles &t, const double2 *x, double2 *y, double gxh,
                  double gyh, hipStream_t st)
{
    hipLaunchKernelGGL(k_apply, dim3(t.nblocks), dim3(kBlock), 0, st, op, t, x, y, gxh, gyh);
}

void launch_reset(Scalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, sc);
}

}  // namespace dl
