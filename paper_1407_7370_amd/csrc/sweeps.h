// gfx950 kernels of the Lanczos short-time propagator for the 2D Dirac
// equation (Beerwerth & Bauke, arXiv:1407.7370).
//
// Stencil sweeps.  One wave64 owns a strip of columns and a chunk of rows and
// marches down the rows: lane l holds column strip*own - halo + l, neighbours
// in x come from the adjacent lanes through DPP wave rotations, neighbours in
// y from a register ring of the last rows, and the rows ahead sit in a
// register FIFO of loads in flight.  The march is unrolled by four so that
// every ring and FIFO slot is a fixed register (no moves).  Row addresses are
// scalar (one base per row) plus a fixed 32-bit lane offset.  No LDS tile and
// no barrier is needed inside the march; the `halo` edge lanes of a wave only
// feed their neighbours.  Reductions are per-lane FP64 sums folded by a fixed
// butterfly, per workgroup, and finally by the last workgroup to finish in
// fixed order, so results are bitwise reproducible.
//
// A sweep p >= 2 fuses one whole Lanczos iteration of Fig. 1 (Sec. 2) into one
// pass over memory: with u_i = gamma_i q_i (gamma_i = ||u_i|| = beta_{i-1})
//   u_p = (A u_{p-1} - alpha_{p-1} u_{p-1}) / gamma_{p-1}
//         - (gamma_{p-1} / gamma_{p-2}) u_{p-2}                  (eq. lanczos_base)
// is formed on the tile plus a one-site rim (A u_{p-1} is recomputed there
// from u_{p-1} with a two-site rim), stored, and A u_p is applied on the tile
// to reduce ||u_p||^2, Re<u_p, A u_p> and Re<u_p, u_{p-1}>.  From these the
// last workgroup forms gamma_p and alpha_p = Re<q_p, A q_p> - beta_{p-1}
// Re<q_p, q_{p-1}>, the modified Gram-Schmidt form of Fig. 1.  The last sweep
// also reduces ||A u_m||^2 and Re<A u_m, u_{m-1}>, from which beta_m (input of
// the error estimate eq. matrix_exponential_error) follows without another
// pass over memory.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

#include "dl_internal.h"
#include "device_reduce.h"

// Device code of the sweeps, shared by the single-grid launches (kernels.hip)
// and the batched launches (batch_kernels.hip).  Internal header; everything
// is in an anonymous namespace (each translation unit instantiates what it
// launches).
namespace dl {
namespace {

template <int K>
using IC = std::integral_constant<int, K>;

// f(IC<0>{}), ..., f(IC<N-1>{}) in order (compile-time unrolled steps).
template <class F, int... K>
__device__ __forceinline__ void unroll_steps(F &&f, std::integer_sequence<int, K...>)
{
    (f(IC<K>{}), ...);
}

struct Sp {
    double r0, i0, r1, i1;  // component 0 (re, im), component 1 (re, im)
};

__device__ __forceinline__ Sp sp_zero() { return Sp{0.0, 0.0, 0.0, 0.0}; }

// DPP wave rotations: wave_ror:1 delivers the value of lane l-1 to lane l,
// wave_rol:1 the value of lane l+1.  Lanes 0 and 63 receive wrapped values
// that only feed rim lanes whose results are discarded.
__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x13C, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x13C, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xF, 0xF, true);
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

// One site of a stored vector: both components in the storage type (aligned
// so that a paired site is one 16-byte access in complex64).
template <class T>
struct alignas(2 * sizeof(T)) Raw {
    T a, b;
};

template <class T>
__device__ __forceinline__ T tzero();
template <>
__device__ __forceinline__ double2 tzero<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ float2 tzero<float2>() { return make_float2(0.0f, 0.0f); }

template <class T>
__device__ __forceinline__ Raw<T> raw_zero() { return Raw<T>{tzero<T>(), tzero<T>()}; }

template <class T>
__device__ __forceinline__ Sp to_sp(const Raw<T> &r)
{
    return Sp{(double)r.a.x, (double)r.a.y, (double)r.b.x, (double)r.b.y};
}

// A FIFO slot's row, taken out of the registers the next load will refill.
// complex64 rows are widened anyway; complex128 rows get a real operation
// (x + 0.0, which the compiler may not drop), so the refill can reuse the
// slot's registers instead of leaving copies of in-flight loads at the loop's
// back edge, which would wait for them.
template <class T>
__device__ __forceinline__ Sp fifo_take(const Raw<T> &r)
{
    if constexpr (sizeof(r.a.x) == 8)
        return Sp{r.a.x + 0.0, r.a.y + 0.0, r.b.x + 0.0, r.b.y + 0.0};
    else
        return to_sp(r);
}

// The value that a later sweep reads back from storage of type T.
template <class T>
__device__ __forceinline__ Sp stored_value(const Sp &s);
template <>
__device__ __forceinline__ Sp stored_value<double2>(const Sp &s) { return s; }
template <>
__device__ __forceinline__ Sp stored_value<float2>(const Sp &s)
{
    return Sp{(double)(float)s.r0, (double)(float)s.i0, (double)(float)s.r1, (double)(float)s.i1};
}

template <class T>
__device__ __forceinline__ Raw<T> to_raw(const Sp &s);
template <>
__device__ __forceinline__ Raw<double2> to_raw<double2>(const Sp &s)
{
    return Raw<double2>{make_double2(s.r0, s.i0), make_double2(s.r1, s.i1)};
}
template <>
__device__ __forceinline__ Raw<float2> to_raw<float2>(const Sp &s)
{
    return Raw<float2>{make_float2((float)s.r0, (float)s.i0), make_float2((float)s.r1, (float)s.i1)};
}

// Buffer access.  Every row of a vector gets its own buffer descriptor
// (scalar registers) whose size is the row length, or zero for a row outside a
// Dirichlet domain; lanes outside the domain use an offset past any row.  The
// hardware returns zero for such loads and drops such stores, so the domain
// boundary costs no branches and no register fills.
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr uint32_t kOob = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer format (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const char *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, (int)bytes, kRsrcWord3);
}

// Rows between scheduling barriers of the recurrence sweep.
#ifndef DL_SCHED_ROWS
#define DL_SCHED_ROWS 1
#endif

// Cache-policy operand of buffer loads and stores: 0 default, 2 the
// nontemporal (streaming) hint, 16 the device-coherent store (sc1: written
// through this XCD's L2 to the coherence point).
constexpr int kPolDefault = 0;
constexpr int kPolStream = 2;
constexpr int kPolCoherent = 16;
// Stores of the Krylov vectors.  Complex64 rows (one 16-byte store per lane,
// whole lines) are written through, so that the kernel's end does not wait
// for the XCD's L2 to write them back (4096^2 sweep 139.6 -> 138.3 us, 1024^2
// mixed step 410 -> 387 us); complex128 rows (two 16-byte halves per lane in
// separate stores) keep the default (written through: 4096^2 324 -> 494 us).
#ifndef DL_SWEEP_STORE_POLICY
#define DL_SWEEP_STORE_POLICY kPolDefault
#endif
#ifndef DL_SWEEP_STORE_POLICY_C64
#define DL_SWEEP_STORE_POLICY_C64 kPolCoherent
#endif

template <class X, int POL = kPolDefault>
__device__ __forceinline__ X ld16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(X) == 16, "16-byte access");
    return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, POL));
}

template <class X, int POL = DL_SWEEP_STORE_POLICY>
__device__ __forceinline__ void st16(__amdgpu_buffer_rsrc_t r, uint32_t off, const X &v)
{
    static_assert(sizeof(X) == 16, "16-byte access");
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), r, off, 0, POL);
}

// Vector views.  Planar: the caller's state layout (two component planes of
// complex128).  Paired: Krylov vectors, both components of a site adjacent.
template <int POL>
struct PlanarT {
    using T = double2;
    const char *base;
    size_t plane_bytes;
    uint32_t row_bytes;  // nx * 16
    __device__ __forceinline__ Raw<double2> load(int jw, bool row_ok, uint32_t off) const
    {
        const char *r = base + (size_t)jw * row_bytes;
        const uint32_t n = row_ok ? row_bytes : 0u;
        Raw<double2> v;
        v.a = ld16<double2, POL>(row_rsrc(r, n), off);
        v.b = ld16<double2, POL>(row_rsrc(r + plane_bytes, n), off);
        return v;
    }
    // Row at address `row` (first plane) with `n` valid bytes (0: returns zeros).
    __device__ __forceinline__ Raw<double2> load_at(const char *row, uint32_t n, uint32_t off) const
    {
        Raw<double2> v;
        v.a = ld16<double2, POL>(row_rsrc(row, n), off);
        v.b = ld16<double2, POL>(row_rsrc(row + plane_bytes, n), off);
        return v;
    }
    static __device__ __forceinline__ uint32_t lane_offset(int colw) { return (uint32_t)colw * 16u; }
};
using Planar = PlanarT<kPolDefault>;
template <class V>
struct is_planar : std::false_type {};
template <int POL>
struct is_planar<PlanarT<POL>> : std::true_type {};

template <class TT, int POL = kPolDefault>
struct Paired {
    using T = TT;
    const char *base;
    uint32_t row_bytes;  // nx * 2 * sizeof(T)
    __device__ __forceinline__ Raw<T> load(int jw, bool row_ok, uint32_t off) const
    {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(base + (size_t)jw * row_bytes, row_ok ? row_bytes : 0u);
        if constexpr (sizeof(T) == 8) {
            return ld16<Raw<T>, POL>(r, off);
        } else {
            Raw<T> v;
            v.a = ld16<T, POL>(r, off);
            v.b = ld16<T, POL>(r, off + 16u);
            return v;
        }
    }
    __device__ __forceinline__ Raw<T> load_at(const char *row, uint32_t n, uint32_t off) const
    {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(row, n);
        if constexpr (sizeof(T) == 8) {
            return ld16<Raw<T>, POL>(r, off);
        } else {
            Raw<T> v;
            v.a = ld16<T, POL>(r, off);
            v.b = ld16<T, POL>(r, off + 16u);
            return v;
        }
    }
    // Store to the row at `row` with `n` valid bytes (0: the store is dropped).
    __device__ __forceinline__ void store_at(const char *row, uint32_t n, uint32_t off, const Raw<T> &v) const
    {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(row, n);
        if constexpr (sizeof(T) == 8) {
            st16<Raw<T>, DL_SWEEP_STORE_POLICY_C64>(r, off, v);
        } else {
            st16(r, off, v.a);
            st16(r, off + 16u, v.b);
        }
    }
    __device__ __forceinline__ void store(int jw, uint32_t off, const Raw<T> &v) const
    {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(base + (size_t)jw * row_bytes, row_bytes);
        if constexpr (sizeof(T) == 8) {
            st16<Raw<T>, DL_SWEEP_STORE_POLICY_C64>(r, off, v);
        } else {
            st16(r, off, v.a);
            st16(r, off + 16u, v.b);
        }
    }
    static __device__ __forceinline__ uint32_t lane_offset(int colw)
    {
        return (uint32_t)colw * (uint32_t)(2 * sizeof(T));
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
    // sweeps touch rows -2 .. ny+1 only (rim of two rows, ny >= 3): one wrap suffices
    const bool inside = r >= 0 && r < op.ny;
    int jw = r < 0 ? r + op.ny : (r >= op.ny ? r - op.ny : r);
    if (!inside && !op.bcy) jw = 0;
    g.jw = jw;
    g.iny = inside || op.bcy;
    g.y = op.ymin + jw * op.hy;
    return g;
}

// Load one site of row r (zero outside a Dirichlet domain; `off` is the lane
// offset, or kOob for a lane outside the domain).  A row that is not `needed`
// gets an empty descriptor: the load returns zeros without touching memory,
// so FIFO refills can be unconditional.
template <class V>
__device__ __forceinline__ Raw<typename V::T> load_row(const V &v, const Op &op, uint32_t off, int r,
                                                       bool needed = true)
{
    const RowGeo rg = row_geo(op, r);
    return v.load(rg.jw, rg.iny && needed, off);
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
// by s, with gx = -s c q A_x and gy = -s c q A_y (Sec. 3 Hamiltonian); the
// optional shift returns (A - shift I) psi.
__device__ __forceinline__ Sp hop(const Op &op, const Sp &c, const Sp &l, const Sp &r, const Sp &d,
                                  const Sp &u, double v, double gx, double gy, double shift = 0.0)
{
    const double d0 = op.mc2 + v - shift, d1 = v - op.mc2 - shift;
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

// Tile of this wave.  The wave index is made wave-uniform explicitly so that
// the whole march (row indices, bounds, addresses) runs on the scalar unit.
struct WaveTask {
    bool active;
    int strip, y0, y1;
};

// Workgroups are dispatched to the eight XCDs of the chip round robin
// (workgroup b to XCD b mod 8), and each XCD has its own L2.  With the XCD
// map on, consecutive logical workgroups -- adjacent strips of one row chunk,
// which share their halo columns -- run on the same XCD.
#ifndef DL_XCD_MAP
#define DL_XCD_MAP 1
#endif
constexpr int kXcds = 8;

__device__ __forceinline__ int logical_block()
{
    const int b = (int)blockIdx.x;
    if (!DL_XCD_MAP) return b;
    const int nb = (int)gridDim.x, q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
    const int first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return first + b / kXcds;
}

__device__ __forceinline__ WaveTask wave_task(const Op &op, const Tiles &t)
{
    WaveTask w;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int task = logical_block() * kWaves + wave;
    w.active = task < t.nstrips * t.nchunks;
    w.strip = task % t.nstrips;
    const int chunk = task / t.nstrips;
    w.y0 = chunk * t.rows;
    w.y1 = min(w.y0 + t.rows, op.ny);
    if (w.y0 >= op.ny) w.active = false;
    return w;
}

// Scalar cursor over the rows of one vector: the (unwrapped) address of row r,
// advanced by one row per step.  Rows outside a Dirichlet domain or outside
// the needed range get a zero-size descriptor: loads return zeros and stores
// are dropped, with no branch.
template <bool PY>
struct RowCursor {
    uint64_t addr;  // base + r * rb
    int r;
    uint32_t rb;    // bytes per row
    uint64_t span;  // ny * rb (periodic wrap)
    int lo;         // first valid row
    uint32_t width; // number of valid rows: lo .. lo + width - 1
    __device__ __forceinline__ const char *ptr(int ny) const
    {
        uint64_t x = addr;
        if constexpr (PY) x = r < 0 ? x + span : (r >= ny ? x - span : x);
        return reinterpret_cast<const char *>(x);
    }
    __device__ __forceinline__ uint32_t bytes() const { return (uint32_t)(r - lo) < width ? rb : 0u; }
    __device__ __forceinline__ void next()
    {
        addr += rb;
        ++r;
    }
};

// Cursor at row r whose valid rows are lo .. hi intersected with the domain
// (Dirichlet) -- every row of the rim is a valid periodic image.
template <bool PY>
__device__ __forceinline__ RowCursor<PY> row_cursor(const void *base, uint32_t rb, int ny, int r, int lo, int hi)
{
    RowCursor<PY> c;
    c.addr = reinterpret_cast<uint64_t>(base) + (uint64_t)((int64_t)r * (int64_t)rb);
    c.r = r;
    c.rb = rb;
    c.span = (uint64_t)ny * rb;
    if (!PY) {
        lo = max(lo, 0);
        hi = min(hi, ny - 1);
    }
    c.lo = lo;
    c.width = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
    return c;
}

// Potential energy (times the operator scale) at column lg, wrapped row jw.
__device__ __forceinline__ double site_pot_row(const Op &op, const LaneGeo &lg, int jw, double y)
{
    double v = 0.0;
    if (op.pot_kind) v = -op.vz / sqrt(lg.x * lg.x + y * y + op.va2);
    if (op.has_table && lg.inx) v += op.vscale * op.vtab[(size_t)jw * op.nx + lg.colw];
    return v;
}

template <class V>
__device__ __forceinline__ V make_view(const void *p, const Op &op)
{
    if constexpr (is_planar<V>::value)
        return V{static_cast<const char *>(p), (size_t)op.nx * op.ny * 16, (uint32_t)op.nx * 16u};
    else
        return V{static_cast<const char *>(p), (uint32_t)(op.nx * 2 * sizeof(typename V::T))};
}

// Load policy of the first iteration's reads of psi.
#ifndef DL_LOAD_POL_FIRST
#define DL_LOAD_POL_FIRST kPolStream
#endif
using PlanarF = PlanarT<DL_LOAD_POL_FIRST>;

// ---------------------------------------------------------------------------
// Lanczos iteration 1: gamma_1 = ||psi||, alpha_1 = Re<psi, A psi>/||psi||^2,
// and for m = 1 also beta_1 = ||A q_1 - alpha_1 q_1||.
// Rows marched: psi rows y0-1 .. y1 (ring slot = row - (y0-1) mod 4).
// ---------------------------------------------------------------------------
// March of one wave of iteration 1 over its tile (acc: ||psi||^2, Re<psi, A psi>,
// ||A psi||^2 of its owned sites).
template <int PF, bool PY, int TERMS>
__device__ __forceinline__ void first_body(const Op &op, const Tiles &t, const WaveTask &wt,
                                           const double2 *__restrict__ psi, const double *__restrict__ field,
                                           double (&acc)[3])
{
    constexpr int U = PF > 4 ? PF : 4;
    static_assert(U % PF == 0 && U % 4 == 0, "FIFO depth must divide the unroll");
    const int lane = threadIdx.x & 63;
    const int ny = op.ny;
    const double gxh = field[0], gyh = field[1];
    if (wt.active) {
        const LaneGeo lg = lane_geo(op, t, wt.strip, lane);
        const double gy = (TERMS & kTermB) ? gyh - op.bqy * lg.x : gyh;
        const PlanarF vin = make_view<PlanarF>(psi, op);
        const uint32_t off = lg.inx ? PlanarF::lane_offset(lg.colw) : kOob;
        const int y0 = wt.y0, y1 = wt.y1, base = y0 - 1;
        RowCursor<PY> cin = row_cursor<PY>(psi, vin.row_bytes, ny, base, base, y1);
        // empty FIFO, march from PF rows early: every load comes from the loop
        // (see recur_body)
        Raw<double2> F[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) F[i] = raw_zero<double2>();
        Sp P[4] = {sp_zero(), sp_zero(), sp_zero(), sp_zero()};
        const double mo = lg.own ? 1.0 : 0.0;
        int R0 = base - PF;
        auto step = [&](auto kc) {
            constexpr int k = decltype(kc)::value & 3;
            constexpr int f = decltype(kc)::value % PF;
            const int R = R0 + decltype(kc)::value;
            __builtin_amdgcn_sched_barrier(0);
            P[k] = fifo_take(F[f]);
            F[f] = vin.load_at(cin.ptr(ny), cin.bytes(), off);
            cin.next();
            // A psi at row R-1, reduced over the owned rows y0 .. y1-1
            const Sp &c = P[(k + 3) & 3];
            double v = 0.0, gx = gxh;
            if constexpr (TERMS != 0) {
                const int jr = min(max(R - 1, 0), ny - 1);
                const double y = op.ymin + jr * op.hy;
                if constexpr (TERMS & kTermPot) v = site_pot_row(op, lg, jr, y);
                if constexpr (TERMS & kTermB) gx = gxh + op.bq * y;
            }
            const Sp y = hop(op, c, sp_left(c), sp_right(c), P[(k + 2) & 3], P[k], v, gx, gy);
            const double m = (unsigned)(R - 1 - y0) < (unsigned)(y1 - y0) ? mo : 0.0;
            acc[0] += m * sp_norm2(c);
            acc[1] += m * sp_redot(c, y);
            acc[2] += m * sp_norm2(y);
        };
        for (; R0 <= y1; R0 += U) unroll_steps(step, std::make_integer_sequence<int, U>{});
    }
}

// Scalar update of iteration 1 from the grid totals (one thread).
__device__ __forceinline__ void first_tail(const double (&tot)[3], double *alpha, double *gamma, Scalars *sc,
                                           int m, int shift)
{
    const double n = tot[0], a = tot[1], yy = tot[2];
    if (!isfinite(n) || !isfinite(a) || !isfinite(yy)) {
        sc->status = 3;
        sc->kstop = -1;
        return;
    }
    if (n == 0.0) {
        gamma[1] = 0.0;
        alpha[1] = 0.0;
        sc->sigma = 0.0;
        sc->keff = 0;
        sc->kstop = 0;
        sc->beta_k = 0.0;
        return;
    }
    const double g = sqrt(n);
    const double al = a / n;
    gamma[1] = g;
    // With the shift on, the later sweeps run on A' = A - alpha_1 I: the same
    // Krylov space, T' = T - alpha_1 I, so alpha'_1 = 0 and the residuals
    // A' u - alpha' u no longer cancel by |alpha| / beta.
    sc->sigma = shift ? al : 0.0;
    alpha[1] = shift ? 0.0 : al;
    sc->scale = fabs(al);
    // fixed dimension m, or the dimension predicted by the previous step
    const int kk = (sc->knext > 0 && sc->knext < m) ? sc->knext : m;
    sc->keff = kk;
    sc->kstop = kk;
    // ||A psi - alpha_1 psi||^2 = ||A psi||^2 - a^2/n
    sc->beta_k = sqrt(fmax(yy - a * (a / n), 0.0)) / g;
}

template <int PF, bool PY, int TERMS>
__global__ __launch_bounds__(kBlock) void k_first(Op op, Tiles t, const double2 *__restrict__ psi,
                                                  const double *__restrict__ field, double *alpha,
                                                  double *gamma, Scalars *sc, double *partials, int m,
                                                  int shift)
{
    if (sc->status != 0) return;
    const WaveTask wt = wave_task(op, t);
    double acc[3] = {0.0, 0.0, 0.0};
    first_body<PF, PY, TERMS>(op, t, wt, psi, field, acc);
    double tot[3];
    if (!grid_reduce(acc, partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) first_tail(tot, alpha, gamma, sc, m, shift);
}

// ---------------------------------------------------------------------------
// Lanczos iteration p >= 2 (see the file comment).  V1, V2: views of u_{p-1},
// u_{p-2}; TO: storage type of u_p (paired layout); PF: FIFO depth in rows;
// PY: periodic in y; TERMS: site-dependent terms present (kTermPot: potential
// or potential table, the diagonal varies; kTermB: magnetic field, the
// coupling varies); absent terms are uniform and computed once.
// Rows marched: R = y0-2 .. y1+1 (u_{p-1} row R enters, u_p row R-1 is formed,
// A u_p row R-2 is applied); ring slot of row r = (r - (y0-2)) mod 4.
// ---------------------------------------------------------------------------

// March of one wave of iteration p >= 2 over its tile (acc: ||u_p||^2,
// Re<u_p, A u_p>, Re<u_p, u_(p-1)> and, in the last iteration, ||A u_p||^2 and
// Re<A u_p, u_(p-1)> of its owned sites).
template <class V1, class V2, class TO, bool HAS2, int PF, bool PY, int TERMS>
__device__ __forceinline__ void recur_body(const PassArgs &a, const WaveTask &wt, double g1, double alpha_pm1,
                                           double (&acc)[5])
{
    // rows are marched U at a time so that every ring and FIFO slot index is a
    // compile-time constant; the rings hold four rows (slot = row mod 4)
    constexpr int U = PF > 4 ? PF : 4;
    static_assert(U % PF == 0 && U % 4 == 0, "FIFO depth must divide the unroll");
    using T1 = typename V1::T;
    using T2 = typename V2::T;
    const Scalars *sc = a.sc;
    const int p = a.pass;
    const Op &op = a.op;
    const int ny = op.ny;
    const int lane = threadIdx.x & 63;
    const double inv_g1 = 1.0 / g1;
    const double ca = alpha_pm1 * inv_g1;
    const double cb = HAS2 ? g1 / a.gamma[p - 2] : 0.0;
    const double sig = sc->sigma;
    const double gxh = a.field[0], gyh = a.field[1];
    if (wt.active) {
        const LaneGeo lg = lane_geo(op, a.t, wt.strip, lane);
        const double gy = (TERMS & kTermB) ? gyh - op.bqy * lg.x : gyh;
        // u_p = cw (A' u_{p-1}) - cc u_{p-1} - cu u_{p-2}; lanes outside the domain
        // get zero coefficients, so their u_p is zero without a select
        const double m = lg.inx ? 1.0 : 0.0;
        const double cw = m * inv_g1, cc = m * ca, cu = m * cb;
        const V1 v1 = make_view<V1>(a.u1, op);
        const V2 v2 = make_view<V2>(a.u2, op);
        const Paired<TO> vo{static_cast<const char *>(a.uo), (uint32_t)(op.nx * 2 * sizeof(TO))};
        const uint32_t off1 = lg.inx ? V1::lane_offset(lg.colw) : kOob;
        const uint32_t off2 = lg.inx ? V2::lane_offset(lg.colw) : kOob;
        const uint32_t offo = lg.own ? Paired<TO>::lane_offset(lg.colw) : kOob;
        const int y0 = wt.y0, y1 = wt.y1, base = y0 - 2;
        // cursors: u_{p-1} rows from base, u_{p-2} rows from base-1, u_p rows from base-1
        RowCursor<PY> c1 = row_cursor<PY>(a.u1, v1.row_bytes, ny, base, base, y1 + 1);
        RowCursor<PY> c2 = row_cursor<PY>(a.u2, v2.row_bytes, ny, base - 1, y0 - 1, y1);
        // the march starts PF rows early with empty FIFOs, so that the first
        // loads are issued by the same loop code as every later refill
        RowCursor<PY> co = row_cursor<PY>(a.uo, vo.row_bytes, ny, base - PF - 1, y0, y1 - 1);
        // FIFOs: u_{p-1} row r in slot (r-base) mod PF, needed rows y0-2 .. y1+1;
        //        u_{p-2} row r-1 in the same slot, needed rows y0-1 .. y1.
        Raw<T1> F1[PF];
        Raw<T2> F2[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            F1[i] = raw_zero<T1>();
            F2[i] = raw_zero<T2>();
        }
        Sp P[4] = {sp_zero(), sp_zero(), sp_zero(), sp_zero()};  // u_{p-1} rows
        Sp Q[4] = {sp_zero(), sp_zero(), sp_zero(), sp_zero()};  // u_p rows
        double Vr[4] = {0.0, 0.0, 0.0, 0.0};                      // potential of the rows (kTermPot)
        const double mo = lg.own ? 1.0 : 0.0;                     // lanes whose sites this wave owns
        int R0 = base - PF;
        // One row R of the march, with no branch: rows the wave does not
        // produce are masked instead.  u_p is formed at row R-1 for every R
        // (the cursor of u_p drops the stores outside rows y0 .. y1-1, a
        // Dirichlet row outside the domain gets zero coefficients) and A u_p
        // at row R-3 enters the reductions only for rows y0 .. y1-1.  The loop
        // blocks are then identical, so the compiler waits for one row of
        // loads at a time while PF rows are in flight; a branch per row makes
        // it wait for all of them.  Rows past y1+1 load nothing (zero-size
        // descriptors) and are discarded.
        auto step = [&](auto kc) {
            constexpr int kk = decltype(kc)::value;
            constexpr int k = kk & 3;   // ring slot of row R
            constexpr int f = kk % PF;  // FIFO slot of row R
            const int R = R0 + kk;
            // keep each group of rows' work in its place: hoisted FIFO reads
            // would make the loop head wait for the rows still in flight
            if constexpr (kk % DL_SCHED_ROWS == 0) __builtin_amdgcn_sched_barrier(0);
            P[k] = fifo_take(F1[f]);
            const Sp o2 = fifo_take(F2[f]);
            // refill: u_{p-1} row R+PF, u_{p-2} row R+PF-1
            F1[f] = v1.load_at(c1.ptr(ny), c1.bytes(), off1);
            c1.next();
            if (HAS2) {
                F2[f] = v2.load_at(c2.ptr(ny), c2.bytes(), off2);
                c2.next();
            }
            // u_p at row R-1, zero outside a Dirichlet domain
            {
                const int rr = R - 1;
                const double mr = (PY || (unsigned)rr < (unsigned)ny) ? 1.0 : 0.0;
                const Sp &c = P[(k + 3) & 3];
                double v = 0.0, gx = gxh;
                if constexpr (TERMS != 0) {
                    // periodic image of the row; rows masked out clamp into the grid
                    const int jw = min(max(rr < 0 ? rr + ny : (rr >= ny ? rr - ny : rr), 0), ny - 1);
                    const double y = op.ymin + jw * op.hy;
                    if constexpr (TERMS & kTermPot) {
                        v = site_pot_row(op, lg, jw, y);
                        Vr[(k + 3) & 3] = v;
                    }
                    if constexpr (TERMS & kTermB) gx = gxh + op.bq * y;
                }
                const Sp w = hop(op, c, sp_left(c), sp_right(c), P[(k + 2) & 3], P[k], v, gx, gy, sig);
                const double cwr = mr * cw, ccr = mr * cc, cur = mr * cu;
                Sp u;
                u.r0 = cwr * w.r0 - ccr * c.r0 - cur * o2.r0;
                u.i0 = cwr * w.i0 - ccr * c.i0 - cur * o2.i0;
                u.r1 = cwr * w.r1 - ccr * c.r1 - cur * o2.r1;
                u.i1 = cwr * w.i1 - ccr * c.i1 - cur * o2.i1;
                const Raw<TO> ur = to_raw<TO>(u);
                Q[(k + 3) & 3] = to_sp(ur);
                vo.store_at(co.ptr(ny), co.bytes(), offo, ur);
            }
            co.next();
            // A u_p at row R-3 and the reductions over rows y0 .. y1-1 (the
            // last pass's two extra ones are formed every pass and reduced
            // only in the last).  Row R-3 rather than R-2: its neighbours
            // R-4 and R-2 were formed in earlier rows, so this product does
            // not wait for the u_p formed just above and the two run side by
            // side.
            {
                const Sp &c = Q[(k + 1) & 3];
                double v = 0.0, gx = gxh;
                if constexpr (TERMS & kTermPot) v = Vr[(k + 1) & 3];
                if constexpr (TERMS & kTermB) gx = gxh + op.bq * (op.ymin + (R - 3) * op.hy);
                const Sp y = hop(op, c, sp_left(c), sp_right(c), Q[k], Q[(k + 2) & 3], v, gx, gy, sig);
                const Sp &prev = P[(k + 1) & 3];  // u_{p-1} row R-3
                const double m = (unsigned)(R - 3 - y0) < (unsigned)(y1 - y0) ? mo : 0.0;
                acc[0] += m * sp_norm2(c);
                acc[1] += m * sp_redot(c, y);
                acc[2] += m * sp_redot(c, prev);
                acc[3] += m * sp_norm2(y);
                acc[4] += m * sp_redot(y, prev);
            }
        };
        for (; R0 <= y1 + 2; R0 += U) unroll_steps(step, std::make_integer_sequence<int, U>{});
    }
}

// Scalar update of iteration p from the grid totals: evaluated from the
// scalars of the iterations before p (the same in every thread that calls
// it), then stored by one thread.
struct RecurTail {
    bool fail;       // a non-finite total: the call is aborted
    bool breakdown;  // invariant Krylov subspace: k_eff = p - 1
    bool last;       // p is the last iteration of the step
    double gp;       // gamma_p = beta_{p-1}
    double al;       // alpha_p
    double scale;    // running scale of the breakdown test
    double beta_k;   // beta_k of the step (last iteration or breakdown)
};

// What the scalar update of iteration p reads besides the sums.
struct TailIn {
    int kstop;
    double g1, sig, scale, alpha_pm1;
};
__device__ __forceinline__ TailIn tail_inputs(const Scalars *sc, const double *alpha, const double *gamma, int p)
{
    return TailIn{sc->kstop, gamma[p - 1], sc->sigma, sc->scale, alpha[p - 1]};
}

__device__ __forceinline__ RecurTail recur_tail_eval(const TailIn &in, int p, int m, const double (&tot)[5])
{
    RecurTail o{};
    o.last = (p == m) || (p == in.kstop);
    const double g1 = in.g1;
    const double sig = in.sig;
    const double n = tot[0], an = tot[1], ov = tot[2], yy = tot[3], yv = tot[4];
    if (!isfinite(n) || !isfinite(an) || !isfinite(ov) || !isfinite(yy) || !isfinite(yv)) {
        o.fail = true;
        return o;
    }
    const double gp = sqrt(n);  // beta_{p-1}
    o.gp = gp;
    // breakdown scale on the unshifted alpha (the reading shared with the oracle)
    const double scale = fmax(in.scale, fabs(in.alpha_pm1 + sig));
    if (gp <= 1e-13 * scale) {
        // invariant Krylov subspace: stop with k_eff = p - 1, beta_k = gamma_p
        o.breakdown = true;
        o.beta_k = gp;
        return o;
    }
    o.scale = fmax(scale, gp);
    const double al = an / n - ov / g1;
    o.al = al;
    if (o.last) {
        // w = A u_m - alpha_m u_m - (gamma_m^2/gamma_{m-1}) u_{m-1} = gamma_m u_{m+1}
        const double bp = n / g1;
        const double w2 = yy + al * al * n + bp * bp * (g1 * g1) - 2.0 * al * an - 2.0 * bp * yv +
                          2.0 * al * bp * ov;
        o.beta_k = sqrt(fmax(w2, 0.0)) / gp;
    }
    return o;
}

__device__ __forceinline__ RecurTail recur_tail_eval(const Scalars *sc, const double *alpha, const double *gamma,
                                                     int p, int m, const double (&tot)[5])
{
    return recur_tail_eval(tail_inputs(sc, alpha, gamma, p), p, m, tot);
}

__device__ __forceinline__ void recur_tail_store(Scalars *sc, double *alpha, double *gamma, int p,
                                                 const RecurTail &o)
{
    if (o.fail) {
        sc->status = 3;
        sc->kstop = -1;
        return;
    }
    gamma[p] = o.gp;
    if (o.breakdown) {
        sc->keff = p - 1;
        sc->kstop = p - 1;
        sc->beta_k = o.beta_k;
        return;
    }
    sc->scale = o.scale;
    alpha[p] = o.al;
    if (o.last) sc->beta_k = o.beta_k;
}

__device__ __forceinline__ void recur_tail(const PassArgs &a, const double (&tot)[5])
{
    recur_tail_store(a.sc, a.alpha, a.gamma, a.pass, recur_tail_eval(a.sc, a.alpha, a.gamma, a.pass, a.m, tot));
}

template <class V1, class V2, class TO, bool HAS2, int PF, bool PY, int TERMS>
__global__ __launch_bounds__(kBlock) void k_recur(PassArgs a)
{
    Scalars *sc = a.sc;
    const int p = a.pass;
    double g1, alpha_pm1;
    if (a.defer && p >= 3) {
        // iteration p-1 left its partials for this kernel: every workgroup
        // folds them in the same order (so all agree bit for bit), takes the
        // scalars of p-1 from its own evaluation and workgroup 0 stores them
        // (iteration p-1 did not run when kstop < p-1)
        if (sc->kstop < p - 1) return;
        __shared__ double red[kWaves][5];
        double tot[5];
        fold_partials(a.prev_partials, a.prev_nblk, red, tot);
        const RecurTail o = recur_tail_eval(sc, a.alpha, a.gamma, p - 1, a.m, tot);
        if (blockIdx.x == 0 && threadIdx.x == 0) recur_tail_store(sc, a.alpha, a.gamma, p - 1, o);
        if (o.fail || o.breakdown || o.last) return;  // kstop < p from here on
        g1 = o.gp;
        alpha_pm1 = o.al;
    } else {
        if (sc->kstop < p) return;
        g1 = a.gamma[p - 1];
        alpha_pm1 = a.alpha[p - 1];
    }
    const WaveTask wt = wave_task(a.op, a.t);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    recur_body<V1, V2, TO, HAS2, PF, PY, TERMS>(a, wt, g1, alpha_pm1, acc);
    if (a.replay) return;  // the second run only regenerates u_p
    if (a.defer) {
        // folded by the next iteration's kernel (or the small exponential's)
        store_partial(acc, a.partials, (int)blockIdx.x);
        return;
    }
    double tot[5];
    if (!grid_reduce(acc, a.partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) recur_tail(a, tot);
}

// ---------------------------------------------------------------------------
// exp(-iT') e_1 for the k x k tridiagonal T' (Sec. 4, any standard method for
// the small exponential; T' = T - sigma I is the shifted matrix of the sweeps)
// in one wave, lane j holding row j.  Two methods, chosen by the half-width R
// of the Gershgorin interval [c0 - R, c0 + R] of T':
//  - R <= ~150: Chebyshev expansion (Tal-Ezer and Kosloff),
//    exp(-iT') = exp(-i c0) sum_n a_n T_n(X), X = (T' - c0 I) / R,
//    a_0 = J_0(R), a_n = 2 (-i)^n J_n(R), with N = R + 10 R^(1/3) + 20 terms
//    (the neglected coefficients sum to below 1e-17).  T_n(X) e_1 follows the
//    three-term recurrence t_{n+1} = 2 X t_n - t_{n-1} in real arithmetic, one
//    tridiagonal product from the neighbouring lanes per term.  The Bessel
//    values J_0..J_N(R) come from Miller's backward recurrence
//    J_{n-1} = (2n/R) J_n - J_{n+1}, started well above N, rescaled when large
//    and normalised by J_0 + 2 sum J_2k = 1.  A few microseconds.
//  - otherwise the eigendecomposition T' = Z Lambda Z^T by implicit symmetric
//    QR steps with Wilkinson shift: lane i holds d_i and the coupling e_i in
//    registers, the bulge chase fetches the next entries by shuffles one step
//    ahead, deflation is a ballot, lane j owns row j of Z in its own LDS
//    column; exp(-iT') e_1 = Z exp(-i Lambda) Z^T e_1.
// Output: coef[j] = c_j / gamma_j with c = ||psi|| exp(-i sigma) exp(-iT') e_1,
// and the step's error estimate beta_k |c_k| (eq. matrix_exponential_error).
// ---------------------------------------------------------------------------
constexpr int kChebMaxTerms = 224;

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = fmin(v, __shfl_xor(v, s, 64));
    return v;
}

__device__ __forceinline__ int cheb_terms(double R)
{
    return (int)ceil(R + 10.0 * cbrt(R) + 20.0);
}

// J_0(R) .. J_N(R) into jb[0..N] (one thread; R > 0).
__device__ void bessel_miller(double R, int N, double *jb)
{
    int M = N + 16 + (int)ceil(2.0 * sqrt((double)N));
    M += M & 1;
    const double ir = 1.0 / R;
    double jp1 = 0.0, j = 1e-300, sum = 0.0;
    for (int n = M; n >= 1; --n) {
        const double jm1 = (2.0 * n * ir) * j - jp1;  // J_{n-1} from J_n, J_{n+1}
        if (n <= N) jb[n] = j;
        if ((n & 1) == 0) sum += 2.0 * j;
        jp1 = j;
        j = jm1;
        if (fabs(j) > 1e250) {
            j *= 1e-250;
            jp1 *= 1e-250;
            sum *= 1e-250;
            for (int i = n; i <= N; ++i) jb[i] *= 1e-250;
        }
    }
    jb[0] = j;
    sum += j;
    const double is = 1.0 / sum;
    for (int i = 0; i <= N; ++i) jb[i] *= is;
    // the expansions read up to three orders past N, in groups of four
    for (int i = N + 1; i <= N + 3; ++i) jb[i] = 0.0;
}

// Start order of Miller's recurrence for J_0 .. J_N (even, as in bessel_miller).
__device__ __forceinline__ int miller_order(int N)
{
    const int M = N + 16 + (int)ceil(2.0 * sqrt((double)N));
    return M + (M & 1);
}

// |J_n| / J_M grows by at most (2M + x)/x per order below M, so from
// J_M = 1e-300 nothing can overflow while M log10((2M + x)/x) < 590.
__device__ __forceinline__ bool miller_safe(double x, int M)
{
    return (double)M * log10((2.0 * M + x) / x) < 590.0;
}

// Miller's backward recurrence with no rescaling and no branch (x > 0, M even,
// miller_safe(x, M)): J_M = 1e-300, J_{M+1} = 0, J_{n-1} = (2n/x) J_n -
// J_{n+1}; put(n, v) receives the unnormalised J_n for n = M .. 0, and the
// return value is the normalising factor 1 / (J_0 + 2 sum_k J_2k).
template <class Put>
__device__ __forceinline__ double miller_run(double x, int M, Put put)
{
    const double tx = 2.0 / x;
    double jp1 = 0.0, j = 1e-300, se = 0.0, nd = (double)M;
    for (int n = M; n >= 2; n -= 2) {
        put(n, j);
        se += j;  // even orders
        const double jm1 = (nd * tx) * j - jp1;
        put(n - 1, jm1);
        const double jm2 = ((nd - 1.0) * tx) * jm1 - j;
        jp1 = jm1;
        j = jm2;
        nd -= 2.0;
    }
    put(0, j);
    return 1.0 / (j + 2.0 * se);
}

// This lane's component of exp(-iT') e_1 for the leading kd x kd block of
// the tridiagonal T' (diagonal d, coupling e to the next row, em to the
// previous one; lanes >= kd must hold d = e = em = 0 outside the block) by the
// Chebyshev expansion.  Returns false, computing nothing, when the spectrum is
// too wide for kChebMaxTerms terms.  Called by the whole wave.
__device__ bool cheb_exp_e1(double d, double e, double em, int kd, int lane, double &cr, double &ci)
{
    // Bessel values up to the start order of the recurrence (N + 47 at most)
    __shared__ double jb[kChebMaxTerms + 48];
    __shared__ double jscale;
    const double rad = fabs(e) + fabs(em);
    const double glo = wave_min(lane < kd ? d - rad : INFINITY);
    const double ghi = wave_max(lane < kd ? d + rad : -INFINITY);
    const double c0 = 0.5 * (glo + ghi), R = 0.5 * (ghi - glo);
    const int N = R > 0.0 ? (R < 1e4 ? cheb_terms(R) : kChebMaxTerms + 1) : 0;
    if (N > kChebMaxTerms) return false;
    __syncthreads();  // jb of a previous call is read up to here
    if (lane == 0) {
        double s = 1.0;
        if (N > 0) {
            const int M = miller_order(N);
            if (miller_safe(R, M))
                s = miller_run(R, M, [&](int n, double v) { jb[n] = v; });
            else
                bessel_miller(R, N, jb);  // rescaled as it goes, normalised
        } else {
            jb[0] = 1.0;
        }
        jscale = s;
    }
    __syncthreads();
    // X = (T' - c0 I) / R on this lane's row (zero rows beyond kd)
    const double ir = N > 0 ? 1.0 / R : 0.0;
    const double xd = lane < kd ? (d - c0) * ir : 0.0, xe = e * ir, xem = em * ir;
    auto xmul = [&](double v) { return xem * from_left(v) + xd * v + xe * from_right(v); };
    const double s1 = jscale, s2 = 2.0 * s1;
    double tm = lane == 0 ? 1.0 : 0.0;  // T_0(X) e_1
    double vr = s1 * jb[0] * tm, vi = 0.0;
    double tc = xmul(tm);  // T_1(X) e_1
    if (N >= 1) vi -= s2 * jb[1] * tc;
    // terms n .. n+3 with n = 2 mod 4: phases (-i)^n = -1, i, 1, -i; the
    // last group runs up to three orders past N (more terms of the same
    // expansion; T_n(X) e_1 stays bounded by 1)
    for (int n = 2; n <= N; n += 4) {
        const double f0 = s2 * jb[n], f1 = s2 * jb[n + 1], f2 = s2 * jb[n + 2], f3 = s2 * jb[n + 3];
        const double t2 = 2.0 * xmul(tc) - tm;
        const double t3 = 2.0 * xmul(t2) - tc;
        const double t4 = 2.0 * xmul(t3) - t2;
        const double t5 = 2.0 * xmul(t4) - t3;
        vr -= f0 * t2;
        vi += f1 * t3;
        vr += f2 * t4;
        vi -= f3 * t5;
        tm = t4;
        tc = t5;
    }
    double sn, cs;
    sincos(c0, &sn, &cs);
    cr = cs * vr + sn * vi;
    ci = cs * vi - sn * vr;
    return true;
}

// Adaptive Krylov dimension (Sec. 4: the estimate can steer k): the
// dimension of the next step, from this step's T.  If this step's estimate
// beta_k ||psi|| |c_k| exceeded ktol, grow by two; otherwise take the smallest
// j >= kmin whose estimate beta_j ||psi|| |(exp(-iT'_j) e_1)_j| for the
// leading j x j block is at most ktol / 2 (the next step's spectrum is close
// to this one's), else keep k.  Called by the whole wave after the
// coefficients of this step are written.
__device__ void predict_k(const double *alpha, const double *gamma, Scalars *sc, int k, int lane, double errk)
{
    const double g1 = gamma[1];
    int knext = k;
    if (errk > sc->ktol) {
        knext = min(k + 2, sc->kmax);
    } else {
        for (int j = max(sc->kmin, 1); j < k; ++j) {
            const double d = (lane < j) ? alpha[lane + 1] : 0.0;
            const double e = (lane + 1 < j) ? gamma[lane + 2] : 0.0;
            double em = from_left(e);
            if (lane == 0) em = 0.0;
            double cr = 0.0, ci = 0.0;
            if (!cheb_exp_e1(d, e, em, j, lane, cr, ci)) break;
            const double cj = __shfl(sqrt(cr * cr + ci * ci), j - 1, 64);
            if (gamma[j + 1] * g1 * cj <= 0.5 * sc->ktol) {
                knext = j;
                break;
            }
        }
    }
    if (lane == 0) sc->knext = max(knext, max(sc->kmin, 1));
}

// Bound of the step's error caused by storing u_2..u_k rounded (mixed
// precision).  The stored vectors satisfy the perturbed Lanczos relation
// A Q = Q T + beta_k q_{k+1} e_k^T - F, column j of F being the rounding of
// u_{j+1} = beta_j q_{j+1}, ||F e_j|| <= (reps beta_j + rabs) / (1 - reps).
// y(t) = ||psi|| Q exp(-itT) e_1 then solves y' = -iAy + i(beta_k q_{k+1} e_k^T
// - F) s(t) with s(t) = ||psi|| exp(-itT) e_1 and y(0) = psi, so for Hermitian
// A the error at t = 1 is at most int_0^1 ||F s(t)|| dt (plus the Krylov term
// of eq. matrix_exponential_error), with no assumption of orthogonality, and
// int_0^1 |s_j(t)| dt <= (int_0^1 |s_j(t)|^2 dt)^(1/2) (Cauchy-Schwarz).
// While the Gershgorin half-width R of T (centre c0) is at most 40 the
// integral is taken by Gauss-Legendre quadrature on [0, 1] with
// min(48, ceil(R) + 10) nodes (|s_j|^2 is a trigonometric sum of frequencies
// below 2R, inside the rule's resolution) and a 1% margin on the integral.
// s(t_q) at every node is one Chebyshev expansion of exp(-i t_q (T - c0 I))
// e_1 = sum_n a_n T_n(X) e_1 (X = (T - c0 I) / R, a_0 = J_0(t_q R), a_n =
// 2 (-i)^n J_n(t_q R)): the vectors T_n(X) e_1 are formed once and shared by
// all nodes, the Bessel values by Miller's backward recurrence, one lane per
// node.  The scalar phase exp(-i t c0) does not change |s_j| and is left
// out.  For 40 < R <= 70: |s_j(t)| <= ||psi|| [exp(t|X|) e_1]_j for X = T -
// c0 I (path sums of X^n), a Taylor series of non-negative terms with N = 3R +
// 40 terms plus its tail bound, capped at 1; beyond R = 70 the factor is 1.
// Lane l handles j = l + 1; beta_j is lane l's coupling e.
constexpr int kBoundNodes = 48;
constexpr int kBoundMinNodes = 8;
constexpr double kBoundMaxR = 40.0;
// terms of the expansion at t R <= R <= 40: ceil(R + 6 R^(1/3) + 12) <= 73
// leaves a truncation below 1e-13
constexpr int kBoundMaxTerms = 73;
// one node's Bessel values J_0 .. J_{N+3} and a slot that takes the
// recurrence's higher orders; an odd row length so the lanes' rows start on
// different LDS banks
constexpr int kBoundRow = kBoundMaxTerms + 6;
// LDS (doubles) of the quadrature: the vectors T_n(X) e_1 (rows of 64) and
// the Bessel rows of the nodes
constexpr int kBoundVecRows = kBoundMaxTerms + 4;
constexpr int kBoundLds = kBoundVecRows * 64 + kBoundNodes * kBoundRow;

// Gauss-Legendre rules on [0, 1] of sizes kBoundMinNodes .. kBoundNodes,
// concatenated (rule n from gl_base(n), nodes ascending), built at compile
// time by Newton's method on P_n from the classical starting guess
// cos(pi (q + 3/4) / (n + 1/2)) (six steps; the rule is symmetric about 1/2).
constexpr int gl_base(int n)
{
    return n * (n - 1) / 2 - kBoundMinNodes * (kBoundMinNodes - 1) / 2;
}
constexpr int kGLTotal = gl_base(kBoundNodes + 1);
struct GLRules {
    double t[kGLTotal];
    double w[kGLTotal];
};
constexpr double cx_cos(double x)
{
    // Taylor series, |x| <= pi
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 24; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
constexpr void cx_legendre(int n, double x, double &p, double &dp)
{
    double p0 = 1.0, p1 = 0.0;
    for (int j = 1; j <= n; ++j) {
        const double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p2) / j;
    }
    p = p0;
    dp = n * (x * p0 - p1) / (x * x - 1.0);
}
constexpr GLRules make_gl_rules()
{
    GLRules g{};
    for (int n = kBoundMinNodes; n <= kBoundNodes; ++n) {
        for (int q = 0; q < (n + 1) / 2; ++q) {
            double x = cx_cos(3.14159265358979323846 * (q + 0.75) / (n + 0.5)), p = 0.0, dp = 1.0;
            for (int it = 0; it < 6; ++it) {
                cx_legendre(n, x, p, dp);
                x -= p / dp;
            }
            cx_legendre(n, x, p, dp);
            const double w = 1.0 / ((1.0 - x * x) * dp * dp);
            g.t[gl_base(n) + q] = 0.5 * (1.0 - x);
            g.w[gl_base(n) + q] = w;
            g.t[gl_base(n) + n - 1 - q] = 0.5 * (1.0 + x);
            g.w[gl_base(n) + n - 1 - q] = w;
        }
    }
    return g;
}
constexpr GLRules kGLRules = make_gl_rules();

// lds: kBoundLds doubles of the calling workgroup's LDS (free on entry,
// reused by the caller afterwards).
__device__ double storage_bound(double d, double e, double em, int k, int lane, double g1, double reps,
                                double rabs, double *lds)
{
    __shared__ double jsc[kBoundNodes], wnode[kBoundNodes];
    if (!(reps > 0.0) && !(rabs > 0.0)) return 0.0;
    const double rad = fabs(e) + fabs(em);
    const double glo = wave_min(lane < k ? d - rad : INFINITY);
    const double ghi = wave_max(lane < k ? d + rad : -INFINITY);
    const double c0 = 0.5 * (glo + ghi), R = 0.5 * (ghi - glo);
    double f = 1.0;
    if (R <= kBoundMaxR) {
        // |s_j|^2 has frequencies below 2R: ceil(R) + 10 nodes integrate it to
        // ~1e-8 relative, far inside the margin; nodes in blocks of four
        // (the padding has zero weight)
        const int nn = min(kBoundNodes, max(kBoundMinNodes, (int)ceil(R) + 10));
        const int nb = (nn + 3) & ~3;
        const int N = R > 0.0 ? min((int)ceil(R + 6.0 * cbrt(R) + 12.0), kBoundMaxTerms) : 0;
        double *vt = lds;                // row n: T_n(X) e_1 (n <= N + 3)
        double *jt = lds + kBoundVecRows * 64;  // row q: J_n(t_q R), unnormalised
        __syncthreads();  // LDS of an earlier use is read up to here
        if (lane < nb) {
            double *row = jt + lane * kBoundRow;
            double s = 0.0, wq = 0.0;
            if (lane < nn) {
                const double x = kGLRules.t[gl_base(nn) + lane] * R;
                wq = kGLRules.w[gl_base(nn) + lane];
                s = 1.0;
                if (x > 0.0) {
                    const int M = miller_order(N), top = N + 4;  // orders above N + 3 land in row[top]
                    if (miller_safe(x, M))
                        s = miller_run(x, M, [&](int n, double v) { row[min(n, top)] = v; });
                    else
                        bessel_miller(x, N, row);  // rescaled as it goes, normalised
                } else {
                    row[0] = 1.0;
                    for (int n = 1; n <= N + 3; ++n) row[n] = 0.0;
                }
            } else {
                for (int n = 0; n <= N + 3; ++n) row[n] = 0.0;
            }
            jsc[lane] = s;
            wnode[lane] = wq;
        }
        const double ir = R > 0.0 ? 1.0 / R : 0.0;
        const double xd = lane < k ? (d - c0) * ir : 0.0, xe = e * ir, xem = em * ir;
        auto xmul = [&](double v) { return xem * from_left(v) + xd * v + xe * from_right(v); };
        double tm = lane == 0 ? 1.0 : 0.0, tc = xmul(tm);
        vt[lane] = tm;
        vt[64 + lane] = tc;
        for (int n = 2; n <= N + 3; ++n) {
            const double tn = 2.0 * xmul(tc) - tm;
            vt[n * 64 + lane] = tn;
            tm = tc;
            tc = tn;
        }
        __syncthreads();
        // per node, halved: a = J_0 v_0 / 2 - J_2 v_2 + J_4 v_4 - ..., b = -J_1 v_1
        // + J_3 v_3 - ..., so that s_j(t_q) = 2 (a + i b) times the
        // normalisation of the node's Bessel values.  The vector needs kk
        // lanes (the power of two >= k); the wave's 64 / kk lane groups take
        // every (64 / kk)-th block of four nodes, and their integrals are
        // added in a fixed order below.
        const int kk = k <= 16 ? 16 : (k <= 32 ? 32 : 64);
        const int jl = lane & (kk - 1), grp = lane / kk, ng = 64 / kk;
        const double v0 = vt[jl], v1 = vt[64 + jl];
        double integral = 0.0;
        for (int q = 4 * grp; q < nb; q += 4 * ng) {
            const double *r0 = jt + q * kBoundRow, *r1 = r0 + kBoundRow, *r2 = r1 + kBoundRow,
                         *r3 = r2 + kBoundRow;
            double a0 = 0.5 * r0[0] * v0, a1 = 0.5 * r1[0] * v0, a2 = 0.5 * r2[0] * v0, a3 = 0.5 * r3[0] * v0;
            double b0 = -r0[1] * v1, b1 = -r1[1] * v1, b2 = -r2[1] * v1, b3 = -r3[1] * v1;
            // orders n .. n+3 with n = 2 mod 4, phases -1, i, 1, -i (up to
            // three orders past N: more terms of the same expansion)
            for (int n = 2; n <= N; n += 4) {
                const double w2 = vt[n * 64 + jl], w3 = vt[(n + 1) * 64 + jl], w4 = vt[(n + 2) * 64 + jl],
                             w5 = vt[(n + 3) * 64 + jl];
                a0 -= r0[n] * w2;
                b0 += r0[n + 1] * w3;
                a1 -= r1[n] * w2;
                b1 += r1[n + 1] * w3;
                a2 -= r2[n] * w2;
                b2 += r2[n + 1] * w3;
                a3 -= r3[n] * w2;
                b3 += r3[n + 1] * w3;
                a0 += r0[n + 2] * w4;
                b0 -= r0[n + 3] * w5;
                a1 += r1[n + 2] * w4;
                b1 -= r1[n + 3] * w5;
                a2 += r2[n + 2] * w4;
                b2 -= r2[n + 3] * w5;
                a3 += r3[n + 2] * w4;
                b3 -= r3[n + 3] * w5;
            }
            // normalised before squaring: the unnormalised sums and their
            // normalising factor each span up to 1e+-270, beyond the range
            // of their squares
            const double s0 = jsc[q], s1 = jsc[q + 1], s2 = jsc[q + 2], s3 = jsc[q + 3];
            a0 *= s0;
            b0 *= s0;
            a1 *= s1;
            b1 *= s1;
            a2 *= s2;
            b2 *= s2;
            a3 *= s3;
            b3 *= s3;
            integral += wnode[q] * (a0 * a0 + b0 * b0) + wnode[q + 1] * (a1 * a1 + b1 * b1) +
                        wnode[q + 2] * (a2 * a2 + b2 * b2) + wnode[q + 3] * (a3 * a3 + b3 * b3);
        }
        // lane j (< k) receives the sum over the groups of component j
        if (kk <= 32) integral += __shfl_xor(integral, 32, 64);
        if (kk <= 16) integral += __shfl_xor(integral, 16, 64);
        f = fmin(1.0, sqrt(4.04 * integral));
    } else if (R <= 30.0 + kBoundMaxR) {
        // X = T - c0 I with entrywise absolute value: |s_j(t)| <= [exp(|X|) e_1]_j
        const double xd = lane < k ? fabs(d - c0) : 0.0, xe = fabs(e), xem = fabs(em);
        const int N = (int)ceil(3.0 * R) + 40;
        double t = lane == 0 ? 1.0 : 0.0, v = t;
        for (int n = 1; n <= N; ++n) {
            t = (xem * from_left(t) + xd * t + xe * from_right(t)) / (double)n;
            v += t;
        }
        const double tail = exp((double)(N + 1) * log(R) + R - lgamma((double)N + 2.0));
        f = fmin(1.0, v + tail);
    }
    double v = (lane + 1 < k) ? f * (reps * fabs(e) + rabs) / (1.0 - reps) : 0.0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    return g1 * v;
}

__device__ __forceinline__ void tridiag_body(const double *alpha, const double *gamma, Scalars *sc, StepStat *stat,
                                             double reps, double rabs)
{
    // eigenvector columns of the QR path; first the storage bound's quadrature
    __shared__ double zpr[(kMaxM + 1) * 64 > kBoundLds ? (kMaxM + 1) * 64 : kBoundLds];
    __shared__ double wre[kMaxM], wim[kMaxM];
    const int lane = threadIdx.x;
    // every scalar of the step read up front, so the loads overlap (the last
    // sweep wrote them just before)
    const int status = sc->status, k = sc->keff;
    const double sigma = sc->sigma, beta_k = sc->beta_k, ktol = sc->ktol;
    if (status != 0) return;
    if (k <= 0) {
        for (int j = lane; j < 2 * (kMaxM + 2); j += 64) sc->coef[j] = 0.0;
        if (lane == 0) {
            sc->cabs_k = 0.0;
            stat->keff = 0;
            stat->err_est = 0.0;
            stat->round_bound = 0.0;
        }
        return;
    }
    double d = (lane < k) ? alpha[lane + 1] : 0.0;
    double e = (lane + 1 < k) ? gamma[lane + 2] : 0.0;  // zero for lanes >= k-1
    const double gl = (lane < k) ? gamma[lane + 1] : 1.0, g1 = gamma[1];
    double em = from_left(e);                           // e_{j-1}
    if (lane == 0) em = 0.0;
    const double rb = storage_bound(d, e, em, k, lane, g1, reps, rabs, zpr);
    double cr = 0.0, ci = 0.0;
    if (!cheb_exp_e1(d, e, em, k, lane, cr, ci)) {
#define ZZ(i) zpr[(i) * 64 + lane]
        for (int i = 0; i < k; ++i) ZZ(i) = (i == lane) ? 1.0 : 0.0;
        const double eps = 2.220446049250313e-16;
        for (int iter = 0; iter < 40 * kMaxM; ++iter) {
            // negligible couplings are set to zero; find the last unreduced block [l, h]
            const double dn = __shfl_down(d, 1, 64);
            const bool live = lane + 1 < k && e != 0.0;
            const bool tiny = live && fabs(e) <= eps * (fabs(d) + fabs(dn));
            if (tiny) e = 0.0;
            const unsigned long long mask = __ballot(live && !tiny);
            if (mask == 0ull) break;
            const int hb = 63 - __clzll(mask);  // highest coupling still live
            const unsigned long long below = ~mask & ((1ull << hb) - 1ull);
            const int l = below ? 64 - __clzll(below) : 0;
            const int h = hb + 1;
            // Wilkinson shift from the trailing 2x2 block of [l, h]
            const double dh1 = __shfl(d, h - 1, 64), dh = __shfl(d, h, 64), eh1 = __shfl(e, h - 1, 64);
            const double delta = 0.5 * (dh1 - dh);
            const double b2 = eh1 * eh1;
            const double mu = dh - b2 / (delta + copysign(sqrt(delta * delta + b2), delta));
            double aq = __shfl(d, l, 64);  // current d_q
            double bq = __shfl(e, l, 64);  // current e_q
            double x = aq - mu, z = bq;
            double aq1n = __shfl(d, l + 1, 64);
            double bq1n = (l + 1 < h) ? __shfl(e, l + 1, 64) : 0.0;
            double zq = ZZ(l);
            for (int q = l; q < h; ++q) {
                const double aq1 = aq1n, bq1 = bq1n;
                // entries of the next step, fetched ahead (lanes > q+1 are untouched so far)
                aq1n = __shfl(d, min(q + 2, 63), 64);
                bq1n = (q + 2 < h) ? __shfl(e, min(q + 2, 63), 64) : 0.0;
                const double zq1 = ZZ(q + 1);
                const double rr = x * x + z * z;
                double c = 1.0, s = 0.0, r = 0.0;
                if (rr > 0.0) {
                    const double ir = rsqrt(rr);
                    c = x * ir;
                    s = -z * ir;
                    r = rr * ir;
                }
                if (q > l && lane == q - 1) e = r;
                const double cc = c * c, ss = s * s, cs = c * s;
                const double dq = cc * aq - 2.0 * cs * bq + ss * aq1;
                const double dq1 = ss * aq + 2.0 * cs * bq + cc * aq1;
                const double eq = cs * (aq - aq1) + (cc - ss) * bq;
                if (lane == q) d = dq;
                ZZ(q) = c * zq - s * zq1;
                zq = s * zq + c * zq1;
                aq = dq1;
                if (q + 1 < h) {
                    x = eq;
                    z = -s * bq1;
                    bq = c * bq1;
                } else {
                    if (lane == q) e = eq;
                    if (lane == q + 1) d = dq1;
                }
            }
            ZZ(h) = zq;
        }
        // c_j = sum_i Z[j][i] exp(-i lambda_i) Z[0][i]; lambda_i is lane i's d
        __syncthreads();
        if (lane < k) {
            double sn, cs;
            sincos(d, &sn, &cs);
            const double z0 = zpr[lane * 64 + 0];
            wre[lane] = z0 * cs;
            wim[lane] = -z0 * sn;
        }
        __syncthreads();
        if (lane < k) {
            for (int i = 0; i < k; ++i) {
                const double zji = ZZ(i);
                cr += zji * wre[i];
                ci += zji * wim[i];
            }
        }
#undef ZZ
    }
    double ck = 0.0;
    if (lane < k) {
        // exp(-iT) = exp(-i sigma) exp(-iT') for the shifted tridiagonal T'
        double ss, sc0;
        sincos(sigma, &ss, &sc0);
        const double tr = g1 * (cr * sc0 + ci * ss), ti = g1 * (ci * sc0 - cr * ss);
        const double ig = 1.0 / gl;
        sc->coef[2 * (lane + 1)] = tr * ig;
        sc->coef[2 * (lane + 1) + 1] = ti * ig;
        ck = sqrt(tr * tr + ti * ti);
        if (lane == k - 1) {
            sc->cabs_k = ck;
            stat->keff = k;
            stat->err_est = beta_k * ck;
            stat->round_bound = rb;
        }
    }
    if (ktol > 0.0) predict_k(alpha, gamma, sc, k, lane, beta_k * __shfl(ck, k - 1, 64));
}

// The scalar update of the step's last iteration from the partials it left
// for the next kernel (one wave; iteration f.pass ran when kstop >= f.pass).
__device__ __forceinline__ void fold_last_tail(double *alpha, double *gamma, Scalars *sc, const TailFold &f)
{
    if (f.pass < 2) return;
    // the partials (inside the table whether or not they are used), the
    // scalars and the chain entries the update reads are loaded together,
    // before the status decides whether to use them: one memory round trip
    // instead of three
    const int status = sc->status;
    const TailIn in = tail_inputs(sc, alpha, gamma, f.pass);
    double tot[5];
    fold_partials_wave(f.partials, f.nblk, tot);
    if (status == 0 && in.kstop >= f.pass) {
        const RecurTail o = recur_tail_eval(in, f.pass, f.pass, tot);
        if (threadIdx.x == 0) recur_tail_store(sc, alpha, gamma, f.pass, o);
        __threadfence_block();
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_tridiag(double *alpha, double *gamma, Scalars *sc, StepStat *stat,
                                                double reps, double rabs, TailFold f)
{
    fold_last_tail(alpha, gamma, sc, f);
    tridiag_body(alpha, gamma, sc, stat, reps, rabs);
}

// The last iteration's scalar update alone, for callers that need the whole
// tridiagonal T before the small exponential runs.
__global__ __launch_bounds__(64) void k_fold_tail(double *alpha, double *gamma, Scalars *sc, TailFold f)
{
    fold_last_tail(alpha, gamma, sc, f);
}

// ---------------------------------------------------------------------------
// Recombination psi_new = sum_j c_j q_j = sum_j (c_j / gamma_j) u_j
// (eq. matrix_exp_approx): a site-local multi-axpy, plus ||psi_new||^2 for the
// step statistics.  A workgroup owns a tile of 256*S sites and streams the
// Krylov vectors one after the other over it (S sites per thread, strided by
// the workgroup so every load is coalesced), so each vector is read in long
// contiguous runs.  The streams are read once and never reused: nontemporal
// loads and stores keep them from displacing cache lines of the other
// streams.
// ---------------------------------------------------------------------------
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    const dv2 v = __builtin_nontemporal_load(reinterpret_cast<const dv2 *>(p));
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ void st_stream(double2 *p, double x, double y)
{
    dv2 v;
    v.x = x;
    v.y = y;
    __builtin_nontemporal_store(v, reinterpret_cast<dv2 *>(p));
}

template <class TB>
__device__ __forceinline__ Raw<TB> ld_site(const char *p);
template <>
__device__ __forceinline__ Raw<float2> ld_site<float2>(const char *p)
{
    const fv4 v = __builtin_nontemporal_load(reinterpret_cast<const fv4 *>(p));
    return Raw<float2>{make_float2(v.x, v.y), make_float2(v.z, v.w)};
}
template <>
__device__ __forceinline__ Raw<double2> ld_site<double2>(const char *p)
{
    return Raw<double2>{ld_stream(reinterpret_cast<const double2 *>(p)),
                        ld_stream(reinterpret_cast<const double2 *>(p) + 1)};
}

// Tiles blk, blk + nblk, ... of the recombination; nrm += ||psi_new||^2 of them.
template <class TB, int S>
__device__ __forceinline__ void combine_body(const CombArgs &a, int blk, int nblk, double &nrm)
{
    const Scalars *sc = a.sc;
    const int k = sc->keff;
    // complex64 form: the coefficients c_j / gamma_j staged once per workgroup
    // in LDS (the FP64 form reads them from the scalars)
    constexpr bool kPairs = sizeof(TB) == 8;
    __shared__ double cs[kPairs ? 2 * (kMaxM + 2) : 1];
    if constexpr (kPairs) {
        for (int i = threadIdx.x; i < 2 * (k + 1); i += kBlock) cs[i] = sc->coef[i];
        __syncthreads();
    }
    auto cf = [&](int i) -> double {
        if constexpr (kPairs)
            return cs[i];
        else
            return sc->coef[i];
    };
    const char *__restrict__ basis = static_cast<const char *>(a.basis);
    const size_t sites = a.sites;
    const size_t tile = (size_t)kBlock * S;
    constexpr size_t kSite = 2 * sizeof(TB);
    if constexpr (!kPairs) {
        // FP64: element by element (one complex128 of one component per lane
        // and slot: element e is component e & 1 of site e >> 1), so that
        // consecutive lanes read consecutive 16-byte elements of the paired
        // basis; a tile of kBlock * S sites is 2 S elements per thread.  Each
        // element is c_1 psi + sum_j c_j u_j in order j = 2..k, as one
        // component of the complex64 site form below.
        const size_t nel = 2 * sites;
        for (size_t s0 = (size_t)blk * tile; s0 < sites; s0 += (size_t)nblk * tile) {
            const size_t e0 = 2 * s0;
            double ar[2 * S], ai[2 * S];
            {
                const double cr = k >= 1 ? cf(2) : 0.0, ci = k >= 1 ? cf(3) : 0.0;
#pragma unroll
                for (int q = 0; q < 2 * S; ++q) {
                    const size_t e = e0 + (size_t)q * kBlock + threadIdx.x;
                    double2 p = make_double2(0.0, 0.0);
                    if (e < nel) p = ld_stream(a.psi + (e & 1) * sites + (e >> 1));
                    ar[q] = cr * p.x - ci * p.y;
                    ai[q] = cr * p.y + ci * p.x;
                }
            }
            for (int j = 2; j <= k; ++j) {
                const double2 *u = reinterpret_cast<const double2 *>(basis + (size_t)(j - 2) * a.vec_bytes);
                double2 v[2 * S];
#pragma unroll
                for (int q = 0; q < 2 * S; ++q) {
                    const size_t e = e0 + (size_t)q * kBlock + threadIdx.x;
                    v[q] = e < nel ? ld_stream(u + e) : make_double2(0.0, 0.0);
                }
                const double cr = sc->coef[2 * j], ci = sc->coef[2 * j + 1];
#pragma unroll
                for (int q = 0; q < 2 * S; ++q) {
                    ar[q] += cr * v[q].x - ci * v[q].y;
                    ai[q] += cr * v[q].y + ci * v[q].x;
                }
            }
#pragma unroll
            for (int q = 0; q < 2 * S; ++q) {
                const size_t e = e0 + (size_t)q * kBlock + threadIdx.x;
                if (e < nel) {
                    st_stream(a.out + (e & 1) * sites + (e >> 1), ar[q], ai[q]);
                    nrm += ar[q] * ar[q] + ai[q] * ai[q];
                }
            }
        }
        return;
    }
    for (size_t s0 = (size_t)blk * tile; s0 < sites; s0 += (size_t)nblk * tile) {
        Sp acc[S];
        {
            const double cr = k >= 1 ? cf(2) : 0.0, ci = k >= 1 ? cf(3) : 0.0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const size_t s = s0 + (size_t)q * kBlock + threadIdx.x;
                double2 p0 = make_double2(0.0, 0.0), p1 = p0;
                if (s < sites) {
                    p0 = ld_stream(a.psi + s);
                    p1 = ld_stream(a.psi + sites + s);
                }
                acc[q].r0 = cr * p0.x - ci * p0.y;
                acc[q].i0 = cr * p0.y + ci * p0.x;
                acc[q].r1 = cr * p1.x - ci * p1.y;
                acc[q].i1 = cr * p1.y + ci * p1.x;
            }
        }
        if constexpr (kPairs) {
            auto load = [&](int j, Raw<TB>(&v)[S]) {
                const char *u = basis + (size_t)(j - 2) * a.vec_bytes;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const size_t s = s0 + (size_t)q * kBlock + threadIdx.x;
                    v[q] = s < sites ? ld_site<TB>(u + s * kSite) : raw_zero<TB>();
                }
            };
            auto add = [&](int j, const Raw<TB>(&v)[S]) {
                const double cr = cf(2 * j), ci = cf(2 * j + 1);
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const Sp w = to_sp(v[q]);
                    acc[q].r0 += cr * w.r0 - ci * w.i0;
                    acc[q].i0 += cr * w.i0 + ci * w.r0;
                    acc[q].r1 += cr * w.r1 - ci * w.i1;
                    acc[q].i1 += cr * w.i1 + ci * w.r1;
                }
            };
            // two vectors at a time, so that 2S loads are in flight before
            // the arithmetic (the terms are still added in order j = 2..k)
            int j = 2;
            for (; j + 1 <= k; j += 2) {
                Raw<TB> v0[S], v1[S];
                load(j, v0);
                load(j + 1, v1);
                add(j, v0);
                add(j + 1, v1);
            }
            if (j <= k) {
                Raw<TB> v[S];
                load(j, v);
                add(j, v);
            }
        }
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const size_t s = s0 + (size_t)q * kBlock + threadIdx.x;
            if (s < sites) {
                st_stream(a.out + s, acc[q].r0, acc[q].i0);
                st_stream(a.out + sites + s, acc[q].r1, acc[q].i1);
                nrm += sp_norm2(acc[q]);
            }
        }
    }
}

__device__ __forceinline__ void combine_tail(const CombArgs &a, const double (&tot)[1])
{
    Scalars *sc = a.sc;
    a.stat->norm2 = tot[0];
    if (!isfinite(tot[0])) {
        sc->status = 3;
        sc->kstop = -1;
        return;
    }
    sc->steps_done += 1;
}

// WPE: minimum resident waves per SIMD asked of the register allocator.
template <class TB, int S, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_combine(CombArgs a)
{
    if (a.sc->status != 0) return;
    if (a.keep != nullptr && blockIdx.x == 0) {
        // the scalars, alpha and gamma are final once the small exponential
        // has run; the recombination changes only the ticket, the step count
        // and, for a non-finite norm, the status (which the caller checks on
        // the live scalars)
        static_assert(sizeof(Scalars) % 8 == 0, "the scalars are copied as 8-byte words");
        constexpr int kWords = (int)(sizeof(Scalars) / 8);
        const auto *src = reinterpret_cast<const unsigned long long *>(a.sc);
        auto *d = reinterpret_cast<unsigned long long *>(a.keep);
        for (int i = threadIdx.x; i < kWords; i += kBlock) d[i] = src[i];
        double *da = reinterpret_cast<double *>(a.keep + a.keep_alpha), *dg = reinterpret_cast<double *>(a.keep + a.keep_gamma);
        for (int i = threadIdx.x; i < a.keep_nab; i += kBlock) {
            da[i] = a.alpha[i];
            dg[i] = a.gamma[i];
        }
    }
    double nrm = 0.0;
    combine_body<TB, S>(a, (int)blockIdx.x, (int)gridDim.x, nrm);
    double accv[1] = {nrm}, tot[1];
    if (!grid_reduce(accv, a.partials, &a.sc->ticket, tot)) return;
    if (threadIdx.x == 0) combine_tail(a, tot);
}

// Recombination terms p0 .. p0 + nv - 1 of the second Lanczos run (AccumArgs):
// out = c_1 psi + ... in term order, the arithmetic per site that of
// combine_body.  Terms beyond k_eff add nothing; the launch holding term k_eff
// (or the first launch when k_eff = 0: psi = 0 gives out = 0) reduces the new
// norm and completes the step.
template <class TB, int S>
__global__ __launch_bounds__(kBlock) void k_accum(AccumArgs a)
{
    Scalars *sc = a.sc;
    if (sc->status != 0) return;
    const int k = sc->keff;
    const int p0 = a.p0;
    const int pend = min(p0 + a.nv - 1, k);  // last term of this launch that counts
    const bool first = p0 == 1;
    if (!first && p0 > k) return;
    const size_t sites = a.sites;
    const size_t tile = (size_t)kBlock * S;
    constexpr size_t kSite = 2 * sizeof(TB);
    double nrm = 0.0;
    for (size_t s0 = (size_t)blockIdx.x * tile; s0 < sites; s0 += (size_t)gridDim.x * tile) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const size_t s = s0 + (size_t)q * kBlock + threadIdx.x;
            if (s >= sites) continue;
            Sp acc;
            if (first) {
                const double cr = k >= 1 ? sc->coef[2] : 0.0, ci = k >= 1 ? sc->coef[3] : 0.0;
                const double2 p0v = ld_stream(a.psi + s), p1v = ld_stream(a.psi + sites + s);
                acc.r0 = cr * p0v.x - ci * p0v.y;
                acc.i0 = cr * p0v.y + ci * p0v.x;
                acc.r1 = cr * p1v.x - ci * p1v.y;
                acc.i1 = cr * p1v.y + ci * p1v.x;
            } else {
                const double2 o0 = a.out[s], o1 = a.out[sites + s];
                acc.r0 = o0.x;
                acc.i0 = o0.y;
                acc.r1 = o1.x;
                acc.i1 = o1.y;
            }
#pragma unroll
            for (int v = 0; v < kAccumTerms; ++v) {
                const int j = p0 + v;
                if (j < 2 || j > pend) continue;
                const Sp w = to_sp(ld_site<TB>(static_cast<const char *>(a.u[v]) + s * kSite));
                const double cr = sc->coef[2 * j], ci = sc->coef[2 * j + 1];
                acc.r0 += cr * w.r0 - ci * w.i0;
                acc.i0 += cr * w.i0 + ci * w.r0;
                acc.r1 += cr * w.r1 - ci * w.i1;
                acc.i1 += cr * w.i1 + ci * w.r1;
            }
            a.out[s] = make_double2(acc.r0, acc.i0);
            a.out[sites + s] = make_double2(acc.r1, acc.i1);
            nrm += sp_norm2(acc);
        }
    }
    if (p0 + a.nv - 1 < k) return;  // term k_eff comes in a later launch
    double accv[1] = {nrm}, tot[1];
    if (!grid_reduce(accv, a.partials, &sc->ticket, tot)) return;
    if (threadIdx.x == 0) {
        a.stat->norm2 = tot[0];
        if (!isfinite(tot[0])) {
            sc->status = 3;
            sc->kstop = -1;
            return;
        }
        sc->steps_done += 1;
    }
}

// sites per thread of the recombination and the occupancy asked for (the
// complex64 form with two vectors in flight: four waves per SIMD; its wide
// form, for grids of at least one wide tile per compute unit and for
// batches, holds 16 sites per thread at one wave per SIMD)
#ifndef DL_COMB_S_MIXED
#define DL_COMB_S_MIXED 4
#endif
#ifndef DL_COMB_S_MIXED_WIDE
#define DL_COMB_S_MIXED_WIDE 16
#endif
#ifndef DL_COMB_BLOCKS_PER_CU
#define DL_COMB_BLOCKS_PER_CU 4
#endif
constexpr int kCombMixed = DL_COMB_S_MIXED;
constexpr int kCombMixedWide = DL_COMB_S_MIXED_WIDE;
constexpr int kCombWpeMixedWide = 1;
constexpr int kCombFp64 = 8;
constexpr int kCombFp64Narrow = 2;  // FP64 grids below four wide tiles per compute unit
#ifndef DL_COMB_WPE_MIXED
#define DL_COMB_WPE_MIXED 4
#endif
constexpr int kCombWpeMixed = DL_COMB_WPE_MIXED;
constexpr int kCombWpeFp64 = 1;
constexpr int kCombWpeFp64Narrow = 4;

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
    const double gy = gyh - op.bqy * lg.x;
    const Planar vin{reinterpret_cast<const char *>(x), plane * 16, (uint32_t)op.nx * 16u};
    const uint32_t off = lg.inx ? Planar::lane_offset(lg.colw) : kOob;
    Sp p0 = sp_zero(), p1 = sp_zero();
    Sp p2 = to_sp(load_row(vin, op, off, wt.y0 - 1));
    for (int R = wt.y0; R <= wt.y1; ++R) {
        p0 = p1;
        p1 = p2;
        p2 = to_sp(load_row(vin, op, off, R));
        if (R - 1 < wt.y0) continue;
        const RowGeo rg = row_geo(op, R - 1);
        const Sp o = hop(op, p1, sp_left(p1), sp_right(p1), p0, p2, site_pot(op, lg, rg),
                         gxh + op.bq * rg.y, gy);
        if (lg.own) {
            const size_t idx = (size_t)(R - 1) * op.nx + lg.colw;
            y[idx] = make_double2(o.r0, o.i0);
            y[plane + idx] = make_double2(o.r1, o.i1);
        }
    }
}

// Scalars to the start-of-call state.  keep_status: an asynchronous call
// leaves a failure of an earlier call in place (its kernels then do nothing)
// until the host has read it.  kmin, kmax, ktol: adaptive Krylov dimension
// (ktol = 0: off).
__global__ void k_reset(Scalars *sc, int keep_status, int kmin, int kmax, double ktol)
{
    if (threadIdx.x == 0) {
        if (!keep_status) sc->status = 0;
        sc->steps_done = 0;
        sc->ticket = 0u;
        sc->kstop = sc->status != 0 ? -1 : 0;
        sc->keff = 0;
        sc->scale = 0.0;
        sc->cabs_k = 0.0;
        sc->beta_k = 0.0;
        sc->sigma = 0.0;
        sc->kmin = kmin;
        sc->kmax = kmax;
        sc->knext = 0;
        sc->ktol = ktol;
    }
}

// End of an asynchronous call: the state after the completed steps is in
// `state` when their number is odd (the steps alternate between the caller's
// psi and the workspace); copy it to psi there, do nothing otherwise.
__global__ __launch_bounds__(kBlock) void k_finish_copy(const Scalars *sc, const double2 *__restrict__ state,
                                                        double2 *__restrict__ psi, size_t n)
{
    if ((sc->steps_done & 1) == 0) return;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        psi[i] = state[i];
}

// FIFO depths (rows of loads in flight per wave).  Dominant sweep at
// 4096^2, four waves per CU: complex64 FIFO 2 / 4 rows 150.6 / 148.9 us,
// complex128 336.8 / 339.5 us.
#ifndef DL_PF_MIXED
#define DL_PF_MIXED 4
#endif
#ifndef DL_PF_FP64
#define DL_PF_FP64 2
#endif
#ifndef DL_WPE_MIXED
#define DL_WPE_MIXED 1
#endif
constexpr int kPfFirst = 4;
constexpr int kPfMixed = DL_PF_MIXED;
constexpr int kPfFp64 = DL_PF_FP64;
// occupancy hint of the complex64 sweeps (1: none).  Three waves per SIMD fit
// them without spills but measured slower than the two the allocator picks.
constexpr int kWpeMixed = DL_WPE_MIXED;

// Load policy of the sweeps per precision (measured on the 4096^2 workload:
// the streaming hint helps the complex64 sweeps and hurts the complex128 ones).
#ifndef DL_LOAD_POL_MIXED
#define DL_LOAD_POL_MIXED kPolStream
#endif
#ifndef DL_LOAD_POL_FP64
#define DL_LOAD_POL_FP64 kPolDefault
#endif
using PlanarM = PlanarT<DL_LOAD_POL_MIXED>;
using PairedM = Paired<float2, DL_LOAD_POL_MIXED>;
using PlanarD = PlanarT<DL_LOAD_POL_FP64>;
using PairedD = Paired<double2, DL_LOAD_POL_FP64>;

template <class K>
int waves_per_cu(K kernel)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, kBlock, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 8;
    }
    return blocks * kWaves;
}


// Kernel families of the recurrence sweep: one launch per grid (single) or
// per batch of packets (batch).
struct SingleRecur {
    template <class V1, class V2, class TO, bool HAS2, int PF, bool PY, int TERMS>
    static constexpr auto get() { return k_recur<V1, V2, TO, HAS2, PF, PY, TERMS>; }
};

// Calls f with the specialisation (periodic y, site terms) of a kernel.
template <template <bool, int> class Pick, class F>
auto dispatch_terms(bool py, int terms, F &&f)
{
    switch ((py ? 4 : 0) | (terms & 3)) {
    case 0: return f(Pick<false, 0>::get());
    case 1: return f(Pick<false, 1>::get());
    case 2: return f(Pick<false, 2>::get());
    case 3: return f(Pick<false, 3>::get());
    case 4: return f(Pick<true, 0>::get());
    case 5: return f(Pick<true, 1>::get());
    case 6: return f(Pick<true, 2>::get());
    default: return f(Pick<true, 3>::get());
    }
}

// The eight specialisations (periodic y, site terms) of one sweep kind.
template <class Fam, class V1, class V2, class TO, bool HAS2, int PF>
struct RecurKind {
    template <bool PY, int TERMS>
    struct Pick {
        static constexpr auto get() { return Fam::template get<V1, V2, TO, HAS2, PF, PY, TERMS>(); }
    };
    template <class F>
    static auto dispatch(bool py, int terms, F &&f) { return dispatch_terms<Pick>(py, terms, f); }
};

template <class Fam, bool M>
using RecurP2 = RecurKind<Fam, std::conditional_t<M, PlanarM, PlanarD>, std::conditional_t<M, PlanarM, PlanarD>,
                          std::conditional_t<M, float2, double2>, false, M ? kPfMixed : kPfFp64>;
template <class Fam, bool M>
using RecurP3 = RecurKind<Fam, std::conditional_t<M, PairedM, PairedD>, std::conditional_t<M, PlanarM, PlanarD>,
                          std::conditional_t<M, float2, double2>, true, M ? kPfMixed : kPfFp64>;
template <class Fam, bool M>
using RecurPn = RecurKind<Fam, std::conditional_t<M, PairedM, PairedD>, std::conditional_t<M, PairedM, PairedD>,
                          std::conditional_t<M, float2, double2>, true, M ? kPfMixed : kPfFp64>;

int op_terms(const Op &op)
{
    return ((op.pot_kind != 0 || op.has_table != 0) ? kTermPot : 0) | (op.bq != 0.0 ? kTermB : 0);
}

template <template <class, bool> class Kind, class Fam, class F>
auto with_kind(bool mixed, bool py, int terms, F &&f)
{
    if (mixed) return Kind<Fam, true>::dispatch(py, terms, f);
    return Kind<Fam, false>::dispatch(py, terms, f);
}

}  // namespace
}  // namespace dl
