// Batched launches of the propagator kernels: one launch per Lanczos
// iteration (and one for the small exponentials, one for the recombination)
// over all packets of a batch.  Each workgroup reads its packet and its
// waves' tiles from device tables; the per-wave marches, the small
// exponential and the recombination are the same device code as the
// single-grid kernels (sweeps.h).  A packet's workgroups form a contiguous
// segment of the grid, and its reductions are folded by the segment's last
// workgroup in fixed order, so every packet's result is reproducible and
// independent of the other packets.
#include <hip/hip_runtime.h>

#include "sweeps.h"

namespace dl {
namespace {

__device__ __forceinline__ WaveTask batch_wave_task(const BatchArgs &b, int entry)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const BatchTask tk = b.tasks[(size_t)entry * kWaves + wave];
    WaveTask w;
    w.strip = tk.strip;
    w.y0 = tk.y0;
    w.y1 = tk.y1;
    w.active = tk.y0 < tk.y1;
    return w;
}

// Resident loop of the batched sweeps: workgroup g runs the block entries
// wg_first[g] .. wg_first[g + 1] - 1, a list the host balanced over the
// resident workgroups (longest first, each to the least loaded).  The entry
// index is a scalar induction variable: the loop and every branch around the
// barriers in `body` stay wave-uniform.
template <class Body>
__device__ __forceinline__ void resident_loop(const BatchArgs &b, Body body)
{
    const int e0 = b.wg_first[blockIdx.x], e1 = b.wg_first[blockIdx.x + 1];
    for (int e = e0; e < e1; ++e) body(e);
}

template <int PF, bool PY, int TERMS>
__global__ __launch_bounds__(kBlock) void k_first_batch(BatchArgs b)
{
    resident_loop(b, [&](int entry) {
        const BatchBlock bb = b.blocks[entry];
        const BatchPacket &pk = b.pk[bb.packet];
        Scalars *sc = pk.sc;
        if (sc->status != 0) return;
        const WaveTask wt = batch_wave_task(b, entry);
        const double2 *in = b.parity ? pk.state : pk.psi;
        double acc[3] = {0.0, 0.0, 0.0};
        first_body<PF, PY, TERMS>(pk.op, pk.tiles[1], wt, in, pk.fields + 2 * b.step, acc);
        double tot[3];
        if (!seg_reduce(acc, b.partials + (size_t)bb.first * kPartialStride, &sc->ticket, bb.nblk, bb.local, tot))
            return;
        if (threadIdx.x == 0) first_tail(tot, pk.alpha, pk.gamma, sc, b.m, 1);
    });
}

template <class V1, class V2, class TO, bool HAS2, int PF, bool PY, int TERMS>
__global__ __launch_bounds__(kBlock) void k_recur_batch(BatchArgs b)
{
    resident_loop(b, [&](int entry) {
        const BatchBlock bb = b.blocks[entry];
        const BatchPacket &pk = b.pk[bb.packet];
        PassArgs a;
        a.op = pk.op;
        a.t = pk.tiles[0];
        const int p = b.pass;
        const double2 *in = b.parity ? pk.state : pk.psi;
        auto bvec = [&](int j) { return static_cast<void *>(pk.basis + (size_t)(j - 2) * pk.vstride); };
        a.u1 = (p - 1 == 1) ? static_cast<const void *>(in) : bvec(p - 1);
        a.u2 = (p - 2 == 1) ? static_cast<const void *>(in) : (p - 2 >= 2 ? bvec(p - 2) : nullptr);
        a.uo = bvec(p);
        a.field = pk.fields + 2 * b.step;
        a.alpha = pk.alpha;
        a.gamma = pk.gamma;
        a.sc = pk.sc;
        a.partials = b.partials + (size_t)bb.first * kPartialStride;
        a.pass = p;
        a.m = b.m;
        a.replay = 0;
        if (a.sc->kstop < p) return;
        const WaveTask wt = batch_wave_task(b, entry);
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        recur_body<V1, V2, TO, HAS2, PF, PY, TERMS>(a, wt, a.gamma[p - 1], a.alpha[p - 1], acc);
        double tot[5];
        if (!seg_reduce(acc, a.partials, &a.sc->ticket, bb.nblk, bb.local, tot)) return;
        if (threadIdx.x == 0) recur_tail(a, tot);
    });
}

// one wave per packet
__global__ __launch_bounds__(64) void k_tridiag_batch(BatchArgs b)
{
    const BatchPacket &pk = b.pk[blockIdx.x];
    tridiag_body(pk.alpha, pk.gamma, pk.sc, pk.stats + b.step, pk.reps, pk.rabs);
}

template <class TB, int S, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_combine_batch(BatchArgs b)
{
    const BatchBlock bb = b.blocks[blockIdx.x];
    const BatchPacket &pk = b.pk[bb.packet];
    if (pk.sc->status != 0) return;
    CombArgs a{};
    a.psi = b.parity ? pk.state : pk.psi;
    a.basis = pk.basis;
    a.vec_bytes = pk.vstride;
    a.sites = pk.sites;
    a.out = b.parity ? pk.psi : pk.state;
    a.sc = pk.sc;
    a.partials = b.partials + (size_t)bb.first * kPartialStride;
    a.stat = pk.stats + b.step;
    double nrm = 0.0;
    combine_body<TB, S>(a, bb.local, bb.nblk, nrm);
    double accv[1] = {nrm}, tot[1];
    if (!seg_reduce(accv, a.partials, &a.sc->ticket, bb.nblk, bb.local, tot)) return;
    if (threadIdx.x == 0) combine_tail(a, tot);
}

// Scalars of every packet to the start-of-call state (one thread per packet).
__global__ void k_reset_batch(const BatchPacket *pk, int n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    Scalars *sc = pk[i].sc;
    sc->status = 0;
    sc->steps_done = 0;
    sc->ticket = 0u;
    sc->kstop = 0;
    sc->keff = 0;
    sc->scale = 0.0;
    sc->cabs_k = 0.0;
    sc->beta_k = 0.0;
    sc->sigma = 0.0;
    sc->kmin = sc->kmax = sc->knext = 0;
    sc->ktol = 0.0;
}

struct BatchRecur {
    template <class V1, class V2, class TO, bool HAS2, int PF, bool PY, int TERMS>
    static constexpr auto get() { return k_recur_batch<V1, V2, TO, HAS2, PF, PY, TERMS>; }
};

template <bool PY, int TERMS>
struct PickFirstBatch {
    static constexpr auto get() { return k_first_batch<kPfFirst, PY, TERMS>; }
};

}  // namespace

void launch_first_batch(const BatchArgs &b, int nblocks, bool py, int terms, hipStream_t st)
{
    dispatch_terms<PickFirstBatch>(py, terms, [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(kBlock), 0, st, b);
        return 0;
    });
}

void launch_recur_batch(const BatchArgs &b, int nblocks, bool mixed, bool py, int terms, hipStream_t st)
{
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(kBlock), 0, st, b);
        return 0;
    };
    if (b.pass == 2)
        with_kind<RecurP2, BatchRecur>(mixed, py, terms, go);
    else if (b.pass == 3)
        with_kind<RecurP3, BatchRecur>(mixed, py, terms, go);
    else
        with_kind<RecurPn, BatchRecur>(mixed, py, terms, go);
}

void launch_tridiag_batch(const BatchArgs &b, int npackets, hipStream_t st)
{
    hipLaunchKernelGGL(k_tridiag_batch, dim3(npackets), dim3(64), 0, st, b);
}

void launch_combine_batch(const BatchArgs &b, int nblocks, bool mixed, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL((k_combine_batch<float2, kCombMixedWide, kCombWpeMixedWide>), dim3(nblocks), dim3(kBlock),
                           0, st, b);
    else
        hipLaunchKernelGGL((k_combine_batch<double2, kCombFp64, kCombWpeFp64>), dim3(nblocks), dim3(kBlock), 0,
                           st, b);
}

void launch_reset_batch(const BatchPacket *pk, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_batch, dim3((n + 63) / 64), dim3(64), 0, st, pk, n);
}

// batches use the wide complex64 form (measured on the 256-packet workload)
int combine_tile_sites(bool mixed) { return kBlock * (mixed ? kCombMixedWide : kCombFp64); }

}  // namespace dl
