// Single-grid launches of the sweep kernels (device code in sweeps.h) and
// the launch-shape queries of the host runtime.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sweeps.h"

namespace dl {

namespace {
template <bool PY, int TERMS>
struct PickFirst {
    static constexpr auto get() { return k_first<kPfFirst, PY, TERMS>; }
};
}  // namespace

int sweep_waves_per_cu(int which, bool mixed, bool py, int terms)
{
    auto occ = [](auto kernel) { return waves_per_cu(kernel); };
    switch (which) {
    case 0: return dispatch_terms<PickFirst>(py, terms, occ);
    case 1: return with_kind<RecurPn, SingleRecur>(mixed, py, terms, occ);
    case 2: return with_kind<RecurP2, SingleRecur>(mixed, py, terms, occ);
    case 3: return with_kind<RecurP3, SingleRecur>(mixed, py, terms, occ);
    default: return waves_per_cu(k_apply);
    }
}

int sweep_terms(const Op &op) { return op_terms(op); }

bool combine_wide(size_t sites, bool mixed, int cus)
{
    // complex64: the wide form from one wide tile per compute unit; FP64: the
    // wide form (8 sites per thread) from four wide tiles per compute unit,
    // below that two sites per thread, so that a small grid still spreads
    // over every compute unit
    return mixed ? sites >= (size_t)cus * kBlock * kCombMixedWide : sites >= (size_t)4 * cus * kBlock * kCombFp64;
}

int combine_grid(size_t sites, bool mixed, int cus, bool wide)
{
    // a fixed number of workgroups per compute unit (four measured best for
    // the tiled stream), never more than there are tiles
    const int S = mixed ? (wide ? kCombMixedWide : kCombMixed) : (wide ? kCombFp64 : kCombFp64Narrow);
    const size_t tile = (size_t)kBlock * S;
    size_t nb = std::min<size_t>((size_t)DL_COMB_BLOCKS_PER_CU * cus, (sites + tile - 1) / tile);
    nb = std::max<size_t>(nb, 1);
    return (int)std::min<size_t>(nb, kMaxBlocks);
}

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
                  double *alpha, double *gamma, Scalars *sc, double *partials, int m, int shift,
                  hipStream_t st)
{
    dispatch_terms<PickFirst>(op.bcy != 0, op_terms(op), [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(t.nblocks), dim3(kBlock), 0, st, op, t, psi, field, alpha, gamma, sc,
                           partials, m, shift);
        return 0;
    });
}

void launch_recur(const PassArgs &a, bool mixed, hipStream_t st)
{
    const dim3 g(a.t.nblocks), b(kBlock);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, g, b, 0, st, a);
        return 0;
    };
    const bool py = a.op.bcy != 0;
    const int terms = op_terms(a.op);
    if (a.pass == 2)
        with_kind<RecurP2, SingleRecur>(mixed, py, terms, go);
    else if (a.pass == 3)
        with_kind<RecurP3, SingleRecur>(mixed, py, terms, go);
    else
        with_kind<RecurPn, SingleRecur>(mixed, py, terms, go);
}

void launch_tridiag(double *alpha, double *gamma, Scalars *sc, StepStat *stat, double reps, double rabs,
                    const TailFold &fold, hipStream_t st)
{
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(64), 0, st, alpha, gamma, sc, stat, reps, rabs, fold);
}

void launch_fold_tail(double *alpha, double *gamma, Scalars *sc, const TailFold &fold, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold_tail, dim3(1), dim3(64), 0, st, alpha, gamma, sc, fold);
}

void launch_combine(const CombArgs &a, bool mixed, bool wide, int nblocks, hipStream_t st)
{
    if (mixed && wide)
        hipLaunchKernelGGL((k_combine<float2, kCombMixedWide, kCombWpeMixedWide>), dim3(nblocks), dim3(kBlock), 0,
                           st, a);
    else if (mixed)
        hipLaunchKernelGGL((k_combine<float2, kCombMixed, kCombWpeMixed>), dim3(nblocks), dim3(kBlock), 0, st, a);
    else if (wide)
        hipLaunchKernelGGL((k_combine<double2, kCombFp64, kCombWpeFp64>), dim3(nblocks), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_combine<double2, kCombFp64Narrow, kCombWpeFp64Narrow>), dim3(nblocks), dim3(kBlock), 0,
                           st, a);
}

void launch_accum(const AccumArgs &a, bool mixed, int nblocks, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL((k_accum<float2, kCombMixed>), dim3(nblocks), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_accum<double2, kCombFp64>), dim3(nblocks), dim3(kBlock), 0, st, a);
}

void launch_apply(const Op &op, const Tiles &t, const double2 *x, double2 *y, double gxh,
                  double gyh, hipStream_t st)
{
    hipLaunchKernelGGL(k_apply, dim3(t.nblocks), dim3(kBlock), 0, st, op, t, x, y, gxh, gyh);
}

void launch_reset(Scalars *sc, hipStream_t st) { launch_reset_call(sc, 0, 0, 0, 0.0, st); }

void launch_reset_call(Scalars *sc, int keep_status, int kmin, int kmax, double ktol, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, sc, keep_status, kmin, kmax, ktol);
}

void launch_finish_copy(const Scalars *sc, const double2 *state, double2 *psi, size_t n, int cus, hipStream_t st)
{
    const size_t blocks = std::min<size_t>((size_t)4 * cus, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_finish_copy, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(kBlock), 0, st, sc, state,
                       psi, n);
}

}  // namespace dl
