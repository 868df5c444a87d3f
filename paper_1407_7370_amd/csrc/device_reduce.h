// Deterministic FP64 reductions shared by the kernels of the library:
// a butterfly inside a wave, then per-workgroup partials folded in fixed order
// by the last workgroup to finish.  Internal header (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include "dl_internal.h"

namespace dl {
namespace {

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV])
{
    // Butterfly: after each stage partner lanes hold bitwise equal sums.
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], s, 64);
}

// This workgroup's partial: the wave sums, then the waves in order (thread 0
// ends with the partial in s).
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double (&red)[kWaves][NV], double (&s)[NV])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    wave_sum(v);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[w][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = red[0][k];
        for (int i = 1; i < kWaves; ++i) a += red[i][k];
        s[k] = a;
    }
}

// The totals of partials[0 .. nblk) folded by the whole workgroup in a fixed
// order (thread t sums partials t, t + kBlock, ...; then the wave sums and
// the waves in order); every thread ends with them.  Device-scope loads: the
// partials may come from other XCDs within this kernel.
template <int NV>
__device__ __forceinline__ void fold_partials(const double *partials, int nblk, double (&red)[kWaves][NV],
                                              double (&tot)[NV])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            s[k] += __hip_atomic_load(&partials[(size_t)b * kPartialStride + k], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
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
}

// The same fold by a single wave (each of the kWaves thread groups of the
// workgroup fold in turn), bit for bit the totals of fold_partials.  With at
// most kBlock partials every group's loads are issued before any sum waits.
template <int NV>
__device__ __forceinline__ void fold_partials_wave(const double *partials, int nblk, double (&tot)[NV])
{
    const int lane = threadIdx.x & 63;
    double s[kWaves][NV];
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[w][k] = 0.0;
    if (nblk <= kBlock) {
        double v[kWaves][NV];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const int b = w * 64 + lane;
#pragma unroll
            for (int k = 0; k < NV; ++k) v[w][k] = b < nblk ? partials[(size_t)b * kPartialStride + k] : 0.0;
        }
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (w * 64 + lane < nblk) s[w][k] += v[w][k];
    } else {
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            for (int b = w * 64 + lane; b < nblk; b += kBlock)
#pragma unroll
                for (int k = 0; k < NV; ++k) s[w][k] += partials[(size_t)b * kPartialStride + k];
    }
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wave_sum(s[w]);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = s[0][k];
        for (int w = 1; w < kWaves; ++w) a += s[w][k];
        tot[k] = a;
    }
}

// Fold the per-lane sums of a segment of `nblk` workgroups (this one is number
// `blk` of the segment) in a fixed order: per-workgroup partials in
// partials[0 .. nblk), a ticket counting the finished workgroups.  Returns true
// in the last workgroup of the segment to finish, where every thread then
// holds the totals; that workgroup also resets the ticket.
//
// Visibility of the partials without a device-wide fence: they are written
// with device-scope atomic stores, which the compiler issues as writes to the
// device's coherence point (not left dirty in this XCD's L2); the wait for
// their completion orders them before the ticket increment; the last
// workgroup reads them with device-scope atomic loads, which do not take a
// line that another XCD's L2 may hold stale.  This is the release/acquire
// pair restricted to the partials.  A full __threadfence() here writes back
// and invalidates the whole L2 of the workgroup's XCD, which the workgroups
// still streaming rows on that XCD then pay for (measured on the 4096^2
// mixed sweep: 147.7 -> 138.5 us; a batched step 6.7 -> 5.6 ms).
template <int NV>
__device__ bool seg_reduce(double (&v)[NV], double *partials, unsigned int *ticket, int nblk, int blk,
                           double (&tot)[NV])
{
    static_assert(NV <= kPartialStride, "partial table stride");
    __shared__ double red[kWaves][NV];
    __shared__ int last;
    double s[NV];
    block_partial(v, red, s);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(&partials[(size_t)blk * kPartialStride + k], s[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        // the partials' stores complete before the ticket is taken
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const unsigned int t = atomicAdd(ticket, 1u);
        last = (t == (unsigned int)nblk - 1u) ? 1 : 0;
    }
    __syncthreads();
    // `last` is the same in every thread; a scalar copy keeps the branch (and
    // the barriers of callers that loop over this) wave-uniform
    if (!__builtin_amdgcn_readfirstlane(last)) return false;
    fold_partials(partials, nblk, red, tot);
    if (threadIdx.x == 0) *ticket = 0u;
    return true;
}

// This workgroup's partial stored for a fold by the next kernel (no ticket).
template <int NV>
__device__ __forceinline__ void store_partial(double (&v)[NV], double *partials, int blk)
{
    static_assert(NV <= kPartialStride, "partial table stride");
    __shared__ double red[kWaves][NV];
    double s[NV];
    block_partial(v, red, s);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[(size_t)blk * kPartialStride + k] = s[k];
}

// The whole grid as one segment.
template <int NV>
__device__ __forceinline__ bool grid_reduce(double (&v)[NV], double *partials, unsigned int *ticket,
                                            double (&tot)[NV])
{
    return seg_reduce(v, partials, ticket, (int)gridDim.x, (int)blockIdx.x, tot);
}

}  // namespace
}  // namespace dl
