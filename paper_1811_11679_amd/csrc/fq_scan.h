// Wavefront and block primitives shared by the kernel translation units:
// decoupled look-back (Merrill & Garland 2016) status words and the look-back
// itself, wave reductions, block-wide exclusive scans (gfx950: 64-wide
// wavefronts, blocks of up to 1024 threads) and the exact fixed-point
// accumulation of FP64 terms used by the estimators.
#pragma once

#include "fq_kernels.h"

namespace fq {

// ---------------------------------------------------------------------------
// decoupled look-back status words: [epoch:24 | flag:2 | value:38]
// ---------------------------------------------------------------------------
constexpr unsigned long long ST_AGG = 1ull, ST_INC = 2ull;
constexpr int ST_VBITS = 38;
constexpr unsigned long long ST_VMASK = (1ull << ST_VBITS) - 1;

__device__ __forceinline__ uint32_t epoch_of(uint32_t t, uint32_t use) { return ((t << 4) | use) & 0xFFFFFFu; }

__device__ __forceinline__ unsigned long long st_pack(uint32_t epoch, unsigned long long flag, long long v)
{
    return ((unsigned long long)epoch << 40) | (flag << ST_VBITS) | ((unsigned long long)v & ST_VMASK);
}

__device__ __forceinline__ void st_store(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long st_load(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// The two halves of a look-back, for a tile that can publish its aggregate
// well before it needs its prefix (other work in between shortens the waits
// of the tiles after it): lookback_publish by one lane, then lookback_wait by
// one whole wavefront with the same aggregate.
static __device__ void lookback_publish(unsigned long long *st, long long tile, uint32_t epoch, long long agg)
{
    st_store(st + tile, st_pack(epoch, tile == 0 ? ST_INC : ST_AGG, agg));
}

static __device__ long long lookback_wait(unsigned long long *st, long long tile, uint32_t epoch, long long agg)
{
    const int lane = lane_id();
    if (tile == 0) return 0;
    long long excl = 0;
    long long j = tile - 1;
    for (;;) {
        const long long idx = j - lane;
        unsigned long long sw = 0;
        if (idx >= 0) sw = st_load(st + idx);
        const uint32_t e = (uint32_t)(sw >> 40);
        const unsigned long long f = (sw >> ST_VBITS) & 3ull;
        const bool valid = idx >= 0 && e == epoch && f != 0;
        const uint64_t inc = __ballot(valid && f == ST_INC);
        const uint64_t bad = __ballot(idx >= 0 && !valid);
        // lanes that count: up to and including the nearest inclusive prefix
        const uint64_t need = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;
        if (bad & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const long long v = (((need >> lane) & 1ull) && valid) ? (long long)(sw & ST_VMASK) : 0;
        excl += wave_sum<long long>(v);
        if (inc) break;
        j -= 64;
    }
    if (lane == 0) st_store(st + tile, st_pack(epoch, ST_INC, excl + agg));
    return excl;
}

// Decoupled look-back, run by one whole wavefront: publishes this tile's
// aggregate, then inspects the 64 preceding tiles at a time until it meets an
// inclusive prefix, publishes its own inclusive prefix and returns the
// exclusive one (to every lane). It waits only on tiles with smaller tickets,
// which are resident and never wait on this tile, so every wait ends.
static __device__ long long lookback(unsigned long long *st, long long tile, uint32_t epoch, long long agg)
{
    if (lane_id() == 0) lookback_publish(st, tile, epoch, agg);
    return lookback_wait(st, tile, epoch, agg);
}

// exclusive block scan of one value per thread (blockDim = 256)
template <typename T>
__device__ T block_excl_scan(T v, T &total, T *lds /* 8 entries */)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    T base = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wid) base += lds[w];
        tot += lds[w];
    }
    total = tot;
    __syncthreads();
    return base + x - v;
}

// two exclusive block scans at once (one pair of barriers)
static __device__ void block_excl_scan2(long long v, long long u, long long &ex_v, long long &ex_u, long long &tot_v,
                                 long long &tot_u, long long *lds /* 16 entries */)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    long long x = v, y = u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long a = __shfl_up(x, o, 64), b = __shfl_up(y, o, 64);
        if (lane >= o) {
            x += a;
            y += b;
        }
    }
    if (lane == 63) {
        lds[wid] = x;
        lds[8 + wid] = y;
    }
    __syncthreads();
    long long bv = 0, bu = 0, tv = 0, tu = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wid) {
            bv += lds[w];
            bu += lds[8 + w];
        }
        tv += lds[w];
        tu += lds[8 + w];
    }
    tot_v = tv;
    tot_u = tu;
    ex_v = bv + x - v;
    ex_u = bu + y - u;
    __syncthreads();
}

// Exact fixed-point accumulation of one FP64 term: |x| 2^64 truncated toward
// zero, split into four 32-bit limbs added with the sign of x (int64 limb
// sums are exact and order independent).
__device__ __forceinline__ void add_limbs4(long long &a0, long long &a1, long long &a2, long long &a3, double x)
{
    if (x == 0.0) return;
    const bool neg = x < 0.0;
    const uint64_t bits = (uint64_t)__double_as_longlong(fabs(x));
    const int ex = (int)((bits >> 52) & 0x7FF);
    const uint64_t mant = (bits & ((1ull << 52) - 1)) | (ex ? (1ull << 52) : 0ull);
    const int sh = (ex ? ex : 1) - 1075 + 64;  // |x| * 2^64 = mant * 2^sh
    uint64_t lo = 0, hi = 0;
    if (sh >= 64) {
        hi = mant << (sh - 64);
    } else if (sh > 0) {
        lo = mant << sh;
        hi = mant >> (64 - sh);
    } else if (sh == 0) {
        lo = mant;
    } else if (sh > -64) {
        lo = mant >> (-sh);
    }
    const long long l0 = (long long)(lo & 0xFFFFFFFFull), l1 = (long long)(lo >> 32);
    const long long l2 = (long long)(hi & 0xFFFFFFFFull), l3 = (long long)(hi >> 32);
    a0 += neg ? -l0 : l0;
    a1 += neg ? -l1 : l1;
    a2 += neg ? -l2 : l2;
    a3 += neg ? -l3 : l3;
}

}  // namespace fq
