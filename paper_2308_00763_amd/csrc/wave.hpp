// Wavefront (64 lanes) and workgroup reductions and scans, and two-float
// (compensated) arithmetic for the reduced-precision cumulative distribution.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pf {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask)
{
    return __shfl_xor(v, mask, kWave);
}

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d)
{
    return __shfl_up(v, (unsigned)d, kWave);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const T o = shfl_xor(v, m);
        v = o > v ? o : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const T o = shfl_xor(v, m);
        v = o < v ? o : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
    return v;
}

// Inclusive prefix sum over the wave (Hillis-Steele).
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T o = shfl_up(v, d);
        if (lane >= d) v += o;
    }
    return v;
}

// Inclusive prefix maximum over the wave.
template <typename T>
__device__ __forceinline__ T wave_incl_max(T v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T o = shfl_up(v, d);
        if (lane >= d && o > v) v = o;
    }
    return v;
}

// Workgroup-wide reductions for a block of NW waves.  `red` is LDS scratch of
// at least NW elements; every thread receives the result.
template <int NW, typename T>
__device__ __forceinline__ T block_max(T v, T* red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = red[i] > r ? red[i] : r;
    return r;
}

template <int NW, typename T>
__device__ __forceinline__ T block_min(T v, T* red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_min(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = red[i] < r ? red[i] : r;
    return r;
}

template <int NW, typename T>
__device__ __forceinline__ T block_sum(T v, T* red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r += red[i];
    return r;
}

// Inclusive prefix sum of one value per thread across the workgroup that is
// monotone for non-negative inputs, whatever the rounding: inside a wave a
// prefix maximum follows the Hillis-Steele sum (maximum is exact and
// associative); across waves the carried offset of wave w is computed as the
// left-to-right sum of the wave totals, which is bit-identical to the last
// result of wave w - 1, so adding a non-negative value to it never goes
// below.  `red` is LDS scratch of at least NW elements.
template <int NW, typename T>
__device__ __forceinline__ T block_incl_sum_monotone(T v, T* red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    T s = wave_incl_sum(v, lane);
    s = wave_incl_max(s, lane);
    __syncthreads();
    if (lane == kWave - 1) red[w] = s;
    __syncthreads();
    if (w == 0) return s;
    T off = red[0];
    for (int i = 1; i < w; ++i) off = off + red[i];
    return off + s;
}

// ---------------------------------------------------------------------------
// Two-float numbers (hi + lo, |lo| <= ulp(hi)/2): error-free transformations
// of Knuth (TwoSum) and Dekker (FastTwoSum, TwoProduct via fused multiply-add).

struct ff {
    float hi, lo;
};

__device__ __forceinline__ ff two_sum(float a, float b)
{
    const float s = a + b;
    const float bb = s - a;
    const float err = (a - (s - bb)) + (b - bb);
    return ff{s, err};
}

__device__ __forceinline__ ff fast_two_sum(float a, float b)
{
    const float s = a + b;
    const float err = b - (s - a);
    return ff{s, err};
}

__device__ __forceinline__ ff two_prod(float a, float b)
{
    const float p = a * b;
    const float err = __builtin_fmaf(a, b, -p);
    return ff{p, err};
}

__device__ __forceinline__ ff ff_add(ff a, ff b)
{
    ff s = two_sum(a.hi, b.hi);
    ff t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ff ff_add_f(ff a, float b)
{
    ff s = two_sum(a.hi, b);
    s.lo += a.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ff ff_mul(ff a, ff b)
{
    ff p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_mul_f(ff a, float b)
{
    ff p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_div(ff a, ff b)
{
    const float q1 = a.hi / b.hi;
    const ff r = ff_add(a, ff_mul_f(b, -q1));
    const float q2 = r.hi / b.hi;
    return fast_two_sum(q1, q2);
}

__device__ __forceinline__ bool ff_lt(ff a, ff b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

__device__ __forceinline__ ff ff_min(ff a, ff b) { return ff_lt(b, a) ? b : a; }
__device__ __forceinline__ ff ff_max(ff a, ff b) { return ff_lt(a, b) ? b : a; }

// floor of a normalised two-float number, as a 64-bit integer.
__device__ __forceinline__ int64_t ff_floor(ff a)
{
    const float fh = floorf(a.hi);
    int64_t r = (int64_t)fh;
    if (fh == a.hi) {
        // hi is an integer: the fraction is in lo
        r += (int64_t)floorf(a.lo);
    }
    return r;
}

}  // namespace pf
