// Wavefront (64 lanes) and workgroup reductions and scans, and two-float
// (compensated) arithmetic for the reduced-precision cumulative distribution.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

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

// ---------------------------------------------------------------------------
// Cross-lane moves through DPP (data-parallel primitives of the VALU; no LDS
// traffic).  Control codes of gfx9: row_shr:n = 0x110 + n (shift within a
// row of 16 lanes), row_bcast:15 = 0x142 (lane 15 of each row to the whole
// next row), row_bcast:31 = 0x143 (lane 31 to rows 2 and 3), wave_shr:1 =
// 0x138 (whole-wave shift by one lane).  Lanes whose source is outside the
// pattern, or whose row is masked off, receive `fill`.

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_i(int v, int fill)
{
    return __builtin_amdgcn_update_dpp(fill, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v, float fill)
{
    return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(v), __float_as_int(fill)));
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v, double fill)
{
    const int lo = dpp_i<CTRL, ROW_MASK>(__double2loint(v), __double2loint(fill));
    const int hi = dpp_i<CTRL, ROW_MASK>(__double2hiint(v), __double2hiint(fill));
    return __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp(int v, int fill) { return dpp_i<CTRL, ROW_MASK>(v, fill); }
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v, float fill) { return dpp_f<CTRL, ROW_MASK>(v, fill); }
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp(double v, double fill) { return dpp_d<CTRL, ROW_MASK>(v, fill); }

struct OpAdd {
    template <typename T> __device__ static T apply(T a, T b) { return a + b; }
    template <typename T> __device__ static T identity() { return T(0); }
};
struct OpMax {
    template <typename T> __device__ static T apply(T a, T b) { return a > b ? a : b; }
    template <typename T> __device__ static T identity()
    {
        if constexpr (std::is_same<T, int>::value) return INT32_MIN;
        else return -INFINITY;
    }
};
struct OpMin {
    template <typename T> __device__ static T apply(T a, T b) { return a < b ? a : b; }
    template <typename T> __device__ static T identity()
    {
        if constexpr (std::is_same<T, int>::value) return INT32_MAX;
        else return INFINITY;
    }
};

// Inclusive scan over the 64 lanes (Hillis-Steele inside each row of 16,
// then the row totals carried by the two row broadcasts).  Every lane must
// be active.  For a sum this is the same association on every call, so the
// result is reproducible bit for bit.
template <typename Op, typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const T id = Op::template identity<T>();
    v = Op::apply(v, dpp<0x111>(v, id));
    v = Op::apply(v, dpp<0x112>(v, id));
    v = Op::apply(v, dpp<0x114>(v, id));
    v = Op::apply(v, dpp<0x118>(v, id));
    v = Op::apply(v, dpp<0x142, 0xA>(v, id));
    v = Op::apply(v, dpp<0x143, 0xC>(v, id));
    return v;
}

// Value of lane 63 (uniform result).
__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
__device__ __forceinline__ double lane63(double v)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Previous lane's value (lane 0 receives `fill`).
template <typename T>
__device__ __forceinline__ T wave_shift_up1(T v, T fill)
{
    return dpp<0x138>(v, fill);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) { return lane63(wave_incl_scan<OpMax>(v)); }
template <typename T>
__device__ __forceinline__ T wave_min(T v) { return lane63(wave_incl_scan<OpMin>(v)); }
template <typename T>
__device__ __forceinline__ T wave_sum(T v) { return lane63(wave_incl_scan<OpAdd>(v)); }

// Inclusive prefix sum / maximum over the wave.
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v, int /*lane*/) { return wave_incl_scan<OpAdd>(v); }
template <typename T>
__device__ __forceinline__ T wave_incl_max(T v, int /*lane*/) { return wave_incl_scan<OpMax>(v); }

// Inclusive prefix maximum of non-negative floats.  Such floats order as
// their bit patterns do as signed integers, so the scan runs on the integers,
// whose DPP maximum steps the compiler folds into single instructions.  Equal,
// bit for bit, to the float scan on non-negative values.
__device__ __forceinline__ float wave_incl_max_nonneg(float v)
{
    return __int_as_float(wave_incl_scan<OpMax>(__float_as_int(v)));
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
