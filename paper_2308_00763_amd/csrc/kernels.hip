// HIP kernels of the per-frame SIR step for gfx950 (CDNA4, wave64).
//
// One step (paper Sec. 4: propagation, likelihood, maximum, weighting,
// normalizing, resampling) runs as three launches on one stream:
//
//   pass A   one workgroup per tile of 1024 particles.  Draws the normals,
//            propagates (Eq. (1)-(2)), stages the row-prefix table of the
//            frame window the tile's particles look at in LDS, sums the disk
//            of Eq. (3) per particle, takes the tile maximum, forms the
//            tile's weights exp(L - m_tile) and their monotone prefix sum (the
//            tile-local cumulative distribution, stored) and the tile's
//            estimate partial sums.
//   combine  one workgroup: global maximum M, factors exp(m_tile - M), the
//            carried cumulative offset of every tile, normaliser Z, estimate,
//            resampling offset u0, each tile's end slot and, in the reduced
//            modes, the origin of the next propagation.
//   pass C   systematic resampling: the particles' end slots
//            e_i = #{j : (j + u0)/N <= C_i}, each particle's first slot marked,
//            a maximum scan over the slots giving every slot its ancestor
//            (the same work whatever the weights), and the gather of the
//            ancestors' propagated positions.
//
// The maximum and weighting are fused into pass A and the cumulative
// distribution is evaluated on the fly in pass C, so the six kernels of the
// paper become three, two of them wide.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "philox.hpp"
#include "pf_internal.hpp"
#include "wave.hpp"

namespace pf {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef double double2_t __attribute__((ext_vector_type(2)));

// Global-memory view of a pointer.  The batched kernels read their filters'
// pointers from memory, where the compiler cannot tell global memory from
// LDS; it then emits generic (flat) accesses, which also count against the
// LDS wait counter, so every LDS wait in a kernel would wait for them too (a
// prefetch would not stay in flight).  Every pointer the kernels take points
// to device memory.
template <typename T>
using gbl_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gbl_t<T>* gbl(T* p)
{
    return (gbl_t<T>*)p;
}

// The bulk outputs that the next kernel reads (pass A's propagated positions
// and tile prefix sums, pass C's resampled state) of a single filter that is
// not FP64 and has at most kWtMaxTiles tiles (StepArgs::wt) are stored at
// device scope: such stores are written through the XCD's L2, so the release
// that ends the kernel finds none of them dirty there to write back, and the
// next kernel, on any XCD, reads them from memory as it would in any case.
// Each store covers whole lines across the wave (one 8- or 16-byte store per
// lane).  That pays where the kernels are short (2^20 FP16 21.0 -> 19.1 us per
// step, FP32 23.2 -> 21.5 us, 2^21 -10 %, 2^23 -2 %) and is even or costs
// where they are long or the stores wide (2^24 FP16 even, the 4096-stream
// batch +20 %, FP64 at 2^20 +53 %), so the kernels that use it (WT) are
// separate instantiations, launched for such filters stepped alone at the
// default sizes.
template <bool WT, typename T>
__device__ __forceinline__ void put(gbl_t<T>* p, const T& v)
{
    static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) % 8 == 0, "store width");
    if constexpr (!WT) {
        *p = v;
    } else if constexpr (sizeof(T) == 2) {
        uint16_t b;
        __builtin_memcpy(&b, &v, 2);
        __hip_atomic_store(reinterpret_cast<gbl_t<uint16_t>*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if constexpr (sizeof(T) == 4) {
        uint32_t b;
        __builtin_memcpy(&b, &v, 4);
        __hip_atomic_store(reinterpret_cast<gbl_t<uint32_t>*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
        for (int i = 0; i < (int)(sizeof(T) / 8); ++i) {
            uint64_t b;
            __builtin_memcpy(&b, reinterpret_cast<const char*>(&v) + 8 * i, 8);
            __hip_atomic_store(reinterpret_cast<gbl_t<uint64_t>*>(p) + i, b, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// 16 bytes per lane written through the L2 (the atomic stores above are at
// most 8 bytes, and two 8-byte stores per lane would each leave every other
// 8 bytes of a line to a later store).  A store of more than 8 bytes reads its
// data registers after it issues, and the next instruction must not rewrite
// them before: the compiler keeps that distance for the stores it emits, but
// cannot see into this one, so the wait states follow it here.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void put16_wt(gbl_t<u32x4_t>* p, u32x4_t v)
{
    __asm__ volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" ::"v"(p), "v"(v) : "memory");
}
// Tile records through such pointers, member by member (a structure's
// implicit copy does not bind to global-memory references).
__device__ __forceinline__ TileRec64 load_rec(const gbl_t<const TileRec64>* p)
{
    return TileRec64{p->m, p->s, p->sx, p->sy};
}
__device__ __forceinline__ TileRec32 load_rec(const gbl_t<const TileRec32>* p)
{
    return TileRec32{p->smax, p->s, p->sx, p->sy};
}
template <typename Rec>
__device__ __forceinline__ void store_rec(gbl_t<Rec>* p, const Rec& r)
{
    if constexpr (sizeof(Rec) == sizeof(TileRec64)) p->m = r.m; else p->smax = r.smax;
    p->s = r.s;
    p->sx = r.sx;
    p->sy = r.sy;
}

// ---------------------------------------------------------------------------
// Disk sums through a row-prefix table.  The disk dx^2 + dy^2 < r^2 is, row by
// row, a run of 2 h(dy) + 1 pixels with h(dy) the largest |dx| on that row, so
// its pixel sum is a sum over rows of two differences of row-prefix sums:
// exactly the integer the per-pixel definition gives, with 2 (2r - 1) table
// reads instead of one read per pixel.  The table holds, for every row of the
// frame window a tile's particles look at, P[c] = sum of the window bytes in
// columns [0, c), as u16 (a window row is at most 128 bytes wide), P[c] at
// entry kPrefBase + c of the row.

__host__ __device__ constexpr int disk_half_width_c(int r, int dy)
{
    int h = 0;
    while ((h + 1) * (h + 1) + dy * dy < r * r) ++h;
    return h;
}

// Offsets of the two prefix entries of every disk row, relative to the table
// entry (row of cy - (r - 1), column of cx - (r - 1)) in u16 elements.
template <int R>
struct DiskRows {
    static constexpr int ROWS = 2 * R - 1;
    int plus[ROWS], minus[ROWS];
    constexpr DiskRows() : plus(), minus()
    {
        for (int i = 0; i < ROWS; ++i) {
            const int dy = i - (R - 1);
            const int h = disk_half_width_c(R, dy);
            plus[i] = i * kPrefPitch + kPrefBase + (R - 1) + h + 1;
            minus[i] = i * kPrefPitch + kPrefBase + (R - 1) - h;
        }
    }
};

__device__ __forceinline__ int disk_half_width(int r, int dy)
{
    const int m = r * r - dy * dy - 1;
    int h = (int)sqrtf((float)m);
    while ((h + 1) * (h + 1) <= m) ++h;
    while (h * h > m) --h;
    return h;
}

// Pixel sum over the disk; `p` points at the table entry of the disk's
// top-left corner (row cy - (r - 1), column cx - (r - 1)).
template <int RC>
__device__ __forceinline__ int disk_sum_prefix(const uint16_t* p, int r)
{
    int s = 0;
    if constexpr (RC > 0) {
        constexpr DiskRows<RC> rows{};
#pragma unroll
        for (int i = 0; i < DiskRows<RC>::ROWS; ++i) s += (int)p[rows.plus[i]] - (int)p[rows.minus[i]];
    } else {
        for (int i = 0; i < 2 * r - 1; ++i) {
            const int h = disk_half_width(r, i - (r - 1));
            const uint16_t* row = p + i * kPrefPitch + kPrefBase + (r - 1);
            s += (int)row[h + 1] - (int)row[-h];
        }
    }
    return s;
}

// The same sum read straight from the frame with edge clamping (used when a
// tile's particles spread wider than the LDS window).
__device__ __forceinline__ int disk_sum_global(const uint8_t* frame, int64_t pitch, int W, int H,
                                               int cx, int cy, int r)
{
    int s = 0;
    for (int dy = -(r - 1); dy <= r - 1; ++dy) {
        const int h = disk_half_width(r, dy);
        const int row = min(max(cy + dy, 0), H - 1);
        const auto* rp = gbl(frame + (int64_t)row * pitch);
        for (int dx = -h; dx <= h; ++dx) s += rp[min(max(cx + dx, 0), W - 1)];
    }
    return s;
}

// ---------------------------------------------------------------------------
// Precision modes.  Each provides: the storage element, loading/storing a
// thread's PPT consecutive particles, propagation, and the pixel cell of a
// particle.  F64 stores absolute positions; the reduced modes store offsets
// from an integer origin cell c (position = c + offset) that follows the
// predicted object position, so the particles that carry the weight sit at
// |offset| <= 1/2, where 16-bit formats are densest.  The pixel of a particle
// is c + floor(offset) + [frac(offset) >= 1/2], computed exactly in float.

// Half-up rounding of a reduced-precision offset to its pixel, clamped to
// [lo, hi]: exact in float for every input (floor and the fraction
// v - floor(v) are exact).  The offset is first clamped to the integers
// [lo - origin, hi - origin], which gives the clamped pixel directly: below
// lo - origin the cell is lo either way, and at the upper bound the fraction
// is 0.
__device__ __forceinline__ int offset_cell(float v, int origin, int lo, int hi)
{
    v = __builtin_amdgcn_fmed3f(v, (float)(lo - origin), (float)(hi - origin));
    const float fl = floorf(v);
    return origin + (int)fl + ((v - fl) >= 0.5f ? 1 : 0);
}

template <int DT>
struct ModeT;

template <>
struct ModeT<PF_F64> {
    using Store = double;
    using Val = double;
    struct Prop {
        double dx, dy, sx, sy;
    };
    static __device__ __forceinline__ Val widen(Store v) { return v; }
    template <int PPT>
    static __device__ __forceinline__ void load(const void* p, int k0, Val* v)
    {
        const auto* q = gbl(reinterpret_cast<const double2_t*>(static_cast<const double*>(p) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) {
            const double2_t a = q[i];
            v[2 * i] = a.x; v[2 * i + 1] = a.y;
        }
    }
    template <int PPT, bool WT = false>
    static __device__ __forceinline__ void store(void* p, int k0, const Val* v)
    {
        auto* q = gbl(reinterpret_cast<double2_t*>(static_cast<double*>(p) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) put<WT>(q + i, double2_t{v[2 * i], v[2 * i + 1]});
    }
    // x <- x + (d + sigma z), each operation rounded (library built without
    // contraction), as Eq. (1)-(2) are written.  draw: the particles' normals;
    // apply: the move (propagate = draw, then apply).
    template <int PPT>
    struct Noise {
        double zx[PPT], zy[PPT];
    };
    template <int PPT>
    static __device__ __forceinline__ void draw(Noise<PPT>& z, const StepArgs& a, int k0, uint32_t t)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), t, a.stream_id, 0u, a.key0, a.key1);
            normal_pair_f64(w, z.zx[i], z.zy[i]);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void apply(Val* x, Val* y, const Prop& pr, const Noise<PPT>& z)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            x[i] = x[i] + (pr.dx + pr.sx * z.zx[i]);
            y[i] = y[i] + (pr.dy + pr.sy * z.zy[i]);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int k0, uint32_t t)
    {
        Noise<PPT> z;
        draw<PPT>(z, a, k0, t);
        apply<PPT>(x, y, pr, z);
    }
    static __device__ __forceinline__ int cell(Val v, int /*origin*/, int lo, int hi)
    {
        double c = floor(v + 0.5);
        c = fmin(fmax(c, (double)lo), (double)hi);
        return (int)c;
    }
};

template <>
struct ModeT<PF_F32> {
    using Store = float;
    using Val = float;
    struct Prop {
        float dx, dy, sx, sy;
    };
    static __device__ __forceinline__ Val widen(Store v) { return v; }
    template <int PPT>
    static __device__ __forceinline__ void load(const void* p, int k0, Val* v)
    {
        const auto* q = gbl(reinterpret_cast<const float2_t*>(static_cast<const float*>(p) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) {
            const float2_t a = q[i];
            v[2 * i] = a.x; v[2 * i + 1] = a.y;
        }
    }
    template <int PPT, bool WT = false>
    static __device__ __forceinline__ void store(void* p, int k0, const Val* v)
    {
        auto* q = gbl(reinterpret_cast<float2_t*>(static_cast<float*>(p) + k0));
        if constexpr (WT && PPT % 4 == 0) {  // one 16-byte store per four particles
#pragma unroll
            for (int i = 0; i < PPT / 4; ++i)
                put16_wt(reinterpret_cast<gbl_t<u32x4_t>*>(q) + i,
                         u32x4_t{__float_as_uint(v[4 * i]), __float_as_uint(v[4 * i + 1]),
                                 __float_as_uint(v[4 * i + 2]), __float_as_uint(v[4 * i + 3])});
        } else {
#pragma unroll
            for (int i = 0; i < PPT / 2; ++i) put<WT>(q + i, float2_t{v[2 * i], v[2 * i + 1]});
        }
    }
    template <int PPT>
    struct Noise {
        float zx[PPT], zy[PPT];
    };
    template <int PPT>
    static __device__ __forceinline__ void draw(Noise<PPT>& z, const StepArgs& a, int k0, uint32_t t)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), t, a.stream_id, 0u, a.key0, a.key1);
            normal_pair_f32(w, z.zx[i], z.zy[i]);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void apply(Val* x, Val* y, const Prop& pr, const Noise<PPT>& z)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            x[i] = x[i] + __builtin_fmaf(pr.sx, z.zx[i], pr.dx);
            y[i] = y[i] + __builtin_fmaf(pr.sy, z.zy[i], pr.dy);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int k0, uint32_t t)
    {
        Noise<PPT> z;
        draw<PPT>(z, a, k0, t);
        apply<PPT>(x, y, pr, z);
    }
    static __device__ __forceinline__ int cell(Val v, int origin, int lo, int hi)
    {
        return offset_cell((float)v, origin, lo, hi);
    }
};

// Half: two particles per 32-bit register; the propagation is one packed
// fused multiply-add (sigma * z + d) and one packed add per pair and axis.
template <>
struct ModeT<PF_F16> {
    using Store = _Float16;
    using Val = _Float16;
    struct Prop {
        half2_t dx, dy, sx, sy;
    };
    static __device__ __forceinline__ Val widen(Store v) { return v; }
    template <int PPT>
    static __device__ __forceinline__ void load(const void* p, int k0, Val* v)
    {
        const auto* q = gbl(reinterpret_cast<const uint32_t*>(static_cast<const _Float16*>(p) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) {
            const half2_t h = __builtin_bit_cast(half2_t, q[i]);
            v[2 * i] = h.x; v[2 * i + 1] = h.y;
        }
    }
    template <int PPT, bool WT = false>
    static __device__ __forceinline__ void store(void* p, int k0, const Val* v)
    {
        auto* q = gbl(reinterpret_cast<uint32_t*>(static_cast<_Float16*>(p) + k0));
        if constexpr (WT && PPT % 4 == 0) {  // one 8-byte store per four particles
#pragma unroll
            for (int i = 0; i < PPT / 4; ++i) {
                const half2_t lo = {v[4 * i], v[4 * i + 1]}, hi = {v[4 * i + 2], v[4 * i + 3]};
                const uint64_t w = (uint64_t)__builtin_bit_cast(uint32_t, lo) |
                                   ((uint64_t)__builtin_bit_cast(uint32_t, hi) << 32);
                put<true>(reinterpret_cast<gbl_t<uint64_t>*>(q) + i, w);
            }
        } else {
#pragma unroll
            for (int i = 0; i < PPT / 2; ++i) {
                const half2_t h = {v[2 * i], v[2 * i + 1]};
                put<WT>(q + i, __builtin_bit_cast(uint32_t, h));
            }
        }
    }
    template <int PPT>
    struct Noise {
        half2_t zx[PPT / 2], zy[PPT / 2];
    };
    template <int PPT>
    static __device__ __forceinline__ void draw(Noise<PPT>& z, const StepArgs& a, int k0, uint32_t t)
    {
#pragma unroll
        for (int i = 0; i < PPT; i += 2) {
            const u32x4 w0 = philox4x32_10((uint32_t)(k0 + i), t, a.stream_id, 0u, a.key0, a.key1);
            const u32x4 w1 = philox4x32_10((uint32_t)(k0 + i + 1), t, a.stream_id, 0u, a.key0, a.key1);
            float zx0, zy0, zx1, zy1;
            normal_pair_f32(w0, zx0, zy0);
            normal_pair_f32(w1, zx1, zy1);
            z.zx[i / 2] = __builtin_convertvector((float2_t){zx0, zx1}, half2_t);
            z.zy[i / 2] = __builtin_convertvector((float2_t){zy0, zy1}, half2_t);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void apply(Val* x, Val* y, const Prop& pr, const Noise<PPT>& z)
    {
#pragma unroll
        for (int i = 0; i < PPT; i += 2) {
            half2_t xx = {x[i], x[i + 1]};
            half2_t yy = {y[i], y[i + 1]};
            xx = xx + __builtin_elementwise_fma(pr.sx, z.zx[i / 2], pr.dx);
            yy = yy + __builtin_elementwise_fma(pr.sy, z.zy[i / 2], pr.dy);
            x[i] = xx.x; x[i + 1] = xx.y;
            y[i] = yy.x; y[i + 1] = yy.y;
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int k0, uint32_t t)
    {
        Noise<PPT> z;
        draw<PPT>(z, a, k0, t);
        apply<PPT>(x, y, pr, z);
    }
    // The same propagation one particle at a time in scalar half arithmetic
    // (each normal cast to half on its own, then a scalar fused multiply-add
    // and add per axis): the straightforward unpacked form, kept to measure
    // what packing two particles per register gains.  Written as explicit
    // instructions so that the compiler cannot pack them again; every
    // operation rounds as its packed lane does, so the results are the same
    // bit for bit.
    template <int PPT>
    static __device__ __forceinline__ void propagate_scalar(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                            int k0, uint32_t t)
    {
        const _Float16 dx = pr.dx.x, dy = pr.dy.x, sx = pr.sx.x, sy = pr.sy.x;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), t, a.stream_id, 0u, a.key0, a.key1);
            float zx, zy;
            normal_pair_f32(w, zx, zy);
            _Float16 hx, hy, mx, my, ox, oy;
            __asm__("v_cvt_f16_f32 %0, %1" : "=v"(hx) : "v"(zx));
            __asm__("v_cvt_f16_f32 %0, %1" : "=v"(hy) : "v"(zy));
            __asm__("v_fma_f16 %0, %1, %2, %3" : "=v"(mx) : "v"(sx), "v"(hx), "v"(dx));
            __asm__("v_fma_f16 %0, %1, %2, %3" : "=v"(my) : "v"(sy), "v"(hy), "v"(dy));
            __asm__("v_add_f16 %0, %1, %2" : "=v"(ox) : "v"(x[i]), "v"(mx));
            __asm__("v_add_f16 %0, %1, %2" : "=v"(oy) : "v"(y[i]), "v"(my));
            x[i] = ox;
            y[i] = oy;
        }
    }
    // A half's value in float, plus one half, is exact (at most 18
    // significant bits), so floor(v + 1/2) is the half-up rounding that
    // offset_cell forms in general; clamping v + 1/2 to the integers
    // [lo - origin, hi - origin] before the floor clamps the cell to
    // [lo, hi] (floor commutes with a clamp to integers).
    static __device__ __forceinline__ int cell(Val v, int origin, int lo, int hi)
    {
        const float f = __builtin_amdgcn_fmed3f((float)v + 0.5f, (float)(lo - origin), (float)(hi - origin));
        return origin + (int)floorf(f);
    }
};

// bfloat16: gfx950 has no packed bfloat16 multiply-add, so the state is
// widened to float, propagated there, and rounded once (to nearest even) to
// bfloat16 by the packed conversion when it is stored.  Within the step the
// likelihood and estimate use the float position in registers; the bfloat16
// rounding reaches the next step's ancestors.
template <>
struct ModeT<PF_BF16> {
    using Store = uint16_t;
    using Val = float;  // widened on load
    struct Prop {
        float dx, dy, sx, sy;
    };
    static __device__ __forceinline__ Val widen(Store v) { return __uint_as_float((uint32_t)v << 16); }
    template <int PPT>
    static __device__ __forceinline__ void load(const void* p, int k0, Val* v)
    {
        const auto* q = gbl(reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(p) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) {
            const uint32_t a = q[i];
            v[2 * i] = __uint_as_float(a << 16);
            v[2 * i + 1] = __uint_as_float(a & 0xFFFF0000u);
        }
    }
    static __device__ __forceinline__ uint32_t pack(float lo, float hi)
    {
        const __bf16 a = (__bf16)lo, b = (__bf16)hi;
        return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
    template <int PPT, bool WT = false>
    static __device__ __forceinline__ void store(void* p, int k0, const Val* v)
    {
        auto* q = gbl(reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(p) + k0));
        if constexpr (WT && PPT % 4 == 0) {  // one 8-byte store per four particles
#pragma unroll
            for (int i = 0; i < PPT / 4; ++i) {
                const uint64_t w = (uint64_t)pack(v[4 * i], v[4 * i + 1]) |
                                   ((uint64_t)pack(v[4 * i + 2], v[4 * i + 3]) << 32);
                put<true>(reinterpret_cast<gbl_t<uint64_t>*>(q) + i, w);
            }
        } else {
#pragma unroll
            for (int i = 0; i < PPT / 2; ++i) put<WT>(q + i, pack(v[2 * i], v[2 * i + 1]));
        }
    }
    template <int PPT>
    struct Noise {
        float zx[PPT], zy[PPT];
    };
    template <int PPT>
    static __device__ __forceinline__ void draw(Noise<PPT>& z, const StepArgs& a, int k0, uint32_t t)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), t, a.stream_id, 0u, a.key0, a.key1);
            normal_pair_f32(w, z.zx[i], z.zy[i]);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void apply(Val* x, Val* y, const Prop& pr, const Noise<PPT>& z)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            x[i] = x[i] + __builtin_fmaf(pr.sx, z.zx[i], pr.dx);
            y[i] = y[i] + __builtin_fmaf(pr.sy, z.zy[i], pr.dy);
        }
    }
    template <int PPT>
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int k0, uint32_t t)
    {
        Noise<PPT> z;
        draw<PPT>(z, a, k0, t);
        apply<PPT>(x, y, pr, z);
    }
    static __device__ __forceinline__ int cell(Val v, int origin, int lo, int hi)
    {
        return offset_cell((float)v, origin, lo, hi);
    }
};

template <int DT>
__device__ __forceinline__ typename ModeT<DT>::Prop make_prop(const StepArgs& a, float ddx, float ddy)
{
    using M = ModeT<DT>;
    typename M::Prop pr;
    if constexpr (DT == PF_F64) {
        pr.dx = a.drift_x; pr.dy = a.drift_y; pr.sx = a.sigma_x; pr.sy = a.sigma_y;
    } else if constexpr (DT == PF_F16) {
        const _Float16 hx = (_Float16)ddx, hy = (_Float16)ddy;
        const _Float16 gx = (_Float16)(float)a.sigma_x, gy = (_Float16)(float)a.sigma_y;
        pr.dx = half2_t{hx, hx}; pr.dy = half2_t{hy, hy};
        pr.sx = half2_t{gx, gx}; pr.sy = half2_t{gy, gy};
    } else {
        pr.dx = ddx; pr.dy = ddy; pr.sx = (float)a.sigma_x; pr.sy = (float)a.sigma_y;
    }
    return pr;
}

// ---------------------------------------------------------------------------
// Pass A.

constexpr int kMaxWavesA = 8;  // pass A runs 128, 256 or 512 threads per tile

struct PassALds {
    uint16_t pref[kPrefPitch * kPrefRows];
    int box[kMaxWavesA][4];
    double red_d[3][kMaxWavesA];
    float red_f[3][kMaxWavesA];
    int red_i[kMaxWavesA];
};

// Source tiles whose prefix sums and propagated positions a gathered state
// loads at once and stages in LDS (a tracking step's output tile has two
// owners on average, at most four in the measured workloads; the double
// mode's 16-byte positions stage two, to keep four workgroups per CU:
// 37 KB of LDS in both modes).  Further owners, if any, are taken one at a
// time from memory.
__host__ __device__ constexpr int gather_stage(int dtype) { return dtype == PF_F64 ? 2 : 4; }

// LDS of a pass A that gathers its state, used before the pass's own LDS (the
// two share the space): slot marks, the candidate tiles' positions, and two
// small exchanges.
template <int DT>
struct GatherLds {
    using Store = typename ModeT<DT>::Store;
    struct alignas(2 * sizeof(Store)) XY {
        Store x, y;
    };
    int32_t marks[kTile];
    XY stage[gather_stage(DT)][kTile];
    int32_t cand[2];
    int32_t red[4];
};

template <int DT>
union PassAGatherLds {
    PassALds a;
    GatherLds<DT> g;
};

template <int DT, int PPT, typename Pre>
__device__ void gather_state(const StepArgs& a, int tile, bool prev_odd, GatherLds<DT>& lds, const int* ev,
                             typename ModeT<DT>::Val* x, typename ModeT<DT>::Val* y, Pre&& pre);

// Pass A of tile `tile` of the filter described by `a`, PPT particles per
// thread (kTile / PPT threads).  GATHER: the filter defers its resampling
// (StepArgs::gather): this step's outputs go to set tn mod 2, and a pending
// resampling of the previous step is gathered for the tile's slots instead
// of loading the state arrays.
template <int DT, int RC, int PPT, bool SCALAR_HALF = false, bool WT = false, bool GATHER = false>
__device__ __forceinline__ void pass_a_tile(const StepArgs& a, int tile, PassALds& lds,
                                            GatherLds<DT>* glds = nullptr)
{
    static_assert(!SCALAR_HALF || DT == PF_F16, "the unpacked propagation is a half-precision variant");
    using M = ModeT<DT>;
    constexpr int kBlockA = kTile / PPT;
    constexpr int kWavesA = kBlockA / 64;
    static_assert(kWavesA >= 1 && kWavesA <= kMaxWavesA && kBlockA * PPT == kTile, "tile shape");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int k0 = tile * kTile + tid * PPT;
    const int n = (int)a.n;
    const int r = RC > 0 ? RC : a.r;

    // A gathering pass A loads the previous step's end-slot column (wave 0)
    // together with the block, before it knows whether a resampling is
    // pending (the column is in bounds either way).
    constexpr int kEv = GATHER ? kGatherMaxTiles / 64 : 1;
    int ev[kEv];
    if constexpr (GATHER) {
        if (wv == 0) {
            const auto* ec = gbl(static_cast<const int32_t*>(a.ecol));
#pragma unroll
            for (int j = 0; j < kEv; ++j) ev[j] = ec[min(lane + 64 * j, (int)a.ntiles - 1)];
        }
    }

    // Origins (reduced modes): stored offsets are relative to ci, the
    // propagated ones to cn; the drift is applied minus the origin change.
    // The step's index is one past the block's count (the combine advances it).
    const auto* blk = gbl(a.blk);
    const uint32_t tn = blk->t + 1u;
    int cnx = 0, cny = 0;
    float ddx = 0.f, ddy = 0.f;
    if constexpr (DT != PF_F64) {
        const int cix = blk->ci_x, ciy = blk->ci_y;
        cnx = blk->cn_x; cny = blk->cn_y;
        ddx = (float)(a.drift_x - (double)(cnx - cix));
        ddy = (float)(a.drift_y - (double)(cny - ciy));
    }
    const typename M::Prop pr = make_prop<DT>(a, ddx, ddy);

    void* out_px = a.px;
    void* out_py = a.py;
    void* out_q = a.q;
    typename M::Val x[PPT], y[PPT];
    if constexpr (GATHER) {
        const bool odd = (tn & 1u) != 0;
        if (odd) {
            out_px = a.px2;
            out_py = a.py2;
            out_q = a.q2;
        }
        if (wv == 0) {  // the column's loads complete here, with the block's
#pragma unroll
            for (int j = 0; j < kEv; ++j) __asm__ volatile("" ::"v"(ev[j]));
        }
        if (blk->pend) {  // uniform
            if constexpr (DT == PF_F64) {
                // (drawn before, the double normals would hold 16 more
                // registers through the gather: three workgroups per CU)
                gather_state<DT, PPT>(a, tile, !odd, *glds, ev, x, y, []() {});
                __syncthreads();  // the gather's LDS is the pass's from here on
                M::template propagate<PPT>(x, y, pr, a, k0, tn);
            } else {
                // the normals are drawn while the candidates' loads are in
                // flight (an empty use of each keeps the compiler from sinking
                // the draws to their use after the gather)
                typename M::template Noise<PPT> nz;
                gather_state<DT, PPT>(a, tile, !odd, *glds, ev, x, y, [&]() {
                    M::template draw<PPT>(nz, a, k0, tn);
                    constexpr int kZ = (int)(sizeof(nz.zx) / sizeof(nz.zx[0]));
#pragma unroll
                    for (int i = 0; i < kZ; ++i) __asm__ volatile("" ::"v"(nz.zx[i]), "v"(nz.zy[i]));
                });
                __syncthreads();  // the gather's LDS is the pass's from here on
                M::template apply<PPT>(x, y, pr, nz);
            }
        } else {
            M::template load<PPT>(a.sx, k0, x);
            M::template load<PPT>(a.sy, k0, y);
            M::template propagate<PPT>(x, y, pr, a, k0, tn);
        }
    } else {
        M::template load<PPT>(a.sx, k0, x);
        M::template load<PPT>(a.sy, k0, y);
        if constexpr (SCALAR_HALF) M::template propagate_scalar<PPT>(x, y, pr, a, k0, tn);
        else M::template propagate<PPT>(x, y, pr, a, k0, tn);
    }
    M::template store<PPT, WT>(out_px, k0, x);
    M::template store<PPT, WT>(out_py, k0, y);

    // Pixel cells, clamped to where clamping the disk pixels changes nothing.
    const int lox = -(r - 1), hix = a.W - 1 + (r - 1);
    const int loy = -(r - 1), hiy = a.H - 1 + (r - 1);
    int cx[PPT], cy[PPT];
    bool valid[PPT];
    int b0 = INT32_MAX, b1 = INT32_MAX, b2 = INT32_MAX, b3 = INT32_MAX;  // min x, min y, -max x, -max y
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        valid[i] = k0 + i < n;
        cx[i] = M::cell(x[i], cnx, lox, hix);
        cy[i] = M::cell(y[i], cny, loy, hiy);
        if (valid[i]) {
            b0 = min(b0, cx[i]); b1 = min(b1, cy[i]);
            b2 = min(b2, -cx[i]); b3 = min(b3, -cy[i]);
        }
    }
    // Bounding box of the tile's cells: four wave reductions, one exchange.
    b0 = wave_min(b0); b1 = wave_min(b1); b2 = wave_min(b2); b3 = wave_min(b3);
    if (lane == 0) {
        lds.box[wv][0] = b0; lds.box[wv][1] = b1; lds.box[wv][2] = b2; lds.box[wv][3] = b3;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kWavesA; ++w) {
        b0 = min(b0, lds.box[w][0]); b1 = min(b1, lds.box[w][1]);
        b2 = min(b2, lds.box[w][2]); b3 = min(b3, lds.box[w][3]);
    }
    const int bx0 = b0, by0 = b1, bx1 = -b2, by1 = -b3;

    // Disk sums over the frame window of the tile: the window's row-prefix
    // table is built in LDS.  A window row is split over LPR lanes (16 for
    // windows up to 64 columns, else 32), four columns per lane, so a wave
    // covers 64 / LPR rows per round; every load of the wave is issued before
    // the first scan, and each lane writes its four prefix values as two
    // 32-bit LDS stores.  When the frame's rows are 4-byte aligned the table
    // starts at the window's first column rounded down to a multiple of 4, so
    // a lane whose four columns lie inside the frame reads them with one
    // aligned 32-bit load (edge lanes read bytes, clamped to the frame).
    // Columns past the window only reach prefix entries no disk reads.
    const int wx0 = bx0 - (r - 1), wy0 = by0 - (r - 1);
    const int ww = bx1 - bx0 + 2 * r - 1, wh = by1 - by0 + 2 * r - 1;
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.frame) | (uintptr_t)a.pitch) & 3) == 0;
    const int xs = aligned ? (wx0 & ~3) : wx0;  // frame column of table column 0
    const int sh = wx0 - xs;
    const int tw = ww + sh;                     // table columns
    const bool in_lds = !a.naive_lik && tw <= kWinMaxW && wh <= kPrefRows;
    int S[PPT];
    if (in_lds) {
        constexpr int kMaxRounds = kPrefRows / (kWavesA * 2);  // 32-lane rows: 2 per wave per round
        const bool narrow = tw <= 64;
        const int lpr = narrow ? 16 : 32;
        const int rpr = 64 / lpr;                 // rows per wave per round
        const int sub = lane / lpr, l = lane - sub * lpr;
        const int c0 = 4 * l;
        const int rows_per_round = kWavesA * rpr;
        const int rounds = (wh + rows_per_round - 1) / rows_per_round;
        uint32_t v[kMaxRounds];
#pragma unroll
        for (int it = 0; it < kMaxRounds; ++it) {
            const int yy = (it * kWavesA + wv) * rpr + sub;
            v[it] = 0;
            if (it < rounds && yy < wh && c0 < tw) {
                const int row = min(max(wy0 + yy, 0), a.H - 1);
                const auto* rp = gbl(a.frame + (int64_t)row * a.pitch);
                const int x = xs + c0;
                uint32_t pk = 0;
                if (aligned && x >= 0 && x + 3 < a.W) {
                    pk = *reinterpret_cast<const gbl_t<uint32_t>*>(rp + x);
                } else {
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb)
                        pk |= (uint32_t)rp[min(max(x + bb, 0), a.W - 1)] << (8 * bb);
                }
                v[it] = pk;
            }
        }
#pragma unroll
        for (int it = 0; it < kMaxRounds; ++it) {
            if (it < rounds) {  // uniform: every lane takes part in the scan
                const int yy = (it * kWavesA + wv) * rpr + sub;
                const int p1 = (int)(v[it] & 0xFF);
                const int p2 = p1 + (int)((v[it] >> 8) & 0xFF);
                const int p3 = p2 + (int)((v[it] >> 16) & 0xFF);
                const int p4 = p3 + (int)(v[it] >> 24);
                // inclusive prefix of the 4-column sums over the lanes of one row
                int sc = p4;
                sc += dpp<0x111>(sc, 0);
                sc += dpp<0x112>(sc, 0);
                sc += dpp<0x114>(sc, 0);
                sc += dpp<0x118>(sc, 0);
                if (!narrow) sc += dpp<0x142, 0xA>(sc, 0);
                const int ex = sc - p4;
                if (yy < wh) {
                    uint16_t* prow = lds.pref + yy * kPrefPitch + kPrefBase;
                    if (l == 0) prow[0] = 0;
                    uint32_t* w32 = reinterpret_cast<uint32_t*>(prow + c0 + 1);
                    w32[0] = (uint32_t)(ex + p1) | ((uint32_t)(ex + p2) << 16);
                    w32[1] = (uint32_t)(ex + p3) | ((uint32_t)(ex + p4) << 16);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int ox = valid[i] ? cx[i] - bx0 + sh : 0, oy = valid[i] ? cy[i] - by0 : 0;
            S[i] = disk_sum_prefix<RC>(lds.pref + oy * kPrefPitch + ox, r);
        }
    } else {
#pragma unroll
        for (int i = 0; i < PPT; ++i)
            S[i] = valid[i] ? disk_sum_global(a.frame, a.pitch, a.W, a.H, cx[i], cy[i], r) : 0;
    }
    // sum over the disk of (I - bg)^2 - (I - fg)^2 = 2 (fg - bg) I - (fg^2 - bg^2)
    const int c1k = 2 * (a.fg - a.bg), c0k = a.nd * (a.fg * a.fg - a.bg * a.bg);
#pragma unroll
    for (int i = 0; i < PPT; ++i) S[i] = c1k * S[i] - c0k;

    // Tile maximum and weights relative to it.
    using Acc = typename std::conditional<DT == PF_F64, double, float>::type;
    Acc wt[PPT];
    Acc tile_m = 0;
    int tile_smax = 0;
    if constexpr (DT == PF_F64) {
        double L[PPT];
        double m = -INFINITY;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            L[i] = (double)S[i] / a.denom;
            if (valid[i]) m = fmax(m, L[i]);
        }
        m = block_max<kWavesA>(m, lds.red_d[0]);
        tile_m = m;
#pragma unroll
        for (int i = 0; i < PPT; ++i) wt[i] = valid[i] ? exp(L[i] - m) : 0.0;
    } else {
        int sm = INT32_MIN;
#pragma unroll
        for (int i = 0; i < PPT; ++i)
            if (valid[i]) sm = max(sm, S[i]);
        sm = block_max<kWavesA>(sm, lds.red_i);
        tile_smax = sm;
#pragma unroll
        for (int i = 0; i < PPT; ++i)
            wt[i] = valid[i] ? __builtin_amdgcn_exp2f((float)(S[i] - sm) * a.beta) : 0.f;
    }

    // Tile-local cumulative weights and estimate partial sums in one
    // exchange: sequential inside the thread; across threads a wave prefix
    // sum made monotone by a prefix maximum, and wave offsets as the
    // left-to-right sum of the wave totals (bit-identical to the previous
    // wave's last value); each value is clamped to its thread's inclusive
    // total, so the tile's sequence never decreases.
    Acc loc[PPT];
    Acc run = 0, ex = 0, ey = 0;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        run = run + wt[i];
        loc[i] = run;
        ex = ex + wt[i] * (Acc)x[i];
        ey = ey + wt[i] * (Acc)y[i];
    }
    Acc sw = wave_incl_sum(run, lane);
    if constexpr (DT == PF_F64) sw = wave_incl_max(sw, lane);
    else sw = wave_incl_max_nonneg(sw);  // the weights are non-negative
    ex = wave_sum(ex);
    ey = wave_sum(ey);
    Acc (*red)[kMaxWavesA];
    if constexpr (DT == PF_F64) red = lds.red_d; else red = lds.red_f;
    if (lane == 63) {
        red[0][wv] = sw;
        red[1][wv] = ex;
        red[2][wv] = ey;
    }
    __syncthreads();
    Acc off = 0;
    if (wv > 0) {
        off = red[0][0];
        for (int w = 1; w < wv; ++w) off = off + red[0][w];
    }
    const Acc incl = wv > 0 ? off + sw : sw;
    const Acc excl = wave_shift_up1(incl, off);
    Acc q[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const Acc v = excl + loc[i];
        q[i] = v < incl ? v : incl;
    }
    if constexpr (DT == PF_F64) {
        auto* qp = gbl(reinterpret_cast<double2_t*>(static_cast<double*>(out_q) + k0));
#pragma unroll
        for (int i = 0; i < PPT / 2; ++i) put<WT>(qp + i, double2_t{q[2 * i], q[2 * i + 1]});
    } else {
        auto* qp = gbl(reinterpret_cast<float2_t*>(static_cast<float*>(out_q) + k0));
        if constexpr (WT && PPT % 4 == 0) {  // one 16-byte store per four particles
#pragma unroll
            for (int i = 0; i < PPT / 4; ++i)
                put16_wt(reinterpret_cast<gbl_t<u32x4_t>*>(qp) + i,
                         u32x4_t{__float_as_uint(q[4 * i]), __float_as_uint(q[4 * i + 1]),
                                 __float_as_uint(q[4 * i + 2]), __float_as_uint(q[4 * i + 3])});
        } else {
#pragma unroll
            for (int i = 0; i < PPT / 2; ++i) put<WT>(qp + i, float2_t{q[2 * i], q[2 * i + 1]});
        }
    }
    if (a.dg_s) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            a.dg_s[k0 + i] = S[i];
            a.dg_w[k0 + i] = (double)wt[i];
        }
    }
    if (a.s_all) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) a.s_all[k0 + i] = S[i];
    }
    if (tid == kBlockA - 1) {
        // the tile total is the last thread's inclusive value
        Acc tx = red[1][0], ty = red[2][0];
        for (int w = 1; w < kWavesA; ++w) {
            tx = tx + red[1][w];
            ty = ty + red[2][w];
        }
        if constexpr (DT == PF_F64) {
            store_rec(gbl(static_cast<TileRec64*>(a.rec)) + tile, TileRec64{tile_m, incl, tx, ty});
        } else {
            store_rec(gbl(static_cast<TileRec32*>(a.rec)) + tile, TileRec32{tile_smax, incl, tx, ty});
        }
    }
}

// Tile of workgroup b when consecutive tiles should share an XCD: workgroups
// are dispatched to the 8 XCDs in turn (b mod 8), and XCD x takes a
// contiguous range of tiles (a bijection of [0, nt) for any nt).
__device__ __forceinline__ int xcd_tile(int b, int nt)
{
    const int x = b & 7, r = b >> 3, q = nt >> 3, rem = nt & 7;
    return x * q + min(x, rem) + r;
}

template <int DT, int RC, int PPT, bool SCALAR_HALF = false, bool WT = false, bool GATHER = false>
__global__ __launch_bounds__(kTile / PPT) void pass_a_kernel(StepArgs a)
{
    if constexpr (GATHER) {
        // consecutive output tiles mostly gather from the same source tiles:
        // on one XCD, the second reads them from its L2
        __shared__ PassAGatherLds<DT> lds;
        pass_a_tile<DT, RC, PPT, SCALAR_HALF, WT, GATHER>(a, xcd_tile((int)blockIdx.x, a.ntiles), lds.a, &lds.g);
    } else {
        __shared__ PassALds lds;
        pass_a_tile<DT, RC, PPT, SCALAR_HALF, WT, GATHER>(a, blockIdx.x, lds);
    }
}

// ---------------------------------------------------------------------------
// End slots.  A particle with normalised cumulative weight C = P / Z ends the
// strata (j + u0) / N <= C, i.e. its end slot is floor(N P / Z - u0) + 1
// (clamped to [0, N]).  With R = N / Z and P = off_t + f_t q inside tile t,
// the slot coordinate is the affine y = (R off_t - u0) + (R f_t) q, capped at
// y_max = R off_{t+1} - u0, whose end slot is the tile's end slot E_t (the
// combine evaluates exactly that expression), so tiles join without gaps.
// The double mode evaluates y in double (the slot coordinate of N <= 2^28
// strata then carries an error far below the 1e-12 resolution of the
// distribution); the reduced modes form the tile's base in two-float
// arithmetic (about 44 bits) and each particle's offset from it in float.

__device__ __forceinline__ int slot_end_of(double y, int n)
{
    const double g = floor(y) + 1.0;
    return g <= 0.0 ? 0 : (g >= (double)n ? n : (int)g);
}

__device__ __forceinline__ int slot_end_of(ff y, int n)
{
    const int64_t g = ff_floor(y) + 1;
    return g <= 0 ? 0 : (g >= n ? n : (int)g);
}

template <int DT>
struct TileSlots;

template <>
struct TileSlots<PF_F64> {
    double base, scale, ymax;
    int E, Eprev;
    // The words the tile's map is built from, one per lane: 0-4 off, f and
    // E of table entry t; 5-6 off of entry t + 1; 7 E of entry t - 1 (0 for
    // the first tile); 8-9 R and 10-11 u0 of the filter's block.  One vector
    // load fetches them and the constructor reads them out, so a streaming
    // kernel loads them one tile ahead and needs no wait for them until it
    // builds the map, after the tile before.
    struct Raw {
        uint32_t w;
        __device__ void load(const StepArgs& a, int t)
        {
            constexpr int kW = (int)(sizeof(TileTab64) / 4);
            const auto* tw = gbl(static_cast<const uint32_t*>(a.tab));
            const auto* bw = gbl(reinterpret_cast<const uint32_t*>(a.blk));
            const int lane = threadIdx.x & 63;
            const gbl_t<const uint32_t>* p =
                lane < 5    ? tw + ((int64_t)kW * t + lane)
                : lane < 7  ? tw + ((int64_t)kW * (t + 1) + (lane - 5))
                : lane == 7 ? tw + ((int64_t)kW * (t - 1) + 4)
                : lane < 10 ? bw + (offsetof(DevBlock, R) / 4 + (lane - 8))
                            : bw + (offsetof(DevBlock, u0) / 4 + (lane - 10));
            w = 0;
            if (lane < 12 && (lane != 7 || t > 0)) w = *p;
        }
        __device__ int word(int l) const { return __builtin_amdgcn_readlane((int)w, l); }
        __device__ double dword(int l) const { return __hiloint2double(word(l + 1), word(l)); }
    };
    static_assert(offsetof(TileTab64, off) == 0 && offsetof(TileTab64, f) == 8 && offsetof(TileTab64, E) == 16,
                  "table word layout");
    static_assert(offsetof(DevBlock, R) % 8 == 0 && offsetof(DevBlock, u0) % 8 == 0, "block word layout");
    TileSlots() = default;
    __device__ explicit TileSlots(const Raw& r)
    {
        init(r.dword(8), r.dword(10), r.dword(0), r.dword(2), r.dword(5), r.word(4), r.word(7));
    }
    __device__ void init(double R, double u0, double off, double f, double off1, int e, int eprev)
    {
        base = R * off - u0;
        scale = R * f;
        ymax = R * off1 - u0;
        E = e;
        Eprev = eprev;
    }
    __device__ int of(double qv, int n) const
    {
        double y = __builtin_fma(scale, qv, base);
        y = y < ymax ? y : ymax;
        return slot_end_of(y, n);
    }
};

// Reduced modes: the tile's base coordinate R off_t - u0 (two-float, up to N)
// is split once into B = floor(hi), an integer that float holds exactly, and
// the float remainder frac = (hi - B) + lo (within about one of zero); a
// particle's coordinate relative to B, frac + (R f_t) q, is at most the
// tile's slot count plus one, so float resolves it to ~1e-4 of a slot, and
// its end slot is B plus the floor, capped at the tile's end slot.
template <>
struct TileSlots<PF_F32> {
    float frac, scale;
    int B, cap, E, Eprev;
    // The map's words, one per lane as in the double mode: 0-3 table entry
    // t; 4 E of entry t - 1 (0 for the first tile); 5-6 R and 7-8 u0 (hi,
    // lo) of the filter's block.
    struct Raw {
        uint32_t w;
        __device__ void load(const StepArgs& a, int t)
        {
            const auto* tw = gbl(static_cast<const uint32_t*>(a.tab));
            const auto* bw = gbl(reinterpret_cast<const uint32_t*>(a.blk));
            const int lane = threadIdx.x & 63;
            const gbl_t<const uint32_t>* p =
                lane < 4    ? tw + (4 * (int64_t)t + lane)
                : lane == 4 ? tw + (4 * (int64_t)(t - 1) + 3)
                : lane < 7  ? bw + (offsetof(DevBlock, R_hi) / 4 + (lane - 5))
                            : bw + (offsetof(DevBlock, u0_hi) / 4 + (lane - 7));
            w = 0;
            if (lane < 9 && (lane != 4 || t > 0)) w = *p;
        }
        __device__ int word(int l) const { return __builtin_amdgcn_readlane((int)w, l); }
        __device__ float fword(int l) const { return __int_as_float(word(l)); }
    };
    static_assert(sizeof(TileTab32) == 16 && offsetof(TileTab32, off_lo) == 4 && offsetof(TileTab32, f) == 8 &&
                  offsetof(TileTab32, E) == 12, "table word layout");
    static_assert(offsetof(DevBlock, R_lo) == offsetof(DevBlock, R_hi) + 4 &&
                  offsetof(DevBlock, u0_lo) == offsetof(DevBlock, u0_hi) + 4, "block word layout");
    TileSlots() = default;
    __device__ explicit TileSlots(const Raw& r)
    {
        init(ff{r.fword(5), r.fword(6)}, ff{r.fword(7), r.fword(8)}, ff{r.fword(0), r.fword(1)}, r.fword(2),
             r.word(3), r.word(4));
    }
    __device__ void init(ff R, ff u0, ff off, float f, int e, int eprev)
    {
        const ff mu0{-u0.hi, -u0.lo};
        const ff base = ff_add(ff_mul(R, off), mu0);
        const float bh = floorf(base.hi);
        B = (int)bh;
        frac = (base.hi - bh) + base.lo;
        scale = ff_mul_f(R, f).hi;
        E = e;
        Eprev = eprev;
        cap = E - B;
    }
    __device__ int of(float qv, int /*n*/) const
    {
        const float y = __builtin_fmaf(scale, qv, frac);
        return B + min((int)floorf(y) + 1, cap);
    }
};

template <int DT>
using TileSlotsT = TileSlots<DT == PF_F64 ? PF_F64 : PF_F32>;

// ---------------------------------------------------------------------------
// Deferred resampling.  A single FP64 or FP32 filter of at most
// kGatherMaxTiles tiles does not run pass C after its combine: the resampled state that pass C would
// write is defined by the step's propagated positions and prefix sums (set t
// mod 2), its table, block and end-slot column, and the next step's pass A
// gathers, for its own tile's slots [lo, hi), exactly the particles that
// pass C would have copied there.  The end slots of a source tile's
// particles are pass C's (TileSlots::of of the same prefix sums, raised to
// the tile's first slot, the last particle ending at the tile's end slot), a
// particle k owning the slots from the end slot of particle k - 1 (or the
// tile's first slot) up to its own.  The source tiles that own [lo, hi) are
// those from the one holding slot lo to the one holding slot hi - 1 (counted
// from the end-slot column: slot s lies in the tile whose index is the
// number of tiles before the last that end at or before s); every particle
// of theirs whose slots meet [lo, hi) marks the first of them, and an
// inclusive maximum scan over the tile's slots gives every slot its owner
// (pass C's fill, over output slots instead of one source tile's slots).
// So the gathered state is bit for bit the state pass C would have written.
template <int DT, int PPT, typename Pre>
__device__ void gather_state(const StepArgs& a, int tile, bool prev_odd, GatherLds<DT>& lds, const int* ev,
                             typename ModeT<DT>::Val* x, typename ModeT<DT>::Val* y, Pre&& pre)
{
    static_assert(PPT == 4 && kTile / PPT == 256, "gathered state: 256 threads, four slots each");
    using M = ModeT<DT>;
    using Store = typename M::Store;
    using XY = typename GatherLds<DT>::XY;
    using Q = typename std::conditional<DT == PF_F64, double, float>::type;
    typedef int32_t I4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = (int)a.n, nt = a.ntiles;
    const int lo = tile * kTile, hi = min(lo + kTile, n);
    const auto* qin = gbl(static_cast<const Q*>(prev_odd ? a.q2 : a.q));
    const auto* xin = gbl(static_cast<const Store*>(prev_odd ? a.px2 : a.px));
    const auto* yin = gbl(static_cast<const Store*>(prev_odd ? a.py2 : a.py));

    // the source tiles holding slots lo and hi - 1 (wave 0, from the end-slot
    // column loaded with the block)
    if (wv == 0) {
        int c0 = 0, c1 = 0;
#pragma unroll
        for (int j = 0; j < kGatherMaxTiles / 64; ++j) {
            if (lane + 64 * j < nt - 1) {
                c0 += ev[j] <= lo ? 1 : 0;
                c1 += ev[j] <= hi - 1 ? 1 : 0;
            }
        }
        c0 = wave_sum(c0);
        c1 = wave_sum(c1);
        if (lane == 0) {
            lds.cand[0] = c0;
            lds.cand[1] = c1;
        }
    }
    *reinterpret_cast<I4*>(lds.marks + PPT * tid) = I4{0, 0, 0, 0};
    __syncthreads();
    const int c0 = __builtin_amdgcn_readfirstlane(lds.cand[0]);
    const int c1 = __builtin_amdgcn_readfirstlane(lds.cand[1]);

    // marks: particle k of candidate c (the c - c0-th) marks the first of its
    // slots in [lo, hi) with (c - c0) kTile + k + 1.  The first S candidates'
    // words, prefix sums and positions are loaded together (one round trip)
    // and their positions staged in LDS; any further candidate is loaded and
    // marked on its own, its owners' positions read from memory.
    constexpr int S = gather_stage(DT);
    const int k = PPT * tid;  // this thread's particles k .. k + 3, and k - 1
    // A candidate tile is read with one vector load per array and thread
    // (the particles k .. k + 3 are contiguous and aligned; the arrays are
    // padded to whole tiles, so the last tile's loads stay inside them and
    // its particles past N are never marked) and one load of particle k - 1's
    // prefix sum.  Element-wise loads issued several times the cache-line
    // requests of pass A's state load and took three times as long; a
    // separate element-wise path for the last tile made the compiler wait
    // for each candidate's loads before issuing the next one's.
    typedef Q Q4 __attribute__((ext_vector_type(4)));
    typedef Store S4 __attribute__((ext_vector_type(4)));
    struct Cand {
        typename TileSlotsT<DT>::Raw raw;
        Q q[PPT + 1];
        Store px[PPT], py[PPT];
    };
    auto load_cand = [&](int c, Cand& cd, bool pos) {
        cd.raw.load(a, c);
        const int first = c * kTile;
        const Q4 qq = *reinterpret_cast<const gbl_t<Q4>*>(qin + first + k);
        cd.q[0] = qin[first + max(k - 1, 0)];
#pragma unroll
        for (int i = 0; i < PPT; ++i) cd.q[i + 1] = qq[i];
        if (pos) {
            const S4 xx = *reinterpret_cast<const gbl_t<S4>*>(xin + first + k);
            const S4 yy = *reinterpret_cast<const gbl_t<S4>*>(yin + first + k);
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                cd.px[i] = xx[i];
                cd.py[i] = yy[i];
            }
        }
    };
    auto mark_cand = [&](int c, const Cand& cd) {
        const int first = c * kTile, tt = min(kTile, n - first);
        const TileSlotsT<DT> ts(cd.raw);
        int e[PPT + 1];
#pragma unroll
        for (int i = 0; i <= PPT; ++i) {
            const int kk = k - 1 + i;
            e[i] = kk < 0 ? ts.Eprev : max(kk == tt - 1 ? ts.E : ts.of(cd.q[i], n), ts.Eprev);
        }
#pragma unroll
        for (int i = 1; i <= PPT; ++i) {
            const int kk = k - 1 + i, b = e[i - 1], en = e[i];
            if (kk < tt && en > b && b < hi && en > lo) lds.marks[max(b, lo) - lo] = (c - c0) * kTile + kk + 1;
        }
    };
    Cand cs[S];
#pragma unroll
    for (int j = 0; j < S; ++j)
        if (c0 + j <= c1) load_cand(c0 + j, cs[j], true);  // uniform
    pre();  // the caller's work that needs no gathered value, while the loads are in flight
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (c0 + j <= c1) {
            mark_cand(c0 + j, cs[j]);
#pragma unroll
            for (int i = 0; i < PPT; ++i) lds.stage[j][k + i] = XY{cs[j].px[i], cs[j].py[i]};
        }
    }
    for (int c = c0 + S; c <= c1; ++c) {
        Cand cd;
        load_cand(c, cd, false);
        mark_cand(c, cd);
    }
    __syncthreads();

    // owners of this thread's four slots: the last mark at or before each
    const I4 mv = *reinterpret_cast<const I4*>(lds.marks + PPT * tid);
    int mk[PPT];
    mk[0] = mv.x;
    mk[1] = max(mk[0], mv.y);
    mk[2] = max(mk[1], mv.z);
    mk[3] = max(mk[2], mv.w);
    const int sc = wave_incl_scan<OpMax>(mk[PPT - 1]);
    if (lane == 63) lds.red[wv] = sc;
    __syncthreads();
    int carry = wave_shift_up1(sc, 0);
    for (int w = 0; w < wv; ++w) carry = max(carry, lds.red[w]);
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int slot = lo + k + i;
        x[i] = 0;
        y[i] = 0;
        if (slot < hi) {
            // every slot of [lo, hi) has an owner; the clamps only keep the
            // reads inside the arrays
            const int m = max(max(carry, mk[i]) - 1, 0);
            const int cr = m / kTile, kk = m - cr * kTile;
            if (cr < S) {
                const XY v = lds.stage[cr][kk];
                x[i] = M::widen(v.x);
                y[i] = M::widen(v.y);
            } else {
                const int src = min(c0 * kTile + m, n - 1);
                x[i] = M::widen(xin[src]);
                y[i] = M::widen(yin[src]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Combine: one workgroup per filter turns the tile records into the tile
// table.  Every thread owns KPER consecutive tiles; the carried
// offsets come from a two-level scan (per wave, then over the wave totals)
// whose total is the normaliser Z; the estimate sums ride on the same
// exchange.  The tiles' end slots are made non-decreasing by an integer
// prefix maximum.  The workgroup size and KPER depend on the filter's tile
// count only (comb_class), so a filter combines the same way alone and in a
// batch.

// Two-float DPP moves and scans.
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ ff dpp_ff(ff v, float fill_hi)
{
    return ff{dpp_f<CTRL, RM>(v.hi, fill_hi), dpp_f<CTRL, RM>(v.lo, 0.f)};
}

__device__ __forceinline__ ff wave_incl_sum_ff(ff v)
{
    v = ff_add(dpp_ff<0x111>(v, 0.f), v);
    v = ff_add(dpp_ff<0x112>(v, 0.f), v);
    v = ff_add(dpp_ff<0x114>(v, 0.f), v);
    v = ff_add(dpp_ff<0x118>(v, 0.f), v);
    v = ff_add(dpp_ff<0x142, 0xA>(v, 0.f), v);
    v = ff_add(dpp_ff<0x143, 0xC>(v, 0.f), v);
    return v;
}

__device__ __forceinline__ ff wave_incl_max_ff(ff v)
{
    const float ninf = -INFINITY;
    v = ff_max(dpp_ff<0x111>(v, ninf), v);
    v = ff_max(dpp_ff<0x112>(v, ninf), v);
    v = ff_max(dpp_ff<0x114>(v, ninf), v);
    v = ff_max(dpp_ff<0x118>(v, ninf), v);
    v = ff_max(dpp_ff<0x142, 0xA>(v, ninf), v);
    v = ff_max(dpp_ff<0x143, 0xC>(v, ninf), v);
    return v;
}

// Accumulator arithmetic of the combine: double in FP64 mode, two-float in
// the reduced modes.
template <int DT>
struct CombAcc;

template <>
struct CombAcc<PF_F64> {
    using T = double;
    static __device__ T zero() { return 0.0; }
    static __device__ T add(T a, T b) { return a + b; }
    static __device__ T min_(T a, T b) { return a < b ? a : b; }
    static __device__ T max_(T a, T b) { return a > b ? a : b; }
    static __device__ T sum_scan(T v) { return wave_incl_sum(v, 0); }
    // the same scan on lanes 0 .. NW - 1 (NW <= 16: its steps inside the first
    // row; the full scan's later steps add zero there)
    template <int NW>
    static __device__ T sum_scan_first(T v)
    {
        if constexpr (NW > 16) return sum_scan(v);
        v = v + dpp<0x111>(v, 0.0);
        if constexpr (NW > 2) v = v + dpp<0x112>(v, 0.0);
        if constexpr (NW > 4) v = v + dpp<0x114>(v, 0.0);
        if constexpr (NW > 8) v = v + dpp<0x118>(v, 0.0);
        return v;
    }
    static __device__ T last(T v) { return lane63(v); }
    static __device__ T up1(T v, T fill) { return wave_shift_up1(v, fill); }
};

template <>
struct CombAcc<PF_F32> {
    using T = ff;
    static __device__ T zero() { return ff{0.f, 0.f}; }
    static __device__ T add(T a, T b) { return ff_add(a, b); }
    static __device__ T min_(T a, T b) { return ff_min(a, b); }
    static __device__ T max_(T a, T b) { return ff_max(a, b); }
    static __device__ T sum_scan(T v) { return wave_incl_sum_ff(v); }
    template <int NW>
    static __device__ T sum_scan_first(T v)
    {
        if constexpr (NW > 16) return sum_scan(v);
        v = ff_add(dpp_ff<0x111>(v, 0.f), v);
        if constexpr (NW > 2) v = ff_add(dpp_ff<0x112>(v, 0.f), v);
        if constexpr (NW > 4) v = ff_add(dpp_ff<0x114>(v, 0.f), v);
        if constexpr (NW > 8) v = ff_add(dpp_ff<0x118>(v, 0.f), v);
        return v;
    }
    static __device__ T last(T v) { return ff{lane63(v.hi), lane63(v.lo)}; }
    static __device__ T up1(T v, T fill) { return ff{wave_shift_up1(v.hi, fill.hi), wave_shift_up1(v.lo, fill.lo)}; }
};

// The map from a cumulative weight P to its end slot, floor(R P - u0) + 1
// with R = N / Z, and the step's resampling offset u0 (counter (0, t,
// stream_id, 1)): double in the FP64 mode, two-float in the reduced modes.
template <bool F64>
struct SlotMap;

// The Philox words of the step's resampling offset (counter (0, t, stream_id, 1)).
__device__ __forceinline__ u32x4 u0_words(const StepArgs& a, uint32_t t)
{
    return philox4x32_10(0u, t, a.stream_id, 1u, a.key0, a.key1);
}

template <>
struct SlotMap<true> {
    double R, mu0, u0;
    __device__ SlotMap(const StepArgs& a, double Z, uint32_t t) : SlotMap(a, Z, u0_words(a, t)) {}
    __device__ SlotMap(const StepArgs& a, double Z, const u32x4& wu)
    {
        u0 = uniform53(wu.v0, wu.v1);
        R = (double)(int)a.n / Z;
        mu0 = -u0;
    }
    __device__ int end_of(double o, int n) const { return slot_end_of(R * o + mu0, n); }
};

template <>
struct SlotMap<false> {
    ff R, mu0, u0;
    __device__ SlotMap(const StepArgs& a, ff Z, uint32_t t) : SlotMap(a, Z, u0_words(a, t)) {}
    __device__ SlotMap(const StepArgs& a, ff Z, const u32x4& wu)
    {
        const int n = (int)a.n;
        const uint64_t bits = ((uint64_t)wu.v0 << 21) | (uint64_t)(wu.v1 >> 11);
        u0 = fast_two_sum((float)(uint32_t)(bits >> 29) * 0x1.0p-24f,
                          (float)(uint32_t)(bits & 0x1FFFFFFFu) * 0x1.0p-53f);
        mu0 = ff{-u0.hi, -u0.lo};
        const ff Nff = fast_two_sum((float)n, (float)(n - (int)(float)n));
        R = ff_div(Nff, Z);
    }
    __device__ int end_of(ff o, int n) const { return slot_end_of(ff_add(ff_mul(R, o), mu0), n); }
};

// The per-filter block after a combine: normaliser, maximum, u0, R, the
// estimate (sx, sy: weighted position sums relative to the maximum) and, in
// the reduced modes, the origin of the next propagation (cnx, cny: the
// block's origin cells as the step found them, read by the caller before its
// first store, so that they come from a scalar load issued at the start and
// not from a memory round trip at the end).  One thread.
template <int DT, bool SET_T = true>
__device__ __forceinline__ void write_block(const StepArgs& a,
                                           typename std::conditional<DT == PF_F64, double, ff>::type Z,
                                           typename std::conditional<DT == PF_F64, double, int>::type gm,
                                           typename std::conditional<DT == PF_F64, double, float>::type sx,
                                           typename std::conditional<DT == PF_F64, double, float>::type sy,
                                           const SlotMap<DT == PF_F64>& sm, uint32_t t, int cnx, int cny)
{
    auto* b = gbl(a.blk);
    if constexpr (SET_T) b->t = t;
    b->pend = a.gather ? 1u : 0u;  // without pass C the resampling stays pending
    if constexpr (DT == PF_F64) {
        b->M = gm;
        b->Z = Z;
        b->u0 = sm.u0;
        b->R = sm.R;
        b->est_x = sx / Z;
        b->est_y = sy / Z;
    } else {
        const float Zf = Z.hi + Z.lo;
        const float ox = (float)cnx + sx / Zf;
        const float oy = (float)cny + sy / Zf;
        // the estimate leaves the device as double (conversion only)
        b->est_x = (double)ox;
        b->est_y = (double)oy;
        b->Zf = Zf;
        b->Smax = gm;
        b->R_hi = sm.R.hi;
        b->R_lo = sm.R.lo;
        b->u0_hi = sm.u0.hi;
        b->u0_lo = sm.u0.lo;
        // the stored positions become relative to this step's origin; the
        // next propagation is centred on the predicted position
        b->ci_x = cnx;
        b->ci_y = cny;
        const float px_ = fminf(fmaxf(ox + (float)a.drift_x, -1.0e6f), 1.0e6f);
        const float py_ = fminf(fmaxf(oy + (float)a.drift_y, -1.0e6f), 1.0e6f);
        b->cn_x = offset_cell(px_, 0, -2000000, 2000000);
        b->cn_y = offset_cell(py_, 0, -2000000, 2000000);
    }
}

// Origin cells of the next propagation as the block holds them before the
// combine (the double mode has none).
template <bool F64>
__device__ __forceinline__ void read_cells(const StepArgs& a, int& cnx, int& cny)
{
    cnx = 0;
    cny = 0;
    if constexpr (!F64) {
        const auto* b = gbl(a.blk);
        cnx = b->cn_x;
        cny = b->cn_y;
    }
}

// Value of a uniform lane l of v.
__device__ __forceinline__ double lane_at(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ ff lane_at(ff v, int l)
{
    return ff{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.hi), l)),
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.lo), l))};
}
__device__ __forceinline__ int lane_at(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// One table entry in a single store (the double mode's entry has a pad word).
__device__ __forceinline__ void put_tab(gbl_t<TileTab32>* p, ff off, float f, int E)
{
    u32x4_t w;
    w[0] = __float_as_uint(off.hi);
    w[1] = __float_as_uint(off.lo);
    w[2] = __float_as_uint(f);
    w[3] = (uint32_t)E;
    *reinterpret_cast<gbl_t<u32x4_t>*>(p) = w;
}
__device__ __forceinline__ void put_tab(gbl_t<TileTab64>* p, double off, double f, int E)
{
    p->off = off;
    p->f = f;
    p->E = E;
}

// Combine of the filter described by `a`, run by one workgroup of NT threads
// that owns KPER consecutive tiles each (at most KPER * NT tiles: one round).
// Its chain is short because it is on the step's critical path: the records
// are loaded once and kept in registers; every wave scans the wave totals
// itself (the same operations on the same values in every wave, so the same
// bits) instead of waiting for one wave to publish them; the end-slot maxima
// travel with the last offsets of the waves in one more exchange; and each
// table entry is stored whole once its end slot is known.  A single-wave
// combine exchanges nothing.
template <int DT, int KPER, int NT>
__device__ __forceinline__ void combine_filter(const StepArgs& a)
{
    constexpr int NW = NT / 64;
    constexpr bool F64 = DT == PF_F64;
    using A = CombAcc<F64 ? PF_F64 : PF_F32>;
    using T = typename A::T;
    using Rec = typename std::conditional<F64, TileRec64, TileRec32>::type;
    using Tab = typename std::conditional<F64, TileTab64, TileTab32>::type;
    using Fv = typename std::conditional<F64, double, float>::type;
    using Mx = typename std::conditional<F64, double, int>::type;
    constexpr int CHUNK = KPER * NT;

    __shared__ Mx red_m[NW];
    __shared__ T red_s[NW];
    __shared__ Fv red_x[NW], red_y[NW];
    __shared__ int red_e[NW];
    __shared__ T red_last[NW];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // A plan captured before the filter was re-initialised larger can hand a
    // filter of more tiles to this class: only the first CHUNK are combined
    // (in bounds; that step's results are meaningless, as documented).
    const int nt = min((int)a.ntiles, CHUNK);
    const int n = (int)a.n;
    const auto* rec = gbl(static_cast<const Rec*>(a.rec));
    auto* tab = gbl(static_cast<Tab*>(a.tab));

    // global maximum of the tile maxima (the loads are unconditional, from a
    // clamped index, so that all of them are in flight at once)
    Rec r[KPER];
#pragma unroll
    for (int k = 0; k < KPER; ++k) r[k] = load_rec(rec + min(tid * KPER + k, nt - 1));
    const uint32_t tn = gbl(a.blk)->t + 1u;  // this step (thread 0 advances the count at the end)
    int cnx, cny;
    read_cells<F64>(a, cnx, cny);
    // the block's words are needed now (the compiler would otherwise sink
    // their loads to the end of the chain); the resampling offset's random
    // words do not depend on the weights: drawn now, they overlap the loads
    // of the records
    __asm__ volatile("" ::"s"(tn), "s"(cnx), "s"(cny));
    const u32x4 wu0 = u0_words(a, tn);
    Mx m = F64 ? (Mx)-INFINITY : (Mx)INT32_MIN;
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        Mx mt;
        if constexpr (F64) mt = r[k].m; else mt = r[k].smax;
        if (tid * KPER + k < nt) m = mt > m ? mt : m;
    }
    m = wave_max(m);
    Mx gm = m;
    if constexpr (NW > 1) {
        if (lane == 0) red_m[wv] = m;
        __syncthreads();
        gm = red_m[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) gm = red_m[w] > gm ? red_m[w] : gm;
    }

    // factors, weighted sums and the inclusive scan of the thread totals
    Fv f[KPER];
    T v[KPER];
    T loc = A::zero();
    Fv ex = 0, ey = 0;
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        const int t = tid * KPER + k;
        f[k] = 0;
        v[k] = A::zero();
        if (t < nt) {
            if constexpr (F64) {
                f[k] = exp(r[k].m - gm);
                v[k] = f[k] * r[k].s;
            } else {
                f[k] = __builtin_amdgcn_exp2f((float)(r[k].smax - gm) * a.beta);
                v[k] = two_prod(f[k], r[k].s);
            }
            ex = ex + f[k] * r[k].sx;
            ey = ey + f[k] * r[k].sy;
        }
        loc = A::add(loc, v[k]);
    }
    const T sw = A::sum_scan(loc);
    const Fv wx = wave_sum(ex), wy = wave_sum(ey);
    T off = A::zero();  // offset of this wave's first tile
    T Z;
    Fv sx = wx, sy = wy;
    if constexpr (NW > 1) {
        if (lane == 63) red_s[wv] = sw;
        if (lane == 0) { red_x[wv] = wx; red_y[wv] = wy; }
        __syncthreads();
        T tv = lane < NW ? red_s[lane] : A::zero();
        tv = A::template sum_scan_first<NW>(tv);
        if (wv > 0) off = lane_at(tv, wv - 1);
        Z = lane_at(tv, NW - 1);
        sx = red_x[0];
        sy = red_y[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) { sx = sx + red_x[w]; sy = sy + red_y[w]; }
    } else {
        Z = A::last(sw);
    }

    // inclusive offsets of the thread's tiles
    const T excl = A::up1(A::add(off, sw), off);
    T o[KPER];
    T run = excl;
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        run = A::add(run, v[k]);
        o[k] = run;
    }

    // End slot of every tile, y = R off_{t+1} - u0 (the expression pass C caps
    // its tiles with), made non-decreasing by a prefix maximum so that the
    // tiles' slot ranges [E_{t-1}, E_t) partition [0, N) whatever the
    // rounding of the offsets; the last tile ends at N.
    const SlotMap<F64> smap(a, Z, wu0);
    int Ek[KPER];
    int mx = 0;
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        const int t = tid * KPER + k;
        Ek[k] = 0;
        if (t < nt) Ek[k] = t == nt - 1 ? n : smap.end_of(o[k], n);
        mx = max(mx, Ek[k]);
    }
    const int sm = wave_incl_scan<OpMax>(mx);
    int e_off = 0;          // end slot of the earlier waves' tiles
    T last_prev = A::zero();  // inclusive offset of the tile before this wave's first
    if constexpr (NW > 1) {
        if (lane == 63) { red_e[wv] = sm; red_last[wv] = run; }
        __syncthreads();
        int tv = lane < NW ? red_e[lane] : 0;
        tv = max(tv, dpp<0x111>(tv, 0));  // prefix maximum over lanes 0 .. NW - 1
        if constexpr (NW > 2) tv = max(tv, dpp<0x112>(tv, 0));
        if constexpr (NW > 4) tv = max(tv, dpp<0x114>(tv, 0));
        if constexpr (NW > 8) tv = max(tv, dpp<0x118>(tv, 0));
        static_assert(NW <= 16, "one combine workgroup holds at most 16 waves");
        if (wv > 0) {
            e_off = lane_at(tv, wv - 1);
            last_prev = red_last[wv - 1];
        }
    }
    int erun = max(e_off, wave_shift_up1(sm, e_off));
    // entry t holds the inclusive offset of tile t - 1 (zero for the first)
    T before = A::up1(run, last_prev);
    int ek[KPER];
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        const int t = tid * KPER + k;
        erun = max(erun, Ek[k]);
        ek[k] = erun;
        if (t < nt) put_tab(tab + t, before, f[k], erun);
        before = o[k];
        if (t == nt - 1) {  // entry nt: the last tile's inclusive offset
            if constexpr (F64) tab[nt].off = o[k];
            else { tab[nt].off_hi = o[k].hi; tab[nt].off_lo = o[k].lo; }
        }
    }
    if (a.ecol) {  // a filter that defers its resampling: the end slots once more, as a column
        auto* ec = gbl(a.ecol);
        if constexpr (KPER == 4) {
            if (tid * KPER + KPER <= nt) {
                typedef int32_t I4 __attribute__((ext_vector_type(4)));
                *reinterpret_cast<gbl_t<I4>*>(ec + tid * KPER) = I4{ek[0], ek[1], ek[2], ek[3]};
            } else {
#pragma unroll
                for (int k = 0; k < KPER; ++k)
                    if (tid * KPER + k < nt) ec[tid * KPER + k] = ek[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < KPER; ++k)
                if (tid * KPER + k < nt) ec[tid * KPER + k] = ek[k];
        }
    }
    if (tid == 0) write_block<DT>(a, Z, gm, sx, sy, smap, tn, cnx, cny);
}

template <int DT, int KPER, int NT>
__global__ __launch_bounds__(NT) void combine_kernel(StepArgs a)
{
    combine_filter<DT, KPER, NT>(a);
}

// ---------------------------------------------------------------------------
// Grouped combine for filters of more than 4096 tiles (combine class 3): the
// tiles form groups of kGroupTiles, and two launches replace the single
// workgroup.
//   group:  one workgroup per group: the group maximum m_g, the tile factors
//           f_t^g = e^{m_t - m_g}, the group-relative exclusive prefix W_t of
//           f_t^g s_t (into the tile table), the group sum S_g and the group's
//           estimate sums; the first workgroup advances the step count;
//   finish: one workgroup per group.  Its first kTopThreads threads take the
//           values over the groups from the group records: M = max m_g,
//           c_g = e^{m_g - M}, the group offsets O_g (exclusive scan of
//           c_g S_g; Z is the total), u0, R and the groups' end slots EB_g
//           (the end slot of O_{g+1}, made non-decreasing; the last group
//           ends at N).  Every workgroup computes them with the same
//           operations on the same values, so they agree bit for bit, and
//           the first one stores the block (estimate, Z, u0, R).  Then
//           off_t = O_g + c_g W_t, f_t = c_g f_t^g, and the tiles' end slots
//           from off_{t+1}, made non-decreasing from EB_{g-1} and capped at
//           EB_g (the group's last tile ends at EB_g).
// A separate launch for the values over the groups cost ~4.7 us per step
// (2^24 particles: 16 groups), more than every finish workgroup spends
// recomputing them while its tiles' entries load.

constexpr int kGroupTiles = 1024;
constexpr int kGroupWaves = kGroupTiles / 64;
constexpr int kTopThreads = 256;  // groups of at most 2^28 particles' tiles

template <int DT>
__global__ __launch_bounds__(kGroupTiles) void combine_group_kernel(StepArgs a)
{
    constexpr bool F64 = DT == PF_F64;
    using A = CombAcc<F64 ? PF_F64 : PF_F32>;
    using T = typename A::T;
    using Rec = typename std::conditional<F64, TileRec64, TileRec32>::type;
    using Tab = typename std::conditional<F64, TileTab64, TileTab32>::type;
    using GRec = typename std::conditional<F64, GroupRec64, GroupRec32>::type;
    using Fv = typename std::conditional<F64, double, float>::type;
    using Mx = typename std::conditional<F64, double, int>::type;
    __shared__ Mx red_m[kGroupWaves];
    __shared__ T red_s[kGroupWaves];
    __shared__ T wave_off[kGroupWaves + 1];
    __shared__ Fv red_x[kGroupWaves], red_y[kGroupWaves];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = blockIdx.x, t = g * kGroupTiles + tid;
    const bool valid = t < a.ntiles;
    Rec rr{};
    if (valid) rr = static_cast<const Rec*>(a.rec)[t];
    Mx m = F64 ? (Mx)-INFINITY : (Mx)INT32_MIN;
    if (valid) {
        if constexpr (F64) m = rr.m; else m = rr.smax;
    }
    m = wave_max(m);
    if (lane == 0) red_m[wv] = m;
    __syncthreads();
    Mx gm = red_m[0];
#pragma unroll
    for (int w = 1; w < kGroupWaves; ++w) gm = red_m[w] > gm ? red_m[w] : gm;

    Fv f = 0, ex = 0, ey = 0;
    T v = A::zero();
    if (valid) {
        if constexpr (F64) {
            f = exp(rr.m - gm);
            v = f * rr.s;
        } else {
            f = __builtin_amdgcn_exp2f((float)(rr.smax - gm) * a.beta);
            v = two_prod(f, rr.s);
        }
        ex = f * rr.sx;
        ey = f * rr.sy;
    }
    const T sw = A::sum_scan(v);
    if (lane == 63) red_s[wv] = sw;
    __syncthreads();
    if (wv == 0) {
        T tv = lane < kGroupWaves ? red_s[lane] : A::zero();
        tv = A::sum_scan(tv);
        if (lane < kGroupWaves) wave_off[lane + 1] = tv;
        if (lane == 0) wave_off[0] = A::zero();
    }
    __syncthreads();
    const T off = wave_off[wv];
    const T excl = A::up1(A::add(off, sw), off);
    if (valid) {
        Tab* tab = static_cast<Tab*>(a.tab);
        tab[t].f = f;
        if constexpr (F64) tab[t].off = excl;
        else { tab[t].off_hi = excl.hi; tab[t].off_lo = excl.lo; }
    }
    ex = wave_sum(ex);
    ey = wave_sum(ey);
    if (lane == 0) { red_x[wv] = ex; red_y[wv] = ey; }
    __syncthreads();
    if (tid == 0) {
        Fv sx = red_x[0], sy = red_y[0];
        for (int w = 1; w < kGroupWaves; ++w) { sx = sx + red_x[w]; sy = sy + red_y[w]; }
        const T S = wave_off[kGroupWaves];
        GRec gr{};
        if constexpr (F64) {
            gr.m = gm; gr.s = S;
        } else {
            gr.smax = gm; gr.s_hi = S.hi; gr.s_lo = S.lo;
        }
        gr.sx = sx;
        gr.sy = sy;
        static_cast<GRec*>(a.grec)[g] = gr;
        // this step's count, read by every finish workgroup (nothing in this
        // launch reads it)
        if (g == 0) a.blk->t = a.blk->t + 1u;
    }
}

template <int DT>
__global__ __launch_bounds__(kGroupTiles) void combine_finish_kernel(StepArgs a)
{
    constexpr bool F64 = DT == PF_F64;
    constexpr int NW = kTopThreads / 64;  // waves that take the values over the groups
    using A = CombAcc<F64 ? PF_F64 : PF_F32>;
    using T = typename A::T;
    using Tab = typename std::conditional<F64, TileTab64, TileTab32>::type;
    using GRec = typename std::conditional<F64, GroupRec64, GroupRec32>::type;
    using Fv = typename std::conditional<F64, double, float>::type;
    using Mx = typename std::conditional<F64, double, int>::type;
    __shared__ T s_off[kGroupTiles];
    __shared__ int red_e[kGroupWaves];
    __shared__ Mx top_m[NW];
    __shared__ T top_s[NW];
    __shared__ T top_off[NW + 1];
    __shared__ Fv top_x[NW], top_y[NW];
    __shared__ int top_e[NW];
    __shared__ T g_off;     // this group's offset O_g
    __shared__ Fv g_c;      // its factor c_g
    __shared__ int g_e[2];  // EB_{g-1}, EB_g

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = (int)a.n;
    const int g = blockIdx.x, t0 = g * kGroupTiles, t = t0 + tid;
    const int ng = (a.ntiles + kGroupTiles - 1) / kGroupTiles;
    const int mt = min(kGroupTiles, a.ntiles - t0);
    const bool valid = tid < mt;
    Tab* tab = static_cast<Tab*>(a.tab);
    // this tile's group-relative entry: its load is in flight while the
    // values over the groups are computed
    T W = A::zero();
    Fv fg = 0;
    if (valid) {
        if constexpr (F64) W = tab[t].off; else W = ff{tab[t].off_hi, tab[t].off_lo};
        fg = tab[t].f;
    }
    const uint32_t tn = a.blk->t;  // this step (the group launch advanced the count)
    int cnx = 0, cny = 0;
    if (g == 0) read_cells<F64>(a, cnx, cny);  // the first workgroup stores the block

    // values over the groups, on threads 0 .. kTopThreads - 1 (thread i: group i)
    const bool top = tid < kTopThreads;  // whole waves
    const bool gv = tid < ng;
    GRec gr{};
    if (gv) gr = static_cast<const GRec*>(a.grec)[tid];
    Mx m = F64 ? (Mx)-INFINITY : (Mx)INT32_MIN;
    if (gv) {
        if constexpr (F64) m = gr.m; else m = gr.smax;
    }
    if (top) {
        m = wave_max(m);
        if (lane == 0) top_m[wv] = m;
    }
    __syncthreads();
    Mx gm = top_m[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) gm = top_m[w] > gm ? top_m[w] : gm;

    Fv c = 0, ex = 0, ey = 0;
    T v = A::zero(), sw = A::zero();
    if (gv) {
        if constexpr (F64) {
            c = exp(gr.m - gm);
            v = c * gr.s;
        } else {
            c = __builtin_amdgcn_exp2f((float)(gr.smax - gm) * a.beta);
            v = ff_mul_f(ff{gr.s_hi, gr.s_lo}, c);
        }
        ex = c * gr.sx;
        ey = c * gr.sy;
    }
    if (top) {
        sw = A::sum_scan(v);
        if (lane == 63) top_s[wv] = sw;
    }
    __syncthreads();
    if (wv == 0) {
        T tv = lane < NW ? top_s[lane] : A::zero();
        tv = A::sum_scan(tv);
        if (lane < NW) top_off[lane + 1] = tv;
        if (lane == 0) top_off[0] = A::zero();
    }
    __syncthreads();
    const T Z = top_off[NW];
    const SlotMap<F64> smap(a, Z, tn);
    T excl = A::zero();
    int sm = 0;
    if (top) {
        const T off = top_off[wv];
        const T incl = A::add(off, sw);
        excl = A::up1(incl, off);
        // end slot of every group (from the next group's offset), made
        // non-decreasing; the last group ends at N
        int e = 0;
        if (gv) e = tid == ng - 1 ? n : smap.end_of(incl, n);
        sm = wave_incl_scan<OpMax>(e);
        if (lane == 63) top_e[wv] = sm;
        ex = wave_sum(ex);
        ey = wave_sum(ey);
        if (lane == 0) { top_x[wv] = ex; top_y[wv] = ey; }
    }
    __syncthreads();
    if (top) {
        int carry = 0;  // end slot of the previous waves' groups
        for (int w = 0; w < wv; ++w) carry = max(carry, top_e[w]);
        sm = max(sm, carry);
        const int ep = wave_shift_up1(sm, carry);  // end slot of the previous group
        if (tid == g) {
            g_off = excl;
            g_c = c;
            g_e[0] = ep;
            g_e[1] = sm;
        }
    }
    if (g == 0 && tid == 0) {
        Fv sx = top_x[0], sy = top_y[0];
        for (int w = 1; w < NW; ++w) { sx = sx + top_x[w]; sy = sy + top_y[w]; }
        if constexpr (F64) tab[a.ntiles].off = Z;
        else { tab[a.ntiles].off_hi = Z.hi; tab[a.ntiles].off_lo = Z.lo; }
        write_block<DT, false>(a, Z, gm, sx, sy, smap, tn, cnx, cny);
    }
    __syncthreads();

    const Fv gc = g_c;
    const int Eprev = g_e[0], E = g_e[1];
    T off;
    Fv f;
    if constexpr (F64) {
        off = g_off + gc * W;
        f = gc * fg;
    } else {
        off = ff_add(g_off, ff_mul_f(W, gc));
        f = gc * fg;
    }
    s_off[tid] = off;
    __syncthreads();
    // the end slot of tile t comes from off_{t+1}; the group's last tile
    // ends where the group does
    int e = 0;
    if (valid) {
        e = tid == mt - 1 ? E : smap.end_of(s_off[tid + 1], n);
        e = min(max(e, Eprev), E);
    }
    int se = wave_incl_scan<OpMax>(e);
    if (lane == 63) red_e[wv] = se;
    __syncthreads();
    for (int w = 0; w < wv; ++w) se = max(se, red_e[w]);
    if (valid) {
        tab[t].f = f;
        tab[t].E = se;
        if constexpr (F64) tab[t].off = off;
        else { tab[t].off_hi = off.hi; tab[t].off_lo = off.lo; }
    }
}

// ---------------------------------------------------------------------------
// Pass C: the slot fill, one tile per workgroup at a time.
//
// The slots of tile t are [E_{t-1}, E_t); inside the tile, particle k owns
// the local slots [b_k, e_k), e_k its local end slot (e_i - E_{t-1},
// non-decreasing, the last one E_t - E_{t-1}) and b_k = e_{k-1} (b_0 = 0).
// Every particle that owns a slot marks its first slot b_k with k + 1: the
// marked slots are distinct and increase with k, so the ancestor of slot j is
// the last mark at or before j, which an inclusive maximum scan over the
// slots fills in (each thread a run of consecutive slots, then a wave scan
// and the wave totals).  The workgroup then writes the ancestors' propagated
// positions to the slots, each thread four consecutive slots that start at a
// global slot divisible by four (one vector store per coordinate; the first
// and last group of a round may be partial): the round's slot i lives at
// entry i + lead of the LDS slot array, lead = its first global slot mod 4.
// A tile that owns more than kSlotRound slots takes several rounds, each
// carrying the last mark of the one before; the work depends only on the
// tile's particle and slot counts, never on how the slots are spread.

constexpr int kSlotRound = 4096;  // slots per round

typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

template <int DT>
struct PassCLds {
    using Store = typename ModeT<DT>::Store;
    struct alignas(2 * sizeof(Store)) XY {
        Store x, y;
    };
    int32_t e[kTile];
    XY xy[kTile];                     // propagated positions of the tile
    alignas(8) uint16_t anc[kSlotRound + 4];  // marks, then tile-local ancestors, of the round's slots
    int32_t red[16];                  // wave totals of the scan (up to 1024 threads)
};

// One tile's pass-C inputs in registers: its particles' cumulative weights
// and propagated positions, thread tid holding particles tid + r BC.  Loaded
// one tile ahead by the streaming kernels.
template <int DT, int BC>
struct PassCIn {
    using Store = typename ModeT<DT>::Store;
    using Q = typename std::conditional<DT == PF_F64, double, float>::type;
    static constexpr int R = kTile / BC;
    Q q[R];
    Store x[R], y[R];

    __device__ void load(const StepArgs& a, int t)
    {
        const int first = t * kTile, tt = min(kTile, (int)a.n - first);
        const auto* qp = gbl(static_cast<const Q*>(a.q) + first);
        const auto* xp = gbl(static_cast<const Store*>(a.px) + first);
        const auto* yp = gbl(static_cast<const Store*>(a.py) + first);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = threadIdx.x + r * BC;
            if (k < tt) {
                q[r] = qp[k];
                x[r] = xp[k];
                y[r] = yp[k];
            }
        }
    }
    // Waits for the loads here (an empty use of every register), so that no
    // wait for them is left to code that later loads the next tile.
    __device__ void settle()
    {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            __asm__ volatile("" ::"v"(q[r]));
            __asm__ volatile("" ::"v"(x[r]));
            __asm__ volatile("" ::"v"(y[r]));
        }
    }
};

// Pass C of tile `t` of the filter described by `a`, BC threads, from its
// inputs `in` and slot map `ts`: end slots and positions to LDS, then the
// slot fill and the scatter.  Every thread takes part; the workgroup is free
// for the next tile when it returns.
template <int DT, int BC, bool WT = false>
__device__ __forceinline__ void pass_c_run(const StepArgs& a, int t, PassCLds<DT>& lds, const PassCIn<DT, BC>& in,
                                           const TileSlotsT<DT>& ts)
{
    using Store = typename ModeT<DT>::Store;
    using XY = typename PassCLds<DT>::XY;
    typedef Store Store4 __attribute__((ext_vector_type(4)));
    int32_t* s_e = lds.e;

    const int n = (int)a.n;
    const int first = t * kTile;
    const int tt = min(kTile, n - first);
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kTile / BC; ++r) {
        const int k = tid + r * BC;
        if (k < tt) {
            // local end slot, at least 0: a particle whose end slot precedes
            // the tile's first slot (the combine's prefix maximum can raise
            // it) owns no slot
            const int e = k == tt - 1 ? ts.E : ts.of(in.q[r], n);
            s_e[k] = max(e - ts.Eprev, 0);
            lds.xy[k] = XY{in.x[r], in.y[r]};
        }
    }
    __syncthreads();
    const int slots = ts.E - ts.Eprev;
    if (slots > 0) {  // uniform over the workgroup
        const int lane = tid & 63, wv = tid >> 6;
        auto* gx = gbl(static_cast<Store*>(a.sx));
        auto* gy = gbl(static_cast<Store*>(a.sy));
        auto* anc_out = a.dg_anc ? gbl(a.dg_anc) : nullptr;
        int carry = 0;  // the last mark of the previous round (none before the first)
        for (int j0 = 0; j0 < slots; j0 += kSlotRound) {
            const int nj = min(kSlotRound, slots - j0);
            const int g0 = ts.Eprev + j0;   // global slot of the round's slot 0
            const int lead = g0 & 3;        // its entry in the slot array
            const int span = nj + lead;     // entries in use
            for (int i = 4 * tid; i < span; i += 4 * BC)
                *reinterpret_cast<u16x4*>(&lds.anc[i]) = u16x4{0, 0, 0, 0};
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kTile / BC; ++r) {
                const int k = tid + r * BC;
                if (k < tt) {
                    const int b = k == 0 ? 0 : s_e[k - 1];
                    if (s_e[k] > b && b >= j0 && b < j0 + nj) lds.anc[b - j0 + lead] = (uint16_t)(k + 1);
                }
            }
            __syncthreads();
            // inclusive maximum scan of the marks; thread tid owns the
            // entries [s0, s0 + spt), spt a multiple of four (entries past
            // the span up to the next multiple of four are cleared)
            const int spt = 4 * ((span + 4 * BC - 1) / (4 * BC));
            const int s0 = tid * spt;
            int run = 0;
            for (int c = s0; c < s0 + spt && c < span; c += 4) {
                const u16x4 v = *reinterpret_cast<const u16x4*>(&lds.anc[c]);
                run = max(run, max(max((int)v.x, (int)v.y), max((int)v.z, (int)v.w)));
            }
            const int sc = wave_incl_scan<OpMax>(run);
            if (lane == 63) lds.red[wv] = sc;
            __syncthreads();
            int m = max(carry, wave_shift_up1(sc, 0));
            for (int w = 0; w < wv; ++w) m = max(m, lds.red[w]);
            for (int c = s0; c < s0 + spt && c < span; c += 4) {
                u16x4 v = *reinterpret_cast<const u16x4*>(&lds.anc[c]);
                m = max(m, (int)v.x); v.x = (uint16_t)(m - 1);
                m = max(m, (int)v.y); v.y = (uint16_t)(m - 1);
                m = max(m, (int)v.z); v.z = (uint16_t)(m - 1);
                m = max(m, (int)v.w); v.w = (uint16_t)(m - 1);
                *reinterpret_cast<u16x4*>(&lds.anc[c]) = v;
            }
            __syncthreads();
            // scatter: group q holds the round's slots 4 q - lead .. + 3, at
            // global slots g0 - lead + 4 q .. + 3
            for (int q = tid; 4 * q < span; q += BC) {
                const int i0 = 4 * q - lead;
                const int gs = g0 - lead + 4 * q;
                const u16x4 v = *reinterpret_cast<const u16x4*>(&lds.anc[4 * q]);
                if (i0 >= 0 && i0 + 4 <= nj) {  // the whole group lies in the round
                    const XY p0 = lds.xy[v.x], p1 = lds.xy[v.y], p2 = lds.xy[v.z], p3 = lds.xy[v.w];
                    if constexpr (WT && sizeof(Store4) == 16) {  // one 16-byte store per group
                        put16_wt(reinterpret_cast<gbl_t<u32x4_t>*>(gx + gs),
                                 __builtin_bit_cast(u32x4_t, Store4{p0.x, p1.x, p2.x, p3.x}));
                        put16_wt(reinterpret_cast<gbl_t<u32x4_t>*>(gy + gs),
                                 __builtin_bit_cast(u32x4_t, Store4{p0.y, p1.y, p2.y, p3.y}));
                    } else {
                        put<WT>(reinterpret_cast<gbl_t<Store4>*>(gx + gs), Store4{p0.x, p1.x, p2.x, p3.x});
                        put<WT>(reinterpret_cast<gbl_t<Store4>*>(gy + gs), Store4{p0.y, p1.y, p2.y, p3.y});
                    }
                    if (anc_out) {
                        typedef int32_t I4 __attribute__((ext_vector_type(4)));
                        *reinterpret_cast<gbl_t<I4>*>(anc_out + gs) =
                            I4{first + v.x, first + v.y, first + v.z, first + v.w};
                    }
                } else {  // the round's first or last group: slot by slot
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u;
                        if (i >= 0 && i < nj) {
                            const int k = v[u];
                            const XY pk = lds.xy[k];
                            put<WT>(gx + gs + u, pk.x);
                            put<WT>(gy + gs + u, pk.y);
                            if (anc_out) anc_out[gs + u] = first + k;
                        }
                    }
                }
            }
            carry = (int)lds.anc[nj - 1 + lead] + 1;
            __syncthreads();
        }
    }
}

// Pass C of one filter over a grid of G <= ntiles workgroups: workgroup g
// takes tiles g, g + G, ... and loads each tile's inputs while it scatters
// the one before, so a workgroup's memory latency overlaps its own slot fill.
template <int DT, int BC, bool WT = false>
__global__ __launch_bounds__(BC, BC >= 256 ? 8 : 1) void pass_c_kernel(StepArgs a)
{
    __shared__ PassCLds<DT> lds;
    const int nt = a.ntiles, G = gridDim.x;
    int t = blockIdx.x;
    PassCIn<DT, BC> cur;
    typename TileSlotsT<DT>::Raw r0;
    r0.load(a, t);
    cur.load(a, t);
    cur.settle();  // one wait for the first tile's words and inputs
    TileSlotsT<DT> ts(r0);
    for (;;) {
        const int tn = t + G;
        // the next tile's table words and inputs are loaded now and used
        // after this tile's scatter
        typename TileSlotsT<DT>::Raw rn;
        PassCIn<DT, BC> nxt;
        if (tn < nt) {  // uniform
            rn.load(a, tn);
            nxt.load(a, tn);
        }
        pass_c_run<DT, BC, WT>(a, t, lds, cur, ts);
        if (tn >= nt) break;
        t = tn;
        cur = nxt;
        ts = TileSlotsT<DT>(rn);
    }
}

// ---------------------------------------------------------------------------
// The straightforward resampler, kept for measuring what pass C gains:
// a normalising kernel writes the normalised cumulative distribution
// C_k = P_k / Z (one division per particle, C_{N-1} = 1), then one thread per
// slot j finds its ancestor, the first k with C_k >= (j + u0) / N, by binary
// search over C in global memory.  Double in the FP64 mode, float otherwise.

template <int DT>
__global__ __launch_bounds__(kBlock) void normalize_naive_kernel(StepArgs a)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int n = (int)a.n;
    if (k >= n) return;
    const int t = k / kTile;
    if constexpr (DT == PF_F64) {
        const TileTab64* tab = static_cast<const TileTab64*>(a.tab);
        const double P = tab[t].off + tab[t].f * static_cast<const double*>(a.q)[k];
        static_cast<double*>(a.cdf)[k] = k == n - 1 ? 1.0 : P / a.blk->Z;
    } else {
        const TileTab32* tab = static_cast<const TileTab32*>(a.tab);
        const float P = (tab[t].off_hi + tab[t].off_lo) + tab[t].f * static_cast<const float*>(a.q)[k];
        static_cast<float*>(a.cdf)[k] = k == n - 1 ? 1.0f : P / a.blk->Zf;
    }
}

template <int DT, int TPB>
__global__ __launch_bounds__(TPB) void resample_naive_kernel(StepArgs a)
{
    using Store = typename ModeT<DT>::Store;
    const int j = blockIdx.x * TPB + threadIdx.x;
    const int n = (int)a.n;
    if (j >= n) return;
    int lo = 0, hi = n - 1;
    if constexpr (DT == PF_F64) {
        const double u = ((double)j + a.blk->u0) / (double)n;
        const double* C = static_cast<const double*>(a.cdf);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (C[mid] >= u) hi = mid; else lo = mid + 1;
        }
    } else {
        const float u = ((float)j + (a.blk->u0_hi + a.blk->u0_lo)) / (float)n;
        const float* C = static_cast<const float*>(a.cdf);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (C[mid] >= u) hi = mid; else lo = mid + 1;
        }
    }
    static_cast<Store*>(a.sx)[j] = static_cast<const Store*>(a.px)[lo];
    static_cast<Store*>(a.sy)[j] = static_cast<const Store*>(a.py)[lo];
    if (a.dg_anc) a.dg_anc[j] = lo;
}

// ---------------------------------------------------------------------------
// Metropolis resampling (Murray, Lee & Jacob, 2016), one thread per slot: a
// chain of B steps from particle j, each proposing a uniform particle i and
// moving when u <= exp(L_i - L_k) (always when L_i >= L_k).  The log-weights
// are the integer disk terms S of pass A over the likelihood's denominator:
// L = S / denom in double in the FP64 mode; the reduced modes compare
// exp2((S_i - S_k) beta) in float.  Proposals gather S from global memory.

template <int DT>
__global__ __launch_bounds__(kBlock) void metropolis_kernel(StepArgs a)
{
    using Store = typename ModeT<DT>::Store;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const int n = (int)a.n;
    if (j >= n) return;
    const int32_t* S = a.s_all;
    const uint32_t t = a.blk->t;  // this step's index (the combine has advanced the count)
    int k = j;
    int Sk = S[k];
    double Lk = (double)Sk / a.denom;
    u32x4 w{0u, 0u, 0u, 0u};
    for (int b = 0; b < a.mh_steps; ++b) {
        if ((b & 1) == 0)
            w = philox4x32_10((uint32_t)j, t, a.stream_id, 2u + (uint32_t)(b >> 1), a.key0, a.key1);
        const uint32_t wi = (b & 1) ? w.v2 : w.v0;
        const uint32_t wu = (b & 1) ? w.v3 : w.v1;
        const int i = (int)(((uint64_t)wi * (uint64_t)(uint32_t)n) >> 32);
        const int Si = S[i];
        if constexpr (DT == PF_F64) {
            const double Li = (double)Si / a.denom;
            if (Li >= Lk || ((double)wu + 0.5) * 0x1.0p-32 <= exp(Li - Lk)) {
                k = i;
                Lk = Li;
            }
        } else {
            if (Si >= Sk ||
                ((float)(wu >> 8) + 0.5f) * 0x1.0p-24f <= __builtin_amdgcn_exp2f((float)(Si - Sk) * a.beta)) {
                k = i;
                Sk = Si;
            }
        }
    }
    static_cast<Store*>(a.sx)[j] = static_cast<const Store*>(a.px)[k];
    static_cast<Store*>(a.sy)[j] = static_cast<const Store*>(a.py)[k];
    if (a.dg_anc) a.dg_anc[j] = k;
}

// ---------------------------------------------------------------------------
// Gumbel-max multinomial resampling: thread per slot i, the argmax over all
// particles j of L_j + G_ij with G_ij = -ln(-ln u) from Philox at counter
// (j / 4, i, t, stream_id) under the key (seed low, seed high ^ 0x47756D62);
// the log weights of 1024 particles at a time are staged in LDS.  Double in
// the FP64 mode; float with the hardware log2 otherwise.  Ties keep the lower
// index.

template <int DT>
__global__ __launch_bounds__(kBlock) void gumbel_kernel(StepArgs a)
{
    using Store = typename ModeT<DT>::Store;
    using Acc = typename std::conditional<DT == PF_F64, double, float>::type;
    __shared__ Acc s_L[kTile];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int n = (int)a.n;
    const uint32_t key1 = a.key1 ^ 0x47756D62u;
    const uint32_t t = a.blk->t;  // this step's index (the combine has advanced the count)
    const float inv = (float)(1.0 / a.denom);
    Acc best = -INFINITY;
    int arg = 0;
    for (int c0 = 0; c0 < n; c0 += kTile) {
        __syncthreads();
        for (int k = threadIdx.x; k < kTile; k += kBlock) {
            const int j = c0 + k;
            if constexpr (DT == PF_F64) s_L[k] = j < n ? (double)a.s_all[j] / a.denom : -INFINITY;
            else s_L[k] = j < n ? (float)a.s_all[j] * inv : -INFINITY;
        }
        __syncthreads();
        if (i < n) {
            const int m = min(kTile, n - c0);
            for (int k = 0; k < m; k += 4) {
                const u32x4 w = philox4x32_10((uint32_t)((c0 + k) >> 2), (uint32_t)i, t, a.stream_id, a.key0, key1);
                const uint32_t ws[4] = {w.v0, w.v1, w.v2, w.v3};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (k + q < m) {
                        Acc g;
                        if constexpr (DT == PF_F64) {
                            g = -log(-log(((double)ws[q] + 0.5) * 0x1.0p-32));
                        } else {
                            const float u = ((float)(ws[q] >> 8) + 0.5f) * 0x1.0p-24f;
                            const float e = -0.6931471805599453f * __builtin_amdgcn_logf(u);  // -ln u
                            g = -0.6931471805599453f * __builtin_amdgcn_logf(e);
                        }
                        const Acc v = s_L[k + q] + g;
                        if (v > best) {
                            best = v;
                            arg = c0 + k + q;
                        }
                    }
                }
            }
        }
    }
    if (i < n) {
        static_cast<Store*>(a.sx)[i] = static_cast<const Store*>(a.px)[arg];
        static_cast<Store*>(a.sy)[i] = static_cast<const Store*>(a.py)[arg];
        if (a.dg_anc) a.dg_anc[i] = arg;
    }
}

// ---------------------------------------------------------------------------
// Rejection resampling (Murray, Lee & Jacob, 2016), one thread per slot: slot
// j first proposes particle j; a proposal c is accepted with probability
// w_c / w_max = exp(L_c - M), M the step's maximum log-likelihood (the
// combine's); after a rejection the next proposal is a uniform particle.  At
// most a.rj_cap trials; a slot that rejects them all keeps its last
// proposal.  Random words of slot j at step t: trials 2q and 2q + 1 use
// counter (j, t, stream_id, 2 + q), words 0-1 and 2-3: the first of each pair
// is the acceptance uniform, the second the next proposal
// floor(word * N / 2^32).  FP64: L = S / denom and exp in double; the
// reduced modes compare ((word >> 8) + 1/2) 2^-24 with
// exp2((S_c - S_max) beta) in float.

template <int DT>
__global__ __launch_bounds__(kBlock) void rejection_kernel(StepArgs a)
{
    using Store = typename ModeT<DT>::Store;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const int n = (int)a.n;
    if (j >= n) return;
    const int32_t* S = a.s_all;
    const DevBlock* blk = a.blk;
    const uint32_t t = blk->t;  // this step's index (the combine has advanced the count)
    int c = j;
    u32x4 w{0u, 0u, 0u, 0u};
    for (int m = 0; m < a.rj_cap; ++m) {
        if ((m & 1) == 0)
            w = philox4x32_10((uint32_t)j, t, a.stream_id, 2u + (uint32_t)(m >> 1), a.key0, a.key1);
        const uint32_t wu = (m & 1) ? w.v2 : w.v0;
        const uint32_t wi = (m & 1) ? w.v3 : w.v1;
        bool accept;
        if constexpr (DT == PF_F64) {
            accept = ((double)wu + 0.5) * 0x1.0p-32 <= exp((double)S[c] / a.denom - blk->M);
        } else {
            accept = ((float)(wu >> 8) + 0.5f) * 0x1.0p-24f <=
                     __builtin_amdgcn_exp2f((float)(S[c] - blk->Smax) * a.beta);
        }
        if (accept) break;
        if (m + 1 < a.rj_cap) c = (int)(((uint64_t)wi * (uint64_t)(uint32_t)n) >> 32);
    }
    static_cast<Store*>(a.sx)[j] = static_cast<const Store*>(a.px)[c];
    static_cast<Store*>(a.sy)[j] = static_cast<const Store*>(a.py)[c];
    if (a.dg_anc) a.dg_anc[j] = c;
}

// ---------------------------------------------------------------------------
// Normalised weights of the latest step for diagnostics: w_k = wt_k f_t / Z.
template <int DT>
__global__ __launch_bounds__(kBlock) void diag_weights_kernel(StepArgs a)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= (int)a.n) return;
    const int t = k / kTile;
    if constexpr (DT == PF_F64) {
        const TileTab64* tab = static_cast<const TileTab64*>(a.tab);
        a.dg_w[k] = a.dg_w[k] * tab[t].f / a.blk->Z;
    } else {
        const TileTab32* tab = static_cast<const TileTab32*>(a.tab);
        a.dg_w[k] = (double)((float)a.dg_w[k] * tab[t].f / a.blk->Zf);
    }
}

// Fill every stored position (including the padding) with one value.
template <typename Store>
__global__ __launch_bounds__(kBlock) void fill_kernel(Store* x, Store* y, int64_t n_pad, Store vx, Store vy)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n_pad) {
        x[k] = vx;
        y[k] = vy;
    }
}

// ---------------------------------------------------------------------------
// Batched step: many independent filters per launch.  Pass A and pass C run
// one workgroup per tile of every stepped filter; the combine one workgroup
// per filter, one launch per combine class.  Each workgroup runs exactly the
// code of the single-filter kernels on its filter's arguments, so a filter's
// results do not depend on the batch it runs in.

// The batch's plan (filter arguments, entries, tile map) does not change while
// a kernel runs, so the kernels read it through the constant address space:
// its uniform reads become scalar loads, which wait on their own counter (a
// tile's arguments can arrive while vector loads of its inputs are in flight)
// and come through the scalar cache.
template <typename T>
using cst_t = __attribute__((address_space(4))) T;
template <typename T>
__device__ __forceinline__ const cst_t<T>* cst(const T* p)
{
    return (const cst_t<T>*)p;
}

__device__ __forceinline__ int tile_entry_of(const BatchArgs& b, int gt) { return cst(b.tile_entry)[gt]; }
__device__ __forceinline__ int tile_base_of(const BatchArgs& b, int e) { return cst(b.entries)[e].tile_base; }

__device__ __forceinline__ StepArgs batch_args(const BatchArgs& b, int e)
{
    static_assert(sizeof(StepArgs) % 4 == 0, "StepArgs copies as 32-bit words");
    const cst_t<BatchEntry>* en = cst(b.entries) + e;
    StepArgs a;
    const cst_t<uint32_t>* src = reinterpret_cast<const cst_t<uint32_t>*>(cst(b.args) + en->fid);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(StepArgs) / 4); ++i) dst[i] = src[i];
    a.frame = en->frame;
    a.pitch = en->pitch;
    a.t = en->t;
    return a;
}

// Pass A over grid tiles of members whose pass-A size is kTile / PPT threads:
// all grid tiles, or the listed ones.
template <int DT, int RC, int PPT>
__global__ __launch_bounds__(kTile / PPT) void pass_a_batch_kernel(BatchArgs b)
{
    __shared__ PassALds lds;
    const int gt = b.a_tiles ? cst(b.a_tiles)[b.entry0 + (int)blockIdx.x] : (int)blockIdx.x;
    const int e = tile_entry_of(b, gt);
    const StepArgs a = batch_args(b, e);
    const int lt = gt - tile_base_of(b, e);
    if (lt >= a.ntiles) return;  // a plan captured before the filter was re-initialised smaller
    pass_a_tile<DT, RC, PPT>(a, lt, lds);
}

template <int DT, int KPER, int NT>
__global__ __launch_bounds__(NT) void combine_batch_kernel(BatchArgs b)
{
    const StepArgs a = batch_args(b, b.entry0 + (int)blockIdx.x);
    combine_filter<DT, KPER, NT>(a);
}

// A filter's arguments by its index in the batch (pass C needs no entry
// fields: no frame, pitch or step index).
__device__ __forceinline__ StepArgs batch_args_of(const BatchArgs& b, int fid)
{
    StepArgs a;
    const cst_t<uint32_t>* src = reinterpret_cast<const cst_t<uint32_t>*>(cst(b.args) + fid);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(StepArgs) / 4); ++i) dst[i] = src[i];
    return a;
}

// Batched pass C over a grid of G <= b.tiles workgroups, streaming as the
// single-filter kernel does: workgroup g takes grid tiles g, g + G, ... of
// whatever filters they belong to.  A grid tile's arguments take three
// dependent scalar loads (its map word, its entry, its filter's arguments),
// so they are pipelined over the stream: while tile t is filled, the inputs
// and slot-map words of t + G are in flight (issued from its arguments,
// complete since the last tile), and so are the arguments of t + 2G, the
// entry of t + 3G and the map word of t + 4G -- one round trip, not three,
// in front of each tile.  A tile past its filter's tiles (a plan captured
// before a smaller re-initialisation) is skipped.  The pipelined arguments
// live in scalar registers; left to itself the compiler takes 100 of them,
// which allows 7 waves per SIMD, so at least 8 workgroups per CU are asked
// for (72 SGPRs in the 16-bit modes, which then run 9 per CU, as many as
// their VGPRs and LDS allow).
template <int DT>
__global__ __launch_bounds__(pass_c_threads(DT, 1 << 30), 8) void pass_c_batch_kernel(BatchArgs b)
{
    constexpr int BC = pass_c_threads(DT, 1 << 30);
    __shared__ PassCLds<DT> lds;
    const int G = gridDim.x, T = b.tiles;
    const int g0 = blockIdx.x;  // < T: the grid has at most T workgroups
    // tile g0: everything now
    int e = tile_entry_of(b, g0);
    StepArgs a0 = batch_args_of(b, cst(b.entries)[e].fid);
    int lt0 = g0 - tile_base_of(b, e);
    PassCIn<DT, BC> cur;
    TileSlotsT<DT> ts;
    if (lt0 < a0.ntiles) {
        typename TileSlotsT<DT>::Raw r0;
        r0.load(a0, lt0);
        cur.load(a0, lt0);
        cur.settle();
        ts = TileSlotsT<DT>(r0);
    }
    // tile g0 + G: its arguments; g0 + 2G: its entry's filter and first
    // tile; g0 + 3G: its entry index (each stage only for tiles of the grid)
    StepArgs a1 = a0;
    int lt1 = 0, fid2 = 0, base2 = 0, e3 = 0;
    if (g0 + G < T) {
        e = tile_entry_of(b, g0 + G);
        a1 = batch_args_of(b, cst(b.entries)[e].fid);
        lt1 = g0 + G - tile_base_of(b, e);
    }
    if (g0 + 2 * G < T) {
        e = tile_entry_of(b, g0 + 2 * G);
        fid2 = cst(b.entries)[e].fid;
        base2 = tile_base_of(b, e);
    }
    if (g0 + 3 * G < T) e3 = tile_entry_of(b, g0 + 3 * G);
    for (int g = g0;; g += G) {
        const int g1 = g + G, g2 = g + 2 * G, g3 = g + 3 * G, g4 = g + 4 * G;
        typename TileSlotsT<DT>::Raw rn;
        PassCIn<DT, BC> nxt;
        if (g1 < T && lt1 < a1.ntiles) {  // uniform: the next tile's words and inputs
            rn.load(a1, lt1);
            nxt.load(a1, lt1);
        }
        StepArgs a2 = a1;
        int fid3 = 0, base3 = 0, e4 = 0;
        if (g2 < T) a2 = batch_args_of(b, fid2);
        if (g3 < T) {
            fid3 = cst(b.entries)[e3].fid;
            base3 = tile_base_of(b, e3);
        }
        if (g4 < T) e4 = tile_entry_of(b, g4);
        if (lt0 < a0.ntiles) pass_c_run<DT, BC>(a0, lt0, lds, cur, ts);
        if (g1 >= T) break;
        a0 = a1;
        lt0 = lt1;
        cur = nxt;
        if (lt0 < a0.ntiles) ts = TileSlotsT<DT>(rn);
        a1 = a2;
        lt1 = g2 - base2;
        fid2 = fid3;
        base2 = base3;
        e3 = e4;
    }
}

__global__ __launch_bounds__(kBlock) void gather_est_kernel(const StepArgs* args, int n, double* out)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k < n) {
        const DevBlock* blk = args[k].blk;
        out[2 * k] = blk->est_x;
        out[2 * k + 1] = blk->est_y;
    }
}

// ---------------------------------------------------------------------------
// Launchers.  With a KTiming the kernel goes through hipExtLaunchKernel, whose
// events take the start and end timestamps of the kernel's own execution.

template <typename Arg>
static hipError_t launch1(void (*kernel)(Arg), dim3 g, dim3 b, hipStream_t s, const KTiming& tm, Arg arg)
{
    if (tm.start || tm.stop) {
        void* args[] = {&arg};
        return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), g, b, args, 0, s, tm.start, tm.stop, 0);
    }
    kernel<<<g, b, 0, s>>>(arg);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_pass_a_t(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    const dim3 g((unsigned)a.ntiles);
    if (a.threads_a == 128) {  // 8 particles per thread
        if (a.r == 5) return launch1(pass_a_kernel<DT, 5, 8>, g, dim3(128), s, tm, a);
        if (a.r == 8) return launch1(pass_a_kernel<DT, 8, 8>, g, dim3(128), s, tm, a);
        return launch1(pass_a_kernel<DT, 0, 8>, g, dim3(128), s, tm, a);
    }
    if (a.threads_a == 512) {  // 2 particles per thread
        if (a.r == 5) return launch1(pass_a_kernel<DT, 5, 2>, g, dim3(512), s, tm, a);
        if (a.r == 8) return launch1(pass_a_kernel<DT, 8, 2>, g, dim3(512), s, tm, a);
        return launch1(pass_a_kernel<DT, 0, 2>, g, dim3(512), s, tm, a);
    }
    const dim3 blk(kBlockA);
    if constexpr (DT == PF_F64 || DT == PF_F32) {
    if (a.gather) {  // the previous step's resampling gathered in (never with the variants)
        if constexpr (DT != PF_F64) {
            if (a.wt) {
                if (a.r == 5) return launch1(pass_a_kernel<DT, 5, kPPT, false, true, true>, g, blk, s, tm, a);
                if (a.r == 8) return launch1(pass_a_kernel<DT, 8, kPPT, false, true, true>, g, blk, s, tm, a);
                return launch1(pass_a_kernel<DT, 0, kPPT, false, true, true>, g, blk, s, tm, a);
            }
        }
        if (a.r == 5) return launch1(pass_a_kernel<DT, 5, kPPT, false, false, true>, g, blk, s, tm, a);
        if (a.r == 8) return launch1(pass_a_kernel<DT, 8, kPPT, false, false, true>, g, blk, s, tm, a);
        return launch1(pass_a_kernel<DT, 0, kPPT, false, false, true>, g, blk, s, tm, a);
    }
    }
    if constexpr (DT != PF_F64) {
        if (a.wt && !a.naive_half) {  // a short step: outputs written through the L2
            if (a.r == 5) return launch1(pass_a_kernel<DT, 5, kPPT, false, true>, g, blk, s, tm, a);
            if (a.r == 8) return launch1(pass_a_kernel<DT, 8, kPPT, false, true>, g, blk, s, tm, a);
            return launch1(pass_a_kernel<DT, 0, kPPT, false, true>, g, blk, s, tm, a);
        }
    }
    if constexpr (DT == PF_F16) {
        if (a.naive_half) {  // the unpacked half propagation
            if (a.r == 5) return launch1(pass_a_kernel<DT, 5, kPPT, true>, g, blk, s, tm, a);
            if (a.r == 8) return launch1(pass_a_kernel<DT, 8, kPPT, true>, g, blk, s, tm, a);
            return launch1(pass_a_kernel<DT, 0, kPPT, true>, g, blk, s, tm, a);
        }
    }
    if (a.r == 5) return launch1(pass_a_kernel<DT, 5, kPPT>, g, blk, s, tm, a);
    if (a.r == 8) return launch1(pass_a_kernel<DT, 8, kPPT>, g, blk, s, tm, a);
    return launch1(pass_a_kernel<DT, 0, kPPT>, g, blk, s, tm, a);
}

template <int DT, int TPB>
static hipError_t launch_naive_res(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    const unsigned gn = (unsigned)((a.n + kBlock - 1) / kBlock);
    normalize_naive_kernel<DT><<<dim3(gn), dim3(kBlock), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch1(resample_naive_kernel<DT, TPB>, dim3((unsigned)((a.n + TPB - 1) / TPB)), dim3(TPB), s, tm, a);
}

// Workgroups of `kernel` (BC threads) resident on the whole device: the
// grid of a streaming pass C (more would only queue behind the first ones).
template <typename K>
static int resident_cap(K kernel, int threads)
{
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess || occ < 1 || cus < 1)
        return 1 << 30;  // unknown: one tile per workgroup
    return occ * cus;
}

template <int DT, int BC>
static hipError_t launch_pass_c_stream(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    if constexpr (DT != PF_F64 && BC == 256) {
        if (a.wt) {  // a short step: the state written through the L2
            static const int capw = resident_cap(pass_c_kernel<DT, BC, true>, BC);
            return launch1(pass_c_kernel<DT, BC, true>, dim3((unsigned)min(a.ntiles, capw)), dim3(BC), s, tm, a);
        }
    }
    static const int cap = resident_cap(pass_c_kernel<DT, BC>, BC);
    return launch1(pass_c_kernel<DT, BC>, dim3((unsigned)min(a.ntiles, cap)), dim3(BC), s, tm, a);
}

template <int DT>
static hipError_t launch_pass_c_t(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    const dim3 g((unsigned)a.ntiles);
    if (a.mh_steps > 0)
        return launch1(metropolis_kernel<DT>, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), s, tm, a);
    if (a.rj_cap > 0)
        return launch1(rejection_kernel<DT>, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), s, tm, a);
    if (a.gumbel)
        return launch1(gumbel_kernel<DT>, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), s, tm, a);
    if (a.naive_res) {
        switch (a.threads_c) {
        case 64: return launch_naive_res<DT, 64>(a, s, tm);
        case 128: return launch_naive_res<DT, 128>(a, s, tm);
        case 512: return launch_naive_res<DT, 512>(a, s, tm);
        case 1024: return launch_naive_res<DT, 1024>(a, s, tm);
        default: return launch_naive_res<DT, 256>(a, s, tm);
        }
    }
    // default: 512 threads while the grid is at most four tiles per CU
    // (latency-bound), else 256 (more workgroups in flight per CU, each
    // streaming tiles); the result does not depend on the choice
    const int bc = a.threads_c ? a.threads_c : pass_c_threads(DT, a.ntiles);
    switch (bc) {
    case 64: return launch_pass_c_stream<DT, 64>(a, s, tm);
    case 128: return launch_pass_c_stream<DT, 128>(a, s, tm);
    case 512: return launch_pass_c_stream<DT, 512>(a, s, tm);
    case 1024: return launch_pass_c_stream<DT, 1024>(a, s, tm);
    default: return launch_pass_c_stream<DT, 256>(a, s, tm);
    }
}

template <int DT>
static hipError_t launch_combine_grouped(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    const int ng = (a.ntiles + kGroupTiles - 1) / kGroupTiles;
    if (ng > kTopThreads) return hipErrorInvalidValue;  // N <= 2^28 keeps ng <= 256
    const dim3 gg((unsigned)ng);
    KTiming t0, t2;
    t0.start = tm.start;
    t2.stop = tm.stop;
    hipError_t e = launch1(combine_group_kernel<DT>, gg, dim3(kGroupTiles), s, t0, a);
    if (e == hipSuccess) e = launch1(combine_finish_kernel<DT>, gg, dim3(kGroupTiles), s, t2, a);
    return e;
}

template <int DT>
static hipError_t launch_combine_t(const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    switch (comb_class(a.ntiles)) {
    case 0: return launch1(combine_kernel<DT, 4, 64>, dim3(1), dim3(64), s, tm, a);
    case 1: return launch1(combine_kernel<DT, 4, 256>, dim3(1), dim3(256), s, tm, a);
    case 2: return launch1(combine_kernel<DT, 4, 1024>, dim3(1), dim3(1024), s, tm, a);
    default: return launch_combine_grouped<DT>(a, s, tm);
    }
}

#define PF_DISPATCH(dtype, call)                         \
    switch (dtype) {                                     \
    case PF_F64: { constexpr int DT = PF_F64; return call; } \
    case PF_F32: { constexpr int DT = PF_F32; return call; } \
    case PF_F16: { constexpr int DT = PF_F16; return call; } \
    case PF_BF16: { constexpr int DT = PF_BF16; return call; } \
    default: return hipErrorInvalidValue;                \
    }

hipError_t launch_pass_a(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_pass_a_t<DT>(a, s, tm))
}

hipError_t launch_combine(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_combine_t<DT>(a, s, tm))
}

hipError_t launch_pass_c(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_pass_c_t<DT>(a, s, tm))
}

template <int DT, int PPT>
static hipError_t launch_batch_pass_a_p(int rc, const BatchArgs& b, int tiles, hipStream_t s, const KTiming& tm)
{
    const dim3 g((unsigned)tiles), blk(kTile / PPT);
    if (rc == 5) return launch1(pass_a_batch_kernel<DT, 5, PPT>, g, blk, s, tm, b);
    if (rc == 8) return launch1(pass_a_batch_kernel<DT, 8, PPT>, g, blk, s, tm, b);
    return launch1(pass_a_batch_kernel<DT, 0, PPT>, g, blk, s, tm, b);
}

template <int DT>
static hipError_t launch_batch_pass_a_t(int rc, int threads_a, const BatchArgs& b, int tiles, hipStream_t s,
                                        const KTiming& tm)
{
    switch (threads_a) {
    case 128: return launch_batch_pass_a_p<DT, 8>(rc, b, tiles, s, tm);
    case 256: return launch_batch_pass_a_p<DT, 4>(rc, b, tiles, s, tm);
    case 512: return launch_batch_pass_a_p<DT, 2>(rc, b, tiles, s, tm);
    default: return hipErrorInvalidValue;
    }
}

template <int DT>
static hipError_t launch_batch_combine_t(int cls, const BatchArgs& b, int count, hipStream_t s, const KTiming& tm)
{
    const dim3 g((unsigned)count);
    switch (cls) {
    case 0: return launch1(combine_batch_kernel<DT, 4, 64>, g, dim3(64), s, tm, b);
    case 1: return launch1(combine_batch_kernel<DT, 4, 256>, g, dim3(256), s, tm, b);
    case 2: return launch1(combine_batch_kernel<DT, 4, 1024>, g, dim3(1024), s, tm, b);
    default: return hipErrorInvalidValue;  // class 3 combines per filter (launch_combine)
    }
}

hipError_t launch_batch_pass_a(int dtype, int rc, int threads_a, const BatchArgs& b, int tiles, hipStream_t s,
                              const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_batch_pass_a_t<DT>(rc, threads_a, b, tiles, s, tm))
}

hipError_t launch_batch_combine(int dtype, int cls, const BatchArgs& b, int count, hipStream_t s, const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_batch_combine_t<DT>(cls, b, count, s, tm))
}

template <int DT>
static hipError_t launch_batch_pass_c_t(const BatchArgs& b, int tiles, hipStream_t s, const KTiming& tm)
{
    constexpr int BC = pass_c_threads(DT, 1 << 30);
    static const int cap = resident_cap(pass_c_batch_kernel<DT>, BC);
    BatchArgs bb = b;
    bb.tiles = tiles;
    return launch1(pass_c_batch_kernel<DT>, dim3((unsigned)min(tiles, cap)), dim3(BC), s, tm, bb);
}

hipError_t launch_batch_pass_c(int dtype, const BatchArgs& b, int tiles, hipStream_t s, const KTiming& tm)
{
    PF_DISPATCH(dtype, launch_batch_pass_c_t<DT>(b, tiles, s, tm))
}

hipError_t launch_gather_est(const StepArgs* args, int n, double* out, hipStream_t s)
{
    gather_est_kernel<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(args, n, out);
    return hipGetLastError();
}

hipError_t launch_step(int dtype, const StepArgs& a, hipStream_t s)
{
    hipError_t e = launch_pass_a(dtype, a, s);
    if (e == hipSuccess) e = launch_combine(dtype, a, s);
    if (e == hipSuccess && !a.gather) e = launch_pass_c(dtype, a, s);  // else the next pass A resamples
    return e;
}

hipError_t launch_diag_weights(int dtype, const StepArgs& a, hipStream_t s)
{
    const dim3 g((unsigned)((a.n + kBlock - 1) / kBlock));
    switch (dtype) {
    case PF_F64: diag_weights_kernel<PF_F64><<<g, kBlock, 0, s>>>(a); break;
    case PF_F32: diag_weights_kernel<PF_F32><<<g, kBlock, 0, s>>>(a); break;
    case PF_F16: diag_weights_kernel<PF_F16><<<g, kBlock, 0, s>>>(a); break;
    case PF_BF16: diag_weights_kernel<PF_BF16><<<g, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// vx, vy: the stored value of every particle (absolute in F64, the offset
// from the origin cell in the reduced modes); converted to the storage type
// with one rounding to nearest even.
hipError_t launch_fill(int dtype, const StepArgs& a, double vx, double vy, hipStream_t s)
{
    const int64_t n_pad = (int64_t)a.ntiles * tile_of(dtype);
    const dim3 g((unsigned)((n_pad + kBlock - 1) / kBlock));
    switch (dtype) {
    case PF_F64:
        fill_kernel<double><<<g, kBlock, 0, s>>>((double*)a.sx, (double*)a.sy, n_pad, vx, vy);
        break;
    case PF_F32:
        fill_kernel<float><<<g, kBlock, 0, s>>>((float*)a.sx, (float*)a.sy, n_pad, (float)vx, (float)vy);
        break;
    case PF_F16:
        fill_kernel<_Float16><<<g, kBlock, 0, s>>>((_Float16*)a.sx, (_Float16*)a.sy, n_pad, (_Float16)vx,
                                                   (_Float16)vy);
        break;
    case PF_BF16: {
        const uint16_t bx = __builtin_bit_cast(uint16_t, (__bf16)(float)vx);
        const uint16_t by = __builtin_bit_cast(uint16_t, (__bf16)(float)vy);
        fill_kernel<uint16_t><<<g, kBlock, 0, s>>>((uint16_t*)a.sx, (uint16_t*)a.sy, n_pad, bx, by);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pf

// ---------------------------------------------------------------------------
// Static step scratch of the filters created with PF_FLAG_STATE_ONLY: the
// tile records and table, group records, propagated positions and
// tile prefix sums of one step, for callers that cannot allocate.  Each
// device holds its own copy at its own address; the array's name is only a
// host-side stand-in, so host code uses the address that
// hipGetSymbolAddress returns on each device, never the name.
static __device__ __align__(256) uint8_t scratch[PF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_addr[kMaxScratchDevices];
}  // namespace

namespace pf {

hipError_t static_scratch_setup(int device, uint8_t** out)
{
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

}  // namespace pf
