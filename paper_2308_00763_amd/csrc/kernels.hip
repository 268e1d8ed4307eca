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
//   pass C   systematic resampling as a merge of two sorted sequences: the
//            particles' end slots e_i = #{j : (j + u0)/N <= C_i} and the slots
//            0..N-1 (merge path: every workgroup takes the same number of
//            particles + slots whatever the weights), gathering the
//            propagated position of each slot's ancestor.
//
// The maximum and weighting are fused into pass A and the cumulative
// distribution is evaluated on the fly in pass C, so the six kernels of the
// paper become three, two of them wide.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "philox.hpp"
#include "pf_internal.hpp"
#include "wave.hpp"

namespace pf {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Disk sums through a row-prefix table.  The disk dx^2 + dy^2 < r^2 is, row by
// row, a run of 2 h(dy) + 1 pixels with h(dy) the largest |dx| on that row, so
// its pixel sum is a sum over rows of two differences of row-prefix sums:
// exactly the integer the per-pixel definition gives, with 2 (2r - 1) table
// reads instead of one read per pixel.  The table holds, for every row of the
// frame window a tile's particles look at, P[c] = sum of the window bytes in
// columns [0, c), as u16 (a window row is at most 128 bytes wide).

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
            plus[i] = i * kPrefPitch + (R - 1) + h + 1;
            minus[i] = i * kPrefPitch + (R - 1) - h;
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
            const uint16_t* row = p + i * kPrefPitch + (r - 1);
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
        const uint8_t* rp = frame + (int64_t)row * pitch;
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

// Half-up rounding of a reduced-precision offset to its pixel: exact in float
// for every input (floor and the fraction v - floor(v) are exact).
__device__ __forceinline__ int offset_cell(float v, int origin, int lo, int hi)
{
    v = fminf(fmaxf(v, (float)(lo - origin) - 1.0f), (float)(hi - origin) + 1.0f);
    const float fl = floorf(v);
    const int c = origin + (int)fl + ((v - fl) >= 0.5f ? 1 : 0);
    return min(max(c, lo), hi);
}

template <int DT>
struct ModeT;

template <>
struct ModeT<PF_F64> {
    static constexpr int PPT = 4;
    using Store = double;
    using Val = double;
    struct Prop {
        double dx, dy, sx, sy;
    };
    static __device__ __forceinline__ void load(const void* p, int64_t k0, Val* v)
    {
        const double2* q = reinterpret_cast<const double2*>(static_cast<const double*>(p) + k0);
        const double2 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    static __device__ __forceinline__ void store(void* p, int64_t k0, const Val* v)
    {
        double2* q = reinterpret_cast<double2*>(static_cast<double*>(p) + k0);
        q[0] = make_double2(v[0], v[1]);
        q[1] = make_double2(v[2], v[3]);
    }
    // x <- x + (d + sigma z), each operation rounded (library built without
    // contraction), as Eq. (1)-(2) are written.
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int64_t k0)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), a.t, a.stream_id, 0u, a.key0, a.key1);
            double zx, zy;
            normal_pair_f64(w, zx, zy);
            x[i] = x[i] + (pr.dx + pr.sx * zx);
            y[i] = y[i] + (pr.dy + pr.sy * zy);
        }
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
    static constexpr int PPT = 4;
    using Store = float;
    using Val = float;
    struct Prop {
        float dx, dy, sx, sy;
    };
    static __device__ __forceinline__ void load(const void* p, int64_t k0, Val* v)
    {
        const float4 a = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + k0);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
    static __device__ __forceinline__ void store(void* p, int64_t k0, const Val* v)
    {
        *reinterpret_cast<float4*>(static_cast<float*>(p) + k0) = make_float4(v[0], v[1], v[2], v[3]);
    }
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int64_t k0)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), a.t, a.stream_id, 0u, a.key0, a.key1);
            float zx, zy;
            normal_pair_f32(w, zx, zy);
            x[i] = x[i] + __builtin_fmaf(pr.sx, zx, pr.dx);
            y[i] = y[i] + __builtin_fmaf(pr.sy, zy, pr.dy);
        }
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
    static constexpr int PPT = 4;
    using Store = _Float16;
    using Val = _Float16;
    struct Prop {
        half2_t dx, dy, sx, sy;
    };
    static __device__ __forceinline__ void load(const void* p, int64_t k0, Val* v)
    {
        const uint2 a = *reinterpret_cast<const uint2*>(static_cast<const _Float16*>(p) + k0);
        const half2_t h0 = __builtin_bit_cast(half2_t, a.x), h1 = __builtin_bit_cast(half2_t, a.y);
        v[0] = h0.x; v[1] = h0.y; v[2] = h1.x; v[3] = h1.y;
    }
    static __device__ __forceinline__ void store(void* p, int64_t k0, const Val* v)
    {
        const half2_t h0 = {v[0], v[1]}, h1 = {v[2], v[3]};
        *reinterpret_cast<uint2*>(static_cast<_Float16*>(p) + k0) =
            make_uint2(__builtin_bit_cast(uint32_t, h0), __builtin_bit_cast(uint32_t, h1));
    }
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int64_t k0)
    {
#pragma unroll
        for (int i = 0; i < PPT; i += 2) {
            const u32x4 w0 = philox4x32_10((uint32_t)(k0 + i), a.t, a.stream_id, 0u, a.key0, a.key1);
            const u32x4 w1 = philox4x32_10((uint32_t)(k0 + i + 1), a.t, a.stream_id, 0u, a.key0, a.key1);
            float zx0, zy0, zx1, zy1;
            normal_pair_f32(w0, zx0, zy0);
            normal_pair_f32(w1, zx1, zy1);
            const half2_t zx = __builtin_convertvector((float2_t){zx0, zx1}, half2_t);
            const half2_t zy = __builtin_convertvector((float2_t){zy0, zy1}, half2_t);
            half2_t xx = {x[i], x[i + 1]};
            half2_t yy = {y[i], y[i + 1]};
            xx = xx + __builtin_elementwise_fma(pr.sx, zx, pr.dx);
            yy = yy + __builtin_elementwise_fma(pr.sy, zy, pr.dy);
            x[i] = xx.x; x[i + 1] = xx.y;
            y[i] = yy.x; y[i + 1] = yy.y;
        }
    }
    static __device__ __forceinline__ int cell(Val v, int origin, int lo, int hi)
    {
        return offset_cell((float)v, origin, lo, hi);
    }
};

// bfloat16: gfx950 has no packed bfloat16 multiply-add, so the state is
// widened to float, propagated there, and rounded once (to nearest even) to
// bfloat16 by the packed conversion when it is stored.  Within the step the
// likelihood and estimate use the float position in registers; the bfloat16
// rounding reaches the next step's ancestors.
template <>
struct ModeT<PF_BF16> {
    static constexpr int PPT = 4;
    using Store = uint16_t;
    using Val = float;  // widened on load
    struct Prop {
        float dx, dy, sx, sy;
    };
    static __device__ __forceinline__ void load(const void* p, int64_t k0, Val* v)
    {
        const uint2 a = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(p) + k0);
        v[0] = __uint_as_float(a.x << 16);
        v[1] = __uint_as_float(a.x & 0xFFFF0000u);
        v[2] = __uint_as_float(a.y << 16);
        v[3] = __uint_as_float(a.y & 0xFFFF0000u);
    }
    static __device__ __forceinline__ uint32_t pack(float lo, float hi)
    {
        const __bf16 a = (__bf16)lo, b = (__bf16)hi;
        return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
    static __device__ __forceinline__ void store(void* p, int64_t k0, const Val* v)
    {
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(p) + k0) = make_uint2(pack(v[0], v[1]), pack(v[2], v[3]));
    }
    static __device__ __forceinline__ void propagate(Val* x, Val* y, const Prop& pr, const StepArgs& a,
                                                     int64_t k0)
    {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const u32x4 w = philox4x32_10((uint32_t)(k0 + i), a.t, a.stream_id, 0u, a.key0, a.key1);
            float zx, zy;
            normal_pair_f32(w, zx, zy);
            x[i] = x[i] + __builtin_fmaf(pr.sx, zx, pr.dx);
            y[i] = y[i] + __builtin_fmaf(pr.sy, zy, pr.dy);
        }
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

struct PassALds {
    uint16_t pref[kPrefPitch * kPrefRows];
    int box[kWaves][4];
    double red_d[3][kWaves];
    float red_f[3][kWaves];
    int red_i[kWaves];
};

template <int DT, int RC>
__global__ __launch_bounds__(kBlock) void pass_a_kernel(StepArgs a)
{
    using M = ModeT<DT>;
    constexpr int PPT = M::PPT;
    constexpr int TILE = kBlock * PPT;
    __shared__ PassALds lds;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int tile = blockIdx.x;
    const int64_t k0 = (int64_t)tile * TILE + (int64_t)tid * PPT;
    const int r = RC > 0 ? RC : a.r;

    // Origins (reduced modes): stored offsets are relative to ci, the
    // propagated ones to cn; the drift is applied minus the origin change.
    const DevBlock* blk = a.blk;
    int cnx = 0, cny = 0;
    float ddx = 0.f, ddy = 0.f;
    if constexpr (DT != PF_F64) {
        const int cix = blk->ci_x, ciy = blk->ci_y;
        cnx = blk->cn_x; cny = blk->cn_y;
        ddx = (float)(a.drift_x - (double)(cnx - cix));
        ddy = (float)(a.drift_y - (double)(cny - ciy));
    }
    const typename M::Prop pr = make_prop<DT>(a, ddx, ddy);

    typename M::Val x[PPT], y[PPT];
    M::load(a.sx, k0, x);
    M::load(a.sy, k0, y);
    M::propagate(x, y, pr, a, k0);
    M::store(a.px, k0, x);
    M::store(a.py, k0, y);

    // Pixel cells, clamped to where clamping the disk pixels changes nothing.
    const int lox = -(r - 1), hix = a.W - 1 + (r - 1);
    const int loy = -(r - 1), hiy = a.H - 1 + (r - 1);
    int cx[PPT], cy[PPT];
    bool valid[PPT];
    int b0 = INT32_MAX, b1 = INT32_MAX, b2 = INT32_MAX, b3 = INT32_MAX;  // min x, min y, -max x, -max y
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        valid[i] = (k0 + i) < a.n;
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
    for (int w = 0; w < kWaves; ++w) {
        b0 = min(b0, lds.box[w][0]); b1 = min(b1, lds.box[w][1]);
        b2 = min(b2, lds.box[w][2]); b3 = min(b3, lds.box[w][3]);
    }
    const int bx0 = b0, by0 = b1, bx1 = -b2, by1 = -b3;

    // Disk sums over the frame window of the tile: the window's row-prefix
    // table is built in LDS.  Each wave takes every fourth window row, two
    // columns per lane; all its row loads are issued before the first scan.
    const int wx0 = bx0 - (r - 1), wy0 = by0 - (r - 1);
    const int ww = bx1 - bx0 + 2 * r - 1, wh = by1 - by0 + 2 * r - 1;
    const bool in_lds = ww <= kWinMaxW && wh <= kPrefRows;
    int S[PPT];
    if (in_lds) {
        constexpr int RPW = kPrefRows / kWaves;
        const int c0 = 2 * lane, c1 = 2 * lane + 1;
        const int col0 = min(max(wx0 + c0, 0), a.W - 1), col1 = min(max(wx0 + c1, 0), a.W - 1);
        int v[RPW];
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int yy = wv + k * kWaves;
            v[k] = 0;
            if (yy < wh) {
                const int row = min(max(wy0 + yy, 0), a.H - 1);
                const uint8_t* rp = a.frame + (int64_t)row * a.pitch;
                const int p0 = c0 < ww ? (int)rp[col0] : 0;
                const int p1 = c1 < ww ? (int)rp[col1] : 0;
                v[k] = p0 | (p1 << 16);
            }
        }
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int yy = wv + k * kWaves;
            if (yy < wh) {
                const int p0 = v[k] & 0xFFFF, p1 = v[k] >> 16;
                const int incl = wave_incl_sum(p0 + p1, lane);
                uint16_t* prow = lds.pref + yy * kPrefPitch;
                if (lane == 0) prow[0] = 0;
                if (c0 < ww) prow[c0 + 1] = (uint16_t)(incl - p1);
                if (c1 < ww) prow[c1 + 1] = (uint16_t)incl;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int ox = valid[i] ? cx[i] - bx0 : 0, oy = valid[i] ? cy[i] - by0 : 0;
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
        m = block_max<kWaves>(m, lds.red_d[0]);
        tile_m = m;
#pragma unroll
        for (int i = 0; i < PPT; ++i) wt[i] = valid[i] ? exp(L[i] - m) : 0.0;
    } else {
        int sm = INT32_MIN;
#pragma unroll
        for (int i = 0; i < PPT; ++i)
            if (valid[i]) sm = max(sm, S[i]);
        sm = block_max<kWaves>(sm, lds.red_i);
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
    sw = wave_incl_max(sw, lane);
    ex = wave_sum(ex);
    ey = wave_sum(ey);
    Acc (*red)[kWaves];
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
    Acc excl = shfl_up(incl, 1);
    if (lane == 0) excl = off;
    Acc q[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const Acc v = excl + loc[i];
        q[i] = v < incl ? v : incl;
    }
    if constexpr (DT == PF_F64) {
        double2* qp = reinterpret_cast<double2*>(static_cast<double*>(a.q) + k0);
        qp[0] = make_double2(q[0], q[1]);
        qp[1] = make_double2(q[2], q[3]);
    } else {
        *reinterpret_cast<float4*>(static_cast<float*>(a.q) + k0) = make_float4(q[0], q[1], q[2], q[3]);
    }
    if (a.dg_s) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            a.dg_s[k0 + i] = S[i];
            a.dg_w[k0 + i] = (double)wt[i];
        }
    }
    if (tid == kBlock - 1) {
        // the tile total is the last thread's inclusive value
        Acc tx = red[1][0], ty = red[2][0];
        for (int w = 1; w < kWaves; ++w) {
            tx = tx + red[1][w];
            ty = ty + red[2][w];
        }
        if constexpr (DT == PF_F64) {
            static_cast<TileRec64*>(a.rec)[tile] = TileRec64{tile_m, incl, tx, ty};
        } else {
            static_cast<TileRec32*>(a.rec)[tile] = TileRec32{tile_smax, incl, tx, ty};
        }
    }
}

// ---------------------------------------------------------------------------
// End slot of a cumulative weight P: #{j in [0, N) : (j + u0)/N <= P / Z}.

template <int DT>
struct SlotMap;

template <>
struct SlotMap<PF_F64> {
    int64_t n;
    double Z, u0, nd;
    // Every comparison is evaluated exactly as (j + u0) / N <= C with
    // C = P / Z, so the result agrees with a direct search of the strata; the
    // floor only gives the starting guess.
    __device__ int64_t operator()(double P) const
    {
        const double C = P / Z;
        double g = floor(nd * C - u0);
        g = fmin(fmax(g, -1.0), (double)(n - 1));
        int64_t j = (int64_t)g;
        while (j + 1 <= n - 1 && ((double)(j + 1) + u0) / nd <= C) ++j;
        while (j >= 0 && ((double)j + u0) / nd > C) --j;
        return j + 1;
    }
};

template <>
struct SlotMap<PF_F32> {
    int64_t n;
    ff R, mu0;  // R = N / Z, mu0 = -u0
    // floor(N P / Z - u0) + 1 in two-float arithmetic (about 44 bits).
    __device__ int64_t operator()(ff P) const
    {
        const ff Y = ff_add(ff_mul(R, P), mu0);
        int64_t g = ff_floor(Y) + 1;
        return g < 0 ? 0 : (g > n ? n : g);
    }
};

// Per-particle end slot e_i from the stored tile-local prefix q_i and the
// tile table; e of a tile's last particle is the tile's stored end slot and
// e_{N-1} = N, so consecutive tiles join exactly.
template <int DT>
struct EndSlot;

template <>
struct EndSlot<PF_F64> {
    const double* q;
    const TileTab64* tab;
    int64_t n;
    int tile;
    SlotMap<PF_F64> sm;
    __device__ EndSlot(const StepArgs& a)
        : q(static_cast<const double*>(a.q)), tab(static_cast<const TileTab64*>(a.tab)), n(a.n),
          tile(tile_of(PF_F64))
    {
        sm.n = a.n; sm.Z = a.blk->Z; sm.u0 = a.blk->u0; sm.nd = (double)a.n;
    }
    __device__ int64_t tile_end(int t) const { return tab[t].E; }
    __device__ int64_t operator()(int64_t i) const
    {
        if (i >= n - 1) return n;
        const int t = (int)(i / tile);
        if (i % tile == tile - 1) return tab[t].E;
        double P = tab[t].off + tab[t].f * q[i];
        const double Pn = tab[t + 1].off;
        P = P < Pn ? P : Pn;
        return sm(P);
    }
};

template <>
struct EndSlot<PF_F32> {
    const float* q;
    const TileTab32* tab;
    int64_t n;
    int tile;
    SlotMap<PF_F32> sm;
    __device__ EndSlot(const StepArgs& a, int tile_size)
        : q(static_cast<const float*>(a.q)), tab(static_cast<const TileTab32*>(a.tab)), n(a.n), tile(tile_size)
    {
        sm.n = a.n;
        sm.R = ff{a.blk->R_hi, a.blk->R_lo};
        sm.mu0 = ff{-a.blk->u0_hi, -a.blk->u0_lo};
    }
    __device__ int64_t tile_end(int t) const { return tab[t].E; }
    __device__ int64_t operator()(int64_t i) const
    {
        if (i >= n - 1) return n;
        const int t = (int)(i / tile);
        if (i % tile == tile - 1) return tab[t].E;
        const TileTab32 tb = tab[t];
        const TileTab32 tn = tab[t + 1];
        ff P = ff_add(ff{tb.off_hi, tb.off_lo}, two_prod(tb.f, q[i]));
        P = ff_min(P, ff{tn.off_hi, tn.off_lo});
        return sm(P);
    }
};

template <int DT>
__device__ __forceinline__ auto make_end_slot(const StepArgs& a)
{
    if constexpr (DT == PF_F64) return EndSlot<PF_F64>(a);
    else return EndSlot<PF_F32>(a, tile_of(DT));
}

// ---------------------------------------------------------------------------
// Combine: one workgroup turns the tile records into the tile table.

constexpr int kCombChunk = 8 * kBlock;  // tiles per round, 8 per thread

template <int DT>
__global__ __launch_bounds__(kBlock) void combine_kernel(StepArgs a)
{
    using Acc = typename std::conditional<DT == PF_F64, double, float>::type;
    __shared__ double red_d[3][kWaves];
    __shared__ float red_f[2][kWaves];
    __shared__ ff red_ff[kWaves];
    __shared__ int red_i[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nt = a.ntiles;
    const int tile = tile_of(DT);
    DevBlock* b = a.blk;
    const u32x4 wu = philox4x32_10(0u, a.t, a.stream_id, 1u, a.key0, a.key1);

    if constexpr (DT == PF_F64) {
        const TileRec64* rec = static_cast<const TileRec64*>(a.rec);
        TileTab64* tab = static_cast<TileTab64*>(a.tab);
        // global maximum (strided, eight loads in flight per thread)
        double m = -INFINITY;
        for (int base = 0; base < nt; base += kCombChunk) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int t = base + k * kBlock + tid;
                if (t < nt) m = fmax(m, rec[t].m);
            }
        }
        const double Mx = block_max<kWaves>(m, red_d[0]);
        SlotMap<PF_F64> sm;
        sm.n = a.n;
        sm.u0 = uniform53(wu.v0, wu.v1);
        sm.nd = (double)a.n;
        // inclusive offsets, chunk by chunk: 8 consecutive tiles per thread
        double carry = 0.0, sx = 0.0, sy = 0.0;
        // The normaliser is needed for the end slots: a first sweep sums the
        // tiles in the same order as the offsets below, so Z equals the last
        // offset bit for bit.
        for (int pass = 0; pass < 2; ++pass) {
            carry = 0.0;
            for (int base = 0; base < nt; base += kCombChunk) {
                const int t0 = base + tid * 8;
                double f[8], v[8];
                double loc = 0.0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = t0 + k;
                    f[k] = 0.0;
                    v[k] = 0.0;
                    if (t < nt) {
                        const TileRec64 rr = rec[t];
                        f[k] = exp(rr.m - Mx);
                        v[k] = f[k] * rr.s;
                        if (pass == 1) {
                            sx = sx + f[k] * rr.sx;
                            sy = sy + f[k] * rr.sy;
                        }
                    }
                    loc = loc + v[k];
                }
                double sw = wave_incl_sum(loc, lane);
                sw = wave_incl_max(sw, lane);
                __syncthreads();
                if (lane == 63) red_d[0][wv] = sw;
                __syncthreads();
                double off = carry;
                for (int w = 0; w < wv; ++w) off = off + red_d[0][w];
                const double incl = off + sw;
                double excl = shfl_up(incl, 1);
                if (lane == 0) excl = off;
                if (pass == 1) {
                    double run = 0.0;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int t = t0 + k;
                        run = run + v[k];
                        double o = excl + run;
                        o = o < incl ? o : incl;
                        if (t < nt) {
                            tab[t].f = f[k];
                            tab[t + 1].off = o;
                            tab[t].E = t == nt - 1 ? a.n : sm(o);
                        }
                    }
                }
                // carry = the chunk's last inclusive value
                double c = carry;
                for (int w = 0; w < kWaves; ++w) c = c + red_d[0][w];
                carry = c;
            }
            if (pass == 0) sm.Z = carry;
        }
        sx = block_sum<kWaves>(sx, red_d[1]);
        sy = block_sum<kWaves>(sy, red_d[2]);
        if (tid == 0) {
            tab[0].off = 0.0;
            b->M = Mx;
            b->Z = sm.Z;
            b->u0 = sm.u0;
            b->est_x = sx / sm.Z;
            b->est_y = sy / sm.Z;
        }
    } else {
        const TileRec32* rec = static_cast<const TileRec32*>(a.rec);
        TileTab32* tab = static_cast<TileTab32*>(a.tab);
        int smx = INT32_MIN;
        for (int base = 0; base < nt; base += kCombChunk) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int t = base + k * kBlock + tid;
                if (t < nt) smx = max(smx, rec[t].smax);
            }
        }
        const int Smax = block_max<kWaves>(smx, red_i);
        SlotMap<PF_F32> sm;
        sm.n = a.n;
        const uint64_t bits = ((uint64_t)wu.v0 << 21) | (uint64_t)(wu.v1 >> 11);
        const ff u0 = fast_two_sum((float)(uint32_t)(bits >> 29) * 0x1.0p-24f,
                                   (float)(uint32_t)(bits & 0x1FFFFFFFu) * 0x1.0p-53f);
        sm.mu0 = ff{-u0.hi, -u0.lo};
        ff carry{0.f, 0.f};
        float sx = 0.f, sy = 0.f;
        for (int pass = 0; pass < 2; ++pass) {
            carry = ff{0.f, 0.f};
            for (int base = 0; base < nt; base += kCombChunk) {
                const int t0 = base + tid * 8;
                float f[8], sv[8];
                ff loc{0.f, 0.f};
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = t0 + k;
                    f[k] = 0.f;
                    sv[k] = 0.f;
                    if (t < nt) {
                        const TileRec32 rr = rec[t];
                        f[k] = __builtin_amdgcn_exp2f((float)(rr.smax - Smax) * a.beta);
                        sv[k] = rr.s;
                        if (pass == 1) {
                            sx = sx + f[k] * rr.sx;
                            sy = sy + f[k] * rr.sy;
                        }
                    }
                    loc = ff_add(loc, two_prod(f[k], sv[k]));
                }
                // monotone inclusive scan of two-float totals over the wave
                ff s = loc;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const ff o{shfl_up(s.hi, d), shfl_up(s.lo, d)};
                    if (lane >= d) s = ff_add(o, s);
                }
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const ff o{shfl_up(s.hi, d), shfl_up(s.lo, d)};
                    if (lane >= d) s = ff_max(o, s);
                }
                __syncthreads();
                if (lane == 63) red_ff[wv] = s;
                __syncthreads();
                ff off = carry;
                for (int w = 0; w < wv; ++w) off = ff_add(off, red_ff[w]);
                const ff incl = ff_add(off, s);
                ff excl{shfl_up(incl.hi, 1), shfl_up(incl.lo, 1)};
                if (lane == 0) excl = off;
                if (pass == 1) {
                    ff run{0.f, 0.f}, prev = excl;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int t = t0 + k;
                        run = ff_add(run, two_prod(f[k], sv[k]));
                        ff o = ff_min(ff_add(excl, run), incl);
                        o = ff_max(o, prev);
                        prev = o;
                        if (t < nt) {
                            tab[t].f = f[k];
                            tab[t + 1].off_hi = o.hi;
                            tab[t + 1].off_lo = o.lo;
                            tab[t].E = t == nt - 1 ? (int32_t)a.n : (int32_t)sm(o);
                        }
                    }
                }
                ff c = carry;
                for (int w = 0; w < kWaves; ++w) c = ff_add(c, red_ff[w]);
                carry = c;
            }
            if (pass == 0) {
                const ff Nff = fast_two_sum((float)a.n, (float)(a.n - (int64_t)(float)a.n));
                sm.R = ff_div(Nff, carry);
            }
        }
        sx = block_sum<kWaves>(sx, red_f[0]);
        sy = block_sum<kWaves>(sy, red_f[1]);
        if (tid == 0) {
            tab[0].off_hi = 0.f;
            tab[0].off_lo = 0.f;
            const float Zf = carry.hi + carry.lo;
            const int cnx = b->cn_x, cny = b->cn_y;
            const float ox = (float)cnx + sx / Zf;
            const float oy = (float)cny + sy / Zf;
            // the estimate leaves the device as double (conversion only)
            b->est_x = (double)ox;
            b->est_y = (double)oy;
            b->Zf = Zf;
            b->Smax = Smax;
            b->R_hi = sm.R.hi;
            b->R_lo = sm.R.lo;
            b->u0_hi = u0.hi;
            b->u0_lo = u0.lo;
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
    (void)tile;
}

// ---------------------------------------------------------------------------
// Pass C: merge-path scatter.
//
// g(i) = e_i + i is strictly increasing; the merge-path split of diagonal d
// (particles among the first d merged items, a particle going before slot j
// when e_i <= j) is the first i with g(i) >= d.  It is found in two levels by
// one wave: over tiles with G_t = g(last particle of tile t) = E_t + last,
// then inside the tile; each level is a 64-ary search (every lane tests one
// candidate, a ballot picks the first true one), so a split costs a few
// memory round trips instead of a binary search's ~20.

template <typename Pred>
__device__ __forceinline__ int64_t wave_first_true(int64_t lo, int64_t hi, int lane, const Pred& pred)
{
    // first k in [lo, hi] with pred(k); pred(hi) is taken as true
    while (lo < hi) {
        const int64_t n = hi - lo;
        if (n <= 64) {
            const bool p = lane < n ? pred(lo + lane) : false;
            const uint64_t m = __ballot(p);
            return m ? lo + __builtin_ctzll(m) : hi;
        }
        const int64_t step = (n + 63) / 64;
        const int64_t k = lo + (int64_t)(lane + 1) * step - 1;
        const bool p = k < hi ? pred(k) : true;
        const uint64_t m = __ballot(p);
        if (!m) return hi;
        const int f = __builtin_ctzll(m);
        const int64_t kf = lo + (int64_t)(f + 1) * step - 1;
        const int64_t nhi = kf < hi ? kf : hi;
        lo = f == 0 ? lo : lo + (int64_t)f * step;
        hi = nhi;
    }
    return lo;
}

template <typename E>
__device__ int64_t merge_split_wave(const E& e, int64_t d, int64_t n, int tile, int ntiles, int lane)
{
    if (d >= 2 * n) return n;
    auto last_of = [&](int64_t t) { const int64_t l = (t + 1) * (int64_t)tile - 1; return l < n - 1 ? l : n - 1; };
    const int64_t t = wave_first_true(0, ntiles - 1, lane, [&](int64_t tt) {
        return e.tile_end((int)tt) + last_of(tt) >= d;
    });
    return wave_first_true(t * (int64_t)tile, last_of(t), lane, [&](int64_t i) { return e(i) + i >= d; });
}

template <int DT>
__global__ __launch_bounds__(kBlock) void pass_c_kernel(StepArgs a)
{
    using Store = typename ModeT<DT>::Store;
    constexpr int D = kScatterItems;
    __shared__ int64_t sp[2];
    __shared__ int32_t s_e[D + 1];
    __shared__ Store s_x[D + 1];
    __shared__ Store s_y[D + 1];

    const int64_t n = a.n;
    const auto e = make_end_slot<DT>(a);
    const int64_t d0 = (int64_t)blockIdx.x * D;
    const int64_t d1 = d0 + D < 2 * n ? d0 + D : 2 * n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (wv < 2) {
        const int64_t i = merge_split_wave(e, wv == 0 ? d0 : d1, n, tile_of(DT), a.ntiles, lane);
        if (lane == 0) sp[wv] = i;
    }
    __syncthreads();
    const int64_t i0 = sp[0], i1 = sp[1];
    const int64_t j0 = d0 - i0, j1 = d1 - i1;
    const int64_t iend = i1 < n - 1 ? i1 : n - 1;
    const int ni = (int)(iend - i0 + 1);
    const Store* px = static_cast<const Store*>(a.px);
    const Store* py = static_cast<const Store*>(a.py);
    for (int k = tid; k < ni; k += kBlock) {
        s_e[k] = (int32_t)e(i0 + k);
        s_x[k] = px[i0 + k];
        s_y[k] = py[i0 + k];
    }
    __syncthreads();
    Store* sx = static_cast<Store*>(a.sx);
    Store* sy = static_cast<Store*>(a.sy);
    for (int64_t j = j0 + tid; j < j1; j += kBlock) {
        // ancestor: the first particle of the range whose end slot exceeds j
        int lo = 0, hi = ni - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_e[mid] > j) hi = mid;
            else lo = mid + 1;
        }
        sx[j] = s_x[lo];
        sy[j] = s_y[lo];
        if (a.dg_anc) a.dg_anc[j] = (int32_t)(i0 + lo);
    }
}

// ---------------------------------------------------------------------------
// Normalised weights of the latest step for diagnostics: w_k = wt_k f_t / Z.
template <int DT>
__global__ __launch_bounds__(kBlock) void diag_weights_kernel(StepArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.n) return;
    const int t = (int)(k / tile_of(DT));
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
// Launchers.

template <int DT>
static hipError_t launch_pass_a_t(const StepArgs& a, hipStream_t s)
{
    const dim3 blk(kBlock);
    const dim3 ga((unsigned)a.ntiles);
    if (a.r == 5) pass_a_kernel<DT, 5><<<ga, blk, 0, s>>>(a);
    else if (a.r == 8) pass_a_kernel<DT, 8><<<ga, blk, 0, s>>>(a);
    else pass_a_kernel<DT, 0><<<ga, blk, 0, s>>>(a);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_pass_c_t(const StepArgs& a, hipStream_t s)
{
    const int64_t items = 2 * a.n;
    const dim3 gc((unsigned)((items + kScatterItems - 1) / kScatterItems));
    pass_c_kernel<DT><<<gc, dim3(kBlock), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_pass_a(int dtype, const StepArgs& a, hipStream_t s)
{
    switch (dtype) {
    case PF_F64: return launch_pass_a_t<PF_F64>(a, s);
    case PF_F32: return launch_pass_a_t<PF_F32>(a, s);
    case PF_F16: return launch_pass_a_t<PF_F16>(a, s);
    case PF_BF16: return launch_pass_a_t<PF_BF16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_combine(int dtype, const StepArgs& a, hipStream_t s)
{
    switch (dtype) {
    case PF_F64: combine_kernel<PF_F64><<<1, kBlock, 0, s>>>(a); break;
    case PF_F32: combine_kernel<PF_F32><<<1, kBlock, 0, s>>>(a); break;
    case PF_F16: combine_kernel<PF_F16><<<1, kBlock, 0, s>>>(a); break;
    case PF_BF16: combine_kernel<PF_BF16><<<1, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass_c(int dtype, const StepArgs& a, hipStream_t s)
{
    switch (dtype) {
    case PF_F64: return launch_pass_c_t<PF_F64>(a, s);
    case PF_F32: return launch_pass_c_t<PF_F32>(a, s);
    case PF_F16: return launch_pass_c_t<PF_F16>(a, s);
    case PF_BF16: return launch_pass_c_t<PF_BF16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(int dtype, const StepArgs& a, hipStream_t s)
{
    hipError_t e = launch_pass_a(dtype, a, s);
    if (e == hipSuccess) e = launch_combine(dtype, a, s);
    if (e == hipSuccess) e = launch_pass_c(dtype, a, s);
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
