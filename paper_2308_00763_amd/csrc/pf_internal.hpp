// Internal layout shared by the kernels and the C-ABI host code of libpf.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pf.h"

namespace pf {

constexpr int kBlock = 256;        // threads per workgroup of the small kernels
// Default threads per pass-C workgroup, whatever the filter's size (a
// workgroup scatters four slots per thread; with 1024-particle tiles more
// threads would idle).  The dtype and tile count stay in the signature for
// the launchers.
__host__ __device__ constexpr int pass_c_threads(int /*dtype*/, int /*ntiles*/)
{
    return 256;
}
constexpr int kWaves = kBlock / 64;
constexpr int kTile = 1024;        // particles per tile (one pass-A and one pass-C workgroup)
constexpr int kPPT = 4;            // particles per pass-A thread
constexpr int kBlockA = kTile / kPPT;  // threads per pass-A workgroup
constexpr int kWavesA = kBlockA / 64;
constexpr int kPrefPitch = 134;    // LDS row-prefix table: u16 entries per window row (67 dwords)
constexpr int kPrefBase = 3;       // entry of P[0] in a row (so P[4l+1..4l+4] is 4-byte aligned)
constexpr int kPrefRows = 64;      // LDS row-prefix table: window rows
constexpr int kWinMaxW = 128;      // widest frame window staged in LDS
constexpr int kMaxRadius = 32;

// Combine configuration of a filter of nt tiles: class 0 = one wave of 64
// threads, four tiles per thread; 1 = 256 threads, four tiles each; 2 = 1024
// threads, four tiles each; 3 = the grouped combine (groups of 1024 tiles).
__host__ __device__ constexpr int comb_class(int nt)
{
    return nt <= 256 ? 0 : nt <= 1024 ? 1 : nt <= 4096 ? 2 : 3;
}
constexpr int kCombClasses = 4;
// Single FP16, BF16 and FP32 filters of at most this many tiles (2^23
// particles) store their bulk outputs written through the L2 (StepArgs::wt).
constexpr int kWtMaxTiles = 8192;
// Single FP64 and FP32 filters of at most this many tiles resampling
// systematically defer the resampling of each step into the next step's
// pass A (StepArgs::gather).
constexpr int kGatherMaxTiles = 1024;

// Particles per thread and tile size per precision mode.
__host__ __device__ constexpr int tile_of(int /*dtype*/) { return kTile; }
__host__ __device__ constexpr int elt_of(int dtype) { return dtype == PF_F64 ? 8 : dtype == PF_F32 ? 4 : 2; }

// Per-filter scalars in device memory (first 256 bytes of the workspace).
struct DevBlock {
    uint32_t t;           // steps taken; the combine advances it, so a step
                          // replayed from a captured graph draws fresh streams
    uint32_t pend;        // 1: the latest step's resampling is pending (the
                          // state arrays are stale; it is defined by that
                          // step's propagated positions, prefix sums, table
                          // and block, and the next pass A gathers it)
    int32_t ci_x, ci_y;   // reduced modes: origin cell of the stored positions
    int32_t cn_x, cn_y;   // reduced modes: origin cell of the next propagation
    double est_x, est_y;  // estimate of the latest step
    // double mode: normaliser, maximum log-likelihood, resampling offset and
    // R = N / Z of the latest step
    double Z, M, u0, R;
    // reduced modes: the same in float / two-float form
    float Zf, u0_hi, u0_lo, R_hi, R_lo;  // R = N / Z
    int32_t Smax;
    uint32_t pad1[2];
};
static_assert(sizeof(DevBlock) <= 256, "DevBlock must fit in 256 bytes");

// Per-tile record written by the first pass: tile maximum and sums relative
// to it.
struct TileRec64 {
    double m, s, sx, sy;
};
struct TileRec32 {
    int32_t smax;
    float s, sx, sy;
};
// Per-tile table written by the combine: cumulative weight before the tile
// (two-float in reduced modes; entry ntiles holds the total), the factor
// exp(m_t - M), and E = the end slot of the tile's last particle.
struct TileTab64 {
    double off, f;
    int32_t E, pad;
};
struct TileTab32 {
    float off_hi, off_lo, f;
    int32_t E;
};

// Grouped combine (filters of more than 4096 tiles, groups of 1024 tiles):
// per group, its maximum and sums relative to it.
struct GroupRec64 {
    double m, s, sx, sy;
};
struct GroupRec32 {
    int32_t smax;
    float s_hi, s_lo, sx, sy;
    int32_t pad[3];
};

// Workspace layout; offsets in bytes from the workspace base.
struct Layout {
    int64_t n, n_pad;
    int tile, ntiles;
    size_t blk, rec, tab, grec, sx, sy, px, py, q, dg_s, dg_w, dg_anc, cdf, s_all, px2, py2, q2, ecol, total;
};

// Whether a filter with parameters p defers its resampling into the next
// step (the second set of propagated positions and prefix sums and the
// end-slot column are then part of its workspace): FP64 or FP32, systematic
// resampling, no diagnostics, variants or static scratch, at most
// kGatherMaxTiles tiles.  Batch members never do.  (The gather reads every
// source tile's prefix sums and positions about twice, at the start of pass
// A; in the 16-bit modes that costs as much as the pass C it saves.)
inline bool gather_eligible(const pf_params& p, int ntiles)
{
    const uint32_t off = PF_FLAG_DIAGNOSTICS | PF_FLAG_STATE_ONLY | PF_FLAG_NAIVE_LIKELIHOOD |
                         PF_FLAG_NAIVE_RESAMPLE | PF_FLAG_NAIVE_HALF | PF_FLAG_METROPOLIS | PF_FLAG_REJECTION |
                         PF_FLAG_GUMBEL_MAX;
    return (p.dtype == PF_F64 || p.dtype == PF_F32) && !(p.flags & off) && ntiles <= kGatherMaxTiles;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Step scratch of a filter: the sections one step writes before it reads
// them (tile records and table, group records, propagated
// positions, tile prefix sums); offsets relative to the scratch's base.
struct ScratchLayout {
    size_t rec, tab, grec, px, py, q, total;
};

inline ScratchLayout make_scratch_layout(const pf_params& p, int ntiles, int64_t n_pad)
{
    ScratchLayout S{};
    const size_t elt = (size_t)elt_of(p.dtype);
    const size_t rec = p.dtype == PF_F64 ? sizeof(TileRec64) : sizeof(TileRec32);
    const size_t tab = p.dtype == PF_F64 ? sizeof(TileTab64) : sizeof(TileTab32);
    const size_t qel = p.dtype == PF_F64 ? 8 : 4;
    const size_t ngroups = ((size_t)ntiles + 1023) / 1024;
    size_t o = 0;
    S.rec = o; o = align256(o + rec * (size_t)ntiles);
    S.tab = o; o = align256(o + tab * (size_t)(ntiles + 1));
    S.grec = o; o = align256(o + 32 * ngroups);
    S.px = o; o = align256(o + elt * (size_t)n_pad);
    S.py = o; o = align256(o + elt * (size_t)n_pad);
    S.q = o; o = align256(o + qel * (size_t)n_pad);
    S.total = o;
    return S;
}

// Workspace layout: the block and the state (positions), then the step
// scratch (absent with PF_FLAG_STATE_ONLY: those offsets are 0 and the step
// points them into the static scratch), then the optional diagnostics and
// variant buffers, and, for a single filter (`single`) that defers its
// resampling, the second set of propagated positions and prefix sums and the
// end-slot column.
inline Layout make_layout(const pf_params& p, bool single = false)
{
    Layout L{};
    L.n = p.n_particles;
    L.tile = tile_of(p.dtype);
    L.ntiles = (int)((L.n + L.tile - 1) / L.tile);
    L.n_pad = (int64_t)L.ntiles * L.tile;
    const size_t elt = (size_t)elt_of(p.dtype);
    const size_t qel = p.dtype == PF_F64 ? 8 : 4;
    size_t o = 0;
    L.blk = o; o += 256;
    L.sx = o; o = align256(o + elt * (size_t)L.n_pad);
    L.sy = o; o = align256(o + elt * (size_t)L.n_pad);
    if (p.flags & PF_FLAG_STATE_ONLY) {
        L.rec = L.tab = L.grec = L.px = L.py = L.q = 0;
    } else {
        const ScratchLayout S = make_scratch_layout(p, L.ntiles, L.n_pad);
        L.rec = o + S.rec;
        L.tab = o + S.tab;
        L.grec = o + S.grec;
        L.px = o + S.px;
        L.py = o + S.py;
        L.q = o + S.q;
        o += S.total;
    }
    if (p.flags & PF_FLAG_DIAGNOSTICS) {
        L.dg_s = o; o = align256(o + 4 * (size_t)L.n_pad);
        L.dg_w = o; o = align256(o + 8 * (size_t)L.n_pad);
        L.dg_anc = o; o = align256(o + 4 * (size_t)L.n_pad);
    } else {
        L.dg_s = L.dg_w = L.dg_anc = 0;
    }
    if (p.flags & PF_FLAG_NAIVE_RESAMPLE) {
        L.cdf = o; o = align256(o + qel * (size_t)L.n_pad);
    } else {
        L.cdf = 0;
    }
    if (p.flags & (PF_FLAG_METROPOLIS | PF_FLAG_GUMBEL_MAX | PF_FLAG_REJECTION)) {
        L.s_all = o; o = align256(o + 4 * (size_t)L.n_pad);
    } else {
        L.s_all = 0;
    }
    if (single && gather_eligible(p, L.ntiles)) {
        L.px2 = o; o = align256(o + elt * (size_t)L.n_pad);
        L.py2 = o; o = align256(o + elt * (size_t)L.n_pad);
        L.q2 = o; o = align256(o + qel * (size_t)L.n_pad);
        L.ecol = o; o = align256(o + 4 * (size_t)L.ntiles);
    } else {
        L.px2 = L.py2 = L.q2 = L.ecol = 0;
    }
    L.total = o;
    return L;
}

// Arguments of the passes (passed by value).
struct StepArgs {
    const uint8_t* frame;
    int64_t pitch;
    int32_t W, H, r, nd;
    int64_t n;
    int32_t ntiles;
    uint32_t t, stream_id, key0, key1;  // t: host copy of the steps taken (kernels read the block's)
    int32_t fg, bg;
    double drift_x, drift_y, sigma_x, sigma_y;
    double denom;       // kappa * N_d (MEAN) or kappa (SUM)
    float beta;         // log2(e) / denom, reduced modes
    DevBlock* blk;
    void* rec;
    void* tab;
    void* grec;         // grouped combine: per-group records
    void* sx;
    void* sy;
    void* px;
    void* py;
    void* q;
    int32_t* dg_s;      // diagnostics (may be null)
    double* dg_w;
    int32_t* dg_anc;
    // implementation variants (measurement of the straightforward step)
    int32_t naive_lik;  // disk sums read every pixel from the frame
    int32_t naive_res;  // normalised CDF + per-slot binary search instead of pass C
    int32_t naive_half; // FP16: propagation one particle at a time in scalar half arithmetic
    int32_t wt;         // single-filter launches: the write-through pass A and pass C (not FP64, <= kWtMaxTiles)
    int32_t threads_a;  // pass A threads per tile: 128, 256 (default) or 512
    int32_t threads_c;  // pass C / naive resampler threads per workgroup: 64 .. 1024 (0: by tile count)
    void* cdf;          // naive resampler: normalised cumulative weights
    int32_t mh_steps;   // Metropolis resampling: steps per slot (0: systematic)
    int32_t rj_cap;     // rejection resampling: most trials per slot (0: systematic)
    int32_t gumbel;     // Gumbel-max multinomial resampling
    int32_t* s_all;     // Metropolis / Gumbel-max: integer disk terms of all particles
    // Deferred resampling (single FP64 and FP32 filters, systematic
    // resampling, at most kGatherMaxTiles tiles): pass A of step t writes its propagated
    // positions and prefix sums to set t mod 2 (set 0: px, py, q; set 1:
    // px2, py2, q2) and, when the block's pend flag is set, takes its state
    // from the previous step's set, gathered through that step's table; the
    // combine writes the tiles' end slots to ecol as well and sets pend.
    int32_t gather;
    void* px2;
    void* py2;
    void* q2;
    int32_t* ecol;
};

// One filter of a batched step: the per-step part of its arguments.
struct BatchEntry {
    const uint8_t* frame;
    int64_t pitch;
    int32_t fid;        // index of the filter's StepArgs in the batch
    int32_t tile_base;  // first tile of the filter in the step's grid
    uint32_t t;         // index of the step
    int32_t pad;
};
static_assert(sizeof(BatchEntry) == 32, "BatchEntry layout");

// Arguments of the batched passes: the filters' static arguments, this
// step's entries (one per stepped filter, grouped by combine class) and the
// map from grid tile to entry.
struct BatchArgs {
    const StepArgs* args;
    const BatchEntry* entries;
    const int32_t* tile_entry;
    const int32_t* a_tiles;  // pass A of a batch with members of several pass-A
                             // sizes: the grid tiles of each size, size by size
                             // (null: workgroup g takes grid tile g)
    int32_t entry0;     // combine: entry of the launch's first workgroup;
                        // listed pass A: index in a_tiles of its first tile
    int32_t tiles;      // pass C: tiles of the step's grid (set by its launcher)
};

// Optional timing of one launch: events stamped by the kernel's own dispatch
// (start and end of its execution), no separate event records.
struct KTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

// The static step scratch of filters created with PF_FLAG_STATE_ONLY
// (kernels.hip): PF_STATIC_SCRATCH_BYTES on every device.  With `device`
// current, static_scratch_setup looks up the array's address on that device
// (once per device; later calls return the address found then).
hipError_t static_scratch_setup(int device, uint8_t** out);

// Host-side launchers (kernels.hip).  launch_step = launch_pass_a,
// launch_combine, launch_pass_c on the same stream (no pass C for a filter
// that defers its resampling).
hipError_t launch_step(int dtype, const StepArgs& a, hipStream_t s);
hipError_t launch_pass_a(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm = KTiming());
hipError_t launch_combine(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm = KTiming());
hipError_t launch_pass_c(int dtype, const StepArgs& a, hipStream_t s, const KTiming& tm = KTiming());
hipError_t launch_fill(int dtype, const StepArgs& a, double vx, double vy, hipStream_t s);
hipError_t launch_diag_weights(int dtype, const StepArgs& a, hipStream_t s);
// Batched passes: pass A and pass C over `tiles` grid tiles, the combine over
// `count` entries of one combine class starting at b.entry0.  rc: the common
// disk radius of the batch when it is 5 or 8, else 0.  Pass A runs the
// members of pass-A size threads_a (128, 256 or 512): every grid tile when
// b.a_tiles is null, else the `tiles` listed from b.a_tiles[b.entry0].
hipError_t launch_batch_pass_a(int dtype, int rc, int threads_a, const BatchArgs& b, int tiles, hipStream_t s,
                               const KTiming& tm = KTiming());
hipError_t launch_batch_combine(int dtype, int cls, const BatchArgs& b, int count, hipStream_t s,
                                const KTiming& tm = KTiming());
hipError_t launch_batch_pass_c(int dtype, const BatchArgs& b, int tiles, hipStream_t s,
                               const KTiming& tm = KTiming());
// out[2k], out[2k+1] = estimate of filter k (device memory).
hipError_t launch_gather_est(const StepArgs* args, int n, double* out, hipStream_t s);

}  // namespace pf
