// C-ABI of libpf (include/pf.h): argument checking, workspace layout,
// stream-ordered launches, and host-side conversion of the state.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pf_internal.hpp"

using namespace pf;

constexpr int kProfEv = 6;  // start and end of pass A, of the combine and of pass C

struct pf_filter {
    pf_params p;
    Layout L;
    hipStream_t stream;
    uint8_t* ws;
    StepArgs args;
    uint32_t t;
    bool poisoned;
    pf_batch* owner;  // the batch this filter belongs to, or null
    // PF_FLAG_STATE_ONLY: the device the filter was created on and the
    // address of the static step scratch there
    int device;
    uint8_t* scratch;
    // per-pass timing (pf_profile_start / pf_profile_read)
    std::vector<hipEvent_t> prof_ev;  // kProfEv events per recorded step
    uint32_t prof_max, prof_used;
};

// A batch of filters in one workspace:
//   [StepArgs x n][BatchEntry x n][tile map: int32 x total tiles]
//   [the same two for a captured step][estimates: 2n doubles]
//   [pass-A tile lists: int32 x total tiles, twice]
//   [filter 0 layout][filter 1 layout]...
// Each step uploads, from a ring of pinned host buffers, the entries of the
// stepped filters (grouped by combine class) and, when the set of stepped
// filters changed, the map from grid tile to entry and, when the stepped
// filters have several pass-A sizes, the grid tiles of each size.
constexpr int kRing = 3;

struct pf_batch {
    int32_t n;
    int dtype;
    int rc;  // common disk radius when 5 or 8, else 0
    hipStream_t stream;
    uint8_t* ws;
    int64_t total_tiles;              // tile capacity of the plan buffers
    int64_t tiles_used;               // tiles of the members as they are now
    StepArgs* d_args;
    BatchEntry* d_entries;
    int32_t* d_tile_entry;
    BatchEntry* d_g_entries;          // plan of a captured step (replays write only these)
    int32_t* d_g_tile_entry;
    int32_t* d_a_tiles;               // pass-A tile lists (members of several pass-A sizes)
    int32_t* d_g_a_tiles;
    double* d_est;
    std::vector<pf_filter*> f;
    std::vector<int> cls;            // combine class of every filter
    std::vector<int> ta;             // pass-A threads of every filter
    std::vector<size_t> slot_bytes;  // bytes of every filter's workspace share
    std::vector<StepArgs> args_host; // host copy of the filters' StepArgs
    uint8_t* h_stage[kRing];
    uint8_t* h_graph;                 // staging read by the copies of a captured step
    hipEvent_t ev[kRing];
    bool ev_used[kRing];
    int ring;
    size_t stage_bytes;
    std::vector<uint8_t> map_active;  // stepped set of the uploaded tile map
    bool map_valid;
    bool poisoned;
};

namespace {

thread_local std::string g_err = "";

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return PF_OK;
}

int hip_fail(pf_filter* h, hipError_t e, const char* what)
{
    if (h) h->poisoned = true;
    return fail(PF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int disk_count_host(int r)
{
    int n = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            if (dx * dx + dy * dy < r * r) ++n;
    return n;
}

int check_params(const pf_params* p)
{
    if (!p) return fail(PF_ERR_INVALID_ARG, "params is NULL");
    if (p->struct_size != sizeof(pf_params))
        return fail(PF_ERR_INVALID_ARG, "struct_size %u != sizeof(pf_params) %zu", p->struct_size,
                    sizeof(pf_params));
    if (p->dtype < PF_F64 || p->dtype > PF_BF16) return fail(PF_ERR_INVALID_ARG, "bad dtype %d", p->dtype);
    if (p->n_particles < 1 || p->n_particles > (int64_t(1) << 28))
        return fail(PF_ERR_INVALID_ARG, "n_particles %lld outside [1, 2^28]", (long long)p->n_particles);
    if (p->disk_radius < 1 || p->disk_radius > kMaxRadius)
        return fail(PF_ERR_INVALID_ARG, "disk_radius %d outside [1, %d]", p->disk_radius, kMaxRadius);
    if (p->width <= 2 * p->disk_radius || p->height <= 2 * p->disk_radius)
        return fail(PF_ERR_INVALID_ARG, "frame %dx%d must exceed 2 * disk_radius", p->width, p->height);
    if (p->width > (1 << 20) || p->height > (1 << 20))
        return fail(PF_ERR_INVALID_ARG, "frame %dx%d larger than 2^20", p->width, p->height);
    if (p->fg < 0 || p->fg > 255 || p->bg < 0 || p->bg > 255)
        return fail(PF_ERR_INVALID_ARG, "fg/bg must be in [0, 255]");
    if (p->lik_norm != PF_LIK_MEAN && p->lik_norm != PF_LIK_SUM)
        return fail(PF_ERR_INVALID_ARG, "bad lik_norm %d", p->lik_norm);
    if (!(p->kappa > 0) || !isfinite(p->kappa)) return fail(PF_ERR_INVALID_ARG, "kappa must be > 0");
    const double v[6] = {p->x0, p->y0, p->drift_x, p->drift_y, p->sigma_x, p->sigma_y};
    for (double d : v)
        if (!isfinite(d) || fabs(d) > 1e6) return fail(PF_ERR_INVALID_ARG, "positions/drift/sigma must be finite, |v| <= 1e6");
    if (p->sigma_x < 0 || p->sigma_y < 0) return fail(PF_ERR_INVALID_ARG, "sigma must be >= 0");
    const uint32_t known = PF_FLAG_DIAGNOSTICS | PF_FLAG_NAIVE_LIKELIHOOD | PF_FLAG_NAIVE_RESAMPLE |
                           (0xFu << PF_THREADS_A_SHIFT) | (0xFu << PF_THREADS_C_SHIFT) | PF_FLAG_METROPOLIS |
                           (0xFFu << PF_METROPOLIS_STEPS_SHIFT) | PF_FLAG_GUMBEL_MAX | PF_FLAG_REJECTION |
                           PF_FLAG_STATE_ONLY | PF_FLAG_NAIVE_HALF | PF_FLAG_TUNED;
    if (p->flags & ~known) return fail(PF_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
    const uint32_t ta = (p->flags >> PF_THREADS_A_SHIFT) & 0xF, tc = (p->flags >> PF_THREADS_C_SHIFT) & 0xF;
    if (ta != 0 && (ta < 2 || ta > 4)) return fail(PF_ERR_INVALID_ARG, "pass A threads field %u outside {2, 3, 4}", ta);
    if (tc > 5) return fail(PF_ERR_INVALID_ARG, "pass C threads field %u outside [0, 5]", tc);
    if ((p->flags & PF_FLAG_TUNED) && (ta || tc))
        return fail(PF_ERR_INVALID_ARG, "PF_FLAG_TUNED takes both threads fields from the tuning table: give them as 0");
    if ((p->flags & PF_FLAG_TUNED) && (p->flags & PF_FLAG_NAIVE_HALF))
        return fail(PF_ERR_INVALID_ARG, "PF_FLAG_NAIVE_HALF runs pass A at its default size: not with PF_FLAG_TUNED");
    const int resamplers = !!(p->flags & PF_FLAG_METROPOLIS) + !!(p->flags & PF_FLAG_NAIVE_RESAMPLE) +
                           !!(p->flags & PF_FLAG_GUMBEL_MAX) + !!(p->flags & PF_FLAG_REJECTION);
    if (resamplers > 1) return fail(PF_ERR_INVALID_ARG, "at most one resampler variant may be chosen");
    if ((p->flags & PF_FLAG_GUMBEL_MAX) && p->n_particles > 65536)
        return fail(PF_ERR_INVALID_ARG, "Gumbel-max resampling takes at most 65536 particles");
    if (!(p->flags & (PF_FLAG_METROPOLIS | PF_FLAG_REJECTION)) && ((p->flags >> PF_METROPOLIS_STEPS_SHIFT) & 0xFFu))
        return fail(PF_ERR_INVALID_ARG, "Metropolis steps or rejection trials given without their resampler");
    if ((p->flags & PF_FLAG_NAIVE_HALF) && p->dtype != PF_F16)
        return fail(PF_ERR_INVALID_ARG, "PF_FLAG_NAIVE_HALF applies to PF_F16 only");
    if ((p->flags & PF_FLAG_NAIVE_HALF) && ((p->flags >> PF_THREADS_A_SHIFT) & 0xF) != 0 &&
        ((p->flags >> PF_THREADS_A_SHIFT) & 0xF) != 3)
        return fail(PF_ERR_INVALID_ARG, "PF_FLAG_NAIVE_HALF runs pass A with 256 threads only");
    if (p->flags & PF_FLAG_STATE_ONLY) {
        if (resamplers || (p->flags & (PF_FLAG_NAIVE_LIKELIHOOD | PF_FLAG_NAIVE_HALF)))
            return fail(PF_ERR_INVALID_ARG, "PF_FLAG_STATE_ONLY takes only the default step");
        const int nt = (int)((p->n_particles + kTile - 1) / kTile);
        const size_t need = make_scratch_layout(*p, nt, (int64_t)nt * kTile).total;
        if (need > PF_STATIC_SCRATCH_BYTES)
            return fail(PF_ERR_INVALID_ARG, "PF_FLAG_STATE_ONLY: the step scratch of %lld particles needs %zu bytes, "
                        "more than the static scratch's %u", (long long)p->n_particles, need,
                        (unsigned)PF_STATIC_SCRATCH_BYTES);
    }
    return PF_OK;
}

int threads_of(uint32_t field, int dflt) { return field == 0 ? dflt : 1 << (field + 5); }

// ---------------------------------------------------------------------------
// Tuning table: (architecture, dtype, bucket) -> (pass-A threads, pass-C
// threads), one per process, guarded by g_tune_mu.

struct TuneEntry {
    std::string arch;
    int32_t dtype, bucket, ta, tc;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

constexpr int kMaxBucket = 28;

int bucket_of(int64_t n)
{
    int b = 0;
    while (b < 62 && (int64_t(1) << b) < n) ++b;
    return b;
}

bool arch_ok(const char* a)
{
    if (!a) return false;
    const size_t len = strlen(a);
    if (len < 1 || len > 31) return false;
    for (size_t i = 0; i < len; ++i) {
        const char c = a[i];
        if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9') || c == '_')) return false;
    }
    return true;
}

// The threads field of a size (0 for the default), or -1.
int field_of(int threads, bool pass_a)
{
    if (threads == 0) return 0;
    for (int f = pass_a ? 2 : 1; f <= (pass_a ? 4 : 5); ++f)
        if (threads == (1 << (f + 5))) return f;
    return -1;
}

int check_tune_entry(const char* arch, int32_t dtype, int32_t bucket, int32_t ta, int32_t tc)
{
    if (!arch_ok(arch)) return fail(PF_ERR_INVALID_ARG, "architecture name must be 1-31 characters of [A-Za-z0-9_]");
    if (dtype < PF_F64 || dtype > PF_BF16) return fail(PF_ERR_INVALID_ARG, "bad dtype %d", dtype);
    if (bucket < 0 || bucket > kMaxBucket) return fail(PF_ERR_INVALID_ARG, "bucket %d outside [0, %d]", bucket, kMaxBucket);
    if (field_of(ta, true) < 0) return fail(PF_ERR_INVALID_ARG, "pass A threads %d not in {0, 128, 256, 512}", ta);
    if (field_of(tc, false) < 0)
        return fail(PF_ERR_INVALID_ARG, "pass C threads %d not in {0, 64, 128, 256, 512, 1024}", tc);
    return PF_OK;
}

void tune_put(const TuneEntry& en)  // caller holds g_tune_mu
{
    for (TuneEntry& o : g_tune)
        if (o.arch == en.arch && o.dtype == en.dtype && o.bucket == en.bucket) {
            o = en;
            return;
        }
    g_tune.push_back(en);
}

void tune_find(const char* arch, int32_t dtype, int64_t n, int32_t* ta, int32_t* tc)
{
    const int b = bucket_of(n);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneEntry* best = nullptr;
    for (const TuneEntry& o : g_tune) {
        if (o.arch != arch || o.dtype != dtype) continue;
        const int d = std::abs(o.bucket - b), bd = best ? std::abs(best->bucket - b) : 1 << 30;
        if (d < bd || (d == bd && best && o.bucket < best->bucket)) best = &o;
    }
    *ta = best ? best->ta : 0;
    *tc = best ? best->tc : 0;
}

// Architecture name of a device without feature suffixes, cached per device.
int device_arch(int dev, std::string* out)
{
    static std::mutex mu;
    static std::vector<std::string> cache;
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0) return fail(PF_ERR_INVALID_ARG, "bad device %d", dev);
    if ((size_t)dev < cache.size() && !cache[(size_t)dev].empty()) {
        *out = cache[(size_t)dev];
        return PF_OK;
    }
    hipDeviceProp_t prop;
    const hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(PF_ERR_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    if ((size_t)dev >= cache.size()) cache.resize((size_t)dev + 1);
    cache[(size_t)dev] = a;
    *out = a;
    return PF_OK;
}

// `p` with PF_FLAG_TUNED replaced by the threads fields of the table entry
// for the stream's device (unchanged without the flag).
int resolve_tuned(const pf_params* p, hipStream_t s, pf_params* out)
{
    *out = *p;
    if (!(p->flags & PF_FLAG_TUNED)) return PF_OK;
    int dev = -1;
    const hipError_t e = hipStreamGetDevice(s, &dev);
    if (e != hipSuccess) return fail(PF_ERR_HIP, "hipStreamGetDevice: %s", hipGetErrorString(e));
    std::string arch;
    if (int rc = device_arch(dev, &arch)) return rc;
    int32_t ta = 0, tc = 0;
    tune_find(arch.c_str(), p->dtype, p->n_particles, &ta, &tc);
    const uint32_t fields = (0xFu << PF_THREADS_A_SHIFT) | (0xFu << PF_THREADS_C_SHIFT);
    out->flags = (p->flags & ~(PF_FLAG_TUNED | fields)) | ((uint32_t)field_of(ta, true) << PF_THREADS_A_SHIFT) |
                 ((uint32_t)field_of(tc, false) << PF_THREADS_C_SHIFT);
    return PF_OK;
}

int live(pf_filter* h)
{
    if (!h) return fail(PF_ERR_INVALID_ARG, "handle is NULL");
    if (h->poisoned) return fail(PF_ERR_STATE, "handle poisoned by an earlier HIP error");
    return PF_OK;
}

// Round a double to the storage precision; returns the stored bits.
uint64_t to_store_bits(int dtype, double v)
{
    switch (dtype) {
    case PF_F64: { uint64_t b; memcpy(&b, &v, 8); return b; }
    case PF_F32: { const float f = (float)v; uint32_t b; memcpy(&b, &f, 4); return b; }
    case PF_F16: { const _Float16 h = (_Float16)v; uint16_t b; memcpy(&b, &h, 2); return b; }
    default: { const __bf16 h = (__bf16)(float)v; uint16_t b; memcpy(&b, &h, 2); return b; }
    }
}

double from_store(int dtype, const uint8_t* src, int64_t k)
{
    switch (dtype) {
    case PF_F64: { double d; memcpy(&d, src + 8 * k, 8); return d; }
    case PF_F32: { float f; memcpy(&f, src + 4 * k, 4); return (double)f; }
    case PF_F16: { _Float16 h; memcpy(&h, src + 2 * k, 2); return (double)(float)h; }
    default: { uint16_t b; memcpy(&b, src + 2 * k, 2); uint32_t u = (uint32_t)b << 16; float f; memcpy(&f, &u, 4); return (double)f; }
    }
}

void* at(pf_filter* h, size_t off) { return h->ws + off; }

DevBlock read_block(pf_filter* h, hipError_t* e)
{
    DevBlock b{};
    *e = hipMemcpyAsync(&b, at(h, h->L.blk), sizeof b, hipMemcpyDeviceToHost, h->stream);
    if (*e == hipSuccess) *e = hipStreamSynchronize(h->stream);
    return b;
}

hipError_t write_block(pf_filter* h, const DevBlock& b)
{
    hipError_t e = hipMemcpyAsync(at(h, h->L.blk), &b, sizeof b, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e;
}

int floor_cell(double v) { return (int)floor(v + 0.5); }

// Fill the handle for a filter with params p (checked) over workspace ws, and
// return its initial device block and the stored value of every particle.
// `single`: a filter of its own (pf_init), which defers its resampling when
// it can; batch members never do.
void setup_filter(pf_filter* h, const pf_params& pr, uint8_t* ws, hipStream_t stream, DevBlock* blk,
                  double* vx, double* vy, bool single = false)
{
    const pf_params* p = &pr;
    const Layout L = make_layout(pr, single);
    h->p = pr;
    h->L = L;
    h->stream = stream;
    h->ws = ws;
    h->t = 0;
    h->poisoned = false;
    h->owner = nullptr;

    StepArgs& a = h->args;
    a.frame = nullptr;
    a.pitch = 0;
    a.W = p->width;
    a.H = p->height;
    a.r = p->disk_radius;
    a.nd = disk_count_host(p->disk_radius);
    a.n = p->n_particles;
    a.ntiles = L.ntiles;
    a.t = 0;
    a.stream_id = p->stream_id;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.fg = p->fg;
    a.bg = p->bg;
    a.drift_x = p->drift_x;
    a.drift_y = p->drift_y;
    a.sigma_x = p->sigma_x;
    a.sigma_y = p->sigma_y;
    a.denom = p->lik_norm == PF_LIK_MEAN ? p->kappa * (double)a.nd : p->kappa;
    a.beta = (float)(1.4426950408889634 / a.denom);
    a.blk = (DevBlock*)at(h, L.blk);
    a.sx = at(h, L.sx);
    a.sy = at(h, L.sy);
    h->device = -1;
    h->scratch = nullptr;
    if (p->flags & PF_FLAG_STATE_ONLY) {
        // the step points these into the static scratch
        a.rec = a.tab = a.grec = a.px = a.py = a.q = nullptr;
    } else {
        a.rec = at(h, L.rec);
        a.tab = at(h, L.tab);
        a.grec = at(h, L.grec);
        a.px = at(h, L.px);
        a.py = at(h, L.py);
        a.q = at(h, L.q);
    }
    if (p->flags & PF_FLAG_DIAGNOSTICS) {
        a.dg_s = (int32_t*)at(h, L.dg_s);
        a.dg_w = (double*)at(h, L.dg_w);
        a.dg_anc = (int32_t*)at(h, L.dg_anc);
    } else {
        a.dg_s = nullptr;
        a.dg_w = nullptr;
        a.dg_anc = nullptr;
    }
    a.naive_lik = (p->flags & PF_FLAG_NAIVE_LIKELIHOOD) ? 1 : 0;
    a.naive_res = (p->flags & PF_FLAG_NAIVE_RESAMPLE) ? 1 : 0;
    a.naive_half = (p->flags & PF_FLAG_NAIVE_HALF) ? 1 : 0;
    // a short 16-bit step stores its bulk outputs written through the L2
    // (single-filter launches at the default sizes; batches store plainly)
    a.wt = p->dtype != PF_F64 && a.ntiles <= kWtMaxTiles ? 1 : 0;
    a.threads_a = threads_of((p->flags >> PF_THREADS_A_SHIFT) & 0xF, kBlockA);
    a.threads_c = threads_of((p->flags >> PF_THREADS_C_SHIFT) & 0xF, 0);
    a.cdf = a.naive_res ? at(h, L.cdf) : nullptr;
    a.mh_steps = 0;
    a.gumbel = (p->flags & PF_FLAG_GUMBEL_MAX) ? 1 : 0;
    if (p->flags & PF_FLAG_METROPOLIS) {
        const int steps = (int)((p->flags >> PF_METROPOLIS_STEPS_SHIFT) & 0xFFu);
        a.mh_steps = steps == 0 ? 32 : steps;
    }
    a.rj_cap = 0;
    if (p->flags & PF_FLAG_REJECTION) {
        const int v = (int)((p->flags >> PF_METROPOLIS_STEPS_SHIFT) & 0xFFu);
        a.rj_cap = v == 0 ? 4096 : 64 * v;
    }
    a.s_all = (p->flags & (PF_FLAG_METROPOLIS | PF_FLAG_GUMBEL_MAX | PF_FLAG_REJECTION)) ? (int32_t*)at(h, L.s_all)
                                                                                        : nullptr;
    // deferred resampling: at the default sizes (the gather assigns four slots
    // to each of 256 threads; a filter given a pass-C size wants its pass C)
    a.gather = L.px2 != 0 && a.threads_a == kBlockA && ((p->flags >> PF_THREADS_C_SHIFT) & 0xF) == 0 ? 1 : 0;
    a.px2 = a.gather ? at(h, L.px2) : nullptr;
    a.py2 = a.gather ? at(h, L.py2) : nullptr;
    a.q2 = a.gather ? at(h, L.q2) : nullptr;
    a.ecol = a.gather ? (int32_t*)at(h, L.ecol) : nullptr;

    DevBlock b{};
    *vx = p->x0;
    *vy = p->y0;
    if (p->dtype != PF_F64) {
        b.ci_x = floor_cell(p->x0);
        b.ci_y = floor_cell(p->y0);
        b.cn_x = floor_cell(p->x0 + p->drift_x);
        b.cn_y = floor_cell(p->y0 + p->drift_y);
        *vx = p->x0 - (double)b.ci_x;
        *vy = p->y0 - (double)b.ci_y;
    }
    b.est_x = p->x0;
    b.est_y = p->y0;
    *blk = b;
}

}  // namespace

extern "C" {

int pf_abi_version(void) { return PF_ABI_VERSION; }

const char* pf_last_error(void) { return g_err.c_str(); }

int pf_tune_set(const char* arch, int32_t dtype, int32_t bucket, int32_t threads_a, int32_t threads_c)
{
    if (int rc = check_tune_entry(arch, dtype, bucket, threads_a, threads_c)) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_put(TuneEntry{arch, dtype, bucket, threads_a, threads_c});
    return ok();
}

int pf_tune_load(const char* path, int32_t* out_entries)
{
    if (!path) return fail(PF_ERR_INVALID_ARG, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return fail(PF_ERR_INVALID_ARG, "cannot open tuning table %s", path);
    std::vector<TuneEntry> got;
    char line[512];
    int ln = 0, rc = PF_OK;
    while (rc == PF_OK && fgets(line, sizeof line, f)) {
        ++ln;
        if (!strchr(line, '\n') && !feof(f)) {
            rc = fail(PF_ERR_INVALID_ARG, "%s:%d: line longer than %zu characters", path, ln, sizeof line - 2);
            break;
        }
        if (char* hash = strchr(line, '#')) *hash = '\0';
        char arch[64], dt[16], extra[8];
        int bucket = 0, ta = 0, tc = 0;
        const int got_n = sscanf(line, "%63s %15s %d %d %d %7s", arch, dt, &bucket, &ta, &tc, extra);
        if (got_n <= 0) continue;  // blank
        if (got_n != 5) {
            rc = fail(PF_ERR_INVALID_ARG, "%s:%d: expected `arch dtype bucket threads_a threads_c`", path, ln);
            break;
        }
        const int dtype = !strcmp(dt, "f64") ? PF_F64 : !strcmp(dt, "f32") ? PF_F32 : !strcmp(dt, "f16") ? PF_F16
                        : !strcmp(dt, "bf16") ? PF_BF16 : -1;
        if (dtype < 0) {
            rc = fail(PF_ERR_INVALID_ARG, "%s:%d: dtype %s is not one of f64 f32 f16 bf16", path, ln, dt);
            break;
        }
        if (check_tune_entry(arch, dtype, bucket, ta, tc)) {
            rc = fail(PF_ERR_INVALID_ARG, "%s:%d: %s", path, ln, g_err.c_str());
            break;
        }
        got.push_back(TuneEntry{arch, dtype, bucket, ta, tc});
    }
    if (rc == PF_OK && ferror(f)) rc = fail(PF_ERR_INVALID_ARG, "error reading %s", path);
    fclose(f);
    if (rc != PF_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const TuneEntry& en : got) tune_put(en);
    }
    if (out_entries) *out_entries = (int32_t)got.size();
    return ok();
}

int pf_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return ok();
}

int pf_tune_lookup(const char* arch, int32_t dtype, int64_t n, int32_t* threads_a, int32_t* threads_c)
{
    if (!arch_ok(arch)) return fail(PF_ERR_INVALID_ARG, "architecture name must be 1-31 characters of [A-Za-z0-9_]");
    if (dtype < PF_F64 || dtype > PF_BF16) return fail(PF_ERR_INVALID_ARG, "bad dtype %d", dtype);
    if (n < 1) return fail(PF_ERR_INVALID_ARG, "n %lld < 1", (long long)n);
    if (!threads_a || !threads_c) return fail(PF_ERR_INVALID_ARG, "output is NULL");
    tune_find(arch, dtype, n, threads_a, threads_c);
    return ok();
}

int pf_launch_config(pf_filter* h, int32_t* threads_a, int32_t* threads_c)
{
    if (!h) return fail(PF_ERR_INVALID_ARG, "handle is NULL");
    if (!threads_a || !threads_c) return fail(PF_ERR_INVALID_ARG, "output is NULL");
    *threads_a = h->args.threads_a;
    if (h->owner)
        *threads_c = pass_c_threads(h->p.dtype, 1 << 30);
    else if (h->args.threads_c)
        *threads_c = h->args.threads_c;
    else
        *threads_c = h->args.naive_res ? 256 : pass_c_threads(h->p.dtype, h->L.ntiles);
    return ok();
}

int pf_workspace_bytes(const pf_params* p, size_t* out_bytes)
{
    if (int rc = check_params(p)) return rc;
    if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
    *out_bytes = make_layout(*p, true).total;
    return ok();
}

int pf_member_bytes(const pf_params* p, size_t* out_bytes)
{
    if (int rc = check_params(p)) return rc;
    if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
    *out_bytes = make_layout(*p).total;
    return ok();
}

int pf_init(const pf_params* p_in, void* d_workspace, size_t workspace_bytes, void* hip_stream, pf_filter** out)
{
    if (int rc = check_params(p_in)) return rc;
    if (!out) return fail(PF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    pf_params tuned;
    if (int rc = resolve_tuned(p_in, (hipStream_t)hip_stream, &tuned)) return rc;
    const pf_params* p = &tuned;
    if (!d_workspace) return fail(PF_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(PF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const Layout L = make_layout(*p, true);
    if (workspace_bytes < L.total)
        return fail(PF_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, L.total);

    pf_filter* h = new (std::nothrow) pf_filter{};
    if (!h) return fail(PF_ERR_INVALID_ARG, "out of host memory");
    DevBlock b;
    double vx, vy;
    setup_filter(h, *p, (uint8_t*)d_workspace, (hipStream_t)hip_stream, &b, &vx, &vy, true);
    hipError_t e = hipSuccess;
    if (p->flags & PF_FLAG_STATE_ONLY) {
        // set-up of the static step scratch on the stream's device, with that
        // device current
        int cur = 0;
        e = hipGetDevice(&cur);
        if (e == hipSuccess) e = hipStreamGetDevice(h->stream, &h->device);
        if (e == hipSuccess && h->device != cur) e = hipSetDevice(h->device);
        if (e == hipSuccess) e = static_scratch_setup(h->device, &h->scratch);
        if (h->device >= 0 && h->device != cur) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
    }
    if (e == hipSuccess) e = write_block(h, b);
    if (e == hipSuccess) e = launch_fill(p->dtype, h->args, vx, vy, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        int rc = hip_fail(h, e, "pf_init");
        delete h;
        return rc;
    }
    *out = h;
    return ok();
}

int pf_step(pf_filter* h, const uint8_t* d_frame, int64_t row_pitch)
{
    if (int rc = live(h)) return rc;
    if (h->p.flags & PF_FLAG_STATE_ONLY)
        return fail(PF_ERR_INVALID_ARG, "a PF_FLAG_STATE_ONLY filter steps through pf_step_static_scratch");
    if (!d_frame) return fail(PF_ERR_INVALID_ARG, "frame is NULL");
    if (row_pitch < h->p.width) return fail(PF_ERR_INVALID_ARG, "row_pitch %lld < width %d", (long long)row_pitch, h->p.width);
    if (h->t == UINT32_MAX) return fail(PF_ERR_INVALID_ARG, "step counter exhausted");
    StepArgs a = h->args;
    a.frame = d_frame;
    a.pitch = row_pitch;
    a.t = h->t + 1;
    hipError_t e;
    if (h->prof_used < h->prof_max) {
        hipEvent_t* ev = &h->prof_ev[kProfEv * (size_t)h->prof_used];
        KTiming ta, tb, tc;
        ta.start = ev[0]; ta.stop = ev[1];
        tb.start = ev[2]; tb.stop = ev[3];
        tc.start = ev[4]; tc.stop = ev[5];
        e = launch_pass_a(h->p.dtype, a, h->stream, ta);
        if (e == hipSuccess) e = launch_combine(h->p.dtype, a, h->stream, tb);
        if (e == hipSuccess && !a.gather) e = launch_pass_c(h->p.dtype, a, h->stream, tc);
        ++h->prof_used;
    } else {
        e = launch_step(h->p.dtype, a, h->stream);
    }
    if (e == hipSuccess && a.dg_w) e = launch_diag_weights(h->p.dtype, a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "pf_step launch");
    h->t = a.t;
    return ok();
}

int pf_step_static_scratch(pf_filter* h, const uint8_t* d_frame, int64_t row_pitch)
{
    if (int rc = live(h)) return rc;
    if (!(h->p.flags & PF_FLAG_STATE_ONLY) || !h->scratch)
        return fail(PF_ERR_INVALID_ARG, "pf_step_static_scratch needs a filter created with PF_FLAG_STATE_ONLY");
    if (!d_frame) return fail(PF_ERR_INVALID_ARG, "frame is NULL");
    if (row_pitch < h->p.width) return fail(PF_ERR_INVALID_ARG, "row_pitch %lld < width %d", (long long)row_pitch, h->p.width);
    if (h->t == UINT32_MAX) return fail(PF_ERR_INVALID_ARG, "step counter exhausted");
    int dev = -1;
    hipError_t e = hipStreamGetDevice(h->stream, &dev);
    if (e != hipSuccess) return hip_fail(h, e, "pf_step_static_scratch");
    if (dev != h->device)
        return fail(PF_ERR_INVALID_ARG, "the filter's stream runs on device %d, its scratch was set up on %d", dev,
                    h->device);
    const ScratchLayout S = make_scratch_layout(h->p, h->L.ntiles, h->L.n_pad);
    StepArgs a = h->args;
    a.frame = d_frame;
    a.pitch = row_pitch;
    a.t = h->t + 1;
    a.rec = h->scratch + S.rec;
    a.tab = h->scratch + S.tab;
    a.grec = h->scratch + S.grec;
    a.px = h->scratch + S.px;
    a.py = h->scratch + S.py;
    a.q = h->scratch + S.q;
    e = launch_step(h->p.dtype, a, h->stream);
    if (e == hipSuccess && a.dg_w) e = launch_diag_weights(h->p.dtype, a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "pf_step_static_scratch launch");
    h->t = a.t;
    return ok();
}

int pf_estimate(pf_filter* h, double out_xy[2])
{
    if (int rc = live(h)) return rc;
    if (!out_xy) return fail(PF_ERR_INVALID_ARG, "out_xy is NULL");
    hipError_t e;
    const DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_estimate");
    out_xy[0] = b.est_x;
    out_xy[1] = b.est_y;
    return ok();
}

int pf_estimate_async(pf_filter* h, double* d_out_xy)
{
    if (int rc = live(h)) return rc;
    if (!d_out_xy) return fail(PF_ERR_INVALID_ARG, "d_out_xy is NULL");
    hipError_t e = hipMemcpyAsync(d_out_xy, (uint8_t*)at(h, h->L.blk) + offsetof(DevBlock, est_x),
                                  2 * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "pf_estimate_async");
    return ok();
}

static int export_positions(pf_filter* h, size_t off_x, size_t off_y, double* x, double* y, const DevBlock& b)
{
    const int64_t n = h->p.n_particles;
    const int dt = h->p.dtype;
    const size_t bytes = (size_t)n * (size_t)elt_of(dt);
    std::vector<uint8_t> buf(bytes);
    const size_t offs[2] = {off_x, off_y};
    double* dst[2] = {x, y};
    const double org[2] = {dt == PF_F64 ? 0.0 : (double)b.ci_x, dt == PF_F64 ? 0.0 : (double)b.ci_y};
    for (int c = 0; c < 2; ++c) {
        if (!dst[c]) continue;
        hipError_t e = hipMemcpyAsync(buf.data(), at(h, offs[c]), bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "export");
        for (int64_t k = 0; k < n; ++k) dst[c][k] = org[c] + from_store(dt, buf.data(), k);
    }
    return PF_OK;
}

// The arguments of a filter that defers its resampling with set 0 pointing
// at the set that step t wrote (the passes read set 0 unless they gather).
static StepArgs args_of_set(const pf_filter* h, uint32_t t)
{
    StepArgs a = h->args;
    if (a.gather && (t & 1u)) {
        a.px = a.px2;
        a.py = a.py2;
        a.q = a.q2;
    }
    return a;
}

// Offsets of the propagated positions that step t wrote.
static void prop_offsets(const pf_filter* h, uint32_t t, size_t* ox, size_t* oy)
{
    const bool odd = h->args.gather && (t & 1u);
    *ox = odd ? h->L.px2 : h->L.px;
    *oy = odd ? h->L.py2 : h->L.py;
}

// Runs the pending resampling of the latest step (pass C over the set it
// wrote) and clears the flag in *b and on the device.
static int materialize(pf_filter* h, DevBlock* b)
{
    const StepArgs a = args_of_set(h, b->t);
    hipError_t e = launch_pass_c(h->p.dtype, a, h->stream);
    if (e == hipSuccess) {
        b->pend = 0;
        e = write_block(h, *b);
    }
    if (e != hipSuccess) return hip_fail(h, e, "resampling of the latest step");
    return PF_OK;
}

int pf_export(pf_filter* h, double* x, double* y, double* w_norm, int32_t* anc, uint32_t* t)
{
    if (int rc = live(h)) return rc;
    const bool diag = (h->p.flags & PF_FLAG_DIAGNOSTICS) != 0;
    if ((w_norm || anc) && !diag) return fail(PF_ERR_INVALID_ARG, "w_norm/anc need PF_FLAG_DIAGNOSTICS");
    hipError_t e;
    DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_export");
    if ((w_norm || anc) && b.t == 0) return fail(PF_ERR_INVALID_ARG, "no step taken yet");
    if ((x || y) && b.pend) {
        if (int rc = materialize(h, &b)) return rc;
    }
    if (int rc = export_positions(h, h->L.sx, h->L.sy, x, y, b)) return rc;
    const int64_t n = h->p.n_particles;
    if (w_norm) {
        e = hipMemcpyAsync(w_norm, at(h, h->L.dg_w), (size_t)n * 8, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "pf_export w_norm");
    }
    if (anc) {
        e = hipMemcpyAsync(anc, at(h, h->L.dg_anc), (size_t)n * 4, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "pf_export anc");
    }
    if (t) *t = b.t;  // the device count (also right after steps replayed from a graph)
    h->t = b.t;
    return ok();
}

int pf_export_step(pf_filter* h, double* x_prop, double* y_prop, int32_t* disk_sum)
{
    if (int rc = live(h)) return rc;
    if (disk_sum && !(h->p.flags & PF_FLAG_DIAGNOSTICS))
        return fail(PF_ERR_INVALID_ARG, "disk_sum needs PF_FLAG_DIAGNOSTICS");
    hipError_t e;
    const DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_export_step");
    if (b.t == 0) return fail(PF_ERR_INVALID_ARG, "no step taken yet");
    if ((x_prop || y_prop) && (h->p.flags & PF_FLAG_STATE_ONLY))
        return fail(PF_ERR_INVALID_ARG, "a PF_FLAG_STATE_ONLY filter keeps no propagated positions");
    size_t ox, oy;
    prop_offsets(h, b.t, &ox, &oy);
    if (int rc = export_positions(h, ox, oy, x_prop, y_prop, b)) return rc;
    if (disk_sum) {
        e = hipMemcpyAsync(disk_sum, at(h, h->L.dg_s), (size_t)h->p.n_particles * 4, hipMemcpyDeviceToHost,
                           h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "pf_export_step disk_sum");
    }
    return ok();
}

int pf_import(pf_filter* h, const double* x, const double* y, uint32_t t)
{
    if (int rc = live(h)) return rc;
    if (!x || !y) return fail(PF_ERR_INVALID_ARG, "x/y is NULL");
    const int64_t n = h->p.n_particles;
    const int dt = h->p.dtype;
    double mx = 0, my = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(x[k]) || !isfinite(y[k]) || fabs(x[k]) > 1e6 || fabs(y[k]) > 1e6)
            return fail(PF_ERR_INVALID_ARG, "position %lld not finite or |v| > 1e6", (long long)k);
        mx += x[k];
        my += y[k];
    }
    mx /= (double)n;
    my /= (double)n;
    hipError_t e;
    DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_import");
    double ox = 0, oy = 0;
    if (dt != PF_F64) {
        b.ci_x = floor_cell(mx);
        b.ci_y = floor_cell(my);
        b.cn_x = floor_cell(mx + h->p.drift_x);
        b.cn_y = floor_cell(my + h->p.drift_y);
        ox = (double)b.ci_x;
        oy = (double)b.ci_y;
    }
    b.est_x = mx;
    b.est_y = my;
    b.t = t;
    b.pend = 0;  // the imported state is the state
    const int elt = elt_of(dt);
    std::vector<uint8_t> bx((size_t)n * elt), by((size_t)n * elt);
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t vx = to_store_bits(dt, x[k] - ox), vy = to_store_bits(dt, y[k] - oy);
        memcpy(bx.data() + (size_t)k * elt, &vx, elt);
        memcpy(by.data() + (size_t)k * elt, &vy, elt);
    }
    e = hipMemcpyAsync(at(h, h->L.sx), bx.data(), bx.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(at(h, h->L.sy), by.data(), by.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = write_block(h, b);
    if (e != hipSuccess) return hip_fail(h, e, "pf_import");
    h->t = t;
    return ok();
}

static void profile_free(pf_filter* h)
{
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    h->prof_ev.clear();
    h->prof_max = h->prof_used = 0;
}

int pf_profile_start(pf_filter* h, uint32_t max_steps)
{
    if (int rc = live(h)) return rc;
    if (max_steps == 0 || max_steps > (1u << 20)) return fail(PF_ERR_INVALID_ARG, "max_steps must be in [1, 2^20]");
    profile_free(h);
    h->prof_ev.resize(kProfEv * (size_t)max_steps);
    for (size_t i = 0; i < h->prof_ev.size(); ++i) {
        const hipError_t e = hipEventCreate(&h->prof_ev[i]);
        if (e != hipSuccess) {
            h->prof_ev.resize(i);
            profile_free(h);
            return hip_fail(h, e, "pf_profile_start");
        }
    }
    h->prof_max = max_steps;
    h->prof_used = 0;
    return ok();
}

int pf_profile_read(pf_filter* h, double out_ms[3], uint32_t* steps)
{
    if (int rc = live(h)) return rc;
    if (!out_ms) return fail(PF_ERR_INVALID_ARG, "out_ms is NULL");
    hipError_t e = hipStreamSynchronize(h->stream);
    double acc[3] = {0, 0, 0};
    for (uint32_t i = 0; e == hipSuccess && i < h->prof_used; ++i) {
        // a filter that defers its resampling runs no pass C (its events stay unused)
        for (int k = 0; k < (h->args.gather ? 2 : 3) && e == hipSuccess; ++k) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, h->prof_ev[kProfEv * i + 2 * k], h->prof_ev[kProfEv * i + 2 * k + 1]);
            acc[k] += ms;
        }
    }
    const uint32_t used = h->prof_used;
    profile_free(h);
    if (e != hipSuccess) return hip_fail(h, e, "pf_profile_read");
    for (int k = 0; k < 3; ++k) out_ms[k] = acc[k];
    if (steps) *steps = used;
    return ok();
}

int pf_destroy(pf_filter* h)
{
    if (h && h->owner) return fail(PF_ERR_INVALID_ARG, "filter belongs to a batch; use pf_batch_destroy");
    if (h) profile_free(h);
    delete h;
    return ok();
}

// ---------------------------------------------------------------------------
// Batches.

struct BatchLayout {
    size_t args, entries, tile_entry, g_entries, g_tile_entry, est, a_tiles, g_a_tiles, filters, total;
    int64_t tiles;
};

// Flags a batch member may carry: diagnostics and the workgroup sizes.
constexpr uint32_t kBatchFlags =
    PF_FLAG_DIAGNOSTICS | PF_FLAG_TUNED | (0xFu << PF_THREADS_A_SHIFT) | (0xFu << PF_THREADS_C_SHIFT);

// Checks a batch's parameters and lays out its workspace; the plan buffers
// hold max(max_tiles, the members' tiles) tiles.
static int check_batch(const pf_params* ps, int32_t n, int64_t max_tiles, BatchLayout* bl,
                       std::vector<size_t>* foff)
{
    if (!ps) return fail(PF_ERR_INVALID_ARG, "params is NULL");
    if (n < 1 || n > (1 << 20)) return fail(PF_ERR_INVALID_ARG, "batch size %d outside [1, 2^20]", n);
    int64_t tiles = 0;
    size_t fbytes = 0;
    if (foff) foff->resize((size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        if (check_params(&ps[k])) return fail(PF_ERR_INVALID_ARG, "filter %d: %s", k, g_err.c_str());
        if (ps[k].dtype != ps[0].dtype) return fail(PF_ERR_INVALID_ARG, "filter %d: dtype differs from filter 0", k);
        if (ps[k].flags & ~kBatchFlags)
            return fail(PF_ERR_INVALID_ARG, "filter %d: implementation variants are not batched", k);
        const Layout L = make_layout(ps[k]);
        if (foff) (*foff)[k] = fbytes;
        fbytes += L.total;
        tiles += L.ntiles;
    }
    if (max_tiles < 0 || max_tiles > INT32_MAX)
        return fail(PF_ERR_INVALID_ARG, "tile capacity %lld outside [0, 2^31 - 1]", (long long)max_tiles);
    if (tiles > INT32_MAX) return fail(PF_ERR_INVALID_ARG, "batch has %lld tiles, more than 2^31 - 1", (long long)tiles);
    if (max_tiles > tiles) tiles = max_tiles;
    size_t o = 0;
    bl->args = o; o = align256(o + sizeof(StepArgs) * (size_t)n);
    bl->entries = o; o = align256(o + sizeof(BatchEntry) * (size_t)n);
    bl->tile_entry = o; o = align256(o + 4 * (size_t)tiles);
    bl->g_entries = o; o = align256(o + sizeof(BatchEntry) * (size_t)n);  // captured steps' plan
    bl->g_tile_entry = o; o = align256(o + 4 * (size_t)tiles);
    bl->est = o; o = align256(o + 16 * (size_t)n);
    bl->a_tiles = o; o = align256(o + 4 * (size_t)tiles);
    bl->g_a_tiles = o; o = align256(o + 4 * (size_t)tiles);
    bl->filters = o; o += fbytes;
    bl->total = o;
    bl->tiles = tiles;
    return PF_OK;
}

static int batch_fail(pf_batch* b, hipError_t e, const char* what)
{
    b->poisoned = true;
    b->map_valid = false;
    for (pf_filter* h : b->f) h->poisoned = true;
    return fail(PF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static int batch_rebind(pf_batch* b, int32_t k, const pf_params* p, uint8_t* ws, size_t share_bytes);

static void batch_free(pf_batch* b)
{
    for (pf_filter* h : b->f) {
        profile_free(h);
        delete h;
    }
    b->f.clear();
    for (int i = 0; i < kRing; ++i) {
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
        if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
    }
    if (b->h_graph) (void)hipHostFree(b->h_graph);
    delete b;
}

int pf_batch_workspace_bytes_cap(const pf_params* ps, int32_t n, int64_t max_tiles, size_t* out_bytes)
{
    BatchLayout bl;
    if (int rc = check_batch(ps, n, max_tiles, &bl, nullptr)) return rc;
    if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
    *out_bytes = bl.total;
    return ok();
}

int pf_batch_workspace_bytes(const pf_params* ps, int32_t n, size_t* out_bytes)
{
    return pf_batch_workspace_bytes_cap(ps, n, 0, out_bytes);
}

int pf_batch_init(const pf_params* ps, int32_t n, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                  pf_batch** out)
{
    return pf_batch_init_cap(ps, n, 0, d_workspace, workspace_bytes, hip_stream, out);
}

int pf_batch_init_cap(const pf_params* ps, int32_t n, int64_t max_tiles, void* d_workspace, size_t workspace_bytes,
                      void* hip_stream, pf_batch** out)
{
    BatchLayout bl;
    std::vector<size_t> foff;
    if (int rc = check_batch(ps, n, max_tiles, &bl, &foff)) return rc;
    if (!out) return fail(PF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d_workspace) return fail(PF_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(PF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < bl.total)
        return fail(PF_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, bl.total);

    pf_batch* b = new (std::nothrow) pf_batch{};
    if (!b) return fail(PF_ERR_INVALID_ARG, "out of host memory");
    b->n = n;
    b->dtype = ps[0].dtype;
    b->stream = (hipStream_t)hip_stream;
    b->ws = (uint8_t*)d_workspace;
    b->total_tiles = bl.tiles;
    b->d_args = (StepArgs*)(b->ws + bl.args);
    b->d_entries = (BatchEntry*)(b->ws + bl.entries);
    b->d_tile_entry = (int32_t*)(b->ws + bl.tile_entry);
    b->d_g_entries = (BatchEntry*)(b->ws + bl.g_entries);
    b->d_g_tile_entry = (int32_t*)(b->ws + bl.g_tile_entry);
    b->d_a_tiles = (int32_t*)(b->ws + bl.a_tiles);
    b->d_g_a_tiles = (int32_t*)(b->ws + bl.g_a_tiles);
    b->d_est = (double*)(b->ws + bl.est);
    b->map_valid = false;
    b->poisoned = false;
    b->ring = 0;
    bool all5 = true, all8 = true;
    for (int32_t k = 0; k < n; ++k) {
        all5 = all5 && ps[k].disk_radius == 5;
        all8 = all8 && ps[k].disk_radius == 8;
    }
    b->rc = all5 ? 5 : all8 ? 8 : 0;

    std::vector<DevBlock> blocks((size_t)n);
    std::vector<StepArgs>& args = b->args_host;
    args.resize((size_t)n);
    b->slot_bytes.resize((size_t)n);
    b->tiles_used = 0;
    std::vector<double> vx((size_t)n), vy((size_t)n);
    b->f.reserve((size_t)n);
    b->cls.resize((size_t)n);
    b->ta.resize((size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        pf_params pk;
        if (resolve_tuned(&ps[k], b->stream, &pk)) {
            const int rc = fail(PF_ERR_HIP, "filter %d: %s", k, g_err.c_str());
            batch_free(b);
            return rc;
        }
        pf_filter* h = new (std::nothrow) pf_filter{};
        if (!h) {
            batch_free(b);
            return fail(PF_ERR_INVALID_ARG, "out of host memory");
        }
        b->f.push_back(h);
        setup_filter(h, pk, b->ws + bl.filters + foff[k], b->stream, &blocks[k], &vx[k], &vy[k]);
        h->owner = b;
        args[k] = h->args;
        b->cls[k] = comb_class(h->L.ntiles);
        b->ta[k] = h->args.threads_a;
        b->slot_bytes[k] = h->L.total;
        b->tiles_used += h->L.ntiles;
    }
    b->stage_bytes = sizeof(BatchEntry) * (size_t)n + 8 * (size_t)bl.tiles;
    hipError_t e = hipSuccess;
    for (int i = 0; i < kRing && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&b->h_stage[i], b->stage_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_graph, b->stage_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_args, args.data(), sizeof(StepArgs) * (size_t)n, hipMemcpyHostToDevice, b->stream);
    for (int32_t k = 0; k < n && e == hipSuccess; ++k) {
        pf_filter* h = b->f[k];
        e = hipMemcpyAsync(at(h, h->L.blk), &blocks[k], sizeof(DevBlock), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = launch_fill(b->dtype, h->args, vx[k], vy[k], b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        const int rc = fail(PF_ERR_HIP, "pf_batch_init: %s", hipGetErrorString(e));
        batch_free(b);
        return rc;
    }
    *out = b;
    return ok();
}

static int batch_live(pf_batch* b)
{
    if (!b) return fail(PF_ERR_INVALID_ARG, "batch is NULL");
    if (b->poisoned) return fail(PF_ERR_STATE, "batch poisoned by an earlier HIP error");
    return PF_OK;
}

int pf_batch_step(pf_batch* b, const uint8_t* const* d_frames, const int64_t* pitches, const uint8_t* active)
{
    if (int rc = batch_live(b)) return rc;
    if (!d_frames || !pitches) return fail(PF_ERR_INVALID_ARG, "frames/pitches is NULL");
    const int32_t n = b->n;
    // check everything before any state changes
    int32_t n_act = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (active && !active[k]) continue;
        const pf_filter* h = b->f[k];
        if (h->poisoned) return fail(PF_ERR_STATE, "filter %d poisoned", k);
        if (!d_frames[k]) return fail(PF_ERR_INVALID_ARG, "filter %d: frame is NULL", k);
        if (pitches[k] < h->p.width)
            return fail(PF_ERR_INVALID_ARG, "filter %d: row_pitch %lld < width %d", k, (long long)pitches[k], h->p.width);
        if (h->t == UINT32_MAX) return fail(PF_ERR_INVALID_ARG, "filter %d: step counter exhausted", k);
        ++n_act;
    }
    if (n_act == 0) return ok();

    // Under stream capture the step is recorded, not run: its entries and tile
    // map go through the staging buffer kept for captured steps to device
    // buffers of their own (copies that every replay repeats, leaving the
    // eager steps' plan alone), and no host wait or event is recorded.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(b->stream, &cap);
    if (e != hipSuccess) return batch_fail(b, e, "pf_batch_step");
    const bool capturing = cap != hipStreamCaptureStatusNone;

    // the stepped set, and whether the uploaded tile map still describes it
    bool same = !capturing && b->map_valid && (int32_t)b->map_active.size() == n;
    if (same)
        for (int32_t k = 0; k < n && same; ++k) same = b->map_active[k] == (uint8_t)(active ? active[k] != 0 : 1);

    const int slot = b->ring;
    uint8_t* stage = b->h_graph;
    if (!capturing) {
        b->ring = (b->ring + 1) % kRing;
        if (b->ev_used[slot]) e = hipEventSynchronize(b->ev[slot]);
        if (e != hipSuccess) return batch_fail(b, e, "pf_batch_step");
        stage = b->h_stage[slot];
    }
    BatchEntry* ent = reinterpret_cast<BatchEntry*>(stage);
    int32_t* tmap = reinterpret_cast<int32_t*>(stage + sizeof(BatchEntry) * (size_t)n);
    int32_t* alist = tmap + b->total_tiles;
    int32_t cls_begin[kCombClasses + 1];
    int32_t ne = 0, tiles = 0;
    for (int c = 0; c < kCombClasses; ++c) {
        cls_begin[c] = ne;
        for (int32_t k = 0; k < n; ++k) {
            if ((active && !active[k]) || b->cls[k] != c) continue;
            const pf_filter* h = b->f[k];
            BatchEntry& en = ent[ne];
            en.frame = d_frames[k];
            en.pitch = pitches[k];
            en.fid = k;
            en.tile_base = tiles;
            en.t = h->t + 1;
            en.pad = 0;
            if (!same)
                for (int i = 0; i < h->L.ntiles; ++i) tmap[tiles + i] = ne;
            tiles += h->L.ntiles;
            ++ne;
        }
    }
    cls_begin[kCombClasses] = ne;

    // pass-A sizes of the stepped filters: one launch per size; with more
    // than one size, each launch reads its grid tiles from a list
    static constexpr int kSizesA[3] = {128, 256, 512};
    int32_t a_count[3] = {0, 0, 0};
    for (int32_t i = 0; i < ne; ++i) {
        const pf_filter* h = b->f[ent[i].fid];
        for (int c = 0; c < 3; ++c)
            if (b->ta[ent[i].fid] == kSizesA[c]) a_count[c] += h->L.ntiles;
    }
    const int sizes_used = (a_count[0] > 0) + (a_count[1] > 0) + (a_count[2] > 0);
    int32_t a_begin[3] = {0, a_count[0], a_count[0] + a_count[1]};
    if (sizes_used > 1 && !same) {
        int32_t fillp[3] = {a_begin[0], a_begin[1], a_begin[2]};
        for (int32_t i = 0; i < ne; ++i) {
            const pf_filter* h = b->f[ent[i].fid];
            const int c = b->ta[ent[i].fid] == 128 ? 0 : b->ta[ent[i].fid] == 256 ? 1 : 2;
            for (int j = 0; j < h->L.ntiles; ++j) alist[fillp[c]++] = ent[i].tile_base + j;
        }
    }

    BatchEntry* d_ent = capturing ? b->d_g_entries : b->d_entries;
    int32_t* d_map = capturing ? b->d_g_tile_entry : b->d_tile_entry;
    int32_t* d_alist = capturing ? b->d_g_a_tiles : b->d_a_tiles;
    e = hipMemcpyAsync(d_ent, ent, sizeof(BatchEntry) * (size_t)ne, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !same)
        e = hipMemcpyAsync(d_map, tmap, 4 * (size_t)tiles, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !same && sizes_used > 1)
        e = hipMemcpyAsync(d_alist, alist, 4 * (size_t)tiles, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !capturing) e = hipEventRecord(b->ev[slot], b->stream);
    if (e == hipSuccess && !capturing) b->ev_used[slot] = true;
    BatchArgs ba;
    ba.args = b->d_args;
    ba.entries = d_ent;
    ba.tile_entry = d_map;
    ba.a_tiles = nullptr;
    ba.entry0 = 0;
    ba.tiles = tiles;
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        if (a_count[c] == 0) continue;
        BatchArgs bp = ba;
        if (sizes_used > 1) {
            bp.a_tiles = d_alist;
            bp.entry0 = a_begin[c];
        }
        e = launch_batch_pass_a(b->dtype, b->rc, kSizesA[c], bp, a_count[c], b->stream);
    }
    for (int c = 0; c < kCombClasses - 1 && e == hipSuccess; ++c) {
        const int32_t cnt = cls_begin[c + 1] - cls_begin[c];
        if (cnt == 0) continue;
        ba.entry0 = cls_begin[c];
        e = launch_batch_combine(b->dtype, c, ba, cnt, b->stream);
    }
    // the largest filters (class 3) combine with the grouped kernels, one
    // filter at a time, exactly as they do alone
    for (int32_t i = cls_begin[kCombClasses - 1]; i < cls_begin[kCombClasses] && e == hipSuccess; ++i) {
        StepArgs a = b->f[ent[i].fid]->args;
        a.t = ent[i].t;
        e = launch_combine(b->dtype, a, b->stream);
    }
    ba.entry0 = 0;
    if (e == hipSuccess) e = launch_batch_pass_c(b->dtype, ba, tiles, b->stream);
    for (int32_t i = 0; i < ne && e == hipSuccess; ++i) {
        const pf_filter* h = b->f[ent[i].fid];
        if (!h->args.dg_w) continue;
        StepArgs a = h->args;
        a.t = ent[i].t;
        e = launch_diag_weights(b->dtype, a, b->stream);
    }
    if (e != hipSuccess) return batch_fail(b, e, "pf_batch_step launch");
    if (capturing) return ok();
    if (!same) {
        b->map_active.resize((size_t)n);
        for (int32_t k = 0; k < n; ++k) b->map_active[k] = (uint8_t)(active ? active[k] != 0 : 1);
        b->map_valid = true;
    }
    for (int32_t i = 0; i < ne; ++i) b->f[ent[i].fid]->t = ent[i].t;
    return ok();
}

int pf_batch_estimates_async(pf_batch* b, double* d_out_2n)
{
    if (int rc = batch_live(b)) return rc;
    if (!d_out_2n) return fail(PF_ERR_INVALID_ARG, "d_out_2n is NULL");
    const hipError_t e = launch_gather_est(b->d_args, b->n, d_out_2n, b->stream);
    if (e != hipSuccess) return batch_fail(b, e, "pf_batch_estimates_async");
    return ok();
}

int pf_batch_estimates(pf_batch* b, double* out_2n)
{
    if (int rc = batch_live(b)) return rc;
    if (!out_2n) return fail(PF_ERR_INVALID_ARG, "out_2n is NULL");
    hipError_t e = launch_gather_est(b->d_args, b->n, b->d_est, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out_2n, b->d_est, 16 * (size_t)b->n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_fail(b, e, "pf_batch_estimates");
    return ok();
}

int pf_batch_reinit(pf_batch* b, int32_t k, const pf_params* p_in)
{
    if (int rc = batch_live(b)) return rc;
    if (k < 0 || k >= b->n) return fail(PF_ERR_INVALID_ARG, "filter index %d outside [0, %d)", k, b->n);
    if (int rc = check_params(p_in)) return rc;
    if (p_in->dtype != b->dtype)
        return fail(PF_ERR_INVALID_ARG, "dtype %d differs from the batch's %d", p_in->dtype, b->dtype);
    if (p_in->flags & ~kBatchFlags) return fail(PF_ERR_INVALID_ARG, "implementation variants are not batched");
    pf_params tuned;
    if (int rc = resolve_tuned(p_in, b->stream, &tuned)) return rc;
    const pf_params* p = &tuned;
    const Layout L = make_layout(*p);
    pf_filter* h = b->f[k];
    if (L.total > b->slot_bytes[k])
        return fail(PF_ERR_WORKSPACE, "filter %d: %zu bytes needed, its share holds %zu", k, L.total, b->slot_bytes[k]);
    if (b->tiles_used - h->L.ntiles + L.ntiles > b->total_tiles)
        return fail(PF_ERR_WORKSPACE, "filter %d: %d tiles would bring the batch to %lld, its plan holds %lld", k,
                    L.ntiles, (long long)(b->tiles_used - h->L.ntiles + L.ntiles), (long long)b->total_tiles);
    return batch_rebind(b, k, p, h->ws, b->slot_bytes[k]);
}

int pf_batch_rebind(pf_batch* b, int32_t k, const pf_params* p_in, void* d_share, size_t share_bytes)
{
    if (int rc = batch_live(b)) return rc;
    if (k < 0 || k >= b->n) return fail(PF_ERR_INVALID_ARG, "filter index %d outside [0, %d)", k, b->n);
    if (int rc = check_params(p_in)) return rc;
    if (p_in->dtype != b->dtype)
        return fail(PF_ERR_INVALID_ARG, "dtype %d differs from the batch's %d", p_in->dtype, b->dtype);
    if (p_in->flags & ~kBatchFlags) return fail(PF_ERR_INVALID_ARG, "implementation variants are not batched");
    if (!d_share) return fail(PF_ERR_INVALID_ARG, "share is NULL");
    if (((uintptr_t)d_share & 255) != 0) return fail(PF_ERR_INVALID_ARG, "share must be 256-byte aligned");
    pf_params tuned;
    if (int rc = resolve_tuned(p_in, b->stream, &tuned)) return rc;
    const Layout L = make_layout(tuned);
    pf_filter* h = b->f[k];
    if (L.total > share_bytes)
        return fail(PF_ERR_WORKSPACE, "filter %d: %zu bytes needed, the share holds %zu", k, L.total, share_bytes);
    if (b->tiles_used - h->L.ntiles + L.ntiles > b->total_tiles)
        return fail(PF_ERR_WORKSPACE, "filter %d: %d tiles would bring the batch to %lld, its plan holds %lld", k,
                    L.ntiles, (long long)(b->tiles_used - h->L.ntiles + L.ntiles), (long long)b->total_tiles);
    return batch_rebind(b, k, &tuned, (uint8_t*)d_share, share_bytes);
}

}  // extern "C"

// Re-initialise member k with checked parameters `p` on the share at `ws`
// (share_bytes long): waits for the stream before and after.
static int batch_rebind(pf_batch* b, int32_t k, const pf_params* p, uint8_t* ws, size_t share_bytes)
{
    pf_filter* h = b->f[k];
    const Layout L = make_layout(*p);
    hipError_t e = hipStreamSynchronize(b->stream);  // earlier work may still read the slot
    if (e != hipSuccess) return batch_fail(b, e, "batch member re-initialisation");
    profile_free(h);
    DevBlock blk;
    double vx, vy;
    b->tiles_used += L.ntiles - h->L.ntiles;
    setup_filter(h, *p, ws, b->stream, &blk, &vx, &vy);
    h->owner = b;
    b->slot_bytes[k] = share_bytes;
    b->args_host[k] = h->args;
    b->cls[k] = comb_class(L.ntiles);
    b->ta[k] = h->args.threads_a;
    b->map_valid = false;
    bool all5 = true, all8 = true;
    for (const pf_filter* g : b->f) {
        all5 = all5 && g->p.disk_radius == 5;
        all8 = all8 && g->p.disk_radius == 8;
    }
    b->rc = all5 ? 5 : all8 ? 8 : 0;
    e = hipMemcpyAsync(b->d_args + k, &b->args_host[k], sizeof(StepArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(at(h, h->L.blk), &blk, sizeof blk, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_fill(b->dtype, h->args, vx, vy, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_fail(b, e, "batch member re-initialisation");
    return ok();
}

extern "C" {

int pf_batch_filter(pf_batch* b, int32_t k, pf_filter** out)
{
    if (!b) return fail(PF_ERR_INVALID_ARG, "batch is NULL");
    if (!out) return fail(PF_ERR_INVALID_ARG, "out is NULL");
    if (k < 0 || k >= b->n) return fail(PF_ERR_INVALID_ARG, "filter index %d outside [0, %d)", k, b->n);
    *out = b->f[k];
    return ok();
}

int pf_batch_destroy(pf_batch* b)
{
    if (!b) return ok();
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return ok();
}

}  // extern "C"
