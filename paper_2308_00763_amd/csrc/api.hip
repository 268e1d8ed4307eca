// C-ABI of libpf (include/pf.h): argument checking, workspace layout,
// stream-ordered launches, and host-side conversion of the state.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "pf_internal.hpp"

using namespace pf;

constexpr int kProfEv = 4;  // before pass A, after pass A, after combine, after pass C

struct pf_filter {
    pf_params p;
    Layout L;
    hipStream_t stream;
    uint8_t* ws;
    StepArgs args;
    uint32_t t;
    bool poisoned;
    // per-pass timing (pf_profile_start / pf_profile_read)
    std::vector<hipEvent_t> prof_ev;  // kProfEv events per recorded step
    uint32_t prof_max, prof_used;
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
    if (p->flags & ~PF_FLAG_DIAGNOSTICS) return fail(PF_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
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

}  // namespace

extern "C" {

int pf_abi_version(void) { return PF_ABI_VERSION; }

const char* pf_last_error(void) { return g_err.c_str(); }

int pf_workspace_bytes(const pf_params* p, size_t* out_bytes)
{
    if (int rc = check_params(p)) return rc;
    if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
    *out_bytes = make_layout(*p).total;
    return ok();
}

int pf_init(const pf_params* p, void* d_workspace, size_t workspace_bytes, void* hip_stream, pf_filter** out)
{
    if (int rc = check_params(p)) return rc;
    if (!out) return fail(PF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d_workspace) return fail(PF_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(PF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const Layout L = make_layout(*p);
    if (workspace_bytes < L.total)
        return fail(PF_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, L.total);

    pf_filter* h = new (std::nothrow) pf_filter{};
    if (!h) return fail(PF_ERR_INVALID_ARG, "out of host memory");
    h->p = *p;
    h->L = L;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (uint8_t*)d_workspace;
    h->t = 0;
    h->poisoned = false;

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
    a.rec = at(h, L.rec);
    a.tab = at(h, L.tab);
    a.sx = at(h, L.sx);
    a.sy = at(h, L.sy);
    a.px = at(h, L.px);
    a.py = at(h, L.py);
    a.q = at(h, L.q);
    if (p->flags & PF_FLAG_DIAGNOSTICS) {
        a.dg_s = (int32_t*)at(h, L.dg_s);
        a.dg_w = (double*)at(h, L.dg_w);
        a.dg_anc = (int32_t*)at(h, L.dg_anc);
    } else {
        a.dg_s = nullptr;
        a.dg_w = nullptr;
        a.dg_anc = nullptr;
    }

    DevBlock b{};
    double vx = p->x0, vy = p->y0;
    if (p->dtype != PF_F64) {
        b.ci_x = floor_cell(p->x0);
        b.ci_y = floor_cell(p->y0);
        b.cn_x = floor_cell(p->x0 + p->drift_x);
        b.cn_y = floor_cell(p->y0 + p->drift_y);
        vx = p->x0 - (double)b.ci_x;
        vy = p->y0 - (double)b.ci_y;
    }
    b.est_x = p->x0;
    b.est_y = p->y0;
    hipError_t e = write_block(h, b);
    if (e == hipSuccess) e = launch_fill(p->dtype, a, vx, vy, h->stream);
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
        e = hipEventRecord(ev[0], h->stream);
        if (e == hipSuccess) e = launch_pass_a(h->p.dtype, a, h->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
        if (e == hipSuccess) e = launch_combine(h->p.dtype, a, h->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
        if (e == hipSuccess) e = launch_pass_c(h->p.dtype, a, h->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[3], h->stream);
        ++h->prof_used;
    } else {
        e = launch_step(h->p.dtype, a, h->stream);
    }
    if (e == hipSuccess && a.dg_w) e = launch_diag_weights(h->p.dtype, a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "pf_step launch");
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

int pf_export(pf_filter* h, double* x, double* y, double* w_norm, int32_t* anc, uint32_t* t)
{
    if (int rc = live(h)) return rc;
    const bool diag = (h->p.flags & PF_FLAG_DIAGNOSTICS) != 0;
    if ((w_norm || anc) && !diag) return fail(PF_ERR_INVALID_ARG, "w_norm/anc need PF_FLAG_DIAGNOSTICS");
    if ((w_norm || anc) && h->t == 0) return fail(PF_ERR_INVALID_ARG, "no step taken yet");
    hipError_t e;
    const DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_export");
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
    if (t) *t = h->t;
    return ok();
}

int pf_export_step(pf_filter* h, double* x_prop, double* y_prop, int32_t* disk_sum)
{
    if (int rc = live(h)) return rc;
    if (h->t == 0) return fail(PF_ERR_INVALID_ARG, "no step taken yet");
    if (disk_sum && !(h->p.flags & PF_FLAG_DIAGNOSTICS))
        return fail(PF_ERR_INVALID_ARG, "disk_sum needs PF_FLAG_DIAGNOSTICS");
    hipError_t e;
    const DevBlock b = read_block(h, &e);
    if (e != hipSuccess) return hip_fail(h, e, "pf_export_step");
    if (int rc = export_positions(h, h->L.px, h->L.py, x_prop, y_prop, b)) return rc;
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
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, h->prof_ev[kProfEv * i + k], h->prof_ev[kProfEv * i + k + 1]);
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
    if (h) profile_free(h);
    delete h;
    return ok();
}

}  // extern "C"
