// rt_abi.cpp -- the extern "C" boundary of libradtex.so (declared in
// include/radtex.h): argument validation, texture handles, workspace sizing,
// kernel dispatch and the event-based kernel timer.
#include "radtex.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

struct rt_texture {
    rt::TexView view;
    int fmt;
    void* owned;  // bucket-major copy made from an atlas, or nullptr
};

namespace {

thread_local std::string g_last_error;

rt_status fail(rt_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
rt_status fail(rt_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

rt_status ok() { return RT_OK; }

rt_status hip_fail(hipError_t e, const char* what) {
    return fail(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t out_align(int C) { return C == 4 ? 16 : (C == 2 ? 8 : 4); }

rt_status check_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(RT_ERR_NO_DEVICE, "no HIP device is visible");
    }
    return RT_OK;
}

rt_status check_tex(const rt_texture* t) {
    if (!t) return fail(RT_ERR_INVALID_ARG, "texture handle is NULL");
    return RT_OK;
}

rt::FragMap fragmap(const rt_fragments* f) {
    return rt::make_fragmap(f->count, f->views, f->height, f->width);
}

rt_status check_frags(const rt_fragments* f, bool need_view = true) {
    if (!f) return fail(RT_ERR_INVALID_ARG, "fragments is NULL");
    if (f->count < 0) return fail(RT_ERR_INVALID_ARG, "fragment count %lld < 0", (long long)f->count);
    if (f->count >= (1ll << 31))
        return fail(RT_ERR_UNSUPPORTED, "fragment count %lld >= 2^31", (long long)f->count);
    const bool flat = f->views == 0 && f->height == 0 && f->width == 0;
    if (!flat) {
        if (f->views <= 0 || f->height <= 0 || f->width <= 0)
            return fail(RT_ERR_INVALID_ARG, "tiling hint views=%d height=%d width=%d: all three "
                        "positive or all three 0", f->views, f->height, f->width);
        if ((int64_t)f->views * f->height * f->width != f->count)
            return fail(RT_ERR_INVALID_ARG, "tiling hint %d x %d x %d does not match count %lld",
                        f->views, f->height, f->width, (long long)f->count);
    }
    if (f->count == 0) return RT_OK;
    if (!f->uv || !f->tbn || (need_view && !f->view))
        return fail(RT_ERR_INVALID_ARG, need_view ? "uv, tbn and view must be non-NULL when count > 0"
                                                  : "uv and tbn must be non-NULL when count > 0");
    if (!aligned(f->uv, 8)) return fail(RT_ERR_INVALID_ARG, "uv must be 8-byte aligned");
    if (!aligned(f->tbn, 4) || (need_view && !aligned(f->view, 4)))
        return fail(RT_ERR_INVALID_ARG, "tbn and view must be 4-byte aligned");
    return RT_OK;
}

// ---------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------
struct Pending {
    int id;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
double g_total_ms[rt::K_COUNT];
int64_t g_launches[rt::K_COUNT];
thread_local hipEvent_t t_open = nullptr;

hipEvent_t pool_get() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_locked() {
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_total_ms[p.id] += ms;
            g_launches[p.id] += 1;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}

}  // namespace

namespace rt {

const char* kernel_name(int id) {
    static const char* names[K_COUNT] = {
        "k_lookup_fwd",   "k_debug_indices", "k_quant_bf16",    "k_quant_fp8",
        "k_atlas_to_buckets", "k_bwd_fragment", "k_fill_u32",   "k_radix_hist",
        "k_scan",         "k_radix_scatter", "k_bucket_ranges", "k_segacc",
        "k_segacc_hot",   "k_combine_hot",   "k_segacc_big",    "k_bake_directions",
        "k_bake_env",     "k_build_mip",     "k_lookup_lod",    "k_pack_bits",
        "k_lookup_light", "k_bake_shadow",   "k_vq_assign",     "k_vq_hist",
        "k_vq_scatter",   "k_vq_pieces",     "k_vq_combine",    "k_lod_bwd_fragment",
        "k_mip_adjoint",  "k_payload",       "k_keys_in_order", "k_plan_keys",
        "k_plan_gather",  "k_permute_rows"};
    return (id >= 0 && id < K_COUNT) ? names[id] : "";
}

namespace {
thread_local int t_prof_suspended = 0;
}

ProfileSuspend::ProfileSuspend() { t_prof_suspended++; }
ProfileSuspend::~ProfileSuspend() { t_prof_suspended--; }

void prof_begin(int, hipStream_t s) {
    if (!g_prof_on || t_prof_suspended) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    t_open = pool_get();
    if (t_open) (void)hipEventRecord(t_open, s);
}

void prof_end(int id, hipStream_t s) {
    if (!g_prof_on || !t_open || t_prof_suspended) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t b = pool_get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_pending.push_back({id, t_open, b});
    t_open = nullptr;
}

}  // namespace rt

#define RT_GUARD_BEGIN try {
#define RT_GUARD_END                                                              \
    }                                                                             \
    catch (const std::bad_alloc&) {                                               \
        return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");              \
    }                                                                             \
    catch (const std::exception& ex) {                                            \
        return fail(RT_ERR_HIP, "internal error: %s", ex.what());                 \
    }                                                                             \
    catch (...) {                                                                 \
        return fail(RT_ERR_HIP, "internal error");                                \
    }

extern "C" {

const char* rt_last_error(void) { return g_last_error.c_str(); }

int32_t rt_version(void) { return RT_VERSION; }

const char* rt_status_string(rt_status s) {
    switch (s) {
    case RT_OK: return "RT_OK";
    case RT_ERR_INVALID_ARG: return "RT_ERR_INVALID_ARG";
    case RT_ERR_UNSUPPORTED: return "RT_ERR_UNSUPPORTED";
    case RT_ERR_OUT_OF_MEMORY: return "RT_ERR_OUT_OF_MEMORY";
    case RT_ERR_WORKSPACE_TOO_SMALL: return "RT_ERR_WORKSPACE_TOO_SMALL";
    case RT_ERR_NO_DEVICE: return "RT_ERR_NO_DEVICE";
    case RT_ERR_HIP: return "RT_ERR_HIP";
    }
    return "unknown rt_status";
}

rt_status rt_create_texture(const rt_texture_desc* d, void* stream, rt_texture** out) {
    RT_GUARD_BEGIN
    if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
    if (!d) return fail(RT_ERR_INVALID_ARG, "desc is NULL");
    if (d->buckets_w < 1 || d->buckets_h < 1)
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d must be at least 1 x 1", d->buckets_w, d->buckets_h);
    if (d->buckets_w > 65536 || d->buckets_h > 65536)
        return fail(RT_ERR_UNSUPPORTED, "bucket matrix %d x %d exceeds 65536 per side", d->buckets_w, d->buckets_h);
    if (d->n < 1) return fail(RT_ERR_INVALID_ARG, "angular resolution n = %d must be >= 1", d->n);
    if (d->n > 64) return fail(RT_ERR_UNSUPPORTED, "angular resolution n = %d exceeds 64", d->n);
    if (d->channels < 1 || d->channels > 4)
        return fail(RT_ERR_INVALID_ARG, "channels = %d must be in 1..4", d->channels);
    if (d->format < RT_FMT_F32 || d->format > RT_FMT_BIT1)
        return fail(RT_ERR_INVALID_ARG, "unknown format %d", d->format);
    if (d->layout != RT_LAYOUT_BUCKET_MAJOR && d->layout != RT_LAYOUT_ATLAS)
        return fail(RT_ERR_INVALID_ARG, "unknown layout %d", d->layout);
    if (d->format == RT_FMT_BIT1) {
        if (d->channels != 1)
            return fail(RT_ERR_INVALID_ARG, "1-bit textures have one channel, not %d", d->channels);
        if (d->layout != RT_LAYOUT_BUCKET_MAJOR)
            return fail(RT_ERR_UNSUPPORTED, "1-bit textures are bucket-major only");
    }
    if (!d->data) return fail(RT_ERR_INVALID_ARG, "data is NULL");
    if (!aligned(d->data, 16)) return fail(RT_ERR_INVALID_ARG, "data must be 16-byte aligned");
    if (d->format == RT_FMT_FP8_E4M3) {
        if (!d->scales) return fail(RT_ERR_INVALID_ARG, "FP8 textures need per-bucket scales");
        if (!aligned(d->scales, 4)) return fail(RT_ERR_INVALID_ARG, "scales must be 4-byte aligned");
    } else if (d->scales) {
        return fail(RT_ERR_INVALID_ARG, "scales must be NULL for F32, BF16 and 1-bit textures");
    }
    rt_status st = check_device();
    if (st != RT_OK) return st;
    rt_texture* t = new rt_texture();
    t->view.data = d->data;
    t->view.scales = d->scales;
    t->view.W = d->buckets_w;
    t->view.H = d->buckets_h;
    t->view.n = d->n;
    t->view.C = d->channels;
    t->fmt = d->format;
    t->owned = nullptr;
    if (d->layout == RT_LAYOUT_ATLAS) {
        const int eb = d->format == RT_FMT_F32 ? 4 : (d->format == RT_FMT_BF16 ? 2 : 1);
        const size_t bytes = (size_t)d->buckets_w * d->buckets_h * d->n * d->n * d->channels * eb;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete t;
            return fail(RT_ERR_OUT_OF_MEMORY, "allocation of %zu bytes for the bucket-major copy failed", bytes);
        }
        e = rt::launch_atlas_to_buckets(d->data, p, d->buckets_w, d->buckets_h, d->n, d->channels,
                                        eb, (hipStream_t)stream);
        if (e != hipSuccess) {
            (void)hipFree(p);
            delete t;
            return hip_fail(e, "atlas re-layout launch");
        }
        t->owned = p;
        t->view.data = p;
    }
    *out = t;
    return ok();
    RT_GUARD_END
}

rt_status rt_create_dictionary_texture(const rt_dictionary_desc* d, rt_texture** out) {
    RT_GUARD_BEGIN
    if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
    if (!d) return fail(RT_ERR_INVALID_ARG, "desc is NULL");
    if (d->buckets_w < 1 || d->buckets_h < 1)
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d must be at least 1 x 1", d->buckets_w, d->buckets_h);
    if (d->buckets_w > 65536 || d->buckets_h > 65536)
        return fail(RT_ERR_UNSUPPORTED, "bucket matrix %d x %d exceeds 65536 per side", d->buckets_w, d->buckets_h);
    if (d->n < 1) return fail(RT_ERR_INVALID_ARG, "angular resolution n = %d must be >= 1", d->n);
    if (d->n > 64) return fail(RT_ERR_UNSUPPORTED, "angular resolution n = %d exceeds 64", d->n);
    if (d->channels < 1 || d->channels > 4)
        return fail(RT_ERR_INVALID_ARG, "channels = %d must be in 1..4", d->channels);
    if (d->format != RT_FMT_F32 && d->format != RT_FMT_BF16)
        return fail(RT_ERR_UNSUPPORTED, "dictionary entries are stored as F32 or BF16, not format %d", d->format);
    if (d->index_bytes != 1 && d->index_bytes != 2 && d->index_bytes != 4)
        return fail(RT_ERR_INVALID_ARG, "index_bytes = %d must be 1, 2 or 4", d->index_bytes);
    if (d->entries < 1) return fail(RT_ERR_INVALID_ARG, "entries = %d must be >= 1", d->entries);
    if ((d->index_bytes == 1 && d->entries > 256) || (d->index_bytes == 2 && d->entries > 65536))
        return fail(RT_ERR_INVALID_ARG, "%d entries do not fit %d-byte entry numbers", d->entries, d->index_bytes);
    if (!d->codebook || !d->index) return fail(RT_ERR_INVALID_ARG, "codebook and index must be non-NULL");
    if (!aligned(d->codebook, 16)) return fail(RT_ERR_INVALID_ARG, "codebook must be 16-byte aligned");
    if (!aligned(d->index, (size_t)d->index_bytes))
        return fail(RT_ERR_INVALID_ARG, "index must be %d-byte aligned", d->index_bytes);
    if (d->gains && !aligned(d->gains, 4)) return fail(RT_ERR_INVALID_ARG, "gains must be 4-byte aligned");
    rt_status st = check_device();
    if (st != RT_OK) return st;
    rt_texture* t = new rt_texture();
    t->view.data = d->codebook;
    t->view.scales = nullptr;
    t->view.W = d->buckets_w;
    t->view.H = d->buckets_h;
    t->view.n = d->n;
    t->view.C = d->channels;
    t->view.index = d->index;
    t->view.gains = d->gains;
    t->view.index_bytes = d->index_bytes;
    t->view.entries = d->entries;
    t->fmt = d->format;
    t->owned = nullptr;
    *out = t;
    return ok();
    RT_GUARD_END
}

rt_status rt_destroy_texture(rt_texture* t) {
    RT_GUARD_BEGIN
    if (!t) return RT_OK;
    if (t->owned) {
        (void)hipDeviceSynchronize();
        (void)hipFree(t->owned);
    }
    delete t;
    return RT_OK;
    RT_GUARD_END
}

rt_status rt_quantize(const rt_texture* src, int32_t dst_format, void* codes, float* scales,
                      void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(src);
    if (st != RT_OK) return st;
    if (src->fmt != RT_FMT_F32 || src->view.index)
        return fail(RT_ERR_INVALID_ARG, "quantiser source must be an F32 texture (not a dictionary)");
    if (!codes) return fail(RT_ERR_INVALID_ARG, "dst_codes is NULL");
    if (dst_format == RT_FMT_BF16) {
        if (scales) return fail(RT_ERR_INVALID_ARG, "BF16 has no scales: dst_scales must be NULL");
        if (!aligned(codes, 8)) return fail(RT_ERR_INVALID_ARG, "dst_codes must be 8-byte aligned");
    } else if (dst_format == RT_FMT_FP8_E4M3) {
        if (!scales) return fail(RT_ERR_INVALID_ARG, "FP8 needs dst_scales");
        if (!aligned(codes, 4) || !aligned(scales, 4))
            return fail(RT_ERR_INVALID_ARG, "dst_codes and dst_scales must be 4-byte aligned");
    } else if (dst_format == RT_FMT_BIT1) {
        if (src->view.C != 1)
            return fail(RT_ERR_INVALID_ARG, "1-bit packing needs a one-channel source, not %d", src->view.C);
        if (scales) return fail(RT_ERR_INVALID_ARG, "1-bit textures have no scales: dst_scales must be NULL");
        if (!aligned(codes, 4)) return fail(RT_ERR_INVALID_ARG, "dst_codes must be 4-byte aligned");
    } else {
        return fail(RT_ERR_INVALID_ARG, "dst_format must be RT_FMT_BF16, RT_FMT_FP8_E4M3 or RT_FMT_BIT1");
    }
    hipError_t e = rt::launch_quantize(src->view, dst_format, codes, scales, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "quantiser launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_lookup_fwd(const rt_texture* t, const rt_fragments* f, float* out, uint32_t flags,
                        void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(t);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (flags & ~(uint32_t)(RT_BUCKET_BILINEAR | RT_FWD_STAGE_BUCKETS))
        return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool staged = (flags & RT_FWD_STAGE_BUCKETS) != 0;
    const int mode = (int)(flags & RT_BUCKET_BILINEAR);
    if (staged && (mode != RT_BUCKET_NEAREST || !rt::lookup_staged_supported(t->view, t->fmt)))
        return fail(RT_ERR_UNSUPPORTED,
                    "RT_FWD_STAGE_BUCKETS needs nearest buckets and a plain F32/BF16/FP8 texture "
                    "whose bucket is a multiple of 16 bytes and at most %d bytes",
                    rt::STAGED_BUCKET_BYTES);
    if (f->count > 0) {
        if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
        if (!aligned(out, out_align(t->view.C)))
            return fail(RT_ERR_INVALID_ARG, "out must be %zu-byte aligned", out_align(t->view.C));
    }
    hipError_t e = staged ? rt::launch_lookup_fwd_staged(t->view, t->fmt, f->uv, f->tbn, f->view,
                                                         out, fragmap(f), (hipStream_t)stream)
                          : rt::launch_lookup_fwd(t->view, t->fmt, mode, f->uv, f->tbn, f->view,
                                                  out, fragmap(f), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lookup launch");
    return ok();
    RT_GUARD_END
}

size_t rt_lookup_bwd_workspace(const rt_texture* t, int64_t count, uint32_t flags) {
    try {
        if (!t || count < 0 || flags > RT_BUCKET_BILINEAR) return 0;
        rt::BwdPlan p;
        if (!rt::plan_backward(t->view.W, t->view.H, t->view.n, t->view.C, count, (int)flags, &p))
            return 0;
        return p.total;
    } catch (...) {
        return 0;
    }
}

namespace {
// The arguments of the backward, checked before anything is enqueued; *plan
// receives the backward's plan.
rt_status check_bwd(const rt_texture* t, const rt_fragments* f, const float* grad_out,
                    const float* grad_tex, const float* grad_view, const float* grad_uv,
                    uint32_t flags, rt::BwdPlan* plan) {
    rt_status st = check_tex(t);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (flags > RT_BUCKET_BILINEAR) return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (t->fmt == RT_FMT_BIT1)
        return fail(RT_ERR_UNSUPPORTED, "1-bit textures have no backward (their values are flags)");
    if (t->view.index)
        return fail(RT_ERR_UNSUPPORTED, "the backward of a bucket dictionary is not supported");
    const int C = t->view.C;
    if (f->count > 0) {
        if (!grad_out) return fail(RT_ERR_INVALID_ARG, "grad_out is NULL");
        if (!aligned(grad_out, out_align(C)))
            return fail(RT_ERR_INVALID_ARG, "grad_out must be %zu-byte aligned", out_align(C));
    }
    if (grad_tex && !aligned(grad_tex, 16)) return fail(RT_ERR_INVALID_ARG, "grad_tex must be 16-byte aligned");
    if (grad_view && !aligned(grad_view, 4)) return fail(RT_ERR_INVALID_ARG, "grad_view must be 4-byte aligned");
    if (grad_uv && !aligned(grad_uv, 8)) return fail(RT_ERR_INVALID_ARG, "grad_uv must be 8-byte aligned");
    if (!rt::plan_backward(t->view.W, t->view.H, t->view.n, C, f->count, (int)flags, plan))
        return fail(RT_ERR_UNSUPPORTED, "sort key (W*H*n*n), bucket size (n*n*C <= 4096) or record count beyond the backward's limits");
    return RT_OK;
}
}  // namespace

rt_status rt_lookup_bwd(const rt_texture* t, const rt_fragments* f, const float* grad_out,
                        float* grad_tex, float* grad_view, float* grad_uv, void* ws,
                        size_t ws_bytes, uint32_t flags, void* stream) {
    RT_GUARD_BEGIN
    rt::BwdPlan plan;
    rt_status st = check_bwd(t, f, grad_out, grad_tex, grad_view, grad_uv, flags, &plan);
    if (st != RT_OK) return st;
    if (!grad_tex && !grad_view && !grad_uv) return ok();  // nothing requested
    if (grad_tex) {
        if (!ws) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
        if (!aligned(ws, 256)) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        if (ws_bytes < plan.total)
            return fail(RT_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, %zu needed", ws_bytes, plan.total);
    }
    hipError_t e = rt::launch_backward(t->view, t->fmt, (int)flags, f->uv, f->tbn, f->view,
                                       grad_out, grad_tex, grad_view, grad_uv, fragmap(f), plan,
                                       ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return ok();
    RT_GUARD_END
}

size_t rt_plan_workspace(const rt_texture* t, int64_t count, uint32_t flags) {
    try {
        if (!t || count < 0 || flags > RT_BUCKET_BILINEAR) return 0;
        rt::BwdPlan p;
        if (!rt::plan_backward(t->view.W, t->view.H, t->view.n, 1, count, rt::MODE_NEAREST, &p))
            return 0;
        return p.sort_total;
    } catch (...) {
        return 0;
    }
}

namespace {
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}
}  // namespace

rt_status rt_plan_fragments(const rt_texture* t, const rt_fragments* f, uint32_t flags,
                            int32_t* order, float* uv_out, float* tbn_out, float* view_out,
                            void* ws, size_t ws_bytes, void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(t);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (flags > RT_BUCKET_BILINEAR) return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    rt::BwdPlan plan;
    if (!rt::plan_backward(t->view.W, t->view.H, t->view.n, 1, f->count, rt::MODE_NEAREST, &plan))
        return fail(RT_ERR_UNSUPPORTED, "sort key (W*H*n*n) beyond 32 bits");
    const int64_t N = f->count;
    if (N == 0) return ok();
    if (!order || !uv_out || !tbn_out || !view_out)
        return fail(RT_ERR_INVALID_ARG, "order, uv_out, tbn_out and view_out must be non-NULL");
    if (!aligned(order, 4) || !aligned(uv_out, 8) || !aligned(tbn_out, 4) || !aligned(view_out, 4))
        return fail(RT_ERR_INVALID_ARG, "order, tbn_out and view_out must be 4-byte and uv_out "
                    "8-byte aligned");
    const void* ins[3] = {f->uv, f->tbn, f->view};
    const size_t insz[3] = {(size_t)N * 8, (size_t)N * 36, (size_t)N * 12};
    const void* outs[4] = {order, uv_out, tbn_out, view_out};
    const size_t outsz[4] = {(size_t)N * 4, (size_t)N * 8, (size_t)N * 36, (size_t)N * 12};
    for (int a = 0; a < 4; a++) {
        for (int b = 0; b < 3; b++)
            if (overlaps(outs[a], outsz[a], ins[b], insz[b]))
                return fail(RT_ERR_INVALID_ARG, "the planned arrays must not overlap the input");
        for (int b = a + 1; b < 4; b++)
            if (overlaps(outs[a], outsz[a], outs[b], outsz[b]))
                return fail(RT_ERR_INVALID_ARG, "the planned arrays must not overlap each other");
    }
    if (!ws) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < plan.sort_total)
        return fail(RT_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, %zu needed", ws_bytes,
                    plan.sort_total);
    hipError_t e = rt::launch_plan(t->view, (int)flags, f->uv, f->tbn, f->view, fragmap(f), plan,
                                   ws, order, uv_out, tbn_out, view_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_plan_permute(const int32_t* order, int64_t count, int32_t row_bytes,
                          const void* src, void* dst, uint32_t direction, void* stream) {
    RT_GUARD_BEGIN
    if (count < 0 || count >= (1ll << 31))
        return fail(RT_ERR_INVALID_ARG, "count %lld outside [0, 2^31)", (long long)count);
    if (direction > RT_PLAN_SCATTER) return fail(RT_ERR_INVALID_ARG, "unknown direction %u", direction);
    if (row_bytes <= 0 || row_bytes % 4 != 0 || row_bytes > 4096)
        return fail(RT_ERR_INVALID_ARG, "row_bytes %d: a multiple of 4 in 4..4096", row_bytes);
    if (count == 0) return ok();
    if (!order || !src || !dst) return fail(RT_ERR_INVALID_ARG, "order, src and dst must be non-NULL");
    if (!aligned(order, 4) || !aligned(src, 4) || !aligned(dst, 4))
        return fail(RT_ERR_INVALID_ARG, "order, src and dst must be 4-byte aligned");
    const size_t bytes = (size_t)count * (size_t)row_bytes;
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (a < b + bytes && b < a + bytes)
        return fail(RT_ERR_INVALID_ARG, "src and dst must not overlap");
    hipError_t e = rt::launch_permute_rows(order, count, row_bytes / 4, src, dst,
                                           direction == RT_PLAN_SCATTER, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "permute launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_lookup_bwd_noalloc(const rt_texture* t, const rt_fragments* f,
                                const float* grad_out, float* grad_tex, float* grad_view,
                                float* grad_uv, uint32_t flags, void* stream) {
    RT_GUARD_BEGIN
    rt::BwdPlan plan;
    rt_status st = check_bwd(t, f, grad_out, grad_tex, grad_view, grad_uv, flags, &plan);
    if (st != RT_OK) return st;
    if (!grad_tex && !grad_view && !grad_uv) return ok();  // nothing requested
    void* ws = nullptr;
    if (grad_tex) {
        if (plan.total > rt::NOALLOC_SCRATCH_BYTES)
            return fail(RT_ERR_WORKSPACE_TOO_SMALL, "this backward needs %zu bytes of workspace, "
                        "more than the %zu bytes of the allocation-free entry's scratch: use "
                        "rt_lookup_bwd with a workspace", plan.total, rt::NOALLOC_SCRATCH_BYTES);
        hipError_t e = rt::noalloc_scratch(&ws);
        if (e != hipSuccess) return hip_fail(e, "scratch address");
    }
    rt::ProfileSuspend quiet;  // the kernel timer would create events
    hipError_t e = rt::launch_backward(t->view, t->fmt, (int)flags, f->uv, f->tbn, f->view,
                                       grad_out, grad_tex, grad_view, grad_uv, fragmap(f), plan,
                                       ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_debug_indices(const rt_texture* t, const rt_fragments* f, int32_t* idx, float* frac,
                           void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(t);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (f->count > 0) {
        if (!idx || !frac) return fail(RT_ERR_INVALID_ARG, "idx and frac must be non-NULL");
        if (!aligned(idx, 16) || !aligned(frac, 8))
            return fail(RT_ERR_INVALID_ARG, "idx must be 16-byte and frac 8-byte aligned");
    }
    rt::prof_begin(rt::K_DEBUG_INDICES, (hipStream_t)stream);
    hipError_t e = rt::launch_debug_indices(t->view, f->uv, f->tbn, f->view, idx, frac,
                                            fragmap(f), (hipStream_t)stream);
    rt::prof_end(rt::K_DEBUG_INDICES, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "debug-indices launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_bake_directions(int32_t n, float* inc, float* refl, void* stream) {
    RT_GUARD_BEGIN
    if (n < 1) return fail(RT_ERR_INVALID_ARG, "angular resolution n = %d must be >= 1", n);
    if (n > 64) return fail(RT_ERR_UNSUPPORTED, "angular resolution n = %d exceeds 64", n);
    if ((inc && !aligned(inc, 4)) || (refl && !aligned(refl, 4)))
        return fail(RT_ERR_INVALID_ARG, "inc and refl must be 4-byte aligned");
    if (!inc && !refl) return ok();
    rt_status st = check_device();
    if (st != RT_OK) return st;
    hipError_t e = rt::launch_bake_directions(n, inc, refl, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bake-directions launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_bake_environment(int32_t W, int32_t H, int32_t n, int32_t C, const float* frames,
                              const rt_env_lobe* lobes, int32_t nlobes, const float* ambient,
                              float* texels, void* stream) {
    RT_GUARD_BEGIN
    if (W < 1 || H < 1)
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d must be at least 1 x 1", W, H);
    if (W > 65536 || H > 65536)
        return fail(RT_ERR_UNSUPPORTED, "bucket matrix %d x %d exceeds 65536 per side", W, H);
    if (n < 1) return fail(RT_ERR_INVALID_ARG, "angular resolution n = %d must be >= 1", n);
    if (n > 64) return fail(RT_ERR_UNSUPPORTED, "angular resolution n = %d exceeds 64", n);
    if (C < 1 || C > 4) return fail(RT_ERR_INVALID_ARG, "channels = %d must be in 1..4", C);
    if (nlobes < 0) return fail(RT_ERR_INVALID_ARG, "nlobes = %d < 0", nlobes);
    if (nlobes > rt::MAX_LOBES)
        return fail(RT_ERR_UNSUPPORTED, "nlobes = %d exceeds %d", nlobes, rt::MAX_LOBES);
    if (nlobes > 0 && !lobes) return fail(RT_ERR_INVALID_ARG, "lobes is NULL");
    if (!ambient) return fail(RT_ERR_INVALID_ARG, "ambient is NULL");
    if (!texels) return fail(RT_ERR_INVALID_ARG, "texels is NULL");
    if (!aligned(texels, out_align(C)))
        return fail(RT_ERR_INVALID_ARG, "texels must be %zu-byte aligned", out_align(C));
    if (frames && !aligned(frames, 4)) return fail(RT_ERR_INVALID_ARG, "frames must be 4-byte aligned");
    rt::EnvParams env;
    memset(&env, 0, sizeof(env));
    env.lobes = nlobes;
    for (int c = 0; c < 4; c++) {
        if (!std::isfinite(ambient[c])) return fail(RT_ERR_INVALID_ARG, "ambient[%d] is not finite", c);
        env.ambient[c] = ambient[c];
    }
    for (int k = 0; k < nlobes; k++) {
        const rt_env_lobe& L = lobes[k];
        const double ax = L.axis[0], ay = L.axis[1], az = L.axis[2];
        const double len = std::sqrt(ax * ax + ay * ay + az * az);
        if (!(len > 0.0) || !std::isfinite(len))
            return fail(RT_ERR_INVALID_ARG, "lobe %d: axis must be finite and non-zero", k);
        if (!(L.sharpness >= 0.f) || !std::isfinite(L.sharpness))
            return fail(RT_ERR_INVALID_ARG, "lobe %d: sharpness must be finite and >= 0", k);
        const double l2 = (double)L.sharpness * 1.4426950408889634;  // lambda log2(e)
        env.lobe[k][0] = (float)(l2 * ax / len);
        env.lobe[k][1] = (float)(l2 * ay / len);
        env.lobe[k][2] = (float)(l2 * az / len);
        env.lobe[k][3] = (float)(-l2);
        for (int c = 0; c < 4; c++) {
            if (!std::isfinite(L.amplitude[c]))
                return fail(RT_ERR_INVALID_ARG, "lobe %d: amplitude[%d] is not finite", k, c);
            env.lobe[k][4 + c] = L.amplitude[c];
        }
    }
    rt_status st = check_device();
    if (st != RT_OK) return st;
    hipError_t e = rt::launch_bake_env(W, H, n, C, frames, env, texels, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bake launch");
    return ok();
    RT_GUARD_END
}

namespace {
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) l++;
    return l;
}
}  // namespace

rt_status rt_build_mip(const rt_texture* src, float* dst, void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(src);
    if (st != RT_OK) return st;
    const rt::TexView& v = src->view;
    if (src->fmt != RT_FMT_F32 || src->view.index)
        return fail(RT_ERR_UNSUPPORTED, "mip levels are built from FP32 textures (not dictionaries)");
    if (!pow2(v.W) || !pow2(v.H))
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d: a mip chain needs powers of two", v.W, v.H);
    if (v.W == 1 && v.H == 1) return fail(RT_ERR_INVALID_ARG, "a 1 x 1 matrix has no next level");
    if (!dst) return fail(RT_ERR_INVALID_ARG, "dst is NULL");
    if (!aligned(dst, 16)) return fail(RT_ERR_INVALID_ARG, "dst must be 16-byte aligned");
    hipError_t e = rt::launch_build_mip(v, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mip launch");
    return ok();
    RT_GUARD_END
}

namespace {
// Shared checks of a mip chain: sizes halve from level 0, one n, C and format,
// no 1-bit or dictionary level.
rt_status check_chain(const rt_texture* const* levels, int32_t nlevels, rt::LevelSet* ls) {
    if (!levels) return fail(RT_ERR_INVALID_ARG, "levels is NULL");
    if (nlevels < 1) return fail(RT_ERR_INVALID_ARG, "nlevels = %d < 1", nlevels);
    if (nlevels > rt::MAX_LEVELS)
        return fail(RT_ERR_UNSUPPORTED, "nlevels = %d exceeds %d", nlevels, rt::MAX_LEVELS);
    for (int l = 0; l < nlevels; l++)
        if (!levels[l]) return fail(RT_ERR_INVALID_ARG, "level %d is NULL", l);
    const rt::TexView& v0 = levels[0]->view;
    for (int l = 0; l < nlevels; l++)
        if (levels[l]->fmt == RT_FMT_BIT1 || levels[l]->view.index)
            return fail(RT_ERR_UNSUPPORTED, "mip chains of 1-bit or dictionary textures are not supported");
    if (nlevels > 1) {
        if (!pow2(v0.W) || !pow2(v0.H))
            return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d: a mip chain needs powers of two", v0.W, v0.H);
        if (nlevels > 1 + log2i(std::max(v0.W, v0.H)))
            return fail(RT_ERR_INVALID_ARG, "%d levels exceed the chain of a %d x %d matrix", nlevels, v0.W, v0.H);
    }
    memset(ls, 0, sizeof(*ls));
    ls->levels = nlevels;
    ls->W = v0.W;
    ls->H = v0.H;
    ls->n = v0.n;
    ls->C = v0.C;
    for (int l = 0; l < nlevels; l++) {
        const rt::TexView& v = levels[l]->view;
        const int w = std::max(v0.W >> l, 1), h = std::max(v0.H >> l, 1);
        if (v.W != w || v.H != h)
            return fail(RT_ERR_INVALID_ARG, "level %d is %d x %d, the chain needs %d x %d", l, v.W, v.H, w, h);
        if (v.n != v0.n || v.C != v0.C || levels[l]->fmt != levels[0]->fmt)
            return fail(RT_ERR_INVALID_ARG, "level %d differs from level 0 in n, channels or format", l);
        ls->data[l] = v.data;
        ls->scales[l] = v.scales;
    }
    return RT_OK;
}

// The LOD backward's plan: the chain's buckets numbered one level after the
// other, two units per fragment (its levels l0 and l0 + 1), sparse keys; then
// the workspace layout (the backward's workspace, the units' weighted
// upstream gradient).
bool plan_lod_backward(const rt_texture* const* levels, int nlevels, int64_t N, int mode,
                       rt::BwdPlan* plan, rt::LodBwdLayout* lay) {
    const rt::TexView& v0 = levels[0]->view;
    int64_t nb = 0;
    for (int l = 0; l < nlevels; l++) nb += (int64_t)levels[l]->view.W * levels[l]->view.H;
    if (nb > INT32_MAX || N > INT64_MAX / 2) return false;
    const int64_t units = 2 * N;
    if (!rt::plan_backward((int)nb, 1, v0.n, v0.C, units, mode, plan, true)) return false;
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t u1 = (size_t)std::max<int64_t>(units, 1);
    lay->off_bwd = 0;
    lay->off_gl = a256(plan->total);
    lay->total = lay->off_gl + a256(u1 * v0.C * 4);
    return true;
}
}  // namespace

rt_status rt_lookup_fwd_lod(const rt_texture* const* levels, int32_t nlevels,
                            const rt_fragments* f, const float* duv, float* out, uint32_t flags,
                            void* stream) {
    RT_GUARD_BEGIN
    rt::LevelSet ls;
    rt_status st = check_chain(levels, nlevels, &ls);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (flags > RT_BUCKET_BILINEAR) return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (f->count > 0) {
        if (!duv) return fail(RT_ERR_INVALID_ARG, "duv is NULL");
        if (!aligned(duv, 16)) return fail(RT_ERR_INVALID_ARG, "duv must be 16-byte aligned");
        if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
        if (!aligned(out, out_align(ls.C)))
            return fail(RT_ERR_INVALID_ARG, "out must be %zu-byte aligned", out_align(ls.C));
    }
    hipError_t e = rt::launch_lookup_lod(ls, levels[0]->fmt, (int)flags, f->uv, f->tbn, f->view,
                                         duv, out, fragmap(f), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lod lookup launch");
    return ok();
    RT_GUARD_END
}

size_t rt_lookup_lod_bwd_workspace(const rt_texture* const* levels, int32_t nlevels, int64_t count,
                                   uint32_t flags) {
    try {
        if (!levels || nlevels < 1 || nlevels > rt::MAX_LEVELS || count < 0 ||
            flags > RT_BUCKET_BILINEAR)
            return 0;
        for (int l = 0; l < nlevels; l++)
            if (!levels[l]) return 0;
        rt::BwdPlan plan;
        rt::LodBwdLayout lay;
        if (!plan_lod_backward(levels, nlevels, count, (int)flags, &plan, &lay)) return 0;
        return lay.total;
    } catch (...) {
        return 0;
    }
}

rt_status rt_lookup_lod_bwd(const rt_texture* const* levels, int32_t nlevels,
                            const rt_fragments* f, const float* duv, const float* grad_out,
                            float* const* grad_levels, float* grad_view, float* grad_uv, void* ws,
                            size_t ws_bytes, uint32_t flags, void* stream) {
    RT_GUARD_BEGIN
    rt::LevelSet ls;
    rt_status st = check_chain(levels, nlevels, &ls);
    if (st != RT_OK) return st;
    st = check_frags(f);
    if (st != RT_OK) return st;
    if (flags > RT_BUCKET_BILINEAR) return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (!grad_levels) return fail(RT_ERR_INVALID_ARG, "grad_levels is NULL");
    for (int l = 0; l < nlevels; l++)
        if (grad_levels[l] && !aligned(grad_levels[l], 16))
            return fail(RT_ERR_INVALID_ARG, "grad_levels[%d] must be 16-byte aligned", l);
    if (grad_view && !aligned(grad_view, 4)) return fail(RT_ERR_INVALID_ARG, "grad_view must be 4-byte aligned");
    if (grad_uv && !aligned(grad_uv, 8)) return fail(RT_ERR_INVALID_ARG, "grad_uv must be 8-byte aligned");
    if (f->count > 0) {
        if (!duv || !grad_out) return fail(RT_ERR_INVALID_ARG, "duv and grad_out must be non-NULL");
        if (!aligned(duv, 16)) return fail(RT_ERR_INVALID_ARG, "duv must be 16-byte aligned");
        if (!aligned(grad_out, out_align(ls.C)))
            return fail(RT_ERR_INVALID_ARG, "grad_out must be %zu-byte aligned", out_align(ls.C));
    }
    rt::BwdPlan plan;
    rt::LodBwdLayout lay;
    if (!plan_lod_backward(levels, nlevels, f->count, (int)flags, &plan, &lay))
        return fail(RT_ERR_UNSUPPORTED, "sort key (W*H*n*n), bucket size (n*n*C <= 4096) or record count beyond the backward's limits");
    bool any = grad_view || grad_uv;
    for (int l = 0; l < nlevels; l++) any = any || grad_levels[l];
    if (!any) return ok();  // nothing requested
    if (f->count > 0) {
        if (!ws) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
        if (!aligned(ws, 256)) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        if (ws_bytes < lay.total)
            return fail(RT_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, %zu needed", ws_bytes, lay.total);
    }
    hipError_t e = rt::launch_lookup_lod_bwd(ls, levels[0]->fmt, (int)flags, f->uv, f->tbn,
                                             f->view, duv, grad_out, grad_levels, grad_view,
                                             grad_uv, fragmap(f), plan, lay, ws,
                                             (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lod backward launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_build_mip_adjoint(const rt_texture* src, const float* grad_dst, float* grad_src,
                               void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(src);
    if (st != RT_OK) return st;
    const rt::TexView& v = src->view;
    if (!pow2(v.W) || !pow2(v.H))
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d: a mip chain needs powers of two", v.W, v.H);
    if (v.W == 1 && v.H == 1) return fail(RT_ERR_INVALID_ARG, "a 1 x 1 matrix has no next level");
    if (!grad_dst || !grad_src) return fail(RT_ERR_INVALID_ARG, "grad_dst and grad_src must be non-NULL");
    if (!aligned(grad_dst, 4) || !aligned(grad_src, 4))
        return fail(RT_ERR_INVALID_ARG, "grad_dst and grad_src must be 4-byte aligned");
    hipError_t e = rt::launch_mip_adjoint(v, grad_dst, grad_src, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mip adjoint launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_lookup_light(const rt_texture* t, const rt_fragments* f, const float* pos,
                          const rt_light* light, float* out, uint32_t flags, void* stream) {
    RT_GUARD_BEGIN
    rt_status st = check_tex(t);
    if (st != RT_OK) return st;
    st = check_frags(f, false);
    if (st != RT_OK) return st;
    if (flags > RT_BUCKET_BILINEAR) return fail(RT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (!light) return fail(RT_ERR_INVALID_ARG, "light is NULL");
    if (light->kind != RT_LIGHT_DIRECTIONAL && light->kind != RT_LIGHT_POINT)
        return fail(RT_ERR_INVALID_ARG, "unknown light kind %d", light->kind);
    if (light->samples < 1 || light->samples > RT_MAX_LIGHT_SAMPLES)
        return fail(RT_ERR_INVALID_ARG, "light samples = %d must be in 1..%d", light->samples,
                    RT_MAX_LIGHT_SAMPLES);
    rt::LightParams lp;
    memset(&lp, 0, sizeof(lp));
    lp.kind = light->kind == RT_LIGHT_POINT ? rt::LIGHT_POINT : rt::LIGHT_DIRECTIONAL;
    lp.samples = light->samples;
    lp.inv_samples = 1.0f / (float)light->samples;
    for (int s = 0; s < light->samples; s++)
        for (int k = 0; k < 3; k++) {
            if (!std::isfinite(light->vec[s][k]))
                return fail(RT_ERR_INVALID_ARG, "light sample %d is not finite", s);
            lp.vec[s][k] = light->vec[s][k];
        }
    if (f->count > 0) {
        if (light->kind == RT_LIGHT_POINT) {
            if (!pos) return fail(RT_ERR_INVALID_ARG, "a point light needs the fragments' positions");
            if (!aligned(pos, 4)) return fail(RT_ERR_INVALID_ARG, "pos must be 4-byte aligned");
        }
        if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
        if (!aligned(out, out_align(t->view.C)))
            return fail(RT_ERR_INVALID_ARG, "out must be %zu-byte aligned", out_align(t->view.C));
    }
    hipError_t e = rt::launch_lookup_light(t->view, t->fmt, (int)flags, f->uv, f->tbn,
                                           light->kind == RT_LIGHT_POINT ? pos : nullptr, lp, out,
                                           fragmap(f), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "light lookup launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_bake_shadow(int32_t W, int32_t H, int32_t n, const float* origins,
                         const float* frames, const float* balls, int32_t nballs,
                         uint32_t* words, void* stream) {
    RT_GUARD_BEGIN
    if (W < 1 || H < 1)
        return fail(RT_ERR_INVALID_ARG, "bucket matrix %d x %d must be at least 1 x 1", W, H);
    if (W > 65536 || H > 65536)
        return fail(RT_ERR_UNSUPPORTED, "bucket matrix %d x %d exceeds 65536 per side", W, H);
    if (n < 1) return fail(RT_ERR_INVALID_ARG, "angular resolution n = %d must be >= 1", n);
    if (n > 64) return fail(RT_ERR_UNSUPPORTED, "angular resolution n = %d exceeds 64", n);
    if (nballs < 0) return fail(RT_ERR_INVALID_ARG, "nballs = %d < 0", nballs);
    if (nballs > rt::MAX_OCCLUDERS)
        return fail(RT_ERR_UNSUPPORTED, "nballs = %d exceeds %d", nballs, rt::MAX_OCCLUDERS);
    if (nballs > 0 && !balls) return fail(RT_ERR_INVALID_ARG, "balls is NULL");
    if (!origins) return fail(RT_ERR_INVALID_ARG, "origins is NULL");
    if (!words) return fail(RT_ERR_INVALID_ARG, "words is NULL");
    if (!aligned(origins, 4) || !aligned(words, 4) || (frames && !aligned(frames, 4)))
        return fail(RT_ERR_INVALID_ARG, "origins, frames and words must be 4-byte aligned");
    rt::Occluders occ;
    memset(&occ, 0, sizeof(occ));
    occ.count = nballs;
    for (int k = 0; k < nballs; k++) {
        for (int c = 0; c < 4; c++) {
            if (!std::isfinite(balls[4 * k + c]))
                return fail(RT_ERR_INVALID_ARG, "ball %d is not finite", k);
            occ.ball[k][c] = balls[4 * k + c];
        }
        if (!(balls[4 * k + 3] > 0.f)) return fail(RT_ERR_INVALID_ARG, "ball %d: radius must be > 0", k);
    }
    rt_status st = check_device();
    if (st != RT_OK) return st;
    hipError_t e = rt::launch_bake_shadow(W, H, n, origins, frames, occ, words, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "shadow bake launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_vq_assign(const float* x, int64_t M, int32_t D, const float* codebook, int32_t K,
                       int32_t* assign, float* dist, void* stream) {
    RT_GUARD_BEGIN
    if (M < 0) return fail(RT_ERR_INVALID_ARG, "M = %lld < 0", (long long)M);
    if (M >= (1ll << 31)) return fail(RT_ERR_UNSUPPORTED, "M = %lld >= 2^31", (long long)M);
    if (D < 1) return fail(RT_ERR_INVALID_ARG, "D = %d must be >= 1", D);
    if (K < 1) return fail(RT_ERR_INVALID_ARG, "K = %d must be >= 1", K);
    if (K > 65536) return fail(RT_ERR_UNSUPPORTED, "K = %d exceeds 65536", K);
    if (M == 0) return ok();
    if (!x || !codebook || !assign)
        return fail(RT_ERR_INVALID_ARG, "x, codebook and assign must be non-NULL");
    if (!aligned(x, 16) || !aligned(codebook, 16))
        return fail(RT_ERR_INVALID_ARG, "x and codebook must be 16-byte aligned");
    if (!aligned(assign, 4) || (dist && !aligned(dist, 4)))
        return fail(RT_ERR_INVALID_ARG, "assign and dist must be 4-byte aligned");
    hipError_t e = rt::launch_vq_assign(x, M, D, codebook, K, assign, dist, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "assignment launch");
    return ok();
    RT_GUARD_END
}

size_t rt_vq_update_workspace(int64_t M, int32_t D, int32_t K) {
    try {
        rt::VqPlan p;
        if (!rt::plan_vq_update(M, D, K, &p)) return 0;
        return p.total;
    } catch (...) {
        return 0;
    }
}

rt_status rt_vq_update(const float* x, int64_t M, int32_t D, const int32_t* assign, int32_t K,
                       float* codebook, int32_t* counts, void* ws, size_t ws_bytes,
                       void* stream) {
    RT_GUARD_BEGIN
    if (M < 1) return fail(RT_ERR_INVALID_ARG, "M = %lld must be >= 1", (long long)M);
    if (D < 1) return fail(RT_ERR_INVALID_ARG, "D = %d must be >= 1", D);
    if (K < 1) return fail(RT_ERR_INVALID_ARG, "K = %d must be >= 1", K);
    rt::VqPlan plan;
    if (!rt::plan_vq_update(M, D, K, &plan))
        return fail(RT_ERR_UNSUPPORTED, "the update takes K <= %d entries and M < 2^31 rows",
                    rt::VQ_MAX_UPDATE_ENTRIES);
    if (!x || !assign || !codebook)
        return fail(RT_ERR_INVALID_ARG, "x, assign and codebook must be non-NULL");
    if (!aligned(x, 4) || !aligned(assign, 4) || !aligned(codebook, 4) ||
        (counts && !aligned(counts, 4)))
        return fail(RT_ERR_INVALID_ARG, "x, assign, codebook and counts must be 4-byte aligned");
    if (!ws) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < plan.total)
        return fail(RT_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, %zu needed", ws_bytes, plan.total);
    hipError_t e = rt::launch_vq_update(x, assign, codebook, counts, plan, ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "update launch");
    return ok();
    RT_GUARD_END
}

rt_status rt_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return RT_OK;
}

rt_status rt_profile_reset(void) {
    RT_GUARD_BEGIN
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_locked();
    for (int k = 0; k < rt::K_COUNT; k++) {
        g_total_ms[k] = 0.0;
        g_launches[k] = 0;
    }
    return RT_OK;
    RT_GUARD_END
}

int32_t rt_profile_kernel_count(void) { return rt::K_COUNT; }

const char* rt_profile_kernel_name(int32_t k) { return rt::kernel_name(k); }

rt_status rt_profile_read(int32_t k, int64_t* launches, double* total_ms) {
    RT_GUARD_BEGIN
    if (k < 0 || k >= rt::K_COUNT) return fail(RT_ERR_INVALID_ARG, "kernel id %d out of range", k);
    if (!launches || !total_ms) return fail(RT_ERR_INVALID_ARG, "outputs are NULL");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_locked();
    *launches = g_launches[k];
    *total_ms = g_total_ms[k];
    return RT_OK;
    RT_GUARD_END
}

}  // extern "C"
