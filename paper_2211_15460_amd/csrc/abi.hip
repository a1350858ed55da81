// C ABI entry points (include/fhv.h): host-side validation, workspace
// queries and dispatch to the kernels' launchers on the caller's stream.
#include <new>
#include <string.h>
#include <vector>

#include "fhv_common.h"

namespace fhv {

// Pairs of HIP events around kernel launches, resolved at the end of a
// profiling session into per-name launch counts and summed durations.
struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    hipError_t err = hipSuccess;

    hipEvent_t take()
    {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) err = r;
        return e;
    }
};

void prof_mark(Profiler* p, const char* name, hipStream_t s, bool start)
{
    hipEvent_t e = p->take();
    if (!e) return;
    hipError_t r = hipEventRecord(e, s);
    if (r != hipSuccess) p->err = r;
    if (start) {
        p->recs.push_back({name, e, nullptr});
    } else if (!p->recs.empty() && p->recs.back().b == nullptr) {
        p->recs.back().b = e;
    } else {
        p->spare.push_back(e);
    }
}

}  // namespace fhv

struct fhv_ctx {
    fhv::Device dev;
    fhv::Profiler prof;
};

namespace {

fhv_status hip_status(hipError_t e) { return e == hipSuccess ? FHV_OK : FHV_EHIP + (int)e; }

bool desc_ok(const fhv_capture_desc* d)
{
    if (!d) return false;
    if (d->mode == FHV_PPFL) return d->width >= 1 && d->width <= 16384 && d->height >= 1 && d->height <= 16384;
    if (d->mode == FHV_POFL) return d->levels >= 1 && d->levels <= 11;
    return false;
}

uint64_t n_head_of(const fhv_capture_desc* d)
{
    return d->mode == FHV_PPFL ? (uint64_t)d->width * d->height : 1ull << (3 * d->levels);
}

fhv_status check_lists(const fhv_lists* L, const fhv_capture_desc* d)
{
    if (!L || !L->head || !L->counter || !L->keys) return FHV_EINVAL;
    if (L->n_head != n_head_of(d)) return FHV_EINVAL;
    if (L->capacity >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (L->capacity > 0 && !L->pool) return FHV_EINVAL;
    if ((uintptr_t)L->pool & 15) return FHV_EINVAL;  // 16-byte records
    return FHV_OK;
}

fhv_status set_device(fhv_ctx* ctx)
{
    return hip_status(hipSetDevice(ctx->dev.id));
}

}  // namespace

extern "C" {

fhv_status fhv_create(fhv_ctx** out, int hip_device)
{
    if (!out) return FHV_EINVAL;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_status(e);
    if (hip_device < 0 || hip_device >= n) return FHV_EINVAL;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e != hipSuccess) return hip_status(e);
    fhv_ctx* c = new (std::nothrow) fhv_ctx;
    if (!c) return FHV_EINVAL;
    c->dev.id = hip_device;
    c->dev.cus = cus > 0 ? cus : 256;
    c->dev.prof = nullptr;
    *out = c;
    return FHV_OK;
}

fhv_status fhv_destroy(fhv_ctx* ctx)
{
    if (!ctx) return FHV_OK;
    for (auto& r : ctx->prof.recs) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->prof.spare) (void)hipEventDestroy(e);
    delete ctx;
    return FHV_OK;
}

fhv_status fhv_profile_begin(fhv_ctx* ctx)
{
    if (!ctx) return FHV_EINVAL;
    for (auto& r : ctx->prof.recs) {
        ctx->prof.spare.push_back(r.a);
        if (r.b) ctx->prof.spare.push_back(r.b);
    }
    ctx->prof.recs.clear();
    ctx->prof.err = hipSuccess;
    ctx->dev.prof = &ctx->prof;
    return FHV_OK;
}

fhv_status fhv_profile_end(fhv_ctx* ctx, fhv_kernel_stat* out, uint32_t cap, uint32_t* n_out)
{
    if (!ctx || (cap > 0 && !out) || !n_out) return FHV_EINVAL;
    ctx->dev.prof = nullptr;
    fhv::Profiler& p = ctx->prof;
    std::vector<fhv_kernel_stat> acc;
    hipError_t err = p.err;
    for (auto& r : p.recs) {
        if (!r.b) continue;
        hipError_t e = hipEventSynchronize(r.b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            err = e;
            continue;
        }
        size_t k = 0;
        while (k < acc.size() && strcmp(acc[k].name, r.name) != 0) ++k;
        if (k == acc.size()) acc.push_back({r.name, 0, 0.0});
        acc[k].launches += 1;
        acc[k].total_ms += ms;
    }
    for (size_t k = 0; k < acc.size() && k < cap; ++k) out[k] = acc[k];
    *n_out = (uint32_t)acc.size();
    return hip_status(err);
}

const char* fhv_status_str(fhv_status s)
{
    switch (s) {
    case FHV_OK: return "ok";
    case FHV_EINVAL: return "invalid argument";
    case FHV_EWORKSPACE: return "workspace too small";
    case FHV_ERANGE: return "size out of range";
    default: return s >= FHV_EHIP ? "HIP runtime error" : "unknown status";
    }
}

size_t fhv_capture_workspace(const fhv_capture_desc* desc, uint32_t n_tri)
{
    if (!desc_ok(desc)) return 0;
    return fhv::capture_ws_bytes(desc, n_tri);
}

fhv_status fhv_capture(fhv_ctx* ctx, const fhv_mesh* mesh, const fhv_capture_desc* desc,
                       const fhv_lists* lists, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !mesh || !desc_ok(desc)) return FHV_EINVAL;
    fhv_status st = check_lists(lists, desc);
    if (st != FHV_OK) return st;
    if (mesh->n_tri > 0 && (!mesh->pos || !mesh->rgba || !mesh->tri || mesh->n_vert == 0))
        return FHV_EINVAL;
    if (mesh->n_tri >= (1u << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::capture_ws_bytes(desc, mesh->n_tri)) return FHV_EWORKSPACE;
    if (mesh->n_tri > 0 && !ws) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    return hip_status(fhv::capture_launch(ctx->dev, mesh, desc, lists, ws, (hipStream_t)stream));
}

size_t fhv_compact_workspace(const fhv_capture_desc* desc, uint64_t capacity)
{
    if (!desc_ok(desc)) return 0;
    return fhv::compact_ws_bytes(desc, n_head_of(desc), capacity);
}

fhv_status fhv_compact(fhv_ctx* ctx, const fhv_lists* lists, const fhv_capture_desc* desc,
                       const fhv_pofa* out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !desc_ok(desc) || !out) return FHV_EINVAL;
    fhv_status st = check_lists(lists, desc);
    if (st != FHV_OK) return st;
    if (!out->n_occ || !out->n_frag) return FHV_EINVAL;
    if (out->cap_frag < lists->capacity) return FHV_EINVAL;
    if (lists->capacity > 0 && !out->frag) return FHV_EINVAL;
    if ((uintptr_t)out->frag & 15) return FHV_EINVAL;
    if (out->cap_occ > 0 && (!out->oct_key || !out->oct_off || !out->oct_cnt)) return FHV_EINVAL;
    if (ws_bytes < fhv::compact_ws_bytes(desc, lists->n_head, lists->capacity)) return FHV_EWORKSPACE;
    if (!ws) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    return hip_status(fhv::compact_launch(ctx->dev, lists, desc, out, ws, (hipStream_t)stream));
}

fhv_status fhv_splat(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                     const fhv_view* views, uint32_t n_views, uint64_t* zbuf, uint32_t* rgba,
                     float* depth, uint8_t* cov, fhv_stream stream)
{
    if (!ctx || !arrays || !desc_ok(desc) || !views) return FHV_EINVAL;
    if (n_views == 0 || n_views > fhv::kMaxViews) return FHV_ERANGE;
    if (!zbuf || !rgba || !depth || !cov || !arrays->n_frag) return FHV_EINVAL;
    if (arrays->cap_frag > 0 && (!arrays->frag || !arrays->oct_key)) return FHV_EINVAL;
    if (arrays->cap_frag >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (((uintptr_t)arrays->frag & 15) || ((uintptr_t)zbuf & 15)) return FHV_EINVAL;
    fhv::ViewArgs va;
    memset(&va, 0, sizeof(va));
    va.n_views = n_views;
    va.width = views[0].width;
    va.height = views[0].height;
    va.all_k1 = 1;
    if (va.width < 1 || va.width > 16384 || va.height < 1 || va.height > 16384) return FHV_ERANGE;
    for (uint32_t v = 0; v < n_views; ++v) {
        if (views[v].width != va.width || views[v].height != va.height) return FHV_EINVAL;
        if (views[v].splat_px < 1 || views[v].splat_px > 64) return FHV_EINVAL;
        memcpy(va.m[v], views[v].m, sizeof(va.m[v]));
        va.k[v] = views[v].splat_px;
        if (views[v].splat_px != 1) va.all_k1 = 0;
        va.c[v] = 0.5f - 0.5f * (float)views[v].splat_px;
    }
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::splat_launch(ctx->dev, arrays, desc, va, zbuf, rgba, depth, cov,
                                        arrays->cap_frag, (hipStream_t)stream));
}

static bool fill_dims_ok(uint32_t levels, uint32_t n, uint32_t h, uint32_t w)
{
    if (levels < 1 || levels > 4 || n == 0 || h == 0 || w == 0) return false;
    const uint32_t m = 1u << (levels - 1);
    return h % m == 0 && w % m == 0;
}

uint64_t fhv_unet_param_count(uint32_t levels)
{
    if (levels < 1 || levels > 4) return 0;
    return fhv::nn::param_count(levels);
}

size_t fhv_fill_workspace(uint32_t levels, uint32_t n_img, uint32_t height, uint32_t width, int training)
{
    if (!fill_dims_ok(levels, n_img, height, width)) return 0;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return 0;
    return fhv::nn::fill_ws_bytes(levels, n_img, height, width, training != 0);
}

fhv_status fhv_fill(fhv_ctx* ctx, uint32_t levels, const float* params, const uint32_t* rgba,
                    const float* depth, const uint8_t* cov, uint32_t n_img, uint32_t height,
                    uint32_t width, uint32_t* out_rgba, float* out_residual, void* ws, size_t ws_bytes,
                    fhv_stream stream)
{
    if (!ctx || !params || !rgba || !depth || !cov || !out_rgba || !ws) return FHV_EINVAL;
    if (!fill_dims_ok(levels, n_img, height, width)) return FHV_EINVAL;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::nn::fill_ws_bytes(levels, n_img, height, width, false)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::nn::fill(ctx->dev, levels, params, rgba, depth, cov, n_img, height, width, out_rgba,
                                    out_residual, ws, (hipStream_t)stream));
}

fhv_status fhv_fill_train_step(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m,
                               float* adam_v, uint32_t step, float lr, const uint32_t* rgba,
                               const float* depth, const uint8_t* cov, const uint32_t* target_rgba,
                               uint32_t n_img, uint32_t height, uint32_t width, float* loss_out,
                               float* grad_out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !params || !rgba || !depth || !cov || !target_rgba || !ws) return FHV_EINVAL;
    if (step > 0 && (!adam_m || !adam_v)) return FHV_EINVAL;
    if (!fill_dims_ok(levels, n_img, height, width)) return FHV_EINVAL;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::nn::fill_ws_bytes(levels, n_img, height, width, true)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::nn::train_step(ctx->dev, levels, params, adam_m, adam_v, step, lr, rgba, depth, cov,
                                          target_rgba, n_img, height, width, loss_out, grad_out, ws,
                                          (hipStream_t)stream));
}

}  // extern "C"
