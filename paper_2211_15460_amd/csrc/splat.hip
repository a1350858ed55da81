// Point splatting of per-octant arrays into novel views (Sec. 3.3): every
// fragment is projected, covers a k x k pixel square (at least one pixel),
// and per pixel the nearest fragment wins, as in deferred shading.
//
//   k_zclear   z-buffers <- ~0 (empty)
//   k_splat    one fragment per thread, all views per fragment read: fp32
//              3x4 transform without fused multiply-adds, footprint, 64-bit
//              atomic minimum of (depth bits << 32 | fragment index), with a
//              plain read first so covered pixels skip the atomic
//   k_resolve  per pixel: winner's colour (w1), depth and coverage
#include <math.h>

#include "fhv_common.h"

namespace fhv {

namespace {

__global__ void __launch_bounds__(kBlock) k_zclear(uint64_t* __restrict__ z, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint4* q = (uint4*)z;
    const uint4 e = make_uint4(~0u, ~0u, ~0u, ~0u);
    const uint64_t nq = n / 2;
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (uint64_t i = t; i < nq; i += stride) q[i] = e;
    if (t == 0 && (n & 1)) z[n - 1] = ~0ull;
}

// Position of array fragment r in the view's input space: PPFL
// (px + 1/2, py + 1/2, depth24), POFL grid position + 1/2.
template <int kMode>
__device__ __forceinline__ void frag_pos(const uint4& r, uint64_t key, uint32_t cap_w, float* x,
                                         float* y, float* z)
{
    if (kMode == FHV_PPFL) {
        const uint32_t px = (uint32_t)(key % cap_w), py = (uint32_t)(key / cap_w);
        *x = (float)px + 0.5f;
        *y = (float)py + 0.5f;
        *z = (float)(r.x & 0xFFFFFFu);
    } else {
        const uint32_t kx = compact3(key >> 2), ky = compact3(key >> 1), kz = compact3(key);
        *x = (float)((kx << 8) | (r.x & 0xFFu)) + 0.5f;
        *y = (float)((ky << 8) | ((r.x >> 8) & 0xFFu)) + 0.5f;
        *z = (float)((kz << 8) | ((r.x >> 16) & 0xFFu)) + 0.5f;
    }
}

// One-pixel footprints: target z-buffer entry of fragment i in view v, or
// none (returns false).
__device__ __forceinline__ bool pixel_of(const ViewArgs& va, uint32_t v, float x, float y, float z,
                                         uint64_t i, uint64_t plane, uint64_t* off,
                                         unsigned long long* zk)
{
    const float* M = va.m[v];
    const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    const float fx = floorf(sx + va.c[v]), fy = floorf(sy + va.c[v]);
    const bool ok = d > 0.0f && fx >= 0.0f && fx < (float)va.width && fy >= 0.0f &&
                    fy < (float)va.height;
    *off = ok ? (uint64_t)v * plane + (uint64_t)(uint32_t)fy * va.width + (uint32_t)fx : 0;
    *zk = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(uint32_t)i;
    return ok;
}

template <int kMode>
__global__ void __launch_bounds__(kBlock)
k_splat(const uint4* __restrict__ frag, const uint64_t* __restrict__ oct_key,
        const uint64_t* __restrict__ n_frag, uint64_t cap_frag, uint64_t cap_occ, uint32_t cap_w,
        ViewArgs va, unsigned long long* __restrict__ zbuf)
{
    const uint64_t nf = *n_frag;
    const uint64_t F = nf < cap_frag ? nf : cap_frag;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t plane = (uint64_t)va.width * va.height;
    if (cap_occ == 0) return;   // no table rows: nothing to draw
    if (va.all_k1) {
        // one pixel per view; two fragments per iteration, and the z-buffer
        // reads of all their views issued before any atomic, so that the
        // memory latencies overlap
        for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i0 < F; i0 += 2 * stride) {
            const uint64_t i1 = i0 + stride;
            const bool h1 = i1 < F;
            const uint4 r0 = frag[i0];
            const uint4 r1 = h1 ? frag[i1] : make_uint4(0, 0, 0, 0);
            const bool v0ok = r0.w < cap_occ, v1ok = h1 && r1.w < cap_occ;
            const uint64_t k0 = oct_key[v0ok ? r0.w : 0];
            const uint64_t k1 = oct_key[v1ok ? r1.w : 0];
            float x0, y0, z0, x1, y1, z1;
            frag_pos<kMode>(r0, k0, cap_w, &x0, &y0, &z0);
            frag_pos<kMode>(r1, k1, cap_w, &x1, &y1, &z1);
            for (uint32_t vb = 0; vb < va.n_views; vb += 2) {
                uint64_t off[4];
                unsigned long long zk[4], cur[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint32_t v = vb + j;
                    const bool vv = v < va.n_views;
                    const uint32_t vc = vv ? v : 0;
                    ok[2 * j] = pixel_of(va, vc, x0, y0, z0, i0, plane, &off[2 * j], &zk[2 * j]) && vv && v0ok;
                    ok[2 * j + 1] = pixel_of(va, vc, x1, y1, z1, i1, plane, &off[2 * j + 1], &zk[2 * j + 1]) && vv && v1ok;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) cur[q] = zbuf[ok[q] ? off[q] : 0];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (ok[q] && zk[q] < cur[q]) atomicMin(zbuf + off[q], zk[q]);
            }
        }
        return;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < F; i += stride) {
        const uint4 r = frag[i];
        if (r.w >= cap_occ) continue;   // table row not stored
        float x, y, z;
        frag_pos<kMode>(r, oct_key[r.w], cap_w, &x, &y, &z);
        for (uint32_t v = 0; v < va.n_views; ++v) {
            const float* M = va.m[v];
            const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
            const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
            const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
            if (!(d > 0.0f)) continue;
            const float fx = floorf(sx + va.c[v]), fy = floorf(sy + va.c[v]);
            if (!(fx > -1073741824.0f && fx < 1073741824.0f)) continue;
            if (!(fy > -1073741824.0f && fy < 1073741824.0f)) continue;
            const int32_t k = (int32_t)va.k[v];
            int32_t xa = (int32_t)fx, ya = (int32_t)fy;
            int32_t xb = xa + k, yb = ya + k;   // exclusive
            xa = xa < 0 ? 0 : xa;
            ya = ya < 0 ? 0 : ya;
            xb = xb > (int32_t)va.width ? (int32_t)va.width : xb;
            yb = yb > (int32_t)va.height ? (int32_t)va.height : yb;
            const unsigned long long zk =
                ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(uint32_t)i;
            unsigned long long* zb = zbuf + (uint64_t)v * plane;
            for (int32_t yy = ya; yy < yb; ++yy)
                for (int32_t xx = xa; xx < xb; ++xx) {
                    unsigned long long* p = zb + (uint64_t)yy * va.width + xx;
                    if (zk < *p) atomicMin(p, zk);
                }
        }
    }
}

// Batches: the fragment's scene is the high part of its key (key >> 3L);
// it draws only into its scene's views, whose matrices are read from device
// memory [scene][view][12]. When every fragment of a wave belongs to one
// scene (the usual case: arrays are in key order) the scene index is made
// wave-uniform so that the matrix reads become scalar loads.
struct BatchArgs {
    uint32_t n_scenes, n_views, width, height, k, shift;
    float c;   // 1/2 - k/2
};

__device__ __forceinline__ void splat_batch_one(const float* __restrict__ vm, uint32_t scene,
                                                const BatchArgs& a, float x, float y, float z, uint32_t i,
                                                unsigned long long* __restrict__ zbuf)
{
    const uint64_t plane = (uint64_t)a.width * a.height;
    const unsigned long long idx = (unsigned long long)i;
    if (a.k == 1) {
        for (uint32_t vb = 0; vb < a.n_views; vb += 4) {
            uint64_t off[4];
            unsigned long long zk[4], cur[4];
            bool ok[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t v = vb + j;
                ok[j] = false;
                off[j] = 0;
                zk[j] = 0;
                if (v < a.n_views) {
                    const uint64_t pl = (uint64_t)scene * a.n_views + v;
                    const float* M = vm + pl * 12;
                    const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
                    const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
                    const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
                    const float fx = floorf(sx + a.c), fy = floorf(sy + a.c);
                    ok[j] = d > 0.0f && fx >= 0.0f && fx < (float)a.width && fy >= 0.0f && fy < (float)a.height;
                    if (ok[j]) off[j] = pl * plane + (uint64_t)(uint32_t)fy * a.width + (uint32_t)fx;
                    zk[j] = ((unsigned long long)__float_as_uint(d) << 32) | idx;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) cur[j] = ok[j] ? zbuf[off[j]] : 0ull;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ok[j] && zk[j] < cur[j]) atomicMin(zbuf + off[j], zk[j]);
        }
        return;
    }
    for (uint32_t v = 0; v < a.n_views; ++v) {
        const uint64_t pl = (uint64_t)scene * a.n_views + v;
        const float* M = vm + pl * 12;
        const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
        const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
        const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
        if (!(d > 0.0f)) continue;
        const float fx = floorf(sx + a.c), fy = floorf(sy + a.c);
        if (!(fx > -1073741824.0f && fx < 1073741824.0f)) continue;
        if (!(fy > -1073741824.0f && fy < 1073741824.0f)) continue;
        const int32_t k = (int32_t)a.k;
        int32_t xa = (int32_t)fx, ya = (int32_t)fy;
        int32_t xb = xa + k, yb = ya + k;   // exclusive
        xa = xa < 0 ? 0 : xa;
        ya = ya < 0 ? 0 : ya;
        xb = xb > (int32_t)a.width ? (int32_t)a.width : xb;
        yb = yb > (int32_t)a.height ? (int32_t)a.height : yb;
        const unsigned long long zk = ((unsigned long long)__float_as_uint(d) << 32) | idx;
        unsigned long long* zb = zbuf + pl * plane;
        for (int32_t yy = ya; yy < yb; ++yy)
            for (int32_t xx = xa; xx < xb; ++xx) {
                unsigned long long* p = zb + (uint64_t)yy * a.width + xx;
                if (zk < *p) atomicMin(p, zk);
            }
    }
}

__global__ void __launch_bounds__(kBlock)
k_splat_batch(const uint4* __restrict__ frag, const uint64_t* __restrict__ oct_key,
              const uint64_t* __restrict__ n_frag, uint64_t cap_frag, uint64_t cap_occ,
              const float* __restrict__ vm, BatchArgs a, unsigned long long* __restrict__ zbuf)
{
    const uint64_t nf = *n_frag;
    const uint64_t F = nf < cap_frag ? nf : cap_frag;
    if (cap_occ == 0) return;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t kmask = (1ull << a.shift) - 1ull;
    // whole waves iterate together (stride and wave bases are multiples of
    // 64), so the ballots below see every lane
    const uint64_t Fw = (F + kWave - 1) & ~(uint64_t)(kWave - 1);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < Fw; i += stride) {
        bool act = i < F;
        const uint4 r = act ? frag[i] : make_uint4(0, 0, 0, 0);
        act = act && r.w < cap_occ;
        const uint64_t key = act ? oct_key[r.w] : 0ull;
        const uint32_t scene = (uint32_t)(key >> a.shift);
        act = act && scene < a.n_scenes;
        const uint64_t live = __ballot(act);
        if (live == 0) continue;
        float x, y, z;
        frag_pos<FHV_POFL>(r, key & kmask, 0, &x, &y, &z);
        const int leader = __ffsll((unsigned long long)live) - 1;
        const uint32_t s0 = uniform32((uint32_t)__shfl((int)scene, leader, kWave));
        const bool one_scene = __ballot(act && scene != s0) == 0;
        if (!act) continue;
        if (one_scene)
            splat_batch_one(vm, s0, a, x, y, z, (uint32_t)i, zbuf);
        else
            splat_batch_one(vm, scene, a, x, y, z, (uint32_t)i, zbuf);
    }
}

__global__ void __launch_bounds__(kBlock)
k_resolve(const unsigned long long* __restrict__ zbuf, const uint4* __restrict__ frag, uint64_t n,
          uint32_t* __restrict__ rgba, float* __restrict__ depth, uint8_t* __restrict__ cov)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += stride) {
        const unsigned long long zk = zbuf[p];
        if (zk == ~0ull) {
            rgba[p] = 0u;
            depth[p] = 0.0f;
            cov[p] = 0;
        } else {
            const uint32_t id = (uint32_t)zk;
            rgba[p] = frag[id].y;
            depth[p] = __uint_as_float((uint32_t)(zk >> 32));
            cov[p] = 1;
        }
    }
}

}  // namespace

hipError_t splat_launch(const Device& dev, const fhv_pofa* a, const fhv_capture_desc* d,
                        const ViewArgs& va, uint64_t* zbuf, uint32_t* rgba, float* depth,
                        uint8_t* cov, uint64_t max_frag, hipStream_t s)
{
    const uint64_t n = (uint64_t)va.n_views * va.width * va.height;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    uint64_t gz = (n / 2 + kBlock - 1) / kBlock;
    gz = gz < 1 ? 1 : (gz > gmax ? gmax : gz);
    hipError_t e;
    {
        ProfScope ps(dev, "splat.zclear", s);
        k_zclear<<<dim3((unsigned)gz), dim3(kBlock), 0, s>>>(zbuf, n);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const uint64_t smax = (uint64_t)dev.cus * dev.tune.splat_wg;
    uint64_t gs = (max_frag + kBlock - 1) / kBlock;
    gs = gs < 1 ? 1 : (gs > smax ? smax : gs);
    {
    ProfScope ps(dev, "splat.splat", s);
    if (d->mode == FHV_PPFL)
        k_splat<FHV_PPFL><<<dim3((unsigned)gs), dim3(kBlock), 0, s>>>(
            (const uint4*)a->frag, a->oct_key, a->n_frag, a->cap_frag, a->cap_occ, d->width, va,
            (unsigned long long*)zbuf);
    else
        k_splat<FHV_POFL><<<dim3((unsigned)gs), dim3(kBlock), 0, s>>>(
            (const uint4*)a->frag, a->oct_key, a->n_frag, a->cap_frag, a->cap_occ, d->width, va,
            (unsigned long long*)zbuf);
    e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    uint64_t gr = (n + kBlock - 1) / kBlock;
    gr = gr < 1 ? 1 : (gr > gmax ? gmax : gr);
    ProfScope ps(dev, "splat.resolve", s);
    k_resolve<<<dim3((unsigned)gr), dim3(kBlock), 0, s>>>((const unsigned long long*)zbuf,
                                                          (const uint4*)a->frag, n, rgba, depth, cov);
    return hipGetLastError();
}

}  // namespace fhv

namespace fhv {

hipError_t splat_batch_launch(const Device& dev, const fhv_pofa* a, uint32_t levels, const BatchViews& bv,
                              uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov,
                              uint64_t max_frag, hipStream_t s)
{
    const uint64_t n = (uint64_t)bv.n_scenes * bv.n_views * bv.width * bv.height;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    uint64_t gz = (n / 2 + kBlock - 1) / kBlock;
    gz = gz < 1 ? 1 : (gz > gmax ? gmax : gz);
    hipError_t e;
    {
        ProfScope ps(dev, "splat.zclear", s);
        k_zclear<<<dim3((unsigned)gz), dim3(kBlock), 0, s>>>(zbuf, n);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    BatchArgs ba;
    ba.n_scenes = bv.n_scenes;
    ba.n_views = bv.n_views;
    ba.width = bv.width;
    ba.height = bv.height;
    ba.k = bv.k;
    ba.shift = 3 * levels;
    ba.c = 0.5f - 0.5f * (float)bv.k;
    const uint64_t smax = (uint64_t)dev.cus * dev.tune.splat_wg;
    uint64_t gs = (max_frag + kBlock - 1) / kBlock;
    gs = gs < 1 ? 1 : (gs > smax ? smax : gs);
    {
        ProfScope ps(dev, "splat.splat", s);
        k_splat_batch<<<dim3((unsigned)gs), dim3(kBlock), 0, s>>>(
            (const uint4*)a->frag, a->oct_key, a->n_frag, a->cap_frag, a->cap_occ, bv.m, ba,
            (unsigned long long*)zbuf);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    uint64_t gr = (n + kBlock - 1) / kBlock;
    gr = gr < 1 ? 1 : (gr > gmax ? gmax : gr);
    ProfScope ps(dev, "splat.resolve", s);
    k_resolve<<<dim3((unsigned)gr), dim3(kBlock), 0, s>>>((const unsigned long long*)zbuf,
                                                          (const uint4*)a->frag, n, rgba, depth, cov);
    return hipGetLastError();
}

}  // namespace fhv
