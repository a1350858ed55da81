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
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < F; i += stride) {
        const uint4 r = frag[i];
        if (r.w >= cap_occ) continue;   // table row not stored
        const uint64_t key = oct_key[r.w];
        float x, y, z;
        if (kMode == FHV_PPFL) {
            const uint32_t px = (uint32_t)(key % cap_w), py = (uint32_t)(key / cap_w);
            x = (float)px + 0.5f;
            y = (float)py + 0.5f;
            z = (float)(r.x & 0xFFFFFFu);
        } else {
            const uint32_t k32 = (uint32_t)key;
            const uint32_t kx = compact3(k32 >> 2), ky = compact3(k32 >> 1), kz = compact3(k32);
            x = (float)((kx << 8) | (r.x & 0xFFu)) + 0.5f;
            y = (float)((ky << 8) | ((r.x >> 8) & 0xFFu)) + 0.5f;
            z = (float)((kz << 8) | ((r.x >> 16) & 0xFFu)) + 0.5f;
        }
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
            int32_t x0 = (int32_t)fx, y0 = (int32_t)fy;
            int32_t x1 = x0 + k, y1 = y0 + k;   // exclusive
            x0 = x0 < 0 ? 0 : x0;
            y0 = y0 < 0 ? 0 : y0;
            x1 = x1 > (int32_t)va.width ? (int32_t)va.width : x1;
            y1 = y1 > (int32_t)va.height ? (int32_t)va.height : y1;
            const unsigned long long zk =
                ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(uint32_t)i;
            unsigned long long* zb = zbuf + (uint64_t)v * plane;
            for (int32_t yy = y0; yy < y1; ++yy)
                for (int32_t xx = x0; xx < x1; ++xx) {
                    unsigned long long* p = zb + (uint64_t)yy * va.width + xx;
                    if (zk < *p) atomicMin(p, zk);
                }
        }
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
    uint64_t gs = (max_frag + kBlock - 1) / kBlock;
    gs = gs < 1 ? 1 : (gs > gmax ? gmax : gs);
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
