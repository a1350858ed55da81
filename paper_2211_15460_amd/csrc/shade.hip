// Shading of the splat's nearest fragments (Sec. 5: a local illumination
// model per fragment, Phong 1975 / Blinn 1977), one thread per pixel: the
// winner's packed normal is unfolded from the octahedron and normalised,
// flipped towards the viewer (surfaces are captured without culling), and
// lit by one directional light with ambient, diffuse and specular terms; the
// specular power is 2^shine, reached by repeated squaring. fp32, every
// operation in the order written and without fused multiply-adds, so that
// the result is reproducible bit for bit.
#include <math.h>

#include "fhv_common.h"

namespace fhv {

namespace {

__global__ void __launch_bounds__(kBlock)
k_shade(const uint4* __restrict__ frag, const unsigned long long* __restrict__ zbuf, uint64_t n_pix,
        uint32_t n_views, ShadeArgs a, float4* __restrict__ out)
{
    const uint64_t n = n_pix * n_views;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += stride) {
        const unsigned long long z = zbuf[p];
        if (z == ~0ull) {
            out[p] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            continue;
        }
        const uint32_t v = (uint32_t)(p / n_pix);
        const float* L = a.l[v];
        const float* V = a.v[v];
        const float* H = a.h[v];
        const uint4 r = frag[(uint32_t)z];
        float px = (float)(int16_t)(r.z & 0xFFFFu) / 32767.0f;
        float py = (float)(int16_t)(r.z >> 16) / 32767.0f;
        const float nz = (1.0f - fabsf(px)) - fabsf(py);
        if (nz < 0.0f) {
            const float tx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
            const float ty = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
            px = tx;
            py = ty;
        }
        const float len = sqrtf((px * px + py * py) + nz * nz);
        float n0 = px / len, n1 = py / len, n2 = nz / len;
        if ((n0 * V[0] + n1 * V[1]) + n2 * V[2] < 0.0f) {
            n0 = -n0;
            n1 = -n1;
            n2 = -n2;
        }
        const float ndl = (n0 * L[0] + n1 * L[1]) + n2 * L[2];
        const float ndh = (n0 * H[0] + n1 * H[1]) + n2 * H[2];
        const float d = ndl > 0.0f ? ndl : 0.0f;
        float sp = (ndl > 0.0f && ndh > 0.0f) ? ndh : 0.0f;
        for (uint32_t k = 0; k < a.shine[v]; ++k) sp = sp * sp;
        const float amb = a.ka[v] + a.kd[v] * d, spec = a.ks[v] * sp;
        out[p] = make_float4((float)(r.y & 0xFFu) / 255.0f * amb + spec,
                             (float)((r.y >> 8) & 0xFFu) / 255.0f * amb + spec,
                             (float)((r.y >> 16) & 0xFFu) / 255.0f * amb + spec, 1.0f);
    }
}

}  // namespace

hipError_t shade_launch(const Device& dev, const fhv_pofa* p, const uint64_t* zbuf, uint32_t n_views,
                        uint64_t n_pix, const ShadeArgs& a, float* out, hipStream_t s)
{
    const uint64_t n = n_pix * n_views;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    uint64_t g = (n + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : (g > gmax ? gmax : g);
    ProfScope ps(dev, "shade", s);
    k_shade<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>((const uint4*)p->frag, (const unsigned long long*)zbuf,
                                                        n_pix, n_views, a, (float4*)out);
    return hipGetLastError();
}

}  // namespace fhv
