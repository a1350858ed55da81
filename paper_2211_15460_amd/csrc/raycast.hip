// Ray casting of per-octant arrays (Sec. 3.3, evaluation by ray casting).
//
// The occupancy of every octree level is rebuilt from the table of occupied
// leaves (Sec. 3.1: coarser levels hold only the occupancy of their
// children, for empty-space skipping), then one lane per output pixel walks
// the octree from the root, descending only into occupied children whose box
// can project onto the pixel, and tests the fragments of every leaf it
// reaches. With an orthographic view the ray of a pixel meets a fragment when
// the fragment projects into that pixel (the one-pixel footprint of the
// splat). The fragments met are kept in a per-lane list ordered by (depth
// bits, index) and composited front to back; when more are met than the list
// holds, the walk is repeated for the fragments behind the last one
// composited, until the transmittance falls below the threshold.
//
//   k_occ_build   one thread per table row: the row's leaf bit and, where
//                 the row is the first of its parent octant, the bits of its
//                 ancestors (rows are in Morton order, so a parent's first
//                 row sets it once)
//   k_raycast     one lane per pixel, 8 x 8 pixels per wave
//
// Workspace: level l (1 <= l <= L) has a bitmap of 8^l bits in Morton order
// (the 8 children of octant n of level l-1 are byte n of level l's bitmap);
// the leaf level has, per 64-bit word, the number of set bits before it,
// which turns a leaf's Morton code into its table row.
#include "fhv_common.h"
#include "scan.h"

namespace fhv {

namespace {

constexpr int kCap = 16;   // fragments a lane keeps per walk

struct OccLayout {
    uint64_t word[kMaxRayLevels + 2];   // u32 offset of level l's bitmap, l = 1..L; [L+1] = end
    uint64_t n64;                       // 64-bit words of the leaf bitmap
};

OccLayout occ_layout(uint32_t L)
{
    OccLayout o{};
    uint64_t w = 0;
    for (uint32_t l = 1; l <= L; ++l) {
        o.word[l] = w;
        const uint64_t bits = 1ull << (3 * l);
        uint64_t words = (bits + 31) / 32;
        words = (words + 1) & ~1ull;   // 8-byte aligned levels
        w += words;
    }
    o.word[L + 1] = w;
    o.n64 = ((1ull << (3 * L)) + 63) / 64;
    return o;
}

__global__ void __launch_bounds__(kBlock)
k_occ_build(const uint64_t* __restrict__ oct_key, const uint64_t* __restrict__ n_occ, uint64_t cap_occ,
            uint32_t* __restrict__ occ, OccLayout lay, uint32_t L)
{
    const uint64_t n = *n_occ < cap_occ ? *n_occ : cap_occ;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) {
        const uint64_t key = oct_key[r];
        const uint64_t prev = r > 0 ? oct_key[r - 1] : ~0ull;
        for (uint32_t l = L; l >= 1; --l) {
            const uint32_t sh = 3 * (L - l);
            const uint64_t b = key >> sh;
            if (l < L && r > 0 && (prev >> sh) == b) break;   // set by an earlier row
            atomicOr(occ + lay.word[l] + (b >> 5), 1u << (b & 31));
        }
    }
}

struct LoadPopc {
    const uint64_t* bits;
    __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)__popcll(bits[i]); }
};

struct RayArgs {
    float m[kMaxViews][12];
    const uint4* frag;
    const uint32_t* oct_off;
    const uint32_t* oct_cnt;
    const uint32_t* occ;
    const uint32_t* rank;   // set leaf bits before each 64-bit word
    OccLayout lay;
    float4* out;            // [V][H][W]
    uint32_t L, width, height, tiles_x, n_tiles;
    float tau;
};

__device__ __forceinline__ float proj(const float* M, int row, float x, float y, float z)
{
    return ((M[4 * row + 0] * x + M[4 * row + 1] * y) + M[4 * row + 2] * z) + M[4 * row + 3];
}

template <int kMode>
__global__ void __launch_bounds__(kBlock) k_raycast(RayArgs a)
{
    // per-lane fragment list, interleaved so that lanes hit distinct banks
    __shared__ uint64_t lst[kCap * kBlock];
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x * (kBlock / kWave) + wv;
    if (tile >= a.n_tiles) return;
    const uint32_t px = (tile % a.tiles_x) * 8 + (lane & 7), py = (tile / a.tiles_x) * 8 + (lane >> 3);
    if (px >= a.width || py >= a.height) return;
    const uint32_t v = blockIdx.y;
    const float* M = a.m[v];
    const uint32_t L = a.L;
    const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
    const float ax = fabsf(M[0]) + fabsf(M[1]) + fabsf(M[2]), ay = fabsf(M[4]) + fabsf(M[5]) + fabsf(M[6]);
    constexpr float kSlack = 0.5f + 0.0625f;   // half a pixel, and room for rounding
    const uint8_t* const occ8 = (const uint8_t*)a.occ;
    const uint64_t* const leaf64 = (const uint64_t*)(a.occ + a.lay.word[L]);
    uint64_t* const my = lst + threadIdx.x;

    // children of octant n (level l, origin o in leaves) that are occupied and
    // whose box can project onto the pixel
    auto expand = [&](uint32_t l, uint32_t n, uint32_t ox, uint32_t oy, uint32_t oz) -> uint32_t {
        uint32_t m = occ8[a.lay.word[l + 1] * 4 + n];
        const uint32_t hc = 1u << (L - l - 1);            // child side in leaves
        const float hw = (float)hc * 128.0f;              // half side in grid units
        uint32_t keep = 0;
        for (uint32_t mm = m; mm; mm &= mm - 1) {
            const uint32_t c = __ffs(mm) - 1;
            const float X = (float)((ox + ((c >> 2) & 1u) * hc) * 256u) + hw;
            const float Y = (float)((oy + ((c >> 1) & 1u) * hc) * 256u) + hw;
            const float Z = (float)((oz + (c & 1u) * hc) * 256u) + hw;
            const float sx = proj(M, 0, X, Y, Z), sy = proj(M, 1, X, Y, Z);
            if (fabsf(sx - pcx) <= hw * ax + kSlack && fabsf(sy - pcy) <= hw * ay + kSlack) keep |= 1u << c;
        }
        return keep;
    };

    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
    uint64_t after = 0;   // keys at or below this were composited (first walk: none)
    bool first = true;
    for (;;) {
        uint32_t n_in = 0;
        bool over = false;
        uint64_t nearest = ~0ull;
        auto take = [&](uint64_t key) {
            if (!first && key <= after) return;
            if (kMode == 0) {
                nearest = key < nearest ? key : nearest;
                return;
            }
            if (n_in == kCap) {
                over = true;
                if (key >= my[(kCap - 1) * kBlock]) return;
                n_in = kCap - 1;   // the farthest kept fragment makes room
            }
            uint32_t j = n_in;
            while (j > 0 && my[(j - 1) * kBlock] > key) {
                my[j * kBlock] = my[(j - 1) * kBlock];
                --j;
            }
            my[j * kBlock] = key;
            ++n_in;
        };
        // depth-first walk without a stack: per level the children still to
        // visit (8 bits each, levels 0..7 and 8..15 in two words)
        uint64_t mlo = 0, mhi = 0;
        auto get_m = [&](uint32_t l) -> uint32_t {
            return (uint32_t)(((l < 8 ? mlo : mhi) >> ((l & 7) * 8)) & 0xFFu);
        };
        auto set_m = [&](uint32_t l, uint32_t m) {
            const uint32_t sh = (l & 7) * 8;
            if (l < 8)
                mlo = (mlo & ~(0xFFull << sh)) | ((uint64_t)m << sh);
            else
                mhi = (mhi & ~(0xFFull << sh)) | ((uint64_t)m << sh);
        };
        uint32_t l = 0, n = 0, ox = 0, oy = 0, oz = 0;
        set_m(0, expand(0, 0, 0, 0, 0));
        for (;;) {
            const uint32_t m = get_m(l);
            if (m == 0) {
                if (l == 0) break;
                --l;
                n >>= 3;
                const uint32_t side = 1u << (L - l);
                ox &= ~(side - 1);
                oy &= ~(side - 1);
                oz &= ~(side - 1);
                continue;
            }
            const uint32_t c = __ffs(m) - 1;
            set_m(l, m & (m - 1));
            const uint32_t hc = 1u << (L - l - 1);
            const uint32_t cx = ox + ((c >> 2) & 1u) * hc, cy = oy + ((c >> 1) & 1u) * hc,
                           cz = oz + (c & 1u) * hc;
            const uint32_t cn = n * 8 + c;
            if (l + 1 < L) {
                ++l;
                n = cn;
                ox = cx;
                oy = cy;
                oz = cz;
                set_m(l, expand(l, n, ox, oy, oz));
                continue;
            }
            // leaf cn: its table row from the set bits before it
            const uint64_t w = leaf64[cn >> 6];
            const uint32_t row = a.rank[cn >> 6] + (uint32_t)__popcll(w & ((1ull << (cn & 63)) - 1ull));
            const uint32_t off = a.oct_off[row], cnt = a.oct_cnt[row];
            for (uint32_t i = off; i < off + cnt; ++i) {
                const uint4 r = a.frag[i];
                const float x = (float)((cx << 8) | (r.x & 0xFFu)) + 0.5f;
                const float y = (float)((cy << 8) | ((r.x >> 8) & 0xFFu)) + 0.5f;
                const float z = (float)((cz << 8) | ((r.x >> 16) & 0xFFu)) + 0.5f;
                const float d = proj(M, 2, x, y, z);
                if (!(d > 0.0f)) continue;
                if (floorf(proj(M, 0, x, y, z)) != (float)px || floorf(proj(M, 1, x, y, z)) != (float)py) continue;
                take(((uint64_t)__float_as_uint(d) << 32) | i);
            }
        }
        // composite what this walk kept, nearest first
        bool done = true;
        if (kMode == 0) {
            if (nearest != ~0ull) {
                const uint32_t rgba = a.frag[(uint32_t)nearest].y;
                C0 = (float)(rgba & 0xFFu) / 255.0f;
                C1 = (float)((rgba >> 8) & 0xFFu) / 255.0f;
                C2 = (float)((rgba >> 16) & 0xFFu) / 255.0f;
                T = 0.0f;
            }
        } else {
            uint32_t j = 0;
            for (; j < n_in; ++j) {
                const uint32_t rgba = a.frag[(uint32_t)my[j * kBlock]].y;
                const float al = (float)(rgba >> 24) / 255.0f;
                const float wgt = T * al;
                C0 = C0 + wgt * ((float)(rgba & 0xFFu) / 255.0f);
                C1 = C1 + wgt * ((float)((rgba >> 8) & 0xFFu) / 255.0f);
                C2 = C2 + wgt * ((float)((rgba >> 16) & 0xFFu) / 255.0f);
                T = T * (1.0f - al);
                if (T < a.tau || T == 0.0f) break;
            }
            done = j < n_in || !over;
            if (!done) after = my[(n_in - 1) * kBlock];
        }
        if (done) break;
        first = false;
    }
    a.out[((size_t)v * a.height + py) * a.width + px] = make_float4(C0, C1, C2, 1.0f - T);
}

}  // namespace

size_t raycast_ws_bytes(uint32_t levels)
{
    if (levels < 1 || levels > kMaxRayLevels) return 0;
    const OccLayout o = occ_layout(levels);
    const size_t occ_b = (size_t)o.word[levels + 1] * 4;
    const size_t rank_b = ((size_t)o.n64 * 4 + 255) & ~(size_t)255;
    const size_t part_b = (scan_partials(o.n64) * 4 + 255) & ~(size_t)255;
    return ((occ_b + 255) & ~(size_t)255) + rank_b + part_b;
}

hipError_t raycast_launch(const Device& dev, const fhv_pofa* p, uint32_t levels, const RayViews& rv,
                          uint32_t mode, float tau, float* out, void* ws, hipStream_t s)
{
    const OccLayout lay = occ_layout(levels);
    const size_t occ_b = (((size_t)lay.word[levels + 1] * 4) + 255) & ~(size_t)255;
    const size_t rank_b = ((size_t)lay.n64 * 4 + 255) & ~(size_t)255;
    uint32_t* occ = (uint32_t*)ws;
    uint32_t* rank = (uint32_t*)((char*)ws + occ_b);
    uint32_t* part = (uint32_t*)((char*)ws + occ_b + rank_b);
    hipError_t e;
    {
        ProfScope ps(dev, "ray.occupancy", s);
        e = fill_u32(occ, lay.word[levels + 1], 0u, s);
        if (e != hipSuccess) return e;
        if (p->cap_occ > 0) {
            uint64_t g = (p->cap_occ + kBlock - 1) / kBlock;
            const uint64_t gmax = (uint64_t)dev.cus * 8;
            g = g > gmax ? gmax : g;
            k_occ_build<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(p->oct_key, p->n_occ, p->cap_occ, occ, lay,
                                                                  levels);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        e = scan<uint32_t>(LoadPopc{(const uint64_t*)(occ + lay.word[levels])}, StoreExcl<uint32_t>{rank},
                           lay.n64, part, (uint32_t*)nullptr, s);
        if (e != hipSuccess) return e;
    }
    RayArgs a;
    for (uint32_t v = 0; v < rv.n_views; ++v)
        for (int k = 0; k < 12; ++k) a.m[v][k] = rv.m[v][k];
    a.frag = (const uint4*)p->frag;
    a.oct_off = p->oct_off;
    a.oct_cnt = p->oct_cnt;
    a.occ = occ;
    a.rank = rank;
    a.lay = lay;
    a.out = (float4*)out;
    a.L = levels;
    a.width = rv.width;
    a.height = rv.height;
    a.tiles_x = (rv.width + 7) / 8;
    a.n_tiles = a.tiles_x * ((rv.height + 7) / 8);
    a.tau = tau;
    const dim3 grid((a.n_tiles + kBlock / kWave - 1) / (kBlock / kWave), rv.n_views);
    ProfScope ps(dev, "ray.cast", s);
    if (mode == FHV_RAY_NEAREST)
        k_raycast<0><<<grid, dim3(kBlock), 0, s>>>(a);
    else
        k_raycast<1><<<grid, dim3(kBlock), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fhv
