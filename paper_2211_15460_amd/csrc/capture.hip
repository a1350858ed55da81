// Capture: rasterize every triangle into per-pixel (PPFL) or per-octant
// (POFL) fragment lists (Sec. 3.1 "Simple Layout" / "Octree Layout",
// Sec. 3.2 FHV_PPFL / FHV_POFL).
//
// Kernels, in stream order:
//   fills     head <- 0xFFFFFFFF, counter <- 0
//   k_setup   one thread per triangle: fixed-point vertices (PPFL: viewport
//             transform; POFL: grid snap, exact integer normal, octahedral
//             packing, tangent frame of the packed normal, projection),
//             orientation, sample bounding box, number of sample tiles of
//             64 samples (8x8, 16x4 or 32x2, a launch choice)
//   scan      inclusive prefix sum of tiles per triangle
//   k_raster  work items are (triangle, tile) pairs; a wave takes a
//             contiguous range of them and processes one tile at a time, one
//             lane per sample: integer edge functions with the top-left
//             rule, integer attribute interpolation, list append
//
// List append (Sec. 3.2): the wave counts its range's covered samples and
// reserves their slots with one atomic add on the global counter (instead
// of one increment per fragment; the slots are the same set). Each lane with
// a slot below the capacity swaps its index into the key's head and stores
// {w0, rgba, normal, previous head} plus the key sidecar. Without a head
// array (batches that only want arrays) the exchange is skipped and the
// link is 0xFFFFFFFF.
//
// The fp64 setup relies on IEEE-correct add, mul, div, sqrt and rint and on
// no contraction into fused multiply-adds (built with -ffp-contract=off):
// the tangent frame is then reproducible operation by operation.
#include <math.h>

#include "fhv_common.h"

namespace fhv {

namespace {

__device__ __forceinline__ int32_t round_snorm(int64_t num, int64_t l1)
{
    const int64_t a = num < 0 ? -num : num;
    const int64_t q = (2 * 32767 * a + l1) / (2 * l1);
    return (int32_t)(num < 0 ? -q : q);
}

// Exact octahedral packing of an integer normal (Cigolle et al. 2014):
// n / |n|_1 folded when n_z < 0, components rounded to multiples of
// 1/32767 with halves away from zero; int16 x | int16 y << 16.
__device__ uint32_t oct_pack(int64_t nx, int64_t ny, int64_t nz)
{
    const int64_t ax = nx < 0 ? -nx : nx, ay = ny < 0 ? -ny : ny, az = nz < 0 ? -nz : nz;
    const int64_t l1 = ax + ay + az;
    if (l1 == 0) return 0;
    int32_t qx, qy;
    if (nz >= 0) {
        qx = round_snorm(nx, l1);
        qy = round_snorm(ny, l1);
    } else {
        qx = round_snorm(nx < 0 ? -(l1 - ay) : (l1 - ay), l1);
        qy = round_snorm(ny < 0 ? -(l1 - ax) : (l1 - ax), l1);
    }
    return (uint32_t)(uint16_t)(int16_t)qx | ((uint32_t)(uint16_t)(int16_t)qy << 16);
}

// Tangent (t) and bitangent (b) of the unit normal decoded from a packed
// normal; basis of Duff et al. (JCGT 2017), t x b = n.
__device__ void tangent_frame(uint32_t nrm, double t[3], double b[3])
{
    double px = (double)(int16_t)(nrm & 0xFFFFu) / 32767.0;
    double py = (double)(int16_t)(nrm >> 16) / 32767.0;
    double pz = 1.0 - fabs(px) - fabs(py);
    if (pz < 0.0) {
        const double tx = (1.0 - fabs(py)) * (px >= 0.0 ? 1.0 : -1.0);
        const double ty = (1.0 - fabs(px)) * (py >= 0.0 ? 1.0 : -1.0);
        px = tx;
        py = ty;
    }
    const double len = sqrt(px * px + py * py + pz * pz);
    const double nx = px / len, ny = py / len, nz = pz / len;
    const double s = copysign(1.0, nz);
    const double a = -1.0 / (s + nz);
    const double c = nx * ny * a;
    t[0] = 1.0 + s * nx * nx * a;
    t[1] = s * c;
    t[2] = -s * nx;
    b[0] = c;
    b[1] = s + ny * ny * a;
    b[2] = -ny;
}

// Sample index range covered by [lo, hi] in 16.8 units: samples sit at
// 256 i + 128, so the first is ceil((lo - 128) / 256), the last
// floor((hi - 128) / 256) (arithmetic shifts round towards -inf).
__device__ __forceinline__ void sample_range(int64_t lo, int64_t hi, int32_t* i0, int32_t* i1)
{
    *i0 = (int32_t)((lo - 128 + 255) >> 8);
    *i1 = (int32_t)((hi - 128) >> 8);
}

// Setup record `tr` of n_rec: triangle tr / copies. POFL projection: the
// tangent frame (FHV_PROJ_NORMAL), or an axis plane: `axis` (2: x-y, 0: y-z,
// 1: z-x), or with three copies per triangle the copy's own (tr mod 3).
__global__ void __launch_bounds__(kBlock)
k_setup(const float* __restrict__ pos, const uint32_t* __restrict__ rgba,
        const uint32_t* __restrict__ tri, const uint8_t* __restrict__ obj, uint32_t n_rec,
        uint32_t mode, uint32_t width, uint32_t height, uint32_t levels, uint32_t tile_shift,
        uint32_t proj, uint32_t axis, uint32_t copies,
        const uint32_t* __restrict__ scene_tri, uint32_t n_scenes,
        TriRec* __restrict__ recs, uint64_t* __restrict__ tiles)
{
    const uint32_t tr = blockIdx.x * kBlock + threadIdx.x;
    if (tr >= n_rec) return;
    const uint32_t t = tr / copies;
    if (copies == 3) axis = tr % 3;
    // scene of a batch: the last s in [0, n_scenes) with scene_tri[s] <= t
    // (only scene_tri[1 .. n_scenes-1] is read, so the result stays in range)
    uint32_t scene = 0;
    if (scene_tri) {
        uint32_t lo = 0, hi = n_scenes - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (scene_tri[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        scene = lo;
    }
    TriRec r;
    int64_t X[3], Y[3];
    int32_t a[3][3];
    uint32_t col[3];
    bool skip = false;
    uint32_t nrm;
    for (int k = 0; k < 3; ++k) col[k] = rgba[tri[3 * (uint64_t)t + k]];
    if (mode == FHV_PPFL) {
        int64_t q[3][3];
        for (int k = 0; k < 3; ++k) {
            const float* p = pos + 3 * (uint64_t)tri[3 * (uint64_t)t + k];
            const double x = p[0], y = p[1], z = p[2];
            if (!(fabs(x) <= 64.0 && fabs(y) <= 64.0 && fabs(z) <= 64.0)) {
                skip = true;
                break;
            }
            X[k] = (int64_t)rint((x + 1.0) * ((double)width * 128.0));
            Y[k] = (int64_t)rint((y + 1.0) * ((double)height * 128.0));
            double zd = rint((z + 1.0) * 0.5 * 16777215.0);
            zd = zd < 0.0 ? 0.0 : (zd > 16777215.0 ? 16777215.0 : zd);
            a[k][0] = (int32_t)zd;
            a[k][1] = a[k][2] = 0;
            q[k][0] = (int64_t)rint(x * 1048576.0);
            q[k][1] = (int64_t)rint(y * 1048576.0);
            q[k][2] = (int64_t)rint(z * 1048576.0);
        }
        if (!skip) {
            const int64_t ux = q[1][0] - q[0][0], uy = q[1][1] - q[0][1], uz = q[1][2] - q[0][2];
            const int64_t vx = q[2][0] - q[0][0], vy = q[2][1] - q[0][1], vz = q[2][2] - q[0][2];
            nrm = oct_pack(uy * vz - uz * vy, uz * vx - ux * vz, ux * vy - uy * vx);
        }
    } else {
        const double G = (double)(1ll << (levels + 8));
        for (int k = 0; k < 3 && !skip; ++k) {
            const float* p = pos + 3 * (uint64_t)tri[3 * (uint64_t)t + k];
            for (int c = 0; c < 3; ++c) {
                const float f = p[c];
                if (!isfinite(f)) {
                    skip = true;
                    break;
                }
                double g = floor((double)f * G);
                g = g < 0.0 ? 0.0 : (g > G - 1.0 ? G - 1.0 : g);
                a[k][c] = (int32_t)g;
            }
        }
        if (!skip) {
            const int64_t ux = a[1][0] - a[0][0], uy = a[1][1] - a[0][1], uz = a[1][2] - a[0][2];
            const int64_t vx = a[2][0] - a[0][0], vy = a[2][1] - a[0][1], vz = a[2][2] - a[0][2];
            const int64_t nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
            if (nx == 0 && ny == 0 && nz == 0) {
                skip = true;
            } else {
                nrm = oct_pack(nx, ny, nz);
                if (proj == FHV_PROJ_NORMAL) {
                    double tt[3], bb[3];
                    tangent_frame(nrm, tt, bb);
                    for (int k = 0; k < 3; ++k) {
                        const double px = (double)a[k][0], py = (double)a[k][1], pz = (double)a[k][2];
                        const double u = px * tt[0] + py * tt[1] + pz * tt[2];
                        const double v = px * bb[0] + py * bb[1] + pz * bb[2];
                        X[k] = (int64_t)rint(2.0 * u);
                        Y[k] = (int64_t)rint(2.0 * v);
                    }
                } else {
                    // axis plane: (u, v) = two grid coordinates in cyclic
                    // order after the axis, exact integers
                    const int cu = (int)((axis + 1) % 3), cv = (int)((axis + 2) % 3);
                    for (int k = 0; k < 3; ++k) {
                        X[k] = 2 * (int64_t)a[k][cu];
                        Y[k] = 2 * (int64_t)a[k][cv];
                    }
                }
            }
        }
    }
    uint64_t n_tiles = 0;
    if (!skip) {
        int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]);
        if (A != 0) {
            int o[3] = {0, 1, 2};
            if (A < 0) {
                o[1] = 2;
                o[2] = 1;
                A = -A;
            }
            int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
            for (int k = 1; k < 3; ++k) {
                xmin = X[k] < xmin ? X[k] : xmin;
                xmax = X[k] > xmax ? X[k] : xmax;
                ymin = Y[k] < ymin ? Y[k] : ymin;
                ymax = Y[k] > ymax ? Y[k] : ymax;
            }
            int32_t i0, i1, j0, j1;
            sample_range(xmin, xmax, &i0, &i1);
            sample_range(ymin, ymax, &j0, &j1);
            if (mode == FHV_PPFL) {
                i0 = i0 < 0 ? 0 : i0;
                j0 = j0 < 0 ? 0 : j0;
                i1 = i1 > (int32_t)width - 1 ? (int32_t)width - 1 : i1;
                j1 = j1 > (int32_t)height - 1 ? (int32_t)height - 1 : j1;
            }
            for (int k = 0; k < 3; ++k) {
                r.x[k] = (int32_t)X[o[k]];
                r.y[k] = (int32_t)Y[o[k]];
                r.rgba[k] = col[o[k]];
                for (int c = 0; c < 3; ++c) r.a[k][c] = a[o[k]][c];
            }
            r.lo_i = i0;
            r.lo_j = j0;
            r.hi_i = i1;
            r.hi_j = j1;
            r.nrm = nrm;
            r.aux = obj ? (uint32_t)obj[t] : 0u;
            r.A = A;
            r.rA = 1.0 / (double)A;
            r.scene = scene;
            r.pad1 = 0;
            r.pad2 = 0;
            if (i1 >= i0 && j1 >= j0) {
                // tiles of (1 << tile_shift) x (64 >> tile_shift) samples
                const uint32_t tx = ((uint32_t)(i1 - i0) >> tile_shift) + 1;
                const uint32_t ty = ((uint32_t)(j1 - j0) >> (6 - tile_shift)) + 1;
                r.tiles_x = tx;
                n_tiles = (uint64_t)tx * ty;
            } else {
                r.tiles_x = 0;
            }
            recs[tr] = r;
        }
    }
    tiles[tr] = n_tiles;
}

// floor((w0 a0 + w1 a1 + w2 a2 + floor(A/2)) / A) for non-negative weights
// and attributes: an fp64 estimate (within 1 of the quotient) corrected by
// the exact remainder, which is small and therefore exact in wrapped
// 64-bit arithmetic even when the numerator itself exceeds 64 bits.
__device__ __forceinline__ uint32_t interp(int64_t w0, int64_t w1, int64_t w2, int32_t a0,
                                           int32_t a1, int32_t a2, int64_t A, double rA)
{
    const int64_t half = A >> 1;
    const double est = ((double)w0 * (double)a0 + (double)w1 * (double)a1 + (double)w2 * (double)a2 +
                        (double)half) * rA;
    int64_t q = (int64_t)floor(est);
    const uint64_t num = (uint64_t)w0 * (uint64_t)(uint32_t)a0 + (uint64_t)w1 * (uint64_t)(uint32_t)a1 +
                         (uint64_t)w2 * (uint64_t)(uint32_t)a2 + (uint64_t)half;
    const int64_t rem = (int64_t)(num - (uint64_t)q * (uint64_t)A);
    if (rem < 0)
        q -= 1;
    else if (rem >= A)
        q += 1;
    return (uint32_t)q;
}

__device__ __forceinline__ uint32_t interp_rgba(int64_t w0, int64_t w1, int64_t w2,
                                                const uint32_t c[3], int64_t A, double rA)
{
    uint32_t out = 0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        const int32_t c0 = (c[0] >> (8 * ch)) & 0xFF, c1 = (c[1] >> (8 * ch)) & 0xFF,
                      c2 = (c[2] >> (8 * ch)) & 0xFF;
        out |= interp(w0, w1, w2, c0, c1, c2, A, rA) << (8 * ch);
    }
    return out;
}

// Edge functions and coverage of one lane's sample in tile `tile` of r.
struct Sample {
    bool cov;
    int32_t i, j;
    int64_t e01, e12, e20;
};

__device__ __forceinline__ Sample sample_of(const TriRec& r, uint32_t tile, int lane, uint32_t ts)
{
    Sample s;
    const uint32_t tx = tile % r.tiles_x, ty = tile / r.tiles_x;
    s.i = r.lo_i + (int32_t)(tx << ts) + (lane & ((1 << ts) - 1));
    s.j = r.lo_j + (int32_t)(ty << (6 - ts)) + (lane >> ts);
    s.cov = s.i <= r.hi_i && s.j <= r.hi_j;
    s.e01 = s.e12 = s.e20 = 0;
    if (s.cov) {
        const int64_t px = 256 * (int64_t)s.i + 128, py = 256 * (int64_t)s.j + 128;
        const int64_t x0 = r.x[0], x1 = r.x[1], x2 = r.x[2];
        const int64_t y0 = r.y[0], y1 = r.y[1], y2 = r.y[2];
        s.e01 = (x1 - x0) * (py - y0) - (y1 - y0) * (px - x0);
        s.e12 = (x2 - x1) * (py - y1) - (y2 - y1) * (px - x1);
        s.e20 = (x0 - x2) * (py - y2) - (y0 - y2) * (px - x2);
        // top-left rule (CCW, y up): an edge owns its samples when it runs
        // downwards, or horizontally towards -x
        const bool o01 = (y1 < y0) || (y1 == y0 && x1 < x0);
        const bool o12 = (y2 < y1) || (y2 == y1 && x2 < x1);
        const bool o20 = (y0 < y2) || (y0 == y2 && x0 < x2);
        s.cov = (s.e01 > 0 || (s.e01 == 0 && o01)) && (s.e12 > 0 || (s.e12 == 0 && o12)) &&
                (s.e20 > 0 || (s.e20 == 0 && o20));
    }
    return s;
}

// Walks work items [w0, w1) (wave-uniform), keeping the owning triangle t
// with its first item `first` and one-past-last item `end`.
struct ItemWalk {
    const uint64_t* incl;
    uint32_t t;
    uint64_t first, end;
    __device__ void start(uint32_t n_tri, uint64_t w0)
    {
        uint32_t lo = 0, hi = n_tri - 1;   // first t with incl[t] > w0
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (incl[mid] > w0)
                hi = mid;
            else
                lo = mid + 1;
        }
        t = uniform32(lo);
        first = t ? incl[t - 1] : 0;
        end = incl[t];
    }
    __device__ void advance(uint64_t w)
    {
        while (w >= end) {
            ++t;
            first = end;
            end = incl[t];
        }
    }
};

// Each wave owns a contiguous range of work items. It first counts the
// covered samples of the whole range, reserves that many pool slots with a
// single atomic add on the counter, and then walks the range again to emit
// the fragments into consecutive slots.
//
// kAct (two-pass capture into arrays, lists and pool unused): kActCount
// adds every fragment to its brick's histogram, kActInsert stores it in its
// brick's staging range with the key's low bits in w3.
template <int kMode, class KeyT, int kAct = kActList>
__global__ void __launch_bounds__(kBlock)
k_raster(const TriRec* __restrict__ recs, const uint64_t* __restrict__ incl, uint32_t n_tri,
         uint32_t width, uint32_t gmax, uint32_t levels, uint32_t ts, uint32_t* __restrict__ head,
         uint4* __restrict__ pool, KeyT* __restrict__ keys, uint64_t cap,
         unsigned long long* __restrict__ counter, BrickSink bs)
{
    const uint64_t total = incl[n_tri - 1];
    const int lane = __lane_id();
    const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / kWave);
    const uint64_t wid = uniform64((uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);
    const uint64_t per = (total + n_waves - 1) / n_waves;
    const uint64_t w0 = wid * per;
    const uint64_t w1 = w0 + per < total ? w0 + per : total;
    if (w0 >= w1) return;
    if (kAct == kActInsert && *bs.skip) return;

    ItemWalk it{incl, 0, 0, 0};
    constexpr int kBatch = 4;   // tiles per step; their memory operations overlap
    unsigned long long base = 0;
    if (kAct == kActList) {
    it.start(n_tri, w0);
    uint64_t n_cov = 0;
    for (uint64_t w = w0; w < w1; w += kBatch) {
        uint32_t tb[kBatch], tile[kBatch];
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            tb[g] = kNil;
            if (w + g < w1) {
                it.advance(w + g);
                tb[g] = it.t;
                tile[g] = (uint32_t)(w + g - it.first);
            }
        }
#pragma unroll
        for (int g = 0; g < kBatch; ++g)
            if (tb[g] != kNil) n_cov += (uint64_t)__popcll(__ballot(sample_of(recs[tb[g]], tile[g], lane, ts).cov));
    }
    if (n_cov == 0) return;
    if (lane == 0) base = atomicAdd(counter, (unsigned long long)n_cov);
    base = __shfl(base, 0, kWave);
    }

    it.start(n_tri, w0);
    for (uint64_t w = w0; w < w1; w += kBatch) {
        bool has[kBatch];
        uint64_t key[kBatch];
        uint32_t w0r[kBatch], w1r[kBatch], nrm[kBatch];
        uint64_t idx[kBatch];
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            has[g] = false;
            key[g] = 0;
            idx[g] = 0;
            if (w + g >= w1) continue;   // wave-uniform
            it.advance(w + g);
            const TriRec& r = recs[it.t];
            const Sample sm = sample_of(r, (uint32_t)(w + g - it.first), lane, ts);
            if (kAct == kActList) {
                const uint64_t mask = __ballot(sm.cov);
                idx[g] = base + (uint64_t)__popcll(mask & lanemask_lt());
                base += (uint64_t)__popcll(mask);
                has[g] = sm.cov && idx[g] < cap;
            } else {
                has[g] = sm.cov;
            }
            if (!has[g]) continue;
            nrm[g] = r.nrm;
            w1r[g] = interp_rgba(sm.e12, sm.e20, sm.e01, r.rgba, r.A, r.rA);
            if (kMode == FHV_PPFL) {
                key[g] = (uint64_t)sm.j * width + (uint32_t)sm.i;
                const uint32_t dz = interp(sm.e12, sm.e20, sm.e01, r.a[0][0], r.a[1][0], r.a[2][0], r.A, r.rA);
                w0r[g] = dz | (r.aux << 24);
            } else {
                // interpolation stays within the vertices' range; the clamp
                // only keeps the key inside the head array
                uint32_t gx = interp(sm.e12, sm.e20, sm.e01, r.a[0][0], r.a[1][0], r.a[2][0], r.A, r.rA);
                uint32_t gy = interp(sm.e12, sm.e20, sm.e01, r.a[0][1], r.a[1][1], r.a[2][1], r.A, r.rA);
                uint32_t gz = interp(sm.e12, sm.e20, sm.e01, r.a[0][2], r.a[1][2], r.a[2][2], r.A, r.rA);
                gx = gx > gmax ? gmax : gx;
                gy = gy > gmax ? gmax : gy;
                gz = gz > gmax ? gmax : gz;
                key[g] = ((uint64_t)r.scene << (3 * levels)) |
                         (spread3(gx >> 8) << 2) | (spread3(gy >> 8) << 1) | spread3(gz >> 8);
                w0r[g] = (gx & 0xFFu) | ((gy & 0xFFu) << 8) | ((gz & 0xFFu) << 16) | (r.aux << 24);
            }
        }
        if (kAct == kActCount) {
#pragma unroll
            for (int g = 0; g < kBatch; ++g)
                if (w + g < w1) wave_hist(key[g], has[g], bs.cnt, bs.bitmap);   // wave-uniform
            continue;
        }
        if (kAct == kActInsert) {
#pragma unroll
            for (int g = 0; g < kBatch; ++g) {
                if (w + g >= w1) continue;   // wave-uniform
                const uint32_t b = (uint32_t)(key[g] >> kBrickShift);
                const uint32_t slot = wave_count_add<true>(bs.cur, b, has[g]);
                if (has[g])
                    bs.stage[bs.off[b] + slot] =
                        make_uint4(w0r[g], w1r[g], nrm[g], (uint32_t)key[g] & (kBrickKeys - 1));
            }
            continue;
        }
        uint32_t prev[kBatch];
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            prev[g] = kNil;
            if (head && has[g]) prev[g] = atomicExch(head + key[g], (uint32_t)idx[g]);
        }
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            if (!has[g]) continue;
            pool[idx[g]] = make_uint4(w0r[g], w1r[g], nrm[g], prev[g]);
            keys[idx[g]] = (KeyT)key[g];
        }
    }
}

}  // namespace

// Setup records per pass: three projected copies of every triangle for
// FHV_PROJ_AXES_1PASS, one otherwise.
static uint64_t records_of(const fhv_capture_desc* d, uint32_t n_tri)
{
    return d->mode == FHV_POFL && d->projection == FHV_PROJ_AXES_1PASS ? 3ull * n_tri : (uint64_t)n_tri;
}

size_t capture_ws_bytes(const fhv_capture_desc* d, uint32_t n_tri)
{
    const uint64_t n = records_of(d, n_tri);
    Carver c{nullptr, 0};
    c.take<TriRec>(n);
    c.take<uint64_t>(n);
    c.take<uint64_t>(n);
    c.take<uint64_t>(scan_partials(n));
    return c.off + 256;
}

// Setup of pass `pass` (of one, or three for 3-Pass/1-Way) and the
// inclusive scan of its tiles per record.
static hipError_t setup_pass(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d, uint32_t pass,
                             const Scenes* sc, TriRec* recs, uint64_t* tiles, uint64_t* incl, uint64_t* part,
                             const char* setup_name, const char* scan_name, hipStream_t s)
{
    const uint64_t n_rec = records_of(d, m->n_tri);
    const uint32_t ts = dev.tune.tile_w == 32 ? 5u : (dev.tune.tile_w == 16 ? 4u : 3u);
    const uint32_t proj = d->mode == FHV_POFL ? d->projection : FHV_PROJ_NORMAL;
    const uint32_t copies = proj == FHV_PROJ_AXES_1PASS ? 3u : 1u;
    // the axis plane of the pass: y-z, z-x, x-y for 3-Pass/1-Way, x-y for
    // 1-Pass/View
    const uint32_t axis = proj == FHV_PROJ_AXES_3PASS ? pass : 2u;
    hipError_t e;
    {
        ProfScope ps(dev, setup_name, s);
        k_setup<<<dim3((unsigned)((n_rec + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(
            m->pos, m->rgba, m->tri, m->obj, (uint32_t)n_rec, d->mode, d->width, d->height, d->levels, ts, proj,
            axis, copies, sc ? sc->scene_tri : nullptr, sc ? sc->n_scenes : 1u, recs, tiles);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    ProfScope ps(dev, scan_name, s);
    return scan_u64(tiles, incl, n_rec, true, part, nullptr, s);
}

hipError_t capture_bricks_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d, void* ws,
                                 int act, const BrickSink& bs, hipStream_t s)
{
    const uint64_t n_rec = records_of(d, m->n_tri);
    Carver c{(char*)ws, 0};
    TriRec* recs = c.take<TriRec>(n_rec);
    uint64_t* tiles = c.take<uint64_t>(n_rec);
    uint64_t* incl = c.take<uint64_t>(n_rec);
    uint64_t* part = c.take<uint64_t>(scan_partials(n_rec));
    if (m->n_tri == 0) return hipSuccess;
    const uint32_t ts = dev.tune.tile_w == 32 ? 5u : (dev.tune.tile_w == 16 ? 4u : 3u);
    const uint32_t passes = d->projection == FHV_PROJ_AXES_3PASS ? 3u : 1u;
    const unsigned grid = (unsigned)(dev.cus * dev.tune.raster_wg);
    const uint32_t gmax = (1u << (d->levels + 8)) - 1u;
    const char* name = act == kActCount ? "arrays.count" : "arrays.insert";
    for (uint32_t pass = 0; pass < passes; ++pass) {
        hipError_t e = setup_pass(dev, m, d, pass, nullptr, recs, tiles, incl, part, "arrays.setup", "arrays.scan", s);
        if (e != hipSuccess) return e;
        ProfScope ps(dev, name, s);
        if (act == kActCount)
            k_raster<FHV_POFL, uint32_t, kActCount><<<dim3(grid), dim3(kBlock), 0, s>>>(
                recs, incl, (uint32_t)n_rec, 0u, gmax, d->levels, ts, nullptr, nullptr, nullptr, 0, nullptr, bs);
        else
            k_raster<FHV_POFL, uint32_t, kActInsert><<<dim3(grid), dim3(kBlock), 0, s>>>(
                recs, incl, (uint32_t)n_rec, 0u, gmax, d->levels, ts, nullptr, nullptr, nullptr, 0, nullptr, bs);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t capture_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d,
                          const fhv_lists* L, void* ws, hipStream_t s, const Scenes* sc)
{
    const uint64_t n_rec = records_of(d, m->n_tri);
    Carver c{(char*)ws, 0};
    TriRec* recs = c.take<TriRec>(n_rec);
    uint64_t* tiles = c.take<uint64_t>(n_rec);
    uint64_t* incl = c.take<uint64_t>(n_rec);
    uint64_t* part = c.take<uint64_t>(scan_partials(n_rec));
    const uint32_t ts = dev.tune.tile_w == 32 ? 5u : (dev.tune.tile_w == 16 ? 4u : 3u);
    hipError_t e;
    {
        ProfScope ps(dev, "capture.reset", s);
        e = L->head ? fill_u32(L->head, L->n_head, kNil, s) : hipSuccess;
        if (e == hipSuccess) e = fill_u64(L->counter, 1, 0, s);
    }
    if (e != hipSuccess || m->n_tri == 0) return e;
    // three passes for 3-Pass/1-Way, one otherwise
    const uint32_t passes = d->mode == FHV_POFL && d->projection == FHV_PROJ_AXES_3PASS ? 3u : 1u;
    const unsigned grid = (unsigned)(dev.cus * dev.tune.raster_wg);
    const uint32_t gmax = d->mode == FHV_POFL ? (1u << (d->levels + 8)) - 1u : 0u;
    const bool wide = L->n_head > (1ull << 32);
    for (uint32_t pass = 0; pass < passes; ++pass) {
        e = setup_pass(dev, m, d, pass, sc, recs, tiles, incl, part, "capture.setup", "capture.scan", s);
        if (e != hipSuccess) return e;
        ProfScope ps(dev, "capture.raster", s);
        if (d->mode == FHV_PPFL)
            k_raster<FHV_PPFL, uint32_t><<<dim3(grid), dim3(kBlock), 0, s>>>(
                recs, incl, (uint32_t)n_rec, d->width, gmax, d->levels, ts, L->head, (uint4*)L->pool,
                (uint32_t*)L->keys, L->capacity, (unsigned long long*)L->counter, BrickSink{});
        else if (!wide)
            k_raster<FHV_POFL, uint32_t><<<dim3(grid), dim3(kBlock), 0, s>>>(
                recs, incl, (uint32_t)n_rec, d->width, gmax, d->levels, ts, L->head, (uint4*)L->pool,
                (uint32_t*)L->keys, L->capacity, (unsigned long long*)L->counter, BrickSink{});
        else
            k_raster<FHV_POFL, uint64_t><<<dim3(grid), dim3(kBlock), 0, s>>>(
                recs, incl, (uint32_t)n_rec, d->width, gmax, d->levels, ts, L->head, (uint4*)L->pool,
                (uint64_t*)L->keys, L->capacity, (unsigned long long*)L->counter, BrickSink{});
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fhv
