// Compaction of fragment lists into per-octant arrays (FHV_POFA, Sec. 3.1
// Fig. 6 and Sec. 3.2): per occupied key a count and an offset, the offsets
// being sums of counts in ascending key (Morton) order, every key's records
// contiguous, ascending by (w0, w1, w2), w3 = the key's table rank.
//
// The paper counts per octant, scans, resets the counters and rasterizes a
// second time. Here the pool is read linearly instead, through the key
// sidecar the capture wrote, and keys are grouped in buckets ("bricks") of
// 512 consecutive keys so that every bucket fits a workgroup's LDS:
//   k_hist     per brick: fragment count (atomic add) and the key's bit
//              in a key bitmap (atomic or); lanes of a wave that hit the
//              same brick or bitmap word combine into one atomic, and no
//              atomic's result is waited for
//   scan       exclusive sums of the brick counts: brick fragment offsets
//              and the list of occupied bricks; total = n_frag
//   k_brick_occ  per occupied brick: distinct keys = popcount of its 16
//              bitmap words
//   scan       exclusive sums of the distinct-key counts: brick rank bases;
//              total = n_occ
//   k_scatter  every pool record to its brick's range of a staging array
//              (slot within the brick from an atomic cursor), its key's low
//              9 bits (the key inside the brick) in w3
//   k_brick_wave / k_brick
//              per brick: counting sort of its records by key inside LDS,
//              a per-key insertion sort into canonical order, then the
//              output records with w3 = rank and the brick's table rows.
//              Bricks of up to 1024 records take one wave each with no
//              workgroup barriers; larger ones a whole workgroup (in place
//              in the output when they exceed LDS)
#include "scan.h"

namespace fhv {

namespace {

constexpr int kLdsRecs = 2048;   // records staged in LDS per brick (32 KiB)

__device__ __forceinline__ uint64_t frag_count(const uint64_t* counter, uint64_t cap)
{
    const uint64_t c = *counter;
    return c < cap ? c : cap;
}

template <class KeyT>
__global__ void __launch_bounds__(kBlock)
k_hist(const KeyT* __restrict__ keys, const uint64_t* __restrict__ counter, uint64_t cap,
       uint32_t* __restrict__ brick_cnt, uint32_t* __restrict__ bitmap)
{
    const uint64_t F = frag_count(counter, cap);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    // the loop bound is rounded up to whole waves so that every lane of a
    // wave takes part in the wave-wide aggregation
    const uint64_t Fw = (F + kWave - 1) & ~(uint64_t)(kWave - 1);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < Fw; i += stride) {
        const bool act = i < F;
        const uint64_t key = act ? (uint64_t)keys[i] : 0u;
        wave_hist(key, act, brick_cnt, bitmap);
    }
}

// Distinct keys of every occupied brick (the list from the count scan):
// the popcount of its kBrickKeys / 32 bitmap words, one lane per word.
__global__ void __launch_bounds__(kBlock)
k_brick_occ(const uint32_t* __restrict__ list, const uint64_t* __restrict__ list_total,
            const uint32_t* __restrict__ bitmap, uint32_t* __restrict__ brick_occ)
{
    constexpr uint32_t kWords = kBrickKeys / 32;   // 16: four bricks per wave
    const uint32_t nl = (uint32_t)(*list_total >> 32);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t nw = (uint64_t)nl * kWords;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < (nw + kWave - 1) / kWave * kWave;
         i += stride) {
        const bool act = i < nw;
        const uint32_t b = act ? list[i / kWords] : 0u;
        uint32_t c = act ? (uint32_t)__popc(bitmap[(uint64_t)b * kWords + i % kWords]) : 0u;
        // sum over the 16 lanes of the brick (aligned groups of 16 lanes)
#pragma unroll
        for (int d = 1; d < (int)kWords; d <<= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
        if (act && i % kWords == 0) brick_occ[b] = c;
    }
}

template <class KeyT>
__global__ void __launch_bounds__(kBlock)
k_scatter(const uint4* __restrict__ pool, const KeyT* __restrict__ keys,
          const uint64_t* __restrict__ counter, uint64_t cap, const uint32_t* __restrict__ brick_off,
          uint32_t* __restrict__ brick_cur, uint4* __restrict__ stage)
{
    const uint64_t F = frag_count(counter, cap);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t Fw = (F + kWave - 1) & ~(uint64_t)(kWave - 1);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < Fw; i += stride) {
        const bool act = i < F;
        const uint64_t key = act ? (uint64_t)keys[i] : 0u;
        const uint32_t b = (uint32_t)(key >> kBrickShift);
        const uint32_t slot = wave_count_add<true>(brick_cur, b, act);
        if (!act) continue;
        uint4 r = pool[i];
        r.w = (uint32_t)key & (kBrickKeys - 1);   // key inside the brick
        stage[brick_off[b] + slot] = r;
    }
}

__device__ __forceinline__ bool rec_less(const uint4& a, const uint4& b)
{
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
}

// 512-entry exclusive scan in LDS by one 256-thread workgroup (2 per thread).
__device__ void scan512(uint32_t* v, uint32_t* tmp)
{
    const int t = threadIdx.x;
    // inclusive Hillis-Steele over 512 values in place
    for (int d = 1; d < 512; d <<= 1) {
        const uint32_t a0 = (2 * t >= d) ? v[2 * t - d] : 0u;
        const uint32_t a1 = (2 * t + 1 >= d) ? v[2 * t + 1 - d] : 0u;
        __syncthreads();
        v[2 * t] += a0;
        v[2 * t + 1] += a1;
        __syncthreads();
    }
    // to exclusive
    tmp[2 * t] = 2 * t ? v[2 * t - 1] : 0u;
    tmp[2 * t + 1] = v[2 * t];
    __syncthreads();
    v[2 * t] = tmp[2 * t];
    v[2 * t + 1] = tmp[2 * t + 1];
    __syncthreads();
}

// Workgroup path for one brick of n records (n above the wave kernel's
// size). Counting sort by key from src into buf (LDS when it fits, else the
// brick's output range), then every record goes to its key's offset plus its
// rank inside the key's run in (w0, w1, w2) order (equal records ordered by
// position), with w3 = the key's table rank. In LDS the placement writes the
// output directly; otherwise it writes the brick's staging range (src, no
// longer needed) and the result is copied to the output.
template <bool kInLds>
__device__ void brick_sort(uint4* __restrict__ buf, uint4* __restrict__ src, uint32_t n,
                           uint32_t* cnt, uint32_t* off, uint32_t* cur, uint32_t* rank,
                           uint32_t* tmp, uint32_t brick, uint32_t base_off, uint32_t base_rank,
                           uint4* __restrict__ out, uint64_t* __restrict__ oct_key,
                           uint32_t* __restrict__ oct_off, uint32_t* __restrict__ oct_cnt,
                           uint64_t cap_occ)
{
    const int t = threadIdx.x;
    cnt[2 * t] = cnt[2 * t + 1] = 0;
    __syncthreads();
    for (uint32_t i = t; i < n; i += kBlock) atomicAdd(cnt + (src[i].w & (kBrickKeys - 1)), 1u);
    __syncthreads();
    for (int k = 0; k < 2; ++k) {
        const uint32_t c = cnt[2 * t + k];
        off[2 * t + k] = c;
        rank[2 * t + k] = c ? 1u : 0u;
    }
    __syncthreads();
    scan512(off, tmp);
    scan512(rank, tmp);
    for (int k = 0; k < 2; ++k) cur[2 * t + k] = off[2 * t + k];
    __syncthreads();
    for (uint32_t i = t; i < n; i += kBlock) {
        const uint4 r = src[i];
        const uint32_t p = atomicAdd(cur + (r.w & (kBrickKeys - 1)), 1u);
        buf[p] = r;
    }
    for (int k = 0; k < 2; ++k) {
        const uint32_t leaf = 2 * t + k, c = cnt[leaf];
        if (c) {
            const uint64_t rk = (uint64_t)base_rank + rank[leaf];
            if (rk < cap_occ) {
                oct_key[rk] = ((uint64_t)brick << kBrickShift) | leaf;
                oct_off[rk] = base_off + off[leaf];
                oct_cnt[rk] = c;
            }
        }
    }
    if (!kInLds) __threadfence();
    __syncthreads();
    uint4* dst = kInLds ? out : src;
    for (uint32_t i = t; i < n; i += kBlock) {
        const uint4 x = buf[i];
        const uint32_t leaf = x.w & (kBrickKeys - 1), lo = off[leaf], c = cnt[leaf];
        uint32_t before = 0;
        for (uint32_t q = lo; q < lo + c; ++q) {
            const uint4 y = buf[q];
            before += (rec_less(y, x) || (q < i && y.x == x.x && y.y == x.y && y.z == x.z)) ? 1u : 0u;
        }
        dst[lo + before] = make_uint4(x.x, x.y, x.z, base_rank + rank[leaf]);
    }
    if (!kInLds) {
        __threadfence();
        __syncthreads();
        for (uint32_t i = t; i < n; i += kBlock) out[i] = src[i];
    }
}

// Orders LDS traffic of one wave: its earlier LDS writes are complete and
// visible to all its lanes before later LDS reads.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

constexpr int kWaveRecs = 1024;            // records per wave-sized brick
constexpr int kSmallRecs = 256;            // bricks up to this size take the smaller variant
constexpr int kKeysPerLane = kBrickKeys / kWave;  // 8

// One wave per brick of kLo < n <= kRecs records, with no workgroup
// barriers (one-wave workgroups; the variant for small bricks needs less
// LDS and fewer registers, so more of them share a compute unit): records
// loaded into registers (kRecs / 64 per lane) are counted per key in LDS,
// the 512 counts scanned across the wave (8 consecutive keys per lane), the
// records grouped by key in LDS through cursors, and every record written
// straight to its final slot: its key's offset plus its rank inside the
// key's run in canonical order, with w3 = the key's table rank.
template <int kRecs, int kLo>
__global__ void __launch_bounds__(kWave)
k_brick_wave(const uint4* __restrict__ stage, const uint32_t* __restrict__ brick_cnt,
             const uint32_t* __restrict__ brick_off, const uint32_t* __restrict__ brick_rank,
             const uint32_t* __restrict__ list, const uint64_t* __restrict__ list_total,
             uint4* __restrict__ frag, uint64_t* __restrict__ oct_key,
             uint32_t* __restrict__ oct_off, uint32_t* __restrict__ oct_cnt, uint64_t cap_occ)
{
    constexpr int kPerLane = kRecs / kWave;
    __shared__ uint4 buf[kRecs];
    __shared__ uint32_t off[kBrickKeys], rank[kBrickKeys], cur[kBrickKeys];
    const int lane = __lane_id();
    const uint32_t nl = (uint32_t)(*list_total >> 32);
    for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
        const uint32_t b = list[li];
        const uint32_t n = brick_cnt[b];
        if (n <= (uint32_t)kLo || n > (uint32_t)kRecs) continue;
        const uint32_t o = brick_off[b], base_rank = brick_rank[b];
        uint4 r[kPerLane];
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const uint32_t i = (uint32_t)(k * kWave + lane);
            r[k] = i < n ? stage[o + i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < kKeysPerLane; ++k) cur[lane * kKeysPerLane + k] = 0;
        wave_lds_sync();
#pragma unroll
        for (int k = 0; k < kPerLane; ++k)
            if ((uint32_t)(k * kWave + lane) < n) atomicAdd(cur + (r[k].w & (kBrickKeys - 1)), 1u);
        wave_lds_sync();
        uint32_t c[kKeysPerLane], s = 0, z = 0;
#pragma unroll
        for (int k = 0; k < kKeysPerLane; ++k) {
            c[k] = cur[lane * kKeysPerLane + k];
            s += c[k];
            z += c[k] ? 1u : 0u;
        }
        uint32_t si = s, zi = z;   // inclusive wave scans
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t a = (uint32_t)__shfl_up((int)si, d, kWave);
            const uint32_t q = (uint32_t)__shfl_up((int)zi, d, kWave);
            if (lane >= d) {
                si += a;
                zi += q;
            }
        }
        uint32_t ps = si - s, pz = zi - z;
#pragma unroll
        for (int k = 0; k < kKeysPerLane; ++k) {
            off[lane * kKeysPerLane + k] = ps;
            cur[lane * kKeysPerLane + k] = ps;
            rank[lane * kKeysPerLane + k] = pz;
            ps += c[k];
            pz += c[k] ? 1u : 0u;
        }
        wave_lds_sync();
#pragma unroll
        for (int k = 0; k < kPerLane; ++k)
            if ((uint32_t)(k * kWave + lane) < n) buf[atomicAdd(cur + (r[k].w & (kBrickKeys - 1)), 1u)] = r[k];
        wave_lds_sync();
        // table rows, 8 consecutive keys per lane
#pragma unroll
        for (int k = 0; k < kKeysPerLane; ++k) {
            const uint32_t leaf = lane * kKeysPerLane + k;
            if (c[k]) {
                const uint64_t rk = (uint64_t)base_rank + rank[leaf];
                if (rk < cap_occ) {
                    oct_key[rk] = ((uint64_t)b << kBrickShift) | leaf;
                    oct_off[rk] = o + off[leaf];
                    oct_cnt[rk] = c[k];
                }
            }
        }
        // every record's place inside its key's run: the number of records
        // of the run that precede it in (w0, w1, w2) order (bitwise equal
        // records are interchangeable; they are ordered by LDS position).
        // Records are taken in their key-grouped LDS order, 64 positions at
        // a time, so a window's loop runs to the longest run it meets, with
        // four reads of each lane in flight per step.
        for (uint32_t w0 = 0; w0 < n; w0 += kWave) {
            const uint32_t q = w0 + (uint32_t)lane;
            const bool valid = q < n;
            const uint4 x = buf[valid ? q : 0];
            const uint32_t leaf = x.w & (kBrickKeys - 1);
            const uint32_t lo = valid ? off[leaf] : 0u;
            const uint32_t len = valid ? cur[leaf] - lo : 0u;   // cur = end of run
            uint32_t mrun = len;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o2 = (uint32_t)__shfl_xor((int)mrun, d, kWave);
                mrun = o2 > mrun ? o2 : mrun;
            }
            uint32_t before = 0;
            for (uint32_t dd = 0; dd < mrun; dd += 4) {
                uint4 y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t e = dd + (uint32_t)u;
                    y[u] = buf[lo + (e < len ? e : 0u)];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t e = dd + (uint32_t)u;
                    const bool lt = rec_less(y[u], x) ||
                                    (lo + e < q && y[u].x == x.x && y[u].y == x.y && y[u].z == x.z);
                    before += (e < len && lt) ? 1u : 0u;
                }
            }
            if (valid) frag[o + lo + before] = make_uint4(x.x, x.y, x.z, base_rank + rank[leaf]);
        }
        wave_lds_sync();
    }
}

__global__ void __launch_bounds__(kBlock)
k_brick(uint4* __restrict__ stage, const uint32_t* __restrict__ brick_cnt,
        const uint32_t* __restrict__ brick_off, const uint32_t* __restrict__ brick_rank,
        const uint32_t* __restrict__ list, const uint64_t* __restrict__ list_total,
        uint4* __restrict__ frag, uint64_t* __restrict__ oct_key,
        uint32_t* __restrict__ oct_off, uint32_t* __restrict__ oct_cnt, uint64_t cap_occ)
{
    __shared__ uint4 lbuf[kLdsRecs];
    __shared__ uint32_t cnt[kBrickKeys], off[kBrickKeys], cur[kBrickKeys], rank[kBrickKeys],
        tmp[kBrickKeys];
    // bricks above the wave kernel's size, taken from the occupied-brick list
    const uint32_t nl = (uint32_t)(*list_total >> 32);
    for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
        const uint32_t b = list[li];
        const uint32_t n = brick_cnt[b];
        if (n <= (uint32_t)kWaveRecs) continue;
        const uint32_t o = brick_off[b];
        if (n <= (uint32_t)kLdsRecs)
            brick_sort<true>(lbuf, stage + o, n, cnt, off, cur, rank, tmp, b, o, brick_rank[b],
                             frag + o, oct_key, oct_off, oct_cnt, cap_occ);
        else
            brick_sort<false>(frag + o, stage + o, n, cnt, off, cur, rank, tmp, b, o,
                              brick_rank[b], frag + o, oct_key, oct_off, oct_cnt, cap_occ);
        __syncthreads();
    }
}

// Scan helpers. Bricks are scanned on (count | occupied << 32): the low
// half of the exclusive prefix is the brick's fragment offset, the high half
// its position in the list of occupied bricks.
struct LoadBrick {
    const uint32_t* cnt;
    __device__ uint64_t operator()(uint64_t i) const
    {
        const uint32_t c = cnt[i];
        return (uint64_t)c | ((uint64_t)(c != 0u) << 32);
    }
};

struct StoreBrick {
    uint32_t* off;
    uint32_t* list;
    __device__ void operator()(uint64_t i, uint64_t v, uint64_t ex) const
    {
        off[i] = (uint32_t)ex;
        if ((uint32_t)v) list[ex >> 32] = (uint32_t)i;
    }
};

struct LoadOcc {
    const uint32_t* occ;
    __device__ uint64_t operator()(uint64_t i) const { return occ[i]; }
};

struct StoreRank {
    uint32_t* rank;
    __device__ void operator()(uint64_t i, uint64_t, uint64_t ex) const { rank[i] = (uint32_t)ex; }
};

__global__ void k_totals(const uint64_t* __restrict__ counter, uint64_t cap,
                         uint64_t* __restrict__ n_frag)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_frag = frag_count(counter, cap);
}

}  // namespace

struct CompactWs {
    uint32_t *brick_cnt, *brick_occ, *brick_cur, *brick_off, *brick_rank, *bitmap;
    uint32_t* list;         // occupied bricks, ascending
    uint64_t* part;         // scan scratch
    uint64_t* list_total;   // (fragments | occupied bricks << 32)
    uint4* stage;
};

static CompactWs carve_compact(void* ws, uint64_t n_head, uint64_t capacity, size_t* bytes)
{
    const uint64_t n_brick = (n_head + kBrickKeys - 1) / kBrickKeys;
    Carver c{(char*)ws, 0};
    CompactWs w;
    // the zero-initialised arrays are adjacent so one fill clears them; the
    // bitmap has kBrickKeys / 32 words for every brick, the last one too
    const uint64_t zlen = 3 * n_brick + n_brick * (kBrickKeys / 32);
    uint32_t* z = c.take<uint32_t>(zlen);
    w.brick_cnt = z;
    w.brick_occ = z ? z + n_brick : nullptr;
    w.brick_cur = z ? z + 2 * n_brick : nullptr;
    w.bitmap = z ? z + 3 * n_brick : nullptr;
    w.list = c.take<uint32_t>(n_brick);
    w.brick_off = c.take<uint32_t>(n_brick);
    w.brick_rank = c.take<uint32_t>(n_brick);
    w.part = c.take<uint64_t>(scan_scratch(n_brick));
    w.list_total = c.take<uint64_t>(1);
    w.stage = c.take<uint4>(capacity);
    if (bytes) *bytes = c.off + 256;
    return w;
}

size_t compact_ws_bytes(const fhv_capture_desc* d, uint64_t n_head, uint64_t capacity)
{
    (void)d;
    size_t b = 0;
    carve_compact(nullptr, n_head, capacity, &b);
    return b;
}

static hipError_t brick_sorts(const Device& dev, const CompactWs& w, const fhv_pofa* out, uint64_t n_brick,
                              const char* name, hipStream_t s);

// Distinct keys per occupied brick, from the bitmap (after the count scan
// has listed the occupied bricks).
static hipError_t brick_occ_launch(const Device& dev, const CompactWs& w, uint64_t n_brick, hipStream_t s)
{
    uint64_t g = (n_brick * (kBrickKeys / 32) + kBlock - 1) / kBlock;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    g = g < 1 ? 1 : (g > gmax ? gmax : g);
    k_brick_occ<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(w.list, w.list_total, w.bitmap, w.brick_occ);
    return hipGetLastError();
}

hipError_t compact_launch(const Device& dev, const fhv_lists* L, const fhv_capture_desc* d,
                          const fhv_pofa* out, void* ws, hipStream_t s)
{
    (void)d;
    const uint64_t n_brick = (L->n_head + kBrickKeys - 1) / kBrickKeys;
    CompactWs w = carve_compact(ws, L->n_head, L->capacity, nullptr);
    hipError_t e;
    uint64_t gb = (L->capacity + kBlock - 1) / kBlock;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    const unsigned grid = (unsigned)(gb < 1 ? 1 : (gb > gmax ? gmax : gb));
    {
        ProfScope ps(dev, "compact.hist", s);
        e = fill_u32(w.brick_cnt, 3 * n_brick + n_brick * (kBrickKeys / 32), 0u, s);
        if (e == hipSuccess) e = fill_u64(w.list_total, 1, 0, s);
        if (e != hipSuccess) return e;
        k_totals<<<dim3(1), dim3(64), 0, s>>>(L->counter, L->capacity, out->n_frag);
        if (L->n_head > (1ull << 32))
            k_hist<uint64_t><<<dim3(grid), dim3(kBlock), 0, s>>>((const uint64_t*)L->keys, L->counter,
                                                             L->capacity, w.brick_cnt, w.bitmap);
        else
            k_hist<uint32_t><<<dim3(grid), dim3(kBlock), 0, s>>>((const uint32_t*)L->keys, L->counter,
                                                             L->capacity, w.brick_cnt, w.bitmap);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(dev, "compact.scan", s);
        e = scan<uint64_t>(LoadBrick{w.brick_cnt}, StoreBrick{w.brick_off, w.list}, n_brick, w.part,
                           w.list_total, s);
        if (e == hipSuccess) e = brick_occ_launch(dev, w, n_brick, s);
        if (e == hipSuccess)
            e = scan<uint64_t>(LoadOcc{w.brick_occ}, StoreRank{w.brick_rank}, n_brick, w.part,
                               (uint64_t*)out->n_occ, s);
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(dev, "compact.scatter", s);
        if (L->n_head > (1ull << 32))
            k_scatter<uint64_t><<<dim3(grid), dim3(kBlock), 0, s>>>((const uint4*)L->pool,
                (const uint64_t*)L->keys, L->counter, L->capacity, w.brick_off, w.brick_cur, w.stage);
        else
            k_scatter<uint32_t><<<dim3(grid), dim3(kBlock), 0, s>>>((const uint4*)L->pool,
                (const uint32_t*)L->keys, L->counter, L->capacity, w.brick_off, w.brick_cur, w.stage);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    return brick_sorts(dev, w, out, n_brick, "compact.brick", s);
}

// Per-brick sorts of the staging array into the output arrays.
static hipError_t brick_sorts(const Device& dev, const CompactWs& w, const fhv_pofa* out, uint64_t n_brick,
                              const char* name, hipStream_t s)
{
    hipError_t e;
    const uint64_t bmax = (uint64_t)dev.cus * 4;
    const unsigned gbrick = (unsigned)(n_brick < bmax ? n_brick : bmax);
    ProfScope ps(dev, name, s);
    const uint64_t wmax = (uint64_t)dev.cus * 64;
    const unsigned gwave = (unsigned)(n_brick < wmax ? n_brick : wmax);
    k_brick_wave<kSmallRecs, 0><<<dim3(gwave ? gwave : 1), dim3(kWave), 0, s>>>(
        w.stage, w.brick_cnt, w.brick_off, w.brick_rank, w.list, w.list_total, (uint4*)out->frag,
        out->oct_key, out->oct_off, out->oct_cnt, out->cap_occ);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_brick_wave<kWaveRecs, kSmallRecs><<<dim3(gwave ? gwave : 1), dim3(kWave), 0, s>>>(
        w.stage, w.brick_cnt, w.brick_off, w.brick_rank, w.list, w.list_total, (uint4*)out->frag,
        out->oct_key, out->oct_off, out->oct_cnt, out->cap_occ);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_brick<<<dim3(gbrick ? gbrick : 1), dim3(kBlock), 0, s>>>(
        w.stage, w.brick_cnt, w.brick_off, w.brick_rank, w.list, w.list_total, (uint4*)out->frag,
        out->oct_key, out->oct_off, out->oct_cnt, out->cap_occ);
    return hipGetLastError();
}

// Two-pass capture into arrays: after the count pass and the scans, the
// fragment total decides whether the arrays hold them; if not, only the
// counts are reported and the insert pass and the sorts do nothing.
__global__ void k_arrays_check(uint64_t* __restrict__ list_total, uint64_t capacity, uint64_t* __restrict__ n_frag,
                               uint64_t* __restrict__ n_occ, uint32_t* __restrict__ skip)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t total = *list_total & 0xFFFFFFFFull;
    *n_frag = total;
    if (total > capacity) {
        *skip = 1u;
        *list_total = total;   // no occupied bricks left to sort
        *n_occ = 0;
    } else {
        *skip = 0u;
    }
}

size_t capture_arrays_ws_bytes(const fhv_capture_desc* d, uint32_t n_tri, uint64_t capacity)
{
    const size_t cap_b = (capture_ws_bytes(d, n_tri) + 255) & ~(size_t)255;
    size_t b = 0;
    carve_compact(nullptr, 1ull << (3 * d->levels), capacity, &b);
    return cap_b + ((b + 255) & ~(size_t)255) + 256;
}

hipError_t capture_arrays_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d,
                                 const fhv_pofa* out, void* ws, hipStream_t s)
{
    const uint64_t n_head = 1ull << (3 * d->levels);
    const uint64_t n_brick = (n_head + kBrickKeys - 1) / kBrickKeys;
    const size_t cap_b = (capture_ws_bytes(d, m->n_tri) + 255) & ~(size_t)255;
    size_t cmp_b = 0;
    CompactWs w = carve_compact((char*)ws + cap_b, n_head, out->cap_frag, &cmp_b);
    uint32_t* skip = (uint32_t*)((char*)ws + cap_b + ((cmp_b + 255) & ~(size_t)255));
    hipError_t e;
    {
        ProfScope ps(dev, "arrays.reset", s);
        e = fill_u32(w.brick_cnt, 3 * n_brick + n_brick * (kBrickKeys / 32), 0u, s);
        if (e == hipSuccess) e = fill_u64(w.list_total, 1, 0, s);
        if (e == hipSuccess) e = fill_u32(skip, 1, 0u, s);
    }
    if (e != hipSuccess) return e;
    BrickSink bs{w.brick_cnt, w.bitmap, w.brick_off, w.brick_cur, w.stage, skip};
    e = capture_bricks_launch(dev, m, d, ws, kActCount, bs, s);
    if (e != hipSuccess) return e;
    {
        ProfScope ps(dev, "arrays.scan", s);
        e = scan<uint64_t>(LoadBrick{w.brick_cnt}, StoreBrick{w.brick_off, w.list}, n_brick, w.part,
                           w.list_total, s);
        if (e == hipSuccess) e = brick_occ_launch(dev, w, n_brick, s);
        if (e == hipSuccess)
            e = scan<uint64_t>(LoadOcc{w.brick_occ}, StoreRank{w.brick_rank}, n_brick, w.part,
                               (uint64_t*)out->n_occ, s);
        if (e == hipSuccess) {
            k_arrays_check<<<dim3(1), dim3(64), 0, s>>>(w.list_total, out->cap_frag, out->n_frag, out->n_occ, skip);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    e = capture_bricks_launch(dev, m, d, ws, kActInsert, bs, s);
    if (e != hipSuccess) return e;
    return brick_sorts(dev, w, out, n_brick, "arrays.brick", s);
}

}  // namespace fhv
