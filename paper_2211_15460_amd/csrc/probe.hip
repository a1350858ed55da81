// Measurement probes: the streaming bandwidths (copy, read only, write only)
// and the rate of uncontended device-scope atomics, the ceilings against which
// the capture (list head exchanges, counters), compaction (brick counts) and
// splat kernels are measured. Each atomic probe touches one word at the start
// of every line of a buffer, once per pass, so no two atomics of a pass meet
// on one line; the buffer's size decides whether the lines live in HBM or
// stay in the last-level cache.
//
//   k_probe_copy     dst <- src in 16-byte vector loads and stores, eight
//                    per thread in flight
//   k_probe_read     every 16 bytes of the buffer loaded once (eight per
//                    thread in flight) and folded into a value that decides
//                    a store which never happens
//   k_probe_write    every 16 bytes of the buffer stored once
//   Each stream comes in two access forms: non-temporal (streamed past the
//   caches) and ordinary (as the library's own kernels access memory, lines
//   allocated in the caches on the way), since which of the two is faster
//   depends on the stream's mix and size.
//   k_probe_atomic   per line and pass: add 1 (u32, result unused), exchange
//                    (u32, result used, as the list insertion does) or
//                    minimum (u64, result unused, each pass storing a smaller
//                    value than the last, as a z-buffer test that wins)
#include "fhv_common.h"

namespace fhv {

namespace {

constexpr int kProbeU = 8;   // 16-byte units per thread and iteration

template <bool kNT>
__device__ __forceinline__ uint4 load16(const uint4* p)
{
    if (!kNT) return *p;
    uint4 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
}

template <bool kNT>
__device__ __forceinline__ void store16(uint4* p, uint4 v)
{
    if (!kNT) {
        *p = v;
        return;
    }
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
}

// All loads of an iteration are issued before its stores, so that enough
// reads are in flight to cover the memory latency.
template <bool kNT>
__global__ void __launch_bounds__(kBlock)
k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + (kProbeU - 1) * stride < n; i += kProbeU * stride) {
        uint4 v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) v[u] = load16<kNT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) store16<kNT>(dst + i + u * stride, v[u]);
    }
    for (; i < n; i += stride) store16<kNT>(dst + i, load16<kNT>(src + i));
}

template <bool kNT>
__global__ void __launch_bounds__(kBlock)
k_probe_read(uint4* __restrict__ buf, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kProbeU - 1) * stride < n; i += kProbeU * stride) {
        uint4 v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) v[u] = load16<kNT>(buf + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const uint4 v = load16<kNT>(buf + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // the probe's buffers are filled with 0xFF bytes, so the fold of an even
    // number of words is 0 and of an odd number ~0: never this value
    if (acc == 0x5A5A5A5Au) buf[0].x = acc;
}

template <bool kNT>
__global__ void __launch_bounds__(kBlock)
k_probe_write(uint4* __restrict__ buf, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint4 v = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) store16<kNT>(buf + i, v);
}

template <uint32_t kOp>
__global__ void __launch_bounds__(kBlock)
k_probe_atomic(uint8_t* __restrict__ buf, uint64_t n_lines, uint32_t line, uint32_t passes)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t r = 0; r < passes; ++r)
        for (uint64_t i = t; i < n_lines; i += stride) {
            uint8_t* p = buf + i * line;
            if (kOp == FHV_PROBE_ADD_U32) {
                atomicAdd((uint32_t*)p, 1u);
            } else if (kOp == FHV_PROBE_EXCH_U32) {
                acc += atomicExch((uint32_t*)p, r + 1u);
            } else {
                const unsigned long long v = ((unsigned long long)(passes - r) << 32) | (uint32_t)i;
                atomicMin((unsigned long long*)p, v);
            }
        }
    // the exchanged values feed a result, so the exchanges must return them;
    // the second word of each line is the probe's own and never an operand
    if (kOp == FHV_PROBE_EXCH_U32 && t < n_lines) ((uint32_t*)(buf + t * line))[1] = acc;
}

}  // namespace

hipError_t probe_launch(const Device& dev, uint32_t kind, void* buf, uint64_t bytes, uint32_t line,
                        uint32_t passes, hipStream_t s)
{
    // the streams launch as the library's own streaming kernels do: up to
    // 32 workgroups per compute unit, each thread looping over the rest
    const uint64_t gmax = (uint64_t)dev.cus * 16, smax = (uint64_t)dev.cus * 32;
    if (kind == FHV_PROBE_COPY || kind == FHV_PROBE_COPY_CACHED) {
        const uint64_t n = bytes / 32;   // 16-byte units per half
        uint64_t g = (n + kBlock - 1) / kBlock;
        g = g < 1 ? 1 : (g > smax ? smax : g);
        const uint4* src = (const uint4*)buf;
        uint4* dst = (uint4*)buf + n;
        if (kind == FHV_PROBE_COPY) {
            ProfScope ps(dev, "probe.copy", s);
            k_probe_copy<true><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(src, dst, n);
        } else {
            ProfScope ps(dev, "probe.copy_cached", s);
            k_probe_copy<false><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(src, dst, n);
        }
        return hipGetLastError();
    }
    if (kind == FHV_PROBE_READ || kind == FHV_PROBE_WRITE || kind == FHV_PROBE_READ_CACHED ||
        kind == FHV_PROBE_WRITE_CACHED) {
        const uint64_t n = bytes / 16;
        uint64_t g = (n + kBlock - 1) / kBlock;
        g = g < 1 ? 1 : (g > smax ? smax : g);
        uint4* b = (uint4*)buf;
        const dim3 grid((unsigned)g), block(kBlock);
        switch (kind) {
        case FHV_PROBE_READ: {
            ProfScope ps(dev, "probe.read", s);
            k_probe_read<true><<<grid, block, 0, s>>>(b, n);
            break;
        }
        case FHV_PROBE_READ_CACHED: {
            ProfScope ps(dev, "probe.read_cached", s);
            k_probe_read<false><<<grid, block, 0, s>>>(b, n);
            break;
        }
        case FHV_PROBE_WRITE: {
            ProfScope ps(dev, "probe.write", s);
            k_probe_write<true><<<grid, block, 0, s>>>(b, n);
            break;
        }
        default: {
            ProfScope ps(dev, "probe.write_cached", s);
            k_probe_write<false><<<grid, block, 0, s>>>(b, n);
            break;
        }
        }
        return hipGetLastError();
    }
    const uint64_t n_lines = bytes / line;
    uint64_t g = (n_lines + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : (g > gmax ? gmax : g);
    uint8_t* b = (uint8_t*)buf;
    switch (kind) {
    case FHV_PROBE_ADD_U32: {
        ProfScope ps(dev, "probe.add_u32", s);
        k_probe_atomic<FHV_PROBE_ADD_U32><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(b, n_lines, line, passes);
        break;
    }
    case FHV_PROBE_EXCH_U32: {
        ProfScope ps(dev, "probe.exch_u32", s);
        k_probe_atomic<FHV_PROBE_EXCH_U32><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(b, n_lines, line, passes);
        break;
    }
    default: {
        ProfScope ps(dev, "probe.min_u64", s);
        k_probe_atomic<FHV_PROBE_MIN_U64><<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(b, n_lines, line, passes);
        break;
    }
    }
    return hipGetLastError();
}

}  // namespace fhv
