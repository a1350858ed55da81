// Measurement probes: the copy bandwidth and the rate of uncontended
// device-scope atomics, the ceilings against which the capture (list head
// exchanges, counters), compaction (brick counts) and splat (64-bit z-buffer
// minima) kernels are measured. Each atomic probe touches one word at the
// start of every line of a buffer, once per pass, so no two atomics of a
// pass meet on one line; the buffer's size decides whether the lines live in
// HBM or stay in the last-level cache.
//
//   k_probe_copy     dst <- src in 16-byte vector loads and stores
//   k_probe_atomic   per line and pass: add 1 (u32, result unused), exchange
//                    (u32, result used, as the list insertion does) or
//                    minimum (u64, result unused, each pass storing a smaller
//                    value than the last, as a z-buffer test that wins)
#include "fhv_common.h"

namespace fhv {

namespace {

// Four 16-byte units per thread and iteration, all loads issued before the
// stores, so that enough reads are in flight to cover the memory latency.
__global__ void __launch_bounds__(kBlock)
k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n)
{
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
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
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    if (kind == FHV_PROBE_COPY) {
        const uint64_t n = bytes / 32;   // 16-byte units per half
        uint64_t g = (n + kBlock - 1) / kBlock;
        g = g < 1 ? 1 : (g > gmax ? gmax : g);
        ProfScope ps(dev, "probe.copy", s);
        k_probe_copy<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>((const uint4*)buf, (uint4*)buf + n, n);
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
