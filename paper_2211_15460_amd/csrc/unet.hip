// Learned hole fill: a U-Net that predicts an RGB residual for a splat image
// (RGBA, depth, coverage), trained and run with bfloat16 MFMA kernels and
// fp32 accumulation. Not part of the paper: it fills the holes the point
// splat leaves (Sec. 3.3 mentions adapting quad sizes or deforming geometry
// for that; this network learns the fill instead).
//
// Network (levels L = 1..4, base 32 channels, C_l = 32 * 2^l):
//   encoder level l: conv3x3 + ReLU, conv3x3 + ReLU, 2x2 max pool (l < L-1)
//   decoder level l (L-2 .. 0): 2x2 stride-2 transposed conv, concat with
//     the encoder output of level l (transposed conv first), conv3x3 + ReLU
//     twice; head: 1x1 conv to 3 channels, a residual on splat RGB / 255.
// Parameters: one fp32 vector, layer after layer: 3x3 conv W[co][ky][kx][ci]
// then b[co]; transposed conv W[dy][dx][co][ci] then b[co]; head W[k][c]
// then b[k].
//
// Activations are NHWC bfloat16 (round to nearest even). The encoder's second
// convolution writes straight into the skip half of its level's concat
// buffer, the decoder's transposed convolution into the other half, so the
// concatenation costs nothing.
//
// Kernels (implicit GEMM on MFMA 16x16x32 bf16, fused bias, ReLU and bf16
// rounding; sums over 32-channel chunks, then taps, in all of them)
//   k_conv3r      full-size 3x3 layers with 32 output channels: persistent,
//                 one loading wave feeding a three-stage LDS ring by direct
//                 buffer-to-LDS loads, weights resident; optionally the
//                 encoder's 2x2 max pool or, for the last layer in inference,
//                 the 1x1 head with the filled image
//   k_conv3a      3x3 layers with 64-multiple output channels: persistent, halo and
//                 weights double-buffered by direct buffer-to-LDS loads;
//                 optionally the 2x2 max pool
//   k_conv3       the other 3x3 layers (also input gradients with flipped
//                 transposed weights) and the 2x2 stride-2 transposed
//                 convolution as a 1x1 product onto (sub-position, channel)
//                 columns, input halo and weights staged in LDS per chunk
//   k_conv        the remaining shapes (8 input channels; gathered input
//                 gradient of the transposed convolution), operands through
//                 buffer resources
//   k_wgrad       weight gradients: GEMM over pixels, every tap per wave, the
//                 operands staged through LDS transposed (pixels contiguous),
//                 four pixel splits per workgroup summed in LDS, fp32 partial
//                 rows and a fixed-order reduction
//   k_colsum      bias gradients, split over pixel ranges the same way
//   elementwise   input packing, max-pool gradient (plus the skip gradient),
//                 ReLU gradient, head with loss in training, Adam, weight
//                 conversion to bf16 layouts
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fhv_common.h"

namespace fhv {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBase = 32;
constexpr int kInPad = 8;   // 6 input channels padded to 8

// fp32 to bf16, round to nearest even: the conversion instruction of
// gfx950 (two values per instruction in f2bf2)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// lo in the low half, hi in the high half
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{lo, hi}, bf16x2));
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum { MODE_SAME3 = 0, MODE_UP2 = 1, MODE_GATHER4 = 2 };

struct ConvArgs {
    const uint16_t* in;   // first input channel of pixel 0
    const uint16_t* wt;   // [Cout][T * Cin] bf16 (UP2: + tap * Cout * Cin)
    const float* bias;    // fp32 [Cout] or null
    uint16_t* out;        // first output channel of pixel 0
    uint32_t in_cs, out_cs;   // elements per pixel
    uint32_t N, H, W;     // row grid: output grid (SAME3, GATHER4), input grid (UP2)
    uint32_t Cin, Cout, T, mode, relu;
    uint16_t* pool;       // 3x3 only, or null: also write the 2x2 max pool of the output
    uint32_t pool_cs;     // elements per pooled pixel
    // 3x3 with 32 output channels only, or null: apply the 1x1 head to the
    // (bf16) output and write the filled image (and the residual, if asked);
    // the convolution's own output is then not stored
    const float* head_w;  // [3][32]
    const float* head_b;  // [3]
    const uint32_t* head_rgba;
    uint32_t* head_out;
    float* head_res;
};

// Buffer resource over `bytes` bytes at p (raw, unswizzled): loads at an
// offset at or beyond `bytes` return zeros, which is how out-of-image taps
// and channels past the end read as zero padding without branches.
constexpr uint32_t kOob = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// rsrc from values that may sit in vector registers, read back as scalars
__device__ __forceinline__ __amdgpu_buffer_rsrc_t srsrc(const void* p, uint32_t bytes)
{
    const uint64_t v = (uint64_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return rsrc((const void*)(lo | (hi << 32)), __builtin_amdgcn_readfirstlane(bytes));
}

__device__ __forceinline__ u32x4 bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

// The bias of this lane's output channel in each of a wave tile's NJ
// 16-channel columns (zero without bias or past Cout).
template <int NJ>
__device__ __forceinline__ void tile_bias(float (&bv)[NJ], const float* __restrict__ bias, uint32_t co0,
                                          uint32_t Cout)
{
    const int l16 = __lane_id() & 15;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t co = co0 + 16 * j + l16;
        bv[j] = (bias && co < Cout) ? bias[co] : 0.0f;
    }
}

// Epilogue of a wave's (16 MI)-pixel x (16 NJ)-channel result tile: bias
// (per column, from tile_bias), ReLU and bf16 rounding, then a pass through
// the wave's own LDS region (pixel-major, pitch 16 NJ + 8) so that each lane
// stores whole 16-byte runs of 8 channels of one pixel. dst(p) is the first
// output channel of the tile's pixel p, or null when that pixel is outside
// the output.
template <int MI, int NJ, class Dst>
__device__ __forceinline__ void store_tile(uint16_t* __restrict__ lds, const floatx4 (&acc)[MI][NJ],
                                           const float (&bv)[NJ], uint32_t co0, uint32_t Cout, bool relu, Dst dst,
                                           int lane = __lane_id())
{
    constexpr int P = 16 * NJ + 8, CH = 2 * NJ;
    const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float b = bv[j];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[i][j][r] + b;
                if (relu) v = v > 0.0f ? v : 0.0f;
                lds[(16 * i + 4 * g + r) * P + 16 * j + l16] = f2bf(v);
            }
    }
    // the wave reads back what its own lanes wrote
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < (16 * MI * CH) / kWave; ++t) {
        const int id = lane + kWave * t, px = id / CH, q = id % CH;
        const u32x4 v = *(const u32x4*)&lds[px * P + q * 8];
        uint16_t* d = dst(px);
        if (d && co0 + 8 * q < Cout) *(u32x4*)(d + 8 * q) = v;
    }
}

template <int MI, int NJ, class Dst>
__device__ __forceinline__ void store_tile(uint16_t* __restrict__ lds, const floatx4 (&acc)[MI][NJ],
                                           const float* __restrict__ bias, uint32_t co0, uint32_t Cout,
                                           bool relu, Dst dst)
{
    float bv[NJ];
    tile_bias<NJ>(bv, bias, co0, Cout);
    store_tile<MI, NJ>(lds, acc, bv, co0, Cout, relu, dst);
}

// 2x2 max pool of four 8-channel bf16 vectors, the window's pixels in
// (0,0), (0,1), (1,0), (1,1) order: per channel the first largest value.
__device__ __forceinline__ u32x4 max4_bf16(const u32x4 (&v)[4])
{
    u32x4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint32_t word = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float m = -INFINITY;
            uint32_t best = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t bb = (v[k][c] >> (16 * h)) & 0xFFFFu;
                if (bf2f((uint16_t)bb) > m) {
                    m = bf2f((uint16_t)bb);
                    best = bb;
                }
            }
            word |= best << (16 * h);
        }
        o[c] = word;
    }
    return o;
}

// The 1x1 head on pixel p from its 32 bf16 channels hp (in LDS): residual
// W h + b (hw: W [3][32], then b [3], in LDS) as a chain of fused
// multiply-adds, added to the splat colour sp (times the fp32 reciprocal of
// 255), clamped, rounded half up; alpha 255.
__device__ __forceinline__ void head_pixel(const ConvArgs& a, const float* hw, const uint16_t* hp, size_t p,
                                           uint32_t sp)
{
    float r[3] = {hw[96], hw[97], hw[98]};
#pragma unroll 1
    for (int c4 = 0; c4 < 4; ++c4) {
        const u32x4 hv = *(const u32x4*)(hp + 8 * c4);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int c = 8 * c4 + e;
            const float v = bf2f((uint16_t)(hv[e >> 1] >> (16 * (e & 1))));
#pragma unroll
            for (int k = 0; k < 3; ++k) r[k] = __builtin_fmaf(hw[k * 32 + c], v, r[k]);   // one rounding per term
        }
    }
    uint32_t o = 0xFF000000u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float v = (float)((sp >> (8 * k)) & 0xFFu) * (1.0f / 255.0f) + r[k];
        v = v < 0.0f ? 0.0f : (v > 1.0f ? 1.0f : v);
        o |= (uint32_t)floorf(v * 255.0f + 0.5f) << (8 * k);
        if (a.head_res) a.head_res[p * 3 + k] = r[k];
    }
    a.head_out[p] = o;
}

// Wave tile (16 MI) pixels of one row x (16 NJ) output channels, MI x NJ
// MFMA 16x16x32 tiles; a workgroup is 4 waves side by side along the row.
// The K loop runs over (tap, 32-channel chunk) pairs. Per tap, the source
// row is wave-uniform and becomes a buffer resource (empty when the row is
// outside the image); per lane only the column offset and its validity
// change. The operands of the next chunk are loaded before the matrix
// products of the current one. kSmall: 8 input channels, where a 32-wide
// K chunk spans four taps (one per lane group).
template <int kMode, int MI, int NJ, bool kSmall>
__global__ void __launch_bounds__(kBlock) k_conv(ConvArgs a)
{
    constexpr int WX = 16 * MI;
    __shared__ __attribute__((aligned(16))) uint16_t epi[kBlock / kWave][16 * MI * (16 * NJ + 8)];
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const int g = lane >> 4, l16 = lane & 15;
    const uint32_t xtiles = (a.W + 4 * WX - 1) / (4 * WX);
    // UP2: the four output sub-positions of a tile are adjacent workgroups,
    // so they share the input tile in cache and write neighbouring pixels
    const uint32_t tapz = kMode == MODE_UP2 ? (blockIdx.x & 3u) : 0u;
    const uint32_t bx = kMode == MODE_UP2 ? (blockIdx.x >> 2) : blockIdx.x;
    const uint32_t row = bx / xtiles;
    const uint32_t x0 = (bx % xtiles) * (4 * WX) + wv * WX;
    if (x0 >= a.W) return;   // whole wave past the row end
    const uint32_t n = row / a.H, y = row % a.H;
    const uint32_t co0 = blockIdx.y * (16 * NJ);
    const uint32_t K = a.T * a.Cin;
    const uint16_t* wt = a.wt + (kMode == MODE_UP2 ? (size_t)tapz * a.Cout * a.Cin : 0);
    const __amdgpu_buffer_rsrc_t wr = rsrc(wt, a.Cout * K * 2);
    const uint32_t nc = a.Cin >> 5;
    const uint32_t total = kSmall ? (K + 31) / 32 : a.T * nc;
    const uint32_t pix_b = a.in_cs * 2;   // bytes per input pixel
    uint32_t wo[NJ];                      // weight row offsets (bytes)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t co = co0 + 16 * j + l16;
        wo[j] = co < a.Cout ? (co * K + g * 8) * 2 : kOob;
    }
    // input rows of the grid the operand is read from
    const uint32_t in_w = kMode == MODE_GATHER4 ? 2 * a.W : a.W;
    const uint32_t in_h = kMode == MODE_GATHER4 ? 2 * a.H : a.H;
    uint32_t xo[MI];   // per-lane column offsets (bytes) before the tap shift
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        const uint32_t x = x0 + 16 * i + l16;
        xo[i] = (kMode == MODE_GATHER4 ? 2 * x : x) * pix_b + g * 16;
    }
    uint32_t ltap = 0, lcc = 0;   // next (tap, chunk) to load
    auto load = [&](u32x4 (&av)[MI], u32x4 (&bv)[NJ]) {
        if (kSmall) {
            // 8 channels: lane group g reads tap 4 * chunk + g, all channels
            const uint32_t k = lcc * 32 + g * 8;
            const bool kok = k < K;
            const uint32_t tap = kok ? k >> 3 : 0;
            const uint32_t dy = (tap * 11) >> 5, dx = tap - 3 * dy;   // tap / 3, tap % 3 for tap < 9
            const int ys = (int)y + (int)dy - 1;
            const bool rok = kok && ys >= 0 && ys < (int)a.H;
            // image n as one buffer resource (the lane groups read different
            // rows): taps outside the image read zeros through the range
            // check, with no branch that would wait for the load
            const __amdgpu_buffer_rsrc_t ir = rsrc(a.in + (size_t)n * a.H * a.W * a.in_cs, a.H * a.W * pix_b);
#pragma unroll
            for (int i = 0; i < MI; ++i) {
                const int xs = (int)(x0 + 16 * i + l16) + (int)dx - 1;
                const bool ok = rok && xs >= 0 && xs < (int)a.W;
                av[i] = bload(ir, ok ? ((uint32_t)ys * a.W + (uint32_t)xs) * pix_b : kOob, 0);
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) bv[j] = bload(wr, kok ? wo[j] - g * 16 + k * 2 : kOob, 0);
            ++lcc;
            return;
        }
        const uint32_t tap = ltap, cb = lcc * 64;   // chunk byte offset
        if (++lcc == nc) {
            lcc = 0;
            ++ltap;
        }
        uint32_t ys, dxb = 0;
        bool rok = true;
        uint32_t lo_ok = 0, hi_ok = 0;   // which shifted columns stay inside
        if (kMode == MODE_SAME3) {
            const uint32_t dy = (tap * 11) >> 5, dx = tap - 3 * dy;
            const int yy = (int)y + (int)dy - 1;
            rok = yy >= 0 && yy < (int)a.H;
            ys = rok ? (uint32_t)yy : 0;
            dxb = dx * pix_b;
            lo_ok = dx == 0;
            hi_ok = dx == 2;
        } else if (kMode == MODE_GATHER4) {
            ys = 2 * y + (tap >> 1);
            dxb = (tap & 1) * pix_b;
        } else {
            ys = y;
        }
        rok = rok && ys < in_h;
        const size_t rbase = ((size_t)n * in_h + (rok ? ys : 0)) * in_w * a.in_cs;
        const __amdgpu_buffer_rsrc_t ir = rsrc(a.in + rbase, rok ? in_w * pix_b : 0u);
#pragma unroll
        for (int i = 0; i < MI; ++i) {
            const uint32_t x = x0 + 16 * i + l16;
            bool ok = x < a.W;
            if (kMode == MODE_SAME3) {
                // column x + dx - 1: invalid left of 0 (dx = 0, x = 0) and
                // right of W - 1 (dx = 2, x = W - 1)
                ok = ok && !(lo_ok && x == 0) && !(hi_ok && x + 1 >= a.W);
            }
            const uint32_t off = kMode == MODE_SAME3 ? xo[i] + dxb - pix_b : xo[i] + dxb;
            av[i] = bload(ir, ok ? off : kOob, cb);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) bv[j] = bload(wr, wo[j], (tap * a.Cin) * 2 + cb);
    };
    floatx4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](const u32x4 (&av)[MI], const u32x4 (&bv)[NJ]) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av[i]), __builtin_bit_cast(bf16x8, bv[j]), acc[i][j], 0, 0, 0);
    };
    // Loads run one chunk ahead without conditions: the one past the end
    // reads in-range memory or zeros (buffer range checks) and is not used.
    u32x4 a0[MI], b0[NJ], a1[MI], b1[NJ];
    load(a0, b0);
    for (uint32_t it = 0; it + 2 <= total; it += 2) {
        load(a1, b1);
        mma(a0, b0);
        load(a0, b0);
        mma(a1, b1);
    }
    if (total & 1) mma(a0, b0);
    store_tile<MI, NJ>(epi[wv], acc, a.bias, co0, a.Cout, a.relu != 0, [&](int px) -> uint16_t* {
        const uint32_t x = x0 + px;
        if (x >= a.W) return nullptr;
        size_t dst;
        if (kMode == MODE_UP2)
            dst = ((size_t)n * 2 * a.H + 2 * y + (tapz >> 1)) * (2 * (size_t)a.W) + 2 * x + (tapz & 1);
        else
            dst = (size_t)row * a.W + x;
        return a.out + dst * a.out_cs + co0;
    });
}

// 3x3 convolution (stride 1, zero padding 1) with Cin a multiple of 32.
// A workgroup computes 2 output rows x TX pixels x (16 NJ) channels; its
// four waves take 64 pixels of one row each and, when TX = 64, half of the
// channels (4 x NJ or 4 x NJ/2 MFMA tiles). TX = 64 halves the halo so that
// two workgroups share a compute unit's LDS and hide each other's loads. Per
// 32-channel chunk, the input halo (4 rows x TX+2 pixels, zero outside the
// image) and the chunk's weights of all nine taps are staged in LDS, so the
// tap loop reads only LDS: the next tap's operands are read while the
// current tap's matrix products run, and the next chunk's halo and weights
// are loaded into registers meanwhile. Rows of 32 channels are padded to
// 48 bf16 (96 B): the 16-byte reads of 16 consecutive rows at 4 channel
// offsets (one MFMA operand) then run at the LDS's full rate, which rows of
// 64 or 80 bytes do not (bank conflicts; measured on gfx950).
//
// kUp: the same structure for the 2x2 stride-2 transposed convolution,
// which is a 1x1 convolution onto 4 Cout columns (sub-position, channel):
// one tap, no halo, and the epilogue scatters each 32-column group to its
// sub-position of the doubled grid.
//
// R = 4 (with TX = 64): four output rows, one per wave, all channels of the
// tile per wave; the halo of 6 rows for 4 output rows re-reads less of the
// input than 4 rows for 2, which matters for the memory-bound full-size
// layers.
template <int NJ, int TX, bool kUp, int R = 2>
__global__ void __launch_bounds__(kBlock) k_conv3(ConvArgs a)
{
    constexpr int T = kUp ? 1 : 9, PAD = kUp ? 0 : 1;
    constexpr int HP = TX + 2 * PAD, RP = R + 2 * PAD, TN = 16 * NJ, PITCH = 48;
    // waves: R = 4 -> one row each; TX = 128 -> (row, 64-pixel half);
    // TX = 64 -> (row, half of the channels)
    constexpr int NW = (R == 4 || TX == 128) ? NJ : NJ / 2;   // MFMA column tiles per wave
    static_assert((R == 2 && (TX == 128 || (TX == 64 && NJ % 2 == 0))) || (R == 4 && TX == 64), "tile shape");
    // element offset of 16-byte chunk q of staged row `row` (a pixel of the
    // halo or an output channel of the weights)
    auto loff = [](uint32_t row, uint32_t q) -> uint32_t { return row * PITCH + q * 8; };
    constexpr int HU = RP * HP * 4, WU = T * TN * 4;     // 16-byte units: halo, weights
    constexpr int HPT = (HU + kBlock - 1) / kBlock, WPT = (WU + kBlock - 1) / kBlock;
    constexpr int HALO = RP * HP * PITCH;                // bf16 elements
    constexpr int STAGE = HALO + T * TN * PITCH, EPI = 4 * 64 * (16 * NW + 8);
    constexpr int EP = 16 * NW + 8;                      // epilogue pitch (bf16 per pixel)
    __shared__ __attribute__((aligned(16))) uint16_t lds[STAGE > EPI ? STAGE : EPI];
    uint16_t* const tile = lds;
    uint16_t* const wts = lds + HALO;
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const int g = lane >> 4, l16 = lane & 15;
    const uint32_t xtiles = (a.W + TX - 1) / TX, ytiles = (a.H + R - 1) / R;
    const uint32_t n_tiles = a.N * ytiles * xtiles;
    const uint32_t wr = R == 4 ? (uint32_t)wv : (uint32_t)wv >> 1;
    const uint32_t wx = (R == 2 && TX == 128) ? ((uint32_t)wv & 1u) * 64u : 0u;
    const uint32_t wco = (R == 2 && TX == 64) ? ((uint32_t)wv & 1u) * (16u * NW) : 0u;   // wave's channel offset
    const uint32_t co0 = blockIdx.y * TN;
    const uint32_t Cin = a.Cin, K = T * Cin, nc = Cin >> 5;
    const uint32_t Cg = kUp ? 4 * a.Cout : a.Cout;   // GEMM columns
    const uint32_t row_b = a.W * a.in_cs * 2;
    const __amdgpu_buffer_rsrc_t wrs = rsrc(a.wt, Cg * K * 2);
    // Workgroups are persistent: a workgroup takes tiles blockIdx.x,
    // blockIdx.x + gridDim.x, ... and every (tile, chunk) unit's operands are
    // loaded while the previous unit is computed (across tiles too).
    struct Geo {
        uint32_t n, y0, x0, r_first;
        __amdgpu_buffer_rsrc_t ir;
    };
    auto geo = [&](uint32_t t) {
        Geo q;
        q.n = t / (xtiles * ytiles);
        const uint32_t rem = t % (xtiles * ytiles);
        q.y0 = (rem / xtiles) * R;
        q.x0 = (rem % xtiles) * TX;
        // input rows y0-PAD .. y0+R-1+PAD of image n, as far as they exist
        q.r_first = q.y0 >= (uint32_t)PAD ? q.y0 - PAD : 0;
        const uint32_t r_last = q.y0 + R - 1 + PAD < a.H ? q.y0 + R - 1 + PAD : a.H - 1;
        q.ir = rsrc(a.in + ((size_t)q.n * a.H + q.r_first) * a.W * a.in_cs, (r_last - q.r_first + 1) * row_b);
        return q;
    };
    // staging units of this thread (16 bytes each): global byte offsets
    // (out-of-range offsets read zeros) and LDS element offsets, recomputed
    // per unit to keep registers for the operands
    auto halo_unit = [&](const Geo& q, int u, uint32_t* go, uint32_t* lo) {
        const uint32_t idx = threadIdx.x + u * kBlock;
        const uint32_t r = idx / (HP * 4), px = (idx % (HP * 4)) >> 2, c = idx & 3;
        const int ys = (int)q.y0 + (int)r - PAD, xs = (int)q.x0 + (int)px - PAD;
        const bool ok = idx < (uint32_t)HU && ys >= 0 && ys < (int)a.H && xs >= 0 && xs < (int)a.W;
        *go = ok ? ((uint32_t)ys - q.r_first) * row_b + (uint32_t)xs * a.in_cs * 2 + c * 16 : kOob;
        *lo = loff(r * HP + px, c);
        return idx < (uint32_t)HU;
    };
    auto wt_unit = [&](int u, uint32_t* go, uint32_t* lo) {
        const uint32_t idx = threadIdx.x + u * kBlock;
        const uint32_t tap = idx / (TN * 4), co = (idx % (TN * 4)) >> 2, c = idx & 3;
        const bool ok = idx < (uint32_t)WU && co0 + co < Cg;
        *go = ok ? ((co0 + co) * K + tap * Cin + c * 8) * 2 : kOob;
        *lo = loff(tap * TN + co, c);
        return idx < (uint32_t)WU;
    };
    u32x4 hst[HPT], wst[WPT];
    auto gload = [&](const Geo& q, uint32_t cc) {
        uint32_t go, lo;
#pragma unroll
        for (int u = 0; u < HPT; ++u) {
            halo_unit(q, u, &go, &lo);
            hst[u] = bload(q.ir, go, cc * 64);
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            wt_unit(u, &go, &lo);
            wst[u] = bload(wrs, go, cc * 64);
        }
    };
    auto lds_put = [&](const Geo& q) {
        uint32_t go, lo;
#pragma unroll
        for (int u = 0; u < HPT; ++u)
            if (halo_unit(q, u, &go, &lo)) *(u32x4*)&tile[lo] = hst[u];
#pragma unroll
        for (int u = 0; u < WPT; ++u)
            if (wt_unit(u, &go, &lo)) *(u32x4*)&wts[lo] = wst[u];
    };
    floatx4 acc[4][NW];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&]() {
        u32x4 av[2][4], bv[2][NW];
        auto rd = [&](int tap, u32x4 (&A)[4], u32x4 (&B)[NW]) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                A[i] = *(const u32x4*)&tile[loff((wr + dy) * HP + wx + 16 * i + l16 + dx, g)];
#pragma unroll
            for (int j = 0; j < NW; ++j) B[j] = *(const u32x4*)&wts[loff(tap * TN + wco + 16 * j + l16, g)];
        };
        rd(0, av[0], bv[0]);
#pragma unroll
        for (int tap = 0; tap < T; ++tap) {
            const int cur = tap & 1;
            if (tap + 1 < T) rd(tap + 1, av[cur ^ 1], bv[cur ^ 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[cur][i]), __builtin_bit_cast(bf16x8, bv[cur][j]), acc[i][j], 0, 0,
                        0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // Epilogue of tile q (the staging area is free: every wave has passed the
    // barrier before it); each wave uses its own part of the LDS.
    auto epilogue = [&](const Geo& q) {
        const uint32_t y = q.y0 + wr;
        if (kUp) {
            // 32 columns at a time, each within one sub-position (Cout is a
            // multiple of 32); the wave's LDS region is reused in order
#pragma unroll
            for (int h = 0; h < NW / 2; ++h) {
                const uint32_t cw = co0 + wco + 32 * h, tz = cw / a.Cout, cb = cw % a.Cout;
                floatx4 part[4][2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    part[i][0] = acc[i][2 * h];
                    part[i][1] = acc[i][2 * h + 1];
                }
                store_tile<4, 2>(lds + wv * 64 * EP, part, a.bias, cb, cw < Cg ? a.Cout : 0u, a.relu != 0,
                                 [&](int px) -> uint16_t* {
                                     const uint32_t x = q.x0 + wx + px;
                                     if (y >= a.H || x >= a.W) return nullptr;
                                     return a.out + (((size_t)q.n * 2 * a.H + 2 * y + (tz >> 1)) * (2 * (size_t)a.W) +
                                                     2 * x + (tz & 1)) * a.out_cs + cb;
                                 });
            }
            return;
        }
        store_tile<4, NW>(lds + wv * 64 * EP, acc, a.bias, co0 + wco, a.Cout, a.relu != 0,
                          [&](int px) -> uint16_t* {
                              const uint32_t x = q.x0 + wx + px;
                              if (y >= a.H || x >= a.W) return nullptr;
                              return a.out + (((size_t)q.n * a.H + y) * a.W + x) * a.out_cs + co0 + wco;
                          });
        if (!a.pool) return;
        // 2x2 max pool of the output rows (even H and W, y0 even), from the
        // waves' epilogue tiles; one thread per pooled pixel and 8 channels,
        // the first largest of the window in (0,0), (0,1), (1,0), (1,1) order
        __syncthreads();
        constexpr int PCH = TN / 8;   // 16-byte channel runs per pooled pixel
        constexpr int RUNS = (TX / 2) * (R / 2) * PCH;
        static_assert(RUNS % kBlock == 0, "whole passes over the pooled runs");
#pragma unroll
        for (int it = 0; it < RUNS / kBlock; ++it) {
            const uint32_t run = threadIdx.x + it * kBlock;
            const uint32_t c8 = run % PCH, p2 = (run / PCH) % (TX / 2), pr = run / (PCH * (TX / 2));
            const uint32_t xs = q.x0 + 2 * p2, ys = q.y0 + 2 * pr;
            if (xs >= a.W || ys >= a.H || co0 + 8 * c8 >= a.Cout) continue;
            u32x4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t r = 2 * pr + (k >> 1), px = 2 * p2 + (k & 1);   // within the tile
                const uint32_t w = R == 4 ? r : (TX == 128 ? 2 * r + px / 64 : 2 * r + (8 * c8) / (16 * NW));
                const uint32_t col = (R == 2 && TX == 64) ? (8 * c8) % (16 * NW) : 8 * c8;
                v[k] = *(const u32x4*)&lds[w * 64 * EP + (px % 64) * EP + col];
            }
            const u32x4 o = max4_bf16(v);
            *(u32x4*)(a.pool + (((size_t)q.n * (a.H / 2) + ys / 2) * (a.W / 2) + xs / 2) * a.pool_cs + co0 + 8 * c8) = o;
        }
    };

    uint32_t t = blockIdx.x, cc = 0;
    if (t >= n_tiles) return;   // whole workgroup
    Geo cur = geo(t);
    gload(cur, 0);
    lds_put(cur);
    __syncthreads();
    for (;;) {
        // the next unit: next chunk, or the first chunk of the next tile
        uint32_t nt = t, ncc = cc + 1;
        if (ncc == nc) {
            ncc = 0;
            nt = t + gridDim.x;
        }
        const bool more = nt < n_tiles;
        Geo nxt = cur;
        if (nt != t && more) nxt = geo(nt);
        if (more) gload(nxt, ncc);
        compute();
        __syncthreads();   // staged operands no longer needed
        if (cc + 1 == nc) {
            epilogue(cur);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
            __syncthreads();   // epilogue reads of the LDS done
        }
        if (!more) break;
        lds_put(nxt);
        __syncthreads();
        t = nt;
        cc = ncc;
        cur = nxt;
    }
}

// Deep 3x3 layers (Cin a multiple of 32, Cout a multiple of 64): a
// workgroup computes 8 output rows x 62 pixels x 64 channels with 8
// computing waves, one row per wave with all 64 channels (4 x 4 MFMA tiles
// per tap), and 1 loading wave. Per 32-channel chunk, the input halo (10
// rows x 64 pixels) and the weights of all nine taps are staged in LDS by
// direct buffer-to-LDS loads (no registers and no LDS write instructions in
// between), double-buffered: the loading wave fills the next (tile, chunk)
// unit while the current one is computed, and it alone waits for those
// loads, so the computing waves never wait on the memory counter (which
// also counts their own output stores). LDS rows are 64 bytes (32 bf16);
// the 16-byte chunk q of row r sits at position q ^ ((r >> 1) & 3), which
// keeps the operand reads of any 16 consecutive rows free of bank conflicts
// (measured on gfx950). Sums run in the same order as in k_conv3 (chunks,
// then taps), so results are the same.
namespace cva {
// A tile is 62 pixels wide so that a halo row is 64 pixels: moving the
// operand window by whole rows (the taps' dy) then leaves the swizzle of
// every lane unchanged and its addresses differ by constants. The waves'
// last two of 64 pixels are computed but not stored.
constexpr int R = 8, TX = 62, HP = TX + 2, RP = R + 2, TN = 64, NW = 4;
constexpr int HSLOTS = RP * HP * 4;     // halo slots (16 bytes each)
constexpr int WSLOTS = 9 * TN * 4;      // weight slots
constexpr int SLOTS = HSLOTS + WSLOTS;
constexpr int HINSTR = HSLOTS / 64;     // halo wave-loads per unit
constexpr int WINSTR = WSLOTS / 64;     // weight wave-loads per unit
constexpr int CWAVES = 8, WAVES = CWAVES + 1;
constexpr int EP = 16 * NW + 8;         // epilogue pitch (bf16 per pixel)
static_assert(HSLOTS % 64 == 0 && WSLOTS % 64 == 0, "whole wave-loads");
static_assert(CWAVES * 64 * EP <= SLOTS * 8, "epilogue fits one stage");
}  // namespace cva

__device__ __forceinline__ uint32_t swz_slot(uint32_t row, uint32_t q)
{
    return row * 4 + (q ^ ((row >> 1) & 3u));
}

__global__ void __launch_bounds__(cva::WAVES * kWave) k_conv3a(ConvArgs a)
{
    using namespace cva;
    __shared__ __attribute__((aligned(16))) uint16_t st[2][SLOTS * 8];
    const int lane = __lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int g = lane >> 4, l16 = lane & 15;
    const bool loader = wv == CWAVES;
    const uint32_t xtiles = (a.W + TX - 1) / TX, ytiles = (a.H + R - 1) / R;
    const uint32_t n_tiles = a.N * ytiles * xtiles, G = gridDim.x, b = blockIdx.x;
    if (b >= n_tiles) return;   // whole workgroup
    const uint32_t co0 = blockIdx.y * TN;
    const uint32_t Cin = a.Cin, K = 9 * Cin, nc = Cin >> 5;
    const uint32_t U = ((n_tiles - 1 - b) / G + 1) * nc;   // (tile, chunk) units of this workgroup
    const uint32_t row_b = a.W * a.in_cs * 2;
    struct Geo {
        uint32_t n, y0, x0;
    };
    auto geo = [&](uint32_t u) {
        // divisions run on the vector unit: the results go back to scalars
        const uint32_t t = b + __builtin_amdgcn_readfirstlane(u / nc) * G;
        Geo q;
        q.n = __builtin_amdgcn_readfirstlane(t / (xtiles * ytiles));
        const uint32_t rem = t - q.n * (xtiles * ytiles);
        const uint32_t ty = __builtin_amdgcn_readfirstlane(rem / xtiles);
        q.y0 = ty * R;
        q.x0 = (rem - ty * xtiles) * TX;
        return q;
    };
    const bool pool = a.pool != nullptr;
    // Barriers are plain s_barrier, the same sequence on both sides: one per
    // unit (its stage is loaded, and every wave is done with the previous
    // unit), plus one at the end of each tile (every wave is done reading the
    // stage the epilogue reuses) and one more with the pool (the epilogue
    // rows are written).
    if (loader) {
        // Unit u (tile u / nc, chunk u % nc) into stage u % 2. Wave-load j < HINSTR fills
        // slots 64 j + i with halo row j / 4, pixel 16 (j % 4) + i / 4, chunk
        // position i % 4; wave-load HINSTR + m the weight rows of tap m / 4,
        // channels 16 (m % 4) + i / 4, the same way.
        const __amdgpu_buffer_rsrc_t wrs = rsrc(a.wt, a.Cout * K * 2);
        uint32_t wcol[4];   // this lane's weight offsets per m % 4 (tap 0, chunk 0)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t co = (uint32_t)(16 * m) + ((uint32_t)lane >> 2);
            const uint32_t qq = ((uint32_t)lane & 3u) ^ (((uint32_t)lane >> 3) & 3u);
            wcol[m] = ((co0 + co) * K) * 2 + qq * 16;
        }
        uint32_t col[4];   // this lane's halo column offsets per j % 4 (chunk 0), kOob outside
        __amdgpu_buffer_rsrc_t ir = wrs;
        uint32_t r_first = 0;
        Geo q{0, 0, 0};
        auto issue = [&](uint32_t u) {
            const uint32_t c = __builtin_amdgcn_readfirstlane(u % nc);
            if (c == 0) {
                q = geo(u);
                r_first = q.y0 >= 1 ? q.y0 - 1 : 0;
                const uint32_t r_last = q.y0 + R < a.H ? q.y0 + R : a.H - 1;
                ir = srsrc(a.in + ((size_t)q.n * a.H + r_first) * a.W * a.in_cs, (r_last - r_first + 1) * row_b);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t px = 16 * k + ((uint32_t)lane >> 2);
                    const uint32_t qq = ((uint32_t)lane & 3u) ^ ((px >> 1) & 3u);
                    const int xs = (int)(q.x0 + px) - 1;
                    col[k] = (xs >= 0 && xs < (int)a.W) ? (uint32_t)xs * a.in_cs * 2 + qq * 16 : kOob;
                }
            }
            uint16_t* stg = st[u & 1];
#pragma unroll
            for (int j = 0; j < HINSTR; ++j) {
                const int ys = (int)q.y0 + (j >> 2) - 1;
                const bool rok = ys >= 0 && ys < (int)a.H;
                const uint32_t off =
                    (rok && col[j & 3] != kOob) ? ((uint32_t)ys - r_first) * row_b + col[j & 3] + c * 64 : kOob;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ir, (__attribute__((address_space(3))) void*)(stg + j * 512),
                                                         16, off, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < WINSTR; ++m)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    wrs, (__attribute__((address_space(3))) void*)(stg + (HINSTR + m) * 512), 16,
                    wcol[m & 3] + (uint32_t)(m >> 2) * Cin * 2 + c * 64, 0, 0, 0);
        };
        issue(0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        for (uint32_t u = 0; u < U; ++u) {
            asm volatile("s_barrier" ::: "memory");   // unit u staged; unit u - 1 done
            if (u + 1 < U) issue(u + 1);              // into the stage unit u - 1 left
            if ((u + 1) % nc == 0) {
                asm volatile("s_barrier" ::: "memory");
                if (pool) asm volatile("s_barrier" ::: "memory");
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        return;
    }
    float bv[NW];
    tile_bias<NW>(bv, a.bias, co0, a.Cout);
    floatx4 acc[4][NW];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // Byte offsets of the operands within a stage: pixel block i of tap
    // (dy, dx) at abase[dx] + 4096 dy + 1024 i (halo row (wv + dy) HP + 16 i
    // + l16 + dx, whose swizzle depends on l16 + dx alone), the weights of
    // column block j of tap t at bbase + 4096 t + 1024 j; the constants go
    // into the LDS instructions' offset field.
    static_assert(HP == 64 && TN == 64, "row strides of 4096 bytes");
    uint32_t abase[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
        abase[dx] = swz_slot((uint32_t)(wv * HP + l16 + dx), (uint32_t)g) * 16;
    const uint32_t bbase = HSLOTS * 16 + swz_slot((uint32_t)l16, (uint32_t)g) * 16;
    auto compute = [&](const uint16_t* stg) {
        const char* sb = (const char*)stg;
        u32x4 av[2][4], bw[2][NW];
        auto rd = [&](int tap, u32x4 (&A)[4], u32x4 (&B)[NW]) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) A[i] = *(const u32x4*)(sb + abase[dx] + (dy * 4096 + i * 1024));
#pragma unroll
            for (int j = 0; j < NW; ++j) B[j] = *(const u32x4*)(sb + bbase + (tap * 4096 + j * 1024));
        };
        rd(0, av[0], bw[0]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int cur = tap & 1;
            if (tap + 1 < 9) rd(tap + 1, av[cur ^ 1], bw[cur ^ 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[cur][i]), __builtin_bit_cast(bf16x8, bw[cur][j]), acc[i][j], 0, 0,
                        0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    for (uint32_t u = 0; u < U; ++u) {
        // unit u staged (the loading wave waited); this wave's reads of the
        // stage the next unit goes to are done
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        uint16_t* stg = st[u & 1];
        compute(stg);
        if ((u + 1) % nc != 0) continue;
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // the epilogue reuses this stage
        const Geo q = geo(u);
        const uint32_t y = q.y0 + (uint32_t)wv;
        uint16_t* ep = stg + wv * 64 * EP;
        // the lane index made opaque here: otherwise the compiler keeps the
        // epilogue's per-lane addresses live across the whole loop
        int ln = lane;
        asm volatile("" : "+v"(ln));
        store_tile<4, NW>(
            ep, acc, bv, co0, a.Cout, a.relu != 0,
            [&](int px) -> uint16_t* {
                const uint32_t x = q.x0 + (uint32_t)px;
                if (px >= TX || y >= a.H || x >= a.W) return nullptr;
                return a.out + (((size_t)q.n * a.H + y) * a.W + x) * a.out_cs + co0;
            },
            ln);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (!pool) continue;
        // 2x2 max pool (even H and W) from the waves' epilogue rows: one
        // thread per pooled pixel and 8 channels
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        constexpr int PCH = TN / 8, RUNS = (TX / 2) * (R / 2) * PCH;
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        for (uint32_t run = tid; run < (uint32_t)RUNS; run += CWAVES * kWave) {
            const uint32_t c8 = run % PCH, p2 = (run / PCH) % (TX / 2), pr = run / (PCH * (TX / 2));
            const uint32_t xs = q.x0 + 2 * p2, ys = q.y0 + 2 * pr;
            if (xs >= a.W || ys >= a.H || co0 + 8 * c8 >= a.Cout) continue;
            u32x4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t r = 2 * pr + (k >> 1), px = 2 * p2 + (k & 1);
                v[k] = *(const u32x4*)&stg[r * 64 * EP + px * EP + 8 * c8];
            }
            *(u32x4*)(a.pool + (((size_t)q.n * (a.H / 2) + ys / 2) * (a.W / 2) + xs / 2) * a.pool_cs + co0 +
                      8 * c8) = max4_bf16(v);
        }
    }
}

// Full-size 3x3 layers with 32 output channels and 32 or 64 input channels
// (the first and last levels of the network, where the input dominates the
// traffic): persistent workgroups of 8 computing waves and 1 loading wave.
// A tile is 8 rows x 62 pixels x 32 channels (one row per computing wave,
// 4 x 2 MFMA tiles per tap), read as 10 halo rows of 64 pixels. The weights
// of every chunk stay in LDS for the whole launch; the halo of each (tile,
// 32-channel chunk) unit goes into one of three LDS stages by direct
// buffer-to-LDS loads, issued two units ahead by the loading wave alone, so
// that its load counter orders nothing but those loads. Rows are 64 bytes
// with the swizzle of k_conv3a; sums run over chunks, then taps, as in
// k_conv3, so results are the same. The epilogue of a tile (and its pool or
// head) uses the tile's own stage once every wave has left it.
namespace cvr {
constexpr int R = 8, TX = 62, HP = TX + 2, RP = R + 2, TN = 32, NW = 2, S = 3, MAXC = 2;
constexpr int HSLOTS = RP * HP * 4;   // 16-byte slots of one unit's halo
constexpr int HINSTR = HSLOTS / 64;   // wave-loads per unit
constexpr int WSLOTS = 9 * TN * 4;    // slots of one chunk's weights
constexpr int WINSTR = WSLOTS / 64;
constexpr int CWAVES = 8, WAVES = CWAVES + 1;
constexpr int EP = 16 * NW + 8;
constexpr int LDS_ELEMS = (S * HSLOTS + MAXC * WSLOTS) * 8;
static_assert(HSLOTS % 64 == 0 && WSLOTS % 64 == 0, "whole wave-loads");
static_assert(CWAVES * 64 * EP <= HSLOTS * 8, "epilogue fits one stage");
static_assert(HINSTR == 40, "the loading wave's wait below allows one unit's loads in flight");
}  // namespace cvr

template <bool kHead>
__global__ void __launch_bounds__(cvr::WAVES * kWave) k_conv3r(ConvArgs a)
{
    using namespace cvr;
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_ELEMS];
    __shared__ float hws[kHead ? 99 : 1];   // the head's weights, then its bias
    uint16_t* const wts = lds + S * HSLOTS * 8;
    // the wave index as a scalar, so that the loading wave's branches and
    // its buffer resources stay scalar
    const int lane = __lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int g = lane >> 4, l16 = lane & 15;
    const bool loader = wv == CWAVES;
    const uint32_t xtiles = (a.W + TX - 1) / TX, ytiles = (a.H + R - 1) / R;
    const uint32_t n_tiles = a.N * ytiles * xtiles, G = gridDim.x, b = blockIdx.x;
    if (b >= n_tiles) return;   // whole workgroup
    const uint32_t Cin = a.Cin, K = 9 * Cin, nc = kHead ? 1 : Cin >> 5;   // the head follows 32 channels
    const uint32_t U = ((n_tiles - 1 - b) / G + 1) * nc;   // units of this workgroup
    const uint32_t row_b = a.W * a.in_cs * 2;
    struct Geo {
        uint32_t n, y0, x0;
    };
    auto geo = [&](uint32_t u) {
        const uint32_t t = b + __builtin_amdgcn_readfirstlane(u / nc) * G;
        Geo q;
        // divisions run on the vector unit: bring the results back to
        // scalars, or every buffer load would be wrapped in a uniformity loop
        q.n = __builtin_amdgcn_readfirstlane(t / (xtiles * ytiles));
        const uint32_t rem = t - q.n * (xtiles * ytiles);
        const uint32_t ty = __builtin_amdgcn_readfirstlane(rem / xtiles);
        q.y0 = ty * R;
        q.x0 = (rem - ty * xtiles) * TX;
        return q;
    };
    // loading wave: the halo of unit u into stage u % S; lane i of wave-load
    // j fills slot 64 j + i, halo row j / 4, pixel 16 (j % 4) + i / 4
    auto issue = [&](uint32_t u) {
        const Geo q = geo(u);
        const uint32_t c = __builtin_amdgcn_readfirstlane(u % nc);
        const uint32_t r_first = q.y0 >= 1 ? q.y0 - 1 : 0;
        const uint32_t r_last = q.y0 + R < a.H ? q.y0 + R : a.H - 1;
        const __amdgpu_buffer_rsrc_t ir =
            srsrc(a.in + ((size_t)q.n * a.H + r_first) * a.W * a.in_cs, (r_last - r_first + 1) * row_b);
        uint32_t col[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t px = 16 * k + (lane >> 2), qq = (uint32_t)(lane & 3) ^ ((px >> 1) & 3u);
            const int xs = (int)(q.x0 + px) - 1;
            col[k] = (xs >= 0 && xs < (int)a.W) ? (uint32_t)xs * a.in_cs * 2 + qq * 16 + c * 64 : kOob;
        }
        uint16_t* stg = lds + (u % S) * HSLOTS * 8;
#pragma unroll
        for (int j = 0; j < HINSTR; ++j) {
            const int ys = (int)q.y0 + (j >> 2) - 1;
            const bool rok = ys >= 0 && ys < (int)a.H;
            const uint32_t off = (rok && col[j & 3] != kOob) ? ((uint32_t)ys - r_first) * row_b + col[j & 3] : kOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ir, (__attribute__((address_space(3))) void*)(stg + j * 512),
                                                     16, off, 0, 0, 0);
        }
    };
    // Barriers are plain s_barrier: __syncthreads would make the loading
    // wave wait for all its loads (they write LDS) at every barrier. Each
    // side waits for what the other needs: the loading wave for its loads,
    // the computing waves for their LDS accesses. Both sides pass the same
    // sequence of barriers: one per unit, plus one (two with the pool) at
    // the end of each tile.
    const bool pool = !kHead && a.pool != nullptr;
    if (loader) {
        // the weights of every chunk, [chunk][tap][channel] rows, then the
        // first two units
        const __amdgpu_buffer_rsrc_t wrs = rsrc(a.wt, a.Cout * K * 2);
        for (uint32_t jj = 0; jj < nc * WINSTR; ++jj) {
            const uint32_t c = jj / WINSTR, j = jj % WINSTR, s3 = j * 64 + (uint32_t)lane;
            const uint32_t wrow = s3 >> 2, qq = (s3 & 3u) ^ ((wrow >> 1) & 3u);
            const uint32_t tap = wrow / TN, co = wrow % TN;
            const uint32_t off = co < a.Cout ? (co * K + tap * Cin + c * 32) * 2 + qq * 16 : kOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                wrs, (__attribute__((address_space(3))) void*)(wts + (c * WSLOTS + j * 64) * 8), 16, off, 0, 0, 0);
        }
        issue(0);
        if (U > 1) issue(1);
        for (uint32_t u = 0; u < U; ++u) {
            // unit u has landed once at most the next unit's loads are in flight
            if (u + 1 < U)
                asm volatile("s_waitcnt vmcnt(40)\n\ts_barrier" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
            if (u + 2 < U) issue(u + 2);   // into the stage that unit u - 1 left
            if ((u + 1) % nc != 0) continue;
            asm volatile("s_barrier" ::: "memory");
            if (pool) asm volatile("s_barrier" ::: "memory");
        }
        return;
    }
    floatx4 acc[4][NW];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // operand byte offsets as in k_conv3a: pixel block i of tap (dy, dx) at
    // abase[dx] + 4096 dy + 1024 i into a stage, the weights of column block
    // j, tap t at bbase + 2048 t + 1024 j into a chunk's weights
    static_assert(HP == 64 && TN == 32, "row strides of 4096 and 2048 bytes");
    uint32_t abase[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) abase[dx] = swz_slot((uint32_t)(wv * HP + l16 + dx), (uint32_t)g) * 16;
    const uint32_t bbase = swz_slot((uint32_t)l16, (uint32_t)g) * 16;
    auto compute = [&](const uint16_t* stg, const uint16_t* wc) {
        const char* sb = (const char*)stg;
        const char* wb = (const char*)wc;
        u32x4 av[2][4], bv[2][NW];
        auto rd = [&](int tap, u32x4 (&A)[4], u32x4 (&B)[NW]) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) A[i] = *(const u32x4*)(sb + abase[dx] + (dy * 4096 + i * 1024));
#pragma unroll
            for (int j = 0; j < NW; ++j) B[j] = *(const u32x4*)(wb + bbase + (tap * 2048 + j * 1024));
        };
        rd(0, av[0], bv[0]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int cur = tap & 1;
            if (tap + 1 < 9) rd(tap + 1, av[cur ^ 1], bv[cur ^ 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[cur][i]), __builtin_bit_cast(bf16x8, bv[cur][j]), acc[i][j], 0, 0,
                        0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (kHead && wv == 0) {   // visible to all after the first barrier
        hws[lane] = a.head_w[lane];
        if (lane < 32) hws[64 + lane] = a.head_w[64 + lane];
        if (lane < 3) hws[96 + lane] = a.head_b[lane];
    }
    const uint32_t y_w = (uint32_t)wv;
    float bv[NW];
    tile_bias<NW>(bv, a.bias, 0, a.Cout);
    for (uint32_t u = 0; u < U; ++u) {
        // unit u staged (the loading wave waited); this wave's reads of the
        // stage the next loads go to are done
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        uint16_t* stg = lds + (u % S) * HSLOTS * 8;
        const uint32_t c = __builtin_amdgcn_readfirstlane(u % nc);
        // the head's splat colour of this lane's pixel, loaded before the
        // tile's last products so that they hide its latency
        // (every lane loads: pixels outside the image read pixel 0)
        uint32_t sp;
        if (kHead && c + 1 == nc) {
            const Geo q = geo(u);
            const uint32_t y = q.y0 + y_w, x = q.x0 + (uint32_t)lane;
            const bool in = lane < TX && y < a.H && x < a.W;
            sp = a.head_rgba[in ? ((size_t)q.n * a.H + y) * a.W + x : 0];
        }
        compute(stg, wts + c * WSLOTS * 8);
        if (c + 1 < nc) continue;
        if (kHead) asm volatile("" : "+v"(sp));   // the load has landed on every path here
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // every wave done with the halo
        const Geo q = geo(u);
        const uint32_t y = q.y0 + y_w;
        uint16_t* ep = stg + wv * 64 * EP;
        int ln = lane;
        asm volatile("" : "+v"(ln));   // keeps the epilogue's per-lane addresses out of the loop
        store_tile<4, NW>(
            ep, acc, bv, 0, a.Cout, a.relu != 0,
            [&](int px) -> uint16_t* {
                const uint32_t x = q.x0 + (uint32_t)px;
                if (kHead || px >= TX || y >= a.H || x >= a.W) return nullptr;
                return a.out + (((size_t)q.n * a.H + y) * a.W + x) * a.out_cs;
            },
            ln);
        if (kHead) {
            const uint32_t x = q.x0 + (uint32_t)lane;
            if (lane < TX && y < a.H && x < a.W)
                head_pixel(a, hws, ep + lane * EP, ((size_t)q.n * a.H + y) * a.W + x, sp);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (!pool) continue;
        // 2x2 max pool (even H and W) from the waves' epilogue rows
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        constexpr int PCH = TN / 8, RUNS = (TX / 2) * (R / 2) * PCH;
        static_assert(RUNS <= CWAVES * kWave, "one pass over the pooled runs");
        const uint32_t run = threadIdx.x;
        if (run < (uint32_t)RUNS) {
            const uint32_t c8 = run % PCH, p2 = (run / PCH) % (TX / 2), pr = run / (PCH * (TX / 2));
            const uint32_t xs = q.x0 + 2 * p2, ys = q.y0 + 2 * pr;
            if (xs < a.W && ys < a.H) {
                u32x4 v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t r = 2 * pr + (k >> 1), px = 2 * p2 + (k & 1);
                    v[k] = *(const u32x4*)&stg[r * 64 * EP + px * EP + 8 * c8];
                }
                *(u32x4*)(a.pool + (((size_t)q.n * (a.H / 2) + ys / 2) * (a.W / 2) + xs / 2) * a.pool_cs + 8 * c8) =
                    max4_bf16(v);
            }
        }
    }
}

// The first encoder level in inference: both of its 3x3 convolutions (the
// 8-channel input to 32 channels, then 32 to 32 with the 2x2 max pool) in
// one kernel, so that the first convolution's full-size output never goes
// to memory. Persistent workgroups of 8 computing waves and 1 loading wave,
// tiles of 8 rows x 62 pixels as in k_conv3r. The loading wave stages each
// tile's input halo (12 rows x 66 pixels x 8 channels, zero outside the
// image) by direct buffer-to-LDS loads, two tiles ahead into a three-stage
// ring. The computing waves run the first convolution over the second one's
// halo (10 rows x 64 pixels; zero where it falls outside the image, which
// is the second convolution's padding) into LDS in k_conv3r's swizzled
// layout, then the second convolution from there. The first convolution's
// products are transposed (weights as the row operand, pixels as the column
// operand), so that a lane ends with 4 consecutive channels of one pixel
// and writes them as one 8-byte word; its K chunks are k_conv's (four taps
// of 8 channels, lane group g taking tap 4 c + g, the chunks in order), so
// both layers sum exactly as the unfused kernels do and the results are
// the same.
namespace cv2 {
constexpr int R = 8, TX = 62, HP = TX + 2, RP = R + 2, IR = R + 4, IP = TX + 4, S = 3;
constexpr int ISLOTS = (IR * IP + 63) / 64 * 64;   // 16-byte slots of one input halo
constexpr int IINSTR = ISLOTS / 64;                // wave-loads per tile
constexpr int HSLOTS = RP * HP * 4;                // the first convolution's output halo
constexpr int WSLOTS = 9 * 32 * 4;                 // the second convolution's weights
constexpr int WINSTR = WSLOTS / 64;
constexpr int CWAVES = 8, WAVES = CWAVES + 1;
constexpr int EP = 16 * 2 + 8;
constexpr int BLOCKS = RP * (HP / 16);             // 16-pixel blocks of the output halo
constexpr int BPW = BLOCKS / CWAVES;               // blocks per computing wave
constexpr int W1SLOTS = 3 * 2 * 64;                // first convolution's weights, one slot per lane and operand
// then the first convolution's bias: 64 floats, one per lane of its load
constexpr int LDS_ELEMS = (2 * HSLOTS + S * ISLOTS + WSLOTS + W1SLOTS) * 8 + 64 * 2;
static_assert(IINSTR == 13, "the loading wave's wait below allows one tile's loads in flight");
static_assert(BLOCKS % CWAVES == 0, "whole blocks per wave");
static_assert(CWAVES * 64 * EP <= HSLOTS * 8, "epilogue rows fit the output halo");
}  // namespace cv2

struct Conv2Args {
    const uint16_t* in;   // 8-channel input (first channel), in_cs elements per pixel
    const uint16_t* w1;   // first convolution [32][9 * 8] bf16
    const float* b1;      // [32]
    const uint16_t* w2;   // second convolution [32][9 * 32] bf16
    const float* b2;      // [32]
    uint16_t* out;        // the second convolution's output (first channel)
    uint16_t* pool;       // its 2x2 max pool (first channel)
    uint32_t in_cs, out_cs, pool_cs, N, H, W;
};

__global__ void __launch_bounds__(cv2::WAVES * kWave) k_conv33(Conv2Args a)
{
    using namespace cv2;
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_ELEMS];
    // the two output halos come first: the second convolution's reads past
    // the end of one (the two unstored pixels of the last row) stay inside
    // the array
    uint16_t* const ist = lds + 2 * HSLOTS * 8;
    uint16_t* const wts = lds + (2 * HSLOTS + S * ISLOTS) * 8;
    uint16_t* const w1s = wts + WSLOTS * 8;
    const float* const b1s = (const float*)(w1s + W1SLOTS * 8);
    const int lane = __lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int g = lane >> 4, l16 = lane & 15;
    const bool loader = wv == CWAVES;
    const uint32_t xtiles = (a.W + TX - 1) / TX, ytiles = (a.H + R - 1) / R;
    const uint32_t n_tiles = a.N * ytiles * xtiles, G = gridDim.x, b = blockIdx.x;
    if (b >= n_tiles) return;   // whole workgroup
    const uint32_t U = (n_tiles - 1 - b) / G + 1;   // tiles of this workgroup
    const uint32_t row_b = a.W * a.in_cs * 2;
    struct Geo {
        uint32_t n, y0, x0;
    };
    auto geo = [&](uint32_t u) {
        const uint32_t t = b + u * G;
        Geo q;
        q.n = __builtin_amdgcn_readfirstlane(t / (xtiles * ytiles));
        const uint32_t rem = t - q.n * (xtiles * ytiles);
        const uint32_t ty = __builtin_amdgcn_readfirstlane(rem / xtiles);
        q.y0 = ty * R;
        q.x0 = (rem - ty * xtiles) * TX;
        return q;
    };
    // loading wave: the input halo of tile u into stage u % S; lane i of
    // wave-load j fills slot 64 j + i, halo pixel (s / IP, s % IP)
    auto issue = [&](uint32_t u) {
        const Geo q = geo(u);
        const int r_first = q.y0 >= 2 ? (int)q.y0 - 2 : 0;
        const int r_last = q.y0 + R + 1 < a.H ? (int)q.y0 + R + 1 : (int)a.H - 1;
        const __amdgpu_buffer_rsrc_t ir = srsrc(a.in + ((size_t)q.n * a.H + (uint32_t)r_first) * a.W * a.in_cs,
                                                (uint32_t)(r_last - r_first + 1) * row_b);
        uint16_t* stg = ist + (u % S) * ISLOTS * 8;
#pragma unroll
        for (int j = 0; j < IINSTR; ++j) {
            const uint32_t s = (uint32_t)(j * 64 + lane), hr = s / IP, hp = s % IP;
            const int ys = (int)q.y0 - 2 + (int)hr, xs = (int)q.x0 - 2 + (int)hp;
            const bool ok = s < (uint32_t)(IR * IP) && ys >= 0 && ys < (int)a.H && xs >= 0 && xs < (int)a.W;
            const uint32_t off = ok ? (uint32_t)(ys - r_first) * row_b + (uint32_t)xs * a.in_cs * 2 : kOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ir, (__attribute__((address_space(3))) void*)(stg + j * 512),
                                                     16, off, 0, 0, 0);
        }
    };
    // Barriers are plain s_barrier, the same sequence on both sides: one
    // before the pipeline starts (tile 0 staged), then three per tile (the
    // tile's output halo written and the next tile's input staged; the
    // tile's output halo read; its epilogue rows written). Tile u's second
    // convolution and tile u + 1's first run in the same phase, on the two
    // output halos in turn.
    if (loader) {
        // the second convolution's weights, [tap][channel] rows
        const __amdgpu_buffer_rsrc_t wrs = rsrc(a.w2, 32 * 9 * 32 * 2);
        for (uint32_t j = 0; j < (uint32_t)WINSTR; ++j) {
            const uint32_t s3 = j * 64 + (uint32_t)lane;
            const uint32_t wrow = s3 >> 2, qq = (s3 & 3u) ^ ((wrow >> 1) & 3u);
            const uint32_t tap = wrow / 32, co = wrow % 32;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, (__attribute__((address_space(3))) void*)(wts + j * 512), 16,
                                                     (co * 9 * 32 + tap * 32) * 2 + qq * 16, 0, 0, 0);
        }
        // the first convolution's weights as the products' row operands:
        // slot 64 (2 c + j) + lane holds, for lane (g, l16), output channel
        // 16 j + l16, K entries 32 c + 8 g .. 32 c + 8 g + 7 (tap 4 c + g;
        // zeros past the ninth tap); then its bias
        const __amdgpu_buffer_rsrc_t w1rs = rsrc(a.w1, 32 * 9 * 8 * 2);
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
            const int c = jj >> 1, j = jj & 1, tap = 4 * c + (lane >> 4);
            const uint32_t off = tap < 9 ? ((16 * j + (lane & 15)) * 72 + 8 * tap) * 2 : kOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(w1rs, (__attribute__((address_space(3))) void*)(w1s + jj * 512), 16,
                                                     off, 0, 0, 0);
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc(a.b1, 32 * 4), (__attribute__((address_space(3))) void*)b1s, 4,
                                                 lane < 32 ? (uint32_t)lane * 4 : kOob, 0, 0, 0);
        issue(0);
        if (U > 1) issue(1);
        // tile 0 has landed once at most tile 1's loads are in flight
        if (U > 1)
            asm volatile("s_waitcnt vmcnt(13)\n\ts_barrier" ::: "memory");
        else
            asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
        if (U > 2) issue(2);
        for (uint32_t u = 0; u < U; ++u) {
            // tile u + 1 (read in this tile's phase) has landed once at most
            // tile u + 2's loads are in flight
            if (u + 2 < U)
                asm volatile("s_waitcnt vmcnt(13)\n\ts_barrier" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
            if (u + 3 < U) issue(u + 3);   // into tile u's stage, read before this barrier
            asm volatile("s_barrier\n\ts_barrier" ::: "memory");
        }
        return;
    }
    float bv[2];
    tile_bias<2>(bv, a.b2, 0, 32);
    // the first convolution's weights as row operands (slot 64 (2 c + j) +
    // lane of w1s), held in registers once they have landed
    u32x4 w1r[2][3];
    floatx4 acc[4][2];
    // second-convolution operand byte offsets as in k_conv3a: pixel block i
    // of tap (dy, dx) at abase[dx] + 4096 dy + 1024 i into the output halo,
    // the weights of column block j, tap t at bbase + 2048 t + 1024 j
    static_assert(HP == 64, "row stride of 4096 bytes");
    uint32_t abase[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) abase[dx] = swz_slot((uint32_t)(wv * HP + l16 + dx), (uint32_t)g) * 16;
    const uint32_t bbase = (2 * HSLOTS + S * ISLOTS) * 16 + swz_slot((uint32_t)l16, (uint32_t)g) * 16;
    const char* const lb = (const char*)lds;
    auto compute2 = [&](int hb) {
        const uint32_t hoff = (uint32_t)hb * HSLOTS * 16;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        u32x4 av[2][4], bw[2][2];
        auto rd = [&](int tap, u32x4 (&A)[4], u32x4 (&B)[2]) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) A[i] = *(const u32x4*)(lb + hoff + abase[dx] + (dy * 4096 + i * 1024));
#pragma unroll
            for (int j = 0; j < 2; ++j) B[j] = *(const u32x4*)(lb + bbase + (tap * 2048 + j * 1024));
        };
        rd(0, av[0], bw[0]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int cur = tap & 1;
            if (tap + 1 < 9) rd(tap + 1, av[cur ^ 1], bw[cur ^ 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[cur][i]), __builtin_bit_cast(bf16x8, bw[cur][j]), acc[i][j], 0, 0,
                        0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // first convolution of tile u into output halo hb: blocks wv, wv + 8,
    // ... of the halo, each 16 pixels of one halo row x 32 channels. All
    // operands of the wave's blocks are read first, then all products
    // issued (ten independent accumulators), then the results written.
    auto conv1 = [&](uint32_t u, int hb) {
        const Geo q = geo(u);
        const uint16_t* in_s = ist + (u % S) * ISLOTS * 8;
        uint16_t* h1 = lds + hb * HSLOTS * 8;
        u32x4 xb[BPW][3];
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            const int blk = wv + CWAVES * k, hr = blk >> 2, hp = 16 * (blk & 3) + l16;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // past the ninth tap: read tap 8 and clear it (no branch)
                const int tap = 4 * c + g, t = tap < 9 ? tap : 8, dy = t / 3, dx = t - 3 * dy;
                const uint32_t keep = tap < 9 ? ~0u : 0u;
                xb[k][c] = *(const u32x4*)&in_s[((hr + dy) * IP + hp + dx) * 8] & keep;
            }
        }
        floatx4 d[BPW][2];
#pragma unroll
        for (int k = 0; k < BPW; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j) d[k][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < BPW; ++k)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    d[k][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w1r[j][c]),
                                                                      __builtin_bit_cast(bf16x8, xb[k][c]), d[k][j], 0,
                                                                      0, 0);
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            const int blk = wv + CWAVES * k, hr = blk >> 2, hp = 16 * (blk & 3) + l16;
            const int y = (int)q.y0 - 1 + hr, x = (int)q.x0 - 1 + hp;
            const bool in = y >= 0 && y < (int)a.H && x >= 0 && x < (int)a.W;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // bias of the 4 channels 16 j + 4 g + r this lane holds
                const floatx4 bj = *(const floatx4*)&b1s[16 * j + 4 * g];
                uint32_t w[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float v0 = d[k][j][2 * h] + bj[2 * h], v1 = d[k][j][2 * h + 1] + bj[2 * h + 1];
                    v0 = v0 > 0.0f ? v0 : 0.0f;
                    v1 = v1 > 0.0f ? v1 : 0.0f;
                    w[h] = in ? f2bf2(v0, v1) : 0u;
                }
                const uint32_t slot = swz_slot((uint32_t)(hr * HP + hp), (uint32_t)(2 * j + (g >> 1)));
                *(uint2*)&h1[slot * 8 + (g & 1) * 4] = make_uint2(w[0], w[1]);
            }
        }
    };
    // tile 0 staged; the first convolution's weights have landed with it
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 2; ++j) w1r[j][c] = *(const u32x4*)&w1s[((2 * c + j) * 64 + lane) * 8];
    conv1(0, 0);
    for (uint32_t u = 0; u < U; ++u) {
        // tile u's output halo complete, tile u + 1 staged; the previous
        // tile's pool reads of the other output halo are done
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        const int hb = (int)(u & 1);
        if (u + 1 < U) conv1(u + 1, hb ^ 1);
        compute2(hb);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // every wave done with tile u's halo
        const Geo q = geo(u);
        uint16_t* h1 = lds + hb * HSLOTS * 8;
        const uint32_t y = q.y0 + (uint32_t)wv;
        int ln = lane;
        asm volatile("" : "+v"(ln));   // keeps the epilogue's per-lane addresses out of the loop
        store_tile<4, 2>(
            h1 + wv * 64 * EP, acc, bv, 0, 32, true,
            [&](int px) -> uint16_t* {
                const uint32_t x = q.x0 + (uint32_t)px;
                if (px >= TX || y >= a.H || x >= a.W) return nullptr;
                return a.out + (((size_t)q.n * a.H + y) * a.W + x) * a.out_cs;
            },
            ln);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // epilogue rows complete
        // 2x2 max pool (even H and W) from the waves' epilogue rows
        constexpr int PCH = 4, RUNS = (TX / 2) * (R / 2) * PCH;
        static_assert(RUNS <= CWAVES * kWave, "one pass over the pooled runs");
        uint32_t run = threadIdx.x;
        asm volatile("" : "+v"(run));
        if (run < (uint32_t)RUNS) {
            const uint32_t c8 = run % PCH, p2 = (run / PCH) % (TX / 2), pr = run / (PCH * (TX / 2));
            const uint32_t xs = q.x0 + 2 * p2, ys = q.y0 + 2 * pr;
            if (xs < a.W && ys < a.H) {
                u32x4 v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t r = 2 * pr + (k >> 1), px = 2 * p2 + (k & 1);
                    v[k] = *(const u32x4*)&h1[r * 64 * EP + px * EP + 8 * c8];
                }
                *(u32x4*)(a.pool + (((size_t)q.n * (a.H / 2) + ys / 2) * (a.W / 2) + xs / 2) * a.pool_cs + 8 * c8) =
                    max4_bf16(v);
            }
        }
    }
}

// The decoder's last level in inference: its 2x2 stride-2 transposed
// convolution (64 to 32 channels) computed inside its first 3x3 convolution
// (over the concatenation of that output with the encoder's 32 skip
// channels, 64 to 32), so that the up-sampled half of the concatenation
// never goes to memory. Persistent workgroups of 8 computing waves and 1
// loading wave, tiles of 8 rows x 62 pixels as in k_conv3r. Per tile the
// loading wave stages the low-resolution input under the tile (6 rows x 33
// pixels x 64 channels) and the skip channels' halo (10 rows x 64 pixels);
// the computing waves compute the up-sampled channels' halo into LDS (zero
// outside the image, which is the 3x3 convolution's padding), then the 3x3
// products over it (chunk 0) and over the skip halo (chunk 1), the order in
// which the unfused kernels sum, so the results are the same. The
// transposed convolution's products are transposed (weights of one
// sub-position as the row operand, 16 low-resolution pixels as the column
// operand, which land on every other pixel of one output row), so a lane
// writes 4 channels of one pixel at once.
namespace cvu {
constexpr int R = 8, TX = 62, HP = TX + 2, RP = R + 2;
constexpr int LR = R / 2 + 2, LP = TX / 2 + 2;           // low-resolution rows and pixels under a tile
constexpr int LSLOTS = (LR * LP * 8 + 63) / 64 * 64;     // 16-byte slots, 8 per low-resolution pixel
constexpr int LINSTR = LSLOTS / 64;
constexpr int HSLOTS = RP * HP * 4;                      // one 32-channel halo
constexpr int HINSTR = HSLOTS / 64;
constexpr int WSLOTS = 2 * 9 * 32 * 4;                   // 3x3 weights, both chunks
constexpr int WINSTR = WSLOTS / 64;
constexpr int USLOTS = 16 * 64;                          // transposed-convolution weights, one slot per lane and operand
constexpr int UINSTR = USLOTS / 64;
constexpr int CWAVES = 8, WAVES = CWAVES + 1;
constexpr int EP = 16 * 2 + 8;
constexpr int ITEMS = RP * 2 * 2;                        // (halo row, column parity, 16-pixel block)
constexpr int IPW = ITEMS / CWAVES;
// LDS layout in 16-byte slots: up-sampled halo (later the epilogue rows),
// skip halo, low-resolution stage, 3x3 weights, transposed-convolution
// weights, its bias (64 floats: one per lane of its load)
constexpr int O_UP = 0, O_SK = HSLOTS, O_LR = 2 * HSLOTS, O_W = O_LR + LSLOTS, O_U = O_W + WSLOTS, O_B = O_U + USLOTS;
constexpr int LDS_ELEMS = (O_B + 16) * 8;
static_assert(LINSTR == 25 && HINSTR == 40, "the loading wave's waits below");
static_assert(ITEMS % CWAVES == 0 && IPW == 5 && CWAVES == 8, "two waves per sub-position, 5 items each");
static_assert(CWAVES * 64 * EP <= HSLOTS * 8, "epilogue rows fit the up-sampled halo");
static_assert(O_SK * 16 + 11264 < 65536 && 18432 + 8 * 2048 + 1024 < 65536, "constant LDS offsets fit");
}  // namespace cvu

struct ConvUpArgs {
    const uint16_t* low;   // decoder input at half resolution (first channel), low_cs elements per pixel
    const uint16_t* wu;    // transposed convolution [4][32][64] bf16 (sub-position 2 dy + dx)
    const float* bu;       // [32]
    const uint16_t* skip;  // the encoder's 32 skip channels (first channel), skip_cs per pixel
    const uint16_t* wt;    // 3x3 convolution [32][9 * 64] bf16 (up-sampled channels first)
    const float* bias;     // [32]
    uint16_t* out;         // output (first channel), out_cs per pixel
    uint32_t low_cs, skip_cs, out_cs, N, H, W;   // H, W: full resolution, even
};

__global__ void __launch_bounds__(cvu::WAVES * kWave) k_conv3u(ConvUpArgs a)
{
    using namespace cvu;
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_ELEMS];
    const int lane = __lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int g = lane >> 4, l16 = lane & 15;
    const bool loader = wv == CWAVES;
    const uint32_t xtiles = (a.W + TX - 1) / TX, ytiles = (a.H + R - 1) / R;
    const uint32_t n_tiles = a.N * ytiles * xtiles, G = gridDim.x, b = blockIdx.x;
    if (b >= n_tiles) return;   // whole workgroup
    const uint32_t U = (n_tiles - 1 - b) / G + 1;   // tiles of this workgroup
    const uint32_t Hl = a.H / 2, Wl = a.W / 2;
    struct Geo {
        uint32_t n, y0, x0;
    };
    auto geo = [&](uint32_t u) {
        const uint32_t t = b + u * G;
        Geo q;
        q.n = __builtin_amdgcn_readfirstlane(t / (xtiles * ytiles));
        const uint32_t rem = t - q.n * (xtiles * ytiles);
        const uint32_t ty = __builtin_amdgcn_readfirstlane(rem / xtiles);
        q.y0 = ty * R;
        q.x0 = (rem - ty * xtiles) * TX;
        return q;
    };
    auto lds_at = [&](int slot) { return (__attribute__((address_space(3))) void*)(lds + slot * 8); };
    // Barriers are plain s_barrier, four per tile on both sides: low-resolution
    // stage loaded, up-sampled halo written, skip halo loaded, products done.
    if (loader) {
        // resident: the 3x3 weights as [chunk][tap][channel] rows of 64
        // bytes (swizzled as in k_conv3r), the transposed convolution's
        // weights as row operands (slot 64 (4 sub + 2 j + c) + lane holds, for
        // lane (g, l16), channel 16 j + l16, inputs 32 c + 8 g .. 32 c + 8 g + 7),
        // then its bias
        const __amdgpu_buffer_rsrc_t wrs = rsrc(a.wt, 32 * 9 * 64 * 2);
        for (int jj = 0; jj < WINSTR; ++jj) {
            const uint32_t c = (uint32_t)jj / (WINSTR / 2), j = (uint32_t)jj % (WINSTR / 2);
            const uint32_t s3 = j * 64 + (uint32_t)lane, wrow = s3 >> 2, qq = (s3 & 3u) ^ ((wrow >> 1) & 3u);
            const uint32_t tap = wrow / 32, co = wrow % 32;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, lds_at(O_W + jj * 64), 16,
                                                     (co * 9 * 64 + tap * 64 + c * 32) * 2 + qq * 16, 0, 0, 0);
        }
        const __amdgpu_buffer_rsrc_t urs = rsrc(a.wu, 4 * 32 * 64 * 2);
        for (int m = 0; m < UINSTR; ++m) {
            const uint32_t sub = (uint32_t)m >> 2, j = ((uint32_t)m >> 1) & 1u, c = (uint32_t)m & 1u;
            const uint32_t co = 16 * j + ((uint32_t)lane & 15u);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(urs, lds_at(O_U + m * 64), 16,
                                                     ((sub * 32 + co) * 64 + 32 * c + 8 * ((uint32_t)lane >> 4)) * 2, 0,
                                                     0, 0);
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc(a.bu, 32 * 4), lds_at(O_B), 4,
                                                 lane < 32 ? (uint32_t)lane * 4 : kOob, 0, 0, 0);
        // the low-resolution pixels under tile u: slot 64 j + i holds pixel
        // (s / 8) / LP, (s / 8) % LP of the stage (from the low-resolution
        // pixel one above and left of the tile's), channel chunk
        // (s % 8) ^ (pixel % 8) (s = 64 j + i)
        auto issue_lr = [&](uint32_t u) {
            const Geo q = geo(u);
            const int ly0 = (int)q.y0 / 2 - 1, lx0 = (int)q.x0 / 2 - 1;
            const int r_first = ly0 >= 0 ? ly0 : 0;
            const int r_last = ly0 + LR - 1 < (int)Hl ? ly0 + LR - 1 : (int)Hl - 1;
            const uint32_t row_b = Wl * a.low_cs * 2;
            const __amdgpu_buffer_rsrc_t ir = srsrc(a.low + ((size_t)q.n * Hl + (uint32_t)r_first) * Wl * a.low_cs,
                                                    (uint32_t)(r_last - r_first + 1) * row_b);
#pragma unroll
            for (int j = 0; j < LINSTR; ++j) {
                const uint32_t s = (uint32_t)(j * 64 + lane), pi = s >> 3, lr = pi / LP, lp = pi % LP;
                const uint32_t qq = (s & 7u) ^ (lp & 7u);
                const int ly = ly0 + (int)lr, lx = lx0 + (int)lp;
                const bool ok = pi < (uint32_t)(LR * LP) && ly >= 0 && ly < (int)Hl && lx >= 0 && lx < (int)Wl;
                const uint32_t off = ok ? (uint32_t)(ly - r_first) * row_b + (uint32_t)lx * a.low_cs * 2 + qq * 16 : kOob;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ir, lds_at(O_LR + j * 64), 16, off, 0, 0, 0);
            }
        };
        // the skip channels' halo of tile u, laid out as k_conv3r's halo
        auto issue_sk = [&](uint32_t u) {
            const Geo q = geo(u);
            const uint32_t r_first = q.y0 >= 1 ? q.y0 - 1 : 0;
            const uint32_t r_last = q.y0 + R < a.H ? q.y0 + R : a.H - 1;
            const uint32_t row_b = a.W * a.skip_cs * 2;
            const __amdgpu_buffer_rsrc_t ir =
                srsrc(a.skip + ((size_t)q.n * a.H + r_first) * a.W * a.skip_cs, (r_last - r_first + 1) * row_b);
            uint32_t col[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t px = 16 * k + ((uint32_t)lane >> 2), qq = ((uint32_t)lane & 3u) ^ ((px >> 1) & 3u);
                const int xs = (int)(q.x0 + px) - 1;
                col[k] = (xs >= 0 && xs < (int)a.W) ? (uint32_t)xs * a.skip_cs * 2 + qq * 16 : kOob;
            }
#pragma unroll
            for (int j = 0; j < HINSTR; ++j) {
                const int ys = (int)q.y0 + (j >> 2) - 1;
                const bool rok = ys >= 0 && ys < (int)a.H;
                const uint32_t off = (rok && col[j & 3] != kOob) ? ((uint32_t)ys - r_first) * row_b + col[j & 3] : kOob;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ir, lds_at(O_SK + j * 64), 16, off, 0, 0, 0);
            }
        };
        issue_lr(0);
        issue_sk(0);
        for (uint32_t u = 0; u < U; ++u) {
            // the low-resolution stage of tile u has landed once at most the
            // skip halo's loads are in flight
            asm volatile("s_waitcnt vmcnt(40)\n\ts_barrier" ::: "memory");
            asm volatile("s_barrier" ::: "memory");   // up-sampled halo written: the stage is free
            if (u + 1 < U) {
                issue_lr(u + 1);
                asm volatile("s_waitcnt vmcnt(25)\n\ts_barrier" ::: "memory");   // skip halo landed
            } else {
                asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
            }
            asm volatile("s_barrier" ::: "memory");   // products done: the skip halo is free
            if (u + 1 < U) issue_sk(u + 1);
        }
        return;
    }
    float bv[2];
    tile_bias<2>(bv, a.bias, 0, 32);
    floatx4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // 3x3 operands as in k_conv3a: pixel block i of tap (dy, dx) at
    // abase[dx] + 4096 dy + 1024 i bytes into a halo, the weights of column
    // block j, tap t, chunk c at bbase + 18432 c + 2048 t + 1024 j
    uint32_t abase[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) abase[dx] = swz_slot((uint32_t)(wv * HP + l16 + dx), (uint32_t)g) * 16;
    const uint32_t bbase = O_W * 16 + swz_slot((uint32_t)l16, (uint32_t)g) * 16;
    const char* const lb = (const char*)lds;
    auto compute = [&](int halo, int c) {
        u32x4 av[2][4], bw[2][2];
        auto rd = [&](int tap, u32x4 (&A)[4], u32x4 (&B)[2]) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) A[i] = *(const u32x4*)(lb + abase[dx] + (halo * 16 + dy * 4096 + i * 1024));
#pragma unroll
            for (int j = 0; j < 2; ++j) B[j] = *(const u32x4*)(lb + bbase + (c * 18432 + tap * 2048 + j * 1024));
        };
        rd(0, av[0], bw[0]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int cur = tap & 1;
            if (tap + 1 < 9) rd(tap + 1, av[cur ^ 1], bw[cur ^ 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[cur][i]), __builtin_bit_cast(bf16x8, bw[cur][j]), acc[i][j], 0, 0,
                        0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    const float* const bus = (const float*)(lds + O_B * 8);
    // this wave's sub-position of the transposed convolution and its
    // weights as row operands (read from LDS once they have landed)
    const int sub = wv >> 1, sy = sub >> 1, sx = sub & 1;
    u32x4 wup[2][2];
    for (uint32_t u = 0; u < U; ++u) {
        // low-resolution stage of tile u loaded; the previous tile's
        // epilogue reads of the up-sampled halo are done
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        const Geo q = geo(u);
        // up-sampled halo: wave wv computes sub-position sub (rows of parity
        // sy, pixels of column parity sx) for 5 of its 10 (row, 16-pixel
        // block) items; halo pixel x0 - 1 + hp has column parity sx when hp
        // has parity 1 - sx (x0 is even), halo row hr row parity sy when hr
        // has parity 1 - sy
        if (u == 0) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    wup[j][c] = *(const u32x4*)(lb + (O_U + (4 * sub + 2 * j + c) * 64 + lane) * 16);
        }
        auto rd1 = [&](int k, u32x4 (&xb)[2]) {
            const int m = 5 * (wv & 1) + k, hr = 2 * (m >> 1) + 1 - sy, blk = m & 1;
            const int lr = (hr + 1 - sy) >> 1, lp = 16 * blk + l16 + 1 - sx;
#pragma unroll
            for (int c = 0; c < 2; ++c)
                xb[c] = *(const u32x4*)(lb + (O_LR + (lr * LP + lp) * 8 + ((4 * c + g) ^ (lp & 7))) * 16);
        };
        // all five items' operands read first, then their products: the
        // items are independent, so one item's products run while another's
        // results are rounded and stored (a loop over the items, each
        // waiting for its own products, left the matrix units idle)
        floatx4 bjs[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) bjs[j] = *(const floatx4*)&bus[16 * j + 4 * g];
        u32x4 xa[IPW][2];
#pragma unroll
        for (int k = 0; k < IPW; ++k) rd1(k, xa[k]);
#pragma unroll
        for (int k = 0; k < IPW; ++k) {
            const int m = 5 * (wv & 1) + k, hr = 2 * (m >> 1) + 1 - sy, blk = m & 1;
            const int hp = 2 * (16 * blk + l16) + 1 - sx;
            floatx4 d[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    d[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, wup[j][c]),
                                                                   __builtin_bit_cast(bf16x8, xa[k][c]), d[j], 0, 0, 0);
            const int y = (int)q.y0 - 1 + hr, x = (int)q.x0 - 1 + hp;
            const bool in = y >= 0 && y < (int)a.H && x >= 0 && x < (int)a.W;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                uint32_t w[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float v0 = d[j][2 * h] + bjs[j][2 * h], v1 = d[j][2 * h + 1] + bjs[j][2 * h + 1];
                    w[h] = in ? f2bf2(v0, v1) : 0u;
                }
                const uint32_t slot = O_UP + swz_slot((uint32_t)(hr * HP + hp), (uint32_t)(2 * j + (g >> 1)));
                *(uint2*)&lds[slot * 8 + (g & 1) * 4] = make_uint2(w[0], w[1]);
            }
        }
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // up-sampled halo complete
        compute(O_UP, 0);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // skip halo loaded
        compute(O_SK, 1);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // every wave done with both halos
        const uint32_t y = q.y0 + (uint32_t)wv;
        int ln = lane;
        asm volatile("" : "+v"(ln));
        store_tile<4, 2>(
            lds + O_UP * 8 + wv * 64 * EP, acc, bv, 0, 32, true,
            [&](int px) -> uint16_t* {
                const uint32_t x = q.x0 + (uint32_t)px;
                if (px >= TX || y >= a.H || x >= a.W) return nullptr;
                return a.out + (((size_t)q.n * a.H + y) * a.W + x) * a.out_cs;
            },
            ln);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
}

struct WgradArgs {
    const uint16_t* gr;   // gradient w.r.t. the layer output (first channel)
    const uint16_t* x;    // layer input (first channel)
    float* part;          // [splits][Cout][T][Cin]
    uint32_t g_cs, x_cs;
    uint32_t N, H, W;     // reduction grid: output grid (SAME3), input grid (UP2)
    uint32_t Cin, Cout, T, mode;
    uint32_t chunks, per_split;   // 32-pixel chunks in total / per split
};

constexpr int kWgradWaves = 4;   // waves (pixel splits) per workgroup, summed in the workgroup

// One wave per (32 output channels, 32 input channels, split), all kT taps
// (9: 3x3, 4: transposed 2x2). Per 32-pixel chunk the operand that does not
// move with the tap (the output gradient for 3x3, the input for the
// transposed convolution) is staged and read once; the other one is staged
// per tap. Staging goes through LDS transposed (pixels contiguous): lane
// (pixel, channel half) loads 2 x 8 channels of its pixel.
template <int kT>
__global__ void __launch_bounds__(kWgradWaves * kWave) k_wgrad(WgradArgs a)
{
    constexpr bool kUpm = kT == 4;   // the transposed convolution
    __shared__ __attribute__((aligned(16))) uint16_t sgw[kWgradWaves][32][40];   // [co][px] per wave
    __shared__ __attribute__((aligned(16))) uint16_t sxw[kWgradWaves][32][40];   // [ci][px] per wave
    __shared__ float red[kT][2][2][4][kWave];   // one wave's accumulators
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    uint16_t (*sg)[40] = sgw[wv];
    uint16_t (*sx)[40] = sxw[wv];
    const int g = lane >> 4, l16 = lane & 15;
    const uint32_t ntc = (a.Cin + 31) / 32;
    const uint32_t co0 = (blockIdx.x / ntc) * 32, ci0 = (blockIdx.x % ntc) * 32;
    const uint32_t split = blockIdx.y * kWgradWaves + (uint32_t)wv;   // this wave's pixel range
    const uint32_t P = a.N * a.H * a.W;
    const uint32_t c_begin = split * a.per_split;
    const uint32_t c_end = c_begin + a.per_split < a.chunks ? c_begin + a.per_split : a.chunks;
    floatx4 acc[kT][2][2];
#pragma unroll
    for (int t = 0; t < kT; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[t][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int pl = lane & 31, hh = lane >> 5;   // staging: pixel, channel half
    // 16-byte loads of this lane's pixel (2 x 8 channels), then their
    // transposed LDS writes: split so that the loads of the next tap are in
    // flight while the current one is written and multiplied
    // (every lane loads, outside the image from element 0, and the zero
    // padding is applied when the values are written: no branch waits for
    // a load)
    struct Ld {
        u32x4 v[2];
        bool ok[2];
    };
    auto load = [&](const uint16_t* base, uint32_t cs, uint32_t c0, uint32_t climit, size_t pix, bool ok, Ld& l) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t ch = c0 + 16 * hh + 8 * q;
            l.ok[q] = ok && ch < climit;
            l.v[q] = *(const u32x4*)(base + (l.ok[q] ? pix * cs + ch : 0));
        }
    };
    auto put = [&](const Ld& l, uint16_t (*dst)[40]) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ch = 16 * hh + 8 * q + 2 * e;
                const uint32_t w = l.ok[q] ? l.v[q][e] : 0u;
                dst[ch][pl] = (uint16_t)(w & 0xFFFFu);
                dst[ch + 1][pl] = (uint16_t)(w >> 16);
            }
    };
    // the workgroup is one wave: ordering its own LDS accesses is enough,
    // and a wider fence would also wait for the loads in flight
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    for (uint32_t c = c_begin; c < c_end; ++c) {
        const uint32_t p = c * 32 + pl;
        const bool pok = p < P;
        const uint32_t n = p / (a.H * a.W), rem = p % (a.H * a.W), y = rem / a.W, xq = rem % a.W;
        // the tap-moving operand of tap t: its loads
        auto load_tap = [&](int tap, Ld& v) {
            if (kUpm) {
                // the gradient lives on the doubled grid
                const size_t gp =
                    ((size_t)n * 2 * a.H + 2 * y + (tap >> 1)) * (2 * (size_t)a.W) + 2 * xq + (tap & 1);
                load(a.gr, a.g_cs, co0, a.Cout, gp, pok, v);
            } else {
                const int ys = (int)y + tap / 3 - 1, xs = (int)xq + tap % 3 - 1;
                const bool ok = pok && ys >= 0 && ys < (int)a.H && xs >= 0 && xs < (int)a.W;
                const size_t xp = ok ? ((size_t)n * a.H + (uint32_t)ys) * a.W + (uint32_t)xs : 0;
                load(a.x, a.x_cs, ci0, a.Cin, xp, ok, v);
            }
        };
        Ld fv, tv[2];
        if (kUpm)
            load(a.x, a.x_cs, ci0, a.Cin, p, pok, fv);
        else
            load(a.gr, a.g_cs, co0, a.Cout, p, pok, fv);
        load_tap(0, tv[0]);
        sync();   // the previous chunk's reads are done
        put(fv, kUpm ? sx : sg);
        sync();
        u32x4 fix[2];   // fragments of the staged operand, the same for every tap
#pragma unroll
        for (int i = 0; i < 2; ++i)
            fix[i] = kUpm ? *(const u32x4*)&sx[16 * i + l16][8 * g] : *(const u32x4*)&sg[16 * i + l16][8 * g];
#pragma unroll
        for (int tap = 0; tap < kT; ++tap) {
            if (tap + 1 < kT) load_tap(tap + 1, tv[(tap + 1) & 1]);
            sync();   // the previous tap's reads are done
            put(tv[tap & 1], kUpm ? sg : sx);
            sync();
            u32x4 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = kUpm ? *(const u32x4*)&sg[16 * i + l16][8 * g] : fix[i];
                bv[i] = kUpm ? fix[i] : *(const u32x4*)&sx[16 * i + l16][8 * g];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[tap][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[i]), __builtin_bit_cast(bf16x8, bv[j]), acc[tap][i][j], 0, 0,
                        0);
        }
    }
    // the waves' sums added in wave order through LDS, then one partial row
    // per workgroup
    for (int w2 = 1; w2 < kWgradWaves; ++w2) {
        if (wv == w2)
#pragma unroll
            for (int tap = 0; tap < kT; ++tap)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) red[tap][i][j][r][lane] = acc[tap][i][j][r];
        __syncthreads();
        if (wv == 0)
#pragma unroll
            for (int tap = 0; tap < kT; ++tap)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[tap][i][j][r] += red[tap][i][j][r][lane];
        __syncthreads();
    }
    if (wv != 0) return;
#pragma unroll
    for (int tap = 0; tap < kT; ++tap)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t co = co0 + 16 * i + 4 * g + r, ci = ci0 + 16 * j + l16;
                    if (co < a.Cout && ci < a.Cin)
                        a.part[(((size_t)blockIdx.y * a.Cout + co) * kT + tap) * a.Cin + ci] = acc[tap][i][j][r];
                }
}

// dst[layout(co, tap, ci)] = sum over splits of part; ci < Creal. The splits
// fall into 16 contiguous groups, each summed in order by one thread, and
// the group sums are added in group order (a fixed order, so results do not
// depend on timing): a workgroup takes 16 elements x 16 groups.
// kind 0: 3x3 conv layout [co][tap][ci]; kind 1: transposed [tap][co][ci].
__global__ void __launch_bounds__(kBlock)
k_wgrad_reduce(const float* __restrict__ part, uint32_t splits, uint32_t Cout, uint32_t T,
               uint32_t Cin, uint32_t Creal, uint32_t kind, float* __restrict__ dst)
{
    constexpr uint32_t E = 16, GR = kBlock / E;
    __shared__ float red[GR][E];
    const size_t n = (size_t)Cout * T * Cin;
    const uint32_t e = threadIdx.x % E, grp = threadIdx.x / E;
    const size_t i = (size_t)blockIdx.x * E + e;
    const uint32_t per = (splits + GR - 1) / GR;
    const uint32_t k0 = grp * per, k1 = k0 + per < splits ? k0 + per : splits;
    float s = 0.0f;
    if (i < n)
        for (uint32_t k = k0; k < k1; ++k) s += part[(size_t)k * n + i];
    red[grp][e] = s;
    __syncthreads();
    if (grp != 0 || i >= n) return;
    float tot = 0.0f;
    for (uint32_t g2 = 0; g2 < GR; ++g2) tot += red[g2][e];
    const uint32_t ci = (uint32_t)(i % Cin), tap = (uint32_t)((i / Cin) % T), co = (uint32_t)(i / ((size_t)Cin * T));
    if (ci >= Creal) return;
    const size_t o = kind == 0 ? ((size_t)co * T + tap) * Creal + ci : ((size_t)tap * Cout + co) * Creal + ci;
    dst[o] = tot;
}

// Column sums of a [P][C] bf16 matrix (row stride cs, both multiples of 8)
// into fp32 partials [splits][C]: thread t adds the 8 channels of group
// t % (C / 8) of rows t / (C / 8), t / (C / 8) + 256 / (C / 8), ... with
// 16-byte loads; the row phases are then added in order.
__global__ void __launch_bounds__(kBlock)
k_colsum(const uint16_t* __restrict__ m, uint32_t cs, uint32_t P, uint32_t C, uint32_t per_split,
         float* __restrict__ part)
{
    __shared__ float red[kBlock * 8];
    const uint32_t t = threadIdx.x;
    const uint32_t G = C / 8, lanes = kBlock / G;   // C / 8 divides 256 (C <= 2048, power of two)
    const uint32_t cg = t % G, ph = t / G;
    const uint32_t r0 = blockIdx.x * per_split, r1 = r0 + per_split < P ? r0 + per_split : P;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (ph < lanes)
        for (uint32_t r = r0 + ph; r < r1; r += lanes) {
            const u32x4 v = *(const u32x4*)(m + (size_t)r * cs + 8 * cg);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += bf2f((uint16_t)(v[e >> 1] >> (16 * (e & 1))));
        }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[ph * C + 8 * cg + e] = s[e];
    __syncthreads();
    for (uint32_t c = t; c < C; c += kBlock) {
        float tot = 0.0f;
        for (uint32_t k = 0; k < lanes; ++k) tot += red[k * C + c];
        part[(size_t)blockIdx.x * C + c] = tot;
    }
}

// dst[i] = sum over k < splits (in order within each thread's stride, then
// a fixed tree) of part[k * n + i]; one workgroup per output value.
__global__ void __launch_bounds__(kBlock)
k_sum_splits(const float* __restrict__ part, uint32_t splits, uint32_t n, float* __restrict__ dst)
{
    __shared__ float red[kBlock];
    const uint32_t i = blockIdx.x;
    float s = 0.0f;
    for (uint32_t k = threadIdx.x; k < splits; k += kBlock) s += part[(size_t)k * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[i] = red[0];
}

// Splat images -> bf16 [P][8]: R, G, B, A / 255, depth - 1 (covered), cov, 0, 0.
__global__ void __launch_bounds__(kBlock)
k_pack_input(const uint32_t* __restrict__ rgba, const float* __restrict__ depth,
             const uint8_t* __restrict__ cov, uint32_t P, uint16_t* __restrict__ out)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    const uint32_t c = rgba[p];
    const bool cv = cov[p] != 0;
    uint16_t v[8];
    for (int k = 0; k < 4; ++k) v[k] = f2bf((float)((c >> (8 * k)) & 0xFFu) / 255.0f);
    v[4] = f2bf(cv ? depth[p] - 1.0f : 0.0f);
    v[5] = f2bf(cv ? 1.0f : 0.0f);
    v[6] = v[7] = 0;
    u32x4 w;
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)v[2 * k] | ((uint32_t)v[2 * k + 1] << 16);
    *(u32x4*)(out + (size_t)p * 8) = w;
}

// Gradient w.r.t. the pooled tensor's source: the pooled gradient goes to
// the first maximum of each window ((0,0), (0,1), (1,0), (1,1)); plus the
// skip gradient; rounded to bf16. Grid over the source (2H x 2W).
__global__ void __launch_bounds__(kBlock)
k_maxpool_bwd(const uint16_t* __restrict__ src, uint32_t src_cs, const uint16_t* __restrict__ dpool,
              const uint16_t* __restrict__ dskip, uint32_t dskip_cs, uint32_t N, uint32_t H,
              uint32_t W, uint32_t C, uint16_t* __restrict__ out)
{
    // one thread per source pixel and 8 channels (16-byte accesses; C, the
    // strides and the channel offsets of the pointers are multiples of 8)
    const uint32_t G = C / 8;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x, tot = (size_t)N * 4 * H * W * G;
    if (t >= tot) return;
    const size_t p = t / G;
    const uint32_t c = (uint32_t)(t - p * G) * 8;
    const uint32_t X = (uint32_t)(p % (2 * W)), Y = (uint32_t)((p / (2 * W)) % (2 * H)),
                   n = (uint32_t)(p / (4 * (size_t)W * H));
    const uint32_t y = Y >> 1, x = X >> 1, me = ((Y & 1) << 1) | (X & 1);
    u32x4 win[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const size_t s = ((size_t)n * 2 * H + 2 * y + (k >> 1)) * (2 * (size_t)W) + 2 * x + (k & 1);
        win[k] = *(const u32x4*)(src + s * src_cs + c);
    }
    const u32x4 sk = *(const u32x4*)(dskip + p * dskip_cs + c);
    const u32x4 dp = *(const u32x4*)(dpool + (((size_t)n * H + y) * W + x) * C + c);
    u32x4 o;
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
        uint32_t word = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float m = -INFINITY;
            uint32_t arg = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) {
                const float v = bf2f((uint16_t)(win[k][e2] >> (16 * h)));
                if (v > m) {
                    m = v;
                    arg = k;
                }
            }
            float g = bf2f((uint16_t)(sk[e2] >> (16 * h)));
            if (arg == me) g += bf2f((uint16_t)(dp[e2] >> (16 * h)));
            word |= (uint32_t)f2bf(g) << (16 * h);
        }
        o[e2] = word;
    }
    *(u32x4*)(out + p * C + c) = o;
}

// dz = dy where y > 0, else 0 (both bf16 [P][C], y with row stride y_cs,
// dy with row stride dy_cs).
__global__ void __launch_bounds__(kBlock)
k_relu_bwd(const uint16_t* __restrict__ dy, uint32_t dy_cs, const uint16_t* __restrict__ y,
           uint32_t y_cs, size_t P, uint32_t C, uint16_t* __restrict__ dz)
{
    // one thread per pixel and 8 channels (16-byte accesses; C, the strides
    // and the channel offsets of the pointers are multiples of 8)
    const uint32_t G = C / 8;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= P * G) return;
    const size_t p = t / G;
    const uint32_t c = (uint32_t)(t - p * G) * 8;
    const u32x4 yv = *(const u32x4*)(y + p * y_cs + c), gv = *(const u32x4*)(dy + p * dy_cs + c);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t lo = bf2f((uint16_t)(yv[k] & 0xFFFFu)) > 0.0f ? gv[k] & 0xFFFFu : 0u;
        const uint32_t hi = bf2f((uint16_t)(yv[k] >> 16)) > 0.0f ? gv[k] & 0xFFFF0000u : 0u;
        o[k] = lo | hi;
    }
    *(u32x4*)(dz + p * C + c) = o;
}

// Head in training: loss = mean over 3P of (rgb / 255 + residual - t / 255)^2.
// Writes dX (bf16 [P][32]) and per-block partial sums: [blocks][32*3 dW, 3 db, 1 loss].
constexpr int kHeadPart = kBase * 3 + 3 + 1;

__global__ void __launch_bounds__(kBlock)
k_head_train(const uint16_t* __restrict__ x, const float* __restrict__ w, const float* __restrict__ b,
             const uint32_t* __restrict__ rgba, const uint32_t* __restrict__ tgt, uint32_t P,
             uint16_t* __restrict__ dx, float* __restrict__ part)
{
    __shared__ float red[kBlock / kWave][kHeadPart];
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const float inv_n = 1.0f / (3.0f * (float)P);
    float xv[kBase], d[3] = {0.f, 0.f, 0.f}, l = 0.0f;
    if (p < P) {
        float r[3] = {b[0], b[1], b[2]};
#pragma unroll
        for (int c4 = 0; c4 < kBase / 8; ++c4) {
            const u32x4 v = *(const u32x4*)(x + (size_t)p * kBase + 8 * c4);
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[8 * c4 + e] = bf2f((uint16_t)(v[e >> 1] >> (16 * (e & 1))));
        }
        for (int c = 0; c < kBase; ++c)
            for (int k = 0; k < 3; ++k) r[k] += w[k * kBase + c] * xv[c];
        const uint32_t s = rgba[p], t = tgt[p];
        for (int k = 0; k < 3; ++k) {
            const float diff = ((float)((s >> (8 * k)) & 0xFFu) / 255.0f + r[k]) -
                               (float)((t >> (8 * k)) & 0xFFu) / 255.0f;
            l += diff * diff;
            d[k] = 2.0f * diff * inv_n;
        }
#pragma unroll
        for (int c4 = 0; c4 < kBase / 8; ++c4) {
            u32x4 o;
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                const int c = 8 * c4 + 2 * e2;
                const uint32_t lo = f2bf(w[c] * d[0] + w[kBase + c] * d[1] + w[2 * kBase + c] * d[2]);
                const uint32_t hi =
                    f2bf(w[c + 1] * d[0] + w[kBase + c + 1] * d[1] + w[2 * kBase + c + 1] * d[2]);
                o[e2] = lo | (hi << 16);
            }
            *(u32x4*)(dx + (size_t)p * kBase + 8 * c4) = o;
        }
    } else {
        for (int c = 0; c < kBase; ++c) xv[c] = 0.0f;
    }
    // block sums of dW[k][c] = d[k] x[c], db[k] = d[k], loss: a butterfly
    // within each wave, then the waves' sums in wave order
    for (int q = 0; q < kHeadPart; ++q) {
        float v;
        if (q < 3 * kBase) v = d[q / kBase] * xv[q % kBase];
        else if (q < 3 * kBase + 3) v = d[q - 3 * kBase];
        else v = l * inv_n;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < (uint32_t)kHeadPart; q += kBlock) {
        float tot = 0.0f;
        for (int k = 0; k < kBlock / kWave; ++k) tot += red[k][q];
        part[(size_t)blockIdx.x * kHeadPart + q] = tot;
    }
}

__global__ void __launch_bounds__(kBlock)
k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
       uint64_t n, float lr, float c1, float c2)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Weight conversion to bf16 layouts, all layers in one launch (per-layer
// launches took a few microseconds each for little work): a table of
// layers, each a range of the concatenated element space.
//   3x3 conv: forward [co][tap][ci_pad] and input-gradient [ci][tap'][co]
//             with tap' = 8 - tap (spatial flip; only when wb is given)
//   transposed 2x2: forward [tap][co][ci] (= parameter layout) and
//             input-gradient [ci][tap][co]
constexpr int kMaxPrep = 32;
struct PrepTable {
    uint32_t n;
    struct Entry {
        uint32_t kind, cout, cin, cpad, start;   // kind 0: 3x3, 1: transposed 2x2
        const float* w;
        uint16_t* wf;
        uint16_t* wb;   // or null
    } e[kMaxPrep];
};

// Eight consecutive elements per thread (every layer's count and start are
// multiples of 8, and so is cpad: the eight share a tap and an output
// channel): one walk of the table, eight conversions, one 16-byte store of
// the forward layout; the backward layout's elements are scattered.
__global__ void __launch_bounds__(kBlock) k_prep_all(PrepTable t, uint32_t total)
{
    const uint32_t g = (blockIdx.x * kBlock + threadIdx.x) * 8;
    if (g >= total) return;
    uint32_t l = 0;
    while (l + 1 < t.n && g >= t.e[l + 1].start) ++l;
    const PrepTable::Entry& y = t.e[l];
    const uint32_t i = g - y.start;
    uint16_t v[8];
    if (y.kind == 0) {
        const uint32_t ci0 = i % y.cpad, tap = (i / y.cpad) % 9, co = i / (y.cpad * 9);
        const float* src = y.w + ((size_t)co * 9 + tap) * y.cin;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t ci = ci0 + (uint32_t)e;
            v[e] = ci < y.cin ? f2bf(src[ci]) : (uint16_t)0;
            if (y.wb && ci < y.cin) y.wb[((size_t)ci * 9 + (8 - tap)) * y.cout + co] = v[e];
        }
    } else {
        const uint32_t ci0 = i % y.cin, co = (i / y.cin) % y.cout, tap = i / (y.cin * y.cout);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[e] = f2bf(y.w[i + e]);
            y.wb[((size_t)(ci0 + e) * 4 + tap) * y.cout + co] = v[e];
        }
    }
    uint4 o;
    o.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    o.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    o.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
    o.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
    *(uint4*)(y.wf + i) = o;
}

}  // namespace nn
}  // namespace fhv

// ---------------------------------------------------------------- host side

namespace fhv {
namespace nn {

namespace {

thread_local const Device* t_dev = nullptr;   // set at the entry points, for ProfScope

Device no_dev{0, 0, nullptr};

inline const Device& cur_dev() { return t_dev ? *t_dev : no_dev; }

struct Layer {
    int kind;   // 0 = 3x3 conv, 1 = transposed conv, 2 = head
    uint32_t cin, cout, cpad;
    uint32_t lvl;          // level of the pixel grid its weight gradient sums over
    size_t off_w, off_b;   // into the parameter vector
    size_t wf_off, wb_off; // into the bf16 weight area (elements)
};

struct Net {
    uint32_t L;
    uint32_t C[4];
    std::vector<Layer> layers;
    size_t n_params = 0, n_wf = 0;

    explicit Net(uint32_t levels) : L(levels)
    {
        for (uint32_t l = 0; l < 4; ++l) C[l] = (uint32_t)kBase << l;
        uint32_t cin = 6;
        for (uint32_t l = 0; l < L; ++l) {
            add(0, cin, C[l], l);
            add(0, C[l], C[l], l);
            cin = C[l];
        }
        for (int l = (int)L - 2; l >= 0; --l) {
            add(1, C[l + 1], C[l], (uint32_t)l + 1);
            add(0, 2 * C[l], C[l], (uint32_t)l);
            add(0, C[l], C[l], (uint32_t)l);
        }
        add(2, C[0], 3, 0);
    }
    void add(int kind, uint32_t cin, uint32_t cout, uint32_t lvl)
    {
        Layer y;
        y.kind = kind;
        y.lvl = lvl;
        y.cin = cin;
        y.cout = cout;
        y.cpad = (cin + 7) / 8 * 8;
        const size_t nw = kind == 0 ? (size_t)cout * 9 * cin : kind == 1 ? (size_t)4 * cout * cin : (size_t)cout * cin;
        y.off_w = n_params;
        y.off_b = n_params + nw;
        n_params += nw + cout;
        const size_t nwf = kind == 0 ? (size_t)cout * 9 * y.cpad : kind == 1 ? (size_t)4 * cout * cin : 0;
        y.wf_off = n_wf;
        y.wb_off = n_wf + nwf;
        n_wf += 2 * nwf;
        layers.push_back(y);
    }
    size_t enc(uint32_t l, uint32_t s) const { return 2 * l + s; }
    size_t dec(uint32_t l) const { return 2 * L + 3 * (L - 2 - l); }   // t2; +1, +2 convs
    size_t head() const { return layers.size() - 1; }
};

constexpr size_t kMaxLayers = 32;

struct Bufs {
    uint16_t* wt;          // bf16 weights (forward and input-gradient layouts)
    uint16_t* x0;
    uint16_t *e0[4], *cat[4], *elast, *pool[4], *d0[4], *d1[4];
    // training
    uint16_t *gh, *dz, *ga, *gb, *dcat[4];
    float *part, *hpart, *grad;
    size_t part_elems, hpart_elems;
    // traced training: every layer's masked output gradient (tz) and input
    // gradient (tg), and every max pool's input gradient (tp), kept in
    // buffers of their own instead of the shared dz, ga and gb
    bool trace;
    uint16_t *tz[kMaxLayers], *tg[kMaxLayers], *tp[4];
};

constexpr uint32_t kWgradTarget = 1024;   // waves per weight-gradient launch

void wgrad_dims(uint32_t P, uint32_t Cin, uint32_t Cout, uint32_t T, uint32_t* splits, uint32_t* per)
{
    (void)T;   // a wave takes every tap
    const uint32_t tiles = (Cout / 32) * ((Cin + 31) / 32);
    const uint32_t chunks = (P + 31) / 32;
    uint32_t s = (kWgradTarget + tiles - 1) / tiles;
    s = s < 1 ? 1 : (s > chunks ? chunks : s);
    *per = (chunks + s - 1) / s;
    *splits = (chunks + *per - 1) / *per;
}

size_t carve(const Net& net, uint32_t N, uint32_t H, uint32_t W, bool training, char* base, Bufs* b,
             bool trace = false)
{
    Carver c{base, 0};
    const uint32_t L = net.L;
    auto P = [&](uint32_t l) { return (size_t)N * (H >> l) * (W >> l); };
    b->wt = c.take<uint16_t>(net.n_wf);
    b->x0 = c.take<uint16_t>(P(0) * kInPad);
    for (uint32_t l = 0; l < L; ++l) {
        b->e0[l] = c.take<uint16_t>(P(l) * net.C[l]);
        if (l + 1 < L) {
            b->cat[l] = c.take<uint16_t>(P(l) * 2 * net.C[l]);
            b->pool[l] = c.take<uint16_t>(P(l + 1) * net.C[l]);
            b->d0[l] = c.take<uint16_t>(P(l) * net.C[l]);
            b->d1[l] = c.take<uint16_t>(P(l) * net.C[l]);
        }
    }
    b->elast = c.take<uint16_t>(P(L - 1) * net.C[L - 1]);
    if (training) {
        size_t mx = 0, mpart = 0;
        for (uint32_t l = 0; l < L; ++l) mx = std::max(mx, P(l) * net.C[l]);
        b->gh = c.take<uint16_t>(P(0) * net.C[0]);
        b->dz = c.take<uint16_t>(mx);
        b->ga = c.take<uint16_t>(mx);
        b->gb = c.take<uint16_t>(mx);
        for (uint32_t l = 0; l + 1 < L; ++l) b->dcat[l] = c.take<uint16_t>(P(l) * 2 * net.C[l]);
        // weight-gradient partials: the largest over the layers
        for (size_t i = 0; i < net.layers.size(); ++i) {
            const Layer& y = net.layers[i];
            if (y.kind == 2) continue;
            uint32_t s, per;
            const uint32_t T = y.kind == 0 ? 9 : 4;
            wgrad_dims((uint32_t)P(y.lvl), y.cpad, y.cout, T, &s, &per);
            mpart = std::max(mpart, (size_t)s * y.cout * T * y.cpad);
            mpart = std::max(mpart, (size_t)1024 * y.cout);   // bias partials
        }
        b->part_elems = mpart;
        b->part = c.take<float>(mpart);
        b->hpart_elems = ((P(0) + kBlock - 1) / kBlock) * kHeadPart;
        b->hpart = c.take<float>(b->hpart_elems);
        b->grad = c.take<float>(net.n_params);
    }
    b->trace = training && trace;
    for (size_t i = 0; i < kMaxLayers; ++i) b->tz[i] = b->tg[i] = nullptr;
    for (uint32_t l = 0; l < 4; ++l) b->tp[l] = nullptr;
    if (b->trace) {
        for (size_t i = 0; i < net.layers.size(); ++i) {
            const Layer& y = net.layers[i];
            if (y.kind == 0) b->tz[i] = c.take<uint16_t>(P(y.lvl) * y.cout);
            if ((y.kind == 0 && i > 0) || y.kind == 1) b->tg[i] = c.take<uint16_t>(P(y.lvl) * y.cin);
        }
        for (uint32_t l = 0; l + 1 < L; ++l) b->tp[l] = c.take<uint16_t>(P(l) * net.C[l]);
    }
    return c.off + 256;
}

unsigned blocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Head applied in the epilogue of the network's last convolution (inference).
struct HeadFuse {
    const float* w;
    const float* b;
    const uint32_t* rgba;
    uint32_t* out;
    float* res;
};

hipError_t conv(const uint16_t* in, uint32_t in_cs, const uint16_t* wt, const float* bias, uint16_t* out,
                uint32_t out_cs, uint32_t N, uint32_t H, uint32_t W, uint32_t Cin, uint32_t Cout,
                int mode, bool relu, hipStream_t s, uint16_t* pool = nullptr, uint32_t pool_cs = 0,
                const HeadFuse* hf = nullptr)
{
    ConvArgs a;
    a.pool = pool;
    a.pool_cs = pool_cs;
    a.head_w = hf ? hf->w : nullptr;
    a.head_b = hf ? hf->b : nullptr;
    a.head_rgba = hf ? hf->rgba : nullptr;
    a.head_out = hf ? hf->out : nullptr;
    a.head_res = hf ? hf->res : nullptr;
    // the fused head needs the 32-channel 3x3 path
    if (hf && (mode != MODE_SAME3 || Cin != 32 || Cout != 32)) return hipErrorInvalidValue;
    // the fused pool needs a 3x3 layer on the staged path, even sizes
    if (pool && (mode != MODE_SAME3 || Cin % 32 != 0 || (H & 1) || (W & 1) || Cout % 8 != 0))
        return hipErrorInvalidValue;
    a.in = in;
    a.wt = wt;
    a.bias = bias;
    a.out = out;
    a.in_cs = in_cs;
    a.out_cs = out_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    a.Cin = Cin;
    a.Cout = Cout;
    a.T = mode == MODE_SAME3 ? 9 : (mode == MODE_GATHER4 ? 4 : 1);
    a.mode = (uint32_t)mode;
    a.relu = relu ? 1u : 0u;
    const unsigned gz = 1, up = mode == MODE_UP2 ? 4 : 1;
    ProfScope ps(cur_dev(), "fill.conv", s);
    const dim3 blk(kBlock);
    const uint32_t rows = N * H;
    if (Cin == 8) {
        if (mode != MODE_SAME3) return hipErrorInvalidValue;
        k_conv<MODE_SAME3, 2, 2, true><<<dim3(rows * ((W + 127) / 128), (Cout + 31) / 32, gz), blk, 0, s>>>(a);
        return hipGetLastError();
    }
    if (Cin % 32 != 0) return hipErrorInvalidValue;
    const dim3 g32(rows * ((W + 255) / 256) * up, (Cout + 31) / 32, gz),
        g64(rows * ((W + 255) / 256) * up, (Cout + 63) / 64, gz);
    const bool narrow = Cout <= 32;
    // staged kernel: with one 32-channel chunk per tile a workgroup has
    // nothing to load ahead within its tile, so workgroups are made
    // persistent (two per compute unit, as LDS and registers allow) and load
    // the next tile during the current one; otherwise one workgroup per tile
    const auto pgrid = [&](uint32_t tiles, uint32_t cols) {
        if (Cin > 32) return dim3(tiles, cols);
        const uint32_t want = (uint32_t)cur_dev().cus * 2 / cols;
        return dim3(std::max(1u, std::min(tiles, want)), cols);
    };
    const uint32_t rows2 = N * ((H + 1) / 2);
    const bool fits62 = (size_t)((W + 61) / 62) * 62 * 10 <= (size_t)W * 11;
    switch (mode) {
    case MODE_SAME3:
        // the 62-pixel tiles of k_conv3r and k_conv3a suit rows whose width
        // they cover with little waste (at most a tenth); narrow rows such
        // as 32, 64 or 128 pixels take the 64-pixel tiles of k_conv3
        if (Cout == 32 && (Cin == 32 || Cin == 64) && (hf || fits62)) {
            const dim3 gr(std::min<uint32_t>(N * ((H + cvr::R - 1) / cvr::R) * ((W + cvr::TX - 1) / cvr::TX),
                                             (uint32_t)cur_dev().cus));
            if (hf)
                k_conv3r<true><<<gr, dim3(cvr::WAVES * kWave), 0, s>>>(a);
            else
                k_conv3r<false><<<gr, dim3(cvr::WAVES * kWave), 0, s>>>(a);
        } else if (narrow)
            k_conv3<2, 64, false, 4><<<pgrid(N * ((H + 3) / 4) * ((W + 63) / 64), (Cout + 31) / 32), blk, 0, s>>>(a);
        else if (Cin % 32 == 0 && Cout % 64 == 0 && fits62)
        {
            // persistent: one workgroup per compute unit over all channel blocks
            const uint32_t tiles = N * ((H + cva::R - 1) / cva::R) * ((W + cva::TX - 1) / cva::TX);
            const uint32_t per = std::max(1u, (uint32_t)cur_dev().cus / (Cout / 64));
            k_conv3a<<<dim3(std::min(tiles, per), Cout / 64), dim3(cva::WAVES * kWave), 0, s>>>(a);
        }
        else
            k_conv3<4, 64, false><<<pgrid(rows2 * ((W + 63) / 64), (Cout + 63) / 64), blk, 0, s>>>(a);
        break;
    case MODE_UP2:
        if (Cout % 32 == 0) {
            // 128 columns per workgroup: the input tile is read once for
            // every 128 of the 4 Cout columns
            k_conv3<8, 64, true><<<pgrid(rows2 * ((W + 63) / 64), (4 * Cout + 127) / 128), blk, 0, s>>>(a);
            break;
        }
        if (narrow) k_conv<MODE_UP2, 4, 2, false><<<g32, blk, 0, s>>>(a);
        else k_conv<MODE_UP2, 4, 4, false><<<g64, blk, 0, s>>>(a);
        break;
    default:
        if (narrow) k_conv<MODE_GATHER4, 4, 2, false><<<g32, blk, 0, s>>>(a);
        else k_conv<MODE_GATHER4, 4, 4, false><<<g64, blk, 0, s>>>(a);
        break;
    }
    return hipGetLastError();
}

// Both convolutions of the first encoder level and its pool, fused
// (inference: the first convolution's output is not kept).
hipError_t conv_first(const uint16_t* in, uint32_t in_cs, const uint16_t* w1, const float* b1, const uint16_t* w2,
                      const float* b2, uint16_t* out, uint32_t out_cs, uint16_t* pool, uint32_t pool_cs, uint32_t N,
                      uint32_t H, uint32_t W, hipStream_t s)
{
    if ((H & 1) || (W & 1) || in_cs != kInPad) return hipErrorInvalidValue;
    Conv2Args a;
    a.in = in;
    a.w1 = w1;
    a.b1 = b1;
    a.w2 = w2;
    a.b2 = b2;
    a.out = out;
    a.pool = pool;
    a.in_cs = in_cs;
    a.out_cs = out_cs;
    a.pool_cs = pool_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    ProfScope ps(cur_dev(), "fill.conv", s);
    const uint32_t tiles = N * ((H + cv2::R - 1) / cv2::R) * ((W + cv2::TX - 1) / cv2::TX);
    k_conv33<<<dim3(std::min<uint32_t>(tiles, (uint32_t)cur_dev().cus)), dim3(cv2::WAVES * kWave), 0, s>>>(a);
    return hipGetLastError();
}

// The decoder's last transposed convolution and first 3x3 convolution,
// fused (inference: the up-sampled channels are not kept).
hipError_t conv_up_first(const uint16_t* low, uint32_t low_cs, const uint16_t* wu, const float* bu,
                         const uint16_t* skip, uint32_t skip_cs, const uint16_t* wt, const float* bias, uint16_t* out,
                         uint32_t out_cs, uint32_t N, uint32_t H, uint32_t W, hipStream_t s)
{
    if ((H & 1) || (W & 1)) return hipErrorInvalidValue;
    ConvUpArgs a;
    a.low = low;
    a.wu = wu;
    a.bu = bu;
    a.skip = skip;
    a.wt = wt;
    a.bias = bias;
    a.out = out;
    a.low_cs = low_cs;
    a.skip_cs = skip_cs;
    a.out_cs = out_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    ProfScope ps(cur_dev(), "fill.conv", s);
    const uint32_t tiles = N * ((H + cvu::R - 1) / cvu::R) * ((W + cvu::TX - 1) / cvu::TX);
    k_conv3u<<<dim3(std::min<uint32_t>(tiles, (uint32_t)cur_dev().cus)), dim3(cvu::WAVES * kWave), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t wgrad(const uint16_t* gr, uint32_t g_cs, const uint16_t* x, uint32_t x_cs, uint32_t N,
                 uint32_t H, uint32_t W, uint32_t Cin, uint32_t Creal, uint32_t Cout, int mode,
                 float* part, size_t part_elems, float* dst, hipStream_t s)
{
    WgradArgs a;
    a.gr = gr;
    a.x = x;
    a.part = part;
    a.g_cs = g_cs;
    a.x_cs = x_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    a.Cin = Cin;
    a.Cout = Cout;
    a.T = mode == MODE_SAME3 ? 9 : 4;
    a.mode = (uint32_t)mode;
    const uint32_t P = N * H * W;
    uint32_t splits = 0;
    wgrad_dims(P, Cin, Cout, a.T, &splits, &a.per_split);
    a.chunks = (P + 31) / 32;
    if ((size_t)splits * Cout * a.T * Cin > part_elems) return hipErrorInvalidValue;
    ProfScope ps(cur_dev(), "fill.wgrad", s);
    const uint32_t groups = (splits + kWgradWaves - 1) / kWgradWaves;   // partial rows
    const dim3 gr_((Cout / 32) * ((Cin + 31) / 32), groups);
    if (a.T == 9)
        k_wgrad<9><<<gr_, dim3(kWgradWaves * kWave), 0, s>>>(a);
    else
        k_wgrad<4><<<gr_, dim3(kWgradWaves * kWave), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_wgrad_reduce<<<dim3((unsigned)(((size_t)Cout * a.T * Cin + 15) / 16)), dim3(kBlock), 0, s>>>(
        part, groups, Cout, a.T, Cin, Creal, mode == MODE_SAME3 ? 0u : 1u, dst);
    return hipGetLastError();
}

hipError_t bgrad(const uint16_t* m, uint32_t cs, uint32_t P, uint32_t C, float* part, float* dst,
                 hipStream_t s)
{
    uint32_t splits = (P + 255) / 256;
    splits = splits > 512 ? 512 : splits;
    const uint32_t per = (P + splits - 1) / splits;
    splits = (P + per - 1) / per;
    k_colsum<<<dim3(splits), dim3(kBlock), 0, s>>>(m, cs, P, C, per, part);
    k_sum_splits<<<dim3(C), dim3(kBlock), 0, s>>>(part, splits, C, dst);
    return hipGetLastError();
}

#define FHV_TRY(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return e_;            \
    } while (0)

hipError_t prep_weights(const Net& net, const float* th, bool training, const Bufs& b, hipStream_t s)
{
    PrepTable t{};
    uint32_t total = 0;
    for (size_t i = 0; i < net.layers.size(); ++i) {
        const Layer& y = net.layers[i];
        if (y.kind != 0 && y.kind != 1) continue;
        if (t.n == (uint32_t)kMaxPrep) return hipErrorInvalidValue;
        PrepTable::Entry& e = t.e[t.n++];
        e.kind = (uint32_t)y.kind;
        e.cout = y.cout;
        e.cin = y.cin;
        e.cpad = y.cpad;
        e.start = total;
        e.w = th + y.off_w;
        e.wf = b.wt + y.wf_off;
        e.wb = y.kind == 1 || (training && i > 0) ? b.wt + y.wb_off : nullptr;
        total += y.kind == 0 ? y.cout * 9 * y.cpad : 4 * y.cout * y.cin;
    }
    if (total) k_prep_all<<<blocks(total / 8), dim3(kBlock), 0, s>>>(t, total);
    return hipGetLastError();
}

// Forward pass up to the head input; returns it (P0 x 32, row stride 32).
hipError_t forward(const Net& net, const float* th, const Bufs& b, uint32_t N, uint32_t H, uint32_t W,
                   hipStream_t s, const uint16_t** head_in, const HeadFuse* hf = nullptr)
{
    const uint32_t L = net.L;
    const uint16_t* h = b.x0;
    uint32_t h_cs = kInPad, cin = kInPad;
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t Hl = H >> l, Wl = W >> l, Cl = net.C[l];
        const Layer& a0 = net.layers[net.enc(l, 0)];
        const Layer& a1 = net.layers[net.enc(l, 1)];
        if (l == 0 && hf && L > 1) {
            // inference: the first level's two convolutions in one kernel
            FHV_TRY(conv_first(h, h_cs, b.wt + a0.wf_off, th + a0.off_b, b.wt + a1.wf_off, th + a1.off_b,
                               b.cat[0] + Cl, 2 * Cl, b.pool[0], Cl, N, Hl, Wl, s));
            h = b.pool[0];
            h_cs = Cl;
            cin = Cl;
            continue;
        }
        FHV_TRY(conv(h, h_cs, b.wt + a0.wf_off, th + a0.off_b, b.e0[l], Cl, N, Hl, Wl, cin, Cl, MODE_SAME3, true, s));
        uint16_t* o1 = l + 1 < L ? b.cat[l] + Cl : b.elast;
        const uint32_t o1_cs = l + 1 < L ? 2 * Cl : Cl;
        // the second convolution of a level above the last also writes its
        // 2x2 max pool (fused into its epilogue)
        FHV_TRY(conv(b.e0[l], Cl, b.wt + a1.wf_off, th + a1.off_b, o1, o1_cs, N, Hl, Wl, Cl, Cl, MODE_SAME3, true, s,
                     l + 1 < L ? b.pool[l] : nullptr, Cl, L == 1 ? hf : nullptr));
        if (l + 1 < L) {
            h = b.pool[l];
            h_cs = Cl;
            cin = Cl;
        }
    }
    h = b.elast;
    h_cs = net.C[L - 1];
    for (int l = (int)L - 2; l >= 0; --l) {
        const uint32_t Hl = H >> l, Wl = W >> l, Cl = net.C[l];
        const Layer& t = net.layers[net.dec(l)];
        const Layer& c0 = net.layers[net.dec(l) + 1];
        const Layer& c1 = net.layers[net.dec(l) + 2];
        if (l == 0 && hf) {
            // inference: the transposed convolution inside the first 3x3 one
            FHV_TRY(conv_up_first(h, h_cs, b.wt + t.wf_off, th + t.off_b, b.cat[0] + Cl, 2 * Cl, b.wt + c0.wf_off,
                                  th + c0.off_b, b.d0[0], Cl, N, Hl, Wl, s));
        } else {
            FHV_TRY(conv(h, h_cs, b.wt + t.wf_off, th + t.off_b, b.cat[l], 2 * Cl, N, Hl / 2, Wl / 2,
                         net.C[l + 1], Cl, MODE_UP2, false, s));
            FHV_TRY(conv(b.cat[l], 2 * Cl, b.wt + c0.wf_off, th + c0.off_b, b.d0[l], Cl, N, Hl, Wl, 2 * Cl, Cl,
                         MODE_SAME3, true, s));
        }
        FHV_TRY(conv(b.d0[l], Cl, b.wt + c1.wf_off, th + c1.off_b, b.d1[l], Cl, N, Hl, Wl, Cl, Cl,
                     MODE_SAME3, true, s, nullptr, 0, l == 0 ? hf : nullptr));
        h = b.d1[l];
        h_cs = Cl;
    }
    *head_in = h;
    return hipSuccess;
}

// Backward through a 3x3 conv layer i with output y (row stride y_cs) given
// the gradient g w.r.t. y (row stride g_cs): weight and bias gradients into
// grad, and (when gin) the input gradient into gin (row stride gin_cs).
hipError_t conv_bwd(const Net& net, size_t i, const Bufs& b, const uint16_t* x, uint32_t x_cs,
                    const uint16_t* y, uint32_t y_cs, const uint16_t* g, uint32_t g_cs, uint16_t* gin,
                    uint32_t gin_cs, uint32_t N, uint32_t Hl, uint32_t Wl, hipStream_t s)
{
    const Layer& ly = net.layers[i];
    const size_t P = (size_t)N * Hl * Wl;
    uint16_t* dz = b.trace ? b.tz[i] : b.dz;
    k_relu_bwd<<<blocks(P * (ly.cout / 8)), dim3(kBlock), 0, s>>>(g, g_cs, y, y_cs, P, ly.cout, dz);
    FHV_TRY(hipGetLastError());
    FHV_TRY(wgrad(dz, ly.cout, x, x_cs, N, Hl, Wl, ly.cpad, ly.cin, ly.cout, MODE_SAME3, b.part,
                  b.part_elems, b.grad + ly.off_w, s));
    FHV_TRY(bgrad(dz, ly.cout, (uint32_t)P, ly.cout, b.part, b.grad + ly.off_b, s));
    if (gin)
        FHV_TRY(conv(dz, ly.cout, b.wt + ly.wb_off, nullptr, gin, gin_cs, N, Hl, Wl, ly.cout, ly.cpad,
                     MODE_SAME3, false, s));
    return hipSuccess;
}

hipError_t backward(const Net& net, const float* th, const Bufs& b, uint32_t N, uint32_t H, uint32_t W,
                    hipStream_t s)
{
    const uint32_t L = net.L;
    // decoder, top level first; g is the gradient w.r.t. the level's output
    const uint16_t* g = b.gh;
    for (uint32_t l = 0; l + 1 < L; ++l) {
        const uint32_t Hl = H >> l, Wl = W >> l, Cl = net.C[l];
        const size_t it = net.dec(l);
        uint16_t* g2 = b.trace ? b.tg[it + 2] : b.ga;
        FHV_TRY(conv_bwd(net, it + 2, b, b.d0[l], Cl, b.d1[l], Cl, g, Cl, g2, Cl, N, Hl, Wl, s));
        FHV_TRY(conv_bwd(net, it + 1, b, b.cat[l], 2 * Cl, b.d0[l], Cl, g2, Cl, b.dcat[l], 2 * Cl, N, Hl,
                         Wl, s));
        // transposed conv: input hin on level l + 1, output gradient = first half of dcat
        const Layer& t = net.layers[it];
        const uint16_t* hin = (l + 2 == L) ? b.elast : b.d1[l + 1];
        const uint32_t Cu = net.C[l + 1];
        FHV_TRY(wgrad(b.dcat[l], 2 * Cl, hin, Cu, N, Hl / 2, Wl / 2, Cu, Cu, Cl, MODE_UP2, b.part,
                      b.part_elems, b.grad + t.off_w, s));
        FHV_TRY(bgrad(b.dcat[l], 2 * Cl, N * Hl * Wl, Cl, b.part, b.grad + t.off_b, s));
        uint16_t* gt = b.trace ? b.tg[it] : b.gb;
        FHV_TRY(conv(b.dcat[l], 2 * Cl, b.wt + t.wb_off, nullptr, gt, Cu, N, Hl / 2, Wl / 2, Cl, Cu,
                     MODE_GATHER4, false, s));
        g = gt;
    }
    // encoder, deepest level first. The gradient stays in one buffer (each
    // layer's ReLU-gradient kernel consumes it before the layer's input
    // gradient overwrites it), except across a max pool, whose gradient
    // kernel reads the pooled gradient and writes the other buffer.
    uint16_t* cur = (uint16_t*)g;
    for (int l = (int)L - 1; l >= 0; --l) {
        const uint32_t Hl = H >> l, Wl = W >> l, Cl = net.C[l];
        const uint16_t* y1 = l + 1 < (int)L ? b.cat[l] + Cl : b.elast;
        const uint32_t y1_cs = l + 1 < (int)L ? 2 * Cl : Cl;
        if (l + 1 < (int)L) {
            uint16_t* nxt = b.trace ? b.tp[l] : (cur == b.ga ? b.gb : b.ga);
            // pooled gradient (cur, on level l + 1) plus the skip gradient
            k_maxpool_bwd<<<blocks((size_t)N * Hl * Wl * (Cl / 8)), dim3(kBlock), 0, s>>>(
                y1, y1_cs, cur, b.dcat[l] + Cl, 2 * Cl, N, Hl / 2, Wl / 2, Cl, nxt);
            FHV_TRY(hipGetLastError());
            cur = nxt;
        }
        // traced: every input gradient into a buffer of its own
        uint16_t* g1 = b.trace ? b.tg[net.enc(l, 1)] : cur;
        FHV_TRY(conv_bwd(net, net.enc(l, 1), b, b.e0[l], Cl, y1, y1_cs, cur, Cl, g1, Cl, N, Hl, Wl, s));
        cur = g1;
        const uint16_t* x0 = l == 0 ? b.x0 : b.pool[l - 1];
        const uint32_t x0_cs = l == 0 ? kInPad : net.C[l - 1];
        uint16_t* g0 = l > 0 ? (b.trace ? b.tg[net.enc(l, 0)] : cur) : nullptr;
        FHV_TRY(conv_bwd(net, net.enc(l, 0), b, x0, x0_cs, b.e0[l], Cl, cur, Cl, g0, l > 0 ? net.C[l - 1] : 0, N,
                         Hl, Wl, s));
        if (g0) cur = g0;
    }
    return hipSuccess;
}

}  // namespace

uint64_t param_count(uint32_t levels) { return Net(levels).n_params; }

// Scope that makes the device's profiler visible to the layer helpers.
struct DevScope {
    explicit DevScope(const Device& d) { t_dev = &d; }
    ~DevScope() { t_dev = nullptr; }
};

size_t fill_ws_bytes(uint32_t levels, uint32_t N, uint32_t H, uint32_t W, bool training, bool trace)
{
    Net net(levels);
    Bufs b;
    return carve(net, N, H, W, training, nullptr, &b, trace);
}

// Where a traced training step leaves every tensor of every layer in its
// workspace: five entries per parameter layer (input, output, gradient
// received for the output, that gradient after the ReLU mask, gradient of
// the input), channels 0 where a layer has no such tensor.
uint32_t trace_tensors(uint32_t levels, uint32_t N, uint32_t H, uint32_t W, fhv_fill_tensor* out, uint32_t cap)
{
    Net net(levels);
    Bufs b;
    // offsets from a stand-in base address (nothing is dereferenced)
    char* const base = (char*)(uintptr_t)4096;
    carve(net, N, H, W, true, base, &b, true);
    const uint32_t L = levels;
    const uint32_t n = (uint32_t)net.layers.size() * 5;
    if (!out) return n;
    auto put = [&](uint32_t k, const uint16_t* p, uint32_t stride, uint32_t ch, uint32_t lvl) {
        if (k >= cap) return;
        fhv_fill_tensor t{};
        if (p && ch) {
            t.offset = (uint64_t)((const char*)p - base);
            t.stride = stride;
            t.channels = ch;
            t.n = N;
            t.height = H >> lvl;
            t.width = W >> lvl;
        }
        out[k] = t;
    };
    for (uint32_t k = 0; k < n && k < cap; ++k) out[k] = fhv_fill_tensor{};
    const auto& C = net.C;
    for (uint32_t l = 0; l < L; ++l) {
        const uint32_t Cl = C[l];
        const uint32_t e1 = (uint32_t)net.enc(l, 0) * 5, e2 = (uint32_t)net.enc(l, 1) * 5;
        // first convolution of encoder level l
        if (l == 0) put(e1 + 0, b.x0, kInPad, kInPad, 0);
        else put(e1 + 0, b.pool[l - 1], C[l - 1], C[l - 1], l);
        put(e1 + 1, b.e0[l], Cl, Cl, l);
        put(e1 + 2, b.tg[net.enc(l, 1)], Cl, Cl, l);
        put(e1 + 3, b.tz[net.enc(l, 0)], Cl, Cl, l);
        if (l > 0) put(e1 + 4, b.tg[net.enc(l, 0)], C[l - 1], C[l - 1], l);
        // second convolution
        put(e2 + 0, b.e0[l], Cl, Cl, l);
        if (l + 1 < L) put(e2 + 1, b.cat[l] + Cl, 2 * Cl, Cl, l);
        else put(e2 + 1, b.elast, Cl, Cl, l);
        if (l + 1 < L) put(e2 + 2, b.tp[l], Cl, Cl, l);
        else if (L > 1) put(e2 + 2, b.tg[net.dec(L - 2)], Cl, Cl, l);
        else put(e2 + 2, b.gh, Cl, Cl, l);
        put(e2 + 3, b.tz[net.enc(l, 1)], Cl, Cl, l);
        put(e2 + 4, b.tg[net.enc(l, 1)], Cl, Cl, l);
    }
    for (int l = (int)L - 2; l >= 0; --l) {
        const uint32_t Cl = C[l], Cu = C[l + 1];
        const uint32_t it = (uint32_t)net.dec((uint32_t)l);
        const uint32_t t5 = it * 5, c15 = (it + 1) * 5, c25 = (it + 2) * 5;
        // transposed convolution from level l + 1
        put(t5 + 0, l + 2 == (int)L ? b.elast : b.d1[l + 1], Cu, Cu, (uint32_t)l + 1);
        put(t5 + 1, b.cat[l], 2 * Cl, Cl, (uint32_t)l);
        put(t5 + 2, b.dcat[l], 2 * Cl, Cl, (uint32_t)l);
        put(t5 + 4, b.tg[it], Cu, Cu, (uint32_t)l + 1);
        // the level's two convolutions
        put(c15 + 0, b.cat[l], 2 * Cl, 2 * Cl, (uint32_t)l);
        put(c15 + 1, b.d0[l], Cl, Cl, (uint32_t)l);
        put(c15 + 2, b.tg[it + 2], Cl, Cl, (uint32_t)l);
        put(c15 + 3, b.tz[it + 1], Cl, Cl, (uint32_t)l);
        put(c15 + 4, b.dcat[l], 2 * Cl, 2 * Cl, (uint32_t)l);
        put(c25 + 0, b.d0[l], Cl, Cl, (uint32_t)l);
        put(c25 + 1, b.d1[l], Cl, Cl, (uint32_t)l);
        if (l == 0) put(c25 + 2, b.gh, Cl, Cl, 0);
        else put(c25 + 2, b.tg[net.dec((uint32_t)l - 1)], Cl, Cl, (uint32_t)l);
        put(c25 + 3, b.tz[it + 2], Cl, Cl, (uint32_t)l);
        put(c25 + 4, b.tg[it + 2], Cl, Cl, (uint32_t)l);
    }
    const uint32_t h5 = (uint32_t)net.head() * 5;
    put(h5 + 0, L > 1 ? b.d1[0] : b.elast, C[0], C[0], 0);
    put(h5 + 4, b.gh, C[0], C[0], 0);
    return n;
}

hipError_t fill(const Device& dev, uint32_t levels, const float* th, const uint32_t* rgba, const float* depth,
                const uint8_t* cov, uint32_t N, uint32_t H, uint32_t W, uint32_t* out, float* residual,
                void* ws, hipStream_t s)
{
    DevScope dscope(dev);
    Net net(levels);
    Bufs b;
    carve(net, N, H, W, false, (char*)ws, &b);
    const uint32_t P = N * H * W;
    {
        ProfScope ps(dev, "fill.misc", s);
        k_pack_input<<<blocks(P), dim3(kBlock), 0, s>>>(rgba, depth, cov, P, b.x0);
        FHV_TRY(hipGetLastError());
        FHV_TRY(prep_weights(net, th, false, b, s));
    }
    // the head runs in the epilogue of the last convolution
    const Layer& hd = net.layers[net.head()];
    const HeadFuse hf{th + hd.off_w, th + hd.off_b, rgba, out, residual};
    const uint16_t* hin = nullptr;
    return forward(net, th, b, N, H, W, s, &hin, &hf);
}

hipError_t train_step(const Device& dev, uint32_t levels, float* th, float* m, float* v, uint32_t step,
                      float lr, const uint32_t* rgba, const float* depth, const uint8_t* cov,
                      const uint32_t* tgt, uint32_t N, uint32_t H, uint32_t W, float* loss, float* grad_out,
                      void* ws, hipStream_t s, bool trace)
{
    DevScope dscope(dev);
    Net net(levels);
    Bufs b;
    carve(net, N, H, W, true, (char*)ws, &b, trace);
    if (grad_out) b.grad = grad_out;
    const uint32_t P = N * H * W;
    k_pack_input<<<blocks(P), dim3(kBlock), 0, s>>>(rgba, depth, cov, P, b.x0);
    FHV_TRY(hipGetLastError());
    FHV_TRY(prep_weights(net, th, true, b, s));
    const uint16_t* hin = nullptr;
    FHV_TRY(forward(net, th, b, N, H, W, s, &hin));
    const Layer& hd = net.layers[net.head()];
    const uint32_t hb = blocks(P);
    k_head_train<<<dim3(hb), dim3(kBlock), 0, s>>>(hin, th + hd.off_w, th + hd.off_b, rgba, tgt, P, b.gh,
                                                   b.hpart);
    FHV_TRY(hipGetLastError());
    // head weight and bias gradients, and the loss
    k_sum_splits<<<dim3(kHeadPart), dim3(kBlock), 0, s>>>(b.hpart, hb, kHeadPart, b.part);
    FHV_TRY(hipGetLastError());
    FHV_TRY(hipMemcpyAsync(b.grad + hd.off_w, b.part, sizeof(float) * 3 * kBase, hipMemcpyDeviceToDevice, s));
    FHV_TRY(hipMemcpyAsync(b.grad + hd.off_b, b.part + 3 * kBase, sizeof(float) * 3, hipMemcpyDeviceToDevice, s));
    if (loss) FHV_TRY(hipMemcpyAsync(loss, b.part + 3 * kBase + 3, sizeof(float), hipMemcpyDeviceToDevice, s));
    FHV_TRY(backward(net, th, b, N, H, W, s));
    if (step > 0) {   // step 0: gradients only
        const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
        k_adam<<<blocks(net.n_params), dim3(kBlock), 0, s>>>(th, m, v, b.grad, net.n_params, lr, c1, c2);
        FHV_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace nn
}  // namespace fhv
