// Learned k-space completion on gfx950: a 6-layer, 32-channel convolutional network on the
// per-bin (transmit angle x receive angle) pair grid of the Eq. 3 decomposition, trained and
// run with BF16 operands and FP32 accumulation on MFMA (v_mfma_f32_32x32x16_bf16).
//
// Grids are channel-last, x[b][h][w][c]: sample b (one bin of one frame), transmit angle h,
// receive angle w of a uniform bank, channel c.  The input grid holds, per bin, the observed
// pairs scaled by 1/scale (scale = root mean square of the observed pairs) in c = 0, 1 and the
// observation mask in c = 2 (c = 3..7 zero); the network predicts the unobserved pairs.
//
//   conv3x3   y[b][h][w][o] = bias[o] + sum_{t,c} W[t][o][c] x[b][h+dy*eh][w+dx*ew][c], t = 3(dy+1)
//             + (dx+1), dilation (eh, ew) per layer, zero outside the grid.  One wave = 32 grid positions of one row x 32
//             output channels: A = weights (rows = output channels, K = 16 (tap, channel)
//             pairs), B = input patch (K x 32 positions), 18 MFMAs for 32 input channels.
//   backward  input gradient = the same convolution of the output gradient with the
//             weights flipped in (dy, dx) and transposed in (o, c); the ReLU derivative is
//             applied on the fly from the stored activation.  Weight gradient: per workgroup a
//             run of grid rows, staged in LDS transposed (channels x positions; the input row
//             pre-shifted by dx so every MFMA operand read is one aligned 16-byte read), the
//             MFMA contracting over positions; the workgroups' partial sums are added in a
//             fixed order afterwards.
//   Adam      FP32 master parameters and moments; BF16 copies (plain and flipped/transposed)
//             rebuilt after every update.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>

#include "../../include/kk.h"
#include "kk_internal.h"

namespace kk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWidth = KK_NET_WIDTH;   // hidden channels
constexpr int kIn = KK_NET_IN;         // channels of the input grid in memory
constexpr int kLayers = KK_NET_LAYERS;
constexpr int kTaps = 9;
constexpr int kMaxGridW = 192;         // weight-gradient staging limit (LDS)

constexpr int kW0 = kTaps * kWidth * kIn;       // weights of layer 0 [9][32][8]
constexpr int kWn = kTaps * kWidth * kWidth;    // weights of layers 1..5 [9][32][32]
__host__ __device__ constexpr int layer_cin(int l) { return l == 0 ? kIn : kWidth; }
__host__ __device__ constexpr int layer_wsize(int l) { return l == 0 ? kW0 : kWn; }
// parameter offsets (floats): per layer W [9][32][cin] then bias [32]
__host__ __device__ constexpr int layer_poff(int l) { return l == 0 ? 0 : (kW0 + kWidth) + (l - 1) * (kWn + kWidth); }
constexpr int kParams = layer_poff(kLayers);
// BF16 weight offsets (elements): plain [9][32][cin] per layer, then flipped/transposed
// [9][32][32] for layers 1..5 (the input gradient of layer 0 is never needed)
__host__ __device__ constexpr int layer_koff(int l) { return l == 0 ? 0 : kW0 + (l - 1) * kWn; }
constexpr int kPlainBf16 = layer_koff(kLayers);
__host__ __device__ constexpr int layer_toff(int l) { return kPlainBf16 + (l - 1) * kWn; }
constexpr int kBf16Weights = kPlainBf16 + (kLayers - 1) * kTaps * kWidth * kWidth;

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
// state: params, m, v, grad (FP32), BF16 weights
constexpr size_t kStateParams = 0;
constexpr size_t kStateM = align256(kParams * 4);
constexpr size_t kStateV = kStateM + align256(kParams * 4);
constexpr size_t kStateG = kStateV + align256(kParams * 4);
constexpr size_t kStateW = kStateG + align256(kParams * 4);
constexpr size_t kStateBytes = kStateW + align256((size_t)kBf16Weights * 2);

__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_float(uint32_t b16) { return __builtin_bit_cast(float, b16 << 16); }

// keep the BF16 halves of word `x` whose counterpart in `m` is > 0
__device__ __forceinline__ uint32_t keep_positive(uint32_t x, uint32_t m) {
    const uint32_t lo = m & 0xFFFFu, hi = m >> 16;
    const uint32_t klo = ((lo & 0x8000u) == 0 && lo != 0) ? 0x0000FFFFu : 0u;
    const uint32_t khi = ((hi & 0x8000u) == 0 && hi != 0) ? 0xFFFF0000u : 0u;
    return x & (klo | khi);
}

constexpr int kRelu = 1, kBias = 2, kMaskIn = 4, kOutF32x2 = 8;

// One 3x3 convolution, 32 output channels, as described above.  in: [*][H][W][CIN] (row b of
// the batch is sample sidx[b] of `in`, or b), mask: [B][H][W][CIN] (kMaskIn), out: BF16
// [B][H][W][32] or, with kOutF32x2, FP32 [B][H][W][2] (channels 0, 1).
template <int CIN, int FLAGS>
__global__ __launch_bounds__(256) void conv3x3_kernel(const uint16_t* __restrict__ in, const int32_t* __restrict__ sidx,
                                                      const uint16_t* __restrict__ mask,
                                                      const uint16_t* __restrict__ wk,
                                                      const float* __restrict__ bias, void* __restrict__ out, int B,
                                                      int H, int W, int dh, int dw) {
    static_assert(CIN == 8 || CIN == 32, "input channels");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wtiles = (W + 31) >> 5;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= (int64_t)B * H * wtiles) return;  // whole wave; no barriers below
    const int wt = (int)(tile % wtiles);
    const int64_t bh = tile / wtiles;
    const int h = (int)(bh % H), b = (int)(bh / H);
    const int bs = sidx ? sidx[b] : b;
    const int col = lane & 31, half = lane >> 5;
    const int w = wt * 32 + col;
    constexpr int kSteps = CIN == 32 ? 2 * kTaps : (kTaps + 1) / 2;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        const int tap = CIN == 32 ? (s >> 1) : 2 * s + half;
        const int ci0 = CIN == 32 ? (s & 1) * 16 + half * 8 : 0;
        u32x4 a = {0u, 0u, 0u, 0u}, x = {0u, 0u, 0u, 0u};
        if (tap < kTaps) {
            a = *reinterpret_cast<const u32x4*>(wk + ((size_t)tap * kWidth + col) * CIN + ci0);
            const int hh = h + (tap / 3 - 1) * dh, ww = w + (tap % 3 - 1) * dw;
            if (hh >= 0 && hh < H && ww >= 0 && ww < W) {
                x = *reinterpret_cast<const u32x4*>(in + (((size_t)bs * H + hh) * W + ww) * CIN + ci0);
                if constexpr ((FLAGS & kMaskIn) != 0) {
                    const u32x4 m = *reinterpret_cast<const u32x4*>(mask + (((size_t)b * H + hh) * W + ww) * CIN + ci0);
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[j] = keep_positive(x[j], m[j]);
                }
            }
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, x), acc,
                                                      0, 0, 0);
    }
    if (w >= W) return;
    const size_t pos = ((size_t)b * H + h) * W + w;
    // lane holds position w and channels g*8 + half*4 + 0..3 in acc[g*4 + 0..3]
    if constexpr ((FLAGS & kOutF32x2) != 0) {
        if (half == 0) {
            float y0 = acc[0], y1 = acc[1];
            if constexpr ((FLAGS & kBias) != 0) {
                y0 += bias[0];
                y1 += bias[1];
            }
            reinterpret_cast<float2*>(out)[pos] = make_float2(y0, y1);
        }
    } else {
        uint16_t* o = static_cast<uint16_t*>(out) + pos * kWidth;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int c0 = g * 8 + half * 4;
            uint32_t p[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                float y0 = acc[g * 4 + 2 * j], y1 = acc[g * 4 + 2 * j + 1];
                if constexpr ((FLAGS & kBias) != 0) {
                    y0 += bias[c0 + 2 * j];
                    y1 += bias[c0 + 2 * j + 1];
                }
                if constexpr ((FLAGS & kRelu) != 0) {
                    y0 = fmaxf(y0, 0.f);
                    y1 = fmaxf(y1, 0.f);
                }
                p[j] = (uint32_t)bf16_bits(y0) | ((uint32_t)bf16_bits(y1) << 16);
            }
            *reinterpret_cast<uint2*>(o + c0) = make_uint2(p[0], p[1]);
        }
    }
}

// Weight and bias gradient partial sums of one 3x3 convolution over grid rows [r0, r1) of the
// batch (row = b * H + h): part[block][(t * 32 + o) * CIN + c] = sum g[b][h][w][o] x[b][h+dy][w+dx][c],
// part[block][9 * 32 * CIN + o] = sum g[b][h][w][o], with g = gout (masked by mask > 0 if given).
// Three waves; wave v owns the output tiles n = v, v+3, v+6 of the (tap, channel) columns.
template <int CIN>
__global__ __launch_bounds__(192) void wgrad_kernel(const uint16_t* __restrict__ gout, const uint16_t* __restrict__ mask,
                                                    const uint16_t* __restrict__ xin, const int32_t* __restrict__ sidx,
                                                    float* __restrict__ part, int B, int H, int W, int rows_per_block,
                                                    int dh, int dw) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[(kWidth + 9 * CIN) * (kMaxGridW + 8)];
    const int stride = W + 8;                     // BF16 elements per LDS row (16-byte pad)
    uint16_t* zT = smem;                          // [32][stride]: gradient, channel-major
    uint16_t* xT = smem + kWidth * stride;        // [3 dx][3 dy][CIN][stride]: shifted input rows
    constexpr int kN = kTaps * CIN;               // (tap, channel) columns
    constexpr int kTiles = (kN + 31) / 32;
    constexpr int kOwn = (kTiles + 2) / 3;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int col = lane & 31, half = lane >> 5;
    const int rows = B * H;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(rows, r0 + rows_per_block);
    floatx16 acc[kOwn];
#pragma unroll
    for (int u = 0; u < kOwn; ++u)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[u][v] = 0.f;
    float bsum = 0.f;  // thread tid < 32: bias gradient of channel tid
    for (int r = r0; r < r1; ++r) {
        const int b = r / H, h = r - (r / H) * H;
        const int bs = sidx ? sidx[b] : b;
        __syncthreads();  // previous row's operand reads are done
        // gradient row, transposed: two positions x 8 channels per item
        for (int it = tid; it < (W / 2) * 4; it += 192) {
            const int w = 2 * (it >> 2), cg = (it & 3) * 8;
            const size_t p = ((size_t)b * H + h) * W + w;
            u32x4 g0 = *reinterpret_cast<const u32x4*>(gout + p * kWidth + cg);
            u32x4 g1 = *reinterpret_cast<const u32x4*>(gout + (p + 1) * kWidth + cg);
            if (mask) {
                const u32x4 m0 = *reinterpret_cast<const u32x4*>(mask + p * kWidth + cg);
                const u32x4 m1 = *reinterpret_cast<const u32x4*>(mask + (p + 1) * kWidth + cg);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    g0[j] = keep_positive(g0[j], m0[j]);
                    g1[j] = keep_positive(g1[j], m1[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t e0 = (g0[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                const uint32_t e1 = (g1[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                *reinterpret_cast<uint32_t*>(zT + (cg + j) * stride + w) = e0 | (e1 << 16);
            }
        }
        // input rows h + dy eh (dy = -1, 0, 1), each stored three times shifted by dx ew:
        // xT[dx+1][dy+1][c][w] = x[h+dy*eh][w+dx*ew][c] (zero outside the grid)
        for (int it = tid; it < 9 * (W / 2) * (CIN / 8); it += 192) {
            const int cgi = it % (CIN / 8);
            const int rest = it / (CIN / 8);
            const int w = 2 * (rest % (W / 2));
            const int sh = rest / (W / 2);  // 0..8 = (dx+1) * 3 + (dy+1)
            const int dxi = sh / 3, dyi = sh - (sh / 3) * 3;
            const int hh = h + (dyi - 1) * dh;
            u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
            if (hh >= 0 && hh < H) {
                const int w0 = w + (dxi - 1) * dw, w1 = w0 + 1;
                const size_t rowp = ((size_t)bs * H + hh) * W;
                if (w0 >= 0 && w0 < W) v0 = *reinterpret_cast<const u32x4*>(xin + (rowp + w0) * CIN + cgi * 8);
                if (w1 >= 0 && w1 < W) v1 = *reinterpret_cast<const u32x4*>(xin + (rowp + w1) * CIN + cgi * 8);
            }
            uint16_t* dst = xT + ((size_t)sh * CIN + cgi * 8) * stride + w;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t e0 = (v0[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                const uint32_t e1 = (v1[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                *reinterpret_cast<uint32_t*>(dst + j * stride) = e0 | (e1 << 16);
            }
        }
        __syncthreads();
        if (tid < kWidth)
            for (int w = 0; w < W; w += 8) {
                const u32x4 z = *reinterpret_cast<const u32x4*>(zT + tid * stride + w);
#pragma unroll
                for (int j = 0; j < 4; ++j) bsum += bf16_float(z[j] & 0xFFFFu) + bf16_float(z[j] >> 16);
            }
        for (int p0 = 0; p0 < W; p0 += 16) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(zT + col * stride + p0 + 8 * half);
#pragma unroll
            for (int u = 0; u < kOwn; ++u) {
                const int n = (wave + 3 * u) * 32 + col;
                u32x4 x = {0u, 0u, 0u, 0u};
                if (wave + 3 * u < kTiles && n < kN) {
                    const int tap = n / CIN, c = n - (n / CIN) * CIN;
                    // tap = 3 (dy+1) + (dx+1) -> shifted copy (dx+1) * 3 + (dy+1)
                    const int sh = (tap % 3) * 3 + tap / 3;
                    x = *reinterpret_cast<const u32x4*>(xT + ((size_t)sh * CIN + c) * stride + p0 + 8 * half);
                }
                acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                                 __builtin_bit_cast(bf16x8, x), acc[u], 0, 0, 0);
            }
        }
    }
    float* pb = part + (size_t)blockIdx.x * (kN * kWidth + kWidth);
#pragma unroll
    for (int u = 0; u < kOwn; ++u) {
        const int n = (wave + 3 * u) * 32 + col;
        if (wave + 3 * u >= kTiles || n >= kN) continue;
        const int tap = n / CIN, c = n - (n / CIN) * CIN;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = (v >> 2) * 8 + half * 4 + (v & 3);
            pb[((size_t)tap * kWidth + o) * CIN + c] = acc[u][v];
        }
    }
    if (tid < kWidth) pb[kN * kWidth + tid] = bsum;
}

// dst[j] = sum over g of part[g * n + j].  A block covers kSumCols columns; its threads split
// the parts into 256 / kSumCols interleaved runs (g = r, r + runs, ...), each summed in order,
// and the runs are then added in run order: the same order on every call (deterministic), and
// many loads in flight per column instead of one chain of nparts dependent adds.
template <int kSumCols>
__global__ __launch_bounds__(256) void sum_parts_kernel(const float* __restrict__ part, int nparts, int n,
                                                        float* __restrict__ dst) {
    constexpr int kRuns = 256 / kSumCols;
    __shared__ float red[256];
    const int c = threadIdx.x % kSumCols, r = threadIdx.x / kSumCols;
    const int j = blockIdx.x * kSumCols + c;
    float s = 0.f;
    if (j < n)
        for (int g = r; g < nparts; g += kRuns) s += part[(size_t)g * n + j];
    red[r * kSumCols + c] = s;
    __syncthreads();
    if (r == 0 && j < n) {
        float t = red[c];
        for (int q = 1; q < kRuns; ++q) t += red[q * kSumCols + c];
        dst[j] = t;
    }
}

hipError_t sum_parts(const float* part, int nparts, int n, float* dst, hipStream_t st) {
    if (n >= 32)
        hipLaunchKernelGGL(sum_parts_kernel<32>, dim3((n + 31) / 32), dim3(256), 0, st, part, nparts, n, dst);
    else
        hipLaunchKernelGGL(sum_parts_kernel<1>, dim3(n), dim3(256), 0, st, part, nparts, n, dst);
    return hipGetLastError();
}

// Masked squared error of the network output against the target (unobserved pairs only):
// gout[p][0..1] = 2 u (out - target) inv_count, gout[p][2..31] = 0; part[block] = sum u |out - target|^2.
__global__ __launch_bounds__(256) void masked_loss_kernel(const float2* __restrict__ out, const float2* __restrict__ target,
                                                          const uint16_t* __restrict__ grid,
                                                          const int32_t* __restrict__ sidx, int B, int HW,
                                                          float inv_count, uint16_t* __restrict__ gout,
                                                          float* __restrict__ part) {
    __shared__ float red[256];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (p < (int64_t)B * HW) {
        const int b = (int)(p / HW), q = (int)(p - (int64_t)b * HW);
        const int bs = sidx ? sidx[b] : b;
        const size_t ps = (size_t)bs * HW + q;
        const bool observed = bf16_float(grid[ps * kIn + 2]) > 0.5f;
        const float2 y = out[p], t = target[ps];
        float gx = 0.f, gy = 0.f;
        if (!observed) {
            const float dx = y.x - t.x, dy = y.y - t.y;
            l = dx * dx + dy * dy;
            gx = 2.f * dx * inv_count;
            gy = 2.f * dy * inv_count;
        }
        uint32_t* g = reinterpret_cast<uint32_t*>(gout + p * kWidth);
        g[0] = (uint32_t)bf16_bits(gx) | ((uint32_t)bf16_bits(gy) << 16);
#pragma unroll
        for (int j = 1; j < kWidth / 2; ++j) g[j] = 0u;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void scale_kernel(float* __restrict__ x, float s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) x[0] *= s;
}

__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// BF16 weights from the FP32 parameters: plain [9][32][cin] per layer, and for layers 1..5 the
// flipped/transposed copy Wt[t][c][o] = W[8 - t][o][c] used by the input gradient.
__global__ void refresh_weights_kernel(const float* __restrict__ params, uint16_t* __restrict__ wk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kPlainBf16) {
        const int l = i < kW0 ? 0 : 1 + (i - kW0) / kWn;
        wk[i] = bf16_bits(params[layer_poff(l) + (i - layer_koff(l))]);
    } else if (i < kBf16Weights) {
        const int j = i - kPlainBf16;
        const int l = 1 + j / (kTaps * kWidth * kWidth);
        const int r = j - (l - 1) * kTaps * kWidth * kWidth;
        const int t = r / (kWidth * kWidth), c = (r / kWidth) % kWidth, o = r % kWidth;
        wk[i] = bf16_bits(params[layer_poff(l) + ((kTaps - 1 - t) * kWidth + o) * kWidth + c]);
    }
}

// Input grids (and targets) of B samples from a decomposition spectrum spec [H][Msrc][kpad]:
// sample b is bin k = bins[b] (or k_first + b); receive column w of the grid is observed when
// g2o[w] = j >= 0, its value then spec[h][obs_src[j]][k]; target (if not NULL) the full grid
// spec[h][w][k] (Msrc == W).  All values divided by the sample's scale.
__global__ __launch_bounds__(256) void prepare_kernel(const float2* __restrict__ spec, int H, int Msrc, int kpad,
                                                      const int32_t* __restrict__ bins, int k_first,
                                                      const int32_t* __restrict__ obs_src, int J,
                                                      const int32_t* __restrict__ g2o, int W,
                                                      uint16_t* __restrict__ grid, float2* __restrict__ target,
                                                      float* __restrict__ scale) {
    __shared__ float red[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int k = bins ? bins[b] : k_first + b;
    float s2 = 0.f;
    for (int q = tid; q < H * J; q += 256) {
        const int h = q / J, j = q - (q / J) * J;
        const float2 v = spec[((size_t)h * Msrc + obs_src[j]) * kpad + k];
        s2 += v.x * v.x + v.y * v.y;
    }
    red[tid] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const float ms = red[0] / (float)(H * J);
    const float sc = ms > 0.f ? sqrtf(ms) : 1.f;
    const float inv = 1.f / sc;
    if (tid == 0) scale[b] = sc;
    for (int q = tid; q < H * W; q += 256) {
        const int h = q / W, w = q - (q / W) * W;
        const int j = g2o[w];
        u32x4 e = {0u, 0u, 0u, 0u};
        if (j >= 0) {
            const float2 v = spec[((size_t)h * Msrc + obs_src[j]) * kpad + k];
            e[0] = (uint32_t)bf16_bits(v.x * inv) | ((uint32_t)bf16_bits(v.y * inv) << 16);
            e[1] = (uint32_t)bf16_bits(1.f);
        }
        const size_t p = (size_t)b * H * W + q;
        *reinterpret_cast<u32x4*>(grid + p * kIn) = e;
        if (target) {
            const float2 v = spec[((size_t)h * Msrc + w) * kpad + k];
            target[p] = make_float2(v.x * inv, v.y * inv);
        }
    }
}

// Completed spectrum: dst[h][w][k] = observed ? spec[h][obs_src[g2o[w]]][k] : out * scale.
__global__ void merge_kernel(const float2* __restrict__ out, const float* __restrict__ scale,
                             const int32_t* __restrict__ bins, int k_first, int B, const float2* __restrict__ spec,
                             int H, int Msrc, int kpad, const int32_t* __restrict__ obs_src,
                             const int32_t* __restrict__ g2o, int W, float2* __restrict__ dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)B * H * W) return;
    const int b = (int)(p / ((int64_t)H * W));
    const int q = (int)(p - (int64_t)b * H * W);
    const int h = q / W, w = q - (q / W) * W;
    const int k = bins ? bins[b] : k_first + b;
    const int j = g2o[w];
    float2 v;
    if (j >= 0) {
        v = spec[((size_t)h * Msrc + obs_src[j]) * kpad + k];
    } else {
        const float2 y = out[p];
        const float s = scale[b];
        v = make_float2(y.x * s, y.y * s);
    }
    dst[((size_t)h * W + w) * kpad + k] = v;
}

__global__ void zero_bytes_kernel(uint4* __restrict__ p, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ------------------------------------------------------------------------------- host side

struct NetWs {
    size_t act, out, g0, g1, part, loss, total;
    int wg_blocks, rows_per_block;
};

size_t act_bytes(int B, int H, int W) { return (size_t)B * H * W * kWidth * 2; }

bool net_ws(int B, int H, int W, NetWs* w) {
    if (B < 1 || H < 1 || W < 16 || W > kMaxGridW || (W % 16) != 0) return false;
    const int rows = B * H;
    w->wg_blocks = rows < 256 ? rows : 256;
    w->rows_per_block = (rows + w->wg_blocks - 1) / w->wg_blocks;
    w->wg_blocks = (rows + w->rows_per_block - 1) / w->rows_per_block;
    const size_t a = align256(act_bytes(B, H, W));
    w->act = 0;                                              // activations of layers 1..5
    w->out = w->act + (kLayers - 1) * a;                     // FP32 [B][H][W][2]
    w->g0 = w->out + align256((size_t)B * H * W * 8);        // gradient ping-pong (BF16)
    w->g1 = w->g0 + a;
    w->part = w->g1 + a;                                     // weight-gradient partials
    w->loss = w->part + align256((size_t)w->wg_blocks * (kTaps * kWidth * kWidth + kWidth) * 4);
    const size_t loss_blocks = ((size_t)B * H * W + 255) / 256;
    w->total = w->loss + align256(loss_blocks * 4);
    return true;
}


// per-layer dilations (eh, ew) from the caller's array, or all 1; false when out of range
bool read_dilation(const int32_t* d, int* out) {
    for (int i = 0; i < 2 * kLayers; ++i) {
        out[i] = d ? d[i] : 1;
        if (out[i] < 1 || out[i] > 64) return false;
    }
    return true;
}

hipError_t conv(int l, int flags, const uint16_t* in, const int32_t* sidx, const uint16_t* mask, const uint16_t* wk,
                const float* bias, void* out, int B, int H, int W, int dh, int dw, hipStream_t st) {
    const int64_t tiles = (int64_t)B * H * ((W + 31) / 32);
    const dim3 g((unsigned)((tiles + 3) / 4)), blk(256);
    if (l == 0) {
        hipLaunchKernelGGL((conv3x3_kernel<kIn, kRelu | kBias>), g, blk, 0, st, in, sidx, mask, wk, bias, out, B, H, W, dh, dw);
    } else if (flags == (kRelu | kBias)) {
        hipLaunchKernelGGL((conv3x3_kernel<kWidth, kRelu | kBias>), g, blk, 0, st, in, sidx, mask, wk, bias, out, B, H,
                           W, dh, dw);
    } else if (flags == (kBias | kOutF32x2)) {
        hipLaunchKernelGGL((conv3x3_kernel<kWidth, kBias | kOutF32x2>), g, blk, 0, st, in, sidx, mask, wk, bias, out, B,
                           H, W, dh, dw);
    } else if (flags == kMaskIn) {
        hipLaunchKernelGGL((conv3x3_kernel<kWidth, kMaskIn>), g, blk, 0, st, in, sidx, mask, wk, bias, out, B, H, W, dh, dw);
    } else if (flags == 0) {
        hipLaunchKernelGGL((conv3x3_kernel<kWidth, 0>), g, blk, 0, st, in, sidx, mask, wk, bias, out, B, H, W, dh, dw);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t forward(const unsigned char* state, const uint16_t* grid, const int32_t* sidx, int B, int H, int W,
                   const int* dil, unsigned char* ws, const NetWs& w, float* out, hipStream_t st) {
    const float* params = reinterpret_cast<const float*>(state + kStateParams);
    const uint16_t* wk = reinterpret_cast<const uint16_t*>(state + kStateW);
    const size_t a = align256(act_bytes(B, H, W));
    const uint16_t* x = grid;
    for (int l = 0; l < kLayers; ++l) {
        const float* bias = params + layer_poff(l) + layer_wsize(l);
        hipError_t e;
        if (l < kLayers - 1) {
            uint16_t* y = reinterpret_cast<uint16_t*>(ws + w.act + l * a);
            e = conv(l, kRelu | kBias, x, l == 0 ? sidx : nullptr, nullptr, wk + layer_koff(l), bias, y, B, H, W,
                     dil[2 * l], dil[2 * l + 1], st);
            x = y;
        } else {
            e = conv(l, kBias | kOutF32x2, x, nullptr, nullptr, wk + layer_koff(l), bias, out, B, H, W, dil[2 * l],
                     dil[2 * l + 1], st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t wgrad(int l, const uint16_t* g, const uint16_t* mask, const uint16_t* x, const int32_t* sidx, float* part,
                 float* dst, int B, int H, int W, int dh, int dw, const NetWs& w, hipStream_t st) {
    if (layer_cin(l) == kIn)
        hipLaunchKernelGGL(wgrad_kernel<kIn>, dim3(w.wg_blocks), dim3(192), 0, st, g, mask, x, sidx, part, B, H, W,
                           w.rows_per_block, dh, dw);
    else
        hipLaunchKernelGGL(wgrad_kernel<kWidth>, dim3(w.wg_blocks), dim3(192), 0, st, g, mask, x, sidx, part, B, H,
                           W, w.rows_per_block, dh, dw);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    return sum_parts(part, w.wg_blocks, layer_wsize(l) + kWidth, dst, st);
}

}  // namespace
}  // namespace kk

extern "C" {

size_t kk_net_param_count(void) { return (size_t)kk::kParams; }

size_t kk_net_state_bytes(void) { return kk::kStateBytes; }

int32_t kk_net_load(void* state, const float* params_host, void* stream) {
    using namespace kk;
    if (!state || !params_host) return KK_E_NULL;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* s = static_cast<unsigned char*>(state);
    if (hipMemcpyAsync(s + kStateParams, params_host, (size_t)kParams * 4, hipMemcpyHostToDevice, st) != hipSuccess)
        return KK_E_HIP;
    // moments and gradient to zero (a kernel, like every other write of the state)
    const int64_t n16 = (int64_t)(kStateW - kStateM) / 16;
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<uint4*>(s + kStateM), n16);
    hipLaunchKernelGGL(refresh_weights_kernel, dim3((kBf16Weights + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const float*>(s + kStateParams), reinterpret_cast<uint16_t*>(s + kStateW));
    if (hipGetLastError() != hipSuccess) return KK_E_HIP;
    return hipStreamSynchronize(st) == hipSuccess ? KK_OK : KK_E_HIP;
}

size_t kk_net_workspace_bytes(int32_t B, int32_t H, int32_t W) {
    kk::NetWs w;
    return kk::net_ws(B, H, W, &w) ? w.total : 0;
}

int32_t kk_net_prepare(const float* spec, int32_t H, int32_t Msrc, int32_t kpad, const int32_t* bins, int32_t k_first,
                       int32_t B, const int32_t* obs_src, int32_t J, const int32_t* grid_to_obs, int32_t W,
                       uint16_t* grid, float* target, float* scale, void* stream) {
    using namespace kk;
    if (!spec || !obs_src || !grid_to_obs || !grid || !scale) return KK_E_NULL;
    if (H < 1 || Msrc < 1 || kpad < 1 || B < 1 || J < 1 || W < 1 || (target && Msrc != W) ||
        (!bins && (k_first < 0 || k_first + B > kpad)))
        return KK_E_ARG;
    hipLaunchKernelGGL(prepare_kernel, dim3(B), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(spec), H, Msrc, kpad, bins, k_first, obs_src, J, grid_to_obs, W,
                       grid, reinterpret_cast<float2*>(target), scale);
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_net_forward(const void* state, const uint16_t* grid, const int32_t* sidx, int32_t B, int32_t H, int32_t W,
                       const int32_t* dilation, float* out, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!state || !grid || !out || !ws) return KK_E_NULL;
    NetWs w;
    int dil[2 * kLayers];
    if (!net_ws(B, H, W, &w) || !read_dilation(dilation, dil)) return KK_E_ARG;
    if (ws_bytes < w.total) return KK_E_WORKSPACE;
    return forward(static_cast<const unsigned char*>(state), grid, sidx, B, H, W, dil, static_cast<unsigned char*>(ws),
                   w, out, (hipStream_t)stream) == hipSuccess
               ? KK_OK
               : KK_E_HIP;
}

int32_t kk_net_backward(void* state, const uint16_t* grid, const float* target, const int32_t* sidx, int32_t B,
                        int32_t H, int32_t W, const int32_t* dilation, float inv_count, float* loss, void* ws,
                        size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!state || !grid || !target || !loss || !ws) return KK_E_NULL;
    NetWs w;
    int dil[2 * kLayers];
    if (!net_ws(B, H, W, &w) || !read_dilation(dilation, dil)) return KK_E_ARG;
    if (!(inv_count > 0.f)) return KK_E_ARG;
    if (ws_bytes < w.total) return KK_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* s = static_cast<unsigned char*>(state);
    unsigned char* wsb = static_cast<unsigned char*>(ws);
    float* grad = reinterpret_cast<float*>(s + kStateG);
    const uint16_t* wk = reinterpret_cast<const uint16_t*>(s + kStateW);
    float* out = reinterpret_cast<float*>(wsb + w.out);
    const size_t a = align256(act_bytes(B, H, W));
    auto act = [&](int l) -> const uint16_t* {  // output of layer l (0-based), l < kLayers - 1
        return reinterpret_cast<const uint16_t*>(wsb + w.act + l * a);
    };
    if (forward(s, grid, sidx, B, H, W, dil, wsb, w, out, st) != hipSuccess) return KK_E_HIP;
    const int HW = H * W;
    const int lblocks = (int)(((int64_t)B * HW + 255) / 256);
    uint16_t* g[2] = {reinterpret_cast<uint16_t*>(wsb + w.g0), reinterpret_cast<uint16_t*>(wsb + w.g1)};
    float* lpart = reinterpret_cast<float*>(wsb + w.loss);
    hipLaunchKernelGGL(masked_loss_kernel, dim3(lblocks), dim3(256), 0, st, reinterpret_cast<const float2*>(out),
                       reinterpret_cast<const float2*>(target), grid, sidx, B, HW, inv_count, g[0], lpart);
    if (sum_parts(lpart, lblocks, 1, loss, st) != hipSuccess) return KK_E_HIP;
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(64), 0, st, loss, inv_count);
    float* part = reinterpret_cast<float*>(wsb + w.part);
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        // g[cur]: gradient at layer l's output (before its ReLU derivative)
        const uint16_t* mask = l < kLayers - 1 ? act(l) : nullptr;
        const uint16_t* x = l > 0 ? act(l - 1) : grid;
        const int dh = dil[2 * l], dw = dil[2 * l + 1];
        if (wgrad(l, g[cur], mask, x, l > 0 ? nullptr : sidx, part, grad + layer_poff(l), B, H, W, dh, dw, w, st) !=
            hipSuccess)
            return KK_E_HIP;
        if (l > 0) {
            // the input gradient is the convolution with the flipped, transposed weights at the
            // same dilation
            if (conv(l, mask ? kMaskIn : 0, g[cur], nullptr, mask, wk + layer_toff(l), nullptr, g[1 - cur], B, H, W,
                     dh, dw, st) != hipSuccess)
                return KK_E_HIP;
            cur = 1 - cur;
        }
    }
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_net_adam(void* state, int32_t step, float lr, void* stream) {
    using namespace kk;
    if (!state) return KK_E_NULL;
    if (step < 1 || !(lr > 0.f)) return KK_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* s = static_cast<unsigned char*>(state);
    float* params = reinterpret_cast<float*>(s + kStateParams);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, step))), c2 = (float)(1.0 / (1.0 - std::pow(0.999, step)));
    hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, params,
                       reinterpret_cast<float*>(s + kStateM), reinterpret_cast<float*>(s + kStateV),
                       reinterpret_cast<const float*>(s + kStateG), kParams, lr, b1, b2, eps, c1, c2);
    hipLaunchKernelGGL(refresh_weights_kernel, dim3((kBf16Weights + 255) / 256), dim3(256), 0, st, params,
                       reinterpret_cast<uint16_t*>(s + kStateW));
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_net_train_step(void* state, const uint16_t* grid, const float* target, const int32_t* sidx, int32_t B,
                          int32_t H, int32_t W, const int32_t* dilation, float inv_count, int32_t step, float lr,
                          float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (step < 1 || !(lr > 0.f)) return KK_E_ARG;
    const int32_t rc =
        kk_net_backward(state, grid, target, sidx, B, H, W, dilation, inv_count, loss, ws, ws_bytes, stream);
    return rc != KK_OK ? rc : kk_net_adam(state, step, lr, stream);
}

int32_t kk_net_read(const void* state, int32_t what, float* host, void* stream) {
    using namespace kk;
    if (!state || !host) return KK_E_NULL;
    size_t off;
    switch (what) {
        case KK_NET_PARAMS: off = kStateParams; break;
        case KK_NET_GRADS: off = kStateG; break;
        case KK_NET_MOMENT1: off = kStateM; break;
        case KK_NET_MOMENT2: off = kStateV; break;
        default: return KK_E_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(host, static_cast<const unsigned char*>(state) + off, (size_t)kParams * 4,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

int32_t kk_net_merge(const float* out, const float* scale, const int32_t* bins, int32_t k_first, int32_t B,
                     const float* spec, int32_t H, int32_t Msrc, int32_t kpad, const int32_t* obs_src,
                     const int32_t* grid_to_obs, int32_t W, float* dst, void* stream) {
    using namespace kk;
    if (!out || !scale || !spec || !obs_src || !grid_to_obs || !dst) return KK_E_NULL;
    if (B < 1 || H < 1 || Msrc < 1 || W < 1 || kpad < 1 || (!bins && (k_first < 0 || k_first + B > kpad)))
        return KK_E_ARG;
    const int64_t n = (int64_t)B * H * W;
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(out), scale, bins, k_first, B,
                       reinterpret_cast<const float2*>(spec), H, Msrc, kpad, obs_src, grid_to_obs, W,
                       reinterpret_cast<float2*>(dst));
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_clear(void* dev, size_t bytes, void* stream) {
    if (!dev) return KK_E_NULL;
    if ((bytes & 15) != 0 || (reinterpret_cast<uintptr_t>(dev) & 15) != 0) return KK_E_ARG;
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return KK_OK;
    hipLaunchKernelGGL(kk::zero_bytes_kernel, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       static_cast<uint4*>(dev), n16);
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

}  // extern "C"
