// Eq. 3 receive plane-wave decomposition on gfx950, evaluated in the temporal-frequency
// domain (Sec. II-F):
//   1. analytic spectra of the N*L zero-padded records (kk_fft.hip, two records per FFT),
//      stored bin-blocked X[k/8][i][l][k%8];
//   2. per bin k the complex contraction Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] with
//      W_k[o][l] = exp(2 pi i r / (n 2^22)), r = (k shift[o][l]) mod (n 2^22), on MFMA
//      (v_mfma_f32_32x32x2_f32: one complex element l per instruction, 16 receive angles x
//      {Re, Im} rows by 32 transmit columns, 8 bins per workgroup held in 8 accumulator tiles);
//   3. inverse FFT of each (i, o) spectrum, first T samples.
// The phase is formed exactly in integers; only the reduced fraction becomes floating point:
// W = E[r >> 22] * exp(2 pi i (r mod 2^22) / (n 2^22)), with E[m] = exp(2 pi i m / n) from the
// FP64-evaluated table and the small second factor (|angle| < 2 pi / n) by its Taylor series.
// Also the DAS comparator entry point (analytic channel data + delay-gather).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kContractThreads = 256;  // 4 waves split the element sum

template <int LOG2N>
__global__ __launch_bounds__(kContractThreads) void contract_kernel(const float2* __restrict__ X,
                                                                     const int32_t* __restrict__ shift,
                                                                     const float2* __restrict__ tw,
                                                                     float2* __restrict__ Y, int ntx, int M,
                                                                     int L, int ncol, int K, int kpad) {
    constexpr int N = 1 << LOG2N;
    constexpr int64_t kMask = (int64_t(1) << (22 + LOG2N)) - 1;
    constexpr float kFine = 6.283185307179586f / (float)N / 4194304.0f;  // 2 pi / (n 2^22)
    __shared__ float2 tab[N];                                             // exp(+2 pi i m / n)
    __shared__ float red[2][kBinBlock][16][64];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int kb = blockIdx.x, rt = blockIdx.y, ct = blockIdx.z;
    for (int m = tid; m < N; m += kContractThreads) {
        const float2 w = tw[m];
        tab[m] = make_float2(w.x, -w.y);
    }
    __syncthreads();

    // B operand (2 x 32): lane -> (part = lane / 32 in {Re, Im}, transmit column lane % 32)
    const int part = lane >> 5;
    const int i = ct * 32 + (lane & 31);
    // A operand (32 x 2): lane -> row lane % 32 = {Re rows 0..15, Im rows 16..31} x 16 angles
    const int row = lane & 31;
    const int ytype = row >> 4;
    const int o = rt * 16 + (row & 15);
    const bool ovalid = o < M;
    const float sgn = (ytype == part) ? 1.0f : (ytype == 0 ? -1.0f : 1.0f);  // Wr, -Wi, Wi, Wr
    const bool use_re = (ytype == part);

    floatx16 acc[kBinBlock];
#pragma unroll
    for (int kk = 0; kk < kBinBlock; ++kk)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[kk][v] = 0.0f;

    for (int l = wave; l < L; l += 4) {
        const float4* src = reinterpret_cast<const float4*>(X + (((size_t)kb * ncol + i) * L + l) * kBinBlock);
        float bv[kBinBlock];
#pragma unroll
        for (int h = 0; h < kBinBlock / 2; ++h) {
            const float4 q = src[h];
            bv[2 * h] = part ? q.y : q.x;
            bv[2 * h + 1] = part ? q.w : q.z;
        }
        const int64_t s = ovalid ? (int64_t)shift[(size_t)o * L + l] : 0;
#pragma unroll
        for (int kk = 0; kk < kBinBlock; ++kk) {
            const int64_t k = (int64_t)kb * kBinBlock + kk;
            const int64_t r = (k * s) & kMask;
            const float2 e = tab[(int)(r >> 22)];
            const float ph = (float)(int)(r & 0x3FFFFF) * kFine;
            const float p2 = ph * ph;
            const float cf = 1.0f - p2 * (0.5f - p2 * (1.0f / 24.0f));
            const float sf = ph * (1.0f - p2 * (1.0f / 6.0f));
            const float wr = e.x * cf - e.y * sf;
            const float wi = e.x * sf + e.y * cf;
            const float a = ovalid ? sgn * (use_re ? wr : wi) : 0.0f;
            acc[kk] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv[kk], acc[kk], 0, 0, 0);
        }
    }
    // sum the four element subsets
    if (wave >= 2) {
#pragma unroll
        for (int kk = 0; kk < kBinBlock; ++kk)
#pragma unroll
            for (int v = 0; v < 16; ++v) red[wave - 2][kk][v][lane] = acc[kk][v];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int kk = 0; kk < kBinBlock; ++kk)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[kk][v] += red[wave][kk][v][lane];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int kk = 0; kk < kBinBlock; ++kk)
#pragma unroll
            for (int v = 0; v < 16; ++v) red[0][kk][v][lane] = acc[kk][v];
    }
    __syncthreads();
    if (wave != 0 || i >= ntx) return;
    // accumulator v of lane holds row (v/4)*8 + (lane/32)*4 + v%4, column lane%32; rows v and
    // v + 8 are Re and Im of the same receive angle
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int ol = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int oo = rt * 16 + ol;
        if (oo < M) {
            float2* dst = Y + ((size_t)i * M + oo) * kpad + (size_t)kb * kBinBlock;
#pragma unroll
            for (int kk = 0; kk < kBinBlock; ++kk) {
                if (kb * kBinBlock + kk < K)
                    dst[kk] = make_float2(acc[kk][v] + red[0][kk][v][lane], acc[kk][v + 8] + red[0][kk][v + 8][lane]);
            }
        }
    }
}

template <int LOG2N>
hipError_t contract(const float2* X, const int32_t* shift, const float2* tw, float2* Y, int ntx, int M, int L,
                    int ncol, int K, int kpad, hipStream_t st) {
    const dim3 grid(kpad / kBinBlock, (M + 15) / 16, ncol / 32);
    hipLaunchKernelGGL((contract_kernel<LOG2N>), grid, dim3(kContractThreads), 0, st, X, shift, tw, Y, ntx, M, L,
                       ncol, K, kpad);
    return hipGetLastError();
}

hipError_t launch_contract(int log2n, const float2* X, const int32_t* shift, const float2* tw, float2* Y, int ntx,
                           int M, int L, int ncol, int K, int kpad, hipStream_t st) {
    switch (log2n) {
        case 8: return contract<8>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        case 9: return contract<9>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        case 10: return contract<10>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        case 11: return contract<11>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        case 12: return contract<12>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        case 13: return contract<13>(X, shift, tw, Y, ntx, M, L, ncol, K, kpad, st);
        default: return hipErrorInvalidValue;
    }
}

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct DecomposeLayout {
    int log2n, K, kpad, ncol;
    size_t tw_off, x_off, y_off, total;
};

bool decompose_layout(const kk_geom* g, int32_t N, int32_t M, int32_t tpad, DecomposeLayout* d) {
    const int lg = log2_exact(tpad);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->T < 1 || g->T > tpad || g->L < 1 || N < 1 || M < 1) return false;
    d->log2n = lg;
    d->K = tpad / 2 + 1;
    d->kpad = (d->K + kBinBlock - 1) / kBinBlock * kBinBlock;
    d->ncol = (N + 31) / 32 * 32;
    d->tw_off = 0;
    d->x_off = align256((size_t)tpad * 8);
    d->y_off = d->x_off + align256((size_t)d->kpad * d->ncol * g->L * 8);
    d->total = d->y_off + align256((size_t)N * M * d->kpad * 8);
    return true;
}

struct DasLayout {
    int log2n, kpad;
    size_t tw_off, x_off, a_off, total;
};

bool das_layout(const kk_geom* g, int32_t N, DasLayout* d) {
    int64_t tp = 1;
    while (tp < g->T) tp *= 2;
    const int lg = log2_exact(tp);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->L < 1 || N < 1) return false;
    d->log2n = lg;
    d->kpad = (int)(tp / 2 + 1 + 7) / 8 * 8;
    d->tw_off = 0;
    d->x_off = align256((size_t)tp * 8);
    d->a_off = d->x_off + align256((size_t)N * g->L * d->kpad * 8);
    d->total = d->a_off + align256((size_t)N * g->L * g->T * 8);
    return true;
}

}  // namespace
}  // namespace kk

extern "C" {

size_t kk_decompose_workspace_bytes(const kk_geom* g, int32_t N, int32_t M, int32_t tpad, int32_t precision) {
    kk::DecomposeLayout d;
    if (!g || precision != KK_PREC_FP32 || !kk::decompose_layout(g, N, M, tpad, &d)) return 0;
    return d.total;
}

int32_t kk_decompose(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M, int32_t tpad,
                     int32_t precision, float* rf_theta, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf || !g || !shift_q || !rf_theta || !ws) return KK_E_NULL;
    if (precision != KK_PREC_FP32) return KK_E_UNSUPPORTED;
    if (N < 1 || M < 1 || g->L < 1 || g->L > 65536 || g->T < 1) return KK_E_ARG;
    DecomposeLayout d;
    if (!decompose_layout(g, N, M, tpad, &d)) return KK_E_ARG;
    if ((int64_t)N * g->L > 0x7fffffff || (int64_t)N * M > 0x7fffffff) return KK_E_ARG;
    if (ws_bytes < d.total) return KK_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* w = static_cast<unsigned char*>(ws);
    float2* tw = reinterpret_cast<float2*>(w + d.tw_off);
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    float2* Y = reinterpret_cast<float2*>(w + d.y_off);
    if (launch_twiddles(tw, d.log2n, st) != hipSuccess) return KK_E_HIP;
    if (launch_fft_forward(rf, N * g->L, g->T, d.log2n, tw, X, true, g->L, d.ncol, d.kpad, st) != hipSuccess)
        return KK_E_HIP;
    if (launch_contract(d.log2n, X, shift_q, tw, Y, N, M, g->L, d.ncol, d.K, d.kpad, st) != hipSuccess)
        return KK_E_HIP;
    if (launch_fft_inverse(Y, N * M, d.kpad, d.log2n, tw, reinterpret_cast<float2*>(rf_theta), g->T, st) !=
        hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

size_t das_workspace_bytes(const kk_geom* g, int32_t N) {
    kk::DasLayout d;
    if (!g || !kk::das_layout(g, N, &d)) return 0;
    return d.total;
}

int32_t das_beamform(const int16_t* rf, int32_t N, const kk_geom* g, const void* plan_host, const void* plan_dev,
                     size_t plan_bytes, float* image, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf || !g || !plan_host || !plan_dev || !image || !ws) return KK_E_NULL;
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (plan_bytes < (size_t)PW_HEADER_WORDS * 4 || h[PW_MAGIC] != kPlanMagic || h[PW_KIND] != kPlanKindDAS ||
        (size_t)h[PW_TOTAL] * 4 > plan_bytes || h[PW_PB] != pairs_per_batch(h[PW_CAP]))
        return KK_E_WORKSPACE;
    if (N < 1 || h[PW_N] != N || h[PW_M] != g->L || h[PW_T] != g->T) return KK_E_ARG;
    DasLayout d;
    if (!das_layout(g, N, &d)) return KK_E_ARG;
    if (ws_bytes < d.total) return KK_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* w = static_cast<unsigned char*>(ws);
    float2* tw = reinterpret_cast<float2*>(w + d.tw_off);
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    float2* A = reinterpret_cast<float2*>(w + d.a_off);
    const int ntr = N * g->L;
    if (launch_twiddles(tw, d.log2n, st) != hipSuccess) return KK_E_HIP;
    if (launch_fft_forward(rf, ntr, g->T, d.log2n, tw, X, false, g->L, 0, d.kpad, st) != hipSuccess) return KK_E_HIP;
    if (launch_fft_inverse(X, ntr, d.kpad, d.log2n, tw, A, g->T, st) != hipSuccess) return KK_E_HIP;
    if (launch_das_gather(A, h, static_cast<const int32_t*>(plan_dev), reinterpret_cast<float2*>(image), st) !=
        hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

}  // extern "C"
