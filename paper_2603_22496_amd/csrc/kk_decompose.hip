// Eq. 3 receive plane-wave decomposition on gfx950, evaluated in the temporal-frequency
// domain (Sec. II-F):
//   1. analytic spectra of the N*L zero-padded records (kk_fft.hip, two records per FFT),
//      stored bin-blocked X[k/8][i][l][k%8];
//   2. per bin k the complex contraction Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] with
//      W_k[o][l] = exp(2 pi i r / (n 2^22)), r = (k shift[o][l]) mod (n 2^22), on MFMA
//      (v_mfma_f32_32x32x2_f32: one complex element l per instruction, 16 receive angles x
//      {Re, Im} rows by 32 transmit columns; 8 bins per workgroup, one per wave, the spectrum
//      staged through LDS 16 elements at a time);
//   3. inverse FFT of each (i, o) spectrum, first T samples.
// The phase is formed exactly in integers; only the reduced fraction becomes floating point:
// W = E[r >> 22] * exp(2 pi i (r mod 2^22) / (n 2^22)), with E[m] = exp(2 pi i m / n) tabulated
// per workgroup from two FP64-evaluated factors and the small second factor (|angle| < 2 pi / n)
// by its Taylor series.
// Also the DAS comparator entry point (analytic channel data + delay-gather).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kContractWaves = kBinBlock;   // one bin of the block per wave
constexpr int kContractThreads = kContractWaves * 64;
constexpr int kChunkL = 16;                  // elements per LDS chunk
constexpr int kRowFloats = kChunkL * kBinBlock * 2 + 4;  // one transmit column + pad (16-byte rows)

// exp(+2 pi i ((k s) mod (n 2^22)) / (n 2^22)) for 0 <= k < 2^23, any int32 s: the turn count
// is reduced exactly with 24-bit products (k s = k s_hi 2^22 + k s_lo, s_lo < 2^22), the coarse
// part m / n is the product of the two factor tables and the remaining fraction (< 1/n turn)
// comes from its Taylor series.
template <int LOG2N>
__device__ __forceinline__ float2 shear_phase(uint32_t k, int32_t s, const float2* fac) {
    constexpr float kFine = 6.283185307179586f / (float)(1 << LOG2N) / 4194304.0f;
    const uint32_t s_lo = (uint32_t)s & 0x3FFFFFu;
    const int32_t s_hi = s >> 22;
    const uint64_t p = (uint64_t)(k & 0xFFFFFFu) * (uint64_t)s_lo;         // 24 x 22-bit product
    const uint32_t plo = (uint32_t)p;
    const uint32_t coarse = ((uint32_t)(p >> 22) + (uint32_t)__mul24((int)k, s_hi)) & ((1u << LOG2N) - 1);
    const float ph = (float)(plo & 0x3FFFFFu) * kFine;
    const float p2 = ph * ph;
    const float cf = __builtin_fmaf(p2, __builtin_fmaf(p2, 1.0f / 24.0f, -0.5f), 1.0f);
    const float sf = ph * __builtin_fmaf(p2, -1.0f / 6.0f, 1.0f);
    const float2 a = fac[coarse >> (LOG2N - 6)], b = fac[64 + (coarse & ((1u << (LOG2N - 6)) - 1))];
    const float2 e = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
    return make_float2(e.x * cf - e.y * sf, e.x * sf + e.y * cf);
}

// exp(+2 pi i m / n) = exp(2 pi i (m >> (log2n - 6)) / 64) exp(2 pi i (m mod n/64) / n): the
// two factor tables, evaluated in FP64
template <int LOG2N>
__device__ __forceinline__ void build_phase_factors(float2* fac, int tid) {
    constexpr int N = 1 << LOG2N;
    if (tid < 64 + N / 64) {
        double sn, cs;
        sincospi(tid < 64 ? 2.0 * tid / 64.0 : 2.0 * (tid - 64) / (double)N, &sn, &cs);
        fac[tid] = make_float2((float)cs, (float)sn);
    }
}

// Global loads of one chunk: spectrum X[kb][i][l0 .. l0+15][0..7] (a contiguous 1 KiB run per
// transmit column i) and the shifts of 4 (receive angle, element) entries per thread.
struct ContractStage {
    float4 v[4];
    int32_t s[4];
};

__device__ __forceinline__ void contract_load(ContractStage& st, const float2* __restrict__ X,
                                              const int32_t* __restrict__ shift, int kb, int ncol, int ct, int L,
                                              int l0, int M, int rt, int tid) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int f = tid + u * kContractThreads;  // float4 index in the 32 x 64 chunk
        const int i = f >> 6, j = f & 63;          // column, float4 within the column's run
        const int l = l0 + (j >> 2);
        st.v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (l < L)
            st.v[u] = reinterpret_cast<const float4*>(X + (((size_t)kb * ncol + ct * 32 + i) * L + l) * kBinBlock)[j & 3];
        // phase entry e = (l_local, bin, angle) of this thread: angle fastest
        const int e = tid + u * kContractThreads;
        const int ol = e & 15, ll = e >> 7;
        const int o = rt * 16 + ol;
        st.s[u] = (o < M && l0 + ll < L) ? shift[(size_t)o * L + l0 + ll] : 0;
    }
}

template <int LOG2N>
__device__ __forceinline__ void contract_store(const ContractStage& st, float* xs, float2* ws, const float2* fac,
                                               int kb, int l0, int L, int M, int rt, int tid) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int f = tid + u * kContractThreads;
        const int i = f >> 6, j = f & 63;
        *reinterpret_cast<float4*>(xs + i * kRowFloats + j * 4) = st.v[u];
        const int e = tid + u * kContractThreads;
        const int ol = e & 15, bin = (e >> 4) & 7, ll = e >> 7;
        const bool valid = rt * 16 + ol < M && l0 + ll < L;
        const float2 w = shear_phase<LOG2N>((uint32_t)(kb * kBinBlock + bin), st.s[u], fac);
        ws[e] = valid ? w : make_float2(0.f, 0.f);
    }
}

// the 16 MFMAs of one chunk: operands for every element read first, then the chain
template <int LOG2N>
__device__ __forceinline__ void contract_mfma(floatx16& acc, const float* xs, const float2* ws, int col, int wave,
                                              int part, int orow, int comp, uint32_t negmask) {
    const float* xrow = xs + col * kRowFloats + wave * 2 + part;
    const float* wrow = reinterpret_cast<const float*>(ws) + (wave * 16 + orow) * 2 + comp;
    float av[kChunkL], bv[kChunkL];
#pragma unroll
    for (int ll = 0; ll < kChunkL; ++ll) {
        bv[ll] = xrow[ll * kBinBlock * 2];
        av[ll] = wrow[ll * kBinBlock * 16 * 2];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep all 32 operand reads in flight ahead of the MFMA chain
#pragma unroll
    for (int ll = 0; ll < kChunkL; ++ll) {
        const float a = __uint_as_float(__float_as_uint(av[ll]) ^ negmask);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv[ll], acc, 0, 0, 0);
    }
}

template <int LOG2N>
__global__ __launch_bounds__(kContractThreads) void contract_kernel(const float2* __restrict__ X,
                                                                     const int32_t* __restrict__ shift,
                                                                     float2* __restrict__ Y, int ntx, int M,
                                                                     int L, int ncol, int kpad) {
    constexpr int N = 1 << LOG2N;
    __shared__ float2 fac[64 + N / 64];
    __shared__ __attribute__((aligned(16))) float xs[2][32 * kRowFloats];
    __shared__ float2 ws[2][kChunkL * kBinBlock * 16];            // [l][bin][angle]
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int kb = blockIdx.x, rt = blockIdx.y, ct = blockIdx.z;
    build_phase_factors<LOG2N>(fac, tid);
    // lane roles.  B (2 x 32): part = lane / 32 in {Re, Im}, transmit column lane % 32.
    // A (32 x 2): row lane % 32 = {Re rows 0..15, Im rows 16..31} x 16 receive angles; the lane
    // supplies Wr (Re row, Re part), -Wi (Re row, Im part), Wi (Im row, Re part), Wr (Im, Im).
    const int part = lane >> 5;
    const int col = lane & 31;
    const int ytype = col >> 4;
    const int orow = col & 15;
    const int comp = (ytype == part) ? 0 : 1;
    const uint32_t negmask = (ytype == 0 && part == 1) ? 0x80000000u : 0u;

    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;

    // chunks c + 1 and c + 2 are in flight (two register stages) while chunk c is multiplied
    ContractStage st[2];
    const int nchunks = (L + kChunkL - 1) / kChunkL;
    contract_load(st[0], X, shift, kb, ncol, ct, L, 0, M, rt, tid);
    if (nchunks > 1) contract_load(st[1], X, shift, kb, ncol, ct, L, kChunkL, M, rt, tid);
    __syncthreads();  // phase factors complete
    contract_store<LOG2N>(st[0], xs[0], ws[0], fac, kb, 0, L, M, rt, tid);
    __syncthreads();
    for (int c = 0; c < nchunks; c += 2) {
        // even chunk c from buffer 0 (stage 1 holds c + 1, stage 0 is free)
        if (c + 2 < nchunks) contract_load(st[0], X, shift, kb, ncol, ct, L, (c + 2) * kChunkL, M, rt, tid);
        contract_mfma<LOG2N>(acc, xs[0], ws[0], col, wave, part, orow, comp, negmask);
        if (c + 1 < nchunks) contract_store<LOG2N>(st[1], xs[1], ws[1], fac, kb, (c + 1) * kChunkL, L, M, rt, tid);
        __syncthreads();
        if (c + 1 >= nchunks) break;
        // odd chunk c + 1 from buffer 1 (stage 0 holds c + 2, stage 1 is free)
        if (c + 3 < nchunks) contract_load(st[1], X, shift, kb, ncol, ct, L, (c + 3) * kChunkL, M, rt, tid);
        contract_mfma<LOG2N>(acc, xs[1], ws[1], col, wave, part, orow, comp, negmask);
        if (c + 2 < nchunks) contract_store<LOG2N>(st[0], xs[0], ws[0], fac, kb, (c + 2) * kChunkL, L, M, rt, tid);
        __syncthreads();
    }
    const int i = ct * 32 + col;
    const int k = kb * kBinBlock + wave;
    if (i >= ntx) return;
    // accumulator v of lane holds row (v/4)*8 + (lane/32)*4 + v%4, column lane%32; rows v and
    // v + 8 are Re and Im of the same receive angle
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int oo = rt * 16 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        if (oo < M) Y[((size_t)i * M + oo) * kpad + k] = make_float2(acc[v], acc[v + 8]);
    }
}

template <int LOG2N>
hipError_t contract(const float2* X, const int32_t* shift, float2* Y, int ntx, int M, int L, int ncol, int kpad,
                    hipStream_t st) {
    // bins 0 .. n/2 - 1; the Nyquist bin is summed by the inverse transform
    const dim3 grid((1 << LOG2N) / 2 / kBinBlock, (M + 15) / 16, ncol / 32);
    hipLaunchKernelGGL((contract_kernel<LOG2N>), grid, dim3(kContractThreads), 0, st, X, shift, Y, ntx, M, L, ncol,
                       kpad);
    return hipGetLastError();
}

hipError_t launch_contract(int log2n, const float2* X, const int32_t* shift, float2* Y, int ntx, int M, int L,
                           int ncol, int kpad, hipStream_t st) {
    switch (log2n) {
        case 8: return contract<8>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        case 9: return contract<9>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        case 10: return contract<10>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        case 11: return contract<11>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        case 12: return contract<12>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        case 13: return contract<13>(X, shift, Y, ntx, M, L, ncol, kpad, st);
        default: return hipErrorInvalidValue;
    }
}

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct DecomposeLayout {
    int log2n, K, kpad, ncol;
    size_t x_off, y_off, total;
};

bool decompose_layout(const kk_geom* g, int32_t N, int32_t M, int32_t tpad, DecomposeLayout* d) {
    const int lg = log2_exact(tpad);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->T < 1 || g->T > tpad || g->L < 1 || N < 1 || M < 1) return false;
    d->log2n = lg;
    d->K = tpad / 2 + 1;
    d->kpad = (d->K + kBinBlock - 1) / kBinBlock * kBinBlock;
    d->ncol = (N + 31) / 32 * 32;
    d->x_off = 0;
    d->y_off = d->x_off + align256((size_t)d->kpad * d->ncol * g->L * 8);
    d->total = d->y_off + align256((size_t)N * M * d->kpad * 8);
    return true;
}

struct DasLayout {
    int log2n, kpad;
    size_t x_off, a_off, p_off, total;
};

bool das_layout(const kk_geom* g, int32_t N, const int32_t* plan_host, DasLayout* d) {
    int64_t tp = 1;
    while (tp < g->T) tp *= 2;
    const int lg = log2_exact(tp);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->L < 1 || N < 1) return false;
    d->log2n = lg;
    d->kpad = (int)(tp / 2 + 1 + 7) / 8 * 8;
    d->x_off = 0;
    d->a_off = d->x_off + align256((size_t)N * g->L * d->kpad * 8);
    d->p_off = d->a_off + align256((size_t)N * g->L * g->T * 8);
    d->total = d->p_off + align256(gather_workspace_bytes(plan_host));
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
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    float2* Y = reinterpret_cast<float2*>(w + d.y_off);
    if (launch_fft_forward(rf, N * g->L, g->T, d.log2n, X, true, g->L, d.ncol, d.kpad, st) != hipSuccess)
        return KK_E_HIP;
    if (launch_contract(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, st) != hipSuccess) return KK_E_HIP;
    NyquistSum nyq{X, shift_q, M, g->L, d.ncol};
    if (launch_fft_inverse(Y, N * M, d.kpad, d.log2n, reinterpret_cast<float2*>(rf_theta), g->T, st, &nyq) !=
        hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

size_t das_workspace_bytes(const kk_geom* g, int32_t N, const void* plan_host, size_t plan_bytes) {
    kk::DasLayout d;
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (!g || !h || !kk::gather_plan_ok(h, plan_bytes, true) || !kk::das_layout(g, N, h, &d)) return 0;
    return d.total;
}

int32_t das_beamform(const int16_t* rf, int32_t N, const kk_geom* g, const void* plan_host, const void* plan_dev,
                     size_t plan_bytes, float* image, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf || !g || !plan_host || !plan_dev || !image || !ws) return KK_E_NULL;
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (!gather_plan_ok(h, plan_bytes, true)) return KK_E_WORKSPACE;
    if (N < 1 || h[PW_N] != N || h[PW_M] != g->L || h[PW_T] != g->T) return KK_E_ARG;
    DasLayout d;
    if (!das_layout(g, N, h, &d)) return KK_E_ARG;
    if (ws_bytes < d.total) return KK_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    unsigned char* w = static_cast<unsigned char*>(ws);
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    float2* A = reinterpret_cast<float2*>(w + d.a_off);
    const int ntr = N * g->L;
    if (launch_fft_forward(rf, ntr, g->T, d.log2n, X, false, g->L, 0, d.kpad, st) != hipSuccess) return KK_E_HIP;
    if (launch_fft_inverse(X, ntr, d.kpad, d.log2n, A, g->T, st) != hipSuccess) return KK_E_HIP;
    if (run_gather(A, h, static_cast<const int32_t*>(plan_dev), reinterpret_cast<float2*>(image), nullptr, 0,
                   w + d.p_off, true, st) != hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

}  // extern "C"
