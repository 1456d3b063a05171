// Eq. 3 receive plane-wave decomposition on gfx950, evaluated in the temporal-frequency
// domain (Sec. II-F):
//   1. analytic spectra of the N*L zero-padded records (kk_fft.hip, two records per FFT),
//      stored bin-blocked X[k/8][i][l][k%8];
//   2. per bin k the complex contraction Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] with
//      W_k[o][l] = exp(2 pi i r / (n 2^22)), r = (k shift[o][l]) mod (n 2^22), on MFMA
//      (v_mfma_f32_32x32x2_f32: one complex element l per instruction, 16 receive angles x
//      {Re, Im} rows by 32 transmit columns; 8 bins per workgroup, one per wave, the spectrum
//      staged through LDS 16 elements at a time in a software pipeline across chunks);
//   3. inverse FFT of each (i, o) spectrum, first T samples.
// The phase is formed exactly in integers; only the reduced fraction becomes floating point:
// W = E[r >> 22] * exp(2 pi i (r mod 2^22) / (n 2^22)), with E[m] = exp(2 pi i m / n) the
// product of two FP64-evaluated factor tables and the small second factor (|angle| < 2 pi / n)
// by its Taylor series.  Within a bin block only the first bin's phase and the one-bin step are
// evaluated so; the other bins are products of the step's powers (a few roundings deep).
// Also the DAS comparator entry point (analytic channel data + delay-gather).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kContractWaves = kBinBlock;   // one bin of the block per wave
constexpr int kContractThreads = kContractWaves * 64;
constexpr int kChunkL = 16;                  // elements per LDS chunk
// One transmit column of a chunk plus a pad of two floats: rows stay 8-byte aligned and
// column c's operand reads land on banks 2c, 2c+1, so a wave's 32 columns x {Re, Im} hit all
// 64 banks once.
constexpr int kRowFloats = kChunkL * kBinBlock * 2 + 2;
// Chunks whose global loads are in flight.  Two measure faster than four or eight: the loop is
// bound by LDS traffic and barriers rather than by load latency, and fewer register stages
// leave fewer zero chunks at the end of a ragged element count.
constexpr int kStages = 2;
// Phases of one element of a chunk: 8 bins x 16 angles, then a pad of 16 (288 words, 32 modulo
// the 64 banks): the phase stores of a wave (two elements per 32-lane half) cover every bank once.
constexpr int kWsL = kBinBlock * 16 + 16;

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

__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
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
// transmit column i) and the shift of this thread's (receive angle, element) entry.
struct ContractStage {
    float4 v[4];
    int32_t s;
};

// Every path issues the same loads (clamped to valid addresses; out-of-range entries are
// zeroed at the store), so the wait before a stage's store can leave the later stages in flight.
__device__ __forceinline__ void contract_load(ContractStage& st, const float2* __restrict__ X,
                                              const int32_t* __restrict__ shift, int kb, int ncol, int ct, int L,
                                              int l0, int M, int rt, int tid) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int f = tid + u * kContractThreads;  // float4 index in the 32 x 64 chunk
        const int i = f >> 6, j = f & 63;          // column, float4 within the column's run
        const int l = min(l0 + (j >> 2), L - 1);
        st.v[u] = reinterpret_cast<const float4*>(X + (((size_t)kb * ncol + ct * 32 + i) * L + l) * kBinBlock)[j & 3];
    }
    const int o = min(rt * 16 + (tid & 15), M - 1), l = min(l0 + ((tid >> 4) & 15), L - 1);
    st.s = shift[(size_t)o * L + l];  // used by threads 0..255, (angle, element) = (tid % 16, tid / 16)
}

// Spectrum rows into LDS, and the phases W[l][bin][angle] of the chunk: thread (angle, l) of
// the first four waves evaluates the phase of the block's first bin exactly and the one-bin
// step D = exp(2 pi i s / (n 2^22)), and forms the other seven bins as products of D, D^2 and
// D^4 (at most five roundings deep).
template <int LOG2N>
__device__ __forceinline__ void contract_store(const ContractStage& st, float* xs, float2* ws, const float2* fac,
                                               int kb, int l0, int L, int M, int rt, int tid) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int f = tid + u * kContractThreads;
        const int i = f >> 6, j = f & 63;
        const bool in = l0 + (j >> 2) < L;
        float2* row = reinterpret_cast<float2*>(xs + i * kRowFloats + j * 4);
        row[0] = in ? make_float2(st.v[u].x, st.v[u].y) : make_float2(0.f, 0.f);
        row[1] = in ? make_float2(st.v[u].z, st.v[u].w) : make_float2(0.f, 0.f);
    }
    if (tid < 256) {  // waves 0..3
        const int ol = tid & 15, ll = tid >> 4;
        const bool valid = rt * 16 + ol < M && l0 + ll < L;
        const float2 w0 = shear_phase<LOG2N>((uint32_t)(kb * kBinBlock), st.s, fac);
        const float2 d1 = shear_phase<LOG2N>(1u, st.s, fac);
        const float2 d2 = cmul2(d1, d1), d4 = cmul2(d2, d2);
        const float2 w1 = cmul2(w0, d1), w2 = cmul2(w0, d2), w3 = cmul2(w1, d2);
        const float2 w[8] = {w0, w1, w2, w3, cmul2(w0, d4), cmul2(w1, d4), cmul2(w2, d4), cmul2(w3, d4)};
        const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
        for (int b = 0; b < kBinBlock; ++b) ws[ll * kWsL + b * 16 + ol] = valid ? w[b] : zero;
    }
}

// MFMA operands of one chunk for one lane: the spectrum value (B) and the phase component (A,
// sign applied) of each of the chunk's 16 elements.
struct ChunkOperands {
    float a[kChunkL];
    float b[kChunkL];
};

__device__ __forceinline__ void read_operands(ChunkOperands& op, const float* xs, const float2* ws, int col, int wave,
                                              int part, int orow, int comp, uint32_t negmask) {
    const float* xrow = xs + col * kRowFloats + wave * 2 + part;
    const float* wrow = reinterpret_cast<const float*>(ws) + (wave * 16 + orow) * 2 + comp;
#pragma unroll
    for (int ll = 0; ll < kChunkL; ++ll) {
        op.b[ll] = xrow[ll * kBinBlock * 2];
        op.a[ll] = __uint_as_float(__float_as_uint(wrow[ll * kWsL * 2]) ^ negmask);
    }
}

// the 16 MFMAs of one chunk, in two interleaved accumulation chains (even and odd elements)
__device__ __forceinline__ void chunk_mfma(floatx16 (&acc)[2], const ChunkOperands& op) {
#pragma unroll
    for (int ll = 0; ll < kChunkL; ++ll)
        acc[ll & 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(op.a[ll], op.b[ll], acc[ll & 1], 0, 0, 0);
}

// Per bin block (8 bins, one per wave), receive-angle tile of 16 and transmit tile of 32:
// Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] over all elements in chunks of 16.  Software pipeline
// across chunks, one workgroup barrier per chunk: while the MFMAs of chunk c run from
// registers, the operands of chunk c+1 are read from LDS and chunk c+2 (spectrum rows and its
// phases) is written to LDS from its register stage, whose global loads were issued kStages
// chunks earlier.  The results leave through LDS as 64-byte runs (8 bins of one (i, o)).
template <int LOG2N>
__device__ __forceinline__ void contract_body(const float2* __restrict__ X, const int32_t* __restrict__ shift,
                                              float2* __restrict__ Y, int ntx, int M, int L, int ncol, int kpad,
                                              int kb, int rt, int ct) {
    constexpr int N = 1 << LOG2N;
    __shared__ float2 fac[64 + N / 64];
    __shared__ __attribute__((aligned(16))) float xs[2][32 * kRowFloats];
    __shared__ float2 ws[2][kChunkL * kWsL];                      // [l][bin][angle] (+ pad per l)
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
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

    floatx16 acc[2];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[0][v] = acc[1][v] = 0.0f;

    // a whole number of pipeline rounds: chunks past the last element are all zero
    const int nchunks = (L + kChunkL * kStages - 1) / (kChunkL * kStages) * kStages;
    ContractStage st[kStages];
    ChunkOperands op[2];
#pragma unroll
    for (int u = 0; u < kStages; ++u) contract_load(st[u], X, shift, kb, ncol, ct, L, u * kChunkL, M, rt, tid);
    __syncthreads();  // phase factors complete
    contract_store<LOG2N>(st[0], xs[0], ws[0], fac, kb, 0, L, M, rt, tid);
    contract_load(st[0], X, shift, kb, ncol, ct, L, kStages * kChunkL, M, rt, tid);
    contract_store<LOG2N>(st[1], xs[1], ws[1], fac, kb, kChunkL, L, M, rt, tid);
    contract_load(st[1], X, shift, kb, ncol, ct, L, (kStages + 1) * kChunkL, M, rt, tid);
    __syncthreads();
    read_operands(op[0], xs[0], ws[0], col, wave, part, orow, comp, negmask);
    __syncthreads();  // every wave has chunk 0's operands before buffer 0 takes chunk 2
    for (int c0 = 0; c0 < nchunks; c0 += kStages) {
#pragma unroll
        for (int u = 0; u < kStages; ++u) {
            const int c = c0 + u;  // chunk c: operands in op[u & 1]; c+1 in LDS buffer (u+1)&1
            chunk_mfma(acc, op[u & 1]);
            read_operands(op[(u + 1) & 1], xs[(u + 1) & 1], ws[(u + 1) & 1], col, wave, part, orow, comp, negmask);
            const int s2 = (u + 2) % kStages;  // register stage of chunk c+2 (static once unrolled)
            // chunk c+2 over chunk c's LDS buffer (read before the previous barrier), then the
            // freed stage takes chunk c+2+kStages (loads past the end re-read valid addresses)
            contract_store<LOG2N>(st[s2], xs[u & 1], ws[u & 1], fac, kb, (c + 2) * kChunkL, L, M, rt, tid);
            contract_load(st[s2], X, shift, kb, ncol, ct, L, (c + 2 + kStages) * kChunkL, M, rt, tid);
            __syncthreads();
        }
    }
    // results to LDS as runs [i][o][bin] (i stride 129 float2, so a half-wave's 32 columns
    // write 64 distinct banks), then out as 64-byte runs, 8 threads per run
    constexpr int kYCol = 16 * kBinBlock + 1;
    static_assert(32 * kYCol * 8 <= (int)sizeof(xs), "result staging fits the spectrum buffers");
    float2* yst = reinterpret_cast<float2*>(&xs[0][0]);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int ol = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        yst[col * kYCol + ol * kBinBlock + wave] = make_float2(acc[0][v] + acc[1][v], acc[0][v + 8] + acc[1][v + 8]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int f = tid + u * kContractThreads;  // float2 f & 7 of run f >> 3
        const int run = f >> 3, q = f & 7;
        const int il = run >> 4, ol = run & 15;
        const int i = ct * 32 + il, o = rt * 16 + ol;
        if (i < ntx && o < M) Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q] = yst[il * kYCol + ol * kBinBlock + q];
    }
}

// ---------------------------------------------------------------------------------------
// Split-precision contraction: the same per-bin product with 16-bit MFMA inputs.  Every
// spectrum value and phase is split as x = hi + lo, hi = round16(x), lo = round16(x - hi)
// (BF16 or FP16), and Y = Wh Xh + Wh Xl + Wl Xh accumulated in FP32 on
// v_mfma_f32_32x32x16_{bf16,f16} (eight complex elements per instruction: K = {Re, Im} x 8).
// The dropped Wl Xl term and the residuals are below 2^-16 (BF16) or 2^-22 (FP16) of the
// terms.  FP16 spectra are first scaled by 2^e so that |X| < 2^15 (|X| <= 2 T 32768 for int16
// records), and Y by 2^-e (both exact).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kXsWords = kBinBlock * 2 * kChunkL + 4;  // per column: [bin][hi, lo][l] + pad (16 B)
constexpr int kWsBlock = 2 * kChunkL + 4;              // per (bin, angle, row type): [hi, lo][l] + pad

template <bool F16>
__device__ __forceinline__ uint32_t half_bits(float x) {
    if constexpr (F16)
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
    else
        return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}
template <bool F16>
__device__ __forceinline__ float half_value(float x) {
    if constexpr (F16)
        return (float)(_Float16)x;
    else
        return (float)(__bf16)x;
}
// (re, im) -> hi pair and lo pair, low half = re
template <bool F16>
__device__ __forceinline__ void split_pair(float re, float im, uint32_t& hi, uint32_t& lo) {
    const float rh = half_value<F16>(re), ih = half_value<F16>(im);
    hi = half_bits<F16>(re) | (half_bits<F16>(im) << 16);
    lo = half_bits<F16>(re - rh) | (half_bits<F16>(im - ih) << 16);
}

template <int LOG2N, bool F16>
__device__ __forceinline__ void split_store(const ContractStage& st, uint32_t* xs, uint32_t* ws, const float2* fac,
                                            int kb, int l0, int L, int M, int rt, int tid, float xscale) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int f = tid + u * kContractThreads;
        const int i = f >> 6, j = f & 63;        // column, float4 (two bins of one element)
        const int l = j >> 2, q = j & 3;
        const bool in = l0 + l < L;
        const float v[4] = {st.v[u].x * xscale, st.v[u].y * xscale, st.v[u].z * xscale, st.v[u].w * xscale};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t hi, lo;
            split_pair<F16>(v[2 * h], v[2 * h + 1], hi, lo);
            uint32_t* d = xs + i * kXsWords + ((2 * q + h) * 2) * kChunkL + l;
            d[0] = in ? hi : 0u;
            d[kChunkL] = in ? lo : 0u;
        }
    }
    if (tid < 256) {  // waves 0..3: phases of (angle, element) for the block's 8 bins
        const int ol = tid & 15, ll = tid >> 4;
        const bool valid = rt * 16 + ol < M && l0 + ll < L;
        const float2 w0 = shear_phase<LOG2N>((uint32_t)(kb * kBinBlock), st.s, fac);
        const float2 d1 = shear_phase<LOG2N>(1u, st.s, fac);
        const float2 d2 = cmul2(d1, d1), d4 = cmul2(d2, d2);
        const float2 w1 = cmul2(w0, d1), w2 = cmul2(w0, d2), w3 = cmul2(w1, d2);
        const float2 w[8] = {w0, w1, w2, w3, cmul2(w0, d4), cmul2(w1, d4), cmul2(w2, d4), cmul2(w3, d4)};
#pragma unroll
        for (int b = 0; b < kBinBlock; ++b) {
            uint32_t rh, rl, ih, il;
            split_pair<F16>(w[b].x, -w[b].y, rh, rl);  // Re rows: (Wr, -Wi)
            split_pair<F16>(w[b].y, w[b].x, ih, il);   // Im rows: (Wi, Wr)
            uint32_t* dr = ws + ((b * 16 + ol) * 2 + 0) * kWsBlock + ll;
            uint32_t* di = ws + ((b * 16 + ol) * 2 + 1) * kWsBlock + ll;
            dr[0] = valid ? rh : 0u;
            dr[kChunkL] = valid ? rl : 0u;
            di[0] = valid ? ih : 0u;
            di[kChunkL] = valid ? il : 0u;
        }
    }
}

// MFMA operands of one chunk: two K-steps of 8 elements, hi and lo of A (phases) and B (spectrum)
struct SplitOperands {
    u32x4 ah[2], al[2], bh[2], bl[2];
};

__device__ __forceinline__ void split_read(SplitOperands& op, const uint32_t* xs, const uint32_t* ws, int col, int g,
                                           int wave) {
    // B lane (g, col): elements 4g..4g+3 of K-step s for transmit col; A lane (g, row col):
    // the same elements for row (angle col % 16, Re/Im col / 16)
    const uint32_t* xb = xs + col * kXsWords + wave * 2 * kChunkL + 4 * g;
    const uint32_t* wa = ws + ((wave * 16 + (col & 15)) * 2 + (col >> 4)) * kWsBlock + 4 * g;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        op.bh[s] = *reinterpret_cast<const u32x4*>(xb + 8 * s);
        op.bl[s] = *reinterpret_cast<const u32x4*>(xb + kChunkL + 8 * s);
        op.ah[s] = *reinterpret_cast<const u32x4*>(wa + 8 * s);
        op.al[s] = *reinterpret_cast<const u32x4*>(wa + kChunkL + 8 * s);
    }
}

template <bool F16>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

template <bool F16>
__device__ __forceinline__ void split_mfma(floatx16 (&acc)[2], const SplitOperands& op) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        acc[s] = mfma16<F16>(op.ah[s], op.bl[s], acc[s]);
        acc[s] = mfma16<F16>(op.al[s], op.bh[s], acc[s]);
        acc[s] = mfma16<F16>(op.ah[s], op.bh[s], acc[s]);
    }
}

// Same workgroup shape and software pipeline as contract_kernel.
template <int LOG2N, bool F16>
__device__ __forceinline__ void contract_split_body(const float2* __restrict__ X, const int32_t* __restrict__ shift,
                                                    float2* __restrict__ Y, int ntx, int M, int L, int ncol,
                                                    int kpad, float xscale, float yscale, int kb, int rt, int ct) {
    constexpr int N = 1 << LOG2N;
    __shared__ float2 fac[64 + N / 64];
    __shared__ __attribute__((aligned(16))) uint32_t xs[2][32 * kXsWords];
    __shared__ __attribute__((aligned(16))) uint32_t ws[2][kBinBlock * 16 * 2 * kWsBlock];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    build_phase_factors<LOG2N>(fac, tid);
    const int g = lane >> 5, col = lane & 31;

    floatx16 acc[2];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[0][v] = acc[1][v] = 0.0f;

    const int nchunks = (L + kChunkL * kStages - 1) / (kChunkL * kStages) * kStages;
    ContractStage st[kStages];
    SplitOperands op[2];
#pragma unroll
    for (int u = 0; u < kStages; ++u) contract_load(st[u], X, shift, kb, ncol, ct, L, u * kChunkL, M, rt, tid);
    __syncthreads();  // phase factors complete
    split_store<LOG2N, F16>(st[0], xs[0], ws[0], fac, kb, 0, L, M, rt, tid, xscale);
    contract_load(st[0], X, shift, kb, ncol, ct, L, kStages * kChunkL, M, rt, tid);
    split_store<LOG2N, F16>(st[1], xs[1], ws[1], fac, kb, kChunkL, L, M, rt, tid, xscale);
    contract_load(st[1], X, shift, kb, ncol, ct, L, (kStages + 1) * kChunkL, M, rt, tid);
    __syncthreads();
    split_read(op[0], xs[0], ws[0], col, g, wave);
    __syncthreads();  // every wave has chunk 0's operands before buffer 0 takes chunk 2
    for (int c0 = 0; c0 < nchunks; c0 += kStages) {
#pragma unroll
        for (int u = 0; u < kStages; ++u) {
            const int c = c0 + u;
            split_mfma<F16>(acc, op[u & 1]);
            split_read(op[(u + 1) & 1], xs[(u + 1) & 1], ws[(u + 1) & 1], col, g, wave);
            const int s2 = (u + 2) % kStages;
            split_store<LOG2N, F16>(st[s2], xs[u & 1], ws[u & 1], fac, kb, (c + 2) * kChunkL, L, M, rt, tid, xscale);
            contract_load(st[s2], X, shift, kb, ncol, ct, L, (c + 2 + kStages) * kChunkL, M, rt, tid);
            __syncthreads();
        }
    }
    constexpr int kYCol = 16 * kBinBlock + 1;
    static_assert(32 * kYCol * 8 <= (int)sizeof(xs), "result staging fits the spectrum buffers");
    float2* yst = reinterpret_cast<float2*>(&xs[0][0]);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int ol = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        yst[col * kYCol + ol * kBinBlock + wave] =
            make_float2((acc[0][v] + acc[1][v]) * yscale, (acc[0][v + 8] + acc[1][v + 8]) * yscale);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int f = tid + u * kContractThreads;
        const int run = f >> 3, q = f & 7;
        const int il = run >> 4, ol = run & 15;
        const int i = ct * 32 + il, o = rt * 16 + ol;
        if (i < ntx && o < M) Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q] = yst[il * kYCol + ol * kBinBlock + q];
    }
}

template <int LOG2N>
__global__ __launch_bounds__(kContractThreads) void contract_kernel(const float2* __restrict__ X,
                                                                     const int32_t* __restrict__ shift,
                                                                     float2* __restrict__ Y, int ntx, int M,
                                                                     int L, int ncol, int kpad) {
    contract_body<LOG2N>(X, shift, Y, ntx, M, L, ncol, kpad, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int LOG2N, bool F16>
__global__ __launch_bounds__(kContractThreads) void contract_split_kernel(
    const float2* __restrict__ X, const int32_t* __restrict__ shift, float2* __restrict__ Y, int ntx, int M, int L,
    int ncol, int kpad, float xscale, float yscale) {
    contract_split_body<LOG2N, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, yscale, blockIdx.x, blockIdx.y,
                                    blockIdx.z);
}

// Grouped launches over the frames of one FFT-length class: block b runs block b - block0
// of frame entry blk[b], in the per-frame grid order (bin block fastest, then receive tile,
// then transmit tile).  PREC: 0 FP32, 1 BF16 hi+lo, 2 FP16 hi+lo.
template <int LOG2N, int PREC>
__global__ __launch_bounds__(kContractThreads) void contract_grouped(const ContractEntry* __restrict__ tab,
                                                                     const int32_t* __restrict__ blk,
                                                                     float2* __restrict__ ws,
                                                                     const int32_t* __restrict__ plan) {
    const ContractEntry e = tab[blk[blockIdx.x]];
    int local = (int)blockIdx.x - e.block0;
    const int kb = local % e.nkb;
    local /= e.nkb;
    const int rt = local % e.nrt, ct = local / e.nrt;
    if constexpr (PREC == 0)
        contract_body<LOG2N>(ws + e.x_off, plan + e.shift_off, ws + e.y_off, e.ntx, e.M, e.L, e.ncol, e.kpad, kb, rt,
                             ct);
    else
        contract_split_body<LOG2N, PREC == 2>(ws + e.x_off, plan + e.shift_off, ws + e.y_off, e.ntx, e.M, e.L, e.ncol,
                                              e.kpad, e.xscale, e.yscale, kb, rt, ct);
}

template <int LOG2N>
hipError_t grouped_contract(int prec, const ContractEntry* tab, const int32_t* blk, int blocks, float2* ws,
                            const int32_t* plan, hipStream_t st) {
    const dim3 g(blocks), b(kContractThreads);
    switch (prec) {
        case KK_PREC_FP32: hipLaunchKernelGGL((contract_grouped<LOG2N, 0>), g, b, 0, st, tab, blk, ws, plan); break;
        case KK_PREC_BF16X3: hipLaunchKernelGGL((contract_grouped<LOG2N, 1>), g, b, 0, st, tab, blk, ws, plan); break;
        case KK_PREC_FP16X3: hipLaunchKernelGGL((contract_grouped<LOG2N, 2>), g, b, 0, st, tab, blk, ws, plan); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int LOG2N, bool F16>
hipError_t contract_split(const float2* X, const int32_t* shift, float2* Y, int ntx, int M, int L, int ncol, int kpad,
                          float xscale, hipStream_t st) {
    const dim3 grid((1 << LOG2N) / 2 / kBinBlock, (M + 15) / 16, ncol / 32);
    hipLaunchKernelGGL((contract_split_kernel<LOG2N, F16>), grid, dim3(kContractThreads), 0, st, X, shift, Y, ntx, M,
                       L, ncol, kpad, xscale, 1.0f / xscale);
    return hipGetLastError();
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

template <bool F16>
hipError_t launch_contract_split(int log2n, const float2* X, const int32_t* shift, float2* Y, int ntx, int M, int L,
                                 int ncol, int kpad, float xscale, hipStream_t st) {
    switch (log2n) {
        case 8: return contract_split<8, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 9: return contract_split<9, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 10: return contract_split<10, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 11: return contract_split<11, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 12: return contract_split<12, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 13: return contract_split<13, F16>(X, shift, Y, ntx, M, L, ncol, kpad, xscale, st);
        default: return hipErrorInvalidValue;
    }
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

}  // namespace

hipError_t launch_contract_grouped(int log2n, int precision, const ContractEntry* tab, const int32_t* blk, int blocks,
                                   float2* ws, const int32_t* plan, hipStream_t st) {
    switch (log2n) {
        case 8: return grouped_contract<8>(precision, tab, blk, blocks, ws, plan, st);
        case 9: return grouped_contract<9>(precision, tab, blk, blocks, ws, plan, st);
        case 10: return grouped_contract<10>(precision, tab, blk, blocks, ws, plan, st);
        case 11: return grouped_contract<11>(precision, tab, blk, blocks, ws, plan, st);
        case 12: return grouped_contract<12>(precision, tab, blk, blocks, ws, plan, st);
        case 13: return grouped_contract<13>(precision, tab, blk, blocks, ws, plan, st);
        default: return hipErrorInvalidValue;
    }
}

namespace {
// bins [from, kpad) of every record of y [n][kpad] set to zero
__global__ void zero_bins_kernel(float2* __restrict__ y, int64_t n, int kpad, int from) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int width = kpad - from;
    if (i >= n * width) return;
    const int64_t r = i / width;
    y[r * kpad + from + (int)(i - r * width)] = make_float2(0.f, 0.f);
}
}  // namespace

int fp16_prescale_exponent(int T) {
    // |X| <= 2 T 32768 (analytic mask x int16 record): 2^e X stays below 2^15
    int e = 15;
    for (int64_t bound = 2 * (int64_t)T * 32768; bound > 1; bound = (bound + 1) / 2) --e;
    return e;
}

namespace {

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
    if (!g || (precision != KK_PREC_FP32 && precision != KK_PREC_BF16X3 && precision != KK_PREC_FP16X3) ||
        !kk::decompose_layout(g, N, M, tpad, &d))
        return 0;
    return d.total;
}

int32_t kk_decompose(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M, int32_t tpad,
                     int32_t precision, float* rf_theta, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf || !g || !shift_q || !rf_theta || !ws) return KK_E_NULL;
    if (precision != KK_PREC_FP32 && precision != KK_PREC_BF16X3 && precision != KK_PREC_FP16X3)
        return KK_E_UNSUPPORTED;
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
    hipError_t ce;
    if (precision == KK_PREC_FP32) {
        ce = launch_contract(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, st);
    } else if (precision == KK_PREC_BF16X3) {
        ce = launch_contract_split<false>(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, 1.0f, st);
    } else {
        const int e = fp16_prescale_exponent(g->T);
        ce = launch_contract_split<true>(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, std::ldexp(1.0f, e), st);
    }
    if (ce != hipSuccess) return KK_E_HIP;
    NyquistSum nyq{X, shift_q, M, g->L, d.ncol};
    if (launch_fft_inverse(Y, N * M, d.kpad, d.log2n, reinterpret_cast<float2*>(rf_theta), g->T, st, &nyq) !=
        hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}

int32_t kk_spectrum_bins(int32_t tpad) {
    const int lg = kk::log2_exact(tpad);
    if (lg < kk::kMinLog2Fft || lg > kk::kMaxLog2Fft) return 0;
    return (tpad / 2 + 1 + kk::kBinBlock - 1) / kk::kBinBlock * kk::kBinBlock;
}

int32_t kk_decompose_spectrum(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M,
                              int32_t tpad, int32_t precision, float* spec, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf || !g || !shift_q || !spec || !ws) return KK_E_NULL;
    if (precision != KK_PREC_FP32 && precision != KK_PREC_BF16X3 && precision != KK_PREC_FP16X3)
        return KK_E_UNSUPPORTED;
    if (N < 1 || M < 1 || g->L < 1 || g->L > 65536 || g->T < 1) return KK_E_ARG;
    DecomposeLayout d;
    if (!decompose_layout(g, N, M, tpad, &d)) return KK_E_ARG;
    if ((int64_t)N * g->L > 0x7fffffff || (int64_t)N * M > 0x7fffffff) return KK_E_ARG;
    if (ws_bytes < d.y_off) return KK_E_WORKSPACE;  // the spectra only; Y is the caller's
    hipStream_t st = (hipStream_t)stream;
    float2* X = static_cast<float2*>(ws);
    float2* Y = reinterpret_cast<float2*>(spec);
    if (launch_fft_forward(rf, N * g->L, g->T, d.log2n, X, true, g->L, d.ncol, d.kpad, st) != hipSuccess)
        return KK_E_HIP;
    hipError_t ce;
    if (precision == KK_PREC_FP32) {
        ce = launch_contract(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, st);
    } else if (precision == KK_PREC_BF16X3) {
        ce = launch_contract_split<false>(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad, 1.0f, st);
    } else {
        ce = launch_contract_split<true>(d.log2n, X, shift_q, Y, N, M, g->L, d.ncol, d.kpad,
                                         std::ldexp(1.0f, fp16_prescale_exponent(g->T)), st);
    }
    if (ce != hipSuccess) return KK_E_HIP;
    const int from = tpad / 2;
    const int64_t n = (int64_t)N * M * (d.kpad - from);
    hipLaunchKernelGGL(zero_bins_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Y, (int64_t)N * M,
                       d.kpad, from);
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_spectrum_inverse(const float* spec, int32_t ntraces, int32_t tpad, int32_t T, float* rf_theta,
                            void* stream) {
    using namespace kk;
    if (!spec || !rf_theta) return KK_E_NULL;
    const int lg = log2_exact(tpad);
    if (ntraces < 1 || T < 1 || T > tpad || lg < kMinLog2Fft || lg > kMaxLog2Fft) return KK_E_ARG;
    const int kpad = kk_spectrum_bins(tpad);
    return launch_fft_inverse(reinterpret_cast<const float2*>(spec), ntraces, kpad, lg,
                              reinterpret_cast<float2*>(rf_theta), T, (hipStream_t)stream) == hipSuccess
               ? KK_OK
               : KK_E_HIP;
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
