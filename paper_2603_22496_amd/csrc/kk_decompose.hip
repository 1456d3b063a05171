// Eq. 3 receive plane-wave decomposition on gfx950, evaluated in the temporal-frequency
// domain (Sec. II-F):
//   1. analytic spectra of the N*L zero-padded records (kk_fft.hip, two records per FFT),
//      stored bin-blocked (spec_index: 64-byte runs of 8 bins per element and transmit); the
//      same launch writes the phase tables of step 2 (PhaseTables);
//   2. per bin k the complex contraction Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] with
//      W_k[o][l] = exp(2 pi i r / (n 2^22)), r = (k shift[o][l]) mod (n 2^22), on MFMA
//      (FP32: v_mfma_f32_16x16x4_f32, two complex elements per instruction, 8 receive angles x
//      {Re, Im} rows by 16 transmit columns, up to 32 angles and 8 bins per workgroup; split
//      precision: v_mfma_f32_32x32x16_{bf16,f16} on hi + lo halves);
//   3. inverse FFT of each (i, o) spectrum, first T samples.
// Every table phase comes from an exact integer turn count evaluated in FP64 and rounded once:
// the anchor W_{8 kb} of each bin block and the in-block steps, W_{8 kb + j} = W_{8 kb} D_j.
// The split-precision path reads D_j itself (one complex product from the anchor); the FP32
// path reads D_1 and D_4 and forms D_j = D_1^j or D_4 D_1^(j-4) (at most three products).
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

// FP32 contraction workgroup: one block of 8 bins, R8 tiles of 8 receive angles
// (contract_r8), 16 transmit columns; wave w takes element quarter w (element pairs 2j, 2j+1
// with j = w (mod 4)), all 8 bins; the quarters are summed at the end in a fixed order.  Two
// workgroups share a CU (at most 256 registers per lane), so one's start and reduction overlap
// the other's element loop.
constexpr int kContractWaves = 4;
constexpr int kContractThreads = kContractWaves * 64;
// Element pairs whose operand loads are in flight per wave (fewer with more accumulators).
template <int R8>
constexpr int contract_depth() { return R8 <= 2 ? 4 : 3; }
// Result staging: per transmit column, 8 R8 angles x 8 bins x {Re, Im} floats and a pad of two
// (the 16 columns of a wave's row then fall in distinct banks).
template <int R8>
constexpr int contract_col_floats() { return 8 * R8 * kBinBlock * 2 + 2; }

// Split-precision workgroup: one bin block, T16 tiles of 16 receive angles (T16 = 2 when
// M > 16, so up to 32 angles share one pass over the spectrum), 32 transmit columns; wave w
// takes bin pair w over all elements.  Two workgroups share a CU.
constexpr int kSplitWaves = 4;
constexpr int kSplitThreads = kSplitWaves * 64;
constexpr int kAnchorChunk = 256;
__host__ __device__ constexpr int split_t16(int M) { return M > 16 ? 2 : 1; }
// staging of the results: float2 per (column, angle, bin) + a pad per column
template <int T16>
constexpr int split_col_float2() { return 16 * T16 * kBinBlock + 1; }
template <int T16>
constexpr int split_lds_float2() {
    return T16 * kAnchorChunk * 16 > 32 * split_col_float2<T16>() ? T16 * kAnchorChunk * 16 : 32 * split_col_float2<T16>();
}
// Anchor loads per thread of one chunk and tile (16-byte pieces, 8 per element).
constexpr int kAnchorLoads = (kAnchorChunk * 8 + kSplitThreads - 1) / kSplitThreads;

// Complex product with a fixed rounding sequence (one product rounded, then one fused
// multiply-add per component), so that every kernel instantiation rounds a phase the same way
// and an angle's result does not depend on the angles computed beside it.
__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// Anchors of elements [c0, c0 + cn) of one bin block and receive tile (split kernel): global ->
// registers -> LDS rows [l - c0][16] (indexes past the chunk re-read its last piece).
__device__ __forceinline__ void stage_anchors(float2* buf, const float2* __restrict__ anc, int c0, int cn, int tid) {
    const float4* src = reinterpret_cast<const float4*>(anc) + (size_t)c0 * 8;
    float4 v[kAnchorLoads];
#pragma unroll
    for (int u = 0; u < kAnchorLoads; ++u) v[u] = src[min(tid + u * kSplitThreads, cn * 8 - 1)];
    float4* dst = reinterpret_cast<float4*>(buf);
#pragma unroll
    for (int u = 0; u < kAnchorLoads; ++u) {
        const int f = tid + u * kSplitThreads;
        if (f < cn * 8) dst[f] = v[u];
    }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Operands of one element pair in flight for one lane: spectrum bins 4q .. 4q+3 of its element
// and transmit (q = its part, 32 bytes), and for each 8-angle tile the anchor and (D_1, D_4) of
// its angle and element.
template <int R8>
struct PairLoads {
    float4 x0, x1;
    float2 a[R8];
    float4 d[R8];
};

// LDS floats of the contraction: partial sums of the element quarters (two wave slots), then
// the result staging.
template <int R8>
constexpr int contract_lds_floats() {
    return 2 * R8 * 2048 > kContractCols * contract_col_floats<R8>() ? 2 * R8 * 2048
                                                                     : kContractCols * contract_col_floats<R8>();
}

// Per bin block (8 bins), R8 x 8 receive angles and 16 transmit columns:
// Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] on v_mfma_f32_16x16x4_f32, one instruction per bin,
// 8-angle tile and element pair: A (16 x 4) row lane % 16 = {Re rows 0..7, Im rows 8..15} x 8
// angles, column lane / 16 = (element e = lane / 32 of the pair, part q = lane / 16 % 2); B
// (4 x 16) row lane / 16 = (e, q), column lane % 16 = transmit; C: lane holds rows
// 4 (lane / 16) + 0..3 of column lane % 16.
//  * Spectrum: each lane loads the 32-byte half run (bins 4q .. 4q+3) of its element and
//    transmit, so a wave reads whole 64-byte runs (16 transmits x 2 elements, 2 KB); one
//    v_permlane16_swap per bin pair (b, b+4) exchanges the halves into the B operands.
//  * Phase: the lane needs one component of W_b for b = 0..7: Re W for (Re row, Re part) and
//    (Im row, Im part), -Im W for (Re row, Im part), Im W for (Im row, Re part), i.e.
//    Re(a' D_b) with a' = a, i a or -i a for the anchor a; D_b = D_1^b (b <= 3) or
//    D_4 D_1^(b-4) (three products at most past the anchor).
//  * The workgroup's angle tile rt covers 8-angle table tiles t8 = rt R8 + t (half t8 % 2 of
//    the 16-angle table tile t8 / 2); tiles past the table re-read its last one (their rows
//    lie past M and are not stored).
//  * Elements past the last one re-read its spectrum and steps; their anchors lie past the end
//    of the anchor view, whose loads then return zero (the element offset is in the
//    bounds-checked vector offset).
template <int R8>
__device__ __forceinline__ void contract_body(const float2* __restrict__ X, const float4* __restrict__ d14,
                                              const float2* __restrict__ anc, float2* __restrict__ Y, int ntx,
                                              int M, int L, int ncol, int kpad, int kb, int rt, int ct,
                                              float* __restrict__ lds) {
    constexpr int kDepth = contract_depth<R8>();
    constexpr int kColF = contract_col_floats<R8>();
    const int tid = threadIdx.x;
    const int e4 = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nrt16 = (M + 15) / 16;

    floatx4 acc[R8][kBinBlock];
#pragma unroll
    for (int t = 0; t < R8; ++t)
#pragma unroll
        for (int b = 0; b < kBinBlock; ++b) acc[t][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // lane roles
    const int e = lane >> 5, q = (lane >> 4) & 1, rowtype = (lane >> 3) & 1, o8 = lane & 7;
    const int c0 = ct * kContractCols;
    const int icol = min(c0 + (lane & 15), ntx - 1) - c0;
    // element l of this lane's operands: spectrum at byte xlane + l xstride of
    // X + spec_index(8 kb, 0, c0) (padding columns past the last transmit, never written, read
    // the last transmit's run; their results are discarded); steps at byte dlane + tile_d[t] +
    // 256 l of D14; anchor at byte alane_t[t] + 128 l of its view
    const uint32_t xlane = (uint32_t)icol * 64 + (uint32_t)q * 32;
    const uint32_t dlane = (uint32_t)o8 * sizeof(float4) + (uint32_t)e * 256;  // + the pair's element
    const size_t xstride = (size_t)ncol * kBinBlock * sizeof(float2);
    const __amdgpu_buffer_rsrc_t xv =
        buffer_view(X + spec_index(kb * kBinBlock, 0, c0, L, ncol), (uint32_t)(L * xstride));
    const __amdgpu_buffer_rsrc_t dv = buffer_view(d14, (uint32_t)nrt16 * L * 256);
    __amdgpu_buffer_rsrc_t av[R8];
    uint32_t tile_d[R8], alane_t[R8];
#pragma unroll
    for (int t = 0; t < R8; ++t) {
        const int t8 = min(rt * R8 + t, 2 * nrt16 - 1);
        tile_d[t] = (uint32_t)(t8 >> 1) * L * 256 + (uint32_t)(t8 & 1) * 128;
        av[t] = buffer_view(anc + ((size_t)kb * nrt16 + (t8 >> 1)) * L * 16, (uint32_t)L * 128);
        alane_t[t] = (uint32_t)o8 * sizeof(float2) + (uint32_t)(t8 & 1) * 64;
    }
    const int last = L - 1;
    const uint32_t xlane_e = xlane + (uint32_t)e * (uint32_t)xstride;  // + the pair's element
    // pair j = elements 2j, 2j + 1 (lanes of element 1 one row further); pairs past the end
    // re-read the last element and the row after it (the next bin block's first row, or for the
    // last block the Nyquist block; the next table row), which the zero anchor of an element
    // past the last one cancels: anchors are read with the element in the bounds-checked vector
    // offset of their view, so that reads past it return zero
    auto load_phase_tile = [&](PairLoads<R8>& d, int t, int j) {
        const uint32_t r = (uint32_t)min(2 * j, last);
        d.d[t] = buffer_load4(dv, dlane, tile_d[t] + r * 256);
        d.a[t] = buffer_load2(av[t], alane_t[t] + (uint32_t)(2 * j + e) * 128, 0);
    };
    auto load_phase = [&](PairLoads<R8>& d, int j) {
#pragma unroll
        for (int t = 0; t < R8; ++t) load_phase_tile(d, t, j);
    };
    auto load_spectrum = [&](PairLoads<R8>& d, int j) {
        const uint32_t r = (uint32_t)min(2 * j, last);
        d.x0 = buffer_load4(xv, xlane_e, r * (uint32_t)xstride);
        d.x1 = buffer_load4(xv, xlane_e + 16, r * (uint32_t)xstride);
    };
    // component of the lane's phases: Re(a' D_b) with a' = a (rowtype == q), i a = (-Im a, Re a)
    // for (Re row, Im part), -i a = (Im a, -Re a) for (Im row, Re part)
    const bool rot = rowtype != q;
    const uint32_t sx = (rowtype == 0 && q == 1) ? 0x80000000u : 0u;
    const uint32_t sy = (rowtype == 1 && q == 0) ? 0x80000000u : 0u;

    // this wave's element pairs j = e4 + 4 t, t < nt, in whole steps of kDepth pairs
    const int npairs = (L + 1) >> 1;
    const int nt = max(0, (npairs - e4 + 3) >> 2);
    // steps of kDepth pairs, kRounds per pass of the loop (with two, a pass's waits count the
    // loads of both its halves, not only its own half's; one at R8 = 4 keeps the registers
    // within 256)
    constexpr int kRounds = R8 == 4 ? 1 : 2;
    const int steps = kRounds * ((nt + kRounds * kDepth - 1) / (kRounds * kDepth));
    PairLoads<R8> buf[kDepth];
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
        load_phase(buf[u], e4 + 4 * u);
        load_spectrum(buf[u], e4 + 4 * u);
    }
    // the loop is entered with these arrived (the compiler issues them in its own order; its
    // waits in the loop then count only the loop's own loads)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    int j = e4;
    for (int it = 0; it < steps; it += kRounds, j += 4 * kRounds * kDepth) {
#pragma unroll
        for (int uu = 0; uu < kRounds * kDepth; ++uu) {
            const int u = uu % kDepth;
            const PairLoads<R8>& c = buf[u];
            // B operands of the 8 bins: (bin i, bin i + 4) from the lane's half runs
            float bop[kBinBlock];
            {
                const float re[4] = {c.x0.x, c.x0.z, c.x1.x, c.x1.z};
                const float im[4] = {c.x0.y, c.x0.w, c.x1.y, c.x1.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const auto sw =
                        __builtin_amdgcn_permlane16_swap(__float_as_uint(re[i]), __float_as_uint(im[i]), false, false);
                    bop[i] = __uint_as_float(sw[0]);
                    bop[i + 4] = __uint_as_float(sw[1]);
                }
            }
            // per 8-angle tile: its A operands Re(a' D_b), D_b = D_1^b (b < 4), D_4 D_1^(b-4), then
            // the tile's loads for the pair kDepth steps ahead (into the same registers), then its
            // products
#pragma unroll
            for (int t = 0; t < R8; ++t) {
                float aop[kBinBlock];
                const float2 a = c.a[t];
                const float2 ap = rot ? make_float2(__uint_as_float(__float_as_uint(a.y) ^ sx),
                                                    __uint_as_float(__float_as_uint(a.x) ^ sy))
                                      : a;
                const float2 d1 = make_float2(c.d[t].x, c.d[t].y), d4 = make_float2(c.d[t].z, c.d[t].w);
                const float2 w1 = cmul2(ap, d1), w2 = cmul2(w1, d1);
                const float2 w4 = cmul2(ap, d4), w5 = cmul2(w4, d1), w6 = cmul2(w5, d1);
                aop[0] = ap.x;
                aop[1] = w1.x;
                aop[2] = w2.x;
                aop[3] = __builtin_fmaf(w2.x, d1.x, -(w2.y * d1.y));
                aop[4] = w4.x;
                aop[5] = w5.x;
                aop[6] = w6.x;
                aop[7] = __builtin_fmaf(w6.x, d1.x, -(w6.y * d1.y));
                __builtin_amdgcn_sched_barrier(0);
                load_phase_tile(buf[u], t, j + 4 * (uu + kDepth));
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int b = 0; b < kBinBlock; ++b)
                    acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[b], bop[b], acc[t][b], 0, 0, 0);
            }
            // the spectrum after the products that read its swapped copy
            __builtin_amdgcn_sched_barrier(0);
            load_spectrum(buf[u], j + 4 * (uu + kDepth));
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // element quarters summed as (q0 + q2) + (q1 + q3): quarters 2, 3 (then 1) hand their sums
    // to the wave two (then one) below through LDS slot e4 % 2
    constexpr int kSlot = R8 * kBinBlock * 4 * 64;  // floats per wave slot
    auto put = [&](int slot) {
        float* d = lds + slot * kSlot + lane;
#pragma unroll
        for (int t = 0; t < R8; ++t)
#pragma unroll
            for (int b = 0; b < kBinBlock; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) d[((t * kBinBlock + b) * 4 + v) * 64] = acc[t][b][v];
    };
    auto add = [&](int slot) {
        const float* d = lds + slot * kSlot + lane;
#pragma unroll
        for (int t = 0; t < R8; ++t)
#pragma unroll
            for (int b = 0; b < kBinBlock; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][b][v] += d[((t * kBinBlock + b) * 4 + v) * 64];
    };
    if (e4 >= 2) put(e4 & 1);
    __syncthreads();
    if (e4 < 2) add(e4);
    __syncthreads();
    if (e4 == 1) put(0);
    __syncthreads();
    if (e4 == 0) add(0);
    __syncthreads();
    // results to LDS as [column][angle][bin][Re, Im], then out as 64-byte runs (8 bins of one
    // (i, o)), 8 threads per run
    if (e4 == 0) {
        const int col = lane & 15;
        const int comp = lane >> 5, o4 = ((lane >> 4) & 1) * 4;
#pragma unroll
        for (int t = 0; t < R8; ++t)
#pragma unroll
            for (int b = 0; b < kBinBlock; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    lds[col * kColF + ((8 * t + o4 + v) * kBinBlock + b) * 2 + comp] = acc[t][b][v];
    }
    __syncthreads();
    const float2* yst = reinterpret_cast<const float2*>(lds);
    constexpr int kAng = 8 * R8;
#pragma unroll
    for (int u = 0; u < kContractCols * kAng * kBinBlock / kContractThreads; ++u) {
        const int f = tid + u * kContractThreads;  // float2 f & 7 of run f >> 3
        const int run = f >> 3, q8 = f & 7;
        const int il = run / kAng, ol = run % kAng;
        const int i = c0 + il, o = rt * kAng + ol;
        if (i < ntx && o < M)
            Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q8] = yst[(il * kColF) / 2 + ol * kBinBlock + q8];
    }
}

// ---------------------------------------------------------------------------------------
// Split-precision contraction: the same per-bin product with 16-bit MFMA inputs.  Every
// spectrum value and phase is split as x = hi + lo, hi = round16(x), lo = round16(x - hi)
// (BF16 or FP16), and Y = Wh Xl + Wl Xh + Wh Xh accumulated in FP32 on
// v_mfma_f32_32x32x16_{bf16,f16} (eight complex elements per instruction: K = 8 elements x
// {Re, Im}; lane l holds K slice 8 (l / 32) .. + 7, i.e. elements 4 (l / 32) .. + 3, of row or
// column l % 32).  The dropped Wl Xl term and the residuals are below 2^-16 (BF16) or 2^-22
// (FP16) of the terms.  The forward transform stores the spectrum already split (its 8 bytes
// per bin: the hi pair and the lo pair), so the B operands are loaded words; FP16 spectra are
// scaled by 2^e before the split so that |X| < 2^15 (|X| <= 2 T 32768 for int16 records), and
// Y by 2^-e here (both exact).  Workgroup: one bin block, 16 T16 receive angles (one or two
// MFMA row tiles per wave), 32 transmits; wave w takes bin pair w over all elements.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool F16>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

// Loads of one group of 8 elements for one lane: its 4 elements' spectrum words (bins 2p and
// 2p+1), and per 16-angle tile the anchors and the lane's own coefficients of both bins.
template <int T16>
struct SplitLoads {
    float4 x[4];  // words of bins 2p, 2p + 1: (hi pair, lo pair, hi pair, lo pair)
    float2 a[T16][4];
    float4 d[T16][4];
};

template <bool F16, int T16>
__device__ __forceinline__ void contract_split_body(const float2* __restrict__ X, const float4* __restrict__ cf,
                                                    const float2* __restrict__ anc, float2* __restrict__ Y, int ntx,
                                                    int M, int L, int ncol, int kpad, float yscale, int kb,
                                                    int rt, int ct, float2* __restrict__ buf) {
    const int tid = threadIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int g = lane >> 5, col = lane & 31, orow = col & 15;
    const int nrt16 = (M + 15) / 16;

    floatx16 acc[T16][2];
#pragma unroll
    for (int t = 0; t < T16; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][0][v] = acc[t][1][v] = 0.0f;

    // the lane's element l = l0 + 4 g + e: spectrum words of bins 2p, 2p+1 at byte
    // xlane + (l0 + e) xstride of X + spec_index(8 kb + 2p, 0, 32 ct) (padding columns read the
    // last transmit's run, results discarded); coefficients at dlane + (l0 + e) 1024 of the
    // (tile, p) slab of Cf (the lane's row entry of the Re part: (Re D, -Im D) for Re rows,
    // (Im D, Re D) for Im rows, both bins); past the last element the wave-uniform part of the
    // element offset stays at the last one, so a lane reads at most 4 rows past its slab (the
    // next bin block or the Nyquist block of the spectrum, the next table slab), and those
    // elements enter with a zero anchor
    const uint32_t xstride = (uint32_t)ncol * kBinBlock * sizeof(float2);
    const int icol = min(ct * 32 + col, ntx - 1) - ct * 32;
    const __amdgpu_buffer_rsrc_t xv =
        buffer_view(X + spec_index(kb * kBinBlock + 2 * p, 0, ct * 32, L, ncol), (uint32_t)L * xstride);
    __amdgpu_buffer_rsrc_t dv[T16];
    const float2* ablk[T16];
#pragma unroll
    for (int t = 0; t < T16; ++t) {
        const int r16 = min(rt * T16 + t, nrt16 - 1);  // tiles past the table re-read its last one
        dv[t] = buffer_view(cf + (size_t)(r16 * 4 + p) * L * 64, (uint32_t)L * 1024);
        ablk[t] = anc + ((size_t)kb * nrt16 + r16) * L * 16;
    }
    const uint32_t xlane = (uint32_t)icol * 64 + (uint32_t)(4 * g) * xstride;
    const uint32_t dlane = (uint32_t)col * sizeof(float4) + (uint32_t)(4 * g) * 1024;
    constexpr int kSplitDepth = 2;  // groups of 8 elements whose loads are in flight per wave

    for (int c0 = 0; c0 < L; c0 += kAnchorChunk) {
        const int cn = min(kAnchorChunk, L - c0);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T16; ++t) stage_anchors(buf + t * kAnchorChunk * 16, ablk[t], c0, cn, tid);
        __syncthreads();
        const int last = c0 + cn - 1;
        auto load_coef = [&](SplitLoads<T16>& q, int l0) {
#pragma unroll
            for (int t = 0; t < T16; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    q.d[t][e] = buffer_load4(dv[t], dlane, (uint32_t)min(l0 + e, L - 1) * 1024);
                    q.a[t][e] = buf[t * kAnchorChunk * 16 + min(l0 + 4 * g + e - c0, cn - 1) * 16 + orow];
                }
        };
        auto load_spectrum = [&](SplitLoads<T16>& q, int l0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) q.x[e] = buffer_load4(xv, xlane, (uint32_t)min(l0 + e, L - 1) * xstride);
        };
        // whole groups of 8 elements in steps of kSplitDepth groups, two steps per pass
        const int groups = (cn + 7) / 8;
        const int steps = 2 * ((groups + 2 * kSplitDepth - 1) / (2 * kSplitDepth));
        SplitLoads<T16> q[kSplitDepth];
#pragma unroll
        for (int u = 0; u < kSplitDepth; ++u) {
            load_coef(q[u], c0 + 8 * u);
            load_spectrum(q[u], c0 + 8 * u);
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the loop counts only its own loads
        int e = c0;
        for (int it = 0; it < steps; it += 2, e += 16 * kSplitDepth) {
#pragma unroll
            for (int uu = 0; uu < 2 * kSplitDepth; ++uu) {
                const int u = uu % kSplitDepth;
                const int l0 = e + 8 * uu;
                const SplitLoads<T16>& c = q[u];
                // B: the stored halves of bins 2p (x, y) and 2p + 1 (z, w) of the 4 elements
                const u32x4 bh0 = {__float_as_uint(c.x[0].x), __float_as_uint(c.x[1].x), __float_as_uint(c.x[2].x),
                                   __float_as_uint(c.x[3].x)};
                const u32x4 bl0 = {__float_as_uint(c.x[0].y), __float_as_uint(c.x[1].y), __float_as_uint(c.x[2].y),
                                   __float_as_uint(c.x[3].y)};
                const u32x4 bh1 = {__float_as_uint(c.x[0].z), __float_as_uint(c.x[1].z), __float_as_uint(c.x[2].z),
                                   __float_as_uint(c.x[3].z)};
                const u32x4 bl1 = {__float_as_uint(c.x[0].w), __float_as_uint(c.x[1].w), __float_as_uint(c.x[2].w),
                                   __float_as_uint(c.x[3].w)};
                // per tile: A row pairs (Re rows (Wr, -Wi), Im rows (Wi, Wr)) from the anchor and the
                // lane's coefficient c, (Re(a) c.x + Im(a) c.y, Re(a) c.y - Im(a) c.x), split
                uint32_t hv[T16][4][4];
#pragma unroll
                for (int t = 0; t < T16; ++t)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float2 an = l0 + 4 * g + k <= last ? c.a[t][k] : make_float2(0.f, 0.f);
                        const float4 cw = c.d[t][k];
                        split16_pair<F16>(__builtin_fmaf(an.x, cw.x, an.y * cw.y),
                                          __builtin_fmaf(an.x, cw.y, -(an.y * cw.x)), hv[t][0][k], hv[t][1][k]);
                        split16_pair<F16>(__builtin_fmaf(an.x, cw.z, an.y * cw.w),
                                          __builtin_fmaf(an.x, cw.w, -(an.y * cw.z)), hv[t][2][k], hv[t][3][k]);
                    }
                // the buffer takes the group kSplitDepth ahead: coefficients and anchors now, the
                // spectrum after the products that read it
                __builtin_amdgcn_sched_barrier(0);
                load_coef(q[u], l0 + 8 * kSplitDepth);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < T16; ++t) {
                    const u32x4 ah0 = {hv[t][0][0], hv[t][0][1], hv[t][0][2], hv[t][0][3]};
                    const u32x4 al0 = {hv[t][1][0], hv[t][1][1], hv[t][1][2], hv[t][1][3]};
                    const u32x4 ah1 = {hv[t][2][0], hv[t][2][1], hv[t][2][2], hv[t][2][3]};
                    const u32x4 al1 = {hv[t][3][0], hv[t][3][1], hv[t][3][2], hv[t][3][3]};
                    acc[t][0] = mfma16<F16>(ah0, bl0, acc[t][0]);
                    acc[t][0] = mfma16<F16>(al0, bh0, acc[t][0]);
                    acc[t][0] = mfma16<F16>(ah0, bh0, acc[t][0]);
                    acc[t][1] = mfma16<F16>(ah1, bl1, acc[t][1]);
                    acc[t][1] = mfma16<F16>(al1, bh1, acc[t][1]);
                    acc[t][1] = mfma16<F16>(ah1, bh1, acc[t][1]);
                }
                __builtin_amdgcn_sched_barrier(0);
                load_spectrum(q[u], l0 + 8 * kSplitDepth);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // results to LDS as [column][angle][bin], then out as 64-byte runs (8 bins of one (i, o))
    constexpr int kCol = split_col_float2<T16>();
    __syncthreads();
#pragma unroll
    for (int t = 0; t < T16; ++t)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int ol = 16 * t + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            buf[col * kCol + ol * kBinBlock + 2 * p] = make_float2(acc[t][0][v] * yscale, acc[t][0][v + 8] * yscale);
            buf[col * kCol + ol * kBinBlock + 2 * p + 1] =
                make_float2(acc[t][1][v] * yscale, acc[t][1][v + 8] * yscale);
        }
    __syncthreads();
    constexpr int kAng = 16 * T16;
#pragma unroll
    for (int u = 0; u < 32 * kAng * kBinBlock / kSplitThreads; ++u) {
        const int f = tid + u * kSplitThreads;
        const int run = f >> 3, q8 = f & 7;
        const int il = run / kAng, ol = run % kAng;
        const int i = ct * 32 + il, o = rt * kAng + ol;
        if (i < ntx && o < M) Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q8] = buf[il * kCol + ol * kBinBlock + q8];
    }
}

// Bin block kb and angle tile rt of workgroup x of a launch over nkb x nrt such workgroups
// (nkb a multiple of 8): the angle tiles of one bin block get ids 8 apart, so they land on one
// XCD (workgroups are dealt to the 8 XCDs in turn) back to back and share its L2 for the
// spectrum they all read.
__device__ __forceinline__ void tile_of(int x, int nrt, int& kb, int& rt) {
    kb = 8 * (x / (8 * nrt)) + (x & 7);
    rt = (x >> 3) % nrt;
}

template <int R8>
__global__ __launch_bounds__(kContractThreads, 2) void contract_kernel(const float2* __restrict__ X,
                                                                        const float4* __restrict__ d14,
                                                                        const float2* __restrict__ anc,
                                                                        float2* __restrict__ Y, int ntx, int M,
                                                                        int L, int ncol, int kpad) {
    __shared__ __attribute__((aligned(16))) float lds[contract_lds_floats<R8>()];
    int kb, rt;
    tile_of(blockIdx.x, contract_angle_tiles(M), kb, rt);
    contract_body<R8>(X, d14, anc, Y, ntx, M, L, ncol, kpad, kb, rt, blockIdx.z, lds);
}

template <bool F16, int T16>
__global__ __launch_bounds__(kSplitThreads, 2) void contract_split_kernel(
    const float2* __restrict__ X, const float4* __restrict__ cf, const float2* __restrict__ anc,
    float2* __restrict__ Y, int ntx, int M, int L, int ncol, int kpad, float yscale) {
    __shared__ __attribute__((aligned(16))) float2 buf[split_lds_float2<T16>()];
    int kb, rt;
    tile_of(blockIdx.x, (M + 16 * T16 - 1) / (16 * T16), kb, rt);
    contract_split_body<F16, T16>(X, cf, anc, Y, ntx, M, L, ncol, kpad, yscale, kb, rt, blockIdx.z, buf);
}

// Grouped launches over the frames of one FFT-length class: block b runs block b - block0
// of frame entry blk[b], in the per-frame grid order (bin block fastest, then receive tile,
// then transmit tile).  PREC: 0 FP32, 1 BF16 hi+lo, 2 FP16 hi+lo.
template <int PREC>
__global__ __launch_bounds__(PREC == 0 ? kContractThreads : kSplitThreads, 2) void contract_grouped(
    const ContractEntry* __restrict__ tab, const int32_t* __restrict__ blk, float2* __restrict__ ws) {
    const ContractEntry e = tab[blk[blockIdx.x]];
    int local = (int)blockIdx.x - e.block0;
    const int kb = local % e.nkb;
    local /= e.nkb;
    const int rt = local % e.nrt, ct = local / e.nrt;
    const PhaseTables pt{nullptr, e.M, reinterpret_cast<float4*>(ws + e.d_off)};
    if constexpr (PREC == 0) {
        __shared__ __attribute__((aligned(16))) float lds[contract_lds_floats<4>()];
        const float4* d14 = pt.d14(e.L);
        const float2* anc = pt.anc(e.L);
        float2* X = ws + e.x_off;
        float2* Y = ws + e.y_off;
        switch (contract_r8(e.M)) {
            case 1: contract_body<1>(X, d14, anc, Y, e.ntx, e.M, e.L, e.ncol, e.kpad, kb, rt, ct, lds); break;
            case 2: contract_body<2>(X, d14, anc, Y, e.ntx, e.M, e.L, e.ncol, e.kpad, kb, rt, ct, lds); break;
            case 3: contract_body<3>(X, d14, anc, Y, e.ntx, e.M, e.L, e.ncol, e.kpad, kb, rt, ct, lds); break;
            default: contract_body<4>(X, d14, anc, Y, e.ntx, e.M, e.L, e.ncol, e.kpad, kb, rt, ct, lds); break;
        }
    } else {
        __shared__ __attribute__((aligned(16))) float2 buf[split_lds_float2<2>()];
        if (split_t16(e.M) == 1)
            contract_split_body<PREC == 2, 1>(ws + e.x_off, pt.cf, pt.anc(e.L), ws + e.y_off, e.ntx, e.M, e.L, e.ncol,
                                              e.kpad, e.yscale, kb, rt, ct, buf);
        else
            contract_split_body<PREC == 2, 2>(ws + e.x_off, pt.cf, pt.anc(e.L), ws + e.y_off, e.ntx, e.M, e.L, e.ncol,
                                              e.kpad, e.yscale, kb, rt, ct, buf);
    }
}

// bins 0 .. n/2 - 1 (the Nyquist bin is summed by the inverse transform)
// FP32: bin blocks x angle tiles of 8 R8 x column groups of 16; split precision: bin blocks x
// angle tiles of 16 T16 x column groups of 32 (x: bin blocks x angle tiles in tile_of order,
// z: column groups)
dim3 contract_grid(int log2n, int precision, int M, int ntx, int ncol) {
    if (precision == KK_PREC_FP32)
        return dim3(contract_bin_blocks(log2n) * contract_angle_tiles(M), 1, (ntx + kContractCols - 1) / kContractCols);
    const int a = 16 * split_t16(M);
    return dim3(contract_bin_blocks(log2n) * ((M + a - 1) / a), 1, ncol / 32);
}

}  // namespace

// FP32 or split-precision contraction of one frame; the phase tables sit at pt.cf.
hipError_t launch_contract(int log2n, int precision, const float2* X, const PhaseTables& pt, float2* Y, int ntx,
                           int L, int ncol, int kpad, float xscale, hipStream_t st) {
    if (log2n < kMinLog2Fft || log2n > kMaxLog2Fft) return hipErrorInvalidValue;
    const dim3 grid = contract_grid(log2n, precision, pt.M, ntx, ncol);
    const dim3 block(precision == KK_PREC_FP32 ? kContractThreads : kSplitThreads);
    const float2* anc = pt.anc(L);
    switch (precision) {
        case KK_PREC_FP32:
            switch (contract_r8(pt.M)) {
                case 1:
                    hipLaunchKernelGGL(contract_kernel<1>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L,
                                       ncol, kpad);
                    break;
                case 2:
                    hipLaunchKernelGGL(contract_kernel<2>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L,
                                       ncol, kpad);
                    break;
                case 3:
                    hipLaunchKernelGGL(contract_kernel<3>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L,
                                       ncol, kpad);
                    break;
                default:
                    hipLaunchKernelGGL(contract_kernel<4>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L,
                                       ncol, kpad);
                    break;
            }
            break;
        case KK_PREC_BF16X3:
            if (split_t16(pt.M) == 1)
                hipLaunchKernelGGL((contract_split_kernel<false, 1>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M,
                                   L, ncol, kpad, 1.0f / xscale);
            else
                hipLaunchKernelGGL((contract_split_kernel<false, 2>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M,
                                   L, ncol, kpad, 1.0f / xscale);
            break;
        case KK_PREC_FP16X3:
            if (split_t16(pt.M) == 1)
                hipLaunchKernelGGL((contract_split_kernel<true, 1>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M, L,
                                   ncol, kpad, 1.0f / xscale);
            else
                hipLaunchKernelGGL((contract_split_kernel<true, 2>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M, L,
                                   ncol, kpad, 1.0f / xscale);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_contract_grouped(int log2n, int precision, const ContractEntry* tab, const int32_t* blk, int blocks,
                                   float2* ws, const int32_t* plan, hipStream_t st) {
    (void)plan;
    if (log2n < kMinLog2Fft || log2n > kMaxLog2Fft) return hipErrorInvalidValue;
    const dim3 g(blocks), b(kContractThreads), bs(kSplitThreads);
    switch (precision) {
        case KK_PREC_FP32: hipLaunchKernelGGL((contract_grouped<0>), g, b, 0, st, tab, blk, ws); break;
        case KK_PREC_BF16X3: hipLaunchKernelGGL((contract_grouped<1>), g, bs, 0, st, tab, blk, ws); break;
        case KK_PREC_FP16X3: hipLaunchKernelGGL((contract_grouped<2>), g, bs, 0, st, tab, blk, ws); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

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
    size_t x_off, d_off, y_off, total;
};

// workspace: spectra (contraction layout), phase tables, contracted spectra [N][M][kpad]
bool decompose_layout(const kk_geom* g, int32_t N, int32_t M, int32_t tpad, DecomposeLayout* d) {
    const int lg = log2_exact(tpad);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->T < 1 || g->T > tpad || g->L < 1 || N < 1 || M < 1) return false;
    d->log2n = lg;
    d->K = tpad / 2 + 1;
    d->kpad = (d->K + kBinBlock - 1) / kBinBlock * kBinBlock;
    d->ncol = (N + 31) / 32 * 32;
    d->x_off = 0;
    d->d_off = d->x_off + align256((size_t)d->kpad * d->ncol * g->L * 8);
    d->y_off = d->d_off + align256(phase_table_bytes(M, g->L, lg));
    d->total = d->y_off + align256((size_t)N * M * d->kpad * 8);
    return true;
}

// Forward transform (with the phase tables unless the workspace holds them already) and the
// per-bin contraction of one frame into Y.
hipError_t decompose_front(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M,
                           int32_t precision, const DecomposeLayout& d, unsigned char* w, float2* Y, hipStream_t st,
                           bool tables_ready = false) {
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    const PhaseTables pt{shift_q, M, reinterpret_cast<float4*>(w + d.d_off)};
    const float xscale = precision == KK_PREC_FP16X3 ? std::ldexp(1.0f, fp16_prescale_exponent(g->T)) : 1.0f;
    hipError_t e = launch_fft_forward(rf, N * g->L, g->T, d.log2n, X, true, g->L, d.ncol, d.kpad, st,
                                      tables_ready ? nullptr : &pt, precision, xscale);
    if (e != hipSuccess) return e;
    return launch_contract(d.log2n, precision, X, pt, Y, N, g->L, d.ncol, d.kpad, xscale, st);
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

namespace {
// kk_decompose and kk_decompose_prepared (tables_ready: the workspace holds the phase tables).
int32_t decompose_call(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M, int32_t tpad,
                       int32_t precision, float* rf_theta, void* ws, size_t ws_bytes, void* stream,
                       bool tables_ready) {
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
    float2* Y = reinterpret_cast<float2*>(w + d.y_off);
    if (decompose_front(rf, N, g, shift_q, M, precision, d, w, Y, st, tables_ready) != hipSuccess) return KK_E_HIP;
    NyquistSum nyq{reinterpret_cast<const float2*>(w + d.x_off), shift_q, M, g->L, d.ncol};
    if (launch_fft_inverse(Y, N * M, d.kpad, d.log2n, reinterpret_cast<float2*>(rf_theta), g->T, st, &nyq) !=
        hipSuccess)
        return KK_E_HIP;
    return KK_OK;
}
}  // namespace

int32_t kk_decompose(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M, int32_t tpad,
                     int32_t precision, float* rf_theta, void* ws, size_t ws_bytes, void* stream) {
    return decompose_call(rf, N, g, shift_q, M, tpad, precision, rf_theta, ws, ws_bytes, stream, false);
}

int32_t kk_decompose_prepare(const kk_geom* g, int32_t N, const int32_t* shift_q, int32_t M, int32_t tpad,
                             int32_t precision, void* ws, size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!g || !shift_q || !ws) return KK_E_NULL;
    if (precision != KK_PREC_FP32 && precision != KK_PREC_BF16X3 && precision != KK_PREC_FP16X3)
        return KK_E_UNSUPPORTED;
    if (N < 1 || M < 1 || g->L < 1 || g->L > 65536 || g->T < 1) return KK_E_ARG;
    DecomposeLayout d;
    if (!decompose_layout(g, N, M, tpad, &d)) return KK_E_ARG;
    if ((int64_t)N * g->L > 0x7fffffff || (int64_t)N * M > 0x7fffffff) return KK_E_ARG;
    if (ws_bytes < d.total) return KK_E_WORKSPACE;
    unsigned char* w = static_cast<unsigned char*>(ws);
    const PhaseTables pt{shift_q, M, reinterpret_cast<float4*>(w + d.d_off)};
    // a blocked forward launch over no records: only its phase-table workgroups
    return launch_fft_forward(nullptr, 0, g->T, d.log2n, reinterpret_cast<float2*>(w + d.x_off), true, g->L, d.ncol,
                              d.kpad, (hipStream_t)stream, &pt) == hipSuccess
               ? KK_OK
               : KK_E_HIP;
}

int32_t kk_decompose_prepared(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M,
                              int32_t tpad, int32_t precision, float* rf_theta, void* ws, size_t ws_bytes,
                              void* stream) {
    return decompose_call(rf, N, g, shift_q, M, tpad, precision, rf_theta, ws, ws_bytes, stream, true);
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
    if (ws_bytes < d.y_off) return KK_E_WORKSPACE;  // spectra and phase steps; Y is the caller's
    hipStream_t st = (hipStream_t)stream;
    float2* Y = reinterpret_cast<float2*>(spec);
    if (decompose_front(rf, N, g, shift_q, M, precision, d, static_cast<unsigned char*>(ws), Y, st) != hipSuccess)
        return KK_E_HIP;
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
