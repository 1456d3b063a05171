// Eq. 3 receive plane-wave decomposition on gfx950, evaluated in the temporal-frequency
// domain (Sec. II-F):
//   1. analytic spectra of the N*L zero-padded records (kk_fft.hip, two records per FFT),
//      stored bin-blocked (spec_index: 64-byte runs of 8 bins per element and transmit); the
//      same launch writes the phase tables of step 2 (PhaseTables);
//   2. per bin k the complex contraction Y_k[o][i] = sum_l W_k[o][l] X_k[l][i] with
//      W_k[o][l] = exp(2 pi i r / (n 2^22)), r = (k shift[o][l]) mod (n 2^22), on MFMA
//      (v_mfma_f32_32x32x2_f32: one complex element l per instruction, 16 receive angles x
//      {Re, Im} rows by 32 transmit columns; 8 bins per workgroup, a bin pair per wave);
//   3. inverse FFT of each (i, o) spectrum, first T samples.
// Every phase comes from an exact integer turn count evaluated in FP64 and rounded once: the
// anchor W_{8 kb} of each bin block and the steps D_j (j = 0..7) within a block, so that
// W_{8 kb + j} = W_{8 kb} D_j is one complex product (two roundings) away from exact.
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

// FP32 contraction workgroup: one block of 8 bins, R8 tiles of 8 receive angles (R8 = 1 when
// M <= 8, else 2: 16 angles), 32 transmit columns; wave w takes column group g = w % 2 (16
// transmits) and element quarter e4 = w / 2 (element pairs 2j, 2j+1 with j = e4 (mod 4)), all 8
// bins; the quarters are summed at the end in a fixed order.
constexpr int kContractWaves = 8;
constexpr int kContractThreads = kContractWaves * 64;
// Element pairs whose operand loads are in flight per wave.
constexpr int kDepth = 4;
// Result staging: per transmit column, 16 angles x 8 bins x {Re, Im} floats and a pad of two
// (the 16 columns of a wave's row then fall in distinct banks).
constexpr int kYColF = 16 * kBinBlock * 2 + 2;
constexpr int kStageFloat2 = 32 * kYColF / 2;

// Split-precision workgroup: the same tile; wave w takes bin pair w % 4 over half w / 4 of the
// elements, the halves summed at the end, with the chunk's anchors staged in LDS.
constexpr int kSplitWaves = 8;
constexpr int kSplitThreads = kSplitWaves * 64;
constexpr int kAnchorChunk = 256;
constexpr int kYCol = 16 * kBinBlock + 1;  // split kernel's staging: float2 per (column, angle, bin) + pad
constexpr int kSplitBuf = kAnchorChunk * 16 > 32 * kYCol ? kAnchorChunk * 16 : 32 * kYCol;
static_assert(kSplitBuf >= 4096, "LDS buffer holds the half sums");
// Anchor loads per thread of one chunk (16-byte pieces, 8 per element).
constexpr int kAnchorLoads = (kAnchorChunk * 8 + kSplitThreads - 1) / kSplitThreads;

__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Raw buffer view of nbytes at p (gfx9 descriptor: 32-bit data format, no swizzle): loads take
// a per-lane and a wave-uniform byte offset with no vector address arithmetic, and loads past
// nbytes return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
__device__ __forceinline__ float2 buffer_load2(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane_off, (int)off, 0));
}
__device__ __forceinline__ float4 buffer_load4(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)lane_off, (int)off, 0));
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

// Per bin block (8 bins), R8 x 8 receive angles and 32 transmit columns:
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
//  * Elements past the last one re-read its spectrum and steps; their anchors lie past the end
//    of the anchor view, whose loads then return zero (the element offset is in the
//    bounds-checked vector offset).
// LDS floats of the contraction: partial sums of the element quarters (four wave slots), then
// the result staging.
template <int R8>
constexpr int contract_lds_floats() { return R8 * 8192 > 32 * kYColF ? R8 * 8192 : 32 * kYColF; }

template <int R8>
__device__ __forceinline__ void contract_body(const float2* __restrict__ X, const float4* __restrict__ d14,
                                              const float2* __restrict__ anc, float2* __restrict__ Y, int ntx,
                                              int M, int L, int ncol, int kpad, int kb, int rt, int ct,
                                              float* __restrict__ lds) {
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int g = wave & 1, e4 = wave >> 1;
    const int nrt = (M + 15) / 16;

    floatx4 acc[R8][kBinBlock];
#pragma unroll
    for (int t = 0; t < R8; ++t)
#pragma unroll
        for (int b = 0; b < kBinBlock; ++b) acc[t][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // lane roles
    const int e = lane >> 5, q = (lane >> 4) & 1, rowtype = (lane >> 3) & 1, o8 = lane & 7;
    const int icol = min(ct * 32 + g * 16 + (lane & 15), ntx - 1) - ct * 32;
    // element l of this lane's operands: spectrum at byte xlane + l xstride of
    // X + spec_index(8 kb, 0, 32 ct) (padding columns past the last transmit, never written, read
    // the last transmit's run; their results are discarded); steps at byte dlane + 256 t + 256 l
    // of D14 + rt L 16; anchor at byte alane + 64 t + 128 l of Anc + (kb nrt + rt) L 16
    const uint32_t xlane = (uint32_t)icol * 64 + (uint32_t)q * 32;
    const uint32_t dlane = (uint32_t)o8 * sizeof(float4) + (uint32_t)e * 256;  // + the pair's element
    const uint32_t alane = (uint32_t)o8 * sizeof(float2);
    const size_t xstride = (size_t)ncol * kBinBlock * sizeof(float2);
    const __amdgpu_buffer_rsrc_t xv =
        buffer_view(X + spec_index(kb * kBinBlock, 0, ct * 32, L, ncol), (uint32_t)(L * xstride));
    const __amdgpu_buffer_rsrc_t dv = buffer_view(d14 + (size_t)rt * L * 16, (uint32_t)L * 256);
    const __amdgpu_buffer_rsrc_t av = buffer_view(anc + ((size_t)kb * nrt + rt) * L * 16, (uint32_t)L * 128);
    const int last = L - 1;
    const uint32_t xlane_e = xlane + (uint32_t)e * (uint32_t)xstride;  // + the pair's element
    // pair j = elements 2j, 2j + 1 (lanes of element 1 one row further); pairs past the end
    // re-read the last element and the row after it (the next bin block's first row, or for the
    // last block the Nyquist block; the next table row), which the zero anchor of an element
    // past the last one cancels: anchors are read with the element in the bounds-checked vector
    // offset of their view, so that reads past it return zero
    auto load_phase = [&](PairLoads<R8>& d, int j) {
        const uint32_t r = (uint32_t)min(2 * j, last);
#pragma unroll
        for (int t = 0; t < R8; ++t) {
            d.d[t] = buffer_load4(dv, dlane + 128 * t, r * 256);
            d.a[t] = buffer_load2(av, alane + 64 * t + (uint32_t)(2 * j + e) * 128, 0);
        }
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
    // steps of kDepth pairs, two per pass of the loop (a pass's waits count the loads of both its
    // halves, not only its own half's)
    const int steps = 2 * ((nt + 2 * kDepth - 1) / (2 * kDepth));
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
    for (int it = 0; it < steps; it += 2, j += 8 * kDepth) {
#pragma unroll
        for (int uu = 0; uu < 2 * kDepth; ++uu) {
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
            // A operands: Re(a' D_b), D_b = D_1^b (b < 4), D_4 D_1^(b-4)
            float aop[R8][kBinBlock];
#pragma unroll
            for (int t = 0; t < R8; ++t) {
                const float2 a = c.a[t];
                const float2 ap = rot ? make_float2(__uint_as_float(__float_as_uint(a.y) ^ sx),
                                                    __uint_as_float(__float_as_uint(a.x) ^ sy))
                                      : a;
                const float2 d1 = make_float2(c.d[t].x, c.d[t].y), d4 = make_float2(c.d[t].z, c.d[t].w);
                const float2 w1 = cmul2(ap, d1), w2 = cmul2(w1, d1);
                const float2 w4 = cmul2(ap, d4), w5 = cmul2(w4, d1), w6 = cmul2(w5, d1);
                aop[t][0] = ap.x;
                aop[t][1] = w1.x;
                aop[t][2] = w2.x;
                aop[t][3] = w2.x * d1.x - w2.y * d1.y;
                aop[t][4] = w4.x;
                aop[t][5] = w5.x;
                aop[t][6] = w6.x;
                aop[t][7] = w6.x * d1.x - w6.y * d1.y;
            }
            // the buffer takes this wave's pair kDepth steps ahead (into the same registers: the
            // phase operands now, the spectrum after the products that read its swapped copy)
            __builtin_amdgcn_sched_barrier(0);
            load_phase(buf[u], j + 4 * (uu + kDepth));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < R8; ++t)
#pragma unroll
                for (int b = 0; b < kBinBlock; ++b)
                    acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[t][b], bop[b], acc[t][b], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            load_spectrum(buf[u], j + 4 * (uu + kDepth));
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // element quarters summed as (q0 + q2) + (q1 + q3): quarters 2, 3 (then 1) hand their sums
    // to the wave below through slot 2 g + (e4 & 1) of LDS
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
    if (e4 >= 2) put(2 * g + (e4 & 1));
    __syncthreads();
    if (e4 < 2) add(2 * g + e4);
    __syncthreads();
    if (e4 == 1) put(2 * g);
    __syncthreads();
    if (e4 == 0) add(2 * g);
    __syncthreads();
    // results to LDS as [column][angle][bin][Re, Im], then out as 64-byte runs (8 bins of one
    // (i, o)), 8 threads per run
    if (e4 == 0) {
        const int col = 16 * g + (lane & 15);
        const int comp = lane >> 5, o4 = ((lane >> 4) & 1) * 4;
#pragma unroll
        for (int t = 0; t < R8; ++t)
#pragma unroll
            for (int b = 0; b < kBinBlock; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    lds[col * kYColF + ((8 * t + o4 + v) * kBinBlock + b) * 2 + comp] = acc[t][b][v];
    }
    __syncthreads();
    const float2* yst = reinterpret_cast<const float2*>(lds);
#pragma unroll
    for (int u = 0; u < 32 * 16 * kBinBlock / kContractThreads; ++u) {
        const int f = tid + u * kContractThreads;  // float2 f & 7 of run f >> 3
        const int run = f >> 3, q8 = f & 7;
        const int il = run >> 4, ol = run & 15;
        const int i = ct * 32 + il, o = rt * 16 + ol;
        if (ol < 8 * R8 && i < ntx && o < M)
            Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q8] = yst[(il * kYColF) / 2 + ol * kBinBlock + q8];
    }
}

// ---------------------------------------------------------------------------------------
// Split-precision contraction: the same per-bin product with 16-bit MFMA inputs.  Every
// spectrum value and phase is split as x = hi + lo, hi = round16(x), lo = round16(x - hi)
// (BF16 or FP16), and Y = Wh Xl + Wl Xh + Wh Xh accumulated in FP32 on
// v_mfma_f32_32x32x16_{bf16,f16} (eight complex elements per instruction: K = 8 elements x
// {Re, Im}; lane l holds K slice 8 (l / 32) .. + 7, i.e. elements 4 (l / 32) .. + 3, of row or
// column l % 32).  The dropped Wl Xl term and the residuals are below 2^-16 (BF16) or 2^-22
// (FP16) of the terms.  FP16 spectra are first scaled by 2^e so that |X| < 2^15 (|X| <= 2 T
// 32768 for int16 records), and Y by 2^-e (both exact).  Same workgroup shape, spectrum
// layout and phase construction as the FP32 kernel.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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
// (first, second) -> hi pair and lo pair, low half = first
template <bool F16>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
    const float ah = half_value<F16>(a), bh = half_value<F16>(b);
    hi = half_bits<F16>(a) | (half_bits<F16>(b) << 16);
    lo = half_bits<F16>(a - ah) | (half_bits<F16>(b - bh) << 16);
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

// Loads of one group of 8 elements for one lane: its 4 elements' spectra (bins 2p and 2p+1),
// anchors and the coefficients of the lane that holds (Re row, Re part) of its angle:
// (Re D, -Im D) of both bins.
struct SplitLoads {
    float4 x[4];
    float2 a[4];
    float4 d[4];
};

template <bool F16>
__device__ __forceinline__ void contract_split_body(const float2* __restrict__ X, const float4* __restrict__ cf,
                                                    const float2* __restrict__ anc, float2* __restrict__ Y, int ntx,
                                                    int M, int L, int ncol, int kpad, float xscale, float yscale,
                                                    int kb, int rt, int ct) {
    __shared__ __attribute__((aligned(16))) float2 buf[kSplitBuf];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int p = wave & 3, h = wave >> 2;
    const int g = lane >> 5, col = lane & 31, orow = col & 15;
    const bool im_row = col >= 16;
    const int nrt = (M + 15) / 16;

    floatx16 acc0, acc1;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.0f;

    const size_t xstride = (size_t)kBinBlock * ncol;  // complex floats between elements
    // padding columns read the last transmit's spectrum (results discarded)
    const float4* xp = reinterpret_cast<const float4*>(
        X + spec_index(kb * kBinBlock + 2 * p, 0, min(ct * 32 + col, ntx - 1), L, ncol));
    const float4* dp = cf + (size_t)(rt * 4 + p) * L * 64 + orow;
    const float2* ablk = anc + ((size_t)kb * nrt + rt) * L * 16;

    for (int c0 = 0; c0 < L; c0 += kAnchorChunk) {
        const int cn = min(kAnchorChunk, L - c0);
        __syncthreads();
        stage_anchors(buf, ablk, c0, cn, tid);
        __syncthreads();
        const int half = (cn + 1) >> 1;
        const int e0 = __builtin_amdgcn_readfirstlane(c0 + h * half);
        const int e1 = __builtin_amdgcn_readfirstlane(min(c0 + cn, e0 + half));
        const int last = e1 - 1;
        auto load = [&](SplitLoads& q, int l0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = min(l0 + 4 * g + e, last);
                q.x[e] = xp[(size_t)l * (xstride / 2)];
                q.d[e] = dp[(size_t)l * 64];
                q.a[e] = buf[(l - c0) * 16 + orow];
            }
        };
        if (e0 < e1) {
            // whole groups of 8 elements, two groups of loads in flight; elements past the
            // last one re-read it and enter with a zero phase
            const int groups = (e1 - e0 + 7) / 8;
            const int steps = (groups + 1) / 2;
            SplitLoads q[2];
            load(q[0], e0);
            asm volatile("" ::: "memory");  // the prologue issues its loads in the loop's order
            load(q[1], e0 + 8);
            asm volatile("" ::: "memory");
            int e = e0;
            for (int it = 0; it < steps; ++it, e += 16) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int l0 = e + 8 * u;
                    const SplitLoads& c = q[u];
                    uint32_t hv[8][4];  // per element: A hi/lo of both bins, B hi/lo of both bins
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool valid = l0 + 4 * g + k <= last;
                        const float2 an = valid ? c.a[k] : make_float2(0.f, 0.f);
                        const float2 w0 = cmul2(an, make_float2(c.d[k].x, -c.d[k].y));
                        const float2 w1 = cmul2(an, make_float2(c.d[k].z, -c.d[k].w));
                        // A row pair: Re rows (Wr, -Wi), Im rows (Wi, Wr)
                        split_pair<F16>(im_row ? w0.y : w0.x, im_row ? w0.x : -w0.y, hv[0][k], hv[1][k]);
                        split_pair<F16>(im_row ? w1.y : w1.x, im_row ? w1.x : -w1.y, hv[2][k], hv[3][k]);
                        const float4 x = c.x[k];
                        split_pair<F16>(x.x * xscale, x.y * xscale, hv[4][k], hv[5][k]);
                        split_pair<F16>(x.z * xscale, x.w * xscale, hv[6][k], hv[7][k]);
                    }
                    const u32x4 ah0 = {hv[0][0], hv[0][1], hv[0][2], hv[0][3]};
                    const u32x4 al0 = {hv[1][0], hv[1][1], hv[1][2], hv[1][3]};
                    const u32x4 ah1 = {hv[2][0], hv[2][1], hv[2][2], hv[2][3]};
                    const u32x4 al1 = {hv[3][0], hv[3][1], hv[3][2], hv[3][3]};
                    const u32x4 bh0 = {hv[4][0], hv[4][1], hv[4][2], hv[4][3]};
                    const u32x4 bl0 = {hv[5][0], hv[5][1], hv[5][2], hv[5][3]};
                    const u32x4 bh1 = {hv[6][0], hv[6][1], hv[6][2], hv[6][3]};
                    const u32x4 bl1 = {hv[7][0], hv[7][1], hv[7][2], hv[7][3]};
                    // this group's operands are in hv: the buffer takes the group two ahead
                    load(q[u], l0 + 16);
                    acc0 = mfma16<F16>(ah0, bl0, acc0);
                    acc0 = mfma16<F16>(al0, bh0, acc0);
                    acc0 = mfma16<F16>(ah0, bh0, acc0);
                    acc1 = mfma16<F16>(ah1, bl1, acc1);
                    acc1 = mfma16<F16>(al1, bh1, acc1);
                    acc1 = mfma16<F16>(ah1, bh1, acc1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    __syncthreads();
    float* red = reinterpret_cast<float*>(buf);
    if (h == 1) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            red[((p * 2 + 0) * 16 + v) * 64 + lane] = acc0[v];
            red[((p * 2 + 1) * 16 + v) * 64 + lane] = acc1[v];
        }
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc0[v] += red[((p * 2 + 0) * 16 + v) * 64 + lane];
            acc1[v] += red[((p * 2 + 1) * 16 + v) * 64 + lane];
        }
    }
    __syncthreads();
    float2* yst = buf;
    if (h == 0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int ol = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            yst[col * kYCol + ol * kBinBlock + 2 * p] = make_float2(acc0[v] * yscale, acc0[v + 8] * yscale);
            yst[col * kYCol + ol * kBinBlock + 2 * p + 1] = make_float2(acc1[v] * yscale, acc1[v + 8] * yscale);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int f = tid + u * kSplitThreads;
        const int run = f >> 3, q = f & 7;
        const int il = run >> 4, ol = run & 15;
        const int i = ct * 32 + il, o = rt * 16 + ol;
        if (i < ntx && o < M) Y[((size_t)i * M + o) * kpad + kb * kBinBlock + q] = yst[il * kYCol + ol * kBinBlock + q];
    }
}

template <int R8>
__global__ __launch_bounds__(kContractThreads) void contract_kernel(const float2* __restrict__ X,
                                                                     const float4* __restrict__ d14,
                                                                     const float2* __restrict__ anc,
                                                                     float2* __restrict__ Y, int ntx, int M,
                                                                     int L, int ncol, int kpad) {
    __shared__ __attribute__((aligned(16))) float lds[contract_lds_floats<R8>()];
    contract_body<R8>(X, d14, anc, Y, ntx, M, L, ncol, kpad, blockIdx.x, blockIdx.y, blockIdx.z, lds);
}

template <bool F16>
__global__ __launch_bounds__(kSplitThreads) void contract_split_kernel(
    const float2* __restrict__ X, const float4* __restrict__ cf, const float2* __restrict__ anc,
    float2* __restrict__ Y, int ntx, int M, int L, int ncol, int kpad, float xscale, float yscale) {
    contract_split_body<F16>(X, cf, anc, Y, ntx, M, L, ncol, kpad, xscale, yscale, blockIdx.x, blockIdx.y,
                             blockIdx.z);
}

// Grouped launches over the frames of one FFT-length class: block b runs block b - block0
// of frame entry blk[b], in the per-frame grid order (bin block fastest, then receive tile,
// then transmit tile).  PREC: 0 FP32, 1 BF16 hi+lo, 2 FP16 hi+lo.
template <int PREC>
__global__ __launch_bounds__(PREC == 0 ? kContractThreads : kSplitThreads) void contract_grouped(
    const ContractEntry* __restrict__ tab, const int32_t* __restrict__ blk, float2* __restrict__ ws) {
    const ContractEntry e = tab[blk[blockIdx.x]];
    int local = (int)blockIdx.x - e.block0;
    const int kb = local % e.nkb;
    local /= e.nkb;
    const int rt = local % e.nrt, ct = local / e.nrt;
    const PhaseTables pt{nullptr, e.M, reinterpret_cast<float4*>(ws + e.d_off)};
    if constexpr (PREC == 0) {
        __shared__ __attribute__((aligned(16))) float lds[contract_lds_floats<2>()];
        if (e.M <= 8)
            contract_body<1>(ws + e.x_off, pt.d14(e.L), pt.anc(e.L), ws + e.y_off, e.ntx, e.M, e.L, e.ncol, e.kpad,
                             kb, rt, ct, lds);
        else
            contract_body<2>(ws + e.x_off, pt.d14(e.L), pt.anc(e.L), ws + e.y_off, e.ntx, e.M, e.L, e.ncol, e.kpad,
                             kb, rt, ct, lds);
    } else
        contract_split_body<PREC == 2>(ws + e.x_off, pt.cf, pt.anc(e.L), ws + e.y_off, e.ntx, e.M, e.L, e.ncol, e.kpad,
                                       e.xscale, e.yscale, kb, rt, ct);
}

// bins 0 .. n/2 - 1 (the Nyquist bin is summed by the inverse transform)
dim3 contract_grid(int log2n, int M, int ncol) { return dim3(contract_bin_blocks(log2n), (M + 15) / 16, ncol / 32); }

}  // namespace

// FP32 or split-precision contraction of one frame; the phase tables sit at pt.cf.
hipError_t launch_contract(int log2n, int precision, const float2* X, const PhaseTables& pt, float2* Y, int ntx,
                           int L, int ncol, int kpad, float xscale, hipStream_t st) {
    if (log2n < kMinLog2Fft || log2n > kMaxLog2Fft) return hipErrorInvalidValue;
    const dim3 grid = contract_grid(log2n, pt.M, ncol);
    const dim3 block(precision == KK_PREC_FP32 ? kContractThreads : kSplitThreads);
    const float2* anc = pt.anc(L);
    switch (precision) {
        case KK_PREC_FP32:
            if (pt.M <= 8)
                hipLaunchKernelGGL(contract_kernel<1>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L, ncol,
                                   kpad);
            else
                hipLaunchKernelGGL(contract_kernel<2>, grid, block, 0, st, X, pt.d14(L), anc, Y, ntx, pt.M, L, ncol,
                                   kpad);
            break;
        case KK_PREC_BF16X3:
            hipLaunchKernelGGL((contract_split_kernel<false>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M, L,
                               ncol, kpad, xscale, 1.0f / xscale);
            break;
        case KK_PREC_FP16X3:
            hipLaunchKernelGGL((contract_split_kernel<true>), grid, block, 0, st, X, pt.cf, anc, Y, ntx, pt.M, L,
                               ncol, kpad, xscale, 1.0f / xscale);
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
    hipError_t e = launch_fft_forward(rf, N * g->L, g->T, d.log2n, X, true, g->L, d.ncol, d.kpad, st,
                                      tables_ready ? nullptr : &pt);
    if (e != hipSuccess) return e;
    const float xscale = precision == KK_PREC_FP16X3 ? std::ldexp(1.0f, fp16_prescale_exponent(g->T)) : 1.0f;
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
