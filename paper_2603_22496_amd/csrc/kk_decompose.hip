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

// Contraction workgroup: one block of 8 bins, 16 receive angles, 32 transmit columns; wave w
// takes the bin pair p = w % 4 (bins 8 kb + 2p, 8 kb + 2p + 1) over half h = w / 4 of the
// elements, and the two halves are summed at the end.
constexpr int kContractWaves = 8;
constexpr int kContractThreads = kContractWaves * 64;
// Elements whose anchor phases W_{8 kb}[o][l] sit in LDS at once.
constexpr int kAnchorChunk = 256;
// Elements whose operand loads are in flight per wave.
constexpr int kDepth = 8;
// Result staging per transmit column: 16 angles x 8 bins and a pad (a half-wave's 32 columns
// then write 64 distinct banks).
constexpr int kYCol = 16 * kBinBlock + 1;
constexpr int kBufFloat2 = 32 * kYCol;  // >= anchors (kAnchorChunk x 16) and the half sums (4096)
static_assert(kBufFloat2 >= kAnchorChunk * 16 && kBufFloat2 >= 4096, "LDS buffer");

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

// Anchor phases of elements [c0, c0 + cn) of one bin block and receive tile:
// anc[(l - c0) 16 + o % 16] = W_{8 kb}[o][l] (zero for o >= M), evaluated exactly.
template <int LOG2N>
__device__ __forceinline__ void build_anchors(float2* anc, const float2* fac, const int32_t* __restrict__ shift,
                                              int kb, int rt, int M, int L, int c0, int cn, int tid) {
    for (int e = tid; e < cn * 16; e += kContractThreads) {
        const int o = rt * 16 + (e & 15), l = c0 + (e >> 4);
        anc[e] = o < M ? shear_phase<LOG2N>((uint32_t)(kb * kBinBlock), shift[(size_t)o * L + l], fac)
                       : make_float2(0.f, 0.f);
    }
}

// Lane roles of v_mfma_f32_32x32x2_f32.  A (32 x 2): row lane % 32 = {Re rows 0..15, Im rows
// 16..31} x 16 receive angles, column lane / 32 = {Re, Im} part of the element; the lane
// supplies Wr (Re row, Re part), -Wi (Re row, Im part), Wi (Im row, Re part), Wr (Im, Im).
// B (2 x 32): part lane / 32 of transmit column lane % 32.
struct LaneRole {
    int part, col, orow;
    bool use_im;
    uint32_t negmask;
    __device__ __forceinline__ explicit LaneRole(int lane) {
        part = lane >> 5;
        col = lane & 31;
        orow = col & 15;
        const int ytype = col >> 4;
        use_im = ytype != part;
        negmask = (ytype == 0 && part == 1) ? 0x80000000u : 0u;
    }
    __device__ __forceinline__ float pick(float2 w) const {
        return __uint_as_float(__float_as_uint(use_im ? w.y : w.x) ^ negmask);
    }
};

// Operands of one element in flight: spectrum (bin 2p + part of this lane's transmit), anchor
// phase of this lane's angle, phase steps {D_2p, D_1}.
struct ElemLoads {
    float2 x;
    float2 a;
    float4 d;
};

// Per bin block (8 bins), receive tile of 16 and transmit tile of 32:
// Y_k[o][i] = sum_l W_k[o][l] X_k[l][i].  W_{8kb+2p} = W_{8kb} D_2p and W_{8kb+2p+1} =
// W_{8kb+2p} D_1 (two roundings from exactly evaluated factors).  The spectrum is read
// straight from global memory: one 8-byte load per lane gives bins 2p (lanes 0..31 Re, 32..63
// Im after one v_permlane32_swap) and 2p+1; no LDS staging and no barrier in the element loop.
// Results leave through LDS as 64-byte runs (8 bins of one (i, o)).
template <int LOG2N>
__device__ __forceinline__ void contract_body(const float2* __restrict__ X, const int32_t* __restrict__ shift,
                                              const float4* __restrict__ phd, float2* __restrict__ Y, int ntx,
                                              int M, int L, int ncol, int kpad, int kb, int rt, int ct) {
    constexpr int N = 1 << LOG2N;
    __shared__ float2 fac[64 + N / 64];
    __shared__ __attribute__((aligned(16))) float2 buf[kBufFloat2];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int p = wave & 3, h = wave >> 2;
    const LaneRole R(lane);
    build_phase_factors<LOG2N>(fac, tid);

    floatx16 acc0, acc1;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.0f;

    // element l of this lane's operands: spectrum X[spec_index(8 kb + 2p + part, l, 32 ct + col)],
    // phase steps PhD[((rt 4 + p) L + l) 16 + orow]
    const size_t xstride = (size_t)kBinBlock * ncol;
    // padding columns past the last transmit (never written) read the last transmit's spectrum,
    // whose lines are fetched anyway; their results are discarded
    const int icol = min(ct * 32 + R.col, ntx - 1);
    const float2* xp = X + spec_index(kb * kBinBlock + 2 * p, 0, icol, L, ncol) + R.part;
    const float4* dp = phd + ((size_t)rt * 4 + p) * L * 16 + R.orow;

    for (int c0 = 0; c0 < L; c0 += kAnchorChunk) {
        const int cn = min(kAnchorChunk, L - c0);
        __syncthreads();  // factor tables complete; the previous chunk's anchors consumed
        build_anchors<LOG2N>(buf, fac, shift, kb, rt, M, L, c0, cn, tid);
        __syncthreads();
        const int half = (cn + 1) >> 1;
        const int e0 = __builtin_amdgcn_readfirstlane(c0 + h * half);
        const int e1 = __builtin_amdgcn_readfirstlane(min(c0 + cn, e0 + half));
        if (e0 < e1) {
            // a whole number of kDepth-element steps; elements past the last one re-read it
            // and enter with a zero phase
            const int last = e1 - 1;
            const int steps = (e1 - e0 + kDepth - 1) / kDepth;
            ElemLoads q[kDepth];
#pragma unroll
            for (int u = 0; u < kDepth; ++u) {
                const int l = min(e0 + u, last);
                q[u].x = xp[(size_t)l * xstride];
                q[u].d = dp[(size_t)l * 16];
                q[u].a = buf[(l - c0) * 16 + R.orow];
                asm volatile("" ::: "memory");  // the prologue issues its loads in the loop's order
            }
            int e = e0;
            for (int it = 0; it < steps; ++it, e += kDepth) {
#pragma unroll
                for (int u = 0; u < kDepth; ++u) {
                    // operands of element e + u from the buffer ...
                    const ElemLoads& c = q[u];
                    const float2 an = e + u <= last ? c.a : make_float2(0.f, 0.f);
                    const auto sw =
                        __builtin_amdgcn_permlane32_swap(__float_as_uint(c.x.x), __float_as_uint(c.x.y), false, false);
                    const float2 w0 = cmul2(an, make_float2(c.d.x, c.d.y));
                    const float2 w1 = cmul2(w0, make_float2(c.d.z, c.d.w));
                    const float a0 = R.pick(w0), a1 = R.pick(w1);
                    // ... then the buffer takes the element kDepth ahead (into the same registers;
                    // the spectrum after the products that read its swapped copy)
                    const int ln = min(e + u + kDepth, last);
                    q[u].d = dp[(size_t)ln * 16];
                    q[u].a = buf[(ln - c0) * 16 + R.orow];
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, __uint_as_float(sw[0]), acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, __uint_as_float(sw[1]), acc1, 0, 0, 0);
                    q[u].x = xp[(size_t)ln * xstride];
                    // keeps each element's refill loads in its own step (the loads stay kDepth
                    // steps ahead of their use instead of being moved next to it)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    // the element halves: waves 4..7 hand their sums to waves 0..3 through LDS
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
    // results to LDS as runs [i][o][bin], then out as 64-byte runs, 8 threads per run
    float2* yst = buf;
    if (h == 0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int ol = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            yst[R.col * kYCol + ol * kBinBlock + 2 * p] = make_float2(acc0[v], acc0[v + 8]);
            yst[R.col * kYCol + ol * kBinBlock + 2 * p + 1] = make_float2(acc1[v], acc1[v + 8]);
        }
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
// anchors and phase steps.
struct SplitLoads {
    float4 x[4];
    float2 a[4];
    float4 d[4];
};

template <int LOG2N, bool F16>
__device__ __forceinline__ void contract_split_body(const float2* __restrict__ X, const int32_t* __restrict__ shift,
                                                    const float4* __restrict__ phd, float2* __restrict__ Y, int ntx,
                                                    int M, int L, int ncol, int kpad, float xscale, float yscale,
                                                    int kb, int rt, int ct) {
    constexpr int N = 1 << LOG2N;
    __shared__ float2 fac[64 + N / 64];
    __shared__ __attribute__((aligned(16))) float2 buf[kBufFloat2];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int p = wave & 3, h = wave >> 2;
    const int g = lane >> 5, col = lane & 31, orow = col & 15;
    const bool im_row = col >= 16;
    build_phase_factors<LOG2N>(fac, tid);

    floatx16 acc0, acc1;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.0f;

    const size_t xstride = (size_t)kBinBlock * ncol;  // complex floats between elements
    // padding columns read the last transmit's spectrum (results discarded)
    const float4* xp = reinterpret_cast<const float4*>(
        X + spec_index(kb * kBinBlock + 2 * p, 0, min(ct * 32 + col, ntx - 1), L, ncol));
    const float4* dp = phd + ((size_t)rt * 4 + p) * L * 16 + orow;

    for (int c0 = 0; c0 < L; c0 += kAnchorChunk) {
        const int cn = min(kAnchorChunk, L - c0);
        __syncthreads();
        build_anchors<LOG2N>(buf, fac, shift, kb, rt, M, L, c0, cn, tid);
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
                q.d[e] = dp[(size_t)l * 16];
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
                        const float2 w0 = cmul2(an, make_float2(c.d[k].x, c.d[k].y));
                        const float2 w1 = cmul2(w0, make_float2(c.d[k].z, c.d[k].w));
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
                                                                     const float4* __restrict__ phd,
                                                                     float2* __restrict__ Y, int ntx, int M,
                                                                     int L, int ncol, int kpad) {
    contract_body<LOG2N>(X, shift, phd, Y, ntx, M, L, ncol, kpad, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int LOG2N, bool F16>
__global__ __launch_bounds__(kContractThreads) void contract_split_kernel(
    const float2* __restrict__ X, const int32_t* __restrict__ shift, const float4* __restrict__ phd,
    float2* __restrict__ Y, int ntx, int M, int L, int ncol, int kpad, float xscale, float yscale) {
    contract_split_body<LOG2N, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, yscale, blockIdx.x, blockIdx.y,
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
    const float4* phd = reinterpret_cast<const float4*>(ws + e.d_off);
    if constexpr (PREC == 0)
        contract_body<LOG2N>(ws + e.x_off, plan + e.shift_off, phd, ws + e.y_off, e.ntx, e.M, e.L, e.ncol, e.kpad, kb,
                             rt, ct);
    else
        contract_split_body<LOG2N, PREC == 2>(ws + e.x_off, plan + e.shift_off, phd, ws + e.y_off, e.ntx, e.M, e.L,
                                              e.ncol, e.kpad, e.xscale, e.yscale, kb, rt, ct);
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
hipError_t contract_split(const float2* X, const int32_t* shift, const float4* phd, float2* Y, int ntx, int M, int L,
                          int ncol, int kpad, float xscale, hipStream_t st) {
    const dim3 grid((1 << LOG2N) / 2 / kBinBlock, (M + 15) / 16, ncol / 32);
    hipLaunchKernelGGL((contract_split_kernel<LOG2N, F16>), grid, dim3(kContractThreads), 0, st, X, shift, phd, Y,
                       ntx, M, L, ncol, kpad, xscale, 1.0f / xscale);
    return hipGetLastError();
}

template <int LOG2N>
hipError_t contract(const float2* X, const int32_t* shift, const float4* phd, float2* Y, int ntx, int M, int L,
                    int ncol, int kpad, hipStream_t st) {
    // bins 0 .. n/2 - 1; the Nyquist bin is summed by the inverse transform
    const dim3 grid((1 << LOG2N) / 2 / kBinBlock, (M + 15) / 16, ncol / 32);
    hipLaunchKernelGGL((contract_kernel<LOG2N>), grid, dim3(kContractThreads), 0, st, X, shift, phd, Y, ntx, M, L,
                       ncol, kpad);
    return hipGetLastError();
}

template <bool F16>
hipError_t launch_contract_split(int log2n, const float2* X, const int32_t* shift, const float4* phd, float2* Y, int ntx,
                                 int M, int L, int ncol, int kpad, float xscale, hipStream_t st) {
    switch (log2n) {
        case 8: return contract_split<8, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 9: return contract_split<9, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 10: return contract_split<10, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 11: return contract_split<11, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 12: return contract_split<12, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        case 13: return contract_split<13, F16>(X, shift, phd, Y, ntx, M, L, ncol, kpad, xscale, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_contract(int log2n, const float2* X, const int32_t* shift, const float4* phd, float2* Y, int ntx,
                           int M, int L, int ncol, int kpad, hipStream_t st) {
    switch (log2n) {
        case 8: return contract<8>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
        case 9: return contract<9>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
        case 10: return contract<10>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
        case 11: return contract<11>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
        case 12: return contract<12>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
        case 13: return contract<13>(X, shift, phd, Y, ntx, M, L, ncol, kpad, st);
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
    size_t x_off, d_off, y_off, total;
};

// workspace: spectra (contraction layout), phase steps, contracted spectra [N][M][kpad]
bool decompose_layout(const kk_geom* g, int32_t N, int32_t M, int32_t tpad, DecomposeLayout* d) {
    const int lg = log2_exact(tpad);
    if (lg < kMinLog2Fft || lg > kMaxLog2Fft || g->T < 1 || g->T > tpad || g->L < 1 || N < 1 || M < 1) return false;
    d->log2n = lg;
    d->K = tpad / 2 + 1;
    d->kpad = (d->K + kBinBlock - 1) / kBinBlock * kBinBlock;
    d->ncol = (N + 31) / 32 * 32;
    d->x_off = 0;
    d->d_off = d->x_off + align256((size_t)d->kpad * d->ncol * g->L * 8);
    d->y_off = d->d_off + align256(phase_step_floats4(M, g->L) * 16);
    d->total = d->y_off + align256((size_t)N * M * d->kpad * 8);
    return true;
}

// Forward transform (with the phase steps) and the per-bin contraction of one frame into Y.
hipError_t decompose_front(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q, int32_t M,
                           int32_t precision, const DecomposeLayout& d, unsigned char* w, float2* Y, hipStream_t st) {
    float2* X = reinterpret_cast<float2*>(w + d.x_off);
    float4* phd = reinterpret_cast<float4*>(w + d.d_off);
    const PhaseSteps ph{shift_q, M, phd};
    hipError_t e = launch_fft_forward(rf, N * g->L, g->T, d.log2n, X, true, g->L, d.ncol, d.kpad, st, &ph);
    if (e != hipSuccess) return e;
    if (precision == KK_PREC_FP32)
        return launch_contract(d.log2n, X, shift_q, phd, Y, N, M, g->L, d.ncol, d.kpad, st);
    if (precision == KK_PREC_BF16X3)
        return launch_contract_split<false>(d.log2n, X, shift_q, phd, Y, N, M, g->L, d.ncol, d.kpad, 1.0f, st);
    return launch_contract_split<true>(d.log2n, X, shift_q, phd, Y, N, M, g->L, d.ncol, d.kpad,
                                       std::ldexp(1.0f, fp16_prescale_exponent(g->T)), st);
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
    float2* Y = reinterpret_cast<float2*>(w + d.y_off);
    if (decompose_front(rf, N, g, shift_q, M, precision, d, w, Y, st) != hipSuccess) return KK_E_HIP;
    NyquistSum nyq{reinterpret_cast<const float2*>(w + d.x_off), shift_q, M, g->L, d.ncol};
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
