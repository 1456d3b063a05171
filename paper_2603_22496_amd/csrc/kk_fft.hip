// Power-of-two FFTs for gfx950 (FP32), used by the decomposition (Sec. II-F: analytic signal by
// a temporal FFT with negative frequencies zeroed, shear by the Fourier shift theorem) and by
// the DAS comparator.
//
// Stockham autosort in LDS with radix-16 passes (register-resident 16-point DFTs built from
// radix-2/4 stages with exact internal constants) and one radix-2/4/8 pass for the remainder,
// 256 threads per transform (512 at 8192 points).  Records enter LDS as 16-byte loads; every
// pass goes through one LDS round trip (the LDS array carries one pad slot per 16 points so
// the strided writes of a radix-16 pass spread over the banks).  A record at most half the
// transform long has a zero upper half, which the first pass skips; an inverse transform whose
// first half of outputs is kept computes only those in its last pass.  The twiddles of a
// butterfly, W^(r k) for r = 1 .. R-1, come from one base twiddle W^k by a power tree (W^r =
// W^(r/2) W^(r - r/2), at most four products deep); the base twiddle exp(-2 pi i m / n) is the
// product of two factors, exp(-2 pi i (m >> (log2n-6)) / 64) and exp(-2 pi i (m mod n/64) / n),
// each evaluated in FP64 by the workgroup into a small LDS table.
// Forward transforms take two real int16 records per workgroup as the real and imaginary parts
// of one complex sequence and unpack them straight into the two masked analytic spectra: for
// 0 < k < n/2, A[k] = Z[k] + conj(Z[n-k]) and
// B[k] = -i (Z[k] - conj(Z[n-k])) (the x2 of the analytic mask absorbs the 1/2 of the unpack);
// A[0] = Re Z[0], B[0] = Im Z[0], likewise at k = n/2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kk_internal.h"

namespace kk {
namespace {

// Threads per transform: 256, and 512 for the 8192-point transform, whose LDS footprint
// (~70 KB) leaves room for only two transforms per CU (so each takes more waves).
template <int LOG2N>
constexpr int fft_threads() { return fft_threads_for(LOG2N); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by exp(-i pi/2) = -i (forward) or exp(+i pi/2) = +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV>
struct Dft<4, INV> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
        const float2 s1 = cadd(v[1], v[3]), d1 = rot90<INV>(csub(v[1], v[3]));
        v[0] = cadd(s0, s1);
        v[2] = csub(s0, s1);
        v[1] = cadd(d0, d1);
        v[3] = csub(d0, d1);
    }
};

template <bool INV>
struct Dft<8, INV> {
    __device__ __forceinline__ static void run(float2* v) {
        constexpr float c = 0.70710678118654752440f;
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        float2 t[4];
        t[0] = o[0];
        t[1] = INV ? make_float2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                   : make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
        t[2] = rot90<INV>(o[2]);
        t[3] = INV ? make_float2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                   : make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], t[k]);
            v[k + 4] = csub(e[k], t[k]);
        }
    }
};

template <bool INV>
struct Dft<16, INV> {
    __device__ __forceinline__ static void run(float2* v) {
        // cos and sin of pi k / 8, k = 0..7
        constexpr float C[8] = {1.0f, 0.92387953251128675613f, 0.70710678118654752440f, 0.38268343236508977173f,
                                0.0f, -0.38268343236508977173f, -0.70710678118654752440f, -0.92387953251128675613f};
        constexpr float S[8] = {0.0f, 0.38268343236508977173f, 0.70710678118654752440f, 0.92387953251128675613f,
                                1.0f, 0.92387953251128675613f, 0.70710678118654752440f, 0.38268343236508977173f};
        float2 e[8], o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        Dft<8, INV>::run(e);
        Dft<8, INV>::run(o);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float2 t;
            if (k == 0) {
                t = o[0];
            } else if (k == 4) {
                t = rot90<INV>(o[4]);
            } else {
                t = cmul(o[k], make_float2(C[k], INV ? S[k] : -S[k]));
            }
            v[k] = cadd(e[k], t);
            v[k + 8] = csub(e[k], t);
        }
    }
};

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Padded LDS positions of a butterfly's R inputs (b + r NB) and outputs (out_index(b, r)) as a
// per-butterfly base plus a constant step in r (NB and NS are 1 or multiples of 16 and R
// divides 16, so the pad term splits exactly).
template <int N, int R>
__device__ __forceinline__ int read_base(int b) { return pad(b); }
template <int N, int R>
constexpr int read_step() { return (N / R) + (N / R) / 16; }
template <int N, int R, int NS>
__device__ __forceinline__ int write_base(int b) {
    if constexpr (NS == 1) return pad(b * R);
    else return pad((b / NS) * NS * R + (b % NS));
}
template <int N, int R, int NS>
constexpr int write_step() { return NS == 1 ? 1 : NS + NS / 16; }

// the two twiddle factor tables: fac[0..63] coarse, fac[64..64+n/64) fine
template <int LOG2N>
__device__ __forceinline__ void make_factors(float2* fac, int tid) {
    constexpr int N = 1 << LOG2N;
    if (tid < 64 + N / 64) {
        double sn, cs;
        sincospi(tid < 64 ? 2.0 * tid / 64.0 : 2.0 * (tid - 64) / (double)N, &sn, &cs);
        fac[tid] = make_float2((float)cs, (float)(-sn));
    }
}

template <int LOG2N>
__device__ __forceinline__ float2 twiddle_of(const float2* fac, int m) {
    constexpr int N = 1 << LOG2N;
    return cmul(fac[m >> (LOG2N - 6)], fac[64 + (m & (N / 64 - 1))]);
}

template <int LOG2N>
struct FftPlan {
    static constexpr int N = 1 << LOG2N;
    static constexpr int P16 = LOG2N / 4;
    static constexpr int REM = 1 << (LOG2N % 4);
    static constexpr int NPASS = P16 + (REM > 1 ? 1 : 0);
    static constexpr int radix(int p) { return p < P16 ? 16 : REM; }
    static constexpr int ns(int p) { return p == 0 ? 1 : ns(p - 1) * radix(p - 1); }
};

// twiddles of butterfly b in a pass with NS already-combined points: v[r] *= W_{NS R}^{r k},
// the powers W^r of the base twiddle by a product tree
template <int LOG2N, int R, int NS, bool INV>
__device__ __forceinline__ void twiddle(float2* v, int b, const float2* fac) {
    constexpr int N = 1 << LOG2N;
    if constexpr (NS > 1) {
        const int k = b % NS;
        constexpr int step = N / (NS * R);
        float2 w[R];
        w[1] = twiddle_of<LOG2N>(fac, k * step);
#pragma unroll
        for (int r = 2; r < R; ++r) w[r] = cmul(w[r / 2], w[r - r / 2]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
    }
}

template <int N, int R, int NS>
__device__ __forceinline__ int out_index(int b, int r) {
    const int k = b % NS;
    return (b / NS) * NS * R + k + r * NS;
}

// one Stockham pass LDS -> LDS (in place: all reads, barrier, all writes, barrier).  HALF: the
// first pass of a sequence whose upper half is zero (a record zero-padded to at least twice its
// length): inputs r >= R/2 of every butterfly (n = b + r N/R >= N/2) are known zeros.
template <int LOG2N, int R, int NS, bool INV, bool HALF = false>
__device__ __forceinline__ void pass_lds(float2* data, const float2* fac, int tid) {
    constexpr int N = 1 << LOG2N;
    constexpr int NB = N / R;
    constexpr int PER = (NB + fft_threads<LOG2N>() - 1) / fft_threads<LOG2N>();
    static_assert(!HALF || NS == 1, "zero upper half only on the first pass");
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * fft_threads<LOG2N>();
        if (b < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[p][r] = (HALF && 2 * r >= R) ? make_float2(0.f, 0.f) : data[read_base<N, R>(b) + r * read_step<N, R>()];
            twiddle<LOG2N, R, NS, INV>(v[p], b, fac);
            Dft<R, INV>::run(v[p]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * fft_threads<LOG2N>();
        if (b < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) data[write_base<N, R, NS>(b) + r * write_step<N, R, NS>()] = v[p][r];
        }
    }
    __syncthreads();
}

template <int LOG2N, int P, bool INV, bool HALF = false>
__device__ __forceinline__ void middle_passes(float2* data, const float2* fac, int tid) {
    using F = FftPlan<LOG2N>;
    if constexpr (P < F::NPASS - 1) {
        pass_lds<LOG2N, F::radix(P), F::ns(P), INV, HALF && P == 0>(data, fac, tid);
        middle_passes<LOG2N, P + 1, INV>(data, fac, tid);
    }
}

// exp(2 pi i ((k s) mod (n 2^22)) / (n 2^22)): the turn count reduced exactly in integers, the
// angle in FP64, rounded once to FP32.
template <int LOG2N>
__device__ __forceinline__ float2 exact_turn(int64_t k, int64_t s) {
    constexpr int64_t period = (int64_t)1 << (LOG2N + 22);
    int64_t r = (k * s) % period;
    if (r < 0) r += period;
    double sn, cs;
    sincospi((double)r / (double)(period >> 1), &sn, &cs);
    return make_float2((float)cs, (float)sn);
}

// The contraction's phase tables (extra workgroups of a blocked forward launch; the layouts
// are those of PhaseTables).  Work item e of table block b: a step entry (rt, l, o % 16) (D_1 ..
// D_7 of its angle and element: its D14 entry, and its four Cf operand lanes for p = 0..3), or
// four anchors W_{8 kb}[o][l] of consecutive angles.
template <int LOG2N>
__device__ __forceinline__ void phase_table_block(const int32_t* __restrict__ shift, int M, int L,
                                                  float4* __restrict__ cf, float4* __restrict__ d14,
                                                  float2* __restrict__ anc, int b) {
    constexpr int nkb = (1 << LOG2N) / 2 / kBinBlock;
    const int nrt = (M + 15) / 16;
    const int64_t e = (int64_t)b * fft_threads<LOG2N>() + threadIdx.x;
    const int64_t ncf = (int64_t)nrt * L * 16;
    if (e < ncf) {
        const int o16 = (int)(e & 15);
        const int64_t rl = e >> 4;
        const int l = (int)(rl % L), rt = (int)(rl / L);
        const int o = rt * 16 + o16;
        float2 d[8];
        if (o < M) {
            const int64_t s = shift[(size_t)o * L + l];
            d[0] = make_float2(1.f, 0.f);
#pragma unroll
            for (int j = 1; j < 8; ++j) d[j] = exact_turn<LOG2N>(j, s);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) d[j] = make_float2(0.f, 0.f);
        }
        d14[((size_t)rt * L + l) * 16 + o16] = make_float4(d[1].x, d[1].y, d[4].x, d[4].y);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const float2 u = d[2 * p], v = d[2 * p + 1];
            float4* row = cf + (((size_t)rt * 4 + p) * L + l) * 64;
            row[o16] = make_float4(u.x, -u.y, v.x, -v.y);        // Re row, Re part: Re W
            row[o16 + 16] = make_float4(u.y, u.x, v.y, v.x);     // Im row, Re part: Im W
            row[o16 + 32] = make_float4(-u.y, -u.x, -v.y, -v.x); // Re row, Im part: -Im W
            row[o16 + 48] = make_float4(u.x, -u.y, v.x, -v.y);   // Im row, Im part: Re W
        }
        return;
    }
    const int64_t a = e - ncf;
    if (a >= (int64_t)nkb * nrt * L * 4) return;
    const int quad = (int)(a & 3);
    int64_t r = a >> 2;
    const int l = (int)(r % L);
    r /= L;
    const int rt = (int)(r % nrt), kb = (int)(r / nrt);
    float2 w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = rt * 16 + quad * 4 + q;
        w[q] = o < M ? exact_turn<LOG2N>((int64_t)kb * kBinBlock, shift[(size_t)o * L + l]) : make_float2(0.f, 0.f);
    }
    float4* dst = reinterpret_cast<float4*>(anc + ((((size_t)kb * nrt + rt) * L + l) * 16 + quad * 4));
    dst[0] = make_float4(w[0].x, w[0].y, w[1].x, w[1].y);
    dst[1] = make_float4(w[2].x, w[2].y, w[3].x, w[3].y);
}

// One record pair per workgroup: the two real records are the real and imaginary parts of one
// complex FFT.  The records enter LDS as 16-byte loads (8 samples), zero-padded to n.
// Blocked (contraction) layout: the pair is transmits i, i+1 of element l and the spectra
// leave as whole 128-byte lines (8 bins of both records, four threads); trace layout:
// records 2 blk, 2 blk + 1, and 64-byte runs (8 bins) of each record.
// Body of block blk of one frame (shared by the per-frame and the grouped launches); blocked
// launches carry the phase-table blocks after the record pairs.
// Spectrum words of bins (k, k+1) = (v.x + i v.y, v.z + i v.w): FP32, or (split = BF16X3 or
// FP16X3) each bin times xscale split in 16-bit halves as (hi pair, lo pair).
__device__ __forceinline__ float4 spectrum_words(float4 v, int split, float xscale) {
    if (split == 0) return v;
    uint32_t h0, l0, h1, l1;
    if (split == 2) {
        split16_pair<true>(v.x * xscale, v.y * xscale, h0, l0);
        split16_pair<true>(v.z * xscale, v.w * xscale, h1, l1);
    } else {
        split16_pair<false>(v.x * xscale, v.y * xscale, h0, l0);
        split16_pair<false>(v.z * xscale, v.w * xscale, h1, l1);
    }
    return make_float4(__uint_as_float(h0), __uint_as_float(l0), __uint_as_float(h1), __uint_as_float(l1));
}

template <int LOG2N, bool BLOCKED>
__device__ __forceinline__ void fft_forward_body(const int16_t* __restrict__ rf, int ntraces, int T,
                                                 float2* __restrict__ out, int L, int ncol, int kpad, int blk,
                                                 const int32_t* __restrict__ shift, int M, float4* __restrict__ cf,
                                                 int split = 0, float xscale = 1.0f) {
    using F = FftPlan<LOG2N>;
    constexpr int N = F::N;
    __shared__ __attribute__((aligned(16))) float2 data[N + N / 16 + 1];  // + the mirror slot of bin 0
    __shared__ float2 fac[64 + N / 64];
    const int tid = threadIdx.x;
    int t0, t1, i0 = 0, l0 = 0;
    bool has1;
    if constexpr (BLOCKED) {
        const int ntx = ntraces / L;
        const int npairs = (ntx + 1) / 2;
        const int tb = cf ? (int)phase_table_blocks(M, L, LOG2N) : 0;
        if (blk < tb) {  // uniform per workgroup, before any barrier
            const PhaseTables pt{shift, M, cf};
            phase_table_block<LOG2N>(shift, M, L, cf, pt.d14(L), pt.anc(L), blk);
            return;
        }
        blk -= tb;
        if (blk >= L * npairs) return;
        l0 = blk % L;
        i0 = 2 * (blk / L);
        t0 = i0 * L + l0;
        t1 = t0 + L;
        has1 = i0 + 1 < ntx;
    } else {
        t0 = 2 * blk;
        t1 = t0 + 1;
        has1 = t1 < ntraces;
    }
    make_factors<LOG2N>(fac, tid);
    const int16_t* a = rf + (size_t)t0 * T;
    const int16_t* b = rf + (size_t)(has1 ? t1 : t0) * T;
    // records at most half the transform long: the first pass never reads the upper half
    const bool half = 2 * T <= N;
    if ((T & 7) == 0) {  // 8-sample groups: 16-byte aligned (records start at multiples of 16 B)
        for (int g = tid; g < (half ? N / 16 : N / 8); g += fft_threads<LOG2N>()) {
            const int n0 = g * 8;
            int16_t xa[8], xb[8];
            if (n0 < T) {
                *reinterpret_cast<uint4*>(xa) = *reinterpret_cast<const uint4*>(a + n0);
                *reinterpret_cast<uint4*>(xb) = *reinterpret_cast<const uint4*>(b + n0);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) xa[j] = xb[j] = 0;
            }
            float2* d = data + pad(n0);  // 8 consecutive entries, no pad slot inside
#pragma unroll
            for (int j = 0; j < 8; ++j) d[j] = make_float2((float)xa[j], has1 ? (float)xb[j] : 0.f);
        }
    } else {
        for (int n = tid; n < N; n += fft_threads<LOG2N>())
            data[pad(n)] = make_float2(n < T ? (float)a[n] : 0.f, (n < T && has1) ? (float)b[n] : 0.f);
    }
    __syncthreads();
    if (half)
        middle_passes<LOG2N, 0, false, true>(data, fac, tid);
    else
        middle_passes<LOG2N, 0, false>(data, fac, tid);
    pass_lds<LOG2N, F::radix(F::NPASS - 1), F::ns(F::NPASS - 1), false>(data, fac, tid);
    // unpack the two real spectra with the analytic mask, two bins per thread and record
    if constexpr (BLOCKED) {
        // bins 2kp, 2kp+1 < n/2 of transmits i0 and i0+1 (zeros for a missing partner): the four
        // threads of one bin block write one 128-byte line (64 bytes per record); bin 0 takes
        // Z[0] alone (the slot read as its mirror Z[n] is the spare one after the data)
        constexpr int TH = fft_threads<LOG2N>();
        constexpr int ITER = (N / 4 + TH - 1) / TH;
        float4* o = reinterpret_cast<float4*>(out + spec_index(2 * tid, l0, i0, L, ncol));
        const size_t ostep = (size_t)(TH / 4) * L * ncol * 4;  // float4s between iterations
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int k = 2 * (tid + it * TH);
            if ((N / 4) % TH != 0 && k >= N / 2) break;
            const float2 z0 = data[pad(k)], z1 = data[pad(k + 1)];
            const float2 m0 = data[pad(N - k)], m1 = data[pad(N - k - 1)];
            float4 A = make_float4(z0.x + m0.x, z0.y - m0.y, z1.x + m1.x, z1.y - m1.y);
            float4 B = make_float4(z0.y + m0.y, m0.x - z0.x, z1.y + m1.y, m1.x - z1.x);
            if (it == 0 && tid == 0) {
                A.x = z0.x;
                A.y = 0.f;
                B.x = z0.y;
                B.y = 0.f;
            }
            o[it * ostep] = spectrum_words(A, split, xscale);
            o[it * ostep + kBinBlock / 2] = spectrum_words(B, split, xscale);
        }
        if (tid == 0) {  // bin n/2 in FP32 (read by the inverse transform's Nyquist sum), then a zero bin
            const float2 z = data[pad(N / 2)];
            float4* q = reinterpret_cast<float4*>(out + spec_index(N / 2, l0, i0, L, ncol));
            q[0] = make_float4(z.x, 0.f, 0.f, 0.f);
            q[kBinBlock / 2] = make_float4(z.y, 0.f, 0.f, 0.f);
        }
        return;
    }
    for (int kp = tid; 2 * kp < kpad; kp += fft_threads<LOG2N>()) {
        float2 A[2], B[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * kp + h;
            A[h] = B[h] = make_float2(0.f, 0.f);
            if (k <= N / 2) {
                const float2 zk = data[pad(k)];
                const float2 zm = data[pad((N - k) & (N - 1))];
                if (k == 0 || k == N / 2) {
                    A[h] = make_float2(zk.x, 0.f);
                    B[h] = make_float2(zk.y, 0.f);
                } else {
                    A[h] = make_float2(zk.x + zm.x, zk.y - zm.y);
                    B[h] = make_float2(zk.y + zm.y, zm.x - zk.x);
                }
            }
        }
        // trace layout: four neighbouring threads complete one 64-byte run of 8 bins per record
        float2* o0 = out + (size_t)t0 * kpad;
        float2* o1 = out + (size_t)t1 * kpad;
        *reinterpret_cast<float4*>(o0 + 2 * kp) = make_float4(A[0].x, A[0].y, A[1].x, A[1].y);
        if (has1) *reinterpret_cast<float4*>(o1 + 2 * kp) = make_float4(B[0].x, B[0].y, B[1].x, B[1].y);
    }
}

// Last inverse pass straight to the output record, scaled by 1/N.  HALF: only the first N/2
// samples are kept, i.e. outputs r < R/2 of every butterfly (n = k + r N/R).
template <int LOG2N, bool HALF>
__device__ __forceinline__ void inverse_last_pass(const float2* data, const float2* fac, float2* __restrict__ o,
                                                  int T, int tid) {
    using F = FftPlan<LOG2N>;
    constexpr int N = F::N;
    {
        constexpr int P = F::NPASS - 1;
        constexpr int R = F::radix(P);
        constexpr int NS = F::ns(P);
        constexpr int NB = N / R;
        constexpr int PER = (NB + fft_threads<LOG2N>() - 1) / fft_threads<LOG2N>();
        constexpr float scale = 1.0f / (float)N;
        static_assert(NS * R == N, "last pass");
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int bb = tid + p * fft_threads<LOG2N>();
            if (bb < NB) {
                float2 v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = data[read_base<N, R>(bb) + r * read_step<N, R>()];
                twiddle<LOG2N, R, NS, true>(v, bb, fac);
                Dft<R, true>::run(v);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (HALF && 2 * r >= R) continue;
                    const int n = out_index<N, R, NS>(bb, r);
                    if (n < T) o[n] = make_float2(v[r].x * scale, v[r].y * scale);
                }
            }
        }
    }
}

// Body of record t of one frame.
template <int LOG2N, bool NYQ>
__device__ __forceinline__ void fft_inverse_body(const float2* __restrict__ in, int kpad, float2* __restrict__ out,
                                                 int T, const NyquistSum& nyq, int t) {
    using F = FftPlan<LOG2N>;
    constexpr int N = F::N;
    constexpr int K = N / 2 + 1;
    __shared__ float2 data[N + N / 16];
    __shared__ float2 fac[64 + N / 64];
    __shared__ float2 wsum[fft_threads<LOG2N>() / 64];
    const int tid = threadIdx.x;
    const float2* y = in + (size_t)t * kpad;
    // first pass inputs, the K non-negative bins (negative bins are zero), loaded first so that
    // the Nyquist sum's loads and the factor tables overlap them
    constexpr int R = F::radix(0);
    constexpr int NB = N / R;
    constexpr int PER = (NB + fft_threads<LOG2N>() - 1) / fft_threads<LOG2N>();
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int bb = tid + p * fft_threads<LOG2N>();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = bb + r * NB;
            v[p][r] = (bb < NB && 2 * r <= R && k < K && !(NYQ && k == N / 2)) ? y[k] : make_float2(0.f, 0.f);
        }
    }
    float2 part = make_float2(0.f, 0.f);
    if constexpr (NYQ) {
        // Eq. 3 at k = n/2: the advance s gives exp(i pi (s mod 2^23) / 2^22)
        const int i = t / nyq.M, o = t - (t / nyq.M) * nyq.M;
        for (int l = tid; l < nyq.L; l += fft_threads<LOG2N>()) {
            const uint32_t s = (uint32_t)nyq.shift[(size_t)o * nyq.L + l];
            const float2 x = nyq.X[spec_index(N / 2, l, i, nyq.L, nyq.ncol)];
            float sn, cs;
            sincospif((float)(s & 0x7FFFFFu) * (1.0f / 4194304.0f), &sn, &cs);
            part.x += cs * x.x - sn * x.y;
            part.y += cs * x.y + sn * x.x;
        }
    }
    make_factors<LOG2N>(fac, tid);
    if constexpr (NYQ) {
        // the sum over elements: within each wave by lane exchanges, then over the waves
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            part.x += __shfl_xor(part.x, m);
            part.y += __shfl_xor(part.y, m);
        }
        if ((tid & 63) == 0) wsum[tid >> 6] = part;
        __syncthreads();
        if (tid == 0) {  // bin n/2 enters butterfly 0 as its input R/2
            float2 ynyq = wsum[0];
#pragma unroll
            for (int w = 1; w < fft_threads<LOG2N>() / 64; ++w) ynyq = cadd(ynyq, wsum[w]);
            v[0][R / 2] = ynyq;
        }
    }
    {  // first pass
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int bb = tid + p * fft_threads<LOG2N>();
            if (bb < NB) {
                Dft<R, true>::run(v[p]);
#pragma unroll
                for (int r = 0; r < R; ++r) data[write_base<N, R, 1>(bb) + r * write_step<N, R, 1>()] = v[p][r];
            }
        }
        __syncthreads();
    }
    middle_passes<LOG2N, 1, true>(data, fac, tid);
    if (2 * T <= N)
        inverse_last_pass<LOG2N, true>(data, fac, out + (size_t)t * T, T, tid);
    else
        inverse_last_pass<LOG2N, false>(data, fac, out + (size_t)t * T, T, tid);
}


template <int LOG2N, bool BLOCKED>
__global__ __launch_bounds__(fft_threads<LOG2N>()) void fft_forward_kernel(const int16_t* __restrict__ rf, int ntraces,
                                                                  int T, float2* __restrict__ out, int L, int ncol,
                                                                  int kpad, const int32_t* __restrict__ shift, int M,
                                                                  float4* __restrict__ cf, int split, float xscale) {
    fft_forward_body<LOG2N, BLOCKED>(rf, ntraces, T, out, L, ncol, kpad, blockIdx.x, shift, M, cf, split, xscale);
}

template <int LOG2N, bool NYQ>
__global__ __launch_bounds__(fft_threads<LOG2N>()) void fft_inverse_kernel(const float2* __restrict__ in, int kpad,
                                                                  float2* __restrict__ out, int T,
                                                                  NyquistSum nyq) {
    fft_inverse_body<LOG2N, NYQ>(in, kpad, out, T, nyq, blockIdx.x);
}

// Grouped launches over the frames of one FFT-length class: block b runs record pair (or
// record) b - block0 of frame entry blk[b].
template <int LOG2N>
__global__ __launch_bounds__(fft_threads<LOG2N>()) void fft_forward_grouped(const FwdEntry* __restrict__ tab,
                                                                   const int32_t* __restrict__ blk,
                                                                   const int16_t* __restrict__ rf,
                                                                   float2* __restrict__ ws,
                                                                   const int32_t* __restrict__ plan) {
    const FwdEntry e = tab[blk[blockIdx.x]];
    fft_forward_body<LOG2N, true>(rf + e.rf_off, e.ntraces, e.T, ws + e.x_off, e.L, e.ncol, e.kpad,
                                  (int)blockIdx.x - e.block0, plan + e.shift_off, e.M,
                                  reinterpret_cast<float4*>(ws + e.d_off), e.split, e.xscale);
}

template <int LOG2N>
__global__ __launch_bounds__(fft_threads<LOG2N>()) void fft_inverse_grouped(const InvEntry* __restrict__ tab,
                                                                   const int32_t* __restrict__ blk,
                                                                   float2* __restrict__ ws,
                                                                   const int32_t* __restrict__ plan) {
    const InvEntry e = tab[blk[blockIdx.x]];
    const NyquistSum nyq{ws + e.x_off, plan + e.shift_off, e.M, e.L, e.ncol};
    fft_inverse_body<LOG2N, true>(ws + e.y_off, e.kpad, ws + e.out_off, e.T, nyq, (int)blockIdx.x - e.block0);
}

template <int LOG2N>
hipError_t fwd(const int16_t* rf, int ntraces, int T, float2* out, bool blocked, int L, int ncol, int kpad,
               hipStream_t st, const PhaseTables* ph, int split, float xscale) {
    if (blocked) {
        // one record pair (transmits i, i+1 of one element) per workgroup, then the phase tables
        const int64_t pairs = (int64_t)L * ((ntraces / L + 1) / 2);
        const int64_t pblocks = ph ? phase_table_blocks(ph->M, L, LOG2N) : 0;
        hipLaunchKernelGGL((fft_forward_kernel<LOG2N, true>), dim3((unsigned)(pairs + pblocks)), dim3(fft_threads<LOG2N>()), 0,
                           st, rf, ntraces, T, out, L, ncol, kpad, ph ? ph->shift : nullptr, ph ? ph->M : 0,
                           ph ? ph->cf : nullptr, split, xscale);
    } else {
        hipLaunchKernelGGL((fft_forward_kernel<LOG2N, false>), dim3((ntraces + 1) / 2), dim3(fft_threads<LOG2N>()), 0, st, rf,
                           ntraces, T, out, L, ncol, kpad, nullptr, 0, nullptr, 0, 1.0f);
    }
    return hipGetLastError();
}

template <int LOG2N>
hipError_t inv(const float2* in, int ntraces, int kpad, float2* out, int T, hipStream_t st, const NyquistSum* nyq) {
    if (nyq)
        hipLaunchKernelGGL((fft_inverse_kernel<LOG2N, true>), dim3(ntraces), dim3(fft_threads<LOG2N>()), 0, st, in, kpad, out,
                           T, *nyq);
    else
        hipLaunchKernelGGL((fft_inverse_kernel<LOG2N, false>), dim3(ntraces), dim3(fft_threads<LOG2N>()), 0, st, in, kpad,
                           out, T, NyquistSum{nullptr, nullptr, 1, 1, 32});
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fft_forward(const int16_t* rf, int ntraces, int T, int log2n, float2* out, bool blocked, int L,
                              int ncol, int kpad, hipStream_t st, const PhaseTables* ph, int split, float xscale) {
    if (split < 0 || split > 2 || (split != 0 && !blocked)) return hipErrorInvalidValue;
    switch (log2n) {
        case 8: return fwd<8>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        case 9: return fwd<9>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        case 10: return fwd<10>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        case 11: return fwd<11>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        case 12: return fwd<12>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        case 13: return fwd<13>(rf, ntraces, T, out, blocked, L, ncol, kpad, st, ph, split, xscale);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fft_forward_grouped(int log2n, const FwdEntry* tab, const int32_t* blk, int blocks,
                                      const int16_t* rf, float2* ws, const int32_t* plan, hipStream_t st) {
    const dim3 g(blocks);
    switch (log2n) {
        case 8: hipLaunchKernelGGL(fft_forward_grouped<8>, g, dim3(fft_threads<8>()), 0, st, tab, blk, rf, ws, plan); break;
        case 9: hipLaunchKernelGGL(fft_forward_grouped<9>, g, dim3(fft_threads<9>()), 0, st, tab, blk, rf, ws, plan); break;
        case 10: hipLaunchKernelGGL(fft_forward_grouped<10>, g, dim3(fft_threads<10>()), 0, st, tab, blk, rf, ws, plan); break;
        case 11: hipLaunchKernelGGL(fft_forward_grouped<11>, g, dim3(fft_threads<11>()), 0, st, tab, blk, rf, ws, plan); break;
        case 12: hipLaunchKernelGGL(fft_forward_grouped<12>, g, dim3(fft_threads<12>()), 0, st, tab, blk, rf, ws, plan); break;
        case 13: hipLaunchKernelGGL(fft_forward_grouped<13>, g, dim3(fft_threads<13>()), 0, st, tab, blk, rf, ws, plan); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_inverse_grouped(int log2n, const InvEntry* tab, const int32_t* blk, int blocks, float2* ws,
                                      const int32_t* plan, hipStream_t st) {
    const dim3 g(blocks);
    switch (log2n) {
        case 8: hipLaunchKernelGGL(fft_inverse_grouped<8>, g, dim3(fft_threads<8>()), 0, st, tab, blk, ws, plan); break;
        case 9: hipLaunchKernelGGL(fft_inverse_grouped<9>, g, dim3(fft_threads<9>()), 0, st, tab, blk, ws, plan); break;
        case 10: hipLaunchKernelGGL(fft_inverse_grouped<10>, g, dim3(fft_threads<10>()), 0, st, tab, blk, ws, plan); break;
        case 11: hipLaunchKernelGGL(fft_inverse_grouped<11>, g, dim3(fft_threads<11>()), 0, st, tab, blk, ws, plan); break;
        case 12: hipLaunchKernelGGL(fft_inverse_grouped<12>, g, dim3(fft_threads<12>()), 0, st, tab, blk, ws, plan); break;
        case 13: hipLaunchKernelGGL(fft_inverse_grouped<13>, g, dim3(fft_threads<13>()), 0, st, tab, blk, ws, plan); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_inverse(const float2* in, int ntraces, int kpad, int log2n, float2* out, int T,
                              hipStream_t st, const NyquistSum* nyq) {
    switch (log2n) {
        case 8: return inv<8>(in, ntraces, kpad, out, T, st, nyq);
        case 9: return inv<9>(in, ntraces, kpad, out, T, st, nyq);
        case 10: return inv<10>(in, ntraces, kpad, out, T, st, nyq);
        case 11: return inv<11>(in, ntraces, kpad, out, T, st, nyq);
        case 12: return inv<12>(in, ntraces, kpad, out, T, st, nyq);
        case 13: return inv<13>(in, ntraces, kpad, out, T, st, nyq);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace kk
