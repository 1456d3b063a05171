// Internal launch interface between the library's HIP translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kk {

// Bins per block of the spectrum layout used by the contraction (one contraction workgroup
// per block).  Bin k of the analytic spectrum of record (i, l) sits at
//   X[(((k / 8) L + l) ncol + i) 8 + k % 8]
// (complex float units, ncol = transmits padded to a multiple of 32): per block and element,
// one 64-byte run of 8 bins per transmit column.  The forward FFT transforms transmits i and
// i+1 of one element together, so its four threads of one block write one whole 128-byte
// line; an FP32 contraction wave reads whole runs.  For the split-precision contraction the
// same 8 bytes of a bin hold its value split in 16-bit halves (split16_pair): the hi pair
// (Re, Im) and the lo pair, each as one 32-bit word with Re in the low half.
constexpr int kBinBlock = 8;

// Raw buffer view of nbytes at p (gfx9 descriptor: 32-bit data format, no swizzle): loads take
// a per-lane and a wave-uniform byte offset with no vector address arithmetic; a load whose
// per-lane offset lies at or past nbytes returns zero (the wave-uniform offset is not part of
// that check, so callers keep it in range themselves).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
__device__ __forceinline__ uint32_t buffer_load1(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)lane_off, (int)off, 0);
}
__device__ __forceinline__ float2 buffer_load2(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane_off, (int)off, 0));
}
__device__ __forceinline__ float4 buffer_load4(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)lane_off, (int)off, 0));
}

// x = hi + lo with hi = round16(x), lo = round16(x - hi), round16 = BF16 or FP16 rounding to
// nearest even: the bits of (hi of a, hi of b) and (lo of a, lo of b), a in the low halves.
typedef float kk_float2v __attribute__((ext_vector_type(2)));
typedef __bf16 kk_bf16x2v __attribute__((ext_vector_type(2)));
typedef _Float16 kk_f16x2v __attribute__((ext_vector_type(2)));
// (a, b) rounded to 16 bits each (one packed conversion), a in the low half
template <bool F16>
__device__ __forceinline__ uint32_t round16_pair(float a, float b) {
    const kk_float2v v = {a, b};
    if constexpr (F16)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, kk_f16x2v));
    else
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, kk_bf16x2v));
}
template <bool F16>
__device__ __forceinline__ void split16_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
    hi = round16_pair<F16>(a, b);
    float ah, bh;
    if constexpr (F16) {
        const kk_f16x2v x = __builtin_bit_cast(kk_f16x2v, hi);
        ah = (float)x[0];
        bh = (float)x[1];
    } else {
        ah = __uint_as_float(hi << 16);
        bh = __uint_as_float(hi & 0xffff0000u);
    }
    lo = round16_pair<F16>(a - ah, b - bh);  // a - ah is exact
}

__host__ __device__ inline size_t spec_index(int k, int l, int i, int L, int ncol) {
    return (((size_t)(k >> 3) * L + l) * ncol + i) * 8 + (k & 7);
}

// Phase tables of the contraction, written by the extra workgroups of a blocked forward launch
// (nrt = receive tiles of 16 angles, nkb = n / 16 bin blocks; rows o >= M are zero), with
// D_j[o][l] = exp(2 pi i ((j shift[o][l]) mod (n 2^22)) / (n 2^22)) the phase step of j bins:
//   coefficients Cf[((rt 4 + p) L + l) 64 + lane] (float4), for lane = the lane of the
//     split-precision contraction's operand A: row r = lane % 32 (Re rows r < 16, Im rows
//     r >= 16, angle o = 16 rt + r % 16) and element part q = lane / 32; (x, y) for j = 2p and
//     (z, w) for j = 2p + 1 are chosen so that the operand is Re(a) x + Im(a) y for the bin
//     block's anchor a: (Re D_j, -Im D_j) for (Re row, Re part) and (Im row, Im part),
//     (Im D_j, Re D_j) for (Im row, Re part), (-Im D_j, -Re D_j) for (Re row, Im part);
//   steps D14[(rt L + l) 16 + o % 16] (float4) = (D_1, D_4)[o][l];
//   anchors Anc[((kb nrt + rt) L + l) 16 + o % 16] (float2) = W_{8 kb}[o][l], the Eq. 3 phase of
//     the first bin of block kb.
// The anchor times the step of the bin's offset in its block gives the bin's phase.
__host__ __device__ inline int contract_bin_blocks(int log2n) { return (1 << log2n) / 2 / kBinBlock; }
// FP32 contraction tiling: R8 tiles of 8 receive angles per workgroup (all M angles in one
// workgroup up to 32; beyond, 24 or 32 per workgroup, whichever pads fewer angles) and 16
// transmit columns per workgroup.
__host__ __device__ inline int contract_r8(int M) {
    if (M <= 32) return (M + 7) / 8;
    return 3 * ((M + 23) / 24) < 4 * ((M + 31) / 32) ? 3 : 4;
}
__host__ __device__ inline int contract_angle_tiles(int M) { return (M + 8 * contract_r8(M) - 1) / (8 * contract_r8(M)); }
constexpr int kContractCols = 16;
__host__ __device__ inline size_t phase_cf_floats4(int M, int L) {
    return (size_t)((M + 15) / 16) * 4 * (size_t)L * 64;
}
__host__ __device__ inline size_t phase_d14_floats4(int M, int L) { return (size_t)((M + 15) / 16) * (size_t)L * 16; }
__host__ __device__ inline size_t phase_anc_floats2(int M, int L, int log2n) {
    return (size_t)contract_bin_blocks(log2n) * ((M + 15) / 16) * (size_t)L * 16;
}
inline size_t phase_table_bytes(int M, int L, int log2n) {
    return (phase_cf_floats4(M, L) + phase_d14_floats4(M, L)) * 16 + phase_anc_floats2(M, L, log2n) * 8;
}

// Threads per workgroup of the FFT kernels for a transform of 2^log2n points.
__host__ __device__ constexpr int fft_threads_for(int log2n) { return log2n >= 13 ? 512 : 256; }
// Work items of the phase tables: one per (rt, l, o % 16) step entry (its Cf lanes for all p and
// its D14 entry), then one per four anchors (kb, rt, l, o % 16 / 4).
__host__ __device__ inline int64_t phase_table_items(int M, int L, int log2n) {
    const int64_t nrt = (M + 15) / 16;
    return nrt * L * 16 + (int64_t)contract_bin_blocks(log2n) * nrt * L * 4;
}
// Workgroups of a blocked forward launch that write the phase tables (before the record pairs).
__host__ __device__ inline int64_t phase_table_blocks(int M, int L, int log2n) {
    const int64_t t = fft_threads_for(log2n);
    return (phase_table_items(M, L, log2n) + t - 1) / t;
}

// Where a blocked forward launch writes the phase tables: Cf at base, then D14, then Anc.
struct PhaseTables {
    const int32_t* shift;  // [M][L] Q.22 advances
    int M;
    float4* cf;            // phase_cf_floats4(M, L) entries
    __host__ __device__ float4* d14(int L) const { return cf + phase_cf_floats4(M, L); }
    __host__ __device__ float2* anc(int L) const {
        return reinterpret_cast<float2*>(cf + phase_cf_floats4(M, L) + phase_d14_floats4(M, L));
    }
};

constexpr int kMinLog2Fft = 8;
constexpr int kMaxLog2Fft = 13;

inline int log2_exact(int64_t n) {
    if (n <= 0 || (n & (n - 1))) return -1;
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    return k;
}

// Analytic spectra of ntraces real int16 records of T samples, zero-padded to 2^log2n
// (mask: DC x1, 1..n/2-1 x2, n/2 x1).  Traces are transformed two per workgroup as the real
// and imaginary parts of one complex FFT.  Output bins k = 0..kpad-1 (zero above n/2):
//   blocked: out[spec_index(k, l, i, L, ncol)] for record t = i L + l (contraction layout;
//            records i and i+1 of element l share a workgroup, a missing partner record of
//            an odd transmit count is written as zeros; of the last block only bin n/2 is
//            written); the launch also writes the phase tables *ph of the contraction (extra
//            workgroups, ahead of the record pairs), when ph is given; split = KK_PREC_BF16X3
//            or KK_PREC_FP16X3 stores bins below n/2 times xscale split in 16-bit halves
//            (bin n/2 stays FP32)
//   else:    out[t * kpad + k]                                   (trace layout)
hipError_t launch_fft_forward(const int16_t* rf, int ntraces, int T, int log2n, float2* out, bool blocked, int L,
                              int ncol, int kpad, hipStream_t st, const PhaseTables* ph = nullptr, int split = 0,
                              float xscale = 1.0f);

// Where the Nyquist bin of record t = i * M + o is not stored but summed by the inverse
// transform itself: Y[n/2] = sum_l exp(i pi shift[o][l] / 2^22) X[i][l][n/2] (Eq. 3 at k = n/2),
// X in the contraction layout (spec_index).
struct NyquistSum {
    const float2* X;
    const int32_t* shift;
    int M, L, ncol;
};

// y[t][n] = (1/2^log2n) sum_{k <= n/2} in[t * kpad + k] exp(+2 pi i k n / 2^log2n), n < T.
hipError_t launch_fft_inverse(const float2* in, int ntraces, int kpad, int log2n, float2* out, int T,
                              hipStream_t st, const NyquistSum* nyq = nullptr);

// Delay-gather with a beamforming plan (KK or DAS): checks of the host copy of the plan, the
// size of the pair-share buffer it needs, and the launch (gather, then the fixed-order share
// reduction and the Eq. 8 / 9 intensity when the plan splits pairs or an intensity is asked).
bool gather_plan_ok(const int32_t* plan_host, size_t plan_bytes, bool das);
size_t gather_workspace_bytes(const int32_t* plan_host);
hipError_t run_gather(const float2* rec, const int32_t* plan_host, const int32_t* plan_dev, float2* image,
                      float* inten, int mode, void* ws, bool das, hipStream_t st);

// FP16 hi+lo contraction: inputs are scaled by 2^e, e from the record length.
int fp16_prescale_exponent(int T);

// ---------------------------------------------------------------------------------------
// Grouped launches of a frame ensemble.  Each launch covers the frames of one shape class;
// its work table (in the device copy of the ensemble plan) has one entry per frame, and a
// per-block table maps block b to its entry (the block then works on block b - block0 of
// that frame, exactly as the per-frame launch would).  Offsets count elements of the buffer
// named: the packed channel data (int16), the workspace (float2), the packed images (float2),
// the packed intensities (float) or the ensemble plan (int32 words).
struct FwdEntry {
    int64_t rf_off;          // channel data of the frame, [N][L][T]
    int64_t x_off;           // workspace: analytic spectra in the contraction layout
    int64_t d_off;           // workspace: phase tables of the contraction (float2 units)
    int32_t ntraces, T, L, ncol, kpad, block0;
    int32_t shift_off, M;    // plan: shift table [M][L]
    int32_t split;           // spectrum format: KK_PREC_* of the contraction
    float xscale;            // split-precision prescale of the spectrum
};
struct ContractEntry {
    int64_t x_off, y_off;    // workspace: spectra in, contracted spectra [N][M][kpad] out
    int64_t d_off;           // workspace: phase tables (float2 units)
    int32_t shift_off;       // plan: shift table [M][L]
    int32_t ntx, M, L, ncol, kpad, nkb, nrt, block0;
    float xscale, yscale;    // split-precision prescale and its inverse
    int32_t pad;
};
struct InvEntry {
    int64_t y_off, out_off, x_off;  // workspace: contracted spectra, RF_theta [N][M][T], spectra
    int32_t shift_off, kpad, T, M, L, ncol, block0, pad;
};
struct GatherEntry {
    int64_t rec_off;         // workspace: RF_theta of the frame
    int64_t out_off;         // images (split == 1) or workspace shares [K][S][X][Z] (split > 1)
    int32_t plan_off;        // plan: the frame's beamforming plan
    int32_t cap, split, n, m, t;
};
struct ReduceEntry {
    int64_t part_off;        // workspace shares (K > 1)
    int64_t img_off;         // images [S][X][Z]
    int64_t inten_off;       // intensities [X][Z], or -1
    int32_t K, S, npix, mode, block0, pad;
};
static_assert(sizeof(FwdEntry) == 64 && sizeof(ContractEntry) == 72 && sizeof(InvEntry) == 56 &&
                  sizeof(GatherEntry) == 40 && sizeof(ReduceEntry) == 48,
              "work table layout");

constexpr int kQueueLists = 8;  // gather work lists, one per XCD

hipError_t launch_fft_forward_grouped(int log2n, const FwdEntry* tab, const int32_t* blk, int blocks,
                                      const int16_t* rf, float2* ws, const int32_t* plan, hipStream_t st);
hipError_t launch_contract_grouped(int log2n, int precision, const ContractEntry* tab, const int32_t* blk,
                                   int blocks, float2* ws, const int32_t* plan, hipStream_t st);
hipError_t launch_fft_inverse_grouped(int log2n, const InvEntry* tab, const int32_t* blk, int blocks, float2* ws,
                                      const int32_t* plan, hipStream_t st);
// n int32 zeros (a kernel, so that it may be captured into a graph).
hipError_t launch_fill_zero(int32_t* p, int n, hipStream_t st);
// Persistent gather of window class cap over items (int2 {entry, unit}; list q =
// items[list_begin[q] .. list_begin[q+1])); counters[kQueueLists] must be zero at launch.
// wg_units (or NULL): [workgroups] units each workgroup took.
hipError_t launch_gather_queue(int cap, const GatherEntry* tab, const int2* items, const int32_t* list_begin,
                               int32_t* counters, int workgroups, const float2* rec, const int32_t* plan,
                               float2* image, float2* part, int32_t* wg_units, hipStream_t st);
hipError_t launch_reduce_grouped(const ReduceEntry* tab, const int32_t* blk, int blocks, const float2* part,
                                 float2* image, float* inten, hipStream_t st);

}  // namespace kk
