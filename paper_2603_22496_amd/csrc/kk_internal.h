// Internal launch interface between the library's HIP translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kk {

// Bins per block of the spectrum layout used by the contraction: the analytic spectrum of
// trace (i, l) is stored as X[k / 8][i][l][k % 8] so that one 64-byte run holds 8 bins.
constexpr int kBinBlock = 8;

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
// and imaginary parts of one complex FFT.  Output bins k = 0..n/2:
//   blocked: out[((k / 8) * ncol + t / L) * L + t % L][k % 8]   (contraction layout)
//   else:    out[t * kpad + k]                                   (trace layout)
hipError_t launch_fft_forward(const int16_t* rf, int ntraces, int T, int log2n, float2* out, bool blocked, int L,
                              int ncol, int kpad, hipStream_t st);

// Where the Nyquist bin of record t = i * M + o is not stored but summed by the inverse
// transform itself: Y[n/2] = sum_l exp(i pi shift[o][l] / 2^22) X[i][l][n/2] (Eq. 3 at k = n/2),
// X in the bin-blocked layout.
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
    int64_t x_off;           // workspace: bin-blocked analytic spectra
    int32_t ntraces, T, L, ncol, kpad, block0;
};
struct ContractEntry {
    int64_t x_off, y_off;    // workspace: spectra in, contracted spectra [N][M][kpad] out
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
static_assert(sizeof(FwdEntry) == 40 && sizeof(ContractEntry) == 64 && sizeof(InvEntry) == 56 &&
                  sizeof(GatherEntry) == 40 && sizeof(ReduceEntry) == 48,
              "work table layout");

constexpr int kQueueLists = 8;  // gather work lists, one per XCD

hipError_t launch_fft_forward_grouped(int log2n, const FwdEntry* tab, const int32_t* blk, int blocks,
                                      const int16_t* rf, float2* ws, hipStream_t st);
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
