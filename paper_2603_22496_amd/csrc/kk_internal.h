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

}  // namespace kk
