// Delay-gather beamforming kernels for gfx950: KK (Eq. 5) per set, DAS (Eq. 4), and the
// Eq. 8 / Eq. 9 compounding epilogue.
//
// One workgroup = one 64 (lateral) x 16 (axial) pixel tile of one set (and one share of its
// pairs when the plan splits them), 16 wave64s: 4 pair groups x 4 axial quarters.  Lane k of
// a wave owns lateral pixel k of the tile and four consecutive axial pixels, so neighbouring
// lanes read neighbouring record samples (adjacent lateral pixels differ by at most ~1 sample
// of delay at lambda/2 pitch) and the LDS gather is broadcast- or stride-1.
//
// Pairs are processed in batches.  For every pair of a batch the workgroup stages into LDS the
// record window the tile touches, as 16-byte entries (R[n], (R[n+1]-R[n]) 2^-16) for
// n = lo .. lo+cap-1 (zero outside [0, T); lo is exact per pair and tile, from the plan), and
// the pair's 64 lateral delays A[p][x].  The axial delays B[p][z] of a wave's four rows are the
// same for all its lanes: they are fetched with scalar loads once per batch, right after the
// barrier, and the window start and LDS slot are folded into them on the scalar unit, so the
// integer part of A + B'' is directly the LDS entry of the sample.  Each pixel-pair then costs
// one integer add, one SDWA shift (entry -> byte address), one SDWA convert of the 16-bit
// fraction, one ds_read_b128 and two adds plus two FMAs:
//   acc += R[idx] + frac * (R[idx+1]-R[idx]) 2^-16 = (1 - w) R[idx] + w R[idx+1], w = frac/65536.
// The four pair groups are reduced through LDS at the end.  Batches are double-buffered: the
// global loads of batch b+1 are issued before batch b is gathered.  DAS adds a third delay term
// (receive table, per pixel and element) read once per batch into registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

constexpr int kWaves = 16;
constexpr int kThreads = kWaves * 64;
constexpr int kGroups = 4;       // pair groups per workgroup
constexpr int kRows = 4;         // axial pixels per lane

struct __attribute__((aligned(8))) F4a8 {
    float x, y, z, w;
};

// (q >> 16) << 4 in one VALU op: SDWA selects the upper 16 bits of q as the shift source.
__device__ __forceinline__ uint32_t entry_byte_offset(uint32_t q) {
    uint32_t a;
    asm("v_lshlrev_b32_sdwa %0, 4, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "=v"(a)
        : "v"(q));
    return a;
}

// Maps the launch index onto a work unit so that each of the 8 XCDs (workgroups are dealt to
// XCDs round-robin) receives a contiguous run of units: tiles are numbered depth-major, so an
// XCD's L2 holds only its depth band of every record.
__device__ __forceinline__ int xcd_remap(int id, int total) {
    const int xcd = id & 7, k = id >> 3;
    const int base = total >> 3, rem = total & 7;
    return xcd * base + (xcd < rem ? xcd : rem) + k;
}

template <int CAP, int PB, bool DAS>
struct Lds {
    static constexpr int kWinBytes = 2 * PB * CAP * 16;
    static constexpr int kABytes = 2 * PB * 64 * 4;
    static constexpr int kCBytes = DAS ? 2 * 2 * 1024 * 4 : 0;  // DAS: two elements per buffer
    static constexpr int kBytes = kWinBytes + kABytes + kCBytes;
    static_assert(kBytes <= 160 * 1024, "LDS budget");
    static_assert(kWinBytes / 16 < 65536, "entry index must fit 16 bits");
    static_assert(3 * 256 * kRows * 8 <= kBytes, "reduction scratch fits the buffers");
};

// Global loads of one batch, held in registers while the previous batch is gathered.
template <int CAP>
struct Prefetch {
    F4a8 v[2][CAP / 64];  // (R[n], R[n+1]) per row of 64 entries, up to two slots per wave
    int32_t a[2];
    int32_t c[2];         // DAS: receive delay of pixel (wave row, lane) for two elements
};

struct PlanView {
    int T, P, N, xpad, zpad, xt, zt, tile, off_rec, off_a, off_b, off_lo, off_c, off_tx;
};

template <int CAP, int PB, bool DAS>
__device__ __forceinline__ void load_batch(Prefetch<CAP>& pf, const float2* __restrict__ rec,
                                           const int32_t* __restrict__ plan, const PlanView& pv, int q0, int nb,
                                           int wave, int lane) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int j = wave + u * kWaves;
        if (j < nb) {
            const int q = q0 + j;
            const int lo = plan[pv.off_lo + pv.tile * pv.P + q];
            const float2* rp = rec + (size_t)plan[pv.off_rec + q] * pv.T;
#pragma unroll
            for (int r = 0; r < CAP / 64; ++r) {
                const int n = lo + r * 64 + lane;
                F4a8 v;
                if ((unsigned)n < (unsigned)(pv.T - 1)) {
                    v = *reinterpret_cast<const F4a8*>(rp + n);
                } else {
                    float2 a = ((unsigned)n < (unsigned)pv.T) ? rp[n] : make_float2(0.f, 0.f);
                    float2 b = ((unsigned)(n + 1) < (unsigned)pv.T) ? rp[n + 1] : make_float2(0.f, 0.f);
                    v.x = a.x;
                    v.y = a.y;
                    v.z = b.x;
                    v.w = b.y;
                }
                pf.v[u][r] = v;
            }
            const int row = DAS ? plan[pv.off_tx + q] : q;  // DAS: transmit delays are per transmit
            pf.a[u] = plan[pv.off_a + row * pv.xpad + pv.xt * 64 + lane];
        }
    }
    if constexpr (DAS) {
        // receive delays of the (at most two) elements of this batch, pixel (row = wave, lane)
        const int l0 = q0 / pv.N;
        const int nl = (q0 + nb - 1) / pv.N - l0 + 1;
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (u < nl)
                pf.c[u] = plan[pv.off_c + ((size_t)(l0 + u) * pv.zpad + pv.zt * 16 + wave) * pv.xpad + pv.xt * 64 +
                               lane];
    }
}

template <int CAP, int PB, bool DAS>
__device__ __forceinline__ void store_batch(const Prefetch<CAP>& pf, unsigned char* lds, int buf, int nb,
                                            const PlanView& pv, int q0, int wave, int lane) {
    using L = Lds<CAP, PB, DAS>;
    float4* win = reinterpret_cast<float4*>(lds);
    int32_t* aslot = reinterpret_cast<int32_t*>(lds + L::kWinBytes);
    const float scale = 1.0f / 65536.0f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int j = wave + u * kWaves;
        if (j < nb) {
            const int slot = buf * PB + j;
#pragma unroll
            for (int r = 0; r < CAP / 64; ++r) {
                const F4a8 v = pf.v[u][r];
                win[slot * CAP + r * 64 + lane] =
                    make_float4(v.x, v.y, (v.z - v.x) * scale, (v.w - v.y) * scale);
            }
            aslot[slot * 64 + lane] = pf.a[u];
        }
    }
    if constexpr (DAS) {
        int32_t* cslot = reinterpret_cast<int32_t*>(lds + L::kWinBytes + L::kABytes);
        const int l0 = q0 / pv.N;
        const int nl = (q0 + nb - 1) / pv.N - l0 + 1;
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (u < nl) cslot[((buf * 2 + u) * 16 + wave) * 64 + lane] = pf.c[u];
    }
}

// pairs of the next batch: at most PB, and for DAS at most two elements (l) per batch
template <int PB, bool DAS>
__device__ __forceinline__ int batch_size(int q, int p_end, int N) {
    int nb = min(PB, p_end - q);
    if (DAS) nb = min(nb, (q / N + 2) * N - q);
    return nb;
}

template <int CAP, int PB, bool DAS>
__global__ __launch_bounds__(kThreads) void gather_kernel(const float2* __restrict__ rec,
                                                          const int32_t* __restrict__ plan,
                                                          float2* __restrict__ out, int n_arg, int m_arg,
                                                          int t_arg) {
    using L = Lds<CAP, PB, DAS>;
    constexpr int kPerGroup = PB / kGroups;
    __shared__ __attribute__((aligned(16))) unsigned char lds[L::kBytes];
    // a device plan that does not describe this call is ignored (uniform early exit)
    if (plan[PW_MAGIC] != kPlanMagic || plan[PW_KIND] != (DAS ? kPlanKindDAS : kPlanKindKK) ||
        plan[PW_N] != n_arg || plan[PW_M] != m_arg || plan[PW_T] != t_arg || plan[PW_CAP] != CAP ||
        plan[PW_PB] != PB)
        return;
    PlanView pv;
    pv.T = plan[PW_T];
    pv.P = plan[PW_P];
    pv.N = plan[PW_N];
    const int S = plan[PW_S], X = plan[PW_X], Z = plan[PW_Z], K = plan[PW_SPLIT];
    const int nxt = plan[PW_NXT], nzt = plan[PW_NZT];
    pv.xpad = plan[PW_XPAD];
    pv.zpad = plan[PW_ZPAD];
    pv.off_rec = plan[PW_OFF_REC];
    pv.off_a = plan[PW_OFF_A];
    pv.off_b = plan[PW_OFF_B];
    pv.off_lo = plan[PW_OFF_LO];
    pv.off_c = plan[PW_OFF_C];
    pv.off_tx = plan[PW_OFF_TX];
    const int off_set = plan[PW_OFF_SET];
    const int ntiles = nxt * nzt;
    // work unit r = (set, pair share, tile)
    const int r = xcd_remap(blockIdx.x, ntiles * S * K);
    const int sh = r / ntiles;
    const int s = sh / K, h = sh - s * K;
    pv.tile = r - sh * ntiles;
    pv.zt = pv.tile / nxt;
    pv.xt = pv.tile - pv.zt * nxt;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int group = wave >> 2, quarter = wave & 3;
    const int set_begin = plan[off_set + s], set_end = plan[off_set + s + 1];
    const int share = (set_end - set_begin + K - 1) / K;
    const int p_begin = min(set_end, set_begin + h * share);
    const int p_end = min(set_end, p_begin + share);

    float2 acc[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) acc[k] = make_float2(0.f, 0.f);

    const float4* win = reinterpret_cast<const float4*>(lds);
    const int32_t* aslot = reinterpret_cast<const int32_t*>(lds + L::kWinBytes);
    const int32_t* cslot = reinterpret_cast<const int32_t*>(lds + L::kWinBytes + L::kABytes);

    Prefetch<CAP> pf;
    int q0 = p_begin;
    int nb = batch_size<PB, DAS>(q0, p_end, pv.N);
    if (nb > 0) {
        load_batch<CAP, PB, DAS>(pf, rec, plan, pv, q0, nb, wave, lane);
        store_batch<CAP, PB, DAS>(pf, lds, 0, nb, pv, q0, wave, lane);
    }
    __syncthreads();
    int buf = 0;
    while (nb > 0) {
        const int q1 = q0 + nb;
        const int nb1 = q1 < p_end ? batch_size<PB, DAS>(q1, p_end, pv.N) : 0;
        if (nb1 > 0) load_batch<CAP, PB, DAS>(pf, rec, plan, pv, q1, nb1, wave, lane);
        // this group's contiguous share of the batch
        const int j0 = group * kPerGroup;
        const int nj = min(kPerGroup, nb - j0);
        // scalar: axial delays of the wave's rows with the window start and LDS slot folded in
        uint32_t bs[kPerGroup][kRows];
#pragma unroll
        for (int jj = 0; jj < kPerGroup; ++jj) {
            if (jj < nj) {
                const int q = q0 + j0 + jj;
                const int row = DAS ? plan[pv.off_tx + q] : q;
                const int lo = plan[pv.off_lo + pv.tile * pv.P + q];
                const uint32_t fold = (uint32_t)((buf * PB + j0 + jj) * CAP - lo) << 16;
                const int32_t* b = plan + pv.off_b + row * pv.zpad + pv.zt * 16 + quarter * kRows;
#pragma unroll
                for (int k = 0; k < kRows; ++k) bs[jj][k] = (uint32_t)b[k] + fold;
            }
        }
        uint32_t cq[2][kRows] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
        int l_first = 0;
        if constexpr (DAS) {
            l_first = q0 / pv.N;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int k = 0; k < kRows; ++k)
                    cq[u][k] = (uint32_t)cslot[((buf * 2 + u) * 16 + quarter * kRows + k) * 64 + lane];
        }
#pragma unroll
        for (int jj = 0; jj < kPerGroup; ++jj) {
            if (jj < nj) {
                const int slot = buf * PB + j0 + jj;
                const uint32_t a = (uint32_t)aslot[slot * 64 + lane];
                uint32_t q[kRows];
                if constexpr (DAS) {
                    const int u = (q0 + j0 + jj) / pv.N - l_first;
#pragma unroll
                    for (int k = 0; k < kRows; ++k) q[k] = a + bs[jj][k] + (u ? cq[1][k] : cq[0][k]);
                } else {
#pragma unroll
                    for (int k = 0; k < kRows; ++k) q[k] = a + bs[jj][k];
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const float w = (float)(q[k] & 0xFFFFu);
                    const float4 e = *reinterpret_cast<const float4*>(reinterpret_cast<const unsigned char*>(win) +
                                                                      entry_byte_offset(q[k]));
                    acc[k].x += e.x;
                    acc[k].y += e.y;
                    acc[k].x = __builtin_fmaf(w, e.z, acc[k].x);
                    acc[k].y = __builtin_fmaf(w, e.w, acc[k].y);
                }
            }
        }
        if (nb1 > 0) store_batch<CAP, PB, DAS>(pf, lds, buf ^ 1, nb1, pv, q1, wave, lane);
        __syncthreads();
        buf ^= 1;
        q0 = q1;
        nb = nb1;
    }
    // reduce the four pair groups
    float2* red = reinterpret_cast<float2*>(lds);
    const int slotpix = (quarter * kRows) * 64 + lane;  // + k * 64
    if (group > 0) {
#pragma unroll
        for (int k = 0; k < kRows; ++k) red[(group - 1) * 1024 + slotpix + k * 64] = acc[k];
    }
    __syncthreads();
    if (group == 0) {
        const int x = pv.xt * 64 + lane;
        const int z0 = pv.zt * 16 + quarter * kRows;
        if (x < X) {
            // unsplit: the image [S][X][Z]; split: share h of it, [K][S][X][Z]
            float2* o = out + (((size_t)h * S + s) * X + x) * Z;
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                float2 v = acc[k];
#pragma unroll
                for (int g = 0; g < kGroups - 1; ++g) {
                    const float2 t = red[g * 1024 + slotpix + k * 64];
                    v.x += t.x;
                    v.y += t.y;
                }
                if (z0 + k < Z) o[z0 + k] = v;
            }
        }
    }
}

// Sum of the K pair shares of each set (fixed order), written as the per-set images, and the
// Eq. 8 / Eq. 9 intensity of the set images when requested.
__global__ void reduce_kernel(const float2* __restrict__ part, int K, int S, int npix, float2* __restrict__ image,
                              float* __restrict__ inten, int mode) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    float2 coh = make_float2(0.f, 0.f);
    float inc = 0.f;
    for (int s = 0; s < S; ++s) {
        float2 v = make_float2(0.f, 0.f);
        for (int h = 0; h < K; ++h) {
            const float2 t = part[((size_t)h * S + s) * npix + i];
            v.x += t.x;
            v.y += t.y;
        }
        if (image) image[(size_t)s * npix + i] = v;
        coh.x += v.x;
        coh.y += v.y;
        inc += v.x * v.x + v.y * v.y;
    }
    if (inten) inten[i] = (mode == KK_COMPOUND_COHERENT) ? coh.x * coh.x + coh.y * coh.y : inc;
}

template <int CAP, bool DAS>
hipError_t launch_gather(const float2* rec, const int32_t* plan_dev, float2* out, int blocks, int n, int m, int t,
                         hipStream_t st) {
    constexpr int PB = pairs_per_batch(CAP);
    hipLaunchKernelGGL((gather_kernel<CAP, PB, DAS>), dim3(blocks), dim3(kThreads), 0, st, rec, plan_dev, out, n, m,
                       t);
    return hipGetLastError();
}

template <bool DAS>
hipError_t dispatch_gather(const float2* rec, const int32_t* h, const int32_t* pd, float2* out, hipStream_t st) {
    const int64_t blocks = (int64_t)h[PW_NXT] * h[PW_NZT] * h[PW_S] * h[PW_SPLIT];
    if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int b = (int)blocks, n = h[PW_N], m = h[PW_M], t = h[PW_T];
    switch (h[PW_CAP]) {
        case 64: return launch_gather<64, DAS>(rec, pd, out, b, n, m, t, st);
        case 128: return launch_gather<128, DAS>(rec, pd, out, b, n, m, t, st);
        case 192: return launch_gather<192, DAS>(rec, pd, out, b, n, m, t, st);
        case 256: return launch_gather<256, DAS>(rec, pd, out, b, n, m, t, st);
        case 320: return launch_gather<320, DAS>(rec, pd, out, b, n, m, t, st);
        case 384: return launch_gather<384, DAS>(rec, pd, out, b, n, m, t, st);
        case 448: return launch_gather<448, DAS>(rec, pd, out, b, n, m, t, st);
        case 512: return launch_gather<512, DAS>(rec, pd, out, b, n, m, t, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t gather_workspace_bytes(const int32_t* h) {
    if (h[PW_SPLIT] <= 1) return 0;
    return (size_t)h[PW_SPLIT] * h[PW_S] * h[PW_X] * h[PW_Z] * 8;
}

bool gather_plan_ok(const int32_t* h, size_t plan_bytes, bool das) {
    return plan_bytes >= (size_t)PW_HEADER_WORDS * 4 && h[PW_MAGIC] == kPlanMagic &&
           h[PW_KIND] == (das ? kPlanKindDAS : kPlanKindKK) && (size_t)h[PW_TOTAL] * 4 <= plan_bytes &&
           h[PW_PB] == pairs_per_batch(h[PW_CAP]) && h[PW_SPLIT] >= 1 && h[PW_SPLIT] <= kMaxSplit;
}

// Gather into the images (unsplit) or into the share buffer followed by the reduction; the
// intensity is written when requested.
hipError_t run_gather(const float2* rec, const int32_t* h, const int32_t* pd, float2* image, float* inten,
                      int mode, void* ws, bool das, hipStream_t st) {
    const int K = h[PW_SPLIT], S = h[PW_S];
    const int64_t npix = (int64_t)h[PW_X] * h[PW_Z];
    float2* dst = K > 1 ? static_cast<float2*>(ws) : image;
    const hipError_t e = das ? dispatch_gather<true>(rec, h, pd, dst, st) : dispatch_gather<false>(rec, h, pd, dst, st);
    if (e != hipSuccess) return e;
    if (K > 1 || inten) {
        const int blocks = (int)((npix + 255) / 256);
        if (K > 1)
            hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, st, static_cast<const float2*>(ws), K, S,
                               (int)npix, image, inten, mode);
        else
            hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, st, image, 1, S, (int)npix,
                               static_cast<float2*>(nullptr), inten, mode);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace kk

extern "C" {

int32_t kk_compound(const float* image, int32_t S, int32_t X, int32_t Z, int32_t mode, float* intensity,
                    void* stream) {
    if (!image || !intensity) return KK_E_NULL;
    if (S < 1 || X < 1 || Z < 1 || (mode != KK_COMPOUND_COHERENT && mode != KK_COMPOUND_INCOHERENT))
        return KK_E_ARG;
    const int64_t npix = (int64_t)X * Z;
    if (npix > 0x7fffffff) return KK_E_ARG;
    const int blocks = (int)((npix + 255) / 256);
    hipLaunchKernelGGL(kk::reduce_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(image), 1, S, (int)npix, static_cast<float2*>(nullptr),
                       intensity, mode);
    return hipGetLastError() == hipSuccess ? KK_OK : KK_E_HIP;
}

size_t kk_beamform_workspace_bytes(const void* plan_host, size_t plan_bytes) {
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (!h || !kk::gather_plan_ok(h, plan_bytes, false)) return 0;
    return kk::gather_workspace_bytes(h);
}

int32_t kk_beamform(const float* rf_theta, int32_t N, int32_t M, int32_t T, const void* plan_host,
                    const void* plan_dev, size_t plan_bytes, float* image, float* intensity, int32_t mode, void* ws,
                    size_t ws_bytes, void* stream) {
    using namespace kk;
    if (!rf_theta || !plan_host || !plan_dev || !image) return KK_E_NULL;
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (!gather_plan_ok(h, plan_bytes, false)) return KK_E_WORKSPACE;
    if (h[PW_N] != N || h[PW_M] != M || h[PW_T] != T || N < 1 || M < 1 || T < 1) return KK_E_ARG;
    if (intensity && mode != KK_COMPOUND_COHERENT && mode != KK_COMPOUND_INCOHERENT) return KK_E_ARG;
    const size_t need = gather_workspace_bytes(h);
    if (need > 0 && (!ws || ws_bytes < need)) return KK_E_WORKSPACE;
    const hipError_t e = run_gather(reinterpret_cast<const float2*>(rf_theta), h, static_cast<const int32_t*>(plan_dev),
                                    reinterpret_cast<float2*>(image), intensity, mode, ws, false,
                                    (hipStream_t)stream);
    return e == hipSuccess ? KK_OK : KK_E_HIP;
}

}  // extern "C"
