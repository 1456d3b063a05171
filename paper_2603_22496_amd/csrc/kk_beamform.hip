// Delay-gather beamforming kernels for gfx950: KK (Eq. 5) per set, DAS (Eq. 4), and the
// Eq. 8 / Eq. 9 compounding epilogue.
//
// One workgroup = one 64 (lateral) x 16 (axial) pixel tile of one set (and one share of its
// pairs when the plan splits them), 16 wave64s.  Each wave takes a contiguous run of the
// share's pairs and forms the whole tile for them: lane k owns lateral pixel k and all 16
// rows, so neighbouring lanes read neighbouring record samples (adjacent lateral pixels
// differ by at most ~1 sample of delay at lambda/2 pitch) and the LDS gather is broadcast- or
// stride-1.  The 16 partial tiles are summed in LDS at the end, in wave order.
//
// A wave owns one LDS window slot.  For its current pair the slot holds the record window
// the tile touches, as 16-byte entries (R[n], (R[n+1]-R[n]) 2^-16) for n = lo .. lo+cap-1
// (zero outside [0, T); lo is exact per pair and tile, from the plan).  While the wave gathers
// pair p it has the window and delays of pair p+1 in flight from global memory into
// registers; it stores that window over its slot after the gather (a wave's LDS operations
// execute in order), so the pair loop has no workgroup barrier at all.  The delays live in
// registers: the lateral delay A[p][x] at the lane's pixel, and the 16 axial delays B[p][z]
// of the tile's rows, with the window start and slot folded in, one per lane of a DPP row.
// The integer part of A + B'' is then directly the LDS entry of the sample, and each
// pixel-pair costs one DPP broadcast add, one SDWA shift (entry -> byte address), one SDWA
// convert of the 16-bit fraction, one ds_read_b128 and two adds plus two FMAs:
//   acc += R[idx] + frac * (R[idx+1]-R[idx]) 2^-16 = (1 - w) R[idx] + w R[idx+1], w = frac/65536.
// DAS adds a third delay term, the receive delay of the pair's element at each pixel, held in
// 16 registers and refetched when the wave's pair run moves to the next element.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

constexpr int kWaves = 16;
constexpr int kThreads = kWaves * 64;
constexpr int kRows = kTileZ;    // axial pixels per lane: the tile's rows
constexpr int kMetaLanes = 64;   // pairs whose slot metadata a wave holds at once

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

// x + bv[lane V of this lane's row of 16 lanes]: one v_add_u32_dpp row_newbcast.
template <int V>
__device__ __forceinline__ uint32_t add_row_broadcast(uint32_t bv, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)bv, 0x150 + V, 0xf, 0xf, true) + x;
}

// Maps the launch index onto a work unit so that each of the 8 XCDs (workgroups are dealt to
// XCDs round-robin) receives a contiguous run of units: tiles are numbered depth-major, so an
// XCD's L2 holds only its depth band of every record.
__device__ __forceinline__ int xcd_remap(int id, int total) {
    const int xcd = id & 7, k = id >> 3;
    const int base = total >> 3, rem = total & 7;
    return xcd * base + (xcd < rem ? xcd : rem) + k;
}

template <int CAP>
struct Lds {
    static constexpr int kWinBytes = kWaves * CAP * 16;
    static constexpr int kRedBytes = kWaves * kRows * 64 * 8;  // partial tiles of all waves
    static constexpr int kBytes = kWinBytes > kRedBytes ? kWinBytes : kRedBytes;
    static_assert(kBytes <= 160 * 1024, "LDS budget");
    static_assert(kWaves * CAP < 65536, "entry index must fit 16 bits");
};

// Window entries of one pair, held in registers from their global load to their LDS store.
template <int CAP>
struct Window {
    F4a8 v[CAP / 64];
};

// Delays of one pair for one wave.
struct PairDelays {
    uint32_t a;     // lateral delay at pixel `lane`
    uint32_t b;     // axial delay of row (lane & 15); window start and slot folded in once loaded
    uint32_t fold;  // (slot start - window start) << 16 (uniform)
};

struct PlanView {
    int T, P, N, xpad, zpad, xt, zt, tile, off_rec, off_a, off_b, off_lo, off_c;
};

template <bool DAS>
__device__ __forceinline__ int delay_row(int q, int N) {
    return DAS ? q % N : q;  // DAS pairs run element-major: p = l N + i, rows are transmits
}

// Window start and record of pairs q0 .. q0+63 (lane j holding pair q0 + j, clamped to qend-1).
struct SlotMeta {
    int32_t lo;
    int32_t rec;
};

__device__ __forceinline__ void load_meta(SlotMeta& m, const int32_t* __restrict__ plan, const PlanView& pv, int q0,
                                          int qend, int lane) {
    const int q = min(q0 + lane, qend - 1);
    m.lo = plan[pv.off_lo + pv.tile * pv.P + q];
    m.rec = plan[pv.off_rec + q];
}

// Issues the global loads of pair q (window entries and delays); j = q - (first pair of the
// metadata run) selects the pair's metadata lane.  A window inside its record is read through a
// buffer view of the record at the window start (a wave-uniform offset, no vector address
// arithmetic); a window over a record edge reads zeros outside the record, sample by sample.
// The delays come through the plan's view at wave-uniform offsets (in range by the plan).
template <int CAP, bool DAS>
__device__ __forceinline__ void load_pair(Window<CAP>& wn, PairDelays& d, const SlotMeta& m, int j,
                                          const float2* __restrict__ rec, __amdgpu_buffer_rsrc_t pview,
                                          const PlanView& pv, int q, int slot0, int lane) {
    const unsigned ulane = (unsigned)lane;
    const int lo = __builtin_amdgcn_readlane(m.lo, j);
    const int ri = __builtin_amdgcn_readlane(m.rec, j);
    const float2* rp = rec + (size_t)ri * pv.T;
    if (lo >= 0 && lo + CAP <= pv.T - 1) {
        // the whole window and its right neighbours lie inside the record
        const __amdgpu_buffer_rsrc_t rv = buffer_view(rp, (uint32_t)pv.T * sizeof(float2));
#pragma unroll
        for (int r = 0; r < CAP / 64; ++r) {
            const float4 v = buffer_load4(rv, (ulane + r * 64) * sizeof(float2), (uint32_t)lo * sizeof(float2));
            wn.v[r] = F4a8{v.x, v.y, v.z, v.w};
        }
    } else {
#pragma unroll
        for (int r = 0; r < CAP / 64; ++r) {
            const int n = lo + r * 64 + lane;
            const float2 a = ((unsigned)n < (unsigned)pv.T) ? rp[n] : make_float2(0.f, 0.f);
            const float2 b = ((unsigned)(n + 1) < (unsigned)pv.T) ? rp[n + 1] : make_float2(0.f, 0.f);
            wn.v[r] = F4a8{a.x, a.y, b.x, b.y};
        }
    }
    const int row = delay_row<DAS>(q, pv.N);
    // (the offsets are uniform; readfirstlane lets the loads take them as scalars)
    const uint32_t oa = (uint32_t)__builtin_amdgcn_readfirstlane((pv.off_a + pv.xt * 64 + row * pv.xpad) * 4);
    const uint32_t ob = (uint32_t)__builtin_amdgcn_readfirstlane((pv.off_b + pv.zt * kRows + row * pv.zpad) * 4);
    d.a = buffer_load1(pview, ulane * 4, oa);
    d.b = buffer_load1(pview, (ulane & 15) * 4, ob);
    d.fold = (uint32_t)(slot0 - lo) << 16;
}

// Folds the window start and the wave's slot into the axial delays once their loads have
// landed (called after the gather of the previous pair, so the loads stay in flight during it).
__device__ __forceinline__ void fold_delays(PairDelays& d) { d.b += d.fold; }

template <int CAP>
__device__ __forceinline__ void store_window(const Window<CAP>& wn, float4* slot, int lane) {
    const float scale = 1.0f / 65536.0f;
#pragma unroll
    for (int r = 0; r < CAP / 64; ++r) {
        const F4a8 v = wn.v[r];
        slot[r * 64 + lane] = make_float4(v.x, v.y, (v.z - v.x) * scale, (v.w - v.y) * scale);
    }
}

// Rows in flight per pipeline step: four for KK; two for DAS, whose 16 receive delays take
// the registers of the other two.
template <bool DAS>
struct Step {
    static constexpr int kRowsPerStep = DAS ? 2 : 4;
};

// One step's samples in flight: their LDS entries and lerp weights.
template <bool DAS>
struct RowSamples {
    float4 e[Step<DAS>::kRowsPerStep];
    float w[Step<DAS>::kRowsPerStep];
};

template <int K, bool DAS>
__device__ __forceinline__ uint32_t row_delay(const PairDelays& d, const uint32_t* c) {
    return add_row_broadcast<K>(d.b, DAS ? d.a + c[K] : d.a);
}

template <int K0, bool DAS>
__device__ __forceinline__ void issue_rows(RowSamples<DAS>& rs, const PairDelays& d, const uint32_t* c,
                                           const unsigned char* win) {
    constexpr int kS = Step<DAS>::kRowsPerStep;
    uint32_t q[kS];
    q[0] = row_delay<K0 + 0, DAS>(d, c);
    q[1] = row_delay<K0 + 1, DAS>(d, c);
    if constexpr (kS == 4) {
        q[2] = row_delay<K0 + 2, DAS>(d, c);
        q[3] = row_delay<K0 + 3, DAS>(d, c);
    }
#pragma unroll
    for (int k = 0; k < kS; ++k) {
        rs.w[k] = (float)(q[k] & 0xFFFFu);
        rs.e[k] = *reinterpret_cast<const float4*>(win + entry_byte_offset(q[k]));
    }
}

template <int K0, bool DAS>
__device__ __forceinline__ void accumulate_rows(float2 (&acc)[kRows], const RowSamples<DAS>& rs) {
#pragma unroll
    for (int k = 0; k < Step<DAS>::kRowsPerStep; ++k) {
        float2& a = acc[K0 + k];
        a.x += rs.e[k].x;
        a.y += rs.e[k].y;
        a.x = __builtin_fmaf(rs.w[k], rs.e[k].z, a.x);
        a.y = __builtin_fmaf(rs.w[k], rs.e[k].w, a.y);
        // pins these rows' arithmetic here, ahead of the next scheduling fence
        asm volatile("" : "+v"(a.x), "+v"(a.y));
    }
}

// Software pipeline over the tile's rows: while a step's samples are accumulated, the reads
// of the next DEPTH-1 steps are in flight; a scheduling fence closes each step so that at most
// DEPTH steps' samples are live.
template <int K0, bool DAS, int DEPTH>
__device__ __forceinline__ void gather_rows(float2 (&acc)[kRows], const PairDelays& d, const uint32_t* c,
                                            RowSamples<DAS>& s0, RowSamples<DAS>& s1, const unsigned char* win) {
    constexpr int kS = Step<DAS>::kRowsPerStep;
    if constexpr (K0 < kRows) {
        RowSamples<DAS> s2;
        constexpr int kAhead = K0 + (DEPTH - 1) * kS;
        if constexpr (kAhead < kRows) issue_rows<kAhead, DAS>(s2, d, c, win);
        accumulate_rows<K0, DAS>(acc, s0);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DEPTH == 3)
            gather_rows<K0 + kS, DAS, DEPTH>(acc, d, c, s1, s2, win);
        else
            gather_rows<K0 + kS, DAS, DEPTH>(acc, d, c, s2, s2, win);
    }
}

// DEPTH 3 where the registers allow it: KK with windows up to 320 entries held in flight.
template <bool DAS, int DEPTH>
__device__ __forceinline__ void gather_pair(float2 (&acc)[kRows], const PairDelays& d, const uint32_t* c,
                                            const unsigned char* win) {
    constexpr int kS = Step<DAS>::kRowsPerStep;
    RowSamples<DAS> s0, s1;
    issue_rows<0, DAS>(s0, d, c, win);
    if constexpr (DEPTH == 3) issue_rows<kS, DAS>(s1, d, c, win);
    gather_rows<0, DAS, DEPTH>(acc, d, c, s0, s1, win);
}

// One work unit (set, pair share, tile) of one plan; unit < 0 takes blockIdx.x through the
// XCD-contiguous remap.  lds: at least Lds<CAP>::kBytes.
template <int CAP, bool DAS>
__device__ __forceinline__ void gather_body(const float2* __restrict__ rec, const int32_t* __restrict__ plan,
                                            float2* __restrict__ out, int n_arg, int m_arg, int t_arg, int unit,
                                            unsigned char* lds) {
    // a device plan that does not describe this call is ignored (uniform early exit)
    if (plan[PW_MAGIC] != kPlanMagic || plan[PW_KIND] != (DAS ? kPlanKindDAS : kPlanKindKK) ||
        plan[PW_N] != n_arg || plan[PW_M] != m_arg || plan[PW_T] != t_arg || plan[PW_CAP] != CAP ||
        plan[PW_PB] != kWaves)
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
    const int off_set = plan[PW_OFF_SET];
    const int ntiles = nxt * nzt;
    // work unit r = (set, pair share, tile)
    const int r = unit >= 0 ? unit : xcd_remap(blockIdx.x, ntiles * S * K);
    const int sh = r / ntiles;
    const int s = sh / K, h = sh - s * K;
    pv.tile = r - sh * ntiles;
    pv.zt = pv.tile / nxt;
    pv.xt = pv.tile - pv.zt * nxt;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int set_begin = plan[off_set + s], set_end = plan[off_set + s + 1];
    const int share = (set_end - set_begin + K - 1) / K;
    const int p_begin = min(set_end, set_begin + h * share);
    const int p_end = min(set_end, p_begin + share);
    // this wave's run of pairs
    const int run = (p_end - p_begin + kWaves - 1) / kWaves;
    const int w_begin = min(p_end, p_begin + wave * run);
    const int w_end = min(p_end, w_begin + run);

    float2 acc[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) acc[k] = make_float2(0.f, 0.f);

    float4* slot = reinterpret_cast<float4*>(lds) + wave * CAP;
    // the plan's words through a buffer view (every offset taken through it is in range)
    const __amdgpu_buffer_rsrc_t pview = buffer_view(plan, 0x7FFFFFFCu);
    if (w_begin < w_end) {
        Window<CAP> wn;
        PairDelays cur, nxt_d;
        SlotMeta meta;
        uint32_t c[DAS ? kRows : 1];
        int c_elem = -1;
        int m_base = w_begin;
        load_meta(meta, plan, pv, m_base, w_end, lane);
        load_pair<CAP, DAS>(wn, cur, meta, 0, rec, pview, pv, w_begin, wave * CAP, lane);
        fold_delays(cur);
        store_window<CAP>(wn, slot, lane);
        // the first pair's delays are complete before the loop, so the loop's only loads in
        // flight during a gather are the next pair's
        asm volatile("" ::"v"(cur.a), "v"(cur.b));
        // pair q gathers with the delays in `use` while pair q + 1's loads land in `next`; the
        // loop runs two pairs per pass with the two delay sets swapping roles (no copies)
        auto step = [&](int q, const PairDelays& use, PairDelays& next) {
            const bool more = q + 1 < w_end;
            if (more) {
                if (q + 1 - m_base == kMetaLanes) {
                    m_base = q + 1;
                    load_meta(meta, plan, pv, m_base, w_end, lane);
                }
                load_pair<CAP, DAS>(wn, next, meta, q + 1 - m_base, rec, pview, pv, q + 1, wave * CAP, lane);
            }
            if constexpr (DAS) {
                const int l = q / pv.N;
                if (l != c_elem) {
                    // receive delays of element l at (lane, rows): C is [L][ZPAD][XPAD]
                    c_elem = l;
                    const int32_t* crow =
                        plan + pv.off_c + ((size_t)l * pv.zpad + pv.zt * kRows) * pv.xpad + pv.xt * 64;
#pragma unroll
                    for (int k = 0; k < kRows; ++k) c[k] = (uint32_t)crow[(unsigned)(k * pv.xpad) + (unsigned)lane];
                }
            }
            gather_pair<DAS, (!DAS && CAP <= 320) ? 3 : 2>(acc, use, c, reinterpret_cast<const unsigned char*>(lds));
            if (more) {
                fold_delays(next);
                // the gather's reads of the slot precede these stores in the wave's LDS order
                __builtin_amdgcn_sched_barrier(0);
                store_window<CAP>(wn, slot, lane);
            }
        };
        for (int q = w_begin; q < w_end; q += 2) {
            step(q, cur, nxt_d);
            if (q + 1 < w_end) step(q + 1, nxt_d, cur);
        }
    }
    // sum the waves' partial tiles in wave order
    __syncthreads();
    float2* red = reinterpret_cast<float2*>(lds);
#pragma unroll
    for (int k = 0; k < kRows; ++k) red[(wave * kRows + k) * 64 + lane] = acc[k];
    __syncthreads();
    const int row = threadIdx.x >> 6;  // pixel (row, lane) of the tile
    float2 v = red[row * 64 + lane];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
        const float2 t = red[(w * kRows + row) * 64 + lane];
        v.x += t.x;
        v.y += t.y;
    }
    const int x = pv.xt * 64 + lane, z = pv.zt * kRows + row;
    // unsplit: the image [S][X][Z]; split: share h of it, [K][S][X][Z]
    if (x < X && z < Z) out[(((size_t)h * S + s) * X + x) * Z + z] = v;
}

template <int CAP, bool DAS>
__global__ __launch_bounds__(kThreads) void gather_kernel(const float2* __restrict__ rec,
                                                          const int32_t* __restrict__ plan,
                                                          float2* __restrict__ out, int n_arg, int m_arg,
                                                          int t_arg) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[Lds<CAP>::kBytes];
    gather_body<CAP, DAS>(rec, plan, out, n_arg, m_arg, t_arg, -1, lds);
}

// Persistent gather over the work units of one window class of a frame ensemble.  The units
// sit in kQueueLists lists; workgroup b starts on list b mod kQueueLists (the XCD the hardware
// places it on when workgroups are dealt to the XCDs in turn) and takes units from its front
// with an atomic counter; once that list is drained it moves on to the next lists, taking
// their remaining units.  Every workgroup stops after one pass over all lists, so the launch
// ends when every list is drained.  A unit's results are written by exactly the workgroup
// that took it, so the images do not depend on the order.  (One class per kernel: a kernel
// holding several classes' bodies needs more registers than any one of them.)
template <int CAP>
__global__ __launch_bounds__(kThreads) void gather_queue_kernel(const GatherEntry* __restrict__ tab,
                                                                const int2* __restrict__ items,
                                                                const int32_t* __restrict__ list_begin,
                                                                int32_t* __restrict__ counters,
                                                                const float2* __restrict__ rec,
                                                                const int32_t* __restrict__ plan,
                                                                float2* __restrict__ image, float2* __restrict__ part,
                                                                int32_t* __restrict__ wg_units) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[Lds<CAP>::kBytes];
    __shared__ int next_item;
    int list = 0;   // lists passed so far (thread 0)
    int taken = 0;  // units this workgroup took (thread 0)
    for (;;) {
        if (threadIdx.x == 0) {
            int got = -1;
            while (list < kQueueLists) {
                const int q = ((int)blockIdx.x + list) % kQueueLists;
                const int i = atomicAdd(&counters[q], 1);
                if (i < list_begin[q + 1] - list_begin[q]) {
                    got = list_begin[q] + i;
                    ++taken;
                    break;
                }
                ++list;
            }
            next_item = got;
        }
        __syncthreads();  // also orders the previous unit's LDS reads before this unit's writes
        const int it = next_item;
        if (it < 0) break;
        const int2 w = items[it];
        const GatherEntry e = tab[w.x];
        if (e.cap == CAP)
            gather_body<CAP, false>(rec + e.rec_off, plan + e.plan_off, (e.split > 1 ? part : image) + e.out_off, e.n,
                                    e.m, e.t, w.y, lds);
        __syncthreads();  // every thread has read next_item and the unit's LDS before they are reused
    }
    // per-workgroup unit counts: their sum equals the number of units when each was taken once
    if (wg_units && threadIdx.x == 0) wg_units[blockIdx.x] = taken;
}

__global__ void fill_zero_kernel(int32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// |v|^2 with one fixed rounding sequence, so that every intensity of the library (the gather's
// share reduction and kk_compound) agrees bit for bit.
__device__ __forceinline__ float norm2(float2 v) { return __builtin_fmaf(v.x, v.x, v.y * v.y); }

// Sum of the K pair shares of each set (fixed order), written as the per-set images, and the
// Eq. 8 / Eq. 9 intensity of the set images when requested.
__device__ __forceinline__ void reduce_body(const float2* __restrict__ part, int K, int S, int npix,
                                            float2* __restrict__ image, float* __restrict__ inten, int mode, int i) {
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
        inc += norm2(v);
    }
    if (inten) inten[i] = (mode == KK_COMPOUND_COHERENT) ? norm2(coh) : inc;
}

__global__ void reduce_kernel(const float2* __restrict__ part, int K, int S, int npix, float2* __restrict__ image,
                              float* __restrict__ inten, int mode) {
    reduce_body(part, K, S, npix, image, inten, mode, blockIdx.x * blockDim.x + threadIdx.x);
}

// Grouped share reduction and compounding: block b covers pixels (b - block0) * 256 .. of
// frame entry blk[b].  The shares sit in the workspace when the frame's plan splits its pairs;
// otherwise the images themselves are the single share (read only, not rewritten).
__global__ __launch_bounds__(256) void reduce_grouped(const ReduceEntry* __restrict__ tab,
                                                     const int32_t* __restrict__ blk, const float2* part,
                                                     float2* image, float* __restrict__ inten) {
    const ReduceEntry e = tab[blk[blockIdx.x]];
    const int i = ((int)blockIdx.x - e.block0) * 256 + (int)threadIdx.x;
    reduce_body(e.K > 1 ? part + e.part_off : image + e.img_off, e.K, e.S, e.npix,
                e.K > 1 ? image + e.img_off : nullptr, e.inten_off >= 0 ? inten + e.inten_off : nullptr, e.mode, i);
}

template <int CAP, bool DAS>
hipError_t launch_gather(const float2* rec, const int32_t* plan_dev, float2* out, int blocks, int n, int m, int t,
                         hipStream_t st) {
    hipLaunchKernelGGL((gather_kernel<CAP, DAS>), dim3(blocks), dim3(kThreads), 0, st, rec, plan_dev, out, n, m, t);
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

hipError_t launch_fill_zero(int32_t* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_gather_queue(int cap, const GatherEntry* tab, const int2* items, const int32_t* list_begin,
                               int32_t* counters, int workgroups, const float2* rec, const int32_t* plan,
                               float2* image, float2* part, int32_t* wg_units, hipStream_t st) {
    const dim3 g(workgroups), b(kThreads);
    switch (cap) {
#define KK_QUEUE_CASE(C)                                                                                        \
    case C:                                                                                                     \
        hipLaunchKernelGGL(gather_queue_kernel<C>, g, b, 0, st, tab, items, list_begin, counters, rec, plan, image, \
                           part, wg_units);                                                                     \
        break;
        KK_QUEUE_CASE(64)
        KK_QUEUE_CASE(128)
        KK_QUEUE_CASE(192)
        KK_QUEUE_CASE(256)
        KK_QUEUE_CASE(320)
        KK_QUEUE_CASE(384)
        KK_QUEUE_CASE(448)
        KK_QUEUE_CASE(512)
#undef KK_QUEUE_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_grouped(const ReduceEntry* tab, const int32_t* blk, int blocks, const float2* part,
                                 float2* image, float* inten, hipStream_t st) {
    hipLaunchKernelGGL(reduce_grouped, dim3(blocks), dim3(256), 0, st, tab, blk, part, image, inten);
    return hipGetLastError();
}

size_t gather_workspace_bytes(const int32_t* h) {
    if (h[PW_SPLIT] <= 1) return 0;
    return (size_t)h[PW_SPLIT] * h[PW_S] * h[PW_X] * h[PW_Z] * 8;
}

bool gather_plan_ok(const int32_t* h, size_t plan_bytes, bool das) {
    return plan_bytes >= (size_t)PW_HEADER_WORDS * 4 && h[PW_MAGIC] == kPlanMagic &&
           h[PW_KIND] == (das ? kPlanKindDAS : kPlanKindKK) && (size_t)h[PW_TOTAL] * 4 <= plan_bytes &&
           h[PW_PB] == pairs_per_batch(h[PW_CAP]) && h[PW_PB] == kWaves && h[PW_SPLIT] >= 1 && h[PW_SPLIT] <= kMaxSplit;
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
