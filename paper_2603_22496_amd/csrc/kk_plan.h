// Layout of the beamforming plans built on the host (kk_beamform_plan, das_plan) and read by
// the gather kernels.  A plan is a flat array of int32 words: a fixed header followed by the
// folded delay tables and the per-tile record windows.  Private to this library.
#pragma once
#include <stdint.h>

namespace kk {

constexpr int32_t kPlanMagic = 0x4B4B5031;  // "KKP1"
constexpr int32_t kPlanKindKK = 0;
constexpr int32_t kPlanKindDAS = 1;

// Pixel tile of one workgroup: 64 lateral pixels (one per lane) by 16 axial pixels.
constexpr int32_t kTileX = 64;
constexpr int32_t kTileZ = 16;

// Largest pair split: a (set, tile) is shared by up to this many workgroups when there are
// fewer (set, tile) units than CUs, their partial images summed in a fixed order afterwards.
constexpr int32_t kMaxSplit = 8;
constexpr int32_t kTargetWorkgroups = 256;  // one per CU of an MI355X

// Window slot capacities (record samples per pair and tile) for which kernels exist.
constexpr int32_t kCaps[] = {64, 128, 192, 256, 320, 384, 448, 512};
constexpr int32_t kNumCaps = 8;

// Pairs in flight per workgroup: one per wave, each wave owning one LDS window slot of cap
// 16-byte entries (at most 16 x 512 x 16 B = 128 KiB).
constexpr int32_t pairs_per_batch(int32_t cap) { return cap > 0 ? 16 : 0; }

enum PlanWord : int32_t {
    PW_MAGIC = 0,
    PW_KIND,
    PW_N,          // transmit angles
    PW_M,          // KK: distinct receive angles; DAS: elements L
    PW_T,          // samples per record
    PW_P,          // pair slots (KK) or N*L (DAS)
    PW_S,          // sets (DAS: 1)
    PW_X,
    PW_Z,
    PW_NXT,        // tiles along x and z
    PW_NZT,
    PW_XPAD,       // n_xt * 64
    PW_ZPAD,       // n_zt * 16
    PW_CAP,        // slot capacity (entries) of the kernel variant
    PW_MAXW,       // largest window any (pair, tile) needs
    PW_PB,         // pairs in flight per workgroup (one per wave)
    PW_OFF_SET,    // int32[S+1]   first pair of each set (pairs grouped by set)
    PW_OFF_REC,    // int32[P]     record index: i*M + o (KK), i*L + l (DAS)
    PW_OFF_A,      // int32[P or N][XPAD]  folded lateral delay (Q16.16, includes t0)
    PW_OFF_B,      // int32[P or N][ZPAD]  folded axial delay
    PW_OFF_LO,     // int32[n_tiles][P]    first record sample of each window
    PW_OFF_C,      // DAS: int32[L][ZPAD][XPAD] receive delay, x fastest; KK: 0
    PW_OFF_TX,     // DAS: int32[P] transmit index of pair p = l N + i (A/B row i); KK: pair index p
    PW_TOTAL,      // plan length in words
    PW_SPLIT,      // pair shares per (set, tile): workgroups = tiles * S * SPLIT
    PW_HEADER_WORDS = 32
};

}  // namespace kk
