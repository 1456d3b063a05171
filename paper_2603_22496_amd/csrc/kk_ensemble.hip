// Frame ensembles on gfx950: many KK frames of different shapes imaged as one unit of work.
//
// Per frame the steps are those of kk_decompose (analytic spectra, the Eq. 3 per-bin
// contraction, inverse transforms) and kk_beamform (the Eq. 5 delay-gather, the pair-share
// sum and the Eq. 8 / Eq. 9 intensity).  Here every step is one launch over all frames of a
// shape class: each block of a grouped launch finds its frame through a per-block table and
// then runs exactly the per-frame kernel body, so results equal the per-frame entry points'.
// Shape classes: the FFT length for the transforms and the contraction (their kernels are
// specialised on it), the window capacity for the gather.  The gather is a persistent launch
// per window class (one workgroup per CU) draining work lists of (frame, set, pair share,
// pixel tile) units, so frames of very different cost balance across the chip.
//
// The plan is built once on the host and copied to the device; a run is a fixed list of
// launches read from the host copy, so it can be captured into one HIP graph.  The
// workspace keeps RF_theta of every frame; the spectra of the decomposition are staged per
// group of frames whose spectra fit a budget, the groups decomposed one after the other.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

namespace kk {
namespace {

constexpr int32_t kEnsMagic = 0x4B4B4531;  // "KKE1"
constexpr int32_t kEnsVersion = 1;
constexpr int kMaxQueueWorkgroups = 1024;   // per-workgroup unit counts kept per class
// units of gather work per (pair share x 1024 pixels): the fixed part (window and delay
// set-up, the end-of-unit reduction) is worth about this many pairs
constexpr int64_t kUnitOverheadPairs = 12;

enum LaunchKind : int32_t { LK_FWD = 0, LK_CONTRACT = 1, LK_INV = 2, LK_GATHER = 3, LK_REDUCE = 4 };

// One launch of a run (host-read).  Offsets in plan words.
struct LaunchRec {
    int32_t kind;
    int32_t arg;       // FFT log2 length, or window capacity (gather)
    int32_t tab_off;   // work table
    int32_t aux_off;   // per-block table, or gather items (int2)
    int32_t aux2_off;  // gather: list bounds [kQueueLists + 1]
    int32_t blocks;    // grid size (grouped), units (gather)
    int32_t slot;      // gather: class index (counter row)
    int32_t pad;
};

struct EnsHeader {
    int32_t magic, version, nframes, precision;
    int32_t total_words, nlaunch, off_launch, off_frames;
    int32_t ngroups, nunits, pad0, pad1;
    int64_t rf_elems, image_elems, inten_elems, ws_bytes;
    int64_t ws_counters, ws_units;  // byte offsets: queue counters [8][kQueueLists], unit counts
    kk_ensemble_tuning tuning;
};

static_assert(sizeof(kk_ensemble_frame_info) % 8 == 0, "frame records pack");

constexpr int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int cap_class(int cap) {
    for (int i = 0; i < kNumCaps; ++i)
        if (kCaps[i] == cap) return i;
    return -1;
}

// Word buffer with aligned appends.
struct Words {
    std::vector<int32_t> w;
    int32_t reserve(int64_t words, int align_words = 16) {
        const int64_t at = align_up((int64_t)w.size(), align_words);
        w.resize((size_t)(at + words), 0);
        return (int32_t)at;
    }
    template <class T>
    int32_t put(const std::vector<T>& v, int align_words = 16) {
        static_assert(sizeof(T) % 4 == 0, "word-sized records");
        const int32_t at = reserve((int64_t)(v.size() * sizeof(T) / 4), align_words);
        if (!v.empty()) std::memcpy(w.data() + at, v.data(), v.size() * sizeof(T));
        return at;
    }
};

struct FrameWork {
    kk_ensemble_frame_info info;
    int log2n, kpad, ncol, cls;
    int64_t x_bytes, d_bytes, y_bytes, x_off_ws, d_off_ws, y_off_ws;  // decomposition buffers within the group region
    std::vector<int32_t> set_begin;                 // S + 1
    int ntiles;
};

bool read_header(const void* plan_host, size_t plan_bytes, EnsHeader* h) {
    if (!plan_host || plan_bytes < sizeof(EnsHeader)) return false;
    std::memcpy(h, plan_host, sizeof(EnsHeader));
    return h->magic == kEnsMagic && h->version == kEnsVersion && h->nframes >= 1 && h->total_words > 0 &&
           (size_t)h->total_words * 4 <= plan_bytes && h->off_launch >= 0 && h->off_frames >= 0;
}

int32_t build_plan(const kk_ensemble_frame* frames, int nf, int precision, const kk_ensemble_tuning& tu,
                   int64_t budget, Words& out) {
    if (!frames) return KK_E_NULL;
    if (nf < 1) return KK_E_ARG;
    if (precision != KK_PREC_FP32 && precision != KK_PREC_BF16X3 && precision != KK_PREC_FP16X3)
        return KK_E_UNSUPPORTED;
    if (tu.queue != 0 && tu.queue != 1) return KK_E_ARG;
    for (int c = 0; c < KK_ENSEMBLE_CLASSES; ++c)
        if (tu.pair_tile[c] < 0) return KK_E_ARG;
    std::vector<FrameWork> fw(nf);
    int64_t rf_elems = 0, img_elems = 0, inten_elems = 0;
    // workspace: queue counters and unit counts, RF_theta of all frames, shares, spectra
    const int64_t ws_counters = 0;
    const int64_t ws_units = 256;
    int64_t ws = align_up(ws_units + (int64_t)KK_ENSEMBLE_CLASSES * kMaxQueueWorkgroups * 4, 256);
    for (int f = 0; f < nf; ++f) {
        const kk_ensemble_frame& fr = frames[f];
        if (!fr.shift_q || !fr.plan) return KK_E_NULL;
        const int32_t* h = static_cast<const int32_t*>(fr.plan);
        if (!gather_plan_ok(h, fr.plan_bytes, false)) return KK_E_WORKSPACE;
        const kk_geom& g = fr.geom;
        const int lg = log2_exact(fr.tpad);
        if (fr.N < 1 || fr.M < 1 || g.L < 1 || g.L > 65536 || g.T < 1 || lg < kMinLog2Fft || lg > kMaxLog2Fft ||
            g.T > fr.tpad || h[PW_N] != fr.N || h[PW_M] != fr.M || h[PW_T] != g.T ||
            (fr.mode != -1 && fr.mode != KK_COMPOUND_COHERENT && fr.mode != KK_COMPOUND_INCOHERENT))
            return KK_E_ARG;
        if ((int64_t)fr.N * g.L > 0x7fffffff || (int64_t)fr.N * fr.M > 0x7fffffff) return KK_E_ARG;
        FrameWork& w = fw[f];
        kk_ensemble_frame_info& in = w.info;
        std::memset(&in, 0, sizeof(in));
        in.N = fr.N;
        in.L = g.L;
        in.T = g.T;
        in.M = fr.M;
        in.S = h[PW_S];
        in.X = h[PW_X];
        in.Z = h[PW_Z];
        in.P = h[PW_P];
        in.tpad = fr.tpad;
        in.cap = h[PW_CAP];
        in.mode = fr.mode;
        w.cls = cap_class(in.cap);
        if (w.cls < 0) return KK_E_WORKSPACE;
        w.log2n = lg;
        w.kpad = (fr.tpad / 2 + 1 + kBinBlock - 1) / kBinBlock * kBinBlock;
        w.ncol = (fr.N + 31) / 32 * 32;
        w.ntiles = h[PW_NXT] * h[PW_NZT];
        w.set_begin.assign(h + h[PW_OFF_SET], h + h[PW_OFF_SET] + in.S + 1);
        int max_set = 0;
        for (int s = 0; s < in.S; ++s) max_set = std::max(max_set, w.set_begin[s + 1] - w.set_begin[s]);
        const int pt = tu.pair_tile[w.cls];
        in.split = pt > 0 ? std::min<int>(kMaxSplit, std::max(1, (max_set + pt - 1) / pt)) : 1;
        const int64_t npix = (int64_t)in.X * in.Z;
        if ((int64_t)w.ntiles * in.S * in.split > 0x7fffffff || npix > 0x7fffffff) return KK_E_ARG;
        in.rf_offset = rf_elems;
        rf_elems = align_up(rf_elems + (int64_t)fr.N * g.L * g.T, 128);
        in.image_offset = img_elems;
        img_elems = align_up(img_elems + (int64_t)in.S * npix, 32);
        in.intensity_offset = -1;
        if (fr.mode >= 0) {
            in.intensity_offset = inten_elems;
            inten_elems = align_up(inten_elems + npix, 64);
        }
        in.rf_theta_offset = ws / 8;
        ws = align_up(ws + (int64_t)fr.N * fr.M * g.T * 8, 256);
        w.x_bytes = align_up((int64_t)w.kpad * w.ncol * g.L * 8, 256);
        w.d_bytes = align_up((int64_t)phase_table_bytes(fr.M, g.L, w.log2n), 256);
        w.y_bytes = align_up((int64_t)fr.N * fr.M * w.kpad * 8, 256);
    }
    for (int f = 0; f < nf; ++f) {
        kk_ensemble_frame_info& in = fw[f].info;
        in.share_offset = -1;
        if (in.split > 1) {
            in.share_offset = ws / 8;
            ws = align_up(ws + (int64_t)in.split * in.S * in.X * in.Z * 8, 256);
        }
    }
    // decomposition groups: consecutive frames whose spectra fit the budget
    const int64_t ws_dec = ws;
    int64_t group_bytes = 0, region = 0;
    int ngroups = 0;
    for (int f = 0; f < nf; ++f) {
        FrameWork& w = fw[f];
        const int64_t need = w.x_bytes + w.d_bytes + w.y_bytes;
        if (f == 0 || (budget > 0 && group_bytes + need > budget)) {
            ++ngroups;
            group_bytes = 0;
        }
        w.info.group = ngroups - 1;
        w.x_off_ws = ws_dec + group_bytes;
        w.d_off_ws = w.x_off_ws + w.x_bytes;
        w.y_off_ws = w.d_off_ws + w.d_bytes;
        group_bytes += need;
        region = std::max(region, group_bytes);
    }
    ws = ws_dec + region;

    // ---- plan words
    Words W;
    const int32_t hdr_words = (int32_t)align_up((int64_t)sizeof(EnsHeader) / 4, 16);
    W.reserve(hdr_words);
    const int32_t off_frames = W.reserve((int64_t)nf * sizeof(kk_ensemble_frame_info) / 4);
    for (int f = 0; f < nf; ++f) {
        const kk_ensemble_frame& fr = frames[f];
        const int32_t* h = static_cast<const int32_t*>(fr.plan);
        const int32_t po = W.reserve(h[PW_TOTAL]);
        std::memcpy(W.w.data() + po, h, (size_t)h[PW_TOTAL] * 4);
        W.w[po + PW_SPLIT] = fw[f].info.split;
        fw[f].info.plan_offset = po;
        const int32_t so = W.reserve((int64_t)fr.M * fr.geom.L);
        std::memcpy(W.w.data() + so, fr.shift_q, (size_t)fr.M * fr.geom.L * 4);
        fw[f].info.shift_offset = so;
    }
    std::vector<LaunchRec> launches;
    auto check_blocks = [](int64_t b) { return b >= 1 && b <= 0x7fffffff; };
    // decomposition: per group, per FFT length present
    for (int gi = 0; gi < ngroups; ++gi) {
        std::vector<int> lgs;
        for (int f = 0; f < nf; ++f)
            if (fw[f].info.group == gi) lgs.push_back(fw[f].log2n);
        std::sort(lgs.begin(), lgs.end());
        lgs.erase(std::unique(lgs.begin(), lgs.end()), lgs.end());
        std::vector<LaunchRec> fwd_l, con_l, inv_l;
        for (int lg : lgs) {
            std::vector<FwdEntry> fe;
            std::vector<ContractEntry> ce;
            std::vector<InvEntry> ie;
            std::vector<int32_t> fb, cb, ib;
            for (int f = 0; f < nf; ++f) {
                const FrameWork& w = fw[f];
                if (w.info.group != gi || w.log2n != lg) continue;
                const kk_ensemble_frame_info& in = w.info;
                const int e = (int)fe.size();
                FwdEntry a{};
                a.rf_off = in.rf_offset;
                a.x_off = w.x_off_ws / 8;
                a.d_off = w.d_off_ws / 8;
                a.shift_off = in.shift_offset;
                a.M = in.M;
                a.ntraces = in.N * in.L;
                a.T = in.T;
                a.L = in.L;
                a.ncol = w.ncol;
                a.kpad = w.kpad;
                a.block0 = (int32_t)fb.size();
                a.split = precision;
                a.xscale = precision == KK_PREC_FP16X3 ? std::ldexp(1.0f, fp16_prescale_exponent(in.T)) : 1.0f;
                // record pairs (transmits i, i+1 of one element), then the phase-table blocks
                const int64_t nfb = (int64_t)in.L * ((in.N + 1) / 2) + phase_table_blocks(in.M, in.L, lg);
                if (!check_blocks((int64_t)fb.size() + nfb)) return KK_E_ARG;
                fb.insert(fb.end(), (size_t)nfb, e);
                fe.push_back(a);
                ContractEntry c{};
                c.x_off = a.x_off;
                c.d_off = a.d_off;
                c.y_off = w.y_off_ws / 8;
                c.shift_off = in.shift_offset;
                c.ntx = in.N;
                c.M = in.M;
                c.L = in.L;
                c.ncol = w.ncol;
                c.kpad = w.kpad;
                c.nkb = (1 << lg) / 2 / kBinBlock;
                // FP32: angle tiles of 8 R8 and column groups of 16; split: angle tiles of 16 or
                // 32 (16 T16) and column groups of 32
                const bool fp32 = precision == KK_PREC_FP32;
                const int a16 = in.M > 16 ? 32 : 16;
                c.nrt = fp32 ? contract_angle_tiles(in.M) : (in.M + a16 - 1) / a16;
                c.block0 = (int32_t)cb.size();
                c.xscale = a.xscale;
                c.yscale = 1.0f / a.xscale;
                const int64_t ncb =
                    (int64_t)c.nkb * c.nrt * (fp32 ? (in.N + kContractCols - 1) / kContractCols : w.ncol / 32);
                if (!check_blocks((int64_t)cb.size() + ncb)) return KK_E_ARG;
                cb.insert(cb.end(), (size_t)ncb, e);
                ce.push_back(c);
                InvEntry v{};
                v.y_off = c.y_off;
                v.out_off = in.rf_theta_offset;
                v.x_off = a.x_off;
                v.shift_off = in.shift_offset;
                v.kpad = w.kpad;
                v.T = in.T;
                v.M = in.M;
                v.L = in.L;
                v.ncol = w.ncol;
                v.block0 = (int32_t)ib.size();
                const int64_t nib = (int64_t)in.N * in.M;
                if (!check_blocks((int64_t)ib.size() + nib)) return KK_E_ARG;
                ib.insert(ib.end(), (size_t)nib, e);
                ie.push_back(v);
            }
            LaunchRec r{};
            r.arg = lg;
            r.kind = LK_FWD;
            r.tab_off = W.put(fe);
            r.aux_off = W.put(fb);
            r.blocks = (int32_t)fb.size();
            fwd_l.push_back(r);
            r.kind = LK_CONTRACT;
            r.tab_off = W.put(ce);
            r.aux_off = W.put(cb);
            r.blocks = (int32_t)cb.size();
            con_l.push_back(r);
            r.kind = LK_INV;
            r.tab_off = W.put(ie);
            r.aux_off = W.put(ib);
            r.blocks = (int32_t)ib.size();
            inv_l.push_back(r);
        }
        launches.insert(launches.end(), fwd_l.begin(), fwd_l.end());
        launches.insert(launches.end(), con_l.begin(), con_l.end());
        launches.insert(launches.end(), inv_l.begin(), inv_l.end());
    }
    // gather: one entry per frame, work lists per window class
    std::vector<GatherEntry> ge(nf);
    for (int f = 0; f < nf; ++f) {
        const kk_ensemble_frame_info& in = fw[f].info;
        GatherEntry& e = ge[f];
        e.rec_off = in.rf_theta_offset;
        e.out_off = in.split > 1 ? in.share_offset : in.image_offset;
        e.plan_off = in.plan_offset;
        e.cap = in.cap;
        e.split = in.split;
        e.n = in.N;
        e.m = in.M;
        e.t = in.T;
    }
    const int32_t gtab = W.put(ge);
    int nunits_total = 0;
    for (int cls = 0; cls < kNumCaps; ++cls) {
        struct Unit {
            int32_t f, r;
            int64_t cost;
        };
        std::vector<Unit> units;
        for (int f = 0; f < nf; ++f) {
            const FrameWork& w = fw[f];
            if (w.cls != cls) continue;
            const int K = w.info.split, S = w.info.S;
            for (int sh = 0; sh < S * K; ++sh) {
                const int s = sh / K, hh = sh - s * K;
                const int sb = w.set_begin[s], se = w.set_begin[s + 1];
                const int share = (se - sb + K - 1) / K;
                const int pb = std::min(se, sb + hh * share), pe = std::min(se, pb + share);
                const int64_t cost = (int64_t)(pe - pb) + kUnitOverheadPairs;
                for (int t = 0; t < w.ntiles; ++t) units.push_back({f, sh * w.ntiles + t, cost});
            }
        }
        if (units.empty()) continue;
        int64_t total = 0;
        for (const Unit& u : units) total += u.cost;
        std::vector<int32_t> bounds(kQueueLists + 1, 0);
        std::vector<int32_t> items;
        items.reserve(units.size() * 2);
        if (tu.queue == 0) {
            std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
            for (int q = 1; q <= kQueueLists; ++q) bounds[q] = (int32_t)units.size();
        } else {
            // contiguous runs of equal cost, in frame order (each list keeps its frames' data
            // in its own XCD's L2)
            int64_t acc = 0;
            int q = 0;
            for (size_t i = 0; i < units.size(); ++i) {
                while (q < kQueueLists - 1 && acc >= total * (q + 1) / kQueueLists) bounds[++q] = (int32_t)i;
                acc += units[i].cost;
            }
            while (q < kQueueLists) bounds[++q] = (int32_t)units.size();
        }
        for (const Unit& u : units) {
            items.push_back(u.f);
            items.push_back(u.r);
        }
        LaunchRec r{};
        r.kind = LK_GATHER;
        r.arg = kCaps[cls];
        r.tab_off = gtab;
        r.aux_off = W.put(items);
        r.aux2_off = W.put(bounds);
        r.blocks = (int32_t)units.size();
        r.slot = cls;
        launches.push_back(r);
        nunits_total += (int)units.size();
    }
    // share sums and intensities
    {
        std::vector<ReduceEntry> re;
        std::vector<int32_t> rb;
        for (int f = 0; f < nf; ++f) {
            const kk_ensemble_frame_info& in = fw[f].info;
            if (in.split <= 1 && in.mode < 0) continue;
            ReduceEntry e{};
            e.part_off = in.split > 1 ? in.share_offset : 0;
            e.img_off = in.image_offset;
            e.inten_off = in.intensity_offset;
            e.K = in.split;
            e.S = in.S;
            e.npix = in.X * in.Z;
            e.mode = in.mode < 0 ? 0 : in.mode;
            e.block0 = (int32_t)rb.size();
            const int64_t nb = ((int64_t)e.npix + 255) / 256;
            if (!check_blocks((int64_t)rb.size() + nb)) return KK_E_ARG;
            rb.insert(rb.end(), (size_t)nb, (int32_t)re.size());
            re.push_back(e);
        }
        if (!re.empty()) {
            LaunchRec r{};
            r.kind = LK_REDUCE;
            r.tab_off = W.put(re);
            r.aux_off = W.put(rb);
            r.blocks = (int32_t)rb.size();
            launches.push_back(r);
        }
    }
    const int32_t off_launch = W.put(launches);
    if ((int64_t)W.w.size() > 0x7fffffff / 4) return KK_E_ARG;
    for (int f = 0; f < nf; ++f)
        std::memcpy(W.w.data() + off_frames + (size_t)f * sizeof(kk_ensemble_frame_info) / 4, &fw[f].info,
                    sizeof(kk_ensemble_frame_info));
    EnsHeader H{};
    H.magic = kEnsMagic;
    H.version = kEnsVersion;
    H.nframes = nf;
    H.precision = precision;
    H.total_words = (int32_t)W.w.size();
    H.nlaunch = (int32_t)launches.size();
    H.off_launch = off_launch;
    H.off_frames = off_frames;
    H.ngroups = ngroups;
    H.nunits = nunits_total;
    H.rf_elems = rf_elems;
    H.image_elems = img_elems;
    H.inten_elems = inten_elems;
    H.ws_bytes = ws;
    H.ws_counters = ws_counters;
    H.ws_units = ws_units;
    H.tuning = tu;
    std::memcpy(W.w.data(), &H, sizeof(H));
    out.w.swap(W.w);
    return KK_OK;
}

int32_t run_plan(const void* plan_host, const void* plan_dev, size_t plan_bytes, const int16_t* rf, float* image,
                 float* intensity, void* ws, size_t ws_bytes, int32_t stages, hipStream_t st) {
    EnsHeader H;
    if (!plan_host || !plan_dev || !rf || !image || !ws) return KK_E_NULL;
    if (!read_header(plan_host, plan_bytes, &H)) return KK_E_WORKSPACE;
    if ((int64_t)ws_bytes < H.ws_bytes) return KK_E_WORKSPACE;
    if (H.inten_elems > 0 && !intensity) return KK_E_NULL;
    if (stages < 0 || stages > KK_STAGE_ALL) return KK_E_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return KK_E_HIP;
    const int workgroups = std::min(cus, kMaxQueueWorkgroups);
    const int32_t* ph = static_cast<const int32_t*>(plan_host);
    const int32_t* pd = static_cast<const int32_t*>(plan_dev);
    unsigned char* wsb = static_cast<unsigned char*>(ws);
    float2* wsf = reinterpret_cast<float2*>(wsb);
    float2* img = reinterpret_cast<float2*>(image);
    int32_t* counters = reinterpret_cast<int32_t*>(wsb + H.ws_counters);
    int32_t* units = reinterpret_cast<int32_t*>(wsb + H.ws_units);
    for (int i = 0; i < H.nlaunch; ++i) {
        LaunchRec r;
        std::memcpy(&r, ph + H.off_launch + (size_t)i * sizeof(LaunchRec) / 4, sizeof(r));
        hipError_t e = hipSuccess;
        switch (r.kind) {
            case LK_FWD:
                if (stages & KK_STAGE_FFT)
                    e = launch_fft_forward_grouped(r.arg, reinterpret_cast<const FwdEntry*>(pd + r.tab_off),
                                                   pd + r.aux_off, r.blocks, rf, wsf, pd, st);
                break;
            case LK_CONTRACT:
                if (stages & KK_STAGE_CONTRACT)
                    e = launch_contract_grouped(r.arg, H.precision,
                                                reinterpret_cast<const ContractEntry*>(pd + r.tab_off),
                                                pd + r.aux_off, r.blocks, wsf, pd, st);
                break;
            case LK_INV:
                if (stages & KK_STAGE_INVERSE)
                    e = launch_fft_inverse_grouped(r.arg, reinterpret_cast<const InvEntry*>(pd + r.tab_off),
                                                   pd + r.aux_off, r.blocks, wsf, pd, st);
                break;
            case LK_GATHER:
                if (stages & KK_STAGE_GATHER) {
                    int32_t* cnt = counters + r.slot * kQueueLists;
                    e = launch_fill_zero(cnt, kQueueLists, st);
                    if (e == hipSuccess)
                        e = launch_gather_queue(r.arg, reinterpret_cast<const GatherEntry*>(pd + r.tab_off),
                                                reinterpret_cast<const int2*>(pd + r.aux_off), pd + r.aux2_off, cnt,
                                                workgroups, wsf, pd, img, wsf, units + r.slot * kMaxQueueWorkgroups,
                                                st);
                }
                break;
            case LK_REDUCE:
                if (stages & KK_STAGE_REDUCE)
                    e = launch_reduce_grouped(reinterpret_cast<const ReduceEntry*>(pd + r.tab_off), pd + r.aux_off,
                                              r.blocks, wsf, img, intensity, st);
                break;
            default: return KK_E_WORKSPACE;
        }
        if (e != hipSuccess) return KK_E_HIP;
    }
    return KK_OK;
}

struct EnsembleGraph {
    hipGraphExec_t exec;
};

float median_of(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.f : v[v.size() / 2];
}

}  // namespace
}  // namespace kk

extern "C" {

void kk_ensemble_default_tuning(kk_ensemble_tuning* t) {
    if (!t) return;
    std::memset(t, 0, sizeof(*t));
    t->queue = 1;
}

int32_t kk_ensemble_plan(const kk_ensemble_frame* frames, int32_t nframes, int32_t precision,
                         const kk_ensemble_tuning* tuning, int64_t spectra_budget, void* plan, size_t plan_bytes,
                         size_t* plan_bytes_out) {
    if (!plan_bytes_out) return KK_E_NULL;
    if (spectra_budget < 0) return KK_E_ARG;
    kk_ensemble_tuning tu;
    kk_ensemble_default_tuning(&tu);
    if (tuning) tu = *tuning;
    kk::Words W;
    const int32_t rc = kk::build_plan(frames, nframes, precision, tu, spectra_budget, W);
    if (rc != KK_OK) return rc;
    const size_t need = W.w.size() * 4;
    *plan_bytes_out = need;
    if (!plan || plan_bytes < need) return KK_E_CAPACITY;
    std::memcpy(plan, W.w.data(), need);
    return KK_OK;
}

int32_t kk_ensemble_query(const void* plan_host, size_t plan_bytes, kk_ensemble_sizes* sizes) {
    if (!plan_host || !sizes) return KK_E_NULL;
    kk::EnsHeader H;
    if (!kk::read_header(plan_host, plan_bytes, &H)) return KK_E_WORKSPACE;
    std::memset(sizes, 0, sizeof(*sizes));
    sizes->rf_elems = H.rf_elems;
    sizes->image_elems = H.image_elems;
    sizes->intensity_elems = H.inten_elems;
    sizes->ws_bytes = H.ws_bytes;
    sizes->units_offset = H.ws_units;
    sizes->nframes = H.nframes;
    sizes->ngroups = H.ngroups;
    sizes->nlaunches = H.nlaunch;
    sizes->nunits = H.nunits;
    sizes->precision = H.precision;
    return KK_OK;
}

int32_t kk_ensemble_frame_query(const void* plan_host, size_t plan_bytes, int32_t f, kk_ensemble_frame_info* info) {
    if (!plan_host || !info) return KK_E_NULL;
    kk::EnsHeader H;
    if (!kk::read_header(plan_host, plan_bytes, &H)) return KK_E_WORKSPACE;
    if (f < 0 || f >= H.nframes) return KK_E_ARG;
    std::memcpy(info,
                static_cast<const int32_t*>(plan_host) + H.off_frames + (size_t)f * sizeof(kk_ensemble_frame_info) / 4,
                sizeof(*info));
    return KK_OK;
}

int32_t kk_ensemble_run(const void* plan_host, const void* plan_dev, size_t plan_bytes, const int16_t* rf,
                        float* image, float* intensity, void* ws, size_t ws_bytes, int32_t stages, void* stream) {
    return kk::run_plan(plan_host, plan_dev, plan_bytes, rf, image, intensity, ws, ws_bytes, stages,
                        (hipStream_t)stream);
}

int32_t kk_ensemble_graph_create(const void* plan_host, const void* plan_dev, size_t plan_bytes, const int16_t* rf,
                                 float* image, float* intensity, void* ws, size_t ws_bytes, void* stream,
                                 void** graph_out) {
    if (!graph_out) return KK_E_NULL;
    if (!stream) return KK_E_ARG;
    *graph_out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return KK_E_HIP;
    const int32_t rc = kk::run_plan(plan_host, plan_dev, plan_bytes, rf, image, intensity, ws, ws_bytes,
                                    KK_STAGE_ALL, st);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (rc != KK_OK || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != KK_OK ? rc : KK_E_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return KK_E_HIP;
    *graph_out = new kk::EnsembleGraph{exec};
    return KK_OK;
}

int32_t kk_ensemble_graph_launch(void* graph, void* stream) {
    if (!graph) return KK_E_NULL;
    return hipGraphLaunch(static_cast<kk::EnsembleGraph*>(graph)->exec, (hipStream_t)stream) == hipSuccess ? KK_OK
                                                                                                          : KK_E_HIP;
}

int32_t kk_ensemble_graph_destroy(void* graph) {
    if (!graph) return KK_E_NULL;
    kk::EnsembleGraph* g = static_cast<kk::EnsembleGraph*>(graph);
    const hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    return e == hipSuccess ? KK_OK : KK_E_HIP;
}

int32_t kk_ensemble_autotune(const kk_ensemble_frame* frames, int32_t nframes, int32_t precision,
                             int64_t spectra_budget, void* plan_dev, size_t plan_dev_bytes, const int16_t* rf,
                             float* image, float* intensity, void* ws, size_t ws_bytes, int32_t reps, void* stream,
                             kk_ensemble_tuning* tuning, float* best_us) {
    using namespace kk;
    if (!tuning || !plan_dev || !rf || !image || !ws) return KK_E_NULL;
    if (reps < 1 || spectra_budget < 0) return KK_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return KK_E_HIP;
    }
    struct Cleanup {
        hipEvent_t a, b;
        ~Cleanup() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } cleanup{e0, e1};
    // plan a candidate, upload it; rc KK_E_WORKSPACE / KK_E_CAPACITY mark candidates that do not fit
    Words W;
    auto prepare = [&](const kk_ensemble_tuning& t) -> int32_t {
        const int32_t rc = build_plan(frames, nframes, precision, t, spectra_budget, W);
        if (rc != KK_OK) return rc;
        EnsHeader H;
        std::memcpy(&H, W.w.data(), sizeof(H));
        if (W.w.size() * 4 > plan_dev_bytes) return KK_E_CAPACITY;
        if ((int64_t)ws_bytes < H.ws_bytes) return KK_E_WORKSPACE;
        if (hipMemcpyAsync(plan_dev, W.w.data(), W.w.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return KK_E_HIP;
        return KK_OK;
    };
    auto time_gather = [&](float* us) -> int32_t {
        std::vector<float> t;
        for (int r = 0; r < reps + 1; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) return KK_E_HIP;
            const int32_t rc = run_plan(W.w.data(), plan_dev, W.w.size() * 4, rf, image, intensity, ws, ws_bytes,
                                        KK_STAGE_GATHER | KK_STAGE_REDUCE, st);
            if (rc != KK_OK) return rc;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return KK_E_HIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return KK_E_HIP;
            if (r > 0) t.push_back(ms * 1000.f);  // the first run warms the new plan's tables
        }
        *us = median_of(t);
        return KK_OK;
    };
    kk_ensemble_tuning best = *tuning;
    int32_t rc = prepare(best);
    if (rc != KK_OK) return rc;
    rc = run_plan(W.w.data(), plan_dev, W.w.size() * 4, rf, image, intensity, ws, ws_bytes, KK_STAGE_ALL, st);
    if (rc != KK_OK) return rc;
    float best_t = 0.f;
    if ((rc = time_gather(&best_t)) != KK_OK) return rc;
    // window classes present, by descending gather work
    std::vector<std::pair<int64_t, int>> cls_work;
    {
        EnsHeader H;
        std::memcpy(&H, W.w.data(), sizeof(H));
        std::vector<int64_t> work(kNumCaps, 0);
        for (int f = 0; f < H.nframes; ++f) {
            kk_ensemble_frame_info in;
            std::memcpy(&in, W.w.data() + H.off_frames + (size_t)f * sizeof(in) / 4, sizeof(in));
            work[cap_class(in.cap)] += (int64_t)in.X * in.Z * in.P;
        }
        for (int c = 0; c < kNumCaps; ++c)
            if (work[c] > 0) cls_work.push_back({-work[c], c});
        std::sort(cls_work.begin(), cls_work.end());
    }
    auto try_candidate = [&](const kk_ensemble_tuning& t) -> int32_t {
        int32_t r = prepare(t);
        if (r == KK_E_CAPACITY || r == KK_E_WORKSPACE) return KK_OK;  // does not fit: skipped
        if (r != KK_OK) return r;
        float us = 0.f;
        if ((r = time_gather(&us)) != KK_OK) return r;
        if (us < best_t) {
            best_t = us;
            best = t;
        }
        return KK_OK;
    };
    {
        kk_ensemble_tuning t = best;
        t.queue = 1 - best.queue;
        if ((rc = try_candidate(t)) != KK_OK) return rc;
    }
    static const int32_t kTiles[] = {0, 512, 256, 128, 64, 32};
    for (const auto& cw : cls_work) {
        const int c = cw.second;
        const int32_t start = best.pair_tile[c];
        for (int32_t pt : kTiles) {
            if (pt == start) continue;
            kk_ensemble_tuning t = best;
            t.pair_tile[c] = pt;
            if ((rc = try_candidate(t)) != KK_OK) return rc;
        }
    }
    *tuning = best;
    if (best_us) *best_us = best_t;
    return KK_OK;
}

}  // extern "C"
