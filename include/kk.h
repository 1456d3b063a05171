/*
 * kk.h - C ABI of the KK (far-field compressive) plane-wave beamforming library for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Khetan & Mertz, "Far-field compressive ultrasound beamforming".  Multi-angle
 * linear-array channel data RF_u(u_l, t) (one record per transmit plane wave theta_i) are
 * decomposed into virtual receive plane waves RF_theta(theta_o, t) (Eq. 3), and images are
 * formed pixel by pixel by summing each selected (theta_i, theta_o) pair at its far-field
 * delay (Eq. 5).  Receive angles follow Eq. 6 (shifted vernier) or Eq. 7 (confocal); sets
 * of Eq. 6 are compounded by Eq. 8 / Eq. 9.  Conventional CPWC delay-and-sum (Eq. 4) is
 * provided on the same data as the comparator.
 *
 * Conventions (all entry points)
 *   - Sizes are int32, angles are radians (FP64), lengths metres, times seconds (SI).
 *   - Arrays are row-major, last index fastest.  Complex samples are interleaved float pairs
 *     (re, im), i.e. "float2".
 *   - Element l sits at u_l = ((2l - (L-1)) pitch) / 2 on z = 0 (origin at the array centre).
 *     Pixel (k, m) sits at x_k = x0 + k dx, z_m = z0 + m dz.  Sample n of a record is time
 *     t0 + n / fs; t = 0 is when the transmitted wavefront crosses the origin.
 *   - All buffers are owned by the caller.  "dev" pointers are device memory on the current
 *     HIP device, "host" pointers are host memory.  The library allocates no device memory,
 *     keeps no global state and is re-entrant.
 *   - Host entry points are synchronous.  Device entry points validate their arguments on
 *     the host, enqueue work on `stream` (a hipStream_t; NULL = the default stream) and
 *     return without synchronising; faults surface at the caller's next synchronisation.
 *   - Every entry point returns a kk_status; on error nothing is written to outputs unless
 *     stated (capacity errors write the required size).
 */
#ifndef KK_H
#define KK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Acquisition geometry: L elements of pitch pitch_m, T samples per record at fs_hz, sound
 * speed c_mps, time of sample 0 t0_s. */
typedef struct kk_geom {
    int32_t L;
    int32_t T;
    double pitch_m;
    double c_mps;
    double fs_hz;
    double t0_s;
} kk_geom;

/* Image grid: X lateral by Z axial pixels, x_k = x0_m + k dx_m, z_m = z0_m + m dz_m. */
typedef struct kk_grid {
    int32_t X;
    int32_t Z;
    double x0_m;
    double dx_m;
    double z0_m;
    double dz_m;
} kk_grid;

typedef enum kk_status {
    KK_OK = 0,
    KK_E_NULL = -1,        /* a required pointer is NULL                                  */
    KK_E_ARG = -2,         /* an argument is out of its documented range                  */
    KK_E_CAPACITY = -3,    /* an output array is too small; required size written back    */
    KK_E_WORKSPACE = -4,   /* workspace or plan buffer too small or not a valid plan      */
    KK_E_RANGE = -5,       /* a delay does not fit the int32 fixed-point tables           */
    KK_E_HIP = -6,         /* a HIP runtime call or kernel launch failed                  */
    KK_E_UNSUPPORTED = -7  /* valid request the library does not implement               */
} kk_status;

/* Receive-angle selection schemes (Sec. II-C, II-D). */
typedef enum kk_scheme {
    KK_SCHEME_SHIFTED = 0,      /* Eq. 6: one set per j in j_list, j in [0, floor(N/2)]      */
    KK_SCHEME_CONFOCAL = 1,     /* Eq. 7: one set                                            */
    KK_SCHEME_SAME = 2,         /* receive angles = transmit angles (redundant control)      */
    KK_SCHEME_FULL_UNIFORM = 3  /* M angles uniform over +-(theta_max + dth_i): dense bank   */
} kk_scheme;

typedef enum kk_precision {
    KK_PREC_FP32 = 0,           /* FP32 transforms and contraction (the parity path)         */
    KK_PREC_BF16X3 = 1,         /* contraction on BF16 MFMA, split hi+lo, 3 products, FP32   */
                                /* accumulate (terms exact to ~2^-16)                        */
    KK_PREC_FP16X3 = 2          /* same on FP16 MFMA with an exact power-of-two prescale     */
                                /* (terms exact to ~2^-22)                                   */
} kk_precision;

typedef enum kk_compound_mode {
    KK_COMPOUND_COHERENT = 0,   /* Eq. 8: I = |sum_s B_s|^2                                   */
    KK_COMPOUND_INCOHERENT = 1  /* Eq. 9: I = sum_s |B_s|^2                                   */
} kk_compound_mode;

/* ---------------------------------------------------------------------------------------
 * kk_select_pairs (host) - transmit angles, distinct receive angles and the pair list.
 *
 * Sec. II-B: theta_i = ((2i - (N-1)) theta_max) / (N-1), dth_i = 2 theta_max / (N-1).
 * Eq. 6: theta_o = sgn(o) dth_i (2|o|/M + j), o = -floor(M/2)..floor(M/2), one set per j.
 * Eq. 7: theta_o = sgn(o) dth_i (2|o|/M + mod(|o|, floor(N/2))), one set.
 * Angles are exact rationals theta_o / dth_i = rx_num / rx_den (lowest terms, den > 0);
 * FP64 values are (n dth_i) / M with n = sgn(o)(2|o| + j M) (Eq. 7 analogue).  Distinct
 * receive angles are de-duplicated on the rationals and sorted ascending.  Pairs are
 * (i, o, s) triples, ordered by set s, then receive index o, then transmit index i; an
 * angle shared by several sets gets one slot per set.  compression = L / (J * M_set)
 * (Sec. II-C), M_set = receive angles per set (2 floor(M/2) + 1 for Eq. 6/7).
 *
 *   scheme      kk_scheme
 *   L, N        elements (>= 1), transmit angles (>= 2)
 *   theta_max   half range of the transmit fan, (0, pi/2)
 *   M           Eq. 6/7: per-set parameter (>= 1); SAME: ignored; FULL_UNIFORM: bank size (>= 2)
 *   j_list, J   Eq. 6 shifts (J >= 1 entries); ignored otherwise (may be NULL)
 *   tx_theta    host out [N]
 *   rx_theta, rx_num, rx_den   host out [cap_rx]; *M_out = number of distinct angles
 *   pairs       host out [cap_p][3] = {i, o, s}; *P_out = number of pair slots
 *   S_out       number of sets;  compression  as above
 * Errors: KK_E_NULL, KK_E_ARG (bad scheme/N/M/j/theta_max, any angle reaching 90 deg),
 * KK_E_CAPACITY (cap_rx or cap_p too small; *M_out and *P_out hold the required sizes).
 * ------------------------------------------------------------------------------------- */
int32_t kk_select_pairs(int32_t scheme, int32_t L, int32_t N, double theta_max, int32_t M,
                        const int32_t* j_list, int32_t J,
                        double* tx_theta,
                        double* rx_theta, int32_t* rx_num, int32_t* rx_den, int32_t cap_rx,
                        int32_t* M_out,
                        int32_t* pairs, int32_t cap_p, int32_t* P_out,
                        int32_t* S_out, double* compression);

/* ---------------------------------------------------------------------------------------
 * kk_build_luts (host) - separable Q16.16 delay tables (Sec. II-F) and the Q.22 shear
 * table of Eq. 3.  Values in samples; FP64, no contraction; rint = round half to even:
 *   lut1[i][k] = rint(((x_k sin th_i) / c) fs 65536)            [N][X]
 *   lut2[i][m] = rint(((z_m cos th_i) / c) fs 65536)            [N][Z]
 *   lut3[o][k] = rint(((-(x_k - x_ref) sin th_o) / c) fs 65536) [M][X]
 *   lut4[o][m] = rint(((z_m cos th_o) / c) fs 65536)            [M][Z]
 *   t0_q      = rint((-t0) fs 65536)
 *   shift_q[o][l] = rint(((d_l sin th_o) / c) fs 2^22)         [M][L]
 * x_ref = u_0 for th_o >= 0, u_{L-1} for th_o < 0; d_l = u_l - u_0 (th_o > 0),
 * u_l - u_{L-1} (th_o < 0), 0 (th_o = 0).  Eq. 3 advances element l by d_l sin(th_o)/c;
 * by stationary phase a scatterer at (x, z) then appears at
 * tau_in + [z cos th_o - (x - x_ref) sin th_o] / c, which lut3 + lut4 encode (Eq. 5's
 * s_o.r/c with th_o mirrored and the origin at the reference edge).
 * *tpad = smallest power of two >= T + ceil(max shift_q / 2^22): the FFT length of Eq. 3's
 * Fourier-shift evaluation (all advanced reads past the record then see zero padding).
 * Any output pointer may be NULL to skip it.  Errors: KK_E_NULL (g, grid, angles),
 * KK_E_ARG (non-positive sizes, c, fs, pitch, dx, dz), KK_E_RANGE (an entry or a composite
 * delay lut1+lut2+lut3+lut4+t0_q outside int32).
 * ------------------------------------------------------------------------------------- */
int32_t kk_build_luts(const kk_geom* g, const kk_grid* grid,
                      const double* tx_theta, int32_t N, const double* rx_theta, int32_t M,
                      int32_t* lut1, int32_t* lut2, int32_t* lut3, int32_t* lut4,
                      int32_t* t0_q, int32_t* shift_q, int32_t* tpad);

/* kk_build_das_rx (host) - DAS receive delays of Eq. 4 (Sec. II-F's third table):
 *   das_rx[k][l][m] = rint((sqrt(dx dx + z_m z_m) / c) fs 65536),  dx = x_k - u_l   [X][L][Z]
 * Errors: KK_E_NULL, KK_E_ARG, KK_E_RANGE. */
int32_t kk_build_das_rx(const kk_geom* g, const kk_grid* grid, int32_t* das_rx);

/* ---------------------------------------------------------------------------------------
 * kk_beamform_plan (host) - per-geometry beamforming plan for kk_beamform.
 *
 * Folds the four tables per pair, A[p][x] = lut1[i][x] + lut3[o][x] + t0_q and
 * B[p][z] = lut2[i][z] + lut4[o][z] (exact integer adds: the composite Q16.16 delay of
 * Eq. 5 is A[p][x] + B[p][z]), groups the pairs by set and records, for every pair and
 * pixel tile, the exact span of record samples the tile reads.  The plan is an opaque
 * byte buffer; copy it to device memory unchanged and pass it to kk_beamform.
 *   pairs [P][3] = {i, o, s} host, 0 <= i < N, 0 <= o < M, 0 <= s < S, every set non-empty
 *   lut1..lut4, t0_q  host tables from kk_build_luts
 *   T           samples per RF_theta record
 *   plan        host out, plan_bytes long; *plan_bytes_out = required size (always written)
 * Errors: KK_E_NULL, KK_E_ARG (sizes, pair entries), KK_E_RANGE (composite delay outside
 * int32), KK_E_CAPACITY (plan_bytes too small, required size in *plan_bytes_out),
 * KK_E_UNSUPPORTED (a tile would need more record samples than fit the on-chip window).
 * Passing plan = NULL with plan_bytes = 0 queries the size (returns KK_E_CAPACITY).
 * ------------------------------------------------------------------------------------- */
int32_t kk_beamform_plan(const int32_t* pairs, int32_t P, int32_t S, int32_t N, int32_t M,
                         int32_t T,
                         const int32_t* lut1, const int32_t* lut2, const int32_t* lut3,
                         const int32_t* lut4, int32_t t0_q, const kk_grid* grid,
                         void* plan, size_t plan_bytes, size_t* plan_bytes_out);

/* ---------------------------------------------------------------------------------------
 * kk_decompose (device) - Eq. 3 receive plane-wave decomposition, evaluated as Sec. II-F
 * describes: analytic (Hilbert) spectrum of each zero-padded record (mask: DC x1,
 * bins 1..tpad/2-1 x2, Nyquist x1, negative bins 0), per temporal-frequency bin k the
 * complex contraction
 *   Y[i][o][k] = sum_l A[i][l][k] exp(2 pi i ((k shift_q[o][l]) mod (tpad 2^22)) / (tpad 2^22))
 * (Fourier shift theorem), and the inverse transform
 *   rf_theta[i][o][n] = (1/tpad) sum_{k <= tpad/2} Y[i][o][k] exp(+2 pi i k n / tpad), n < T.
 *   rf        dev in  int16 [N][L][T]
 *   shift_q   dev in  int32 [M][L] (kk_build_luts)
 *   tpad      FFT length from kk_build_luts (a power of two)
 *   precision KK_PREC_FP32 (the parity path), or KK_PREC_BF16X3 / KK_PREC_FP16X3: the
 *             contraction on 16-bit MFMA with hi+lo split operands (W X ~ Wh Xh + Wh Xl +
 *             Wl Xh, FP32 accumulate); transforms stay FP32.  Each term is exact to about
 *             2^-16 (BF16) or 2^-22 (FP16) of its size; FP16 inputs are scaled by an exact
 *             power of two chosen from T so that no value exceeds 2^15.
 *   rf_theta  dev out complex float [N][M][T]
 *   ws        dev workspace of at least kk_decompose_workspace_bytes() bytes
 * Limits: 1 <= N, 1 <= M, 1 <= L <= 65536, 1 <= T <= tpad, tpad in {256, ..., 8192}.
 * Errors: KK_E_NULL, KK_E_ARG, KK_E_WORKSPACE, KK_E_UNSUPPORTED (precision), KK_E_HIP.
 * ------------------------------------------------------------------------------------- */
size_t kk_decompose_workspace_bytes(const kk_geom* g, int32_t N, int32_t M, int32_t tpad,
                                    int32_t precision);
int32_t kk_decompose(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q,
                     int32_t M, int32_t tpad, int32_t precision, float* rf_theta,
                     void* ws, size_t ws_bytes, void* stream);

/* kk_decompose_prepare (device) - the geometry-dependent part of kk_decompose (Eq. 3, Sec.
 * II-F): the contraction's phase tables, the phase of the first bin of every 8-bin block and the
 * steps to the other bins (each from an exact integer turn count of shift_q, evaluated in FP64
 * and rounded once), written into ws.  They depend only on g, N, M, tpad and the contents of
 * shift_q, like a beamforming plan: a workspace prepared once serves any number of
 * kk_decompose_prepared calls with those same arguments.
 * Errors: as kk_decompose.
 * kk_decompose_prepared (device) - kk_decompose on a workspace that kk_decompose_prepare has
 * prepared for the same g, N, M, tpad and shift table (the caller guarantees it; other inputs
 * give wrong results, not errors): the same arguments and results, bit for bit, without
 * rewriting the tables.  kk_decompose writes them in every call and may use any workspace. */
int32_t kk_decompose_prepare(const kk_geom* g, int32_t N, const int32_t* shift_q, int32_t M,
                             int32_t tpad, int32_t precision, void* ws, size_t ws_bytes,
                             void* stream);
int32_t kk_decompose_prepared(const int16_t* rf, int32_t N, const kk_geom* g,
                              const int32_t* shift_q, int32_t M, int32_t tpad, int32_t precision,
                              float* rf_theta, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * kk_beamform (device) - Eq. 5 per set:
 *   image[s][k][m] = sum_{p in set s} v_p,  q = A[p][k] + B[p][m] (Q16.16 samples),
 *   idx = floor(q / 65536), w = (q mod 65536) / 65536,
 *   v_p = (1 - w) R_p[idx] + w R_p[idx + 1],  R_p = rf_theta[i_p][o_p], zero outside [0, T).
 *   rf_theta  dev in complex float [N][M][T]
 *   plan      dev copy of a kk_beamform_plan buffer for the same N, M, T
 *   image     dev out complex float [S][X][Z]
 *   intensity dev out float [X][Z] or NULL: Eq. 8 (mode COHERENT) or Eq. 9 (INCOHERENT)
 *             of the S images, written in the same call
 *   ws        dev workspace of kk_beamform_workspace_bytes(plan) bytes (0 and NULL allowed
 *             when that is 0): partial images when the plan shares a tile's pairs among
 *             several workgroups (few tiles x sets); they are summed in a fixed order, so
 *             results are deterministic
 * Errors: KK_E_NULL, KK_E_ARG (N, M, T differ from the plan's), KK_E_WORKSPACE (plan header
 * invalid, workspace too small), KK_E_HIP.  The plan header is read from host memory: pass
 * its host copy too.
 * ------------------------------------------------------------------------------------- */
size_t kk_beamform_workspace_bytes(const void* plan_host, size_t plan_bytes);
int32_t kk_beamform(const float* rf_theta, int32_t N, int32_t M, int32_t T,
                    const void* plan_host, const void* plan_dev, size_t plan_bytes,
                    float* image, float* intensity, int32_t mode,
                    void* ws, size_t ws_bytes, void* stream);

/* kk_compound (device) - Eq. 8 / Eq. 9 of S per-set images image [S][X][Z] (complex)
 * into intensity [X][Z] (float).  Errors: KK_E_NULL, KK_E_ARG, KK_E_HIP. */
int32_t kk_compound(const float* image, int32_t S, int32_t X, int32_t Z, int32_t mode,
                    float* intensity, void* stream);

/* ---------------------------------------------------------------------------------------
 * das_plan (host) - per-geometry plan for das_beamform (Eq. 4): folded transmit delays
 * A[i][x] = lut1[i][x] + t0_q, B[i][z] = lut2[i][z], the receive table das_rx re-laid out
 * for coalesced reads, and per (transmit, element, tile) the exact record span.
 *   lut1 [N][X], lut2 [N][Z], das_rx [X][L][Z] host (kk_build_luts / kk_build_das_rx)
 * Same buffer protocol and errors as kk_beamform_plan.
 * ------------------------------------------------------------------------------------- */
int32_t das_plan(int32_t N, const kk_geom* g, const int32_t* lut1, const int32_t* lut2,
                 const int32_t* das_rx, int32_t t0_q, const kk_grid* grid,
                 void* plan, size_t plan_bytes, size_t* plan_bytes_out);

/* das_beamform (device) - conventional CPWC delay-and-sum, Eq. 4, on the analytic channel
 * data (FFT length tpad_das = smallest power of two >= T, same mask as kk_decompose):
 *   image[k][m] = sum_{i, l} lerp(RFa[i][l], A[i][k] + B[i][m] + das_rx[k][l][m])
 *   rf        dev in int16 [N][L][T]
 *   plan      host and dev copies of a das_plan buffer
 *   image     dev out complex float [X][Z]
 *   ws        dev workspace of at least das_workspace_bytes(g, N, plan) bytes (analytic
 *             spectra, analytic channel data, partial images of a split plan)
 * Errors: KK_E_NULL, KK_E_ARG, KK_E_WORKSPACE, KK_E_HIP. */
size_t das_workspace_bytes(const kk_geom* g, int32_t N, const void* plan_host, size_t plan_bytes);
int32_t das_beamform(const int16_t* rf, int32_t N, const kk_geom* g,
                     const void* plan_host, const void* plan_dev, size_t plan_bytes,
                     float* image, void* ws, size_t ws_bytes, void* stream);

/* =======================================================================================
 * Frame ensembles: many KK frames of uneven shapes (element counts, transmit and receive
 * angle sets, record lengths, grids) imaged as one unit of work.
 *
 * Every frame goes through the steps of kk_decompose and kk_beamform (Eq. 3, Eq. 5, and
 * Eq. 8 / Eq. 9 when an intensity is asked for), but each step runs as one launch over all
 * frames of a shape class instead of one launch per frame: the forward transforms,
 * contractions and inverse transforms per FFT length, and the delay-gather as one persistent
 * work-queue launch per window class over every (frame, set, pair share, pixel tile) unit.
 * Results equal the per-frame entry points' for the same precision and pair split.
 *
 * Buffers: the channel data of all frames is one packed int16 array, the images one packed
 * complex array and the intensities one packed float array; kk_ensemble_frame_query gives
 * each frame's offsets.  The workspace holds RF_theta of every frame (all at once), the pair
 * shares of split frames, the queue counters, and the spectra of one decomposition group:
 * frames are decomposed in groups whose spectra fit the budget given to kk_ensemble_plan.
 * ===================================================================================== */

typedef struct kk_ensemble_frame {
    kk_geom geom;              /* this frame's acquisition (L, T, pitch, c, fs, t0)            */
    int32_t N;                 /* transmit angles                                              */
    int32_t M;                 /* distinct receive angles                                      */
    int32_t tpad;              /* FFT length (kk_build_luts)                                   */
    int32_t mode;              /* intensity: KK_COMPOUND_COHERENT or _INCOHERENT, -1 for none  */
    const int32_t* shift_q;    /* host [M][L] shear table (kk_build_luts)                      */
    const void* plan;          /* host kk_beamform_plan buffer for this (N, M, T) and grid     */
    size_t plan_bytes;
} kk_ensemble_frame;

#define KK_ENSEMBLE_CLASSES 8  /* window classes: 64, 128, ..., 512 record samples per tile */

/* Launch-shape choices of an ensemble (what kk_ensemble_autotune searches). */
typedef struct kk_ensemble_tuning {
    int32_t pair_tile[KK_ENSEMBLE_CLASSES]; /* per window class: pairs per gather work unit
                                               (a set is split into ceil(set / pair_tile)
                                               shares, at most 8); 0 = whole sets        */
    int32_t queue;             /* 0: one work list, units in descending cost order;
                                  1: one list per XCD, frames in order, equal cost per list,
                                     drained lists take the others' remaining units      */
    int32_t reserved[7];       /* zero                                                   */
} kk_ensemble_tuning;

typedef struct kk_ensemble_frame_info {
    int64_t rf_offset;         /* int16 elements into the packed channel data: [N][L][T]       */
    int64_t image_offset;      /* complex elements into the packed images: [S][X][Z]           */
    int64_t intensity_offset;  /* float elements into the packed intensities: [X][Z]; -1: none */
    int64_t rf_theta_offset;   /* complex elements into the workspace: RF_theta [N][M][T]      */
    int64_t share_offset;      /* complex elements into the workspace: shares [K][S][X][Z], -1 */
    int32_t N, L, T, M, S, X, Z, P, tpad;
    int32_t cap;               /* window class (record samples per pair and tile)              */
    int32_t split;             /* pair shares per set (K)                                      */
    int32_t group;             /* decomposition group                                          */
    int32_t mode;
    int32_t plan_offset;       /* int32 words into the ensemble plan: this frame's plan copy    */
    int32_t shift_offset;      /* int32 words into the ensemble plan: its shear table          */
    int32_t reserved;
} kk_ensemble_frame_info;

typedef struct kk_ensemble_sizes {
    int64_t rf_elems;          /* packed channel data length (int16 elements)                  */
    int64_t image_elems;       /* packed images length (complex elements)                      */
    int64_t intensity_elems;   /* packed intensities length (float elements)                   */
    int64_t ws_bytes;          /* workspace                                                    */
    int64_t units_offset;      /* workspace byte offset of the per-workgroup unit counts:
                                  int32 [KK_ENSEMBLE_CLASSES][1024], row = window class index  */
    int32_t nframes, ngroups, nlaunches, nunits;  /* frames, decomposition groups, kernel
                                  launches of a full run, gather work units                    */
    int32_t precision;
    int32_t reserved[3];
} kk_ensemble_sizes;

/* Stages of kk_ensemble_run (bit mask). */
enum {
    KK_STAGE_FFT = 1,          /* analytic spectra                                             */
    KK_STAGE_CONTRACT = 2,     /* Eq. 3 per-bin contraction                                    */
    KK_STAGE_INVERSE = 4,      /* inverse transforms -> RF_theta                               */
    KK_STAGE_GATHER = 8,       /* Eq. 5 delay-gather                                           */
    KK_STAGE_REDUCE = 16,      /* pair-share sums and Eq. 8 / 9 intensities                    */
    KK_STAGE_ALL = 31
};

/* kk_ensemble_default_tuning (host): whole sets, per-XCD lists. */
void kk_ensemble_default_tuning(kk_ensemble_tuning* tuning);

/* kk_ensemble_plan (host) - the ensemble plan: frame offsets, the copied per-frame plans and
 * shear tables, the work tables of every grouped launch and the gather work lists.  Opaque
 * bytes; copy to device memory unchanged.
 *   frames, nframes   frame descriptions (nframes >= 1); their plans must be KK plans
 *   precision         KK_PREC_* for every contraction of the ensemble
 *   tuning            launch shapes (NULL: kk_ensemble_default_tuning)
 *   spectra_budget    bytes of workspace the decomposition spectra of one group may use;
 *                     0 = all frames in one group.  A frame larger than the budget forms a
 *                     group of its own.
 *   plan, plan_bytes  host out; *plan_bytes_out = required size (always written)
 * Errors: KK_E_NULL, KK_E_ARG (a frame's sizes, mode or plan disagree), KK_E_WORKSPACE (a
 * frame's plan is not a valid KK plan), KK_E_UNSUPPORTED (precision), KK_E_CAPACITY (plan
 * too small; plan = NULL with plan_bytes = 0 queries the size). */
int32_t kk_ensemble_plan(const kk_ensemble_frame* frames, int32_t nframes, int32_t precision,
                         const kk_ensemble_tuning* tuning, int64_t spectra_budget,
                         void* plan, size_t plan_bytes, size_t* plan_bytes_out);

/* kk_ensemble_query / kk_ensemble_frame_query (host) - sizes of the packed buffers and the
 * workspace, and frame f's offsets and shapes.  Errors: KK_E_NULL, KK_E_WORKSPACE (not an
 * ensemble plan), KK_E_ARG (f out of range). */
int32_t kk_ensemble_query(const void* plan_host, size_t plan_bytes, kk_ensemble_sizes* sizes);
int32_t kk_ensemble_frame_query(const void* plan_host, size_t plan_bytes, int32_t f,
                                kk_ensemble_frame_info* info);

/* kk_ensemble_run (device) - enqueue the selected stages of the whole ensemble on stream
 * (KK_STAGE_ALL for a complete run; a stage reads what the previous stages last wrote).
 *   plan_host, plan_dev  host and device copies of a kk_ensemble_plan buffer
 *   rf          dev in  packed int16 channel data
 *   image       dev out packed complex images
 *   intensity   dev out packed intensities (NULL allowed when no frame asks for one)
 *   ws          dev workspace of kk_ensemble_sizes.ws_bytes bytes
 * The launch list is fixed by the plan, so the same call can be captured into a graph.
 * Errors: KK_E_NULL, KK_E_WORKSPACE (plan or workspace), KK_E_ARG (stages), KK_E_HIP. */
int32_t kk_ensemble_run(const void* plan_host, const void* plan_dev, size_t plan_bytes,
                        const int16_t* rf, float* image, float* intensity, void* ws,
                        size_t ws_bytes, int32_t stages, void* stream);

/* kk_ensemble_graph_create (host) - capture a complete kk_ensemble_run with these buffers on
 * `stream` (a created stream, not NULL) into an executable HIP graph; *graph_out receives an
 * opaque handle owned by the caller until kk_ensemble_graph_destroy.  The graph keeps the
 * device addresses: the buffers must stay allocated while it is used.
 * kk_ensemble_graph_launch enqueues one replay on `stream`.
 * Errors: KK_E_NULL, KK_E_ARG (NULL stream), the errors of kk_ensemble_run, KK_E_HIP. */
int32_t kk_ensemble_graph_create(const void* plan_host, const void* plan_dev, size_t plan_bytes,
                                 const int16_t* rf, float* image, float* intensity, void* ws,
                                 size_t ws_bytes, void* stream, void** graph_out);
int32_t kk_ensemble_graph_launch(void* graph, void* stream);
int32_t kk_ensemble_graph_destroy(void* graph);

/* kk_ensemble_autotune (host, synchronous) - measure launch shapes on the device and return
 * the fastest: the gather queue layout, then per window class present the pair tile (from
 * whole sets down to 32 pairs), each timed as the median of `reps` gather + reduce runs on
 * the caller's data after one full run.  Candidates whose plan or workspace exceeds
 * plan_dev_bytes / ws_bytes are skipped.  *tuning is the starting point and receives the
 * result; *best_us (may be NULL) the gather + reduce time of the result.
 * plan_dev (plan_dev_bytes) is device scratch for the candidate plans; it holds the last
 * candidate's plan on return.  Errors: as kk_ensemble_plan and kk_ensemble_run. */
int32_t kk_ensemble_autotune(const kk_ensemble_frame* frames, int32_t nframes, int32_t precision,
                             int64_t spectra_budget, void* plan_dev, size_t plan_dev_bytes,
                             const int16_t* rf, float* image, float* intensity, void* ws,
                             size_t ws_bytes, int32_t reps, void* stream,
                             kk_ensemble_tuning* tuning, float* best_us);

/* =======================================================================================
 * Spectra: the decomposition stopped before its inverse transform, and the inverse alone.
 * ===================================================================================== */

/* kk_spectrum_bins (host) - bins per record of a spectrum for FFT length tpad:
 * kpad = tpad/2 + 1 rounded up to a multiple of 8; 0 if tpad is not a supported length. */
int32_t kk_spectrum_bins(int32_t tpad);

/* kk_decompose_spectrum (device) - the per-bin contraction of kk_decompose (Eq. 3 via the
 * Fourier shift, analytic mask as there), without the inverse transform:
 *   spec[i][o][k] = sum_l A[i][l][k] exp(2 pi i ((k shift_q[o][l]) mod (tpad 2^22)) / (tpad 2^22))
 * for k < tpad/2; bins tpad/2 .. kpad-1 are set to zero.
 *   spec   dev out complex float [N][M][kpad], kpad = kk_spectrum_bins(tpad)
 *   ws     dev workspace of at least kk_decompose_workspace_bytes(g, N, M, tpad, precision)
 * Other arguments, limits and errors as kk_decompose. */
int32_t kk_decompose_spectrum(const int16_t* rf, int32_t N, const kk_geom* g, const int32_t* shift_q,
                              int32_t M, int32_t tpad, int32_t precision, float* spec, void* ws,
                              size_t ws_bytes, void* stream);

/* kk_spectrum_inverse (device) - rf_theta[t][n] = (1/tpad) sum_{k <= tpad/2} spec[t][k]
 * exp(+2 pi i k n / tpad), n < T, for ntraces records of kpad bins (the inverse transform of
 * kk_decompose; bin tpad/2 taken from spec).
 *   spec dev in complex float [ntraces][kpad];  rf_theta dev out complex float [ntraces][T]
 * Errors: KK_E_NULL, KK_E_ARG (sizes, tpad not a supported length, T > tpad), KK_E_HIP. */
int32_t kk_spectrum_inverse(const float* spec, int32_t ntraces, int32_t tpad, int32_t T,
                            float* rf_theta, void* stream);

/* =======================================================================================
 * Learned k-space completion (a network on the per-bin pair grid).
 *
 * One bin k of a decomposition spectrum over a uniform receive bank is a complex grid of
 * H transmit angles x W receive angles; every (theta_i, theta_o) pair is one k-space sample
 * (Sec. II-B).  A compressive acquisition observes J of the W receive columns.  The network
 * (KK_NET_LAYERS 3x3 convolutions, KK_NET_WIDTH channels, ReLU between them; BF16 weights
 * and activations, FP32 accumulation on MFMA, FP32 master parameters and Adam moments)
 * maps the observed grid to the full grid:
 *   grid  [B][H][W][KK_NET_IN] BF16: c0, c1 = Re, Im of the observed pairs / scale (0 where
 *         unobserved), c2 = 1 where observed, c3..7 = 0; scale = RMS of the observed pairs
 *   out   [B][H][W][2] FP32: the predicted grid / scale
 * and the completed spectrum keeps every observed pair and takes out * scale elsewhere.
 * Training minimises the mean squared error over unobserved pairs (Adam).
 * Parameters (FP32, kk_net_param_count of them): per layer l the weights W[9][32][cin]
 * (tap t = 3 (dy+1) + (dx+1), output channel, input channel; cin = KK_NET_IN for l = 0,
 * KK_NET_WIDTH after) then the bias [32]; the last layer's output channels 2..31 must be zero.
 * Layer l reads its input at (h + dy eh_l, w + dx ew_l): `dilation` is a host array
 * [KK_NET_LAYERS][2] = (eh_l, ew_l), 1..64, or NULL for all 1.
 * Limits: 16 <= W <= 192 with W a multiple of 16; H >= 1; B >= 1.
 * ===================================================================================== */
#define KK_NET_LAYERS 6
#define KK_NET_WIDTH 32
#define KK_NET_IN 8

enum { KK_NET_PARAMS = 0, KK_NET_GRADS = 1, KK_NET_MOMENT1 = 2, KK_NET_MOMENT2 = 3 };

/* Sizes: parameters, the device state (parameters, gradient, moments, BF16 weights), and the
 * workspace of a batch of B grids of H x W (0 if the shape is not supported). */
size_t kk_net_param_count(void);
size_t kk_net_state_bytes(void);
size_t kk_net_workspace_bytes(int32_t B, int32_t H, int32_t W);

/* kk_net_load (host, synchronous) - parameters from host memory into the device state; Adam
 * moments and gradient zeroed; BF16 weights built.  kk_net_read (host, synchronous) - copy
 * the parameters, gradient or moments (KK_NET_*) back.  Errors: KK_E_NULL, KK_E_ARG, KK_E_HIP. */
int32_t kk_net_load(void* state, const float* params_host, void* stream);
int32_t kk_net_read(const void* state, int32_t what, float* host, void* stream);

/* kk_net_prepare (device) - input grids (and training targets) of B bins of a spectrum
 * spec [H][Msrc][kpad]: sample b is bin bins[b] (dev, or k_first + b when bins is NULL); grid
 * column w is observed when grid_to_obs[w] = j >= 0, with the value spec[h][obs_src[j]][k];
 * target (dev [B][H][W][2] or NULL; needs Msrc == W) = spec[h][w][k] / scale; scale dev [B].
 * obs_src [J], grid_to_obs [W]: dev int32.  Errors: KK_E_NULL, KK_E_ARG, KK_E_HIP. */
int32_t kk_net_prepare(const float* spec, int32_t H, int32_t Msrc, int32_t kpad, const int32_t* bins,
                       int32_t k_first, int32_t B, const int32_t* obs_src, int32_t J,
                       const int32_t* grid_to_obs, int32_t W, uint16_t* grid, float* target,
                       float* scale, void* stream);

/* kk_net_forward (device) - out = network(grid); batch row b reads grid sample sidx[b] (dev,
 * or b when sidx is NULL).  ws: kk_net_workspace_bytes(B, H, W).  dilation as above.
 * Errors: KK_E_NULL, KK_E_ARG (shape), KK_E_WORKSPACE, KK_E_HIP. */
int32_t kk_net_forward(const void* state, const uint16_t* grid, const int32_t* sidx, int32_t B,
                       int32_t H, int32_t W, const int32_t* dilation, float* out, void* ws,
                       size_t ws_bytes, void* stream);

/* kk_net_backward (device) - forward pass, loss and parameter gradient of a batch:
 *   loss (dev float) = inv_count * sum over unobserved pairs of |out - target|^2
 * (inv_count = 1 / (2 x unobserved pairs in the batch)); target dev [*][H][W][2] indexed like
 * grid.  The gradient stays in the state (kk_net_read KK_NET_GRADS).  kk_net_adam (device) -
 * one Adam update (b1 0.9, b2 0.999, eps 1e-8, step >= 1) from that gradient, then the BF16
 * weights.  kk_net_train_step = kk_net_backward + kk_net_adam.
 * Errors: KK_E_NULL, KK_E_ARG, KK_E_WORKSPACE, KK_E_HIP. */
int32_t kk_net_backward(void* state, const uint16_t* grid, const float* target, const int32_t* sidx,
                        int32_t B, int32_t H, int32_t W, const int32_t* dilation, float inv_count,
                        float* loss, void* ws, size_t ws_bytes, void* stream);
int32_t kk_net_adam(void* state, int32_t step, float lr, void* stream);
int32_t kk_net_train_step(void* state, const uint16_t* grid, const float* target, const int32_t* sidx,
                          int32_t B, int32_t H, int32_t W, const int32_t* dilation, float inv_count,
                          int32_t step, float lr, float* loss, void* ws, size_t ws_bytes, void* stream);

/* kk_net_merge (device) - completed spectrum of B bins: dst[h][w][k] = spec[h][obs_src[j]][k]
 * where column w is observed (j = grid_to_obs[w] >= 0), else out[b][h][w] * scale[b]; dst dev
 * complex float [H][W][kpad] (other bins untouched).  Errors: KK_E_NULL, KK_E_ARG, KK_E_HIP. */
int32_t kk_net_merge(const float* out, const float* scale, const int32_t* bins, int32_t k_first,
                     int32_t B, const float* spec, int32_t H, int32_t Msrc, int32_t kpad,
                     const int32_t* obs_src, const int32_t* grid_to_obs, int32_t W, float* dst,
                     void* stream);

/* kk_clear (device) - zero `bytes` bytes at dev (16-byte aligned, a multiple of 16), by a
 * kernel (so that it may be captured into a graph).  Errors: KK_E_NULL, KK_E_ARG, KK_E_HIP. */
int32_t kk_clear(void* dev, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * kk_beamform_static (device) - kk_beamform without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as kk_beamform minus ws: the
 * partial images of a split plan sit in a fixed device array inside the library, one copy per
 * GPU of kk_beamform_static_max_bytes() bytes (16 MiB), held until the process ends.
 * The call allocates nothing.  Errors: as kk_beamform; KK_E_WORKSPACE also when the plan needs
 * more than kk_beamform_static_max_bytes() (kk_beamform_workspace_bytes(plan) tells), KK_E_HIP
 * when the array's address cannot be obtained.  Every call on one GPU uses that GPU's array:
 * calls that overlap in time on one GPU (several streams or threads) race and must not be
 * issued; calls in one stream are ordered and safe.
 * ------------------------------------------------------------------------------------- */
size_t kk_beamform_static_max_bytes(void);
int32_t kk_beamform_static(const float* rf_theta, int32_t N, int32_t M, int32_t T,
                           const void* plan_host, const void* plan_dev, size_t plan_bytes,
                           float* image, float* intensity, int32_t mode, void* stream);

/* Human-readable name of a kk_status value (static string, never NULL). */
const char* kk_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* KK_H */
