#!/usr/bin/env python3
"""Benchmark of the KK beamforming hot path on one MI355X.

Workload (the plain-KK-vs-DAS configuration): 128-element linear array, pitch 0.3 mm,
5 MHz pulse sampled at 20 MHz, 2048 int16 samples per record, 31 plane-wave transmits in
+-15 deg; two shifted-vernier receive sets (Eq. 6, j = 0 and 15, M = 7: 13 distinct
receive angles, 434 pair slots, 9.14x compression); speckle phantom of 1e5 scatterers with
8 point targets and a 2 mm anechoic cyst (seeded, synthetic); 256 lateral x 512 axial
pixels at lambda/2.

One step = one KK frame from int16 channel data resident in HBM: decomposition (analytic
FFT, per-bin MFMA contraction, inverse FFT), gather beamforming of both sets and Eq. 9
compounding.  Selection, delay tables and plans are per-geometry setup, built before timing
(as the paper's Table II excludes them).  The K timed frames run with --streams frames in
flight (frame k on stream k mod F, each stream with its own outputs and workspace), so one
frame's small kernels overlap the next frame's; the one-stream frame time is reported beside it.
Printed: one JSON line.
  value            pixel*pair / s of the whole frame (X Z P / step time), in Gpixel*pair/s
  frames_per_s     KK frames per second;  das_frames_per_s  DAS (Eq. 4) on the same data
  roofline         the gather kernel (Eq. 5, the step the metric counts) against the VALU issue
                   bound; traffic from the committed PMC byte-counter summary when it matches
                   the kernel source, else null
  stage_rooflines  every stage of the frame against its own bound, from live stage timings
  graph            the same frame captured as one HIP graph: replays checked against the eager
                   frame, mean replay time and the p10 / median / p90 of single replays
  clocks           shader / memory clock levels the amdgpu kernel driver reports after the timed loop
  cpu_baseline     the FP64 oracle, unmodified, on a bounded sample on this host
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KK beamform Gpixel·pair/s and frames/s vs GPU DAS at rel-L2 ≤1e-5 (FP32)"
# VALU issue rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-operations per second,
# and the algorithmic lane-operations per pixel*pair of a delay-gather: one delay add, two for
# index and fraction, four for the complex interpolate-accumulate, one address operation.
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_PIXEL_PAIR = 8
# Eq. 4's receive delay is not separable in (x, z): one more add per pixel*(transmit, element)
DAS_OPS_PER_GATHER = 9
HBM_BYTES_PER_S = 8.0e12
MFMA_FP32_FLOPS = 157.3e12
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "gather_vernier_traffic.md")
GATHER_SOURCE = os.path.join(ROOT, "paper_2603_22496_amd", "csrc", "kk_beamform.hip")


def measured_gather_traffic():
    """HBM bytes per gather launch from the committed byte-counter summary, or None when the
    kernel source has changed since the counters were taken."""
    try:
        vals = {}
        for line in open(TRAFFIC_SUMMARY):
            if "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        src = hashlib.sha256(open(GATHER_SOURCE, "rb").read()).hexdigest()
        if vals.get("source_sha256") != src:
            return None
        return int(float(vals["gather_traffic_bytes"]))
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--streams", type=int, default=3, help="frames in flight on separate HIP streams in the timed loop")
    ap.add_argument("--settle-s", type=float, default=0.5, help="seconds of untimed frames before the warm-up steps")
    ap.add_argument("--cpu-frames", type=int, default=128,
                    help="whole oracle frames timed on the host's cores for cpu_baseline (0: skip)")
    ap.add_argument("--no-full-bank", action="store_true", help="skip the 128-angle bank frame report")
    ap.add_argument("--no-das", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle check of the timed frame")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the split-precision decomposition report on the large workload")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched frame-ensemble report")
    ap.add_argument("--ensemble-frames", type=int, default=200)
    ap.add_argument("--ensemble-steps", type=int, default=5, help="timed graph replays of the ensemble")
    ap.add_argument("--ensemble-density", type=float, default=0.05,
                    help="scatterers per lambda^2 of the ensemble medium (input generation cost only)")
    ap.add_argument("--ensemble-precision", choices=("fp32", "bf16x3", "fp16x3"), default="bf16x3",
                    help="decomposition arithmetic of the ensemble")
    ap.add_argument("--ensemble-budget-gb", type=float, default=4.0,
                    help="workspace for the decomposition spectra of one frame group")
    ap.add_argument("--no-completion", action="store_true", help="skip the k-space completion report")
    ap.add_argument("--completion-eval", type=int, default=8, help="evaluation phantoms of the completion report")
    ap.add_argument("--no-study", action="store_true", help="skip the scheme / compounding image-metric study")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (HBM byte-counter calibration)")
    return ap.parse_args()


def timed(fn, steps, warmup, torch, repeats=1):
    """ms per call; with repeats > 1 the best of that many timed loops (a stage's steady state:
    the first loop of back-to-back launches of one kernel in a process can run several times
    slower than every later one)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        best = ms if best is None else min(best, ms)
    return best


def graph_report(frame, img, inten, args, torch, np):
    """One frame (decomposition, gather, Eq. 9 intensity) captured as a HIP graph: outputs of
    three replays (eager work between them) against the eager frame, the mean frame time over
    args.steps back-to-back replays and the spread of 100 individually timed replays."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        frame()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref_img, ref_int = img.clone(), inten.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        frame()
    identical = True
    for _ in range(3):
        img.zero_()
        inten.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        identical &= bool(torch.equal(img, ref_img)) and bool(torch.equal(inten, ref_int))
        frame()                                   # eager work between replays
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    mean_us = e0.elapsed_time(e1) / args.steps * 1e3
    per = []
    for _ in range(100):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        b.synchronize()
        per.append(a.elapsed_time(b) * 1e3)
    del g
    p10, p50, p90 = np.percentile(per, [10, 50, 90])
    return {"identical_to_eager": identical, "frame_us_mean": round(mean_us, 2),
            "frame_us_p10": round(float(p10), 2), "frame_us_median": round(float(p50), 2),
            "frame_us_p90": round(float(p90), 2), "replays": args.steps}


# ---------------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, timed on this host before the GPU is touched (its
# worker processes are plain forks of a process that has not initialised the GPU).

_CPU = {}


def _oracle_vernier_frame(_):
    """One whole oracle frame (Eq. 3 decomposition, then the Eq. 5 gather of every set) in a
    forked worker; returns its seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import frame as OF
    with threadpool_limits(limits=1):
        t = time.time()
        OF.kk_image(_CPU["rf"], _CPU["sel"], _CPU["luts"], _CPU["X"], _CPU["Z"])
        return time.time() - t


def oracle_stages(ds, sel, luts, w, das_luts=None, das_stride=1):
    """Seconds per stage of one oracle frame in the paper's Table II columns (FFT, compress,
    IFFT, beamform; DAS when its tables are given), one thread.  DAS may be evaluated on every
    das_stride-th pixel only and scaled up (its time is linear in the pixel count)."""
    import numpy as np
    from oracle import beamform as OB
    from oracle.decompose import shear_phases
    from oracle.spectrum import analytic_signal, analytic_spectrum, inverse_bins
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t = time.time()
        A = analytic_spectrum(ds.rf, luts["tpad"])
        t_fft = time.time() - t
        shift = luts["shift"]
        Y = np.empty((A.shape[0], shift.shape[0], A.shape[2]), dtype=np.complex128)
        t = time.time()
        for o in range(shift.shape[0]):
            W = shear_phases(shift[o:o + 1], luts["tpad"])[0]
            Y[:, o, :] = (A * W[None, :, :]).sum(axis=1)
        t_contract = time.time() - t
        t = time.time()
        R = inverse_bins(Y, luts["tpad"], w.T)
        t_inverse = time.time() - t
        t = time.time()
        OB.kk_beamform(R, sel["pairs"], sel["S"], luts["lut1"], luts["lut2"], luts["lut3"], luts["lut4"],
                       luts["t0_q"], w.X, w.Z)
        t_gather = time.time() - t
        out = {"fft": t_fft, "compress": t_contract, "ifft": t_inverse, "beamform": t_gather}
        if das_luts is not None:
            tp = 1
            while tp < w.T:
                tp *= 2
            t = time.time()
            rfa = analytic_signal(ds.rf, tp)
            npix = w.X * w.Z
            flat = np.arange(0, npix, das_stride)
            OB.das_beamform(rfa, das_luts["lut1"], das_luts["lut2"], das_luts["rx"], das_luts["t0_q"], w.X, w.Z,
                            pixels=(flat // w.Z, flat % w.Z))
            out["das"] = (time.time() - t) * npix / len(flat)
    return out


def cpu_baseline(C, ds, w, frames, log):
    """The oracle's throughput on this host's cores (min(affinity, 16) forked workers, one frame
    each at a time, `frames` whole vernier frames), and per-stage single-thread times (median
    of 3) on the vernier and tiny workloads."""
    import multiprocessing as mp
    import numpy as np
    from oracle import frame as OF
    sel, luts = OF.tables(w)
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    _CPU.update(rf=ds.rf, sel=sel, luts=luts, X=w.X, Z=w.Z)
    t = time.time()
    with mp.get_context("fork").Pool(cores) as pool:
        per = pool.map(_oracle_vernier_frame, range(frames), chunksize=1)
    wall = time.time() - t
    pixpair = w.X * w.Z * len(sel["pairs"])
    log("cpu baseline: %d oracle frames on %d workers in %.2fs wall (%.2f s/frame in a worker)"
        % (frames, cores, wall, float(np.median(per))))
    das_luts = OF.das_tables(w)
    med = lambda runs: {k: round(float(np.median([r[k] for r in runs])), 4) for k in runs[0]}
    stages = med([oracle_stages(ds, sel, luts, w, das_luts, das_stride=64) for _ in range(3)])
    tw = C.TINY
    tds = C.tiny_dataset(0)
    tsel, tluts = OF.tables(tw)
    tiny = med([oracle_stages(tds, tsel, tluts, tw, OF.das_tables(tw)) for _ in range(3)])
    tiny_frame = sum(v for k, v in tiny.items() if k != "das")
    return {
        "value": round(frames * pixpair / wall / 1e9, 5),
        "unit": "Gpixel·pair/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d whole vernier KK frames (decomposition + gather of both sets, FP64 numpy oracle), one frame per "
                  "worker process at a time on %d forked workers: %.2f s wall = %.2f frames/s"
                  % (frames, cores, wall, frames / wall),
        "frames_per_s": round(frames / wall, 3),
        "single_thread_stages_s_median_of_3": {
            "vernier": stages, "vernier_das_note": "DAS on every 64th pixel, scaled to the whole grid",
            "tiny": tiny, "tiny_frame_s": round(tiny_frame, 4),
            "tiny_gpixel_pair_per_s": round(tw.X * tw.Z * len(tsel["pairs"]) / tiny_frame / 1e9, 5)},
        "affinity_cores": len(os.sched_getaffinity(0)),
        "cpu": cpu_model(),
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gpu_clocks():
    """Current shader and memory clock levels as the amdgpu driver's sysfs files mark them (None
    where they are unavailable).  Read as files: no helper program is started."""
    import glob
    found = {}
    for key, name in (("sclk", "pp_dpm_sclk"), ("mclk", "pp_dpm_mclk"), ("fclk", "pp_dpm_fclk")):
        for path in sorted(glob.glob("/sys/class/drm/card*/device/" + name)):
            try:
                with open(path) as f:
                    for line in f:
                        if line.rstrip().endswith("*"):
                            found.setdefault(key, line.split(":", 1)[-1].replace("*", "").strip())
            except OSError:
                continue
    return found or None


def precision_report(kk, C, torch, np, args):
    """Large workload (192 elements, 75 transmits, 4096 samples, Eq. 6 j = 0, 37, M = 9,
    384 x 768 pixels): the decomposition (phase tables prepared once) in FP32 and in the two
    split-precision forms, each timed, set against its unfused HBM bound, and compared with the
    FP64 oracle (sampled pixels of the beamformed sets) and with the FP32 run (whole image)."""
    import oracle as O
    from oracle import frame as OF
    w = C.LARGE
    ds = C.speckle_dataset(w, seed=3, n_scat=20_000)
    su = kk.make_setup(w, with_das=False)
    dev = torch.device("cuda", 0)
    rf, sh, pd = kk.to_device(ds.rf), kk.to_device(su.luts["shift"]), kk.to_device(su.plan)
    sel_o, luts_o = OF.tables(w)                       # the oracle's own selection and tables
    R64 = O.decompose(ds.rf, luts_o["shift"], luts_o["tpad"])
    rng = np.random.default_rng(1)
    xi, zi = rng.integers(0, w.X, 400), rng.integers(0, w.Z, 400)
    ref = OF.kk_image(None, sel_o, luts_o, w.X, w.Z, pixels=(xi, zi), rf_theta=R64)
    out = {"workload": "large: 192 el, 75 tx in +-18 deg, 4096 samples, Eq.6 j=0,37 M=9 (%d pairs), %dx%d px"
                       % (len(su.sel["pairs"]), w.X, w.Z)}
    img32 = None
    for name, prec in (("fp32", kk.PREC_FP32), ("bf16x3", kk.PREC_BF16X3), ("fp16x3", kk.PREC_FP16X3)):
        rt = torch.empty((w.N, su.M, w.T), dtype=torch.complex64, device=dev)
        ws = torch.empty(kk.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad, prec), dtype=torch.uint8,
                         device=dev)
        # the phase tables once per geometry, as in the vernier frames
        kk.decompose_prepare(su.geom, w.N, sh, su.M, su.tpad, ws, precision=prec)
        ms = timed(lambda: kk.decompose(rf, su.geom, sh, su.M, su.tpad, out=rt, ws=ws, precision=prec, prepared=True),
                   max(5, args.steps // 10), 2, torch)
        img = kk.beamform(rt, su.plan, pd)
        torch.cuda.synchronize()
        got = img.cpu().numpy()
        if img32 is None:
            img32 = got
        out[name] = {
            "decompose_us": round(ms * 1e3, 2),
            "frac_unfused_hbm": round(_decompose_bytes(w.N, w.L, w.T, su.M, su.tpad) / HBM_BYTES_PER_S / (ms * 1e-3), 4),
            "rel_l2_rf_theta_vs_fp64": float(np.linalg.norm(rt.cpu().numpy() - R64) / np.linalg.norm(R64)),
            "rel_l2_image_vs_fp64": float(np.linalg.norm(got[:, xi, zi] - ref) / np.linalg.norm(ref)),
            "rel_l2_image_vs_fp32": float(np.linalg.norm(got - img32) / np.linalg.norm(img32)),
        }
        print("bench: precision %s decompose %.2f us" % (name, ms * 1e3), file=sys.stderr, flush=True)
    return out


def _decompose_bytes(N, L, T, M, tpad):
    """Algorithmic HBM bytes of one unfused decomposition: int16 records in, analytic spectra
    out and in, sheared spectra out and in, RF_theta out."""
    K = tpad // 2 + 1
    return N * L * T * 2 + 2 * N * L * K * 8 + 2 * N * M * K * 8 + N * M * T * 8


def ensemble_report(kk, C, torch, np, args):
    """Batched form: an ensemble of uneven frames (64-192 elements, 15-75 transmits, 1-3 Eq. 6
    sets at 4-16x compression, grids 128 x 256 to 384 x 768) imaging one speckle medium whose
    scatterers move up to 50 um per frame; decomposition in --ensemble-precision (default BF16
    hi+lo: on MI355X 25.3 ms per replay against 27.0 ms in FP32 and 26.1 ms in FP16 hi+lo), FP32
    beamforming, Eq. 9 intensities.  Planned once, launch shapes autotuned on the device, then
    timed as graph replays (all frames per replay).  Compared with the same frames through the
    per-frame entry points on one stream and with three frames in flight on three streams (whose
    images must equal the ensemble's)."""
    dev = torch.device("cuda", 0)
    t0 = time.time()
    wls = C.ensemble_workloads(args.ensemble_frames, seed=4000)
    med = C.ensemble_medium(wls, seed=4001, per_lambda2=args.ensemble_density)
    sus = [kk.make_setup(w) for w in wls]
    inputs = [kk.setup_frame_input(su, kk.COMPOUND_INCOHERENT) for su in sus]
    prec = {"fp32": kk.PREC_FP32, "bf16x3": kk.PREC_BF16X3, "fp16x3": kk.PREC_FP16X3}[args.ensemble_precision]
    E = kk.Ensemble(inputs, precision=prec, spectra_budget=int(args.ensemble_budget_gb * (1 << 30)))
    t_plan = time.time() - t0
    t0 = time.time()
    for f, w in enumerate(wls):
        E.frame_rf(f).copy_(torch.from_numpy(C.ensemble_dataset(w, med, f).rf))
    torch.cuda.synchronize()
    t_sim = time.time() - t0
    print("bench: ensemble %d frames planned in %.1fs, simulated in %.1fs; %d groups, %d launches, %d units"
          % (len(wls), t_plan, t_sim, E.sizes.ngroups, E.sizes.nlaunches, E.sizes.nunits), file=sys.stderr,
          flush=True)
    stream = torch.cuda.Stream()

    def ev_time(fn, reps, warm=1):
        for _ in range(warm):
            fn()
        stream.synchronize()
        t = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            t.append(a.elapsed_time(b))
        return float(np.median(t))

    gather_stages = kk.STAGE_GATHER | kk.STAGE_REDUCE
    dec_stages = kk.STAGE_FFT | kk.STAGE_CONTRACT | kk.STAGE_INVERSE
    E.run(stream=stream)
    ms_gather_default = ev_time(lambda: E.run(gather_stages, stream), 3)
    default = E.tuning.as_dict()
    t0 = time.time()
    tuning, tuned_us = E.autotune(reps=3, stream=stream)
    t_tune = time.time() - t0
    print("bench: ensemble autotune %.1fs: %s, gather+reduce %.3f -> %.3f ms"
          % (t_tune, tuning.as_dict(), ms_gather_default, tuned_us * 1e-3), file=sys.stderr, flush=True)
    g = E.graph(stream)
    try:
        ms = ev_time(lambda: g.launch(stream), args.ensemble_steps, warm=2)
    finally:
        g.destroy()
    ms_dec = ev_time(lambda: E.run(dec_stages, stream), 3)
    ms_gat = ev_time(lambda: E.run(gather_stages, stream), 3)
    E.run(stream=stream)
    stream.synchronize()
    print("bench: ensemble %.3f ms per replay (%.1f frames/s); decompose %.3f ms, gather+reduce %.3f ms"
          % (ms, len(wls) * 1e3 / ms, ms_dec, ms_gat), file=sys.stderr, flush=True)

    # the same frames through the per-frame entry points, with the ensemble's pair splits
    SPLIT_WORD = 24
    per = []
    max_ws = max(kk.decompose_workspace_bytes(su.geom, su.N, su.M, su.tpad, prec) for su in sus)
    dws = torch.empty(max_ws, dtype=torch.uint8, device=dev)
    for f, su in enumerate(sus):
        i = E.info[f]
        plan = su.plan.copy()
        plan[SPLIT_WORD] = i.split
        bws = kk.beamform_workspace_bytes(plan)
        per.append(dict(su=su, plan=plan, plan_dev=kk.to_device(plan), shift=kk.to_device(su.luts["shift"]),
                        rt=torch.empty((su.N, su.M, su.T), dtype=torch.complex64, device=dev),
                        img=torch.empty((i.S, i.X, i.Z), dtype=torch.complex64, device=dev),
                        inten=torch.empty((i.X, i.Z), dtype=torch.float32, device=dev),
                        bws=torch.zeros(bws, dtype=torch.uint8, device=dev) if bws else None, rf=E.frame_rf(f)))

    def per_frame_loop():
        for d in per:
            su = d["su"]
            kk.decompose(d["rf"], su.geom, d["shift"], su.M, su.tpad, out=d["rt"], ws=dws,
                         precision=prec, stream=stream)
            kk.beamform(d["rt"], d["plan"], d["plan_dev"], image=d["img"], intensity=d["inten"],
                        mode=kk.COMPOUND_INCOHERENT, ws=d["bws"], stream=stream)

    ms_loop = ev_time(per_frame_loop, 2)
    stream.synchronize()

    # the same per-frame calls with three frames in flight (frame f on stream f mod 3, each stream
    # with its own decomposition workspace), timed between device-wide synchronisations
    side = [torch.cuda.Stream() for _ in range(3)]
    side_ws = [dws] + [torch.empty_like(dws) for _ in range(2)]

    def per_frame_streams():
        for f, d in enumerate(per):
            su, st = d["su"], side[f % 3]
            kk.decompose(d["rf"], su.geom, d["shift"], su.M, su.tpad, out=d["rt"], ws=side_ws[f % 3],
                         precision=prec, stream=st)
            kk.beamform(d["rt"], d["plan"], d["plan_dev"], image=d["img"], intensity=d["inten"],
                        mode=kk.COMPOUND_INCOHERENT, ws=d["bws"], stream=st)

    per_frame_streams()
    torch.cuda.synchronize()
    best = None
    for _ in range(2):
        t0 = time.perf_counter()
        per_frame_streams()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3
        best = dt if best is None else min(best, dt)
    ms_loop3 = best
    print("bench: ensemble frames through the per-frame entry points: %.3f ms on one stream, %.3f ms on three"
          % (ms_loop, ms_loop3), file=sys.stderr, flush=True)
    same = sum(int(torch.equal(d["img"], E.frame_image(f)) and torch.equal(d["inten"], E.frame_intensity(f)))
               for f, d in enumerate(per))
    pixpair = sum(i.X * i.Z * i.P for i in E.info)
    dec_bytes = sum(_decompose_bytes(i.N, i.L, i.T, i.M, i.tpad) for i in E.info)
    return {
        "workload": "%d uneven frames: 64-192 el, 15-75 tx in +-10..18 deg, Eq.6 J=1-3 sets at 4-16x, "
                    "grids 128x256..384x768 px, one speckle medium (%.2f/lambda^2) moving <=50 um/frame"
                    % (len(wls), args.ensemble_density),
        "precision": "%s decomposition, f32 beamform, Eq.9 intensities" % args.ensemble_precision,
        "frames": len(wls),
        "pixel_pairs": pixpair,
        "ms_per_ensemble": round(ms, 4),
        "frames_per_s": round(len(wls) * 1e3 / ms, 1),
        "gpixpair_per_s": round(pixpair / (ms * 1e-3) / 1e9, 2),
        "stages_ms": {"decompose": round(ms_dec, 4), "gather_reduce": round(ms_gat, 4)},
        "graph_launches": int(E.sizes.nlaunches) + sum(1 for c in set(i.cap for i in E.info)),
        "decompose_groups": int(E.sizes.ngroups),
        "gather_units": int(E.sizes.nunits),
        "tuning_default": default,
        "tuning": tuning.as_dict(),
        "gather_reduce_ms_default_tuning": round(ms_gather_default, 4),
        "gather_reduce_ms_tuned": round(tuned_us * 1e-3, 4),
        "per_frame_loop_ms": round(ms_loop, 4),
        "speedup_vs_per_frame_loop": round(ms_loop / ms, 2),
        "per_frame_loop_3_streams_ms": round(ms_loop3, 4),
        "speedup_vs_per_frame_loop_3_streams": round(ms_loop3 / ms, 2),
        "frames_identical_to_per_frame_path": "%d/%d" % (same, len(wls)),
        "stage_rooflines": {
            "decompose": {"bound": "hbm", "bytes_unfused": dec_bytes,
                          "frac_unfused": round(dec_bytes / HBM_BYTES_PER_S / (ms_dec * 1e-3), 4)},
            "gather": {"bound": "alu", "lane_ops": OPS_PER_PIXEL_PAIR * pixpair,
                       "frac": round(OPS_PER_PIXEL_PAIR * pixpair / VALU_LANE_OPS / (ms_gat * 1e-3), 4)},
        },
        "setup_s": {"plan": round(t_plan, 1), "simulate": round(t_sim, 1), "autotune": round(t_tune, 1)},
    }


def completion_report(kk, C, torch, np, args):
    """k-space completion on the vernier geometry, for each observed receive-angle set (13 of 128
    bank columns: Eq. 6 j = 0, 15; Eq. 6 j = 0, 7, 15; Eq. 7): images of evaluation phantoms
    (seeds 12000..) from plain compressed KK and from the completed spectrum, against the fully
    sampled 128-angle KK image (GPU FP32, all pixels; FP64 oracle at sampled pixels for two
    phantoms), with the trained weights committed in the package."""
    from paper_2603_22496_amd import completion as CP
    from oracle import frame as OF
    mean = lambda v: round(float(np.mean(v)), 4) if v else None
    sets, first = {}, None
    rng = np.random.default_rng(5)
    pix = [(rng.integers(0, C.VERNIER.X, 300), rng.integers(0, C.VERNIER.Z, 300)) for _ in range(2)]
    refs, refs64 = {}, {}
    for name in CP.OBSERVED:
        cs = CP.setup(observed=name)
        d = CP.Device(cs)
        loaded = CP.load(CP.weights_path(name))
        W = len(cs.full.sel["rx_theta"])
        net = kk.Net(loaded[0], CP.BATCH, cs.w.N, W, dilation=loaded[1].get("dilation")) if loaded else None
        meta = loaded[1] if loaded else None
        use_net = bool(meta and meta.get("use_net"))
        errs = {"compressed": [], "compressed_best_gain": [], "completed": [], "completed_best_gain": []}
        errs64 = {"compressed_best_gain": [], "completed": [], "completed_best_gain": []}
        for e in range(args.completion_eval):
            seed = CP.EVAL_SEED0 + e
            ds = CP.phantom(cs, seed, meta["scatterers"] if meta else 1000)
            rf = kk.to_device(ds.rf)
            if seed not in refs:
                refs[seed] = CP.full_image(cs, d, rf).cpu().numpy()
            ref = refs[seed]
            comp = CP.complete_image(cs, d, rf, None).cpu().numpy()
            a, b = CP.scaled_error(comp, ref)
            errs["compressed"].append(a)
            errs["compressed_best_gain"].append(b)
            done = None
            if net is not None:
                done = CP.complete_image(cs, d, rf, net).cpu().numpy()
                a, b = CP.scaled_error(done, ref)
                errs["completed"].append(a)
                errs["completed_best_gain"].append(b)
            if e < 2 and not args.no_parity:   # the oracle checks the outputs; it produces none of them
                xi, zi = pix[e]
                if seed not in refs64:
                    sel_o, luts_o = OF.tables(cs.w, scheme=C.SCHEME_FULL_UNIFORM, M=W, j_list=(0,))
                    refs64[seed] = OF.kk_image(ds.rf, sel_o, luts_o, cs.w.X, cs.w.Z, pixels=(xi, zi))[0]
                r64 = refs64[seed]
                errs64["compressed_best_gain"].append(CP.scaled_error(comp[0, xi, zi], r64)[1])
                if done is not None:
                    a, b = CP.scaled_error(done[0, xi, zi], r64)
                    errs64["completed"].append(a)
                    errs64["completed_best_gain"].append(b)
        out = {
            "selection": "Eq. %d, %s" % (7 if CP.OBSERVED[name][0] == C.SCHEME_CONFOCAL else 6,
                                         "M = %d, j = %s" % (CP.OBSERVED[name][1], list(CP.OBSERVED[name][2]))),
            "observed_columns": cs.cols.tolist(),
            "rel_l2_vs_fully_sampled_gpu": {k: mean(v) for k, v in errs.items()},
            "rel_l2_vs_fp64_fully_sampled_sampled_pixels": {k: mean(v) for k, v in errs64.items()},
            "product_path": "network" if use_net else "fallback: plain compressed KK",
        }
        if meta:
            out["training"] = {k: meta[k] for k in ("fit_phantoms", "validation_phantoms", "scatterers", "epochs",
                                                    "bins_per_phantom", "batch", "seconds", "validation")}
            out["training"]["final_loss"] = meta["history"][-1] if meta.get("history") else None
        if first is None:
            rf = kk.to_device(CP.phantom(cs, CP.EVAL_SEED0, 300).rf)
            ms_c = timed(lambda: CP.complete_image(cs, d, rf, None), 5, 2, torch)
            ms_n = timed(lambda: CP.complete_image(cs, d, rf, net), 3, 1, torch) if net is not None else None
            first = {"compressed": round(ms_c, 3), "completed": round(ms_n, 3) if ms_n else None}
        sets[name] = out
        del d
    return {
        "workload": "vernier geometry (128 el, 31 tx, 2048 samples, 256x512 px); 128-angle bank, 13 columns "
                    "observed (403 of 3968 pairs, 9.8x); 6x3x3 conv, 32 ch, BF16/FP32 on MFMA",
        "eval_phantoms": args.completion_eval,
        "observed_sets": sets,
        "ms_per_frame_vernier_set": first,
    }


def study_report(np):
    """Scheme / compounding image metrics on synthetic phantoms (gCNR of an anechoic cyst, lateral
    FWHM of point targets) against DAS on the same data, N = 15 and N = 7."""
    from paper_2603_22496_amd import study as ST
    rep = ST.run(log=lambda s: print("bench: " + s, file=sys.stderr, flush=True))
    out = {"geometry": rep["geometry"], "results": {}}
    for n, res in rep["results"].items():
        out["results"][n] = {name: {"compression": r["compression"], "gcnr": r["gcnr"],
                                    "fwhm_mm_mean": round(float(np.nanmean(r["fwhm_mm"])), 3)}
                             for name, r in res.items()}
    return out


def full_bank_report(kk, C, torch, np, ds, img_vernier, args, log):
    """The same channel data beamformed over the dense 128-angle receive bank (all 3968 pairs,
    one set): one-stream frame time, and the vernier frame's coherent compound compared with the
    fully sampled image (raw rel-L2, rel-L2 after the best complex gain, envelope correlation)."""
    from oracle import frame as OF
    w = C.FULL
    su = kk.make_setup(w)
    dev = torch.device("cuda", 0)
    rf = kk.to_device(ds.rf)
    shift, pd = kk.to_device(su.luts["shift"]), kk.to_device(su.plan)
    rt = torch.empty((w.N, su.M, w.T), dtype=torch.complex64, device=dev)
    ws = torch.empty(kk.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad), dtype=torch.uint8, device=dev)
    img = torch.empty((1, w.X, w.Z), dtype=torch.complex64, device=dev)
    inten = torch.empty((w.X, w.Z), dtype=torch.float32, device=dev)
    bws = torch.zeros(max(1, kk.beamform_workspace_bytes(su.plan)), dtype=torch.uint8, device=dev)

    def frame():
        kk.decompose(rf, su.geom, shift, su.M, su.tpad, out=rt, ws=ws)
        kk.beamform(rt, su.plan, pd, image=img, intensity=inten, mode=kk.COMPOUND_INCOHERENT, ws=bws)

    ms = timed(frame, max(10, args.steps // 4), 3, torch, repeats=2)
    ms_dec = timed(lambda: kk.decompose(rf, su.geom, shift, su.M, su.tpad, out=rt, ws=ws), max(10, args.steps // 4),
                   3, torch, repeats=2)
    frame()
    torch.cuda.synchronize()
    full = img.cpu().numpy()[0]
    coh = img_vernier.sum(axis=0)
    a = full.ravel().astype(np.complex128)
    b = coh.ravel().astype(np.complex128)
    gain = np.vdot(b, a) / np.vdot(b, b)
    env_a, env_b = np.abs(a), np.abs(b)
    ea, eb = env_a - env_a.mean(), env_b - env_b.mean()
    P = len(su.sel["pairs"])
    out = {
        "workload": "128-angle uniform receive bank over +-16 deg, all %d pairs, one set, same data and grid" % P,
        "frame_us_one_stream": round(ms * 1e3, 2), "decompose_us": round(ms_dec * 1e3, 2),
        "frames_per_s": round(1e3 / ms, 1), "gpixel_pair_per_s": round(w.X * w.Z * P / (ms * 1e-3) / 1e9, 1),
        "plan_split": int(su.plan[24]),
        "vernier_vs_full": {
            "rel_l2": round(float(np.linalg.norm(b - a) / np.linalg.norm(a)), 4),
            "rel_l2_after_best_complex_gain": round(float(np.linalg.norm(gain * b - a) / np.linalg.norm(a)), 4),
            "envelope_correlation": round(float(np.dot(ea, eb) / np.sqrt(np.dot(ea, ea) * np.dot(eb, eb))), 4),
            "compression": round(float(C.VERNIER.L / 14.0), 2)},
    }
    if not args.no_parity:
        sel, luts = OF.tables(w)
        rng = np.random.default_rng(3)
        xi, zi = rng.integers(0, w.X, 200), rng.integers(0, w.Z, 200)
        ref = OF.kk_image(ds.rf, sel, luts, w.X, w.Z, pixels=(xi, zi))[0]
        out["rel_l2_vs_fp64_oracle_sampled"] = float(np.linalg.norm(full[xi, zi] - ref) / np.linalg.norm(ref))
    log("full bank: %.2f us/frame (decompose %.2f us), vernier vs full %s"
        % (ms * 1e3, ms_dec * 1e3, json.dumps(out["vernier_vs_full"])))
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (--gpus 1); KK frames would shard frame-parallel across GPUs, "
              "but no multi-GPU path is provided", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2603_22496_amd import configs as C

    def log(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    w = C.VERNIER
    t0 = time.time()
    ds = C.speckle_dataset(w, seed=2, n_scat=100_000)
    log("vernier data generated in %.1fs" % (time.time() - t0))
    # the CPU baseline first: its workers are forks of this process before it touches the GPU
    cpu = cpu_baseline(C, ds, w, args.cpu_frames, log) if args.cpu_frames > 0 else None

    from paper_2603_22496_amd import kk
    if not os.path.exists(kk.LIB_PATH):
        from paper_2603_22496_amd.build import build_all
        build_all()
    torch.cuda.set_device(0)
    t0 = time.time()
    su = kk.make_setup(w, with_das=not args.no_das)
    t_setup = time.time() - t0
    P = len(su.sel["pairs"])
    S = su.sel["S"]
    log("workload vernier N=%d L=%d T=%d M=%d P=%d S=%d grid %dx%d tpad=%d (setup %.1fs)"
        % (w.N, w.L, w.T, su.M, P, S, w.X, w.Z, su.tpad, t_setup))

    dev = torch.device("cuda", 0)
    rf = kk.to_device(ds.rf)
    shift = kk.to_device(su.luts["shift"])
    plan_dev = kk.to_device(su.plan)
    rt = torch.empty((w.N, su.M, w.T), dtype=torch.complex64, device=dev)
    ws = torch.empty(kk.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad), dtype=torch.uint8, device=dev)
    img = torch.empty((S, w.X, w.Z), dtype=torch.complex64, device=dev)
    inten = torch.empty((w.X, w.Z), dtype=torch.float32, device=dev)
    bws = torch.zeros(max(1, kk.beamform_workspace_bytes(su.plan)), dtype=torch.uint8, device=dev)

    # the phase tables of the decomposition depend on the geometry only (like the plan): written
    # once per workspace by kk_decompose_prepare, outside the timed frames
    kk.decompose_prepare(su.geom, w.N, shift, su.M, su.tpad, ws)

    def frame():
        kk.decompose(rf, su.geom, shift, su.M, su.tpad, out=rt, ws=ws, prepared=True)
        kk.beamform(rt, su.plan, plan_dev, image=img, intensity=inten, mode=kk.COMPOUND_INCOHERENT, ws=bws)

    def decompose_only():
        kk.decompose(rf, su.geom, shift, su.M, su.tpad, out=rt, ws=ws, prepared=True)

    def decompose_unprepared():
        kk.decompose(rf, su.geom, shift, su.M, su.tpad, out=rt, ws=ws)

    def prepare_only():
        kk.decompose_prepare(su.geom, w.N, shift, su.M, su.tpad, ws)

    def gather_only():
        kk.beamform(rt, su.plan, plan_dev, image=img, intensity=inten, mode=kk.COMPOUND_INCOHERENT, ws=bws)

    split = int(su.plan[kk.PLAN_WORD_SPLIT])

    def gather_kernel_only():
        # the gather kernel alone: no intensity, and (unsplit plan) no share reduction
        kk.beamform(rt, su.plan, plan_dev, image=img, ws=bws)

    # The timed region: K frames bracketed by synchronisation, frame k on stream k mod F with its
    # own channel data (each stream's records are those of the phantom rotated in time by a
    # different number of samples, so no stream re-reads another's input from the caches),
    # outputs and workspaces; the tables and plan are shared read-only, as a scanner's stream
    # of independent frames runs.
    nstreams = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    bufs = [dict(rf=rf, rt=rt, ws=ws, img=img, inten=inten, bws=bws)]
    for k in range(1, nstreams):
        b = {key: torch.empty_like(v) for key, v in bufs[0].items() if key != "rf"}
        b["rf"] = torch.roll(rf, shifts=97 * k, dims=2).contiguous()
        kk.decompose_prepare(su.geom, w.N, shift, su.M, su.tpad, b["ws"])
        bufs.append(b)

    def frame_on(b, st):
        kk.decompose(b["rf"], su.geom, shift, su.M, su.tpad, out=b["rt"], ws=b["ws"], stream=st, prepared=True)
        kk.beamform(b["rt"], su.plan, plan_dev, image=b["img"], intensity=b["inten"], mode=kk.COMPOUND_INCOHERENT,
                    ws=b["bws"], stream=st)

    def frames(k0, count):
        for k in range(k0, k0 + count):
            frame_on(bufs[k % nstreams], streams[k % nstreams])

    # Settle before the warm-up steps: in a fresh process the first ~10 ms of back-to-back frames
    # run slower than every later loop (clocks and queues ramping up), which no fixed count of
    # warm-up frames covers.
    t_settle = time.time()
    while time.time() - t_settle < args.settle_s:
        frames(0, 64)
        torch.cuda.synchronize()
    frames(0, args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    cur = torch.cuda.current_stream()
    wall0 = time.time()
    e0.record(cur)
    for st in streams:
        st.wait_event(e0)
    frames(0, args.steps)
    for st in streams:
        cur.wait_stream(st)
    e1.record(cur)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    log("%d KK frames on %d streams in %.3fs wall, %.2f us/frame" % (args.steps, nstreams, wall, ms * 1e3))
    # every stream's last frame against the same input's frame computed alone on one stream
    streams_ok = True
    for b in bufs:
        chk = dict(rf=b["rf"], rt=torch.empty_like(rt), ws=torch.empty_like(ws), img=torch.empty_like(img),
                   inten=torch.empty_like(inten), bws=torch.zeros_like(bws))
        # the check frame takes the unprepared entry point (tables written in the call)
        kk.decompose(chk["rf"], su.geom, shift, su.M, su.tpad, out=chk["rt"], ws=chk["ws"], stream=cur)
        kk.beamform(chk["rt"], su.plan, plan_dev, image=chk["img"], intensity=chk["inten"],
                    mode=kk.COMPOUND_INCOHERENT, ws=chk["bws"], stream=cur)
        torch.cuda.synchronize()
        streams_ok &= bool(torch.equal(chk["img"], b["img"])) and bool(torch.equal(chk["inten"], b["inten"]))
    # one frame at a time on one stream (frame latency)
    ms_single = timed(frame, args.steps, 5, torch, repeats=2)
    log("one stream %.2f us/frame" % (ms_single * 1e3))

    graph_rep = graph_report(frame, img, inten, args, torch, np)
    log("graph replay %s" % json.dumps(graph_rep))

    ms_dec = timed(decompose_only, args.steps, 5, torch, repeats=3)
    ms_dec_unprepared = timed(decompose_unprepared, args.steps, 5, torch, repeats=3)
    ms_prepare = timed(prepare_only, max(10, args.steps // 4), 3, torch, repeats=2)
    kk.decompose_prepare(su.geom, w.N, shift, su.M, su.tpad, ws)
    ms_gather = timed(gather_only, args.steps, 5, torch, repeats=3)
    ms_gather_kernel = timed(gather_kernel_only, args.steps, 5, torch, repeats=3)
    res = {}
    if not args.no_das:
        das_dev = kk.to_device(su.das_plan)
        dimg = torch.empty((w.X, w.Z), dtype=torch.complex64, device=dev)
        dws = torch.zeros(kk.das_workspace_bytes(su.geom, w.N, su.das_plan), dtype=torch.uint8, device=dev)
        das_steps = max(10, args.steps // 4)
        ms_das = timed(lambda: kk.das_beamform(rf, su.geom, su.das_plan, das_dev, image=dimg, ws=dws),
                       das_steps, 3, torch, repeats=2)
        res["das_ms"] = ms_das
        log("DAS %.2f us/frame" % (ms_das * 1e3))

    def section(name, fn):
        """An extra report: a Python-level failure in it is recorded in the JSON line instead of
        ending the run before the headline is printed."""
        try:
            return fn()
        except Exception as exc:
            import traceback
            traceback.print_exc()
            log("%s section failed: %s" % (name, exc))
            return {"error": "%s: %s" % (type(exc).__name__, exc)}

    frame()
    torch.cuda.synchronize()
    img_host = img.cpu().numpy()
    if not args.no_full_bank:
        res["full"] = section("full bank", lambda: full_bank_report(kk, C, torch, np, ds, img_host, args, log))

    if not args.no_precision:
        res["precision"] = section("precision", lambda: precision_report(kk, C, torch, np, args))

    if not args.no_ensemble:
        res["ensemble"] = section("ensemble", lambda: ensemble_report(kk, C, torch, np, args))

    if not args.no_completion:
        res["completion"] = section("completion", lambda: completion_report(kk, C, torch, np, args))
        if "error" not in res["completion"]:
            for name, o in res["completion"]["observed_sets"].items():
                log("completion %s %s" % (name, json.dumps(o["rel_l2_vs_fully_sampled_gpu"])))

    if not args.no_study:
        res["study"] = section("study", lambda: study_report(np))

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # parity of this very frame against the FP64 oracle at sampled pixels, the oracle using its
    # own selection and tables (the oracle is test infrastructure: it checks the timed output,
    # it never produces it)
    rel = None
    if not args.no_parity:
        from oracle import frame as OF
        sel_o, luts_o = OF.tables(w)
        assert np.array_equal(np.asarray(sel_o["pairs"]), su.sel["pairs"])
        for key in ("lut1", "lut2", "lut3", "lut4", "shift"):
            assert np.array_equal(luts_o[key], su.luts[key]), key
        rng = np.random.default_rng(0)
        xi, zi = rng.integers(0, w.X, 500), rng.integers(0, w.Z, 500)
        ref = OF.kk_image(ds.rf, sel_o, luts_o, w.X, w.Z, pixels=(xi, zi))
        rel = float(np.linalg.norm(img_host[:, xi, zi] - ref) / np.linalg.norm(ref))

    pixpair = w.X * w.Z * P
    gather_rate = pixpair / (ms_gather_kernel * 1e-3)
    achieved = OPS_PER_PIXEL_PAIR * gather_rate / 1e12
    peak = VALU_LANE_OPS / 1e12
    # stage rooflines: algorithmic bytes or work of each stage over its live time
    K = su.tpad // 2 + 1
    rec_bytes = w.N * w.L * w.T * 2                     # int16 channel data
    spec_bytes = w.N * w.L * K * 8                      # analytic spectra (materialised)
    y_bytes = w.N * su.M * K * 8                        # sheared spectra
    rt_bytes = w.N * su.M * w.T * 8                     # RF_theta records
    dec_unfused = rec_bytes + 2 * spec_bytes + 2 * y_bytes + rt_bytes
    dec_fused = rec_bytes + rt_bytes
    dec_flops = 8.0 * su.M * w.L * w.N * K
    t_dec = ms_dec * 1e-3
    t_dec_bound = dec_unfused / HBM_BYTES_PER_S
    t_gather_bound = OPS_PER_PIXEL_PAIR * pixpair / VALU_LANE_OPS
    stage_roofs = {
        "decompose": {"bound": "hbm", "time_us": round(ms_dec * 1e3, 2),
                      "bytes_unfused": dec_unfused, "frac_unfused": round(t_dec_bound / t_dec, 4),
                      "bytes_fused_minimum": dec_fused,
                      "frac_fused_minimum": round(dec_fused / HBM_BYTES_PER_S / t_dec, 4),
                      "mfma_flops": dec_flops, "frac_mfma": round(dec_flops / MFMA_FP32_FLOPS / t_dec, 4)},
        "beamform": {"bound": "alu", "time_us": round(ms_gather * 1e3, 2),
                     "lane_ops": OPS_PER_PIXEL_PAIR * pixpair,
                     "frac": round(t_gather_bound / (ms_gather * 1e-3), 4),
                     "note": "gather kernel and the Eq. 9 intensity pass (kk_beamform with intensity); the gather "
                             "kernel alone is in roofline"},
    }
    out = {
        "metric": METRIC,
        "value": round(pixpair / (ms * 1e-3) / 1e9, 2),
        "unit": "Gpixel·pair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded speckle + points + cyst phantom, int16 channel data)",
        "config": {
            "workload": "vernier: 128 el pitch 0.3 mm, fc 5 MHz, fs 20 MHz, 2048 samples, 31 tx in +-15 deg, "
                        "Eq.6 sets j=0,15 M=7 (13 rx angles, 434 pairs, 9.14x), 256x512 px, Eq.9 compounding",
            "N": w.N, "L": w.L, "T": w.T, "M": su.M, "P": P, "S": S, "X": w.X, "Z": w.Z, "tpad": su.tpad,
        },
        "frames_per_s": round(1e3 / ms, 1),
        "streams": nstreams,
        "streams_match_single_frames": streams_ok,
        "stages_us": {"decompose": round(ms_dec * 1e3, 2),
                      "decompose_writing_phase_tables": round(ms_dec_unprepared * 1e3, 2),
                      "phase_tables_per_geometry": round(ms_prepare * 1e3, 2),
                      "gather": round(ms_gather * 1e3, 2),
                      "gather_kernel": round(ms_gather_kernel * 1e3, 2),
                      "frame": round(ms * 1e3, 2), "frame_one_stream": round(ms_single * 1e3, 2)},
        "beamform_gpixpair_per_s": round(gather_rate / 1e9, 1),
        "rel_l2_vs_fp64_oracle": rel,
        "roofline": {
            "bound": "alu",
            "kernel": "gather_kernel (kk_beamform)",
            "achieved": round(achieved, 3),
            "peak": round(peak, 3),
            "unit": "TOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_gather_traffic(),
            "ops_per_pixel_pair": OPS_PER_PIXEL_PAIR,
            "pixel_pairs_per_launch": pixpair,
        },
        # the whole frame against the sum of its stages' bounds (decomposition at its unfused HBM
        # bound, gather at its VALU bound), for the timed loop and for one frame at a time
        "frame_roofline": {"bound_us": round((t_dec_bound + t_gather_bound) * 1e6, 2),
                           "frac_timed_loop": round((t_dec_bound + t_gather_bound) / (ms * 1e-3), 4),
                           "frac_one_stream": round((t_dec_bound + t_gather_bound) / (ms_single * 1e-3), 4)},
        "stage_rooflines": stage_roofs,
        "graph": graph_rep,
        "clocks": gpu_clocks(),
    }
    for key, name in (("full", "full_bank"), ("precision", "precision_large"), ("ensemble", "ensemble"),
                      ("completion", "completion"), ("study", "study")):
        if key in res:
            out[name] = res[key]
    if "das_ms" in res:
        das_units = w.X * w.Z * w.N * w.L                 # pixel x (transmit, element) gathers
        das_frac = round(DAS_OPS_PER_GATHER * das_units / VALU_LANE_OPS / (res["das_ms"] * 1e-3), 4)
        out["stage_rooflines"]["das"] = {
            "bound": "alu", "time_us": round(res["das_ms"] * 1e3, 2), "lane_ops": DAS_OPS_PER_GATHER * das_units,
            "frac": das_frac, "note": "analytic transforms and the DAS gather, against the gather's VALU bound"}
        out["das_frames_per_s"] = round(1e3 / res["das_ms"], 1)
        out["stages_us"]["das"] = round(res["das_ms"] * 1e3, 2)
        out["kk_over_das_speedup"] = round(res["das_ms"] / ms_single, 2)   # both one frame at a time
        out["kk_over_das_context"] = {"kk_gather_frac": stage_roofs["beamform"]["frac"], "das_frac": das_frac,
                                      "pair_ratio": round(w.N * w.L / P, 2)}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
