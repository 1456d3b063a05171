"""GPU parity of the frame-ensemble path (kk_ensemble_*) against the per-frame entry points and
the FP64 oracle.

Every step of an ensemble runs the per-frame kernels' bodies, so each frame's RF_theta, images
and intensity must equal, bit for bit, what kk_decompose + kk_beamform give for that frame
with the same precision and the same pair split.  Small frames are also checked against the
FP64 oracle (Eq. 3 and Eq. 5 to rel-L2 1e-5 in FP32).  The work queue must hand out every
gather unit exactly once, graph replays must repeat the eager run, and re-planning with
autotuned launch shapes must keep the results.
"""
import numpy as np
import pytest

from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu

SPLIT_WORD = 24    # beamforming plan header word: pair shares per (set, tile)
TOL_ORACLE = 1e-5


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def kk():
    import torch
    from paper_2603_22496_amd import kk as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K.lib()
    return K


def _frames(K, n, seed, L_range=(16, 48), N_range=(5, 15), scale=(0.25, 0.5), modes=None):
    ws = C.ensemble_workloads(n, seed=seed, L_range=L_range, N_range=N_range, scale_range=scale)
    med = C.ensemble_medium(ws, seed=seed + 1, per_lambda2=0.3)
    sus, inputs, data = [], [], []
    for f, w in enumerate(ws):
        su = K.make_setup(w)
        mode = (modes[f % len(modes)] if modes else K.COMPOUND_INCOHERENT)
        sus.append(su)
        inputs.append(K.setup_frame_input(su, mode))
        data.append(C.ensemble_dataset(w, med, f).rf)
    return ws, sus, inputs, data


def _load(E, data):
    import torch
    for f, rf in enumerate(data):
        E.frame_rf(f).copy_(torch.from_numpy(rf))
    torch.cuda.synchronize()


def _per_frame(K, E, f, su, rf, precision):
    """kk_decompose + kk_beamform (+ intensity) of frame f with the ensemble's pair split."""
    import torch
    i = E.info[f]
    plan = su.plan.copy()
    plan[SPLIT_WORD] = i.split
    rt = K.decompose(K.to_device(rf), su.geom, K.to_device(su.luts["shift"]), su.M, su.tpad, precision=precision)
    inten = torch.zeros((i.X, i.Z), dtype=torch.float32, device="cuda") if i.mode >= 0 else None
    img = K.beamform(rt, plan, K.to_device(plan), intensity=inten, mode=max(i.mode, 0))
    torch.cuda.synchronize()
    return rt.cpu().numpy(), img.cpu().numpy(), None if inten is None else inten.cpu().numpy()


def _check_equal_per_frame(K, E, sus, data, precision, frames=None):
    import torch
    torch.cuda.synchronize()
    for f in (range(len(sus)) if frames is None else frames):
        rt, img, inten = _per_frame(K, E, f, sus[f], data[f], precision)
        np.testing.assert_array_equal(E.frame_rf_theta(f).cpu().numpy(), rt, err_msg="RF_theta frame %d" % f)
        np.testing.assert_array_equal(E.frame_image(f).cpu().numpy(), img, err_msg="image frame %d" % f)
        if inten is not None:
            np.testing.assert_array_equal(E.frame_intensity(f).cpu().numpy(), inten, err_msg="intensity %d" % f)


@pytest.mark.parametrize("precision,queue,budget", [
    (0, 1, 0),             # FP32, per-XCD lists, one decomposition group
    (0, 0, 8 << 20),       # FP32, one list, several groups
    (1, 1, 8 << 20),       # BF16 hi+lo, several groups
    (2, 0, 0),             # FP16 hi+lo
])
def test_ensemble_equals_per_frame_path(kk, precision, queue, budget):
    print("ensemble vs per-frame: precision %d queue %d budget %d" % (precision, queue, budget), flush=True)
    ws, sus, inputs, data = _frames(kk, 7, seed=11 + precision,
                                    modes=[kk.COMPOUND_INCOHERENT, -1, kk.COMPOUND_COHERENT])
    t = kk.default_tuning()
    t.queue = queue
    E = kk.Ensemble(inputs, precision=precision, tuning=t, spectra_budget=budget)
    if budget:
        assert E.sizes.ngroups >= 2
    _load(E, data)
    E.run()
    _check_equal_per_frame(kk, E, sus, data, precision)


def test_ensemble_split_pairs_equal_per_frame_path(kk):
    # pair tiles small enough that every frame's sets are shared by several workgroups
    ws, sus, inputs, data = _frames(kk, 6, seed=23)
    t = kk.default_tuning()
    for c in range(kk.ENSEMBLE_CLASSES):
        t.pair_tile[c] = 4
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32, tuning=t)
    assert all(i.split > 1 for i in E.info)
    _load(E, data)
    E.run()
    _check_equal_per_frame(kk, E, sus, data, kk.PREC_FP32)


def test_ensemble_against_oracle(kk):
    ws, sus, inputs, data = _frames(kk, 3, seed=31, modes=[kk.COMPOUND_COHERENT])
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32)
    _load(E, data)
    E.run()
    import torch
    torch.cuda.synchronize()
    for f, su in enumerate(sus):
        ref = OR.tables(su, ws[f]).kk_image(data[f])
        got = E.frame_image(f).cpu().numpy()
        rel = _rel(got, ref)
        print("frame %d (L %d N %d M %d S %d %dx%d) rel-L2 %.3e" % (f, su.geom.L, su.N, su.M, su.sel["S"],
                                                                  su.grid.X, su.grid.Z, rel), flush=True)
        assert rel <= TOL_ORACLE, rel
        coh = np.abs(ref.sum(axis=0)) ** 2
        assert _rel(E.frame_intensity(f).cpu().numpy(), coh) <= 2 * TOL_ORACLE


def test_queue_hands_out_each_unit_once(kk):
    import torch
    ws, sus, inputs, data = _frames(kk, 8, seed=41, L_range=(16, 64), scale=(0.25, 0.75))
    for queue in (0, 1):
        t = kk.default_tuning()
        t.queue = queue
        E = kk.Ensemble(inputs, precision=kk.PREC_FP32, tuning=t)
        _load(E, data)
        E.ws.zero_()
        E.run()
        torch.cuda.synchronize()
        counts = E.unit_counts()
        per_class = {}
        for i in E.info:
            nt = ((i.X + 63) // 64) * ((i.Z + 15) // 16)
            c = kk.WINDOW_CLASSES.index(i.cap)
            per_class[c] = per_class.get(c, 0) + nt * i.S * i.split
        for c in range(kk.ENSEMBLE_CLASSES):
            assert int(counts[c].sum()) == per_class.get(c, 0), (queue, c, int(counts[c].sum()), per_class)
        assert sum(per_class.values()) == E.sizes.nunits


def test_graph_replays_repeat_eager_run(kk):
    import torch
    ws, sus, inputs, data = _frames(kk, 5, seed=51, modes=[kk.COMPOUND_INCOHERENT, kk.COMPOUND_COHERENT])
    t = kk.default_tuning()
    for c in range(kk.ENSEMBLE_CLASSES):
        t.pair_tile[c] = 32          # shares, so the graph holds the share reduction too
    E = kk.Ensemble(inputs, precision=kk.PREC_BF16X3, tuning=t, spectra_budget=8 << 20)
    _load(E, data)
    E.run()
    torch.cuda.synchronize()
    ref_img, ref_int = E.image.cpu().numpy(), E.intensity.cpu().numpy()
    stream = torch.cuda.Stream()
    g = E.graph(stream)
    try:
        for rep in range(3):
            E.image.zero_()
            E.intensity.zero_()
            E.ws.zero_()
            # unrelated eager work between replays
            a = torch.randn(256, 256, device="cuda")
            (a @ a).sum().item()
            torch.cuda.synchronize()
            g.launch(stream)
            stream.synchronize()
            np.testing.assert_array_equal(E.image.cpu().numpy(), ref_img, err_msg="replay %d" % rep)
            np.testing.assert_array_equal(E.intensity.cpu().numpy(), ref_int, err_msg="replay %d" % rep)
    finally:
        g.destroy()


def test_autotune_keeps_results(kk):
    import torch
    ws, sus, inputs, data = _frames(kk, 6, seed=61, L_range=(32, 64), scale=(0.5, 0.75))
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32)
    _load(E, data)
    tuning, us = E.autotune(reps=2)
    print("autotuned:", tuning.as_dict(), "%.1f us" % us, flush=True)
    assert us > 0
    assert tuning.queue in (0, 1)
    for c in range(kk.ENSEMBLE_CLASSES):
        assert tuning.pair_tile[c] in (0, 512, 256, 128, 64, 32)
    E.run()
    torch.cuda.synchronize()
    _check_equal_per_frame(kk, E, sus, data, kk.PREC_FP32)


def test_ensemble_errors(kk):
    import ctypes
    import torch
    ws, sus, inputs, data = _frames(kk, 2, seed=71)
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32)
    L = kk.lib()
    b = list(E._bufs())
    # workspace too small
    st = L.kk_ensemble_run(*b[:7], 16, kk.STAGE_ALL, kk._stream(None))
    assert st == kk.KK_E_WORKSPACE
    # bad stage mask
    assert L.kk_ensemble_run(*b, 64, kk._stream(None)) == kk.KK_E_ARG
    # NULL workspace
    b2 = list(b)
    b2[6] = None
    assert L.kk_ensemble_run(*b2, kk.STAGE_ALL, kk._stream(None)) == kk.KK_E_NULL
    # not an ensemble plan
    bogus = np.zeros(64, np.int32)
    assert L.kk_ensemble_run(bogus.ctypes.data_as(ctypes.c_void_p), b[1], bogus.nbytes, *b[3:],
                             kk.STAGE_ALL, kk._stream(None)) == kk.KK_E_WORKSPACE
    # graph capture needs a created stream
    h = ctypes.c_void_p(0)
    assert L.kk_ensemble_graph_create(*b, None, ctypes.byref(h)) == kk.KK_E_ARG
    torch.cuda.synchronize()
