"""Every record-window class of the gather kernels (Eq. 5 for KK, Eq. 4 for DAS) against the FP64
oracle at every pixel.

A beamforming plan picks the smallest window class (64 .. 512 record samples per pair and
64 x 16 pixel tile) that holds the widest window any (pair, tile) needs; a separate kernel is
compiled per class (classes above 320 samples run a shallower row pipeline).  The window
width grows with the pixel pitch and the angular fan, so the tiny array imaged at coarser
pitches (lambda / 2 at lower centre frequencies) and wider fans reaches each class.  Each case
asserts the class the plan chose, runs the whole frame (kk_decompose + kk_beamform) with the
plan's pair split and with no split, the DAS comparator on the same data, and one frame
ensemble holding all eight cases (one persistent gather launch per class).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import frame as OF
from paper_2603_22496_amd import configs as C
from paper_2603_22496_amd.phantom import make_dataset, seeded_points
from tests import oracle_ref as OR

TOL = 1e-5
CAP_WORD, SPLIT_WORD = 13, 24   # plan header words: window class, pair shares per (set, tile)

# window class -> (centre frequency, fan half-width in degrees, scheme, M, set list)
CASES = {
    64: (20e6, 10.0, C.SCHEME_FULL_UNIFORM, 16, (0,)),
    128: (10e6, 20.0, C.SCHEME_SHIFTED, 7, (0, 2)),
    192: (5e6, 20.0, C.SCHEME_SHIFTED, 7, (0, 2)),
    256: (3.5e6, 20.0, C.SCHEME_FULL_UNIFORM, 16, (0,)),
    320: (3.5e6, 35.0, C.SCHEME_SHIFTED, 7, (0, 2)),
    384: (2.5e6, 25.0, C.SCHEME_SHIFTED, 7, (0, 2)),
    448: (2e6, 20.0, C.SCHEME_SHIFTED, 7, (0, 2)),
    512: (1.6e6, 20.0, C.SCHEME_SHIFTED, 7, (0, 2)),
}


def _workload(cap):
    fc, th, scheme, M, jl = CASES[cap]
    return replace(C.TINY, name="class%d" % cap, fc=fc, theta_max_deg=th, scheme=scheme, M=M, j_list=jl)


def _dataset(w, cap):
    half = (w.X - 1) * w.dx / 2.0
    z_hi = w.z0 + (w.Z - 1) * w.dz
    return make_dataset(w.acquisition(), seeded_points(500 + cap, amplitudes=(1.0, -0.6, 0.4),
                                                       x_range=(-half, half), z_range=(w.z0, z_hi)))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("cap", sorted(CASES))
def test_geometry_reaches_its_window_class(cap):
    """Host only: the plan of each case selects the class the case is named for."""
    from paper_2603_22496_amd import kk
    su = kk.make_setup(_workload(cap))
    assert int(su.plan[CAP_WORD]) == cap


@pytest.fixture(scope="module")
def kk():
    import torch
    from paper_2603_22496_amd import kk as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K.lib()
    return K


_REF = {}


def _case(K, cap):
    """(workload, dataset, library setup with DAS plan, oracle tables, oracle KK image, oracle DAS image)"""
    if cap not in _REF:
        w = _workload(cap)
        ds = _dataset(w, cap)
        su = K.make_setup(w, with_das=True)
        ot = OR.tables(su, w)
        dt = OR.das_tables(w, su.luts, K.build_das_rx(su.geom, su.grid))
        _REF[cap] = (w, ds, su, ot, ot.kk_image(ds.rf), OF.das_image(ds.rf, dt, w.X, w.Z))
    return _REF[cap]


@pytest.mark.gpu
@pytest.mark.parametrize("cap", sorted(CASES))
def test_kk_frame_every_window_class(kk, cap):
    import torch
    w, ds, su, ot, ref, _ = _case(kk, cap)
    print("window class", cap, "fc", w.fc, "fan", w.theta_max_deg, "split", int(su.plan[SPLIT_WORD]), flush=True)
    assert int(su.plan[CAP_WORD]) == cap
    rt = kk.decompose(kk.to_device(ds.rf), su.geom, kk.to_device(su.luts["shift"]), su.M, su.tpad)
    for split in sorted({int(su.plan[SPLIT_WORD]), 1, 3}):
        plan = su.plan.copy()
        plan[SPLIT_WORD] = split
        img = kk.beamform(rt, plan, kk.to_device(plan))
        torch.cuda.synchronize()
        got = img.cpu().numpy()
        for s in range(ot.sel["S"]):
            assert _rel(got[s], ref[s]) <= TOL, (cap, split, s, _rel(got[s], ref[s]))


@pytest.mark.gpu
@pytest.mark.parametrize("cap", sorted(CASES))
def test_das_frame_on_the_same_geometries(kk, cap):
    import torch
    w, ds, su, _, _, ref = _case(kk, cap)
    print("DAS on window-class geometry", cap, "DAS class", int(su.das_plan[CAP_WORD]), flush=True)
    img = kk.das_beamform(kk.to_device(ds.rf), su.geom, su.das_plan, kk.to_device(su.das_plan))
    torch.cuda.synchronize()
    assert _rel(img.cpu().numpy(), ref) <= TOL


@pytest.mark.gpu
def test_ensemble_holding_every_window_class(kk):
    import torch
    print("ensemble of the eight window classes", flush=True)
    caps = sorted(CASES)
    cases = [_case(kk, c) for c in caps]
    inputs = [kk.setup_frame_input(su, kk.COMPOUND_COHERENT) for (_, _, su, _, _, _) in cases]
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32)
    assert sorted({int(i.cap) for i in E.info}) == caps
    for f, (_, ds, _, _, _, _) in enumerate(cases):
        E.frame_rf(f).copy_(torch.from_numpy(ds.rf))
    torch.cuda.synchronize()
    E.run()
    torch.cuda.synchronize()
    for f, (w, _, _, ot, ref, _) in enumerate(cases):
        got = E.frame_image(f).cpu().numpy()
        for s in range(ot.sel["S"]):
            assert _rel(got[s], ref[s]) <= TOL, (caps[f], s, _rel(got[s], ref[s]))
