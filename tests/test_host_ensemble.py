"""Host-side checks of the frame-ensemble planner (kk_ensemble_plan / _query / _frame_query):
packed-buffer offsets, workspace regions, decomposition groups, pair splits and errors.  No
device calls."""
import ctypes

import numpy as np
import pytest

from paper_2603_22496_amd import configs as C


@pytest.fixture(scope="module")
def kk():
    from paper_2603_22496_amd import kk as K
    K.lib()
    return K


@pytest.fixture(scope="module")
def frames(kk):
    ws = C.ensemble_workloads(10, seed=5, L_range=(16, 96), N_range=(5, 31), scale_range=(0.25, 1.0))
    sus = [kk.make_setup(w) for w in ws]
    modes = [kk.COMPOUND_INCOHERENT, -1, kk.COMPOUND_COHERENT]
    return ws, sus, [kk.setup_frame_input(su, modes[i % 3]) for i, su in enumerate(sus)]


def _spans(E):
    return [(i.rf_offset, i.N * i.L * i.T) for i in E.info]


def _disjoint(spans):
    s = sorted((a, a + n) for a, n in spans if n > 0)
    return all(s[k][1] <= s[k + 1][0] for k in range(len(s) - 1))


def test_workload_draws_follow_the_batched_form():
    ws = C.ensemble_workloads(200)
    assert len(ws) == 200
    for w in ws:
        assert 64 <= w.L <= 192 and 15 <= w.N <= 75
        assert 1 <= len(w.j_list) <= 3 and w.M % 2 == 1
        comp = w.L / (len(w.j_list) * w.M)
        assert 4.0 - 1e-9 <= comp <= 16.0 + 1e-9, (w.L, w.j_list, w.M)
        assert 128 <= w.X <= 384 and 256 <= w.Z <= 768
        assert w.T % 64 == 0 and w.T >= 4 * w.Z + 128
        assert all(0 <= j <= w.N // 2 for j in w.j_list)
    # uneven: the shapes really differ
    assert len({(w.L, w.N, w.X) for w in ws}) > 150


def test_medium_moves_by_at_most_the_step():
    ws = C.ensemble_workloads(4, seed=9)
    x, z, a, vx, vz = C.ensemble_medium(ws, per_lambda2=0.05)
    sp = np.hypot(vx, vz)
    assert sp.max() <= 50e-6 + 1e-15 and sp.min() >= 0
    assert len(x) == len(z) == len(a) > 100


def test_plan_offsets_and_regions(kk, frames):
    ws, sus, inputs = frames
    E = kk.Ensemble(inputs, precision=kk.PREC_BF16X3, allocate=False)
    s = E.sizes
    assert s.nframes == len(inputs) and s.precision == kk.PREC_BF16X3 and s.ngroups == 1
    assert _disjoint(_spans(E))
    assert max(a + n for a, n in _spans(E)) <= s.rf_elems
    for f, (i, su, x) in enumerate(zip(E.info, sus, inputs)):
        assert (i.N, i.L, i.T, i.M) == (su.N, su.geom.L, su.T, su.M)
        assert (i.S, i.X, i.Z, i.P) == (su.sel["S"], su.grid.X, su.grid.Z, len(su.sel["pairs"]))
        assert i.tpad == su.tpad and i.mode == x.mode and i.split == 1 and i.share_offset == -1
        assert i.rf_offset % 128 == 0 and i.image_offset % 32 == 0 and i.rf_theta_offset % 32 == 0
        assert i.cap == int(su.plan[13])
        if x.mode < 0:
            assert i.intensity_offset == -1
        else:
            assert i.intensity_offset % 64 == 0 and i.intensity_offset + i.X * i.Z <= s.intensity_elems
        assert i.image_offset + i.S * i.X * i.Z <= s.image_elems
        assert (i.rf_theta_offset + i.N * i.M * i.T) * 8 <= s.ws_bytes
    assert _disjoint([(i.image_offset, i.S * i.X * i.Z) for i in E.info])
    assert _disjoint([(i.rf_theta_offset, i.N * i.M * i.T) for i in E.info])
    # units: every (set, pixel tile) once when nothing is split
    assert s.nunits == sum(((i.X + 63) // 64) * ((i.Z + 15) // 16) * i.S for i in E.info)
    # one launch per stage and FFT length, one gather per window class, one reduction
    n_lg = len({i.tpad for i in E.info})
    n_cap = len({i.cap for i in E.info})
    assert s.nlaunches == 3 * n_lg + n_cap + 1


def test_pair_tiles_set_the_splits(kk, frames):
    ws, sus, inputs = frames
    t = kk.default_tuning()
    for c in range(kk.ENSEMBLE_CLASSES):
        t.pair_tile[c] = 20
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32, tuning=t, allocate=False)
    for i, su in zip(E.info, sus):
        pairs = su.sel["pairs"]
        max_set = max(int(np.sum(pairs[:, 2] == s)) for s in range(su.sel["S"]))
        assert i.split == min(8, max(1, -(-max_set // 20)))
        if i.split > 1:
            assert i.share_offset >= 0 and i.share_offset % 32 == 0
            assert (i.share_offset + i.split * i.S * i.X * i.Z) * 8 <= E.sizes.ws_bytes
        else:
            assert i.share_offset == -1
    assert E.sizes.nunits == sum(((i.X + 63) // 64) * ((i.Z + 15) // 16) * i.S * i.split for i in E.info)
    regions = [(i.rf_theta_offset, i.N * i.M * i.T) for i in E.info] + \
              [(i.share_offset, i.split * i.S * i.X * i.Z) for i in E.info if i.split > 1]
    assert _disjoint(regions)


def test_spectra_budget_forms_groups(kk, frames):
    ws, sus, inputs = frames
    one = kk.Ensemble(inputs, precision=kk.PREC_FP32, allocate=False)
    budget = 48 << 20
    E = kk.Ensemble(inputs, precision=kk.PREC_FP32, spectra_budget=budget, allocate=False)
    groups = [i.group for i in E.info]
    assert groups == sorted(groups) and groups[0] == 0 and E.sizes.ngroups == groups[-1] + 1 > 1
    # a group's spectra fit the budget unless it is a single frame
    def spectra(i):
        kpad = (i.tpad // 2 + 1 + 7) // 8 * 8
        ncol = (i.N + 31) // 32 * 32
        a = lambda v: (v + 255) // 256 * 256
        return a(kpad * ncol * i.L * 8) + a(i.N * i.M * kpad * 8)
    for g in range(E.sizes.ngroups):
        members = [i for i in E.info if i.group == g]
        tot = sum(spectra(i) for i in members)
        assert tot <= budget or len(members) == 1
    assert E.sizes.ws_bytes < one.sizes.ws_bytes
    # offsets of the packed buffers do not depend on the grouping
    assert [(i.rf_offset, i.image_offset, i.rf_theta_offset) for i in E.info] == \
           [(i.rf_offset, i.image_offset, i.rf_theta_offset) for i in one.info]


def test_plan_errors(kk, frames):
    ws, sus, inputs = frames
    L = kk.lib()
    E = kk.Ensemble(inputs[:2], precision=kk.PREC_FP32, allocate=False)
    arr = E._frames
    need = ctypes.c_size_t(0)
    t = kk.default_tuning()
    assert L.kk_ensemble_plan(arr, 2, 7, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_UNSUPPORTED
    assert L.kk_ensemble_plan(arr, 0, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    assert L.kk_ensemble_plan(None, 2, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_NULL
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(t), -1, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    # size query
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_CAPACITY
    assert need.value == E.plan_host.nbytes
    # a bad queue layout / pair tile
    bad = kk.default_tuning()
    bad.queue = 3
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(bad), 0, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    bad = kk.default_tuning()
    bad.pair_tile[1] = -4
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(bad), 0, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    # a frame whose description disagrees with its plan, a bad mode, a corrupt plan
    keep = (arr[0].N, arr[0].mode, arr[0].plan_bytes)
    arr[0].N = keep[0] + 1
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    arr[0].N = keep[0]
    arr[0].mode = 5
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_ARG
    arr[0].mode = keep[1]
    arr[0].plan_bytes = 16
    assert L.kk_ensemble_plan(arr, 2, 0, ctypes.byref(t), 0, None, 0, ctypes.byref(need)) == kk.KK_E_WORKSPACE
    arr[0].plan_bytes = keep[2]
    # queries
    sz = kk.EnsembleSizes()
    bogus = np.zeros(64, np.int32)
    assert L.kk_ensemble_query(bogus.ctypes.data_as(ctypes.c_void_p), bogus.nbytes, ctypes.byref(sz)) == \
        kk.KK_E_WORKSPACE
    fi = kk.EnsembleFrameInfo()
    p = E.plan_host
    assert L.kk_ensemble_frame_query(p.ctypes.data_as(ctypes.c_void_p), p.nbytes, 2, ctypes.byref(fi)) == kk.KK_E_ARG
    assert L.kk_ensemble_frame_query(p.ctypes.data_as(ctypes.c_void_p), p.nbytes, 1, ctypes.byref(fi)) == kk.KK_OK
    assert L.kk_ensemble_query(p.ctypes.data_as(ctypes.c_void_p), 64, ctypes.byref(sz)) == kk.KK_E_WORKSPACE
