"""GPU parity of kk_beamform and kk_compound (Eq. 5, 8, 9) against the FP64 oracle.

The record fed to both sides is the oracle's RF_theta rounded to complex64, so these tests
isolate the gather kernel: pair selection, tables and plan are bit-exact (host tests), the
kernel's error is FP32 accumulation only.  Full-size workloads compare sampled pixels that
the oracle evaluates one by one.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu

TOL_BF = 2e-6      # beamform alone: FP32 sums of <= 4000 terms of comparable size


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


def _case(K, w, ds, scheme=None, M=None, jl=None, seed=0):
    """Library setup, the oracle's tables (checked equal to the library's) and the oracle's
    RF_theta rounded to complex64."""
    su = K.make_setup(w, scheme=scheme, M=M, j_list=jl)
    ot = OR.tables(su, w, scheme, M, jl)
    R32 = ot.decompose(ds.rf).astype(np.complex64)
    return su, ot, R32


SPLIT_WORD = 24    # plan header word: pair shares per (set, tile)


def _run(K, su, R32, plan=None):
    import torch
    plan = su.plan if plan is None else plan
    rt = K.to_device(R32)
    pd = K.to_device(plan)
    img = K.beamform(rt, plan, pd)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def _oracle_img(ot, R32, pixels=None):
    return ot.kk_image(rf_theta=R32.astype(np.complex128), pixels=pixels)


@pytest.mark.parametrize("scheme,M,jl", [
    (C.SCHEME_FULL_UNIFORM, 16, (0,)),
    (C.SCHEME_SHIFTED, 7, (0, 1, 2)),
    (C.SCHEME_CONFOCAL, 9, (0,)),
])
def test_tiny_all_pixels(kk, scheme, M, jl):
    ds = C.tiny_dataset(0)
    su, ot, R32 = _case(kk, C.TINY, ds, scheme, M, jl)
    got = _run(kk, su, R32)
    ref = _oracle_img(ot, R32)
    assert got.shape == ref.shape
    assert _rel(got, ref) <= TOL_BF, _rel(got, ref)


def test_ragged_grid_and_record_edges(kk):
    # X, Z not multiples of the 64 x 16 tile; a late record start pushes many delays past
    # the record end and a shallow grid puts others before its start
    w = replace(C.TINY, X=70, Z=37, t0=4e-6, z0=2e-3)
    acq = w.acquisition()
    from paper_2603_22496_amd.phantom import make_dataset, seeded_points
    ds = make_dataset(acq, seeded_points(11, z_range=(4e-3, 12e-3)))
    su, ot, R32 = _case(kk, w, ds, C.SCHEME_SHIFTED, 5, (0, 2))
    got = _run(kk, su, R32)
    ref = _oracle_img(ot, R32)
    assert _rel(got, ref) <= TOL_BF


def test_random_record_values(kk):
    # arbitrary complex records (not band-limited) exercise every lerp weight and edge
    w = replace(C.TINY, X=128, Z=48)
    su = kk.make_setup(w, scheme=C.SCHEME_SHIFTED, M=7, j_list=(0, 2))
    ot = OR.tables(su, w, C.SCHEME_SHIFTED, 7, (0, 2))
    rng = np.random.default_rng(3)
    R32 = (rng.standard_normal((w.N, su.M, w.T)) + 1j * rng.standard_normal((w.N, su.M, w.T))).astype(np.complex64)
    got = _run(kk, su, R32)
    ref = _oracle_img(ot, R32)
    assert _rel(got, ref) <= TOL_BF


def test_pair_split_factors(kk):
    # every share count gives the oracle's image: shares of unequal length, empty shares
    # (more shares than batches), and the partial images summed in the fixed order
    w = replace(C.TINY, X=70, Z=37)
    ds = C.tiny_dataset(6)
    su, ot, R32 = _case(kk, w, ds, C.SCHEME_SHIFTED, 5, (0, 1))
    ref = _oracle_img(ot, R32)
    base = _run(kk, su, R32)
    for k in (1, 2, 3, 5, 8):
        plan = su.plan.copy()
        plan[SPLIT_WORD] = k
        assert kk.beamform_workspace_bytes(plan) == (0 if k == 1 else k * su.sel["S"] * w.X * w.Z * 8)
        got = _run(kk, su, R32, plan)
        assert _rel(got, ref) <= TOL_BF, (k, _rel(got, ref))
        if k == 1:
            assert np.array_equal(got.view(np.uint32), base.view(np.uint32))


@pytest.mark.parametrize("wname", ["vernier", "full"])
def test_full_size_sampled_pixels(kk, wname):
    w = C.WORKLOADS[wname]
    ds = C.speckle_dataset(C.VERNIER, seed=2, n_scat=20000)
    su, ot, R32 = _case(kk, w, ds)
    if wname == "full":   # one set: fewer tiles than CUs, the plan splits the pairs
        assert su.plan[SPLIT_WORD] > 1
    got = _run(kk, su, R32)
    rng = np.random.default_rng(7)
    xi = rng.integers(0, w.X, 400)
    zi = rng.integers(0, w.Z, 400)
    # tile corners and the grid edges too
    xi = np.concatenate([xi, [0, w.X - 1, 63, 64, 0, w.X - 1]])
    zi = np.concatenate([zi, [0, w.Z - 1, 15, 16, w.Z - 1, 0]])
    ref = _oracle_img(ot, R32, pixels=(xi, zi))
    assert _rel(got[:, xi, zi], ref) <= TOL_BF


def test_compounding_matches_oracle(kk):
    import torch
    ds = C.tiny_dataset(4)
    su, ot, R32 = _case(kk, C.TINY, ds, C.SCHEME_SHIFTED, 5, (0, 1, 2))
    rt, pd = kk.to_device(R32), kk.to_device(su.plan)
    for mode, fn in ((kk.COMPOUND_COHERENT, O.coherent), (kk.COMPOUND_INCOHERENT, O.incoherent)):
        inten = torch.empty((su.grid.X, su.grid.Z), dtype=torch.float32, device="cuda")
        img = kk.beamform(rt, su.plan, pd, intensity=inten, mode=mode)
        I2 = kk.compound(img, mode)
        torch.cuda.synchronize()
        ref = fn(_oracle_img(ot, R32))
        assert _rel(inten.cpu().numpy(), ref) <= 2 * TOL_BF
        assert np.array_equal(inten.cpu().numpy(), I2.cpu().numpy())


def test_deterministic(kk):
    ds = C.tiny_dataset(5)
    su, ot, R32 = _case(kk, C.TINY, ds)
    a = _run(kk, su, R32)
    b = _run(kk, su, R32)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    plan = su.plan.copy()
    plan[SPLIT_WORD] = 4
    a = _run(kk, su, R32, plan)
    b = _run(kk, su, R32, plan)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_argument_errors(kk):
    import torch
    ds = C.tiny_dataset(0)
    su, ot, R32 = _case(kk, C.TINY, ds)
    rt, pd = kk.to_device(R32), kk.to_device(su.plan)
    with pytest.raises(kk.KKError) as e:          # record count differs from the plan's
        kk.beamform(rt[:, :-1].contiguous(), su.plan, pd)
    assert e.value.status == kk.KK_E_ARG
    bad = su.plan.copy()
    bad[0] = 0
    with pytest.raises(kk.KKError) as e:
        kk.beamform(rt, bad, pd)
    assert e.value.status == kk.KK_E_WORKSPACE
    split = su.plan.copy()
    split[SPLIT_WORD] = 2
    small = torch.empty(kk.beamform_workspace_bytes(split) - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(kk.KKError) as e:          # share buffer too small
        kk.beamform(rt, split, kk.to_device(split), ws=small)
    assert e.value.status == kk.KK_E_WORKSPACE
    split[SPLIT_WORD] = 9                         # beyond the largest split
    with pytest.raises(kk.KKError) as e:
        kk.beamform(rt, split, pd)
    assert e.value.status == kk.KK_E_WORKSPACE
