"""Split-precision decomposition: the Eq. 3 contraction on 16-bit MFMA with hi+lo operands
(W X ~ Wh Xh + Wh Xl + Wl Xh, FP32 accumulate), against the FP64 oracle.

Bars from the arithmetic.  A value split as hi + lo (each rounded to 16 bits) is exact to
u^2 of its size, u = 2^-8 (BF16) or 2^-11 (FP16); the dropped Wl Xl term is of the same
order, so each product term carries a relative error below ~3 u^2 (4.6e-5 for BF16, 7e-7 for
FP16), largely independent from term to term.  With the FP32 transforms (~1e-6) the rel-L2
bars are 2e-5 for BF16X3 and the FP32 path's 1e-5 for FP16X3 (whose exact power-of-two prescale
keeps int16 spectra, up to 2 T 32768, below the FP16 range).
"""
import numpy as np
import pytest

import oracle as O
from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu


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


def _tol(K, prec):
    return {K.PREC_BF16X3: 2e-5, K.PREC_FP16X3: 1e-5}[prec]


@pytest.mark.parametrize("prec_name", ["PREC_BF16X3", "PREC_FP16X3"])
@pytest.mark.parametrize("N,L,T,M,tpad,seed", [
    (3, 5, 200, 4, 256, 1),
    (5, 7, 333, 17, 512, 2),       # two 16-angle MFMA tiles in one workgroup
    (4, 9, 700, 32, 1024, 7),      # 32 angles in one workgroup
    (3, 5, 400, 45, 512, 8),       # two 32-angle workgroups, the second past the tables
    (33, 6, 1000, 3, 1024, 3),     # two transmit tiles
    (1, 3, 5000, 2, 8192, 6),      # longest records: the FP16 prescale's extreme
])
def test_full_range_records(kk, prec_name, N, L, T, M, tpad, seed):
    import torch
    prec = getattr(kk, prec_name)
    rng = np.random.default_rng(seed)
    rf = rng.integers(-32768, 32767, size=(N, L, T)).astype(np.int16)   # full int16 range
    shift = rng.integers(-2 ** 31, 2 ** 31 - 1, size=(M, L)).astype(np.int32)
    g = kk.geom(L, T, 0.3e-3, 1540.0, 20e6, 0.0)
    out = kk.decompose(kk.to_device(rf), g, kk.to_device(shift), M, tpad, precision=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert _rel(got, O.decompose(rf, shift, tpad)) <= _tol(kk, prec)


@pytest.mark.parametrize("prec_name", ["PREC_BF16X3", "PREC_FP16X3"])
def test_vernier_frame_per_dtype(kk, prec_name):
    import torch
    prec = getattr(kk, prec_name)
    w = C.VERNIER
    ds = C.speckle_dataset(w, seed=2, n_scat=20000)
    su = kk.make_setup(w)
    ot = OR.tables(su, w)
    R64 = ot.decompose(ds.rf)
    rf, sh, pd = kk.to_device(ds.rf), kk.to_device(su.luts["shift"]), kk.to_device(su.plan)
    rt = kk.decompose(rf, su.geom, sh, su.M, su.tpad, precision=prec)
    rt32 = kk.decompose(rf, su.geom, sh, su.M, su.tpad)
    img = kk.beamform(rt, su.plan, pd)
    img32 = kk.beamform(rt32, su.plan, pd)
    torch.cuda.synchronize()
    assert _rel(rt.cpu().numpy(), R64) <= _tol(kk, prec)
    rng = np.random.default_rng(0)
    xi, zi = rng.integers(0, w.X, 300), rng.integers(0, w.Z, 300)
    ref = ot.kk_image(rf_theta=R64, pixels=(xi, zi))
    assert _rel(img.cpu().numpy()[:, xi, zi], ref) <= _tol(kk, prec)
    # against the FP32 run over the whole image
    assert _rel(img.cpu().numpy(), img32.cpu().numpy()) <= _tol(kk, prec)


@pytest.fixture(scope="module")
def large_case(kk):
    """The large workload at full size (192 elements, 75 transmits, 4096 samples, FFT length 8192,
    Eq. 6 j = 0, 37, 1350 pair slots, 384 x 768 pixels) with its FP64 oracle records."""
    w = C.LARGE
    ds = C.speckle_dataset(w, seed=3, n_scat=20_000)
    su = kk.make_setup(w)
    ot = OR.tables(su, w)
    return w, ds, su, ot, ot.decompose(ds.rf)


@pytest.mark.parametrize("prec_name", ["PREC_FP32", "PREC_BF16X3", "PREC_FP16X3"])
def test_large_frame_full_size(kk, large_case, prec_name):
    import torch
    prec = getattr(kk, prec_name)
    w, ds, su, ot, R64 = large_case
    print("large frame", prec_name, flush=True)
    rf, sh, pd = kk.to_device(ds.rf), kk.to_device(su.luts["shift"]), kk.to_device(su.plan)
    rt = kk.decompose(rf, su.geom, sh, su.M, su.tpad, precision=prec)
    img = kk.beamform(rt, su.plan, pd)
    torch.cuda.synchronize()
    tol = 1e-5 if prec == kk.PREC_FP32 else _tol(kk, prec)
    assert _rel(rt.cpu().numpy(), R64) <= tol
    rng = np.random.default_rng(4)
    xi, zi = rng.integers(0, w.X, 300), rng.integers(0, w.Z, 300)
    ref = ot.kk_image(rf_theta=R64, pixels=(xi, zi))
    assert _rel(img.cpu().numpy()[:, xi, zi], ref) <= tol


def test_precision_errors(kk):
    import torch
    w = C.TINY
    su = kk.make_setup(w)
    rf = kk.to_device(C.tiny_dataset(0).rf)
    with pytest.raises(kk.KKError) as e:
        kk.decompose(rf, su.geom, kk.to_device(su.luts["shift"]), su.M, su.tpad, precision=7)
    assert e.value.status == kk.KK_E_UNSUPPORTED
    assert kk.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad, kk.PREC_BF16X3) == \
        kk.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad, kk.PREC_FP32)
    torch.cuda.synchronize()
