"""Whole KK frames (kk_decompose + kk_beamform) on randomly drawn small geometries against the FP64
oracle at every pixel: element and transmit counts, record lengths (also not multiples of 8),
receive schemes and set lists, fan widths, ragged grids and record start times all vary, so
windows run off both record ends, tiles are partial and FFT lengths change from case to case."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def kk():
    import torch
    from paper_2603_22496_amd import kk as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K.lib()
    return K


def _draw(case):
    rng = np.random.default_rng(7000 + case)
    N = int(rng.integers(3, 18))
    scheme = C.SCHEME_CONFOCAL if case % 3 == 2 else C.SCHEME_SHIFTED
    M = int(rng.choice([3, 5, 7, 9]))
    J = 1 if scheme == C.SCHEME_CONFOCAL else int(rng.integers(1, 4))
    jl = tuple(int(j) for j in rng.choice(N // 2 + 1, size=min(J, N // 2 + 1), replace=False))
    w = replace(C.TINY, name="random%d" % case, L=int(rng.integers(8, 49)), N=N,
                theta_max_deg=float(rng.uniform(5.0, 20.0)), scheme=scheme, M=M, j_list=jl,
                X=int(rng.integers(30, 141)), Z=int(rng.integers(17, 81)), z0=float(rng.uniform(2e-3, 12e-3)),
                t0=float(rng.uniform(-1e-6, 3e-6)))
    # records long enough for the deepest echo, plus a random tail (any length, also odd)
    reach = 2.0 * (w.z0 + w.Z * w.dz) + w.X * w.dx + w.L * w.pitch
    T = int(np.ceil((reach / w.c + max(w.t0, 0.0)) * w.fs)) + int(rng.integers(0, 400))
    return replace(w, T=T), int(rng.integers(0, 1 << 30))


@pytest.mark.parametrize("case", range(24))
def test_random_frame_against_oracle(kk, case):
    import torch
    from paper_2603_22496_amd.phantom import make_dataset, seeded_points
    w, seed = _draw(case)
    print("random frame", case, "L", w.L, "N", w.N, "T", w.T, "scheme", w.scheme, "M", w.M, "j", w.j_list,
          "grid", w.X, w.Z, flush=True)
    half = (w.X - 1) * w.dx / 2.0
    z_hi = w.z0 + (w.Z - 1) * w.dz
    ds = make_dataset(w.acquisition(), seeded_points(seed, amplitudes=(1.0, -0.7, 0.5, 0.3),
                                                     x_range=(-half, half), z_range=(w.z0, z_hi)))
    su = kk.make_setup(w)
    rt = kk.decompose(kk.to_device(ds.rf), su.geom, kk.to_device(su.luts["shift"]), su.M, su.tpad)
    img = kk.beamform(rt, su.plan, kk.to_device(su.plan))
    torch.cuda.synchronize()
    got = img.cpu().numpy()
    ot = OR.tables(su, w)                          # the oracle's own selection and tables
    R = ot.decompose(ds.rf)
    np.testing.assert_allclose(rt.cpu().numpy(), R, rtol=0, atol=TOL * float(np.abs(R).max()) * 4)
    ref = ot.kk_image(rf_theta=R)
    for s in range(su.sel["S"]):
        rel = float(np.linalg.norm(got[s] - ref[s]) / np.linalg.norm(ref[s]))
        assert rel <= TOL, (s, rel)
