"""GPU run of a reduced scheme study: the anechoic cyst is detected by DAS and KK (gCNR), and a
larger Eq. 6 shift j (broader k_x support, Sec. II-C) does not widen point targets."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def report():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_22496_amd import configs as C
    from paper_2603_22496_amd import study as ST
    g = ST.StudyGeometry(X=160, Z=240)
    schemes = [("KK j=0 M19", C.SCHEME_SHIFTED, 19, (0,), None),
               ("KK j=6 M19", C.SCHEME_SHIFTED, 19, (6,), None),
               ("KK incoherent j=0,3,6 M19", C.SCHEME_SHIFTED, 19, (0, 3, 6), "inc")]
    return ST.run(N_list=(15,), g=g, schemes=schemes, per_lambda2=1.5,
                  log=lambda s: print(s, flush=True))["results"]["N=15"]


def test_cyst_is_detected(report):
    for name in ("DAS", "KK j=0 M19", "KK incoherent j=0,3,6 M19"):
        print(name, report[name]["gcnr"], flush=True)
        assert 0.5 < report[name]["gcnr"] <= 1.0, name


def test_larger_shift_does_not_widen_points(report):
    w0 = np.array(report["KK j=0 M19"]["fwhm_mm"])
    w6 = np.array(report["KK j=6 M19"]["fwhm_mm"])
    assert np.all(np.isfinite(w0)) and np.all(np.isfinite(w6))
    print("FWHM j=0", w0, "j=6", w6, flush=True)
    assert np.mean(w6) <= np.mean(w0) * 1.02


def test_compression_and_kx(report):
    assert report["KK j=0 M19"]["compression"] == pytest.approx(192 / 19, abs=0.006)   # reported to 2 decimals
    assert report["KK incoherent j=0,3,6 M19"]["compression"] == pytest.approx(192 / 57, abs=0.006)
    assert report["KK j=6 M19"]["kx"]["support"] > 1.5 * report["KK j=0 M19"]["kx"]["support"]
