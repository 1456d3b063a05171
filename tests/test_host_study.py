"""CPU pins of the study's image metrics (closed forms) and of the k_x statistics of the
paper's receive-angle schemes (Sec. II-C, II-D)."""
import math

import numpy as np
import pytest

from paper_2603_22496_amd import configs as C
from paper_2603_22496_amd import study as ST


def test_gcnr_closed_forms():
    r = np.random.default_rng(0)
    a = r.uniform(0, 1, 200_000)
    assert ST.gcnr(a, a) == pytest.approx(0.0, abs=1e-12)
    assert ST.gcnr(a, a + 5.0) == pytest.approx(1.0)
    # two uniform densities on [0, 1] and [0.5, 1.5]: overlap 1/2
    assert ST.gcnr(a, a + 0.5, bins=150) == pytest.approx(0.5, abs=0.02)
    # two unit Gaussians 2 apart: overlap 2 Phi(-1)
    g = r.standard_normal(400_000)
    ovl = 2 * 0.5 * math.erfc(1.0 / math.sqrt(2.0))
    assert ST.gcnr(g, g + 2.0, bins=400) == pytest.approx(1 - ovl, abs=0.02)


def test_fwhm_closed_forms():
    x = np.arange(-200, 201) * 0.01
    sig = 0.37
    g = np.exp(-x ** 2 / (2 * sig ** 2))
    assert ST.fwhm(g, 0.01) == pytest.approx(2 * math.sqrt(2 * math.log(2)) * sig, rel=1e-3)
    tri = np.maximum(0, 1 - np.abs(x) / 0.8)
    assert ST.fwhm(tri, 0.01) == pytest.approx(0.8, rel=1e-9)
    assert math.isnan(ST.fwhm(np.ones(10), 1.0))


def _sel(scheme, N, M, jl, L=192, th=12.0):
    from paper_2603_22496_amd import kk
    return kk.select_pairs(scheme, L, N, math.radians(th), M, jl)


def test_kx_statistics_of_the_schemes():
    N, M = 15, 7
    dth = math.radians(2 * 12.0 / (N - 1))
    s0 = _sel(C.SCHEME_SHIFTED, N, M, (0,))
    k0 = ST.kx_stats(s0["tx_theta"], s0["rx_theta"], s0["pairs"], dth)
    # Eq. 6, j = 0: the positive receive angles alone step by 2/M transmit steps (the paper's
    # approximate figure); with the mirrored negative angles the fractional parts of th_o - th_i
    # fill every 1/M, all N M differences distinct; support (N - 1) + 2 (M - 1)/M, about the
    # transmit support (1 + 2/N)
    assert k0["min_step"] == pytest.approx(1.0 / M, abs=1e-8)
    assert k0["distinct"] == N * M
    assert k0["support"] == pytest.approx((N - 1) + 2.0 * (M - 1) / M, abs=1e-9)
    assert k0["max_multiplicity"] == 1
    # j = floor(N/2): about twice the support with sparser sampling
    s7 = _sel(C.SCHEME_SHIFTED, N, M, (7,))
    k7 = ST.kx_stats(s7["tx_theta"], s7["rx_theta"], s7["pairs"], dth)
    assert 1.8 * k0["support"] <= k7["support"] <= 2.2 * k0["support"]
    # same angles: unit steps, highly redundant (the zero difference N times)
    ss = _sel(C.SCHEME_SAME, N, N, (0,))
    ks = ST.kx_stats(ss["tx_theta"], ss["rx_theta"], ss["pairs"], dth)
    assert ks["min_step"] == pytest.approx(1.0) and ks["max_multiplicity"] == N
    # confocal Eq. 7: a triangle-like histogram
    sc = _sel(C.SCHEME_CONFOCAL, N, 21, (0,))
    kc = ST.kx_stats(sc["tx_theta"], sc["rx_theta"], sc["pairs"], dth)
    assert kc["triangle_corr"] > 0.85
    assert kc["triangle_corr"] > k0["triangle_corr"]


def test_scaled_j_sets():
    assert ST.scaled_j((0, 3, 6), 15) == (0, 3, 6)
    assert ST.scaled_j((0, 3, 6), 7) == (0, 1, 3)
    assert all(j <= 31 // 2 for j in ST.scaled_j((0, 3, 6), 31))
