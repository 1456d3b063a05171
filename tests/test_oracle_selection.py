"""Pins for the oracle's angle selection (Sec. II-C, II-D; Eq. 6, Eq. 7; Table II).

Every expected value here comes from the paper (printed compression ratios, the Fig. 2 /
Fig. 3 setting and the support claims of Sec. II-C) or from exact rational arithmetic
done by hand on the printed equations, never from the oracle itself.
"""
import json
import math
import os
from collections import Counter
from fractions import Fraction

import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SCHEMES = {"shifted": O.SHIFTED, "confocal": O.CONFOCAL}


def _fig2():
    with open(os.path.join(GOLD, "fig2_setting.json")) as f:
        return json.load(f)


def _dtheta_units(sel, N):
    """Delta theta / dth_i for every pair, exact (rx rational minus tx rational)."""
    return [Fraction(sel["rx_num"][o], sel["rx_den"][o]) - Fraction(2 * i - (N - 1), 2)
            for (i, o, _) in sel["pairs"]]


def test_table2_compression_ratios():
    with open(os.path.join(GOLD, "table2_compression.json")) as f:
        g = json.load(f)
    for n_tx in g["transmit_counts"]:
        for row in g["rows"]:
            sel = O.select_pairs(SCHEMES[row["scheme"]], g["L"], n_tx, math.radians(24.0),
                                 row["M"], row["j_list"][str(n_tx)])
            assert round(sel["compression"], 1) == row["printed"], row["label"]


def test_eq6_angles_fig2_by_hand():
    # Eq. 6 with dth_i = 24/14 deg = 12/7 deg: theta_o = sgn(o) (2|o|/15 + j) * 12/7 deg
    g = _fig2()
    N, M = g["N"], g["M"]
    for j in (0, 3, 7):
        sel = O.select_pairs(O.SHIFTED, 192, N, math.radians(g["theta_max_deg"]), M, [j])
        expect = sorted(((o > 0) - (o < 0)) * (Fraction(2 * abs(o), 15) + j) * Fraction(12, 7)
                        for o in range(-7, 8))
        got = [math.degrees(t) for t in sel["rx_theta"]]
        assert len(got) == 15
        for e, v in zip(expect, got):
            assert abs(float(e) - v) < 1e-12
    # the outermost j = 0 angle is 14/15 of a transmit step: 1.6 degrees
    sel0 = O.select_pairs(O.SHIFTED, 192, 15, math.radians(12.0), 15, [0])
    assert abs(math.degrees(sel0["rx_theta"][-1]) - 1.6) < 1e-12


def test_eq7_angles_by_hand():
    # Eq. 7, N = M = 15: mod(|o|, 7) = |o| for |o| < 7, 0 at |o| = 7
    sel = O.select_pairs(O.CONFOCAL, 192, 15, math.radians(12.0), 15)
    expect = sorted(((o > 0) - (o < 0)) * (Fraction(2 * abs(o), 15) + (abs(o) % 7)) * Fraction(12, 7)
                    for o in range(-7, 8))
    got = [math.degrees(t) for t in sel["rx_theta"]]
    assert max(abs(float(e) - v) for e, v in zip(expect, got)) < 1e-12
    # largest angle: |o| = 6 -> (12/15 + 6) * 12/7 = 11.657... deg, not |o| = 7
    assert abs(got[-1] - float((Fraction(12, 15) + 6) * Fraction(12, 7))) < 1e-12


def test_support_j0_is_one_plus_two_over_n():
    # Sec. II-C: Delta k_x = Delta k_ix (1 + 2/N) for the j = 0 vernier (exact when M = N)
    g = _fig2()
    N = g["N"]
    sel = O.select_pairs(O.SHIFTED, 192, N, math.radians(12.0), g["M"], [0])
    d = _dtheta_units(sel, N)
    assert (max(d) - min(d)) / (N - 1) == 1 + Fraction(2, N)


def test_support_jmax_roughly_doubles_and_density_halves():
    g = _fig2()
    N = g["N"]
    s0 = O.select_pairs(O.SHIFTED, 192, N, math.radians(12.0), g["M"], [0])
    sj = O.select_pairs(O.SHIFTED, 192, N, math.radians(12.0), g["M"], [g["j_max"]])
    d0, dj = _dtheta_units(s0, N), _dtheta_units(sj, N)
    ratio = (max(dj) - min(dj)) / (N - 1)
    assert 1.9 < ratio < 2.2
    # same number of samples over ~twice the range: density per transmit step halves
    h0 = Counter(math.floor(v + Fraction(1, 2)) for v in d0)
    hj = Counter(math.floor(v + Fraction(1, 2)) for v in dj)
    core0 = [h0[k] for k in range(-6, 7)]
    corej = [hj[k] for k in range(-13, 14)]
    assert all(c == g["M"] for c in core0)                     # j = 0: uniform, M per step
    assert all(abs(c - g["M"] / 2) <= 1 for c in corej)         # j = floor(N/2): ~M/2 per step


def test_step_within_transmit_is_two_over_m():
    # Sec. II-C: consecutive receive angles of the j = 0 set are 2 dth_i / M apart
    sel = O.select_pairs(O.SHIFTED, 192, 15, math.radians(12.0), 15, [0])
    r = [Fraction(n, d) for n, d in zip(sel["rx_num"], sel["rx_den"])]
    assert all(b - a == Fraction(2, 15) for a, b in zip(r, r[1:]))


def test_intermediate_j_is_bimodal():
    # Sec. II-C: dense sampling for |k_x| below ~(N/2 - j) k_ix, sparser beyond
    g = _fig2()
    N, j = g["N"], g["bimodal_j"]
    sel = O.select_pairs(O.SHIFTED, 192, N, math.radians(12.0), g["M"], [j])
    h = Counter(math.floor(v + Fraction(1, 2)) for v in _dtheta_units(sel, N))
    inner = [h[k] for k in range(-3, 4)]
    outer = [h[k] for k in list(range(-10, -5)) + list(range(6, 11))]
    assert min(inner) == g["M"]
    assert max(outer) <= (g["M"] + 1) // 2 + 1


def test_confocal_histogram_is_triangle_like():
    # Sec. II-D / Fig. 3c: density peaks at 0 and falls off continuously
    g = _fig2()
    N = g["N"]
    sel = O.select_pairs(O.CONFOCAL, 192, N, math.radians(12.0), g["M"])
    d = _dtheta_units(sel, N)
    h = Counter(math.floor(v + Fraction(1, 2)) for v in d)
    ks = sorted(h)
    peak = max(h.values())
    assert h[0] == peak
    for k in ks:
        if k > 0:
            assert h[k] <= h[k - 1] + 1
        if k < 0:
            assert h[k] <= h[k + 1] + 1
    # roughly linear fall-off: halfway out, about half the peak count
    half = (max(ks) - min(ks)) // 4
    assert 0.3 * peak <= (h[half] + h[-half]) / 2 <= 0.7 * peak
    assert len(set(d)) == len(d)                                  # no redundancy


def test_same_angle_strategy_is_redundant():
    # Sec. II-C: same tx and rx angles give redundant k_x samples with steps dk_ix
    sel = O.select_pairs(O.SAME, 192, 15, math.radians(12.0), 15)
    d = _dtheta_units(sel, 15)
    c = Counter(d)
    assert max(c.values()) == 15
    assert len(c) == 29
    assert all(v.denominator == 1 for v in c)
    assert sel["rx_theta"] == sel["tx_theta"]
    v = O.select_pairs(O.SHIFTED, 192, 15, math.radians(12.0), 15, [0])
    assert max(Counter(_dtheta_units(v, 15)).values()) == 1


def test_pair_layout_and_shared_broadside():
    sel = O.select_pairs(O.SHIFTED, 128, 31, math.radians(15.0), 7, [0, 15])
    assert sel["S"] == 2
    assert len(sel["rx_theta"]) == 13                 # theta_o = 0 shared by both sets
    assert len(sel["pairs"]) == 31 * 14
    zero = sel["rx_num"].index(0)
    for s in range(2):
        assert sum(1 for (i, o, ss) in sel["pairs"] if ss == s and o == zero) == 31
    # ordering: set, then receive index, then transmit index
    assert sel["pairs"] == sorted(sel["pairs"], key=lambda p: (p[2], p[1], p[0]))
    assert abs(sel["compression"] - 128 / 14) < 1e-15
    assert sel["rx_theta"] == sorted(sel["rx_theta"])


def test_uniform_bank_spacing_and_range():
    sel = O.select_pairs(O.FULL_UNIFORM, 16, 5, math.radians(10.0), 16)
    deg = [math.degrees(t) for t in sel["rx_theta"]]
    assert abs(deg[0] + 15.0) < 1e-12 and abs(deg[-1] - 15.0) < 1e-12
    assert all(abs((b - a) - 2.0) < 1e-12 for a, b in zip(deg, deg[1:]))
    assert len(sel["pairs"]) == 80 and sel["compression"] == 1.0


def test_transmit_angles_uniform_antisymmetric():
    tx = O.tx_angles(31, math.radians(15.0))
    assert tx[0] == -tx[-1] and tx[15] == 0.0
    assert all(abs(math.degrees(b - a) - 1.0) < 1e-12 for a, b in zip(tx, tx[1:]))


@pytest.mark.parametrize("args", [
    (O.SHIFTED, 128, 1, 0.2, 7, [0]),          # N < 2
    (O.SHIFTED, 128, 31, 0.2, 7, [16]),        # j > floor(N/2)
    (O.SHIFTED, 128, 31, 0.2, 7, [-1]),
    (O.SHIFTED, 128, 31, 1.6, 7, [0]),         # theta_max >= 90 deg
    (O.SHIFTED, 128, 31, 0.2, 0, [0]),         # M < 1
    (O.FULL_UNIFORM, 128, 31, 0.2, 1, [0]),
    (7, 128, 31, 0.2, 7, [0]),                 # unknown scheme
    (O.SHIFTED, 128, 3, 1.5, 7, [1]),          # receive angle beyond 90 deg
])
def test_selection_rejects_bad_arguments(args):
    with pytest.raises(ValueError):
        O.select_pairs(*args)
