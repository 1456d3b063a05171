"""Host half of libkk.so against the oracle (no GPU needed).

* every function declared in include/kk.h is exported;
* selection: angles bit-identical, rationals and pair lists identical (Eq. 6/7, same,
  uniform bank) over many argument sets;
* delay tables, shear table, t0, FFT length and the DAS receive table bit-identical to the
  oracle's independent FP64 evaluation;
* plans: the folded delays equal the table sums exactly, and every delay a tile can produce
  lands inside that tile's record window (so every LDS access of the gather kernel is in
  bounds by construction); error statuses.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2603_22496_amd import configs as C
from paper_2603_22496_amd import kk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# word indices of the plan header (paper_2603_22496_amd/csrc/kk_plan.h)
PW = dict(MAGIC=0, KIND=1, N=2, M=3, T=4, P=5, S=6, X=7, Z=8, NXT=9, NZT=10, XPAD=11, ZPAD=12, CAP=13,
          MAXW=14, PB=15, OFF_SET=16, OFF_REC=17, OFF_A=18, OFF_B=19, OFF_LO=20, OFF_C=21, OFF_TX=22,
          TOTAL=23, SPLIT=24)


def _check_split(h, units, min_set_pairs):
    # pair shares per (set, tile): up to 8, grown while the launch has fewer than 256 workgroups
    # and every share keeps at least two batches of pairs
    k, pb = h["SPLIT"], h["PB"]
    assert 1 <= k <= 8
    assert k == 1 or (units * (k - 1) < 256 and min_set_pairs >= k * 2 * pb)
    assert k == 8 or units * k >= 256 or min_set_pairs < (k + 1) * 2 * pb


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(kk.LIB_PATH):
        from paper_2603_22496_amd.build import build_libkk
        build_libkk()


def _declared():
    src = open(os.path.join(ROOT, "include", "kk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|size_t|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 12
    L = ctypes.CDLL(kk.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(kk.EXPORTS) == names


SELECT_CASES = [
    (kk.SCHEME_SHIFTED, 128, 31, math.radians(15.0), 7, (0, 15)),
    (kk.SCHEME_SHIFTED, 192, 15, math.radians(24.0), 7, (0, 3, 6)),
    (kk.SCHEME_SHIFTED, 192, 15, math.radians(24.0), 19, (0, 3, 6)),
    (kk.SCHEME_SHIFTED, 192, 75, math.radians(18.0), 9, (0, 37)),
    (kk.SCHEME_SHIFTED, 64, 7, math.radians(10.0), 8, (0, 3)),       # even M: M+1 angles
    (kk.SCHEME_SHIFTED, 64, 7, math.radians(10.0), 1, (2,)),
    (kk.SCHEME_CONFOCAL, 192, 15, math.radians(12.0), 15, (0,)),
    (kk.SCHEME_CONFOCAL, 192, 15, math.radians(24.0), 57, (0,)),
    (kk.SCHEME_CONFOCAL, 192, 7, math.radians(24.0), 21, (0,)),
    (kk.SCHEME_CONFOCAL, 32, 3, math.radians(5.0), 5, (0,)),         # floor(N/2) = 1
    (kk.SCHEME_SAME, 192, 15, math.radians(12.0), 15, (0,)),
    (kk.SCHEME_SAME, 16, 2, math.radians(1.0), 1, (0,)),
    (kk.SCHEME_FULL_UNIFORM, 16, 5, math.radians(10.0), 16, (0,)),
    (kk.SCHEME_FULL_UNIFORM, 128, 31, math.radians(15.0), 128, (0,)),
    (kk.SCHEME_FULL_UNIFORM, 128, 31, math.radians(15.0), 2, (0,)),
]


@pytest.mark.parametrize("case", SELECT_CASES)
def test_selection_bit_identical_to_oracle(case):
    scheme, L, N, th, M, jl = case
    a = kk.select_pairs(scheme, L, N, th, M, jl)
    b = O.select_pairs(scheme, L, N, th, M, jl)
    assert np.array_equal(np.asarray(a["tx_theta"]).view(np.int64), np.asarray(b["tx_theta"]).view(np.int64))
    assert np.array_equal(np.asarray(a["rx_theta"]).view(np.int64), np.asarray(b["rx_theta"]).view(np.int64))
    assert list(a["rx_num"]) == b["rx_num"] and list(a["rx_den"]) == b["rx_den"]
    assert [tuple(p) for p in a["pairs"]] == [tuple(p) for p in b["pairs"]]
    assert a["S"] == b["S"] and a["compression"] == b["compression"]


@pytest.mark.parametrize("args,status", [
    ((kk.SCHEME_SHIFTED, 128, 1, 0.2, 7, (0,)), kk.KK_E_ARG),
    ((kk.SCHEME_SHIFTED, 128, 31, 0.2, 7, (16,)), kk.KK_E_ARG),
    ((kk.SCHEME_SHIFTED, 128, 31, 1.6, 7, (0,)), kk.KK_E_ARG),
    ((kk.SCHEME_SHIFTED, 128, 31, 0.2, 0, (0,)), kk.KK_E_ARG),
    ((kk.SCHEME_FULL_UNIFORM, 128, 31, 0.2, 1, (0,)), kk.KK_E_ARG),
    ((9, 128, 31, 0.2, 7, (0,)), kk.KK_E_ARG),
    ((kk.SCHEME_SHIFTED, 128, 3, 1.5, 7, (1,)), kk.KK_E_ARG),
])
def test_selection_errors_match_oracle(args, status):
    with pytest.raises(kk.KKError) as e:
        kk.select_pairs(*args)
    assert e.value.status == status
    with pytest.raises(ValueError):
        O.select_pairs(*args)


def test_selection_capacity_protocol():
    L = kk.lib()
    tx = np.zeros(31)
    m, p, s = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    comp = ctypes.c_double()
    jl = np.array([0, 15], dtype=np.int32)
    small_d = np.zeros(4)
    small_i = np.zeros(12, dtype=np.int32)
    st = L.kk_select_pairs(0, 128, 31, math.radians(15.0), 7, kk._ip(jl), 2, kk._dpp(tx), kk._dpp(small_d),
                           kk._ip(small_i), kk._ip(small_i), 4, ctypes.byref(m), kk._ip(small_i), 4,
                           ctypes.byref(p), ctypes.byref(s), ctypes.byref(comp))
    assert st == kk.KK_E_CAPACITY and m.value == 13 and p.value == 434 and s.value == 2
    st = L.kk_select_pairs(0, 128, 31, math.radians(15.0), 7, None, 2, kk._dpp(tx), None, None, None, 0,
                           ctypes.byref(m), None, 0, ctypes.byref(p), ctypes.byref(s), ctypes.byref(comp))
    assert st == kk.KK_E_NULL


def _both_luts(w, scheme=None, M=None, jl=None):
    sel = O.select_pairs(w.scheme if scheme is None else scheme, w.L, w.N, w.theta_max,
                         w.M if M is None else M, w.j_list if jl is None else jl)
    ora = O.build_luts(w.L, w.T, w.pitch, w.c, w.fs, w.t0, w.X, w.Z, w.x0, w.dx, w.z0, w.dz,
                       sel["tx_theta"], sel["rx_theta"])
    g = kk.geom(w.L, w.T, w.pitch, w.c, w.fs, w.t0)
    gr = kk.grid(w.X, w.Z, w.x0, w.dx, w.z0, w.dz)
    lib = kk.build_luts(g, gr, sel["tx_theta"], sel["rx_theta"])
    return sel, ora, lib, g, gr


@pytest.mark.parametrize("wname", ["tiny", "vernier", "full", "large"])
def test_luts_bit_identical_to_oracle(wname):
    _, ora, lib, _, _ = _both_luts(C.WORKLOADS[wname])
    for k in ("lut1", "lut2", "lut3", "lut4", "shift"):
        assert np.array_equal(ora[k], lib[k]), k
    assert ora["t0_q"] == lib["t0_q"] and ora["tpad"] == lib["tpad"]


@pytest.mark.parametrize("t0", [0.0, 3.0e-6, -1.25e-6, 1.0 / 3.0 * 1e-6])
def test_luts_bit_identical_with_record_start(t0):
    w = C.TINY
    sel = O.select_pairs(O.SHIFTED, w.L, w.N, w.theta_max, 7, (0, 2))
    ora = O.build_luts(w.L, w.T, w.pitch, w.c, w.fs, t0, w.X, w.Z, w.x0, w.dx, w.z0, w.dz,
                       sel["tx_theta"], sel["rx_theta"])
    lib = kk.build_luts(kk.geom(w.L, w.T, w.pitch, w.c, w.fs, t0), kk.grid(w.X, w.Z, w.x0, w.dx, w.z0, w.dz),
                        sel["tx_theta"], sel["rx_theta"])
    for k in ("lut1", "lut2", "lut3", "lut4", "shift"):
        assert np.array_equal(ora[k], lib[k]), k
    assert ora["t0_q"] == lib["t0_q"]


@pytest.mark.parametrize("wname", ["tiny", "vernier"])
def test_das_rx_bit_identical_to_oracle(wname):
    w = C.WORKLOADS[wname]
    g = kk.geom(w.L, w.T, w.pitch, w.c, w.fs, w.t0)
    gr = kk.grid(w.X, w.Z, w.x0, w.dx, w.z0, w.dz)
    assert np.array_equal(kk.build_das_rx(g, gr),
                          O.das_rx_table(w.L, w.pitch, w.c, w.fs, w.X, w.Z, w.x0, w.dx, w.z0, w.dz))


def test_table_errors():
    w = C.TINY
    g = kk.geom(w.L, w.T, w.pitch, w.c, w.fs, w.t0)
    gr = kk.grid(w.X, w.Z, w.x0, w.dx, w.z0, w.dz)
    with pytest.raises(kk.KKError) as e:
        kk.build_luts(kk.geom(w.L, w.T, w.pitch, w.c, 2e12, 0.0), gr, [0.1], [0.1])
    assert e.value.status == kk.KK_E_RANGE
    with pytest.raises(kk.KKError) as e:
        kk.build_luts(kk.geom(w.L, w.T, w.pitch, -1.0, w.fs, 0.0), gr, [0.1], [0.1])
    assert e.value.status == kk.KK_E_ARG
    with pytest.raises(kk.KKError) as e:
        kk.build_luts(g, kk.grid(0, w.Z, w.x0, w.dx, w.z0, w.dz), [0.1], [0.1])
    assert e.value.status == kk.KK_E_ARG
    assert kk.lib().kk_build_luts(None, None, None, 0, None, 0, None, None, None, None, None, None,
                                  None) == kk.KK_E_NULL


def _hdr(plan):
    return {k: int(plan[v]) for k, v in PW.items()}


def _check_kk_plan(plan, sel, ora, w):
    h = _hdr(plan)
    assert h["MAGIC"] == 0x4B4B5031 and h["KIND"] == 0 and h["TOTAL"] == plan.size
    P, S = len(sel["pairs"]), sel["S"]
    assert h["P"] == P and h["S"] == S and h["X"] == w.X and h["Z"] == w.Z
    nxt, nzt, xpad, zpad = h["NXT"], h["NZT"], h["XPAD"], h["ZPAD"]
    assert xpad == nxt * 64 >= w.X and zpad == nzt * 16 >= w.Z
    cap, pb = h["CAP"], h["PB"]
    assert h["MAXW"] <= cap and cap % 64 == 0 and pb % 4 == 0 and pb >= 4
    # LDS footprint of the kernel variant (two buffers of pb slots)
    assert pb == 16 and pb * cap * 16 <= 131072 and pb * cap < 65536
    sets = plan[h["OFF_SET"]:h["OFF_SET"] + S + 1]
    assert sets[0] == 0 and sets[-1] == P and np.all(np.diff(sets) > 0)
    order = [p for s in range(S) for p in range(P) if sel["pairs"][p][2] == s]
    Md = len(sel["rx_theta"])
    rec = plan[h["OFF_REC"]:h["OFF_REC"] + P]
    A = plan[h["OFF_A"]:h["OFF_A"] + P * xpad].reshape(P, xpad).astype(np.int64)
    B = plan[h["OFF_B"]:h["OFF_B"] + P * zpad].reshape(P, zpad).astype(np.int64)
    lo = plan[h["OFF_LO"]:h["OFF_LO"] + nxt * nzt * P].reshape(nxt * nzt, P).astype(np.int64)
    xr = np.minimum(np.arange(xpad), w.X - 1)
    zr = np.minimum(np.arange(zpad), w.Z - 1)
    for q, p in enumerate(order):
        i, o, s = sel["pairs"][p]
        assert rec[q] == i * Md + o
        assert q >= sets[s] and q < sets[s + 1]
        assert np.array_equal(A[q], ora["lut1"][i, xr].astype(np.int64) + ora["lut3"][o, xr] + ora["t0_q"])
        assert np.array_equal(B[q], ora["lut2"][i, zr].astype(np.int64) + ora["lut4"][o, zr])
    for t in range(nxt * nzt):
        zt, xt = divmod(t, nxt)
        a = A[:, xt * 64:(xt + 1) * 64]
        b = B[:, zt * 16:(zt + 1) * 16]
        idx = (a[:, :, None] + b[:, None, :]) >> 16              # [P][64][16]
        rel = idx - lo[t][:, None, None]
        assert rel.min() >= 0 and rel.max() <= cap - 1
        assert rel.min(axis=(1, 2)).max() == 0                     # lo is exact
    _check_split(h, nxt * nzt * S, int(np.diff(sets).min()))
    need = kk.beamform_workspace_bytes(plan)
    assert need == (0 if h["SPLIT"] == 1 else h["SPLIT"] * S * w.X * w.Z * 8)


# "full": one set over a 128-angle bank, fewer (set, tile) units than CUs, so pairs are split
@pytest.mark.parametrize("wname", ["tiny", "vernier", "full"])
def test_kk_plan_windows_cover_every_delay(wname):
    w = C.WORKLOADS[wname]
    sel, ora, lib, g, gr = _both_luts(w)
    plan = kk.beamform_plan(sel["pairs"], sel["S"], w.N, len(sel["rx_theta"]), w.T, lib, gr)
    _check_kk_plan(plan, sel, ora, w)


def test_kk_plan_ragged_grid_and_start_time():
    w = C.TINY
    from dataclasses import replace
    w2 = replace(w, X=70, Z=37, t0=2e-6)
    sel, ora, lib, g, gr = _both_luts(w2, scheme=O.SHIFTED, M=5, jl=(0, 1, 2))
    plan = kk.beamform_plan(sel["pairs"], sel["S"], w2.N, len(sel["rx_theta"]), w2.T, lib, gr)
    _check_kk_plan(plan, sel, ora, w2)


def test_kk_plan_errors():
    w = C.TINY
    sel, _, lib, g, gr = _both_luts(w)
    Md = len(sel["rx_theta"])
    bad = np.array(sel["pairs"], dtype=np.int32)
    bad[3, 1] = Md
    with pytest.raises(kk.KKError) as e:
        kk.beamform_plan(bad, sel["S"], w.N, Md, w.T, lib, gr)
    assert e.value.status == kk.KK_E_ARG
    with pytest.raises(kk.KKError) as e:     # set 1 declared but empty
        kk.beamform_plan(sel["pairs"], 2, w.N, Md, w.T, lib, gr)
    assert e.value.status == kk.KK_E_ARG
    # a grid so coarse that a tile spans more record than any window slot holds
    coarse = kk.grid(w.X, w.Z, w.x0, 40 * w.dx, w.z0, 40 * w.dz)
    l2 = kk.build_luts(g, coarse, sel["tx_theta"], sel["rx_theta"])
    with pytest.raises(kk.KKError) as e:
        kk.beamform_plan(sel["pairs"], sel["S"], w.N, Md, w.T, l2, coarse)
    assert e.value.status == kk.KK_E_UNSUPPORTED


def test_das_plan_windows_cover_every_delay():
    w = C.TINY
    sel, ora, lib, g, gr = _both_luts(w)
    rx = kk.build_das_rx(g, gr)
    plan = kk.das_plan(w.N, g, lib, rx, gr)
    h = _hdr(plan)
    assert h["KIND"] == 1 and h["TOTAL"] == plan.size and h["MAXW"] <= h["CAP"]
    N, L = w.N, w.L
    nxt, nzt, xpad, zpad = h["NXT"], h["NZT"], h["XPAD"], h["ZPAD"]
    P = N * L
    A = plan[h["OFF_A"]:h["OFF_A"] + N * xpad].reshape(N, xpad).astype(np.int64)
    B = plan[h["OFF_B"]:h["OFF_B"] + N * zpad].reshape(N, zpad).astype(np.int64)
    Cc = plan[h["OFF_C"]:h["OFF_C"] + L * zpad * xpad].reshape(L, zpad, xpad).astype(np.int64)
    lo = plan[h["OFF_LO"]:h["OFF_LO"] + nxt * nzt * P].reshape(nxt * nzt, P).astype(np.int64)
    rec = plan[h["OFF_REC"]:h["OFF_REC"] + P]
    txr = plan[h["OFF_TX"]:h["OFF_TX"] + P]
    xr = np.minimum(np.arange(xpad), w.X - 1)
    zr = np.minimum(np.arange(zpad), w.Z - 1)
    assert np.array_equal(Cc, np.transpose(rx[xr][:, :, zr], (1, 2, 0)))
    for i in range(N):
        assert np.array_equal(A[i], ora["lut1"][i, xr].astype(np.int64) + ora["t0_q"])
        assert np.array_equal(B[i], ora["lut2"][i, zr])
    for p in range(P):
        l, i = divmod(p, N)
        assert rec[p] == i * L + l and txr[p] == i
    for t in range(nxt * nzt):
        zt, xt = divmod(t, nxt)
        for p in range(P):
            l, i = divmod(p, N)
            q = (A[i, xt * 64:(xt + 1) * 64][None, :] + B[i, zt * 16:(zt + 1) * 16][:, None]
                 + Cc[l, zt * 16:(zt + 1) * 16, xt * 64:(xt + 1) * 64])
            rel = (q >> 16) - lo[t, p]
            assert rel.min() == 0 and rel.max() <= h["CAP"] - 1
    _check_split(h, nxt * nzt, P)
    need = kk.das_workspace_bytes(g, N, plan)
    part = 0 if h["SPLIT"] == 1 else h["SPLIT"] * w.X * w.Z * 8
    assert need >= part + N * L * w.T * 8 and need > 0
