"""Expected values of the GPU parity tests, built from the oracle alone.

Every reference record or image comes from the oracle's own pair selection and delay tables
(oracle.frame).  The library's selection and tables for the same acquisition (the Setup the
GPU side runs with) are compared with them bit for bit first, so a table bug at any geometry
a test draws fails that test instead of entering both sides of the comparison.
"""
from __future__ import annotations

import numpy as np

import oracle as O
from oracle import frame as OF


class OracleTables:
    """The oracle's selection (sel) and tables (luts) of one acquisition."""

    def __init__(self, sel: dict, luts: dict, X: int, Z: int):
        self.sel, self.luts, self.X, self.Z = sel, luts, X, Z

    def decompose(self, rf):
        return O.decompose(rf, self.luts["shift"], self.luts["tpad"])

    def kk_image(self, rf=None, pixels=None, rf_theta=None):
        return OF.kk_image(rf, self.sel, self.luts, self.X, self.Z, pixels=pixels, rf_theta=rf_theta)


def assert_tables_equal(su, sel: dict, luts: dict) -> None:
    """The library's selection and tables (a kk.Setup) equal the oracle's bit for bit."""
    assert su.sel["S"] == sel["S"]
    assert np.array_equal(np.asarray(su.sel["pairs"], dtype=np.int64).reshape(-1, 3),
                          np.asarray(sel["pairs"], dtype=np.int64).reshape(-1, 3)), "pairs"
    for k in ("tx_theta", "rx_theta"):
        a = np.asarray(su.sel[k], dtype=np.float64)
        b = np.asarray(sel[k], dtype=np.float64)
        assert a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64)), k
    for k in ("rx_num", "rx_den"):
        assert np.array_equal(np.asarray(su.sel[k], dtype=np.int64), np.asarray(sel[k], dtype=np.int64)), k
    for k in ("lut1", "lut2", "lut3", "lut4", "shift"):
        assert np.array_equal(np.asarray(su.luts[k]), np.asarray(luts[k])), k
    assert int(su.luts["t0_q"]) == int(luts["t0_q"]) and int(su.tpad) == int(luts["tpad"])


def tables(su, w, scheme=None, M=None, j_list=None) -> OracleTables:
    """The oracle's tables for workload w (with the same overrides the Setup su was built
    with), checked equal to su's."""
    sel, luts = OF.tables(w, scheme, M, j_list)
    assert_tables_equal(su, sel, luts)
    return OracleTables(sel, luts, w.X, w.Z)


def das_tables(w, lib_luts: dict, lib_rx: np.ndarray) -> dict:
    """The oracle's DAS tables for workload w, checked equal to the library's."""
    luts = OF.das_tables(w)
    for k in ("lut1", "lut2"):
        assert np.array_equal(np.asarray(lib_luts[k]), luts[k]), k
    assert int(lib_luts["t0_q"]) == int(luts["t0_q"])
    assert np.array_equal(np.asarray(lib_rx), luts["rx"]), "rx"
    return luts
