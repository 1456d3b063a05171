"""One acquisition end to end from the oracle's own selection and tables (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  This module composes the other
oracle steps and holds no arithmetic of its own:

  tables(w)          pair selection (Eq. 6 / Eq. 7 / same-angle / uniform bank, Sec. II-C/D)
                     and the delay and shear tables (Sec. II-F) of one acquisition;
  kk_image(rf, ...)  Eq. 3 decomposition followed by the Eq. 5 gather, per set;
  das_image(rf, ...) the analytic channel data followed by the Eq. 4 gather.

`w` is any object with the acquisition's attributes (L, T, N, pitch, c, fs, t0,
theta_max, scheme, M, j_list, X, Z, x0, dx, z0, dz); nothing here imports the library.
"""
from __future__ import annotations

from .beamform import das_beamform, kk_beamform
from .decompose import decompose
from .luts import build_luts, das_rx_table
from .selection import select_pairs
from .spectrum import analytic_signal


def tables(w, scheme=None, M=None, j_list=None) -> tuple[dict, dict]:
    """(selection, tables) of one acquisition; scheme, M and j_list override w's."""
    sel = select_pairs(w.scheme if scheme is None else scheme, w.L, w.N, w.theta_max,
                       w.M if M is None else M, w.j_list if j_list is None else j_list)
    luts = build_luts(w.L, w.T, w.pitch, w.c, w.fs, w.t0, w.X, w.Z, w.x0, w.dx, w.z0, w.dz,
                      sel["tx_theta"], sel["rx_theta"])
    return sel, luts


def kk_image(rf, sel: dict, luts: dict, X: int, Z: int, pixels=None, rf_theta=None):
    """Per-set KK images complex128 [S][X][Z] (or [S][npix]) of int16 channel data rf
    [N][L][T]; rf_theta, when given, replaces the decomposition (an already computed
    Eq. 3 output of the same tables)."""
    R = decompose(rf, luts["shift"], luts["tpad"]) if rf_theta is None else rf_theta
    return kk_beamform(R, sel["pairs"], sel["S"], luts["lut1"], luts["lut2"], luts["lut3"], luts["lut4"],
                       luts["t0_q"], X, Z, pixels=pixels)


def das_tables(w) -> dict:
    """Transmit tables (LUT1, LUT2, t0_q) and the receive table of Eq. 4."""
    _, luts = tables(w)
    luts = dict(luts)
    luts["rx"] = das_rx_table(w.L, w.pitch, w.c, w.fs, w.X, w.Z, w.x0, w.dx, w.z0, w.dz)
    return luts


def das_image(rf, luts: dict, X: int, Z: int, pixels=None):
    """DAS image complex128 [X][Z] (or [npix]); the analytic records use the DAS FFT length
    (smallest power of two >= T)."""
    T = rf.shape[-1]
    tp = 1
    while tp < T:
        tp *= 2
    rfa = analytic_signal(rf, tp)
    return das_beamform(rfa, luts["lut1"], luts["lut2"], luts["rx"], luts["t0_q"], X, Z, pixels=pixels)
