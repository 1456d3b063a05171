"""Delay-gather beamforming: Eq. 5 (KK) and Eq. 4 (DAS) (oracle).

KK, Eq. 5: B(r) = sum over pairs (theta_i, theta_o) of RF_theta(theta_o, tau_in + tau_out)
with tau_in from LUT1 + LUT2 and tau_out from LUT3 + LUT4 (receive reading in luts.py);
one image per set s (Eq. 8/9 compound the sets).  DAS, Eq. 4: B(r) = sum over
(theta_i, u_l) of the analytic RF_u(u_l, tau_in + tau_out) with tau_out from the receive
table.  Sample n of a record is time t0 + n/fs, so t0_q is added to every delay.

Sample lookup (the paper states only that delays come from tables): linear
interpolation of the complex record with zero outside [0, T).  For a Q16.16 delay q:
  idx = floor(q / 65536), w = (q mod 65536) / 65536,
  v = (1 - w) R[idx] + w R[idx + 1].
"""
from __future__ import annotations

import numpy as np

INT32_MIN, INT32_MAX = -(2 ** 31), 2 ** 31 - 1


def lerp_gather(R: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Linear interpolation of the complex record R[T] at Q16.16 sample positions q."""
    q = np.asarray(q, dtype=np.int64)
    T = R.shape[0]
    idx = q >> 16
    w = (q & 0xFFFF).astype(np.float64) / 65536.0

    def at(n):
        ok = (n >= 0) & (n < T)
        return np.where(ok, R[np.clip(n, 0, T - 1)], 0.0)

    return (1.0 - w) * at(idx) + w * at(idx + 1)


def _pixels(X, Z, pixels):
    if pixels is None:
        xi = np.repeat(np.arange(X), Z)
        zi = np.tile(np.arange(Z), X)
    else:
        xi, zi = (np.asarray(a, dtype=np.int64) for a in pixels)
    return xi, zi


def kk_beamform(rf_theta: np.ndarray, pairs, S: int, lut1, lut2, lut3, lut4, t0_q: int,
                X: int, Z: int, pixels=None) -> np.ndarray:
    """Per-set KK images.

    rf_theta complex [N][M][T]; pairs [P][3] = (i, o, s); LUT1 [N][X], LUT2 [N][Z],
    LUT3 [M][X], LUT4 [M][Z].  Returns complex128 [S][X][Z], or [S][npix] for a pixel
    subset given as (x indices, z indices).
    """
    xi, zi = _pixels(X, Z, pixels)
    out = np.zeros((S, xi.shape[0]), dtype=np.complex128)
    l1 = np.asarray(lut1, dtype=np.int64)
    l2 = np.asarray(lut2, dtype=np.int64)
    l3 = np.asarray(lut3, dtype=np.int64)
    l4 = np.asarray(lut4, dtype=np.int64)
    for (i, o, s) in np.asarray(pairs).reshape(-1, 3):
        q = l1[i, xi] + l2[i, zi] + l3[o, xi] + l4[o, zi] + int(t0_q)
        if q.size and (q.max() > INT32_MAX or q.min() < INT32_MIN):
            raise OverflowError("composite delay outside int32")
        out[s] += lerp_gather(rf_theta[i, o], q)
    return out.reshape(S, X, Z) if pixels is None else out


def das_beamform(rfa: np.ndarray, lut1, lut2, rx, t0_q: int, X: int, Z: int,
                 pixels=None) -> np.ndarray:
    """DAS image (Eq. 4) from the analytic channel data rfa complex [N][L][T] and the
    receive table rx [X][L][Z].  Returns complex128 [X][Z] (or [npix])."""
    xi, zi = _pixels(X, Z, pixels)
    N, L, _ = rfa.shape
    out = np.zeros(xi.shape[0], dtype=np.complex128)
    l1 = np.asarray(lut1, dtype=np.int64)
    l2 = np.asarray(lut2, dtype=np.int64)
    rx = np.asarray(rx)
    for l in range(L):
        r = rx[xi, l, zi].astype(np.int64)
        for i in range(N):
            q = l1[i, xi] + l2[i, zi] + r + int(t0_q)
            if q.size and (q.max() > INT32_MAX or q.min() < INT32_MIN):
                raise OverflowError("composite delay outside int32")
            out += lerp_gather(rfa[i, l], q)
    return out.reshape(X, Z) if pixels is None else out
