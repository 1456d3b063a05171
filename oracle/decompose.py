"""Receive plane-wave decomposition, Eq. 3 (oracle).

RF_theta(theta_o, t) = sum_l RF_u(u_l, t + d_l sin(theta_o)/c), performed as Sec. II-F
describes: in the temporal-frequency domain by the Fourier shift theorem, on the analytic
spectrum.  A time advance by s samples multiplies bin k by exp(+2 pi i k s / T').

The advance s[o][l] is the Q.22 integer of the shear table, so the phase in turns is
r / (T' 2^22) with r = (k s) mod (T' 2^22) taken exactly in integers; the sum over l of
Eq. 3 is a plain sum (no 1/L).

  Y[i][o][k] = sum_l A[i][l][k] exp(2 pi i r[o][l][k] / (T' 2^22))
  RF_theta[i][o][n] = (1/T') sum_{k<=T'/2} Y[i][o][k] exp(+2 pi i k n / T'),  n < T
"""
from __future__ import annotations

import numpy as np

from .spectrum import analytic_spectrum, inverse_bins

Q22_BITS = 22


def shear_phases(shift: np.ndarray, tpad: int) -> np.ndarray:
    """W[o][l][k] = exp(2 pi i ((k s) mod (T' 2^22)) / (T' 2^22)), complex128."""
    K = tpad // 2 + 1
    period = np.int64(tpad) << np.int64(Q22_BITS)
    k = np.arange(K, dtype=np.int64)
    r = (k[None, None, :] * shift.astype(np.int64)[:, :, None]) % period
    turns = r.astype(np.float64) / float(period)
    return np.exp(2j * np.pi * turns)


def decompose(rf: np.ndarray, shift: np.ndarray, tpad: int) -> np.ndarray:
    """rf int16 [N][L][T], shift int32 [M][L] -> RF_theta complex128 [N][M][T]."""
    N, L, T = rf.shape
    M = shift.shape[0]
    if shift.shape[1] != L:
        raise ValueError("shear table does not match the element count")
    A = analytic_spectrum(rf, tpad)                      # [N][L][K]
    out = np.empty((N, M, T), dtype=np.complex128)
    for o in range(M):
        W = shear_phases(shift[o:o + 1], tpad)[0]        # [L][K]
        Y = (A * W[None, :, :]).sum(axis=1)              # [N][K]
        out[:, o, :] = inverse_bins(Y, tpad, T)
    return out


def decompose_spectrum(rf: np.ndarray, shift: np.ndarray, tpad: int) -> np.ndarray:
    """The per-bin contraction output Y[i][o][k] before the inverse transform."""
    A = analytic_spectrum(rf, tpad)
    Y = np.empty((rf.shape[0], shift.shape[0], tpad // 2 + 1), dtype=np.complex128)
    for o in range(shift.shape[0]):
        W = shear_phases(shift[o:o + 1], tpad)[0]
        Y[:, o, :] = (A * W[None, :, :]).sum(axis=1)
    return Y
