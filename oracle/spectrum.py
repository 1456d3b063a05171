"""Analytic (Hilbert) spectrum and inverse transform (oracle).

Sec. II-F: the RF data are made complex by a Hilbert transform computed as a temporal
Fourier transform with the negative frequencies set to zero.  Reading fixed here: the
one-sided mask that keeps the real part equal to the input (DC x1, bins 1..T'/2-1 x2,
Nyquist x1, negative bins 0), on the record zero-padded to the FFT length T'.

  A[k] = H[k] * sum_{n<T} x[n] exp(-2 pi i k n / T'),   k = 0..T'/2
  inverse: y[n] = (1/T') sum_{k=0}^{T'/2} Y[k] exp(+2 pi i k n / T'),   n = 0..T-1

numpy's FFT (pocketfft, FP64) is the transform primitive.
"""
from __future__ import annotations

import numpy as np


def analytic_mask(tpad: int) -> np.ndarray:
    K = tpad // 2 + 1
    h = np.full(K, 2.0)
    h[0] = 1.0
    h[-1] = 1.0
    return h


def analytic_spectrum(rf: np.ndarray, tpad: int) -> np.ndarray:
    """rf[..., T] (any real dtype) -> A[..., T'/2 + 1] complex128."""
    x = np.asarray(rf, dtype=np.float64)
    if x.shape[-1] > tpad:
        raise ValueError("record longer than the FFT length")
    X = np.fft.rfft(x, n=tpad, axis=-1)
    return X * analytic_mask(tpad)


def inverse_bins(Y: np.ndarray, tpad: int, T: int) -> np.ndarray:
    """Y[..., T'/2 + 1] (non-negative bins only) -> y[..., T] complex128."""
    full = np.zeros(Y.shape[:-1] + (tpad,), dtype=np.complex128)
    full[..., : tpad // 2 + 1] = Y
    return np.fft.ifft(full, axis=-1)[..., :T]


def analytic_signal(rf: np.ndarray, tpad: int) -> np.ndarray:
    """Complex analytic record, first T samples (Eq. 4's RF_u made complex)."""
    T = rf.shape[-1]
    return inverse_bins(analytic_spectrum(rf, tpad), tpad, T)
