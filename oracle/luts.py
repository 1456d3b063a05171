"""Delay look-up tables and the integer shear table (oracle).

Sec. II-F ("Computational Implementation") splits the delays into separable tables:
LUT1 = x sin(theta_i)/c and LUT2 = z cos(theta_i)/c (together tau_in of Eq. 4/5), LUT3 /
LUT4 the receive analogues with theta_o, and for DAS a receive table
sqrt((x - u_l)^2 + z^2)/c.  Here every table holds delays in samples as Q16.16
fixed point, so any sum of table entries is an exact integer add.

Receive delay of Eq. 5.  Eq. 3 advances element l by d_l sin(theta_o)/c with
d_l = u_l - u_0 for theta_o > 0 and d_l = u_l - u_{L-1} for theta_o < 0.  A scatterer at
r then appears in RF_theta at tau_in + [z cos(theta_o) - (x - x_ref) sin(theta_o)]/c
(stationary phase over l), with x_ref = u_0 for theta_o >= 0 and u_{L-1} for theta_o < 0.
That is the paper's s_o . r / c with theta_o mirrored and the origin moved to the
reference edge; it is the reading used here (the printed Eq. 3 and Eq. 5 disagree in sign).

Exact operation order (FP64, no contraction), rint = round half to even:
  LUT1[i][x] = rint(((x_k sin th_i) / c) fs 65536)
  LUT2[i][z] = rint(((z_k cos th_i) / c) fs 65536)
  LUT3[o][x] = rint(((-(x_k - x_ref(o)) sin th_o) / c) fs 65536)
  LUT4[o][z] = rint(((z_k cos th_o) / c) fs 65536)
  t0_q       = rint((-t0) fs 65536)              (sample n is time t0 + n / fs)
  shift[o][l] = rint(((d_l sin th_o) / c) fs 2^22) (Q.22 samples, >= 0)
  rx[x][l][z] = rint((sqrt(dx dx + z_k z_k) / c) fs 65536), dx = x_k - u_l
The products "fs 65536" are evaluated left to right: ((v * fs) * 65536).
sin / cos come from libm (Python's math module), sqrt is correctly rounded.

FFT length (Sec. II-F, Fourier shift): T' is the smallest power of two >= T + S_max with
S_max = ceil(max shift / 2^22), so every advanced read past the record sees zero padding.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import element_positions, grid_axis, next_pow2

Q16 = 65536.0
Q22 = 4194304.0
INT32_MIN, INT32_MAX = -(2 ** 31), 2 ** 31 - 1


def _rint(v: float) -> int:
    """Round half to even (Python's round on floats)."""
    return int(round(v))


def _check32(v: int) -> int:
    if not (INT32_MIN <= v <= INT32_MAX):
        raise OverflowError("delay outside int32")
    return v


def x_reference(theta_o: float, u: list[float]) -> float:
    return u[0] if theta_o >= 0.0 else u[-1]


def shear_table(L: int, pitch: float, c: float, fs: float, rx_theta) -> list[list[int]]:
    """shift[o][l] in Q.22 samples (Eq. 3)."""
    u = element_positions(L, pitch)
    out = []
    for th in rx_theta:
        s = math.sin(th)
        if th > 0.0:
            ref = u[0]
        elif th < 0.0:
            ref = u[L - 1]
        else:
            ref = 0.0
        row = []
        for l in range(L):
            d = u[l] - ref
            row.append(_check32(_rint((((d * s) / c) * fs) * Q22)))
        out.append(row)
    return out


def fft_length(T: int, shift) -> int:
    smax_q = max((max(r) for r in shift), default=0)
    smax_q = max(smax_q, 0)
    s_max = (smax_q + (1 << 22) - 1) >> 22
    return next_pow2(T + s_max)


def build_luts(L, T, pitch, c, fs, t0, X, Z, x0, dx, z0, dz, tx_theta, rx_theta) -> dict:
    """LUT1..LUT4, t0_q, shear table and FFT length (int tables as numpy int32)."""
    u = element_positions(L, pitch)
    xs = grid_axis(X, x0, dx)
    zs = grid_axis(Z, z0, dz)
    lut1 = [[_check32(_rint((((x * math.sin(th)) / c) * fs) * Q16)) for x in xs] for th in tx_theta]
    lut2 = [[_check32(_rint((((z * math.cos(th)) / c) * fs) * Q16)) for z in zs] for th in tx_theta]
    lut3 = []
    for th in rx_theta:
        xr = x_reference(th, u)
        s = math.sin(th)
        lut3.append([_check32(_rint((((-(x - xr) * s) / c) * fs) * Q16)) for x in xs])
    lut4 = [[_check32(_rint((((z * math.cos(th)) / c) * fs) * Q16)) for z in zs] for th in rx_theta]
    t0_q = _check32(_rint(((-t0) * fs) * Q16))
    shift = shear_table(L, pitch, c, fs, rx_theta)
    return dict(
        lut1=np.array(lut1, dtype=np.int32).reshape(len(tx_theta), X),
        lut2=np.array(lut2, dtype=np.int32).reshape(len(tx_theta), Z),
        lut3=np.array(lut3, dtype=np.int32).reshape(len(rx_theta), X),
        lut4=np.array(lut4, dtype=np.int32).reshape(len(rx_theta), Z),
        t0_q=t0_q,
        shift=np.array(shift, dtype=np.int32).reshape(len(rx_theta), L),
        tpad=fft_length(T, shift),
    )


def das_rx_table(L, pitch, c, fs, X, Z, x0, dx, z0, dz) -> np.ndarray:
    """DAS receive delays rx[x][l][z] (Eq. 4's tau_out), Q16.16 int32.

    Elementwise numpy IEEE operations in the stated order; identical per element to the
    scalar definition (no trigonometry is involved)."""
    u = np.array(element_positions(L, pitch), dtype=np.float64)
    xs = np.array(grid_axis(X, x0, dx), dtype=np.float64)
    zs = np.array(grid_axis(Z, z0, dz), dtype=np.float64)
    d = xs[:, None, None] - u[None, :, None]
    zz = zs[None, None, :]
    r = np.sqrt(d * d + zz * zz)
    v = np.rint(((r / c) * fs) * Q16)
    if v.size and (v.max() > INT32_MAX or v.min() < INT32_MIN):
        raise OverflowError("delay outside int32")
    return v.astype(np.int32)
