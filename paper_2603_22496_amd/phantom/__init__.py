"""Seeded synthetic phantoms and int16 channel data for linear-array plane-wave imaging.

This module is the shared input generator: it draws scatterers and simulates what a
linear array records, and it holds none of the beamforming method's arithmetic (no
angle selection, delay tables, decomposition or beamforming).  Acquisition parameters
(element positions, transmit angles) are computed here from their physical definition
and passed to the forward model explicitly.

Forward model (far-field plane-wave transmit, spherical receive, no attenuation or
directivity), evaluated in FP64 by ``rfsim.c``:

    rf[i][l][n] = sum_s a_s p(t0 + n/fs - (x_s sin th_i + z_s cos th_i)/c - |r_s - (u_l,0)|/c)

Pulse: Gaussian-windowed cosine at fc whose envelope FWHM is ``cycles`` periods,
truncated at 4 sigma.  Quantisation: q = clip(rint(G rf), -32768, 32767) with
G = 16384 / max|rf| unless a gain is given.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rfsim.c")
_LIB = os.path.join(_HERE, "_rfsim.so")
_lib = None


def build_rfsim(force: bool = True) -> str:
    """Compile the forward-model helper with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_rfsim(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.kk_rfsim.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp, dp, dp, dp]
        lib.kk_rfsim.restype = None
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Acquisition:
    """Linear array at z = 0 centred on x = 0, plane-wave transmits uniform in +-theta_max."""
    L: int
    T: int
    N: int
    pitch: float
    c: float
    fs: float
    fc: float
    theta_max: float            # radians
    t0: float = 0.0             # time of sample 0 (s); t = 0 when the wavefront crosses the origin
    cycles: float = 1.5         # envelope FWHM in periods of fc

    def element_x(self) -> np.ndarray:
        return np.array([((2 * l - (self.L - 1)) * self.pitch) / 2.0 for l in range(self.L)])

    def tx_angles(self) -> np.ndarray:
        if self.N == 1:
            return np.zeros(1)
        return np.array([((2 * i - (self.N - 1)) * self.theta_max) / (self.N - 1) for i in range(self.N)])

    def sigma(self) -> float:
        return self.cycles / (self.fc * 2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclass
class Scatterers:
    x: np.ndarray
    z: np.ndarray
    a: np.ndarray

    @staticmethod
    def points(pts) -> "Scatterers":
        arr = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        return Scatterers(arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy())

    def __len__(self):
        return int(self.x.shape[0])


def simulate(acq: Acquisition, sc: Scatterers) -> np.ndarray:
    """FP64 channel data [N][L][T] of the scatterers (before quantisation)."""
    lib = _load()
    out = np.empty((acq.N, acq.L, acq.T), dtype=np.float64)
    th = np.ascontiguousarray(acq.tx_angles(), dtype=np.float64)
    ex = np.ascontiguousarray(acq.element_x(), dtype=np.float64)
    sx = np.ascontiguousarray(sc.x, dtype=np.float64)
    sz = np.ascontiguousarray(sc.z, dtype=np.float64)
    sa = np.ascontiguousarray(sc.a, dtype=np.float64)
    lib.kk_rfsim(acq.N, acq.L, acq.T, _dp(th), _dp(ex), acq.c, acq.fs, acq.t0, acq.fc,
                 acq.sigma(), 4.0, len(sc), _dp(sx), _dp(sz), _dp(sa), _dp(out))
    return out


def quantise(rf: np.ndarray, gain: float | None = None) -> tuple[np.ndarray, float]:
    """int16 channel data; returns (q, gain)."""
    if gain is None:
        peak = float(np.max(np.abs(rf)))
        gain = 16384.0 / peak if peak > 0 else 1.0
    q = np.clip(np.rint(rf * gain), -32768, 32767).astype(np.int16)
    return q, gain


# ----------------------------------------------------------------------------- phantoms

def seeded_points(seed: int, amplitudes=(1.0, 0.5, 0.25), x_range=(-2e-3, 2e-3),
                  z_range=(10e-3, 30e-3)) -> Scatterers:
    rng = np.random.default_rng(seed)
    n = len(amplitudes)
    x = rng.uniform(x_range[0], x_range[1], n)
    z = rng.uniform(z_range[0], z_range[1], n)
    return Scatterers(x, z, np.asarray(amplitudes, dtype=np.float64))


def speckle_phantom(seed: int, n_scat: int, x_range, z_range, points=(), cysts=()) -> Scatterers:
    """Uniform random speckle with N(0,1) amplitudes, anechoic cysts (scatterers removed
    inside each (xc, zc, radius)), plus explicit point targets (x, z, a)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(x_range[0], x_range[1], n_scat)
    z = rng.uniform(z_range[0], z_range[1], n_scat)
    a = rng.standard_normal(n_scat)
    keep = np.ones(n_scat, dtype=bool)
    for (xc, zc, r) in cysts:
        keep &= (x - xc) ** 2 + (z - zc) ** 2 > r * r
    x, z, a = x[keep], z[keep], a[keep]
    if len(points):
        p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
        x = np.concatenate([x, p[:, 0]])
        z = np.concatenate([z, p[:, 1]])
        a = np.concatenate([a, p[:, 2]])
    return Scatterers(x, z, a)


@dataclass
class Dataset:
    acq: Acquisition
    scatterers: Scatterers
    rf: np.ndarray              # int16 [N][L][T]
    gain: float
    meta: dict = field(default_factory=dict)


def make_dataset(acq: Acquisition, sc: Scatterers, gain: float | None = None, meta=None) -> Dataset:
    rf = simulate(acq, sc)
    q, g = quantise(rf, gain)
    return Dataset(acq, sc, q, g, dict(meta or {}))
