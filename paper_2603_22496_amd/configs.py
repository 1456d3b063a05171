"""Workload definitions: synthetic linear-array plane-wave acquisitions and image grids.

Shapes follow the linear-array CPWC acquisitions of the paper (Table I: 192-element
probe, ~5 MHz centre frequency, ~20 MHz sampling, 2048-2944 samples per trace), scaled
to the sizes below.  Every phantom is drawn from a seeded PCG64 generator.

  tiny      16 elements, pitch 0.3 mm, 1024 samples, 5 transmits in +-10 deg, 3 seeded
            point scatterers (1.0, 0.5, 0.25) at depth 10-30 mm; 16 uniform receive
            angles over +-15 deg, all 80 pairs; 64 x 64 pixels at lambda/2 from z = 10 mm.
  vernier   128 elements, pitch 0.3 mm, 2048 samples, 31 transmits in +-15 deg; two
            shifted-vernier sets (Eq. 6, j = 0 and 15, M = 7 each; 434 pair slots,
            9.14x compression); 1e5-scatterer speckle, 8 point targets and a 2 mm
            anechoic cyst; 256 lateral x 512 axial pixels at lambda/2 from z = 0.
  full      same data, 128 uniform receive angles over +-16 deg, all 3968 pairs.
  large     192 elements, 4096 samples, 75 transmits in +-18 deg; Eq. 6 sets j = 0, 37
            with M = 9 (1350 pair slots, 10.7x); 384 x 768 pixels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from .phantom import Acquisition, Dataset, make_dataset, seeded_points, speckle_phantom

SCHEME_SHIFTED = 0      # Eq. 6, one set per entry of the j list
SCHEME_CONFOCAL = 1     # Eq. 7
SCHEME_SAME = 2         # receive angles = transmit angles
SCHEME_FULL_UNIFORM = 3 # M angles uniform over +-(theta_max + transmit step)


@dataclass(frozen=True)
class Workload:
    name: str
    L: int
    T: int
    N: int
    pitch: float
    c: float
    fs: float
    fc: float
    theta_max_deg: float
    scheme: int
    M: int
    j_list: tuple
    X: int                  # lateral pixels
    Z: int                  # axial pixels
    z0: float
    t0: float = 0.0

    @property
    def theta_max(self) -> float:
        return math.radians(self.theta_max_deg)

    @property
    def wavelength(self) -> float:
        return self.c / self.fc

    @property
    def dx(self) -> float:
        return self.wavelength / 2.0

    @property
    def dz(self) -> float:
        return self.wavelength / 2.0

    @property
    def x0(self) -> float:
        return -((self.X - 1) * self.dx) / 2.0

    def acquisition(self) -> Acquisition:
        return Acquisition(L=self.L, T=self.T, N=self.N, pitch=self.pitch, c=self.c, fs=self.fs,
                           fc=self.fc, theta_max=self.theta_max, t0=self.t0)

    def with_selection(self, scheme: int, M: int, j_list=(0,), name=None) -> "Workload":
        d = dict(self.__dict__)
        d.update(scheme=scheme, M=M, j_list=tuple(j_list), name=name or self.name)
        return Workload(**d)


TINY = Workload("tiny", L=16, T=1024, N=5, pitch=0.3e-3, c=1540.0, fs=20e6, fc=5e6,
                theta_max_deg=10.0, scheme=SCHEME_FULL_UNIFORM, M=16, j_list=(0,),
                X=64, Z=64, z0=10e-3)

VERNIER = Workload("vernier", L=128, T=2048, N=31, pitch=0.3e-3, c=1540.0, fs=20e6, fc=5e6,
                   theta_max_deg=15.0, scheme=SCHEME_SHIFTED, M=7, j_list=(0, 15),
                   X=256, Z=512, z0=0.0)

FULL = VERNIER.with_selection(SCHEME_FULL_UNIFORM, 128, (0,), name="full")

LARGE = Workload("large", L=192, T=4096, N=75, pitch=0.3e-3, c=1540.0, fs=20e6, fc=5e6,
                 theta_max_deg=18.0, scheme=SCHEME_SHIFTED, M=9, j_list=(0, 37),
                 X=384, Z=768, z0=0.0)

WORKLOADS = {w.name: w for w in (TINY, VERNIER, FULL, LARGE)}


def tiny_dataset(seed: int = 0) -> Dataset:
    """Three seeded point scatterers, amplitudes 1.0 / 0.5 / 0.25, depth 10-30 mm."""
    w = TINY
    return make_dataset(w.acquisition(), seeded_points(seed), meta=dict(workload=w.name, seed=seed))


def speckle_dataset(w: Workload, seed: int = 2, n_scat: int = 100_000) -> Dataset:
    """Speckle (uniform positions, N(0,1) amplitudes, ~3 per lambda^2 at 1e5 over the
    field), 8 point targets of amplitude 10 at x = -8 mm, z = 10..70 mm, and an anechoic
    cyst of radius 2 mm at (0, 40 mm) scaled to the record depth."""
    half_ap = (w.L - 1) * w.pitch / 2.0 + w.pitch / 2.0
    depth = w.T * w.c / (2.0 * w.fs)
    zc = 40e-3 * depth / 78.8e-3
    pts = [(-8e-3 * half_ap / 19.2e-3, (10e-3 + k * 60e-3 / 7) * depth / 78.8e-3, 10.0) for k in range(8)]
    sc = speckle_phantom(seed, n_scat, (-half_ap, half_ap), (1e-3, depth - 0.8e-3),
                         points=pts, cysts=[(0.0, zc, 2e-3)])
    return make_dataset(w.acquisition(), sc, meta=dict(workload=w.name, seed=seed, n_scat=n_scat))
