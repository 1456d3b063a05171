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
  ensemble  frames of uneven shapes (ensemble_workloads): each draws 64-192 elements,
            15-75 transmits, J = 1-3 Eq. 6 sets with odd M giving 4-16x compression, and a
            grid from 128 x 256 to 384 x 768 pixels with a record long enough for its depth;
            all frames image one moving speckle medium (ensemble_dataset).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

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


# ----------------------------------------------------------------------------- ensembles

ENSEMBLE_PITCH = 0.3e-3
ENSEMBLE_C = 1540.0
ENSEMBLE_FS = 20e6
ENSEMBLE_FC = 5e6


def ensemble_workloads(n_frames: int = 200, seed: int = 4000, L_range=(64, 192), N_range=(15, 75),
                       scale_range=(1.0, 3.0), compression=(4.0, 16.0)) -> list:
    """Seeded frame shapes of a batched ensemble.  Per frame: L and N uniform integers; the
    transmit half range uniform in 10-18 deg; J uniform in 1..3 Eq. 6 sets with j spread over
    0..floor(N/2); M odd with L / (J M) inside the compression range; a grid of 128 s lateral x
    256 s axial pixels at lambda/2 (s uniform in scale_range), x centred, from z = 0; T covers
    the grid depth (4 samples per axial pixel at fs = 4 fc) plus 128 samples, rounded up to 64."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_frames):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        th = float(rng.uniform(10.0, 18.0))
        J = int(rng.integers(1, 4))
        lo, hi = L / (compression[1] * J), L / (compression[0] * J)
        Ms = [m for m in range(1, 4 * L, 2) if lo <= m <= hi]
        if not Ms:
            Ms = [max(1, int(round(hi)) | 1)]
        M = int(Ms[int(rng.integers(0, len(Ms)))])
        half = N // 2
        j_list = tuple(sorted({(k * half) // (J - 1) for k in range(J)})) if J > 1 else (0,)
        s = float(rng.uniform(scale_range[0], scale_range[1]))
        X = max(16, int(round(128 * s)))
        Z = max(16, int(round(256 * s)))
        T = (4 * Z + 128 + 63) // 64 * 64
        out.append(Workload("ensemble%d" % f, L=L, T=T, N=N, pitch=ENSEMBLE_PITCH, c=ENSEMBLE_C, fs=ENSEMBLE_FS,
                            fc=ENSEMBLE_FC, theta_max_deg=th, scheme=SCHEME_SHIFTED, M=M, j_list=j_list, X=X, Z=Z,
                            z0=0.0))
    return out


def ensemble_medium(workloads, seed: int = 4001, per_lambda2: float = 0.5, max_step: float = 50e-6):
    """One speckle medium covering every frame's field: uniform positions, N(0,1) amplitudes,
    per_lambda2 scatterers per lambda^2, and a velocity per scatterer of uniform direction and
    speed uniform in [0, max_step] per frame.  Returns (x, z, a, vx, vz)."""
    lam = ENSEMBLE_C / ENSEMBLE_FC
    half = max(max((w.L - 1) * w.pitch / 2.0 + w.pitch / 2.0, (w.X - 1) * w.dx / 2.0) for w in workloads)
    depth = max(w.T * w.c / (2.0 * w.fs) for w in workloads)
    area = 2 * half * depth
    n = max(1, int(round(per_lambda2 * area / (lam * lam))))
    rng = np.random.default_rng(seed)
    x = rng.uniform(-half, half, n)
    z = rng.uniform(1e-3, depth, n)
    a = rng.standard_normal(n)
    sp = rng.uniform(0.0, max_step, n)
    ang = rng.uniform(0.0, 2 * math.pi, n)
    return x, z, a, sp * np.cos(ang), sp * np.sin(ang)


def ensemble_dataset(w: Workload, medium, frame: int) -> Dataset:
    """Channel data of frame `frame` of the ensemble: the medium moved by `frame` steps, the
    scatterers inside this frame's field (its aperture or grid, whichever is wider, plus 5 mm,
    and its record depth)."""
    from .phantom import Scatterers
    x, z, a, vx, vz = medium
    xf, zf = x + frame * vx, z + frame * vz
    half = max((w.L - 1) * w.pitch / 2.0 + w.pitch / 2.0, (w.X - 1) * w.dx / 2.0) + 5e-3
    depth = w.T * w.c / (2.0 * w.fs)
    keep = (np.abs(xf) <= half) & (zf > 0) & (zf <= depth)
    sc = Scatterers(xf[keep].copy(), zf[keep].copy(), a[keep].copy())
    return make_dataset(w.acquisition(), sc, meta=dict(workload=w.name, frame=frame))
