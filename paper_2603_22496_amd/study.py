"""Scheme and compounding study on synthetic phantoms (image metrics).

Compares receive-angle schemes (Eq. 6 with j = 0, 3, 6; confocal Eq. 7; Eq. 6 sets j = 0, 3, 6
compounded coherently, Eq. 8, or incoherently, Eq. 9) with conventional CPWC DAS (Eq. 4) on
the same seeded channel data, at two compression levels (M = 7 per set: 27.4x single, 9.1x
compounded or confocal with M = 21; M = 19 per set: 10.1x single, 3.4x compounded or confocal
with M = 57), and for N = 7 and N = 15 transmits (the acquisition / processing trade-off).

Metrics:
  gCNR      generalized contrast-to-noise ratio of an anechoic cyst: 1 minus the overlap of the
            intensity histograms (common bins) inside the cyst and in a background annulus
  FWHM      lateral full width at half maximum of point-target envelopes (linear interpolation
            at the half-maximum crossings)
  k_x       the difference angles dth = th_o - th_i of a pair set (proportional to k_x in the
            paraxial limit, Sec. II-C): support, smallest step and largest multiplicity in units
            of the transmit step, and the correlation of its histogram with a triangle over the
            same support (the DAS transfer function the confocal scheme imitates)

Every image comes from the library's GPU path; the metrics are plain numpy.
"""
from __future__ import annotations

import json
import math
import sys
from dataclasses import dataclass, replace

import numpy as np

from . import configs as C
from . import kk
from .phantom import Scatterers, make_dataset, speckle_phantom


# ----------------------------------------------------------------------------- metrics

def gcnr(inside: np.ndarray, outside: np.ndarray, bins: int = 200) -> float:
    """1 - sum_b min(p_in(b), p_out(b)) over common histogram bins spanning both samples."""
    a = np.asarray(inside, dtype=np.float64).ravel()
    b = np.asarray(outside, dtype=np.float64).ravel()
    lo, hi = min(a.min(), b.min()), max(a.max(), b.max())
    if hi <= lo:
        return 0.0
    edges = np.linspace(lo, hi, bins + 1)
    pa = np.histogram(a, edges)[0] / a.size
    pb = np.histogram(b, edges)[0] / b.size
    return float(1.0 - np.minimum(pa, pb).sum())


def fwhm(profile: np.ndarray, dx: float) -> float:
    """Full width at half maximum of a single-peaked profile sampled every dx (linear
    interpolation of the two half-maximum crossings around the peak); nan when a crossing is
    outside the profile."""
    p = np.asarray(profile, dtype=np.float64)
    k = int(np.argmax(p))
    half = p[k] / 2.0
    i = k
    while i > 0 and p[i] > half:
        i -= 1
    j = k
    while j < p.size - 1 and p[j] > half:
        j += 1
    if p[i] > half or p[j] > half:
        return float("nan")
    left = i + (half - p[i]) / (p[i + 1] - p[i])
    right = j - 1 + (p[j - 1] - half) / (p[j - 1] - p[j])
    return float((right - left) * dx)


def kx_stats(tx_theta, rx_theta, pairs, dth_i: float) -> dict:
    """Statistics of dth = rx_theta[o] - tx_theta[i] over the (i, o, s) pairs, in units of the
    transmit step dth_i."""
    d = np.array([rx_theta[o] - tx_theta[i] for i, o, _ in np.asarray(pairs)]) / dth_i
    u, cnt = np.unique(np.round(d, 9), return_counts=True)
    steps = np.diff(u)
    support = float(u[-1] - u[0])
    nb = 41
    hist, edges = np.histogram(d, bins=nb, range=(u[0], u[-1] + 1e-12))
    ctr = 0.5 * (edges[:-1] + edges[1:])
    mid = 0.5 * (u[0] + u[-1])
    tri = np.maximum(0.0, 1.0 - np.abs(ctr - mid) / (support / 2.0 + 1e-12))
    h = hist.astype(np.float64)
    corr = float(np.corrcoef(h, tri)[0, 1]) if h.std() > 0 else 0.0
    return dict(pairs=int(len(d)), distinct=int(len(u)), support=support,
                min_step=float(steps.min()) if steps.size else 0.0,
                max_multiplicity=int(cnt.max()), triangle_corr=corr)


# ----------------------------------------------------------------------------- workload

@dataclass(frozen=True)
class StudyGeometry:
    L: int = 192
    pitch: float = 0.23e-3        # the paper's linear probe (Table I)
    c: float = 1540.0
    fc: float = 5.2e6
    fs: float = 20.83e6
    T: int = 2048
    theta_max_deg: float = 12.0   # +-12 deg transmit fan (Fig. 2)
    X: int = 288                  # lateral pixels at lambda / 2
    Z: int = 320                  # axial pixels at lambda / 2 from z0
    z0: float = 8e-3


def workload(g: StudyGeometry, N: int) -> C.Workload:
    return C.Workload("study", L=g.L, T=g.T, N=N, pitch=g.pitch, c=g.c, fs=g.fs, fc=g.fc,
                      theta_max_deg=g.theta_max_deg, scheme=C.SCHEME_SHIFTED, M=7, j_list=(0,), X=g.X, Z=g.Z,
                      z0=g.z0)


CYST = (0.0, 25e-3, 3.5e-3)                       # x, z, radius
POINTS = [(-6e-3, 15e-3), (0.0, 15e-3), (6e-3, 15e-3), (0.0, 38e-3)]


def phantoms(g: StudyGeometry, seed: int = 21, per_lambda2: float = 3.0):
    """(speckle with the anechoic cyst, isolated point targets) scatterers."""
    lam = g.c / g.fc
    half = g.X * lam / 4.0 + 2e-3
    z_lo, z_hi = g.z0 - 2e-3, g.z0 + g.Z * lam / 2.0 + 2e-3
    n = int(per_lambda2 * (2 * half) * (z_hi - z_lo) / (lam * lam))
    sp = speckle_phantom(seed, n, (-half, half), (z_lo, z_hi), cysts=[CYST])
    pts = Scatterers.points([(x, z, 1.0) for x, z in POINTS])
    return sp, pts


# ----------------------------------------------------------------------------- runs

SCHEMES = [
    # name, scheme, M, j list, compounding (None: one set; "coh" / "inc")
    ("KK j=0", C.SCHEME_SHIFTED, 7, (0,), None),
    ("KK j=3", C.SCHEME_SHIFTED, 7, (3,), None),
    ("KK j=6", C.SCHEME_SHIFTED, 7, (6,), None),
    ("KK confocal", C.SCHEME_CONFOCAL, 21, (0,), None),
    ("KK coherent j=0,3,6", C.SCHEME_SHIFTED, 7, (0, 3, 6), "coh"),
    ("KK incoherent j=0,3,6", C.SCHEME_SHIFTED, 7, (0, 3, 6), "inc"),
    ("KK j=0 M19", C.SCHEME_SHIFTED, 19, (0,), None),
    ("KK j=6 M19", C.SCHEME_SHIFTED, 19, (6,), None),
    ("KK confocal M57", C.SCHEME_CONFOCAL, 57, (0,), None),
    ("KK coherent j=0,3,6 M19", C.SCHEME_SHIFTED, 19, (0, 3, 6), "coh"),
    ("KK incoherent j=0,3,6 M19", C.SCHEME_SHIFTED, 19, (0, 3, 6), "inc"),
]


def _masks(w: C.Workload):
    x = w.x0 + w.dx * np.arange(w.X)
    z = w.z0 + w.dz * np.arange(w.Z)
    X, Z = np.meshgrid(x, z, indexing="ij")
    r = np.hypot(X - CYST[0], Z - CYST[1])
    inside = r < 0.8 * CYST[2]
    outside = (r > 1.3 * CYST[2]) & (r < 2.2 * CYST[2])
    return inside, outside


def _metrics(w, inten: np.ndarray, inten_pts: np.ndarray) -> dict:
    inside, outside = _masks(w)
    db = 10 * np.log10(inten / inten.max() + 1e-12)
    widths = []
    for (px, pz) in POINTS:
        zi = int(round((pz - w.z0) / w.dz))
        xi = int(round((px - w.x0) / w.dx))
        zs = slice(max(zi - 3, 0), min(zi + 4, w.Z))
        col = np.sqrt(inten_pts[:, zs]).max(axis=1)   # envelope, axial max near the target depth
        lo, hi = max(xi - 20, 0), min(xi + 21, w.X)   # +-3 mm: the neighbouring targets are 6 mm away
        widths.append(fwhm(col[lo:hi], w.dx) * 1e3)
    return dict(gcnr=round(gcnr(db[inside], db[outside]), 4),
                fwhm_mm=[round(v, 3) for v in widths])


def scaled_j(j_list, N: int):
    """The j = 0, 3, 6 sets of N = 15 scaled to N transmits (j <= floor(N / 2))."""
    return tuple(sorted({min(N // 2, int(round(j * N / 15.0))) for j in j_list}))


def run(N_list=(15, 7), seed: int = 21, log=None, g: StudyGeometry | None = None, schemes=None,
        per_lambda2: float = 3.0) -> dict:
    """The study on the GPU; returns a JSON-ready report."""
    import torch
    g = StudyGeometry() if g is None else g
    schemes = SCHEMES if schemes is None else schemes
    sp, pts = phantoms(g, seed, per_lambda2)
    out = dict(geometry=dict(L=g.L, pitch_mm=g.pitch * 1e3, fc_MHz=g.fc / 1e6, fs_MHz=g.fs / 1e6, T=g.T,
                             theta_max_deg=g.theta_max_deg, grid=[g.X, g.Z], cyst=CYST, points=POINTS,
                             speckle_scatterers=len(sp)), results={})
    for N in N_list:
        w = workload(g, N)
        ds = make_dataset(w.acquisition(), sp)
        dp = make_dataset(w.acquisition(), pts)
        rf, rfp = kk.to_device(ds.rf), kk.to_device(dp.rf)
        res = {}
        # DAS reference on the same data
        su = kk.make_setup(w, with_das=True)
        dplan = kk.to_device(su.das_plan)
        das = kk.das_beamform(rf, su.geom, su.das_plan, dplan)
        dasp = kk.das_beamform(rfp, su.geom, su.das_plan, dplan)
        torch.cuda.synchronize()
        res["DAS"] = dict(compression=1.0, **_metrics(w, np.abs(das.cpu().numpy()) ** 2,
                                                      np.abs(dasp.cpu().numpy()) ** 2))
        for name, scheme, M, jl, comp in schemes:
            jl = scaled_j(jl, N)
            su = kk.make_setup(w, scheme=scheme, M=M, j_list=jl)
            sh, pd = kk.to_device(su.luts["shift"]), kk.to_device(su.plan)
            mode = kk.COMPOUND_INCOHERENT if comp == "inc" else kk.COMPOUND_COHERENT
            ims = []
            for data in (rf, rfp):
                rt = kk.decompose(data, su.geom, sh, su.M, su.tpad)
                inten = torch.empty((w.X, w.Z), dtype=torch.float32, device=rt.device)
                kk.beamform(rt, su.plan, pd, intensity=inten, mode=mode)
                ims.append(inten.cpu().numpy().astype(np.float64))
            dth = 2 * g.theta_max_deg / (N - 1)
            res[name] = dict(compression=round(su.sel["compression"], 2), sets=su.sel["S"], j=list(jl),
                             kx=kx_stats(su.sel["tx_theta"], su.sel["rx_theta"], su.sel["pairs"], math.radians(dth)),
                             **_metrics(w, ims[0], ims[1]))
            if log:
                log("study N=%d %-28s gCNR %.3f FWHM %s" % (N, name, res[name]["gcnr"], res[name]["fwhm_mm"]))
        out["results"]["N=%d" % N] = res
    return out


def main():
    import torch
    torch.cuda.set_device(0)
    rep = run(log=lambda s: print(s, file=sys.stderr, flush=True))
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
