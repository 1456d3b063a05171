"""Compounding of per-set images (oracle), Sec. II-C.

Eq. 8 (coherent):   I = | sum_j B^(j) |^2
Eq. 9 (incoherent): I = sum_j | B^(j) |^2
Single image (Sec. II-D, confocal): I = |B|^2
"""
from __future__ import annotations

import numpy as np


def coherent(B: np.ndarray) -> np.ndarray:
    """B complex [S][X][Z] -> I [X][Z]."""
    s = B.sum(axis=0)
    return (s * np.conj(s)).real


def incoherent(B: np.ndarray) -> np.ndarray:
    return (B * np.conj(B)).real.sum(axis=0)


def intensity(B: np.ndarray) -> np.ndarray:
    return (B * np.conj(B)).real
