"""Geometry of the linear array, transmit plane waves and image grid (oracle).

Sec. II-A/B: the array lies at z = 0; transmit tilt angles are uniform in
[-theta_max, theta_max] with step delta_theta_i = 2 theta_max / (N - 1).

Readings fixed here (the paper does not state them):
  * element coordinate u_l = ((2l - (L-1)) pitch) / 2, l = 0..L-1: origin at the array
    centre (Eq. 3's edge references u_1 / u_L become u_0 / u_{L-1} in 0-based indexing);
  * theta_i = ((2i - (N-1)) theta_max) / (N-1), i = 0..N-1, evaluated in that order in FP64;
  * pixel coordinates x_k = x0 + k dx and z_k = z0 + k dz in FP64.
"""
from __future__ import annotations


def element_positions(L: int, pitch: float) -> list[float]:
    """u_l, metres, array centred on x = 0."""
    return [((2 * l - (L - 1)) * pitch) / 2.0 for l in range(L)]


def tx_angles(N: int, theta_max: float) -> list[float]:
    """Uniform transmit tilt angles (radians), Sec. II-B (delta_theta_i = 2 theta_max/(N-1))."""
    if N < 2:
        raise ValueError("need N >= 2 transmit angles")
    return [(float(2 * i - (N - 1)) * theta_max) / float(N - 1) for i in range(N)]


def tx_step(N: int, theta_max: float) -> float:
    """delta_theta_i = 2 theta_max / (N - 1), Sec. II-B."""
    return (2.0 * theta_max) / float(N - 1)


def grid_axis(n: int, origin: float, step: float) -> list[float]:
    return [origin + k * step for k in range(n)]


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p
