"""Receive-angle selection and angle pairs (oracle).

Follows Sec. II-C ("Contrast versus resolution") and Sec. II-D ("Confocal KK
beamforming"):

  Eq. 6  theta_o = sgn(o) dth_i (2|o|/M + j),              o = -floor(M/2)..floor(M/2),
         j an integer in [0, floor(N/2)]; one beamforming set per j.
  Eq. 7  theta_o = sgn(o) dth_i (2|o|/M + mod(|o|, floor(N/2))), one set.
  same   theta_o = theta_i (the redundant strategy of Sec. II-C, kept as a control).
  uniform bank  M angles uniform over +-(theta_max + dth_i) (a "fully sampled" receive
         set; not in the paper, used as the dense reference).

Every angle is carried as an exact rational theta / dth_i = num/den (Python integers), so
de-duplication across sets and ordering are exact.  The FP64 value of an Eq. 6/7 angle is
(n * dth_i) / M with n = sgn(o)(2|o| + j M) (or the Eq. 7 analogue), evaluated in that
order.  Distinct receive angles are sorted by value.  Pairs are listed set by set, within
a set by distinct-angle index, then by transmit index; an angle present in several sets
(theta_o = 0 is in every Eq. 6 set) gives one pair slot per set, because Eq. 8/9 sum the
per-set images.  Compression = L / (J * M_set), Sec. II-C, where M_set is the number of
receive angles per set (2 floor(M/2) + 1 for Eq. 6/7, i.e. M when M is odd).
"""
from __future__ import annotations

import math
from fractions import Fraction

from .geometry import tx_angles, tx_step

SHIFTED, CONFOCAL, SAME, FULL_UNIFORM = 0, 1, 2, 3


def _sgn(o: int) -> int:
    return (o > 0) - (o < 0)


def eq6_numerators(M: int, j: int) -> list[int]:
    """n(o) = sgn(o)(2|o| + j M) so that theta_o = n dth_i / M  (Eq. 6)."""
    h = M // 2
    return [_sgn(o) * (2 * abs(o) + j * M) for o in range(-h, h + 1)]


def eq7_numerators(M: int, N: int) -> list[int]:
    """n(o) = sgn(o)(2|o| + mod(|o|, floor(N/2)) M)  (Eq. 7)."""
    h = M // 2
    hn = N // 2
    return [_sgn(o) * (2 * abs(o) + (abs(o) % hn) * M) for o in range(-h, h + 1)]


def select_pairs(scheme: int, L: int, N: int, theta_max: float, M: int, j_list=(0,)) -> dict:
    """Angle sets and pair list for one acquisition.

    Returns dict(tx_theta[N], rx_theta[Md], rx_num[Md], rx_den[Md], pairs [P][3] = (i, o, s),
    S (number of sets), compression).
    """
    if N < 2 or L < 1 or M < 1:
        raise ValueError("need N >= 2, L >= 1, M >= 1")
    if not (0.0 < theta_max < math.pi / 2):
        raise ValueError("theta_max out of (0, pi/2)")
    tx = tx_angles(N, theta_max)
    dth = tx_step(N, theta_max)

    # each set: list of (exact rational theta/dth_i, FP64 angle)
    sets: list[list[tuple[Fraction, float]]] = []
    if scheme == SHIFTED:
        if len(j_list) < 1:
            raise ValueError("empty j list")
        for j in j_list:
            if not (0 <= j <= N // 2):
                raise ValueError("j must lie in [0, floor(N/2)]")
            sets.append([(Fraction(n, M), (float(n) * dth) / float(M)) for n in eq6_numerators(M, j)])
    elif scheme == CONFOCAL:
        sets.append([(Fraction(n, M), (float(n) * dth) / float(M)) for n in eq7_numerators(M, N)])
    elif scheme == SAME:
        sets.append([(Fraction(2 * i - (N - 1), 2), tx[i]) for i in range(N)])
    elif scheme == FULL_UNIFORM:
        if M < 2:
            raise ValueError("uniform bank needs M >= 2")
        th_hi = theta_max + dth
        sets.append([(Fraction((2 * k - (M - 1)) * (N + 1), 2 * (M - 1)),
                      (float(2 * k - (M - 1)) * th_hi) / float(M - 1)) for k in range(M)])
    else:
        raise ValueError("unknown scheme")

    for st in sets:
        for _, th in st:
            if not (abs(th) < math.pi / 2):
                raise ValueError("receive angle reaches 90 degrees")

    distinct: dict[Fraction, float] = {}
    for st in sets:
        for fr, th in st:
            distinct.setdefault(fr, th)
    keys = sorted(distinct)
    index = {fr: o for o, fr in enumerate(keys)}

    pairs = []
    for s, st in enumerate(sets):
        for o in sorted(index[fr] for fr, _ in st):
            for i in range(N):
                pairs.append((i, o, s))

    m_set = len(sets[0])
    return dict(
        tx_theta=tx,
        rx_theta=[distinct[k] for k in keys],
        rx_num=[k.numerator for k in keys],
        rx_den=[k.denominator for k in keys],
        pairs=pairs,
        S=len(sets),
        compression=L / (len(sets) * m_set),
    )
