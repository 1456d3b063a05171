"""High-precision reference arithmetic for pins (Decimal, 50 digits).

Independent of the oracle's FP64 evaluation: sin / cos by Taylor series and sqrt by
Decimal's correctly rounded square root, on the exact values of the FP64 inputs.
"""
from decimal import Decimal, getcontext

getcontext().prec = 50


def D(x) -> Decimal:
    return Decimal(float(x)) if not isinstance(x, Decimal) else x


def dsin(x) -> Decimal:
    x = D(x)
    term, total, n = x, x, 1
    while True:
        term = -term * x * x / ((2 * n) * (2 * n + 1))
        if abs(term) < Decimal(10) ** -48:
            return total
        total += term
        n += 1


def dcos(x) -> Decimal:
    x = D(x)
    term, total, n = Decimal(1), Decimal(1), 1
    while True:
        term = -term * x * x / ((2 * n - 1) * (2 * n))
        if abs(term) < Decimal(10) ** -48:
            return total
        total += term
        n += 1


def dsqrt(x) -> Decimal:
    return D(x).sqrt()
