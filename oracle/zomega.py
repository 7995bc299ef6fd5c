"""Exact arithmetic in Z[w], w = e^{i pi/4}, for the oracle: TEST INFRASTRUCTURE ONLY.

An element is a 4-tuple of Python ints (c0, c1, c2, c3) meaning c0 + c1 w + c2 w^2 + c3 w^3;
w^4 = -1.  A scalar of the method is such an element times sqrt2^e (the paper writes
subterm values as A + B sqrt2 + i (C + D sqrt2) with "simple fractional numbers", Section
3.3 step 5; with A = c0, B = (c1 - c3)/2, C = c2, D = (c1 + c3)/2 that is the same set).

Canonical form of z * sqrt2^e: zero is ((0, 0, 0, 0), 0); otherwise divide by sqrt2 while
the quotient stays in Z[w], raising e each time.  Since sqrt2 = w - w^3,
z / sqrt2 = ((c1 - c3)/2, (c0 + c2)/2, (c1 + c3)/2, (c2 - c0)/2), which is integral exactly
when c1 = c3 and c0 = c2 (mod 2).  Two scalars are equal iff their canonical forms are.
"""

import cmath
import math
from typing import Tuple

ZW = Tuple[int, int, int, int]

ZERO: ZW = (0, 0, 0, 0)
ONE: ZW = (1, 0, 0, 0)


def omega_pow(k: int) -> ZW:
    k %= 8
    c = [0, 0, 0, 0]
    if k < 4:
        c[k] = 1
    else:
        c[k - 4] = -1
    return tuple(c)


def add(a: ZW, b: ZW) -> ZW:
    return tuple(x + y for x, y in zip(a, b))


def sub(a: ZW, b: ZW) -> ZW:
    return tuple(x - y for x, y in zip(a, b))


def neg(a: ZW) -> ZW:
    return tuple(-x for x in a)


def mul(a: ZW, b: ZW) -> ZW:
    r = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            if i + j < 4:
                r[i + j] += a[i] * b[j]
            else:
                r[i + j - 4] -= a[i] * b[j]
    return tuple(r)


def scale(a: ZW, k: int) -> ZW:
    return tuple(k * x for x in a)


def conj(a: ZW) -> ZW:
    """complex conjugate: w -> w^{-1} = -w^3, w^2 -> -w^2, w^3 -> -w"""
    return (a[0], -a[3], -a[2], -a[1])


def times_sqrt2(a: ZW) -> ZW:
    c0, c1, c2, c3 = a
    return (c1 - c3, c0 + c2, c1 + c3, c2 - c0)


def divisible_by_sqrt2(a: ZW) -> bool:
    c0, c1, c2, c3 = a
    return (c1 - c3) % 2 == 0 and (c0 + c2) % 2 == 0


def div_sqrt2(a: ZW) -> ZW:
    c0, c1, c2, c3 = a
    assert divisible_by_sqrt2(a)
    return ((c1 - c3) // 2, (c0 + c2) // 2, (c1 + c3) // 2, (c2 - c0) // 2)


def canonical(a: ZW, e: int) -> Tuple[ZW, int]:
    a = tuple(int(v) for v in a)
    if a == ZERO:
        return ZERO, 0
    while divisible_by_sqrt2(a):
        a = div_sqrt2(a)
        e += 1
    return a, e


def to_complex(a: ZW, e: int = 0) -> complex:
    w = cmath.exp(1j * math.pi / 4)
    z = a[0] + a[1] * w + a[2] * w * w + a[3] * w ** 3
    return z * (math.sqrt(2) ** e)


def scalar_equal(a: ZW, ea: int, b: ZW, eb: int) -> bool:
    return canonical(a, ea) == canonical(b, eb)


def mul_scalar(a: ZW, ea: int, b: ZW, eb: int) -> Tuple[ZW, int]:
    return canonical(mul(a, b), ea + eb)


def add_scalar(a: ZW, ea: int, b: ZW, eb: int) -> Tuple[ZW, int]:
    """sum of two scalars with possibly different sqrt2 exponents, exactly"""
    while ea > eb:
        a = times_sqrt2(a)
        ea -= 1
    while eb > ea:
        b = times_sqrt2(b)
        eb -= 1
    return canonical(add(a, b), ea)
