"""Pure-Python Ball Mapper for tiny inputs (TEST INFRASTRUCTURE ONLY).

Written independently of ``bm_oracle.c`` so the two can check each other:

* ``sqdist_f64`` uses Python floats, which are IEEE binary64 with round to
  nearest and no fused multiply-add, summing the squared coordinate
  differences left to right — the same rounding sequence the C oracle must
  produce, so any contraction or reordering in the C build shows up as a
  bitwise difference.
* ``sqdist_exact`` is the exact real squared distance as a Fraction.
* ``greedy`` keeps an explicit set of uncovered points and always takes the
  earliest one in the given order (Sec. 2.2); ``edges_bruteforce`` tests every
  landmark pair against every point (Sec. 2.1, nerve 1-skeleton).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def widen(points) -> list[list[float]]:
    """Exact widening of float16/32/64 coordinates to Python floats."""
    return np.asarray(points).astype(np.float64).tolist()


def sqdist_f64(a, b) -> float:
    acc = 0.0
    for ak, bk in zip(a, b):
        t = ak - bk
        acc = acc + t * t
    return acc


def sqdist_exact(a, b) -> Fraction:
    return sum(((Fraction(ak) - Fraction(bk)) ** 2 for ak, bk in zip(a, b)), Fraction(0))


def greedy(points, eps: float, order=None):
    """Returns (landmarks, rows, edges) with rows as lists of ascending indices."""
    w = widen(points)
    n = len(w)
    e2 = eps * eps
    order = list(range(n)) if order is None else [int(o) for o in order]
    uncovered = set(range(n))
    landmarks, rows = [], []
    for p in order:
        if p not in uncovered:
            continue
        ball = [x for x in range(n) if sqdist_f64(w[p], w[x]) < e2]
        landmarks.append(p)
        rows.append(ball)
        uncovered.difference_update(ball)
    return landmarks, rows, edges_bruteforce(rows, n)


def edges_bruteforce(rows, n: int):
    sets = [set(r) for r in rows]
    out = []
    for i in range(len(rows)):
        for j in range(i + 1, len(rows)):
            if any(x in sets[i] and x in sets[j] for x in range(n)):
                out.append((i, j))
    return out
