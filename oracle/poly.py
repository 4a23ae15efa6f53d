"""Polynomials over GF(65537), coefficient lists lowest degree first (Sec. II-B).

Plain quadratic routines: schoolbook product, formal derivative, Horner
evaluation, and the product of linear factors built one factor at a time.
"""
from __future__ import annotations

import numpy as np

from .field import P


def mul(a, b) -> np.ndarray:
    """Schoolbook product c_m = sum_{i+j=m} a_i b_j (the classic quadratic product)."""
    a = np.asarray(a, dtype=np.int64) % P
    b = np.asarray(b, dtype=np.int64) % P
    if a.size == 0 or b.size == 0:
        return np.zeros(0, dtype=np.int64)
    out = np.zeros(a.size + b.size - 1, dtype=np.int64)
    for i, ai in enumerate(a):
        if ai:
            out[i:i + b.size] = (out[i:i + b.size] + ai * b) % P
    return out


def derivative(a) -> np.ndarray:
    """Formal derivative: coefficient i of a' is (i+1) a_(i+1) (Sec. II-B, step 2)."""
    a = np.asarray(a, dtype=np.int64) % P
    if a.size <= 1:
        return np.zeros(1, dtype=np.int64)
    return (a[1:] * np.arange(1, a.size, dtype=np.int64)) % P


def evaluate(a, x):
    """Horner evaluation of a(x); ``x`` may be an int or an int64 array."""
    a = np.asarray(a, dtype=np.int64) % P
    x = np.asarray(x, dtype=np.int64) % P
    acc = np.zeros_like(x)
    for c in a[::-1]:
        acc = (acc * x + c) % P
    return acc


def from_roots(xs) -> np.ndarray:
    """prod_j (x - x_j), multiplying one linear factor at a time (Sec. II-B, A(x))."""
    xs = np.asarray(xs, dtype=np.int64) % P
    c = np.zeros(xs.size + 1, dtype=np.int64)
    c[0] = 1
    deg = 0
    for xj in xs:
        # (c(x)) * (x - xj): new_m = c_(m-1) - xj c_m
        shifted = np.concatenate([[0], c[:deg + 1]])
        scaled = np.concatenate([(xj * c[:deg + 1]) % P, [0]])
        c[:deg + 2] = (shifted - scaled) % P
        deg += 1
    return c


def trim(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64) % P
    nz = np.nonzero(a)[0]
    return a[: nz[-1] + 1] if nz.size else a[:1] * 0
