"""Fourier transform over GF(65537) (Sec. II-A).

* ``dft``      -- the definition A_j = sum_i a_i r^(i j), read as the evaluation
                  A_j = a(r^j) of the polynomial a(x) at 1, r, ..., r^(n-1)
                  (Sec. II-A, polynomial view); quadratic cost.
* ``idft``     -- the inverse definition, a_j = n^(-1) sum_i A_i r^(-i j).
* ``fnt``      -- the same transform by divide and conquer (the Cooley-Tukey
                  split the paper names for the FNT), O(n log n); pinned to
                  ``dft`` by the tests.
* ``ifnt``     -- its inverse (root r^(-1), then the factor n^(-1)).

Arrays may carry trailing lane axes: the transform runs along axis 0, every
other axis is an independent lane (the paper applies the code to every
16-bit lane of a packet, Sec. II-B).
"""
from __future__ import annotations

import numpy as np

from .field import P, inverse, powers, root


def _as_rows(a) -> np.ndarray:
    return np.asarray(a, dtype=np.int64) % P


def dft(a, r: int | None = None) -> np.ndarray:
    """A_j = sum_{i<n} a_i r^(i j) for 0 <= j < n (Sec. II-A, DFT definition).

    Computed as a(r^j) by Horner's rule at every point r^j at once.  ``r``
    defaults to the n-th root 3^(65536/n) of Sec. II-B.
    """
    a = _as_rows(a)
    n = a.shape[0]
    if r is None:
        r = root(n)
    pts = powers(r, n).reshape((n,) + (1,) * (a.ndim - 1))
    acc = np.zeros(a.shape, dtype=np.int64)
    for i in range(n - 1, -1, -1):
        acc = (acc * pts + a[i]) % P
    return acc


def idft(A, r: int | None = None) -> np.ndarray:
    """a_j = n^(-1) sum_i A_i r^(-i j) (Sec. II-A, inverse DFT definition)."""
    A = _as_rows(A)
    n = A.shape[0]
    if r is None:
        r = root(n)
    return (dft(A, inverse(r)) * inverse(n)) % P


def fnt(a, r: int | None = None) -> np.ndarray:
    """Divide-and-conquer transform with the same result as ``dft``.

    Split the input into even- and odd-indexed halves, transform each with
    root r^2, and recombine A_j = E_j + r^j O_j, A_(j+n/2) = E_j - r^j O_j
    (r^(n/2) = -1 because r has order n).
    """
    a = _as_rows(a)
    n = a.shape[0]
    if r is None:
        r = root(n)
    if n == 1:
        return a.copy()
    if n % 2:
        raise ValueError("divide-and-conquer transform needs an even length")
    r2 = (r * r) % P
    even = fnt(a[0::2], r2)
    odd = fnt(a[1::2], r2)
    half = n // 2
    tw = powers(r, half).reshape((half,) + (1,) * (a.ndim - 1))
    t = (odd * tw) % P
    return np.concatenate([(even + t) % P, (even - t) % P], axis=0)


def ifnt(A, r: int | None = None) -> np.ndarray:
    """Inverse of ``fnt``: transform with r^(-1), then multiply by n^(-1)."""
    A = _as_rows(A)
    n = A.shape[0]
    if r is None:
        r = root(n)
    return (fnt(A, inverse(r)) * inverse(n)) % P
