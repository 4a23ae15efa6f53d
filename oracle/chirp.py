"""Chirp evaluation of a polynomial on a geometric sequence (Sec. II-B, steps 3 and 5).

Test infrastructure: a plain CPU reference, never part of the product path.

Sec. II-B observes that the decoder's evaluation points form a sub-sequence
of a geometric progression and reduces the evaluation of a polynomial on it
to one polynomial product, of which only the middle coefficients are used
(Sec. III: the middle product).  With t_i = i(i-1)/2 one has
t_(i+j) = t_i + t_j + i j, so for any nonzero q

    c(a q^i) = sum_j c_j a^j q^(i j) = q^(-t_i) sum_j (c_j a^j q^(-t_j)) q^(t_(i+j)).

The paper writes b_i for q^(t_i) (b_(i+1) = q^i b_i) and c_i for the
coefficients divided by b_i; its printed sum is garbled (it multiplies the
undivided coefficients by b_(i+j)), read here as the identity above.  The sum
over j is coefficient L-1+i of the product of u reversed (u_j = c_j a^j
q^(-t_j), j < L) by v (v_m = q^(t_m), m < L+M-1): the coefficients of degrees
L-1 .. L+M-2, the middle ones.

Here every step is written out plainly: the exponents t_i, the two sequences,
one schoolbook product (poly.mul), the middle slice and the final scaling.
"""
from __future__ import annotations

import numpy as np

from . import poly
from .field import P, inverse, power


def tri(i: int) -> int:
    """t_i = i (i - 1) / 2."""
    return i * (i - 1) // 2


def chirp_eval(c, q: int, M: int, a: int = 1) -> np.ndarray:
    """c(a q^i) for i < M, by the chirp identity and one middle product.

    c: coefficients, lowest degree first, shape [L] or [L, lanes...].
    q, a: nonzero residues.
    """
    c = np.asarray(c, dtype=np.int64) % P
    L = c.shape[0]
    q %= P
    a %= P
    if q == 0 or a == 0:
        raise ValueError("q and a must be nonzero")
    qinv = inverse(q)
    # u_j = c_j a^j q^(-t_j), reversed; v_m = q^(t_m)
    s = np.array([power(a, j) * power(qinv, tri(j)) % P for j in range(L)], dtype=np.int64)
    u = (c * s.reshape((L,) + (1,) * (c.ndim - 1))) % P
    v = np.array([power(q, tri(m)) for m in range(L + M - 1)], dtype=np.int64)
    flat = u.reshape(L, -1)
    out = np.zeros((M, flat.shape[1]), dtype=np.int64)
    for col in range(flat.shape[1]):
        prod = poly.mul(flat[::-1, col], v)          # degrees 0 .. 2L+M-3
        out[:, col] = prod[L - 1:L - 1 + M]          # the middle coefficients
    scale = np.array([power(qinv, tri(i)) for i in range(M)], dtype=np.int64)
    out = (out * scale[:, None]) % P
    return out.reshape((M,) + c.shape[1:])


def horner_points(c, q: int, M: int, a: int = 1) -> np.ndarray:
    """The same values by Horner's rule at each point a q^i (for the pins)."""
    pts = np.array([a * power(q, i) % P for i in range(M)], dtype=np.int64)
    c = np.asarray(c, dtype=np.int64) % P
    acc = np.zeros((M,) + c.shape[1:], dtype=np.int64)
    x = pts.reshape((M,) + (1,) * (c.ndim - 1))
    for j in range(c.shape[0] - 1, -1, -1):
        acc = (acc * x + c[j]) % P
    return acc
