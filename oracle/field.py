"""The prime field GF(65537) (Sec. II-A, the transform over a finite field).

Residues are the integers 0 .. p-1; addition and product are taken modulo p.
The paper fixes q = 65537, the Fermat prime 2^16 + 1 (Sec. II-B), and uses the
primitive root 3; a transform of size n = 2^i uses the root 3^(2^(16-i))
(Sec. II-B, root selection).

Everything here works on Python ints or on numpy int64 arrays; products of
two residues are below 2^33, so int64 never overflows.
"""
from __future__ import annotations

import numpy as np

P = 65537            # the Fermat prime 2^16 + 1 (Sec. II-B)
GENERATOR = 3        # primitive root of GF(65537) (Sec. II-A example)
ORDER = P - 1        # multiplicative group order, 2^16


def add(a, b):
    return (a + b) % P


def sub(a, b):
    return (a - b) % P


def mul(a, b):
    return (a * b) % P


def power(a: int, e: int) -> int:
    """a^e mod p for a Python int base; negative e uses the inverse."""
    a %= P
    if e < 0:
        return pow(inverse(a), -e, P)
    return pow(a, e, P)


def inverse(a: int) -> int:
    """Multiplicative inverse by Fermat's little theorem: a^(p-2)."""
    a %= P
    if a == 0:
        raise ZeroDivisionError("0 has no inverse in GF(65537)")
    return pow(a, P - 2, P)


def order(a: int) -> int:
    """Multiplicative order: the least e > 0 with a^e = 1 (Sec. II-A)."""
    a %= P
    if a == 0:
        raise ValueError("0 has no multiplicative order")
    x, e = a, 1
    while x != 1:
        x = (x * a) % P
        e += 1
    return e


def is_power_of_two(n: int) -> bool:
    return n > 0 and (n & (n - 1)) == 0


def root(n: int) -> int:
    """The n-th root of unity r_n = 3^(2^16 / n) for n = 2^i <= 2^16 (Sec. II-B)."""
    if not is_power_of_two(n) or n > ORDER:
        raise ValueError(f"transform size must be a power of two <= 65536, got {n}")
    return pow(GENERATOR, ORDER // n, P)


def powers(x: int, count: int) -> np.ndarray:
    """[x^0, x^1, ..., x^(count-1)] mod p as an int64 array (sequential products)."""
    out = np.empty(count, dtype=np.int64)
    acc = 1
    for i in range(count):
        out[i] = acc
        acc = (acc * x) % P
    return out


def inverse_array(a: np.ndarray) -> np.ndarray:
    """Element-wise inverse of a nonzero int64 array by square-and-multiply of a^(p-2)."""
    a = np.asarray(a, dtype=np.int64) % P
    if np.any(a == 0):
        raise ZeroDivisionError("0 has no inverse in GF(65537)")
    result = np.ones_like(a)
    base = a.copy()
    e = P - 2
    while e:
        if e & 1:
            result = (result * base) % P
        base = (base * base) % P
        e >>= 1
    return result
