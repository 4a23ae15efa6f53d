"""Encoder, decoders and locator quantities of the FNT-based RS code (Sec. II-B).

Layout: a codeword block is an int64 array [symbols, lanes...]; every lane is
an independent codeword (the code is applied to each 16-bit lane of a packet).

Readings of the paper taken here (the paper is terse or garbled at these
points):

* the root has order n (not n-1): r_n = 3^(65536/n) (Sec. II-B root choice);
* encoding is e_i = s(r^i) in natural order i = 0..n-1 (Sec. II-B);
* the decoder uses the first k received positions in ascending order
  (Sec. II-B: decoding uses the earliest k points received);
* step 5 forms the power series S_j = -N'(r^(-j-1)), j = 0..k-1, which is the
  unscaled evaluation of N'(y) = sum_i n_i y^(z_i) at the inverse roots, and
  step 6 keeps P(x) = (A(x) S(x)) mod x^k.  P has degree < k and equals
  A(x) * sum_i n_i/(x - x_i) exactly, so truncating A*S at x^k recovers it.
"""
from __future__ import annotations

import numpy as np

from . import poly
from .field import P, inverse, inverse_array, powers, root
from .transform import fnt, ifnt


def _rows(a) -> np.ndarray:
    return np.asarray(a, dtype=np.int64) % P


def _check_nk(n: int, k: int) -> None:
    if n < 1 or n > 65536 or (n & (n - 1)):
        raise ValueError(f"n must be a power of two in [1, 65536], got {n}")
    if k < 1 or k > n:
        raise ValueError(f"need 1 <= k <= n, got k={k}, n={n}")


def eval_points(n: int, positions) -> np.ndarray:
    """x_i = r^(z_i) for received positions z_i (Sec. II-B, x_i = r^(z_i))."""
    r = root(n)
    tab = powers(r, n)
    return tab[np.asarray(positions, dtype=np.int64)]


# ---------------------------------------------------------------------------
# Encoder (Sec. II-B): e = FNT_n(s_0..s_(k-1), 0..0), i.e. e_i = s(r^i).
# ---------------------------------------------------------------------------

def encode(s, n: int, rows=None) -> np.ndarray:
    """e_i = s(r^i) = sum_{j<k} s_j r^(i j), by Horner's rule in x = r^i.

    This is the Vandermonde / generator-matrix view of the encoder: the first k
    rows of the FNT matrix form the generator matrix (Sec. II-A), and the
    encoder applies the FNT to the zero-padded source (Sec. II-B).  ``rows``
    restricts the output to the listed indices i (for sampled checks).
    """
    s = _rows(s)
    k = s.shape[0]
    _check_nk(n, k)
    r = root(n)
    idx = np.arange(n, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    x = powers(r, n)[idx].reshape((idx.size,) + (1,) * (s.ndim - 1))
    acc = np.zeros((idx.size,) + s.shape[1:], dtype=np.int64)
    for j in range(k - 1, -1, -1):
        acc = (acc * x + s[j]) % P
    return acc


# ---------------------------------------------------------------------------
# Decoders.  Both solve sum_{j<k} s_j x_i^j = v_i for the received points.
# ---------------------------------------------------------------------------

def _first_k(positions, k: int, n: int) -> np.ndarray:
    z = np.asarray(positions, dtype=np.int64)
    if z.size < k:
        raise ValueError(f"need at least k={k} received positions, got {z.size}")
    z = np.sort(z)
    if np.any(np.diff(z) == 0) or z[0] < 0 or z[-1] >= n:
        raise ValueError("positions must be distinct and in [0, n)")
    return z[:k]


def decode_gauss(n: int, positions, v) -> np.ndarray:
    """Solve the k x k Vandermonde system V_R s = v by Gauss-Jordan elimination mod p.

    V_R[i][j] = x_i^j is the generator matrix restricted to the received rows;
    it is invertible because the x_i are pairwise distinct (Sec. II-A), which
    is the MDS property.  Pivot: the first nonzero entry of the column.
    Cost k^3, meant for small k.
    """
    v = _rows(v)
    k = v.shape[0]
    z = _first_k(positions, k, n)
    x = eval_points(n, z)
    M = np.empty((k, k), dtype=np.int64)
    M[:, 0] = 1
    for j in range(1, k):
        M[:, j] = (M[:, j - 1] * x) % P
    B = v.reshape(k, -1).copy()
    for c in range(k):
        nz = np.nonzero(M[c:, c])[0]
        piv = c + int(nz[0])
        if piv != c:
            M[[c, piv]] = M[[piv, c]]
            B[[c, piv]] = B[[piv, c]]
        inv = inverse(int(M[c, c]))
        M[c] = (M[c] * inv) % P
        B[c] = (B[c] * inv) % P
        f = M[:, c].copy()
        f[c] = 0
        M = (M - f[:, None] * M[c][None, :]) % P
        B = (B - f[:, None] * B[c][None, :]) % P
    return B.reshape(v.shape)


def lagrange_denominators(x) -> np.ndarray:
    """d_i = prod_{j != i} (x_i - x_j), the Lagrange denominators (Sec. II-B)."""
    x = np.asarray(x, dtype=np.int64) % P
    k = x.size
    d = np.ones(k, dtype=np.int64)
    for j in range(k):
        f = (x - x[j]) % P
        f[j] = 1
        d = (d * f) % P
    return d


def decode_lagrange(n: int, positions, v) -> np.ndarray:
    """P(x) = sum_i v_i prod_{j != i} (x - x_j)/(x_i - x_j) (Sec. II-B, Lagrange form).

    The numerator prod_{j != i}(x - x_j) = A(x)/(x - x_i) is obtained by
    synthetic division of A(x) = prod_j (x - x_j); coefficient m of P is
    sum_i (v_i / d_i) q_i[m].  Quadratic in k per lane.
    """
    v = _rows(v)
    k = v.shape[0]
    z = _first_k(positions, k, n)
    x = eval_points(n, z)
    A = poly.from_roots(x)                      # degree k, monic
    c = (inverse_array(lagrange_denominators(x))[:, None] * v.reshape(k, -1)) % P
    out = np.zeros_like(c)
    q = np.zeros(k, dtype=np.int64)             # q_i[m] for the current m, all i
    for m in range(k - 1, -1, -1):
        # A(x)/(x - x_i): q[k-1] = a_k, q[m-1] = a_m + x_i q[m]
        q = (A[m + 1] + x * q) % P
        out[m] = (q @ c) % P
    return out.reshape(v.shape)


def decode_erasure_free(e) -> np.ndarray:
    """All n symbols received: s = first k of FNT_n^(-1)(e) (Sec. II-B)."""
    return ifnt(e)


# ---------------------------------------------------------------------------
# Locator quantities and the six-step interpolation (Sec. II-B, steps 1-6).
# ---------------------------------------------------------------------------

def locator(n: int, positions, with_w: bool = True) -> dict:
    """Quantities that depend only on the received positions (steps 1-3).

    A     -- A(x) = prod_i (x - x_i), k+1 coefficients, monic (step 1)
    dA    -- A'(x), k coefficients (step 2)
    w     -- w_i = 1 / A'(x_i) = 1 / prod_{j != i}(x_i - x_j) (step 3 and
             the identity A_i(x_i) = A'(x_i))
    Ahat  -- FNT_(2k) of (a_0 .. a_(k-1), 0 .. 0), used for the low product
             of step 6 (requires 2k a power of two <= 65536: the transform
             has power-of-two lengths, Sec. II-A)
    """
    z = np.asarray(positions, dtype=np.int64)
    k = z.size
    x = eval_points(n, z)
    A = poly.from_roots(x)
    dA = poly.derivative(A)
    out = {"x": x, "A": A, "dA": dA}
    if with_w:
        out["w"] = inverse_array(lagrange_denominators(x))
    if 2 * k <= 65536 and k & (k - 1) == 0:
        pad = np.zeros(2 * k, dtype=np.int64)
        pad[:k] = A[:k]
        out["Ahat"] = fnt(pad)
    return out


def step5_series(n: int, positions, nvals, count: int) -> np.ndarray:
    """S_j = -N'(r^(-j-1)), j < count, with N'(y) = sum_i n_i y^(z_i) (Sec. II-B, step 5).

    This is the power series of sum_i n_i / (x - x_i) modulo x^count, written
    as one evaluation of N' per coefficient.
    """
    z = np.asarray(positions, dtype=np.int64)
    nv = _rows(nvals).reshape(z.size, -1)
    rinv = inverse(root(n))
    tab = powers(rinv, n)
    j = np.arange(1, count + 1, dtype=np.int64)
    E = (j[:, None] * z[None, :]) % n           # exponent of r^(-1)
    out = np.zeros((count, nv.shape[1]), dtype=np.int64)
    for c0 in range(0, count, 512):
        blk = tab[E[c0:c0 + 512]]               # [rows, k]
        out[c0:c0 + 512] = (P - (blk @ nv) % P) % P
    return out.reshape((count,) + np.asarray(nvals).shape[1:])


def decode_six_step(n: int, positions, v) -> np.ndarray:
    """The interpolation of Sec. II-B in the paper's six steps, quadratic building blocks.

    1. A(x) = prod (x - x_i);  2. A'(x);  3. A'(x_i);  4. n_i = v_i / A'(x_i);
    5. S(x) = sum_i n_i/(x - x_i) mod x^k = -sum_j N'(r^(-j-1)) x^j;
    6. P(x) = A(x) S(x) truncated to degree < k.
    """
    v = _rows(v)
    k = v.shape[0]
    z = _first_k(positions, k, n)
    x = eval_points(n, z)
    A = poly.from_roots(x)                                   # step 1
    dA = poly.derivative(A)                                  # step 2
    dAx = poly.evaluate(dA, x)                               # step 3
    nvals = (inverse_array(dAx)[:, None] * v.reshape(k, -1)) % P   # step 4
    S = step5_series(n, z, nvals, k)                         # step 5
    out = np.zeros_like(S)
    for i in range(k):                                       # step 6, mod x^k
        out[i:] = (out[i:] + A[i] * S[: k - i]) % P
    return out.reshape(v.shape)


# ---------------------------------------------------------------------------
# Systematic code (Sec. II-C): the source vector, interpolated on the first k
# positions, gives k intermediate symbols; the codeword is the same transform
# of the intermediate symbols, so its first k symbols are the source.
# ---------------------------------------------------------------------------

def systematic_intermediate(s, n: int) -> np.ndarray:
    """The intermediate symbols: coefficients of the degree < k polynomial
    taking the value s_j at x = r^j, j < k (Sec. II-C, interpolation on the
    first k positions)."""
    s = _rows(s)
    k = s.shape[0]
    _check_nk(n, k)
    return decode_lagrange(n, np.arange(k, dtype=np.int64), s)


def systematic_encode(s, n: int, rows=None) -> np.ndarray:
    """e = FNT_n of the zero-padded intermediate symbols (Sec. II-C);
    ``rows`` restricts the output as in ``encode``."""
    return encode(systematic_intermediate(s, n), n, rows=rows)


def systematic_decode(n: int, positions, v) -> np.ndarray:
    """The source from k received symbols (Sec. II-C): the intermediate
    symbols by the interpolation of Sec. II-B, then their transform at the
    first k positions."""
    v = _rows(v)
    k = v.shape[0]
    inter = decode_lagrange(n, positions, v)
    return encode(inter, n, rows=np.arange(k, dtype=np.int64))


# ---------------------------------------------------------------------------
# Code lengths that are not a power of two (Sec. II-B: puncturing), and the
# 16-bit transport of symbols (Sec. II-B: every value but 65536 fits in 16
# bits; the positions holding 65536 travel in the symbol's header).
# ---------------------------------------------------------------------------

def padded_length(n: int) -> int:
    """N = the smallest power of two >= n: the transform length of a code of length n."""
    if n < 1 or n > 65536:
        raise ValueError(f"n must be in [1, 65536], got {n}")
    N = 1
    while N < n:
        N *= 2
    return N


def encode_punctured(s, n: int, rows=None) -> np.ndarray:
    """The code of length n: the first n symbols of the code of length N =
    padded_length(n) (the others are never sent)."""
    N = padded_length(n)
    idx = np.arange(n, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise ValueError("rows must lie in [0, n)")
    return encode(s, N, rows=idx)


def decode_punctured(n: int, positions, v) -> np.ndarray:
    """Decoding from k received symbols of a code of length n: the received
    points are r_N^z, z < n, with N = padded_length(n)."""
    z = np.asarray(positions, dtype=np.int64)
    if z.size and (z.min() < 0 or z.max() >= n):
        raise ValueError("positions must lie in [0, n)")
    return decode_lagrange(padded_length(n), z, v)


def pack16(symbol) -> tuple:
    """One encoding symbol (a vector of residues) as 16-bit words plus the
    positions holding 65536, which are sent as 0."""
    v = np.asarray(symbol, dtype=np.int64)
    if np.any((v < 0) | (v > 65536)):
        raise ValueError("residues must lie in [0, 65536]")
    esc = np.nonzero(v == 65536)[0].astype(np.int64)
    return (v % 65536).astype(np.uint16), esc


def unpack16(words, escapes) -> np.ndarray:
    """Inverse of pack16."""
    v = np.asarray(words, dtype=np.int64).copy()
    v[np.asarray(escapes, dtype=np.int64)] = 65536
    return v
