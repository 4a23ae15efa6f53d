"""Direct (quadratic) encoding and decoding of the FNT-based RS code (Sec. III).

Test infrastructure: a plain CPU reference, never part of the product path.

Besides the FNT-based algorithms, Sec. III lists quadratic ones, which the
paper uses for small k (Sec. IV uses them for k <= 256):

* systematic code, Table I, "direct encoding": the n - k non-systematic
  symbols are computed from the k source symbols in O((n-k) k) per lane;
* systematic code, Table I, "direct intermediate & FNT": the k intermediate
  symbols are obtained by a direct O(k^2) product, then one FNT_n;
* systematic code, Table II, "direct decoding": only the missing source
  symbols are recomputed from the received ones, in less than O((n-k) k);
* the non-systematic code's classic quadratic schemes (the footnote of
  Sec. III): encoding by the generator (Vandermonde) matrix, decoding by the
  inverse of its k received rows.

All of them are products with fixed matrices whose entries come from the
Lagrange basis of the relevant point set.  Here every matrix is written out
from its definition, entry by entry, with plain modular products; the
products with the data use numpy matrix products reduced mod p.

Points: position z of a code of length n is x_z = r_n^z (Sec. II-B); the
systematic code's source occupies positions 0..k-1 (Sec. II-C).
"""
from __future__ import annotations

import numpy as np

from . import codec, poly
from .field import P, inverse_array


def _matmul(M, X) -> np.ndarray:
    """(M X) mod p for residue matrices (exact: int64 partial sums per row chunk)."""
    M = np.asarray(M, dtype=np.int64) % P
    X = np.asarray(X, dtype=np.int64) % P
    flat = X.reshape(X.shape[0], -1)
    out = np.zeros((M.shape[0], flat.shape[1]), dtype=np.int64)
    # 65536^2 * 2048 < 2^63: accumulate at most 2048 terms before reducing
    for j0 in range(0, M.shape[1], 2048):
        out = (out + M[:, j0:j0 + 2048] @ flat[j0:j0 + 2048]) % P
    return out.reshape((M.shape[0],) + X.shape[1:])


def lagrange_values(xs, ys) -> np.ndarray:
    """B[t][i] = L_i(y_t): the Lagrange basis of the points xs, evaluated at ys.

    L_i(y) = prod_{m != i} (y - x_m) / (x_i - x_m) (Sec. II-B, Lagrange form),
    by direct products: O(|ys| k^2) modular products, for small codes only.
    """
    xs = np.asarray(xs, dtype=np.int64) % P
    ys = np.asarray(ys, dtype=np.int64) % P
    k = xs.size
    den = inverse_array(codec.lagrange_denominators(xs))          # 1 / prod_{m != i} (x_i - x_m)
    B = np.ones((ys.size, k), dtype=np.int64)
    for m in range(k):
        f = (ys[:, None] - xs[m]) % P                             # (y_t - x_m), for every i != m
        col = np.ones((ys.size, k), dtype=np.int64) * f
        col[:, m] = 1
        B = (B * col) % P
    return (B * den[None, :]) % P


def inverse_vandermonde(n: int, positions) -> np.ndarray:
    """W with W V_R = I, V_R[i][j] = x_i^j over the received points x_i (Sec. III).

    Row j of W holds coefficient j of every Lagrange basis polynomial:
    L_i(x) = w_i A(x)/(x - x_i), A(x) = prod_i (x - x_i), w_i = 1/A'(x_i),
    and A(x)/(x - x_i) comes from A by synthetic division.  So the
    non-systematic quadratic decoder is s = W v (k^2 per lane).
    """
    z = np.asarray(positions, dtype=np.int64)
    x = codec.eval_points(n, z)
    k = x.size
    A = poly.from_roots(x)
    w = inverse_array(codec.lagrange_denominators(x))
    W = np.zeros((k, k), dtype=np.int64)
    q = np.zeros(k, dtype=np.int64)
    for j in range(k - 1, -1, -1):
        q = (A[j + 1] + x * q) % P           # coefficient j of A(x)/(x - x_i), every i
        W[j] = (q * w) % P
    return W


def generator_rows(n: int, k: int, rows) -> np.ndarray:
    """G[t][j] = x_{rows[t]}^j, the rows of the generator (Vandermonde) matrix."""
    x = codec.eval_points(n, rows)
    G = np.empty((x.size, k), dtype=np.int64)
    G[:, 0] = 1
    for j in range(1, k):
        G[:, j] = (G[:, j - 1] * x) % P
    return G


def encode_direct(s, n: int) -> np.ndarray:
    """Non-systematic quadratic encoder: e = G s with G[i][j] = r_n^(i j)."""
    s = np.asarray(s, dtype=np.int64) % P
    return _matmul(generator_rows(n, s.shape[0], np.arange(n)), s)


def decode_direct(n: int, positions, v) -> np.ndarray:
    """Non-systematic quadratic decoder: s = W v, W the inverse of V_R."""
    v = np.asarray(v, dtype=np.int64) % P
    k = v.shape[0]
    z = np.sort(np.asarray(positions, dtype=np.int64))[:k]
    return _matmul(inverse_vandermonde(n, z), v)


def parity_matrix(n: int, k: int) -> np.ndarray:
    """C[t][j] = L_j(x_(k+t)), t < n-k: the Lagrange basis of the systematic
    points x_0..x_(k-1) at the other positions (Table I, direct encoding)."""
    xs = codec.eval_points(n, np.arange(k))
    ys = codec.eval_points(n, np.arange(k, n))
    return lagrange_values(xs, ys)


def systematic_encode_direct(s, n: int) -> np.ndarray:
    """Systematic codeword by direct encoding: rows 0..k-1 are the source and
    rows k..n-1 are C s, O((n-k) k) per lane (Sec. III, Table I)."""
    s = np.asarray(s, dtype=np.int64) % P
    k = s.shape[0]
    return np.concatenate([s, _matmul(parity_matrix(n, k), s)], axis=0)


def systematic_encode_intermediate(s, n: int) -> np.ndarray:
    """Systematic codeword by direct intermediate symbols and one FNT_n:
    i = W_0 s with W_0 the inverse Vandermonde of positions 0..k-1 (O(k^2)
    per lane), then e = FNT_n(i, 0, ..., 0) (Sec. III, Table I)."""
    s = np.asarray(s, dtype=np.int64) % P
    k = s.shape[0]
    inter = _matmul(inverse_vandermonde(n, np.arange(k)), s)
    return codec.encode(inter, n)


def systematic_decode_direct(n: int, positions, v) -> np.ndarray:
    """Source of a systematic codeword from k received symbols, recomputing
    only the missing source symbols (Sec. III, Table II, direct decoding).

    positions: ascending received positions (the first k are used), v their
    symbols.  A source position m < k that was received is copied; a missing
    one is s_m = sum_i v_i L_i(x_m) over the received points.
    """
    v = np.asarray(v, dtype=np.int64) % P
    k = v.shape[0]
    z = np.sort(np.asarray(positions, dtype=np.int64))[:k]
    out = np.zeros(v.shape, dtype=np.int64)
    got = {int(p): i for i, p in enumerate(z)}
    missing = [m for m in range(k) if m not in got]
    for m in range(k):
        if m in got:
            out[m] = v[got[m]]
    if missing:
        B = lagrange_values(codec.eval_points(n, z), codec.eval_points(n, missing))
        out[missing] = _matmul(B, v)
    return out


def direct_decode_cost(n: int, positions, k: int) -> int:
    """Products per lane of systematic direct decoding: k per missing source symbol."""
    z = set(int(p) for p in np.sort(np.asarray(positions))[:k])
    return k * sum(1 for m in range(k) if m not in z)


def inverse_check(n: int, positions) -> np.ndarray:
    """W V_R (should be the identity): helper for the pins."""
    z = np.sort(np.asarray(positions, dtype=np.int64))
    k = z.size
    return _matmul(inverse_vandermonde(n, z), generator_rows(n, k, z))


__all__ = ["lagrange_values", "inverse_vandermonde", "generator_rows", "encode_direct", "decode_direct",
           "parity_matrix", "systematic_encode_direct", "systematic_encode_intermediate",
           "systematic_decode_direct", "direct_decode_cost", "inverse_check"]
