"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module holds random-number generation and sampling only: nothing here
computes anything of the coding method itself (no field arithmetic, no
transform, no interpolation).  Both the HIP path and the CPU checker are fed
from these generators, so the two see identical inputs.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used in counter mode: the i-th draw of a
stream with seed ``s`` is ``mix64(s + (i + 1) * GAMMA)``.

Workload recipes (the paper's own experiments use synthetic source data at
code rate 1/2 with k swept; no public dataset is involved):

* source symbols: every 16-bit lane of every source symbol is uniform in
  [0, 65535] and stored as a uint32 residue;
* erasures: the received set is a uniform random k-subset of the n positions
  (the k positions whose 64-bit keys are smallest), returned ascending;
* worst-case pattern: every erasure among the first k positions, i.e. the
  received set is {k, ..., n-1};
* uneven batch: k = 2^U with U uniform over {6..14}, rate uniform over
  {1/2, 1/4} (n = 2k or 4k), payload bytes 2*floor(2^V / 2) with V uniform
  on [8, 14], so lanes = floor(2^V / 2) lies in [128, 8192].
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Draws ``offset .. offset+count-1`` of the stream ``seed`` as uint64."""
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
    return mix64(ctr)


def source(seed: int, batch: int, k: int, lanes: int) -> np.ndarray:
    """Uniform 16-bit source symbols, shape [batch, k, lanes], dtype uint32."""
    z = stream(seed, batch * k * lanes)
    return (z >> np.uint64(48)).astype(np.uint32).reshape(batch, k, lanes)


def residues(seed: int, shape, with_top: bool = True) -> np.ndarray:
    """Uniform residues in [0, 65536] (17-bit values), dtype uint32.

    With ``with_top`` a few entries are forced to 65536, the one residue that
    does not fit in 16 bits, so that every test exercises it.
    """
    count = int(np.prod(shape))
    z = stream(seed, count)
    v = ((z >> np.uint64(32)) % np.uint64(65537)).astype(np.uint32)
    if with_top and count:
        pick = (stream(seed ^ 0x5A5A5A5A, 4) % np.uint64(count)).astype(np.int64)
        v[pick] = 65536
    return v.reshape(shape)


def received_positions(seed: int, n: int, k: int) -> np.ndarray:
    """Ascending uniform random k-subset of range(n), dtype uint32."""
    keys = stream(seed, n)
    order = np.argsort(keys, kind="stable")
    return np.sort(order[:k]).astype(np.uint32)


def erased_first_k(n: int, k: int) -> np.ndarray:
    """Received set when every erasure falls among the first k positions."""
    return np.arange(n - k, n, dtype=np.uint32) if n - k < k else np.arange(k, n, dtype=np.uint32)[:k]


def uneven_batch(seed: int, count: int):
    """Sizes of the uneven batch: list of (k, n, lanes) tuples."""
    z = stream(seed, 3 * count).reshape(count, 3)
    out = []
    for a, b, c in z:
        u = 6 + int(a % np.uint64(9))
        k = 1 << u
        n = k * (2 if int(b >> np.uint64(63)) == 0 else 4)
        v = 8.0 + 6.0 * (float(c >> np.uint64(11)) / float(1 << 53))
        lanes = int(2.0 ** v) // 2
        lanes = max(128, min(8192, lanes))
        out.append((k, n, lanes))
    return out
