"""Seeded synthetic input vectors.

``label_keyed_block_vector`` gives every row of a symmetry block a value that
depends only on (seed, representative label, row-within-representative k,
column v).  Because the value is a function of the representative's *label*
and not of its position in any table, a CPU reference can evaluate the same
input at any representative it reaches on its own, without ever reading a
table built by the code under test.

The hash is the SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) used
as a stateless integer mixer; it is input generation only.
"""
from __future__ import annotations

import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def label_keyed_values(seed: int, labels, k, v):
    """Uniform values in [-1, 1) keyed by (seed, label, k, v); broadcasts."""
    labels = np.asarray(labels, dtype=np.uint64)
    k = np.asarray(k, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = mix64(np.uint64(seed) * _GAMMA + np.uint64(1))
        h = mix64(h ^ labels)
        h = mix64(h ^ (k * np.uint64(1 << 16) + v + np.uint64(0x5A5A)))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def label_keyed_block_vector(seed: int, rep_labels, counts, nvec: int):
    """Block vector X (D x nvec) for a block whose rows are (rep, k), k < counts[rep].

    ``rep_labels`` and ``counts`` are in block row order (representatives in
    ascending label order, inactive ones with count 0 allowed).
    """
    rep_labels = np.asarray(rep_labels, dtype=np.uint64)
    counts = np.asarray(counts, dtype=np.int64)
    lab = np.repeat(rep_labels, counts)
    starts = np.repeat(np.cumsum(counts) - counts, counts)
    kk = np.arange(len(lab), dtype=np.int64) - starts
    vv = np.arange(nvec, dtype=np.uint64)[None, :]
    return label_keyed_values(seed, lab[:, None], kk[:, None].astype(np.uint64), vv)


def dense_uniform(seed: int, shape):
    """Plain seeded uniform [-1, 1) array (numpy PCG64)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


def _i64(c: int) -> int:
    """An unsigned 64-bit constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def label_keyed_values_torch(seed: int, labels, k, v):
    """``label_keyed_values`` with torch int64 tensors (any device); same values bit for bit.

    uint64 arithmetic is done in int64: products wrap modulo 2^64 and a
    logical right shift is an arithmetic shift with the sign-extended bits
    masked off.  Returns float64 in [-1, 1).
    """
    import torch

    def srl(x, s):
        return (x >> s) & ((1 << (64 - s)) - 1)

    def mix(z):
        z = (z ^ srl(z, 30)) * _i64(int(_M1))
        z = (z ^ srl(z, 27)) * _i64(int(_M2))
        return z ^ srl(z, 31)

    with np.errstate(over="ignore"):
        h0 = int(mix64(np.uint64(seed) * _GAMMA + np.uint64(1)))
    h = mix(torch.as_tensor(labels, dtype=torch.int64) ^ _i64(h0))
    kv = torch.as_tensor(k, dtype=torch.int64) * (1 << 16) + torch.as_tensor(v, dtype=torch.int64) + 0x5A5A
    h = mix(h ^ kv)
    return srl(h, 11).to(torch.float64) * (2.0 ** -52) - 1.0
