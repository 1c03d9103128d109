"""Sector and block dimensions by counting (paper Section 2.1, Eq. 13).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

* ``sector_dim``: number of labels whose N base-d digits sum to A = Ns + M,
  i.e. the coefficient of x^A in (1 + x + ... + x^(d-1))^N, by the digit-by-
  digit counting recursion.
* ``block_dims_by_characters``: D_{M,Gamma} = (1/|G|) sum_g chi_Gamma(g)^* F_M(g),
  where F_M(g) is the trace of U(g) on the M sector: the number of sector
  states fixed by g, i.e. the coefficient of x^A in prod_{cycles c of g}
  sum_a x^(a |c|) (a state is fixed iff it is constant on every cycle).
  This is the multiplicity of Gamma in the permutation representation of the
  sector, which equals the single-row block dimension of Eq. (13).
"""
from __future__ import annotations

import numpy as np

from .group import Group, cycle_type


def poly_mul(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                if y:
                    out[i + j] += x * y
    return out


def sector_dim(N: int, two_s: int, two_M: int) -> int:
    d = two_s + 1
    if (N * two_s + two_M) % 2:
        return 0
    A = (N * two_s + two_M) // 2
    if A < 0 or A > N * two_s:
        return 0
    counts = [1]                     # counts[a] = ways for the digits so far to sum to a
    for _ in range(N):
        counts = poly_mul(counts, [1] * d)
    return counts[A]


def fixed_count(perm, two_s: int, two_M: int) -> int:
    d = two_s + 1
    N = len(perm)
    A2 = N * two_s + two_M
    if A2 % 2:
        return 0
    A = A2 // 2
    poly = [1]
    for L in cycle_type(perm):
        f = [0] * (L * (d - 1) + 1)
        for a in range(d):
            f[a * L] = 1
        poly = poly_mul(poly, f)
    return poly[A] if 0 <= A < len(poly) else 0


def block_dims_by_characters(G: Group, irreps, two_s: int, two_M: int):
    """D_{M,Gamma} = (1/|G|) sum_g chi(g)^* F_M(g), F_M(g) = states of sector M fixed by U(g).

    For G x Z2 (M = 0 only) the elements U(g) F fix the states counted by
    ``spinflip.flip_fixed_count``."""
    if getattr(G, "flip", False):
        from .spinflip import flip_fixed_count
        if two_M != 0:
            raise ValueError("the spin flip maps sector M to -M; G x Z2 needs M = 0")
        F = np.array([fixed_count(p, two_s, 0) for p in G.base.perms] +
                     [flip_fixed_count(p, two_s) for p in G.base.perms], dtype=np.float64)
    else:
        F = np.array([fixed_count(p, two_s, two_M) for p in G.perms], dtype=np.float64)
    dims = []
    for ir in irreps:
        val = np.sum(np.conj(ir.chars) * F) / G.order
        dims.append(int(round(val.real)))
        # characters carry ~1e-14 rounding; F reaches ~1e11, so allow that scale
        assert abs(val - round(val.real)) < 1e-6 + 1e-12 * ir.dim * float(F.max())
    return dims
