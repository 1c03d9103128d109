"""G x Z2 for the M = 0 sector: the global spin flip.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

The paper resolves its M = 0 production blocks further by the global spin
flip (Section 2.3 and the note to Table 2; the 5x8 block of Section 4.3 is one
flip-parity half).  The flip F sends the digit a_k of every site to
(d - 1) - a_k; on labels of Eq. (2) it is n -> (d^N - 1) - n.  It commutes with
every site permutation and, at M = 0, maps the sector onto itself and commutes
with H, so G' = G x Z2 is a symmetry group of the M = 0 sector.

Conventions of this oracle (the library uses the same ones):

* element (g, f) acts as U(g) F^f and has index f |G| + g, so the |G|
  elements of G come first, in their own order, then the same elements
  composed with F;
* the irreps of G' are Gamma^p with rho'(g, f) = p^f rho_Gamma(g), p = +1 or
  -1, indexed 2 i + (p < 0) for the i-th irrep of G.

Everything else (representatives as orbit minima, the smallest index among
minimisers as the connecting element, stabilizers, n_Gamma, V_S, the explicit
basis of Eq. (12)) is the plain definition in ``basis`` applied to G', which
reaches the flip through ``FlipGroup``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .group import Group, cycle_type
from .irreps import Irrep


@dataclass
class FlipGroup:
    """G x Z2 acting on labels of an M = 0 sector (see the module text)."""
    base: Group
    flip = True

    @property
    def order(self) -> int:
        return 2 * self.base.order

    @property
    def N(self) -> int:
        return self.base.N

    @property
    def inv(self) -> np.ndarray:
        return np.concatenate([self.base.inv, self.base.inv + self.base.order])

    @property
    def mul(self) -> np.ndarray:
        n = self.base.order
        m = self.base.mul
        out = np.empty((2 * n, 2 * n), dtype=np.int64)
        for f1 in (0, 1):
            for f2 in (0, 1):
                out[f1 * n:(f1 + 1) * n, f2 * n:(f2 + 1) * n] = m + ((f1 ^ f2) * n)
        return out


def flip_labels(labels, N: int, d: int) -> np.ndarray:
    """Labels of F|n>: every digit a -> d - 1 - a, i.e. n -> d^N - 1 - n."""
    return (d ** N - 1) - np.asarray(labels, dtype=np.int64)


def flip_irreps(irreps) -> list:
    """Gamma^+ and Gamma^- of G x Z2 for every irrep Gamma of G, in the order 2i, 2i+1."""
    out = []
    for ir in irreps:
        for p in (1.0, -1.0):
            out.append(Irrep(ir.dim, np.concatenate([ir.rho, p * ir.rho]),
                             np.concatenate([ir.chars, p * ir.chars]), ir.indicator))
    return out


def flip_fixed_count(perm, two_s: int) -> int:
    """Number of states n with U(g) F n = n (all such states have M = 0).

    Along a cycle of length L the digits must alternate a, d-1-a: an even
    cycle leaves d choices, an odd cycle needs a = d-1-a, i.e. the middle
    digit, which exists only for odd d (integer s)."""
    d = two_s + 1
    c = 1
    for L in cycle_type(perm):
        c *= d if L % 2 == 0 else (1 if d % 2 == 1 else 0)
    return c
