"""Real forms of irreps of complex and quaternionic type (indicators 0, -1).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

In the paper, irreps whose indicator is 0 or -1 stay complex unitary
matrices and run on a path in complex arithmetic (Section 3).  The library keeps
real arithmetic instead, and this module states what it computes:

* An irrep Gamma of complex type (indicator 0, dimension d) and its conjugate
  Gamma* are taken together as one real representation of dimension 2d, the
  realification rho_R(g) = [[Re rho(g), -Im rho(g)], [Im rho(g), Re rho(g)]].
  It is orthogonal, a homomorphism, irreducible over the reals (its real
  commutant is two-dimensional, spanned by 1 and the complex structure
  J = [[0, -1], [1, 0]]), its character is 2 Re chi, its indicator is 0.
* Row alpha of rho_R satisfies the one orthogonality relation the block
  construction of Eqs. (10)-(12) and the gather form of Eq. (15) use:
  (2d / |G|) sum_g rho_R(g)[alpha, m] rho_R(g)[alpha, m'] = delta(m, m').
  So Eq. (12) built with rho_R (any row) gives an H-invariant real block;
  it is the real form of the complex row block of Gamma and Gamma*: real
  dimension 2 D_Gamma, every eigenvalue of the Gamma block twice.
* Trace weight (the d_Gamma factor of Eq. (4)): the pair contributes
  d Tr_Gamma f(H) + d Tr_Gamma* f(H) = d Tr_{rho_R block} f(H), so a realified
  pair enters with weight d = dim(rho_R) / 2, a real-type irrep with d.
  The whole spectrum of the sector is therefore the union over real forms of
  weight copies of each block's spectrum, which the tests check by exact
  diagonalization.

* An irrep Gamma of quaternionic type (indicator -1, d even) is equivalent to
  its conjugate; its realification rho_R (same formula, dimension 2d) is
  irreducible over the reals with a four-dimensional real commutant (the
  quaternions), character 2 chi, and its rows satisfy the same relation (the
  commutant's non-identity elements are antisymmetric, so they do not reach
  the diagonal).  Its row block is again the real form of the complex Gamma
  block (real dimension 2 D_Gamma, every level of the Gamma block twice, and
  the Gamma block's levels come in pairs themselves).  Gamma contributes
  d Tr_Gamma f(H) = (d / 2) Tr_{rho_R block} f(H): trace weight
  d / 2 = dim(rho_R) / 4.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .group import Group
from .irreps import Irrep


@dataclass
class RealForm:
    irrep: Irrep        # real orthogonal matrices (dim d for real type, 2d when realified)
    weight: int         # trace weight in the thermal sums
    kind: str           # "real", "complex pair" or "quaternionic"


def realify(ir: Irrep) -> Irrep:
    """rho_R = [[Re rho, -Im rho], [Im rho, Re rho]] of a complex- or
    quaternionic-type irrep (the indicator is kept: 0 or -1)."""
    if ir.indicator not in (0, -1):
        raise ValueError("realification applies to irreps with indicator 0 or -1")
    re, im = ir.rho.real, ir.rho.imag
    rho = np.block([[re, -im], [im, re]])
    chars = np.trace(rho, axis1=1, axis2=2).astype(complex)   # = 2 Re chi
    return Irrep(2 * ir.dim, rho, chars, ir.indicator)


def real_forms(G: Group, irreps) -> list:
    """One real form per real-type irrep, per conjugate pair of complex-type
    irreps (the first of the pair in the given order is realified) and per
    quaternionic irrep (realified, weight d / 2).

    Order: dimension of the real form ascending, then its character over the
    canonical class order descending (rounded to 1e-9), as for the irreps."""
    rep_class = [c[0] for c in G.classes]
    out, used = [], set()
    for i, ir in enumerate(irreps):
        if i in used:
            continue
        if ir.indicator == 1:
            out.append(RealForm(ir, ir.dim, "real"))
        elif ir.indicator == 0:
            conj = [j for j, o in enumerate(irreps)
                    if j != i and j not in used and o.dim == ir.dim and np.allclose(o.chars, np.conj(ir.chars), atol=1e-8)]
            if len(conj) != 1:
                raise AssertionError("complex-type irrep without a unique conjugate")
            used.add(conj[0])
            out.append(RealForm(realify(ir), ir.dim, "complex pair"))
        else:
            if ir.dim % 2:
                raise AssertionError("a quaternionic irrep has even dimension")
            out.append(RealForm(realify(ir), ir.dim // 2, "quaternionic"))
        used.add(i)

    def key(f):
        cc = f.irrep.chars[rep_class].real
        return (f.irrep.dim, tuple(-np.round(cc, 9)))

    out.sort(key=key)
    return out
