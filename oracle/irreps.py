"""Irreducible representations from the regular representation (paper Section 3).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

In the paper each irrep is obtained numerically, as matrices, by decomposing
the regular representation, and an irrep whose Frobenius-Schur indicator is +1
is then changed to a real orthogonal basis.  The construction here:

1. Left and right regular representations L(g), R(g) (|G| x |G| permutation
   matrices); every R(g) commutes with every L(h).
2. A random Hermitian element S = A + A^H, A = sum_g c_g R(g), of the right
   regular algebra.  Each eigenspace of S is L-invariant and, for generic c,
   carries exactly one copy of one irrep; rho(g) = Q^H L(g) Q on it.
3. Distinct irreps are told apart by their characters.  For indicator +1 the
   same construction with a *real symmetric* S (real c_g, S = A + A^T) yields
   real eigenspaces and thus the irrep in real orthogonal form.

Irrep order: dimension ascending, then the character vector over the canonical
class order (element order, class size, smallest member) descending
lexicographically by real parts rounded to 1e-9, ties broken by imaginary
parts.  The trivial irrep comes first.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .group import Group


@dataclass
class Irrep:
    dim: int
    rho: np.ndarray          # (|G|, d, d) float64 (real form) or complex128
    chars: np.ndarray        # (|G|,) complex128
    indicator: int           # Frobenius-Schur: +1 real, 0 complex, -1 quaternionic

    @property
    def is_real(self) -> bool:
        return not np.iscomplexobj(self.rho)


def regular_reps(G: Group):
    """Dense L(g), R(g) (only used by tests; the split below works on indices)."""
    n = G.order
    Lm = np.zeros((n, n, n))
    Rm = np.zeros((n, n, n))
    ar = np.arange(n)
    for g in range(n):
        Lm[g, G.mul[g, ar], ar] = 1.0                # e_y -> e_{g y}
        Rm[g, G.mul[ar, G.inv[g]], ar] = 1.0         # e_y -> e_{y g^-1}
    return Lm, Rm


def right_algebra_element(G: Group, c):
    """A = sum_g c_g R(g) as a dense matrix: A[x, y] = c[x^-1 y]."""
    return np.asarray(c)[G.mul[G.inv][:, :]]


def restrict_left(G: Group, Q):
    """rho(g) = Q^H L(g) Q for all g; (L(g) Q)[x] = Q[g^-1 x]."""
    n = G.order
    LQ = Q[G.mul[G.inv[:, None], np.arange(n)[None, :]]]      # (|G|, n, m)
    return np.einsum("xi,gxj->gij", Q.conj(), LQ)


def _clusters(w, tol):
    groups, start = [], 0
    for i in range(1, len(w) + 1):
        if i == len(w) or w[i] - w[i - 1] > tol:
            groups.append((start, i))
            start = i
    return groups


def _split(G: Group, real: bool, seed: int):
    rng = np.random.default_rng(seed)
    n = G.order
    if real:
        c = rng.standard_normal(n)
    else:
        c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = right_algebra_element(G, c)
    S = A + A.conj().T
    w, Q = np.linalg.eigh(S)
    tol = 1e-7 * max(1.0, np.ptp(w))
    out = []
    for a, b in _clusters(w, tol):
        Qc = Q[:, a:b]
        rho = restrict_left(G, Qc)
        if real:
            rho = rho.real
        out.append(rho)
    return out


def _char_key(chars_by_class):
    return tuple(np.round(chars_by_class.real, 6)) + tuple(np.round(chars_by_class.imag, 6))


def compute_irreps(G: Group, seed: int = 12345) -> list:
    n = G.order
    rep_class = [c[0] for c in G.classes]
    found = {}
    for attempt in range(5):
        found.clear()
        ok = True
        for rho in _split(G, real=False, seed=seed + attempt):
            chars = np.trace(rho, axis1=1, axis2=2)
            if abs(np.vdot(chars, chars).real / n - 1.0) > 1e-8:
                ok = False
                break
            key = _char_key(chars[rep_class])
            found.setdefault(key, (rho, chars))
        if ok and sum(r.shape[1] ** 2 for r, _ in found.values()) == n:
            break
    else:
        raise RuntimeError("irrep construction failed")
    # real forms for indicator +1
    real_forms = {}
    for attempt in range(5):
        for rho in _split(G, real=True, seed=seed + 100 + attempt):
            chars = np.trace(rho, axis1=1, axis2=2)
            if abs(np.dot(chars, chars) / n - 1.0) > 1e-8:
                continue
            real_forms.setdefault(_char_key(chars[rep_class].astype(complex)), rho)
        need = [k for k, (r, ch) in found.items()
                if abs(np.sum(ch[G.mul[np.arange(n), np.arange(n)]]).real / n - 1.0) < 1e-8]
        if all(k in real_forms for k in need):
            break
    irreps = []
    for key, (rho, chars) in found.items():
        ind = np.sum(chars[G.mul[np.arange(n), np.arange(n)]]) / n
        indicator = int(round(ind.real))
        if indicator == 1:
            rho = real_forms[key]
            chars = np.trace(rho, axis1=1, axis2=2).astype(complex)
        irreps.append(Irrep(rho.shape[1], rho, chars, indicator))

    def sort_key(ir):
        cc = ir.chars[rep_class]
        re = np.round(cc.real, 9)
        im = np.round(cc.imag, 9)
        return (ir.dim, tuple(-re), tuple(-im))

    irreps.sort(key=sort_key)
    return irreps


def check_irreps(G: Group, irreps, tol=1e-10) -> float:
    """Largest residual of homomorphism, unitarity and great orthogonality."""
    n = G.order
    worst = 0.0
    for ir in irreps:
        rho = ir.rho
        prod = np.einsum("gij,hjk->ghik", rho, rho)
        worst = max(worst, np.max(np.abs(prod - rho[G.mul])))
        eye = np.eye(ir.dim)
        worst = max(worst, np.max(np.abs(np.einsum("gji,gjk->gik", rho.conj(), rho) - eye)))
    for a, A in enumerate(irreps):
        for b, B in enumerate(irreps):
            m = np.einsum("gij,gkl->ijkl", A.rho.conj(), B.rho) * (A.dim / n)
            if a == b:
                d = A.dim
                ref = np.einsum("ik,jl->ijkl", np.eye(d), np.eye(d))
            else:
                ref = 0.0
            worst = max(worst, np.max(np.abs(m - ref)))
    return worst
