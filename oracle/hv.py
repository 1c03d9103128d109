"""Hamiltonian action in the symmetry-adapted basis, by plain definition.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

Y = Psi^H H_M Psi X, with Psi the explicit Eq. (12) basis and H_M the sector
Hamiltonian of Eqs. (1)-(3).  This never uses the closed-form matrix element
of Eq. (15); it therefore checks that formula as well as any kernel built on
it.  For blocks too large to expand, ``sampled_rows`` evaluates selected output
rows <psi_{p,k'}| H |Psi x> by expanding psi_p over its orbit, applying H to
each orbit state, and reading (Psi x) at every reached state after a brute-
force orbit search (every group element applied).
"""
from __future__ import annotations

import numpy as np

from .basis import apply_all, canonicalize, stab_data, stabilizer
from .sector import digits, from_digits, ladder_factor


def block_matrix(block, H):
    Psi = block.Psi
    M = (Psi.conj().T @ (H @ Psi))
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M)


def apply(block, H, X):
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    return np.asarray(block.Psi.conj().T @ (H @ (block.Psi @ X)))


def _flips(labels, N, two_s, bonds, J):
    """All (target label, coefficient, source position) of the off-diagonal part."""
    d = two_s + 1
    dig = digits(labels, N, d)
    two_m = 2 * dig - two_s
    pw = d ** np.arange(N, dtype=np.int64)
    out_t, out_c, out_src = [], [], []
    for (i, j), Jb in zip(bonds, J):
        for up_i in (True, False):
            ok = (dig[:, i] < d - 1) & (dig[:, j] > 0) if up_i else (dig[:, i] > 0) & (dig[:, j] < d - 1)
            src = np.nonzero(ok)[0]
            if len(src) == 0:
                continue
            c = 0.5 * Jb * ladder_factor(two_s, two_m[src, i], up_i) * ladder_factor(two_s, two_m[src, j], not up_i)
            delta = pw[i] - pw[j] if up_i else pw[j] - pw[i]
            out_t.append(labels[src] + delta)
            out_c.append(c)
            out_src.append(src)
    if not out_t:
        return np.zeros(0, np.int64), np.zeros(0), np.zeros(0, np.int64)
    return np.concatenate(out_t), np.concatenate(out_c), np.concatenate(out_src)


class _RepCache:
    def __init__(self, G, irrep, N, d):
        self.G, self.irrep, self.N, self.d = G, irrep, N, d
        self.cache = {}

    def get(self, r):
        if r not in self.cache:
            S = stabilizer(self.G, int(r), self.N, self.d)
            n, V = stab_data(self.irrep, S)
            imgs = apply_all(self.G, np.array([r]), self.N, self.d)[0]
            self.cache[r] = (n, V, len(S), imgs)
        return self.cache[r]


def psi_values(G, irrep, alpha, rc, r, b):
    """psi_{r,k,alpha}(b) for all k (vector over k) at an orbit state b of r."""
    n, V, nS, imgs = rc.get(r)
    d, Gn = irrep.dim, G.order
    lam = d * nS / Gn
    gs = np.nonzero(imgs == b)[0]
    coef = np.conj(irrep.rho[gs])[:, alpha, :].sum(axis=0) @ V
    return coef * (d / (Gn * np.sqrt(lam)))


def sampled_rows(G, irrep, alpha, N, two_s, bonds, J, p_labels, xfun, nvec):
    """Rows (p, k') of Psi^H H Psi X for representatives p (labels).

    ``xfun(rep_label, n)`` returns the (n, nvec) slice of X at representative
    rep_label.  Returns a list of (n_p, nvec) arrays.
    """
    d = two_s + 1
    rc = _RepCache(G, irrep, N, d)
    out = []
    for p in p_labels:
        p = int(p)
        n_p, V_p, nS_p, imgs_p = rc.get(p)
        if n_p == 0:
            out.append(np.zeros((0, nvec)))
            continue
        orbit = np.unique(imgs_p)
        # coefficients psi_p(b) for each orbit state b, (len(orbit), n_p)
        cpsi = np.stack([psi_values(G, irrep, alpha, rc, p, b) for b in orbit])
        # H applied at each orbit state: diagonal + flips
        dig = digits(orbit, N, d)
        m = dig - two_s / 2.0
        diag = np.zeros(len(orbit))
        for (i, j), Jb in zip(bonds, J):
            diag += Jb * m[:, i] * m[:, j]
        tgt, c, src = _flips(orbit, N, two_s, bonds, J)
        # (Psi x)(b) for b in orbit and for every flip target
        allb = np.concatenate([orbit, tgt])
        reps, _ = canonicalize(G, allb, N, d)
        psix = np.zeros((len(allb), nvec), dtype=np.result_type(irrep.rho.dtype, np.float64))
        for q in range(len(allb)):
            r = int(reps[q])
            n_r = rc.get(r)[0]
            if n_r == 0:
                continue
            pv = psi_values(G, irrep, alpha, rc, r, int(allb[q]))      # (n_r,)
            psix[q] = pv @ np.asarray(xfun(r, n_r)).reshape(n_r, nvec)
        hpsix = diag[:, None] * psix[:len(orbit)]
        np.add.at(hpsix, src, c[:, None] * psix[len(orbit):])
        out.append(np.conj(cpsi).T @ hpsix)
    return out
