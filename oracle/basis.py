"""Symmetry-adapted basis of one (M, Gamma, alpha) block (paper Section 2.3).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

Plain-definition steps:

* orbit of n: {U(g) n : g in G}; representative r = the smallest label
  (Section 2.3); the connecting element of a label a is the smallest group
  index h with U(h) a = r (brute force over every g).
* Stab(r) = {g : U(g) r = r} (Eq. 8); L_r = |G| / |Stab(r)|.
* n_Gamma(r) = (1/|Stab|) sum_{h in Stab} chi(h)^* (Section 2.3).
* V_S: orthonormal basis of the range of P_S = (1/|S|) sum_{h in S} rho(h)^*
  (the Gram matrix of Eq. (10) is (d|S|/|G|) P_S, so its non-zero eigenvalue
  is lambda = d|S|/|G| and its eigenvectors span range(P_S), Eq. (11)).  The
  basis is fixed by modified Gram-Schmidt over the columns of P_S in index
  order, a column dropped when its residual norm is below 1e-8, signs such
  that the diagonal of the triangular factor is positive.
* psi_{r,k,alpha} = d/(|G| sqrt(lambda)) sum_g [rho(g)^* V_r]_{alpha,k} U(g)|r>
  (Eq. 12), assembled as the columns of a sparse D_M x D matrix Psi in the
  order (representative ascending, k ascending).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .group import Group
from .irreps import Irrep
from .sector import digits, enumerate_sector


def apply_all(G: Group, labels, N: int, d: int) -> np.ndarray:
    """(len(labels), |G|) array of the labels of U(g)|n>.

    For G x Z2 (``spinflip.FlipGroup``) the columns |G|..2|G|-1 are U(g) F|n>."""
    if getattr(G, "flip", False):
        from .spinflip import flip_labels
        labels = np.asarray(labels, dtype=np.int64)
        return np.hstack([apply_all(G.base, labels, N, d), apply_all(G.base, flip_labels(labels, N, d), N, d)])
    dig = digits(labels, N, d)
    pw = (d ** G.perms).T            # (N, |G|): weight of site k under g is d^{perm_g[k]}
    return dig @ pw


def canonicalize(G: Group, labels, N: int, d: int, chunk: int = 1 << 16):
    """(rep label, connecting element h) with U(h) a = rep; h smallest among minimisers."""
    labels = np.asarray(labels, dtype=np.int64)
    reps = np.empty(len(labels), dtype=np.int64)
    hs = np.empty(len(labels), dtype=np.int64)
    for s in range(0, len(labels), chunk):
        imgs = apply_all(G, labels[s:s + chunk], N, d)
        h = np.argmin(imgs, axis=1)                 # first minimiser = smallest index
        reps[s:s + chunk] = imgs[np.arange(len(h)), h]
        hs[s:s + chunk] = h
    return reps, hs


def stabilizer(G: Group, r: int, N: int, d: int) -> np.ndarray:
    imgs = apply_all(G, np.array([r]), N, d)[0]
    return np.nonzero(imgs == r)[0]


def mgs_range(P, tol=1e-8):
    cols = []
    for j in range(P.shape[1]):
        v = P[:, j].astype(P.dtype, copy=True)
        for q in cols:
            v = v - np.vdot(q, v) * q
        nrm = np.linalg.norm(v)
        if nrm < tol:
            continue
        cols.append(v / nrm)
    if not cols:
        return np.zeros((P.shape[0], 0), dtype=P.dtype)
    return np.stack(cols, axis=1)


@dataclass
class SectorReps:
    N: int
    two_s: int
    two_M: int
    labels: np.ndarray       # all sector labels, ascending
    canon: np.ndarray        # representative of each sector label
    canon_h: np.ndarray      # connecting element of each sector label
    reps: np.ndarray         # sorted representative labels
    stab_sets: list          # per distinct stabilizer (first-appearance order): index array
    stab_id: np.ndarray      # per representative


def sector_reps(G: Group, N: int, two_s: int, two_M: int) -> SectorReps:
    d = two_s + 1
    labels = enumerate_sector(N, two_s, two_M)
    canon, h = canonicalize(G, labels, N, d)
    reps = np.unique(canon)
    stab_sets, stab_id, index = [], np.empty(len(reps), dtype=np.int64), {}
    for i, r in enumerate(reps):
        S = tuple(stabilizer(G, int(r), N, d).tolist())
        if S not in index:
            index[S] = len(stab_sets)
            stab_sets.append(np.array(S, dtype=np.int64))
        stab_id[i] = index[S]
    return SectorReps(N, two_s, two_M, labels, canon, h, reps, stab_sets, stab_id)


@dataclass
class Block:
    sec: SectorReps
    irrep: Irrep
    alpha: int
    n_stab: np.ndarray       # n_Gamma per distinct stabilizer
    V_stab: list             # V_S per distinct stabilizer (d x n)
    n_rep: np.ndarray        # n_Gamma per representative
    offsets: np.ndarray      # exclusive prefix sum of n_rep
    L_rep: np.ndarray        # orbit length per representative
    Psi: sp.csr_matrix       # D_M x D

    @property
    def D(self) -> int:
        return int(self.n_rep.sum())


def stab_data(irrep: Irrep, S: np.ndarray):
    rho = irrep.rho
    P = np.conj(rho[S]).sum(axis=0) / len(S)
    n_char = np.sum(np.conj(irrep.chars[S])).real / len(S)
    n = int(round(n_char))
    V = mgs_range(P)
    if V.shape[1] != n:
        raise AssertionError(f"MGS rank {V.shape[1]} != character count {n}")
    return n, V


def build_block(G: Group, irrep: Irrep, sec: SectorReps, alpha: int = 0, with_psi: bool = True) -> Block:
    d = irrep.dim
    Gn = G.order
    n_stab, V_stab = [], []
    for S in sec.stab_sets:
        n, V = stab_data(irrep, S)
        n_stab.append(n)
        V_stab.append(V)
    n_stab = np.array(n_stab, dtype=np.int64)
    n_rep = n_stab[sec.stab_id]
    offsets = np.concatenate([[0], np.cumsum(n_rep)[:-1]]).astype(np.int64)
    L_rep = np.array([Gn // len(sec.stab_sets[s]) for s in sec.stab_id], dtype=np.int64)
    Psi = None
    if with_psi:
        Psi = explicit_psi(G, irrep, sec, alpha, n_rep, offsets, V_stab)
    return Block(sec, irrep, alpha, n_stab, V_stab, n_rep, offsets, L_rep, Psi)


def explicit_psi(G, irrep, sec, alpha, n_rep, offsets, V_stab):
    d = irrep.dim
    Gn = G.order
    N, dd = sec.N, sec.two_s + 1
    active = np.nonzero(n_rep > 0)[0]
    D = int(n_rep.sum())
    rows, cols, vals = [], [], []
    if len(active):
        imgs = apply_all(G, sec.reps[active], N, dd)              # (nact, |G|)
        pos = np.searchsorted(sec.labels, imgs)
        rhoc = np.conj(irrep.rho)                                  # (|G|, d, d)
        for ai, i in enumerate(active):
            S = sec.stab_sets[sec.stab_id[i]]
            lam = d * len(S) / Gn
            V = V_stab[sec.stab_id[i]]
            coef = (rhoc[:, alpha, :] @ V) * (d / (Gn * np.sqrt(lam)))  # (|G|, n)
            for k in range(n_rep[i]):
                rows.append(pos[ai])
                cols.append(np.full(Gn, offsets[i] + k))
                vals.append(coef[:, k])
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
    else:
        r = c = np.zeros(0, dtype=np.int64)
        v = np.zeros(0)
    dtype = np.complex128 if np.iscomplexobj(irrep.rho) else np.float64
    return sp.csr_matrix((v.astype(dtype), (r, c)), shape=(len(sec.labels), D))
