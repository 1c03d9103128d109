"""M-sector basis and the Heisenberg Hamiltonian (paper Section 2.1, Eqs. 1-3).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

Labels follow Eq. (2): n = sum_k a_k d^k with a_k = m_k + s the k-th base-d
digit (d = 2s + 1).  A sector holds the labels whose digits sum to Ns + M;
they are returned in ascending label order.  H_M is built entry by entry from
Eq. (1): the diagonal J m_i m_j per bond and, for each bond and each sign, the
flip s_i^+ s_j^- or s_i^- s_j^+ with the coefficient of Eq. (3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def enumerate_sector(N: int, two_s: int, two_M: int) -> np.ndarray:
    d = two_s + 1
    A2 = N * two_s + two_M
    if A2 % 2:
        return np.zeros(0, dtype=np.int64)
    A = A2 // 2
    # build labels digit by digit from the highest site down; keep partial sums
    labels = np.zeros(1, dtype=np.int64)
    sums = np.zeros(1, dtype=np.int64)
    for k in range(N - 1, -1, -1):
        remaining_max = k * (d - 1)      # max sum of the digits still to place
        new_l, new_s = [], []
        for a in range(d):
            s2 = sums + a
            ok = (s2 <= A) & (s2 + remaining_max >= A)
            new_l.append(labels[ok] * d + a)
            new_s.append(s2[ok])
        labels = np.concatenate(new_l)
        sums = np.concatenate(new_s)
    return np.sort(labels)


def digits(labels, N: int, d: int) -> np.ndarray:
    labels = np.asarray(labels, dtype=np.int64)
    out = np.empty((len(labels), N), dtype=np.int64)
    x = labels.copy()
    for k in range(N):
        out[:, k] = x % d
        x //= d
    return out


def from_digits(dig, d: int) -> np.ndarray:
    dig = np.asarray(dig, dtype=np.int64)
    w = d ** np.arange(dig.shape[1], dtype=np.int64)
    return dig @ w


def ladder_factor(two_s: int, two_m: np.ndarray, up: bool) -> np.ndarray:
    """sqrt(s(s+1) - m(m +/- 1)) with m given as 2m (float64)."""
    s = two_s / 2.0
    m = two_m / 2.0
    val = s * (s + 1) - m * (m + 1) if up else s * (s + 1) - m * (m - 1)
    return np.sqrt(np.maximum(val, 0.0))


def diag_energy(dig, bonds, J, two_s: int) -> np.ndarray:
    m = dig - two_s / 2.0
    e = np.zeros(len(dig))
    for (i, j), Jb in zip(bonds, J):
        e += Jb * m[:, i] * m[:, j]
    return e


def hamiltonian(labels, N: int, two_s: int, bonds, J) -> sp.csr_matrix:
    """Sparse H_M (FP64) in the given sorted label basis."""
    d = two_s + 1
    labels = np.asarray(labels, dtype=np.int64)
    D = len(labels)
    dig = digits(labels, N, d)
    rows, cols, vals = [np.arange(D)], [np.arange(D)], [diag_energy(dig, bonds, J, two_s)]
    pw = d ** np.arange(N, dtype=np.int64)
    two_m = 2 * dig - two_s
    for (i, j), Jb in zip(bonds, J):
        for up_i in (True, False):
            # up_i: s_i^+ s_j^- ; else s_i^- s_j^+
            if up_i:
                ok = (dig[:, i] < d - 1) & (dig[:, j] > 0)
            else:
                ok = (dig[:, i] > 0) & (dig[:, j] < d - 1)
            src = np.nonzero(ok)[0]
            if len(src) == 0:
                continue
            fi = ladder_factor(two_s, two_m[src, i], up_i)
            fj = ladder_factor(two_s, two_m[src, j], not up_i)
            c = 0.5 * Jb * fi * fj
            delta = pw[i] - pw[j] if up_i else pw[j] - pw[i]
            tgt = labels[src] + delta
            pos = np.searchsorted(labels, tgt)
            assert np.all(labels[pos] == tgt)
            # H|src> contains c |tgt>  ->  H[tgt, src] = c
            rows.append(pos)
            cols.append(src)
            vals.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return sp.csr_matrix((v, (r, c)), shape=(D, D))


def permute_labels(labels, perm, N: int, d: int) -> np.ndarray:
    """Labels of U(g)|n>: the digit on site k moves to site perm[k]."""
    dig = digits(labels, N, d)
    pw = d ** np.asarray(perm, dtype=np.int64)
    return dig @ pw
