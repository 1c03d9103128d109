"""Permutation group from site-permutation generators (paper Section 3).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

The paper closes user generators into the full group; here the closure is a
plain breadth-first search over products (not Dimino's algorithm).  Elements
are sorted lexicographically by their image arrays, so the identity is element
0.  Composition follows U(g)U(h) = U(gh) with pi_{gh}(k) = pi_g(pi_h(k)) (the
homomorphism convention stated with Appendix A).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Group:
    perms: np.ndarray     # (|G|, N) int64, lexicographically sorted
    mul: np.ndarray       # (|G|, |G|) index of g*h
    inv: np.ndarray       # (|G|,)
    classes: list         # list of sorted index lists, in canonical class order
    class_of: np.ndarray  # (|G|,) class index
    order_of: np.ndarray  # (|G|,) element order

    @property
    def order(self) -> int:
        return len(self.perms)

    @property
    def N(self) -> int:
        return self.perms.shape[1]


def close(gens, N: int, max_order: int = 65535) -> Group:
    gens = [tuple(int(x) for x in g) for g in np.asarray(gens).reshape(-1, N)]
    for g in gens:
        if sorted(g) != list(range(N)):
            raise ValueError("generator is not a permutation")
    ident = tuple(range(N))
    seen = {ident}
    frontier = [ident]
    while frontier:
        nxt = []
        for g in frontier:
            for s in gens:
                h = tuple(g[s[k]] for k in range(N))   # g * s
                if h not in seen:
                    seen.add(h)
                    nxt.append(h)
                    if len(seen) > max_order:
                        raise ValueError("group too large")
        frontier = nxt
    elems = sorted(seen)
    perms = np.array(elems, dtype=np.int64)
    index = {e: i for i, e in enumerate(elems)}
    n = len(elems)
    mul = np.empty((n, n), dtype=np.int64)
    for i in range(n):
        gi = perms[i]
        comp = gi[perms]          # row j: g_i(g_j(k))
        for j in range(n):
            mul[i, j] = index[tuple(comp[j])]
    inv = np.empty(n, dtype=np.int64)
    for i in range(n):
        inv[i] = int(np.nonzero(mul[i] == 0)[0][0])
    order_of = np.empty(n, dtype=np.int64)
    for i in range(n):
        k, x = 1, i
        while x != 0:
            x = mul[x, i]
            k += 1
        order_of[i] = k
    # conjugacy classes
    cls_id = -np.ones(n, dtype=np.int64)
    raw = []
    for i in range(n):
        if cls_id[i] >= 0:
            continue
        members = sorted({int(mul[mul[x, i], inv[x]]) for x in range(n)})
        for m in members:
            cls_id[m] = len(raw)
        raw.append(members)
    # canonical class order: (element order, class size, smallest member index)
    order = sorted(range(len(raw)), key=lambda c: (order_of[raw[c][0]], len(raw[c]), raw[c][0]))
    classes = [raw[c] for c in order]
    class_of = np.empty(n, dtype=np.int64)
    for ci, c in enumerate(classes):
        class_of[c] = ci
    return Group(perms, mul, inv, classes, class_of, order_of)


def cycle_type(perm) -> tuple:
    perm = list(perm)
    seen = [False] * len(perm)
    lens = []
    for k in range(len(perm)):
        if not seen[k]:
            L, x = 0, k
            while not seen[x]:
                seen[x] = True
                x = perm[x]
                L += 1
            lens.append(L)
    return tuple(sorted(lens))
