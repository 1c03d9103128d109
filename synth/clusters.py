"""Synthetic cluster inputs: site geometry, bond lists and symmetry generators.

This module produces *inputs* only (the cluster graph and the site-permutation
generators a user would hand to the library); it contains none of the method's
arithmetic.  Both the CPU oracle and the GPU path's tests read from here.

Conventions
-----------
* Sites of the polyhedra are numbered lexicographically by their coordinates
  rounded to 1e-6 (a canonical numbering independent of construction order).
* A generator is a permutation array ``perm`` with ``perm[k]`` = the site that
  site ``k`` is carried to by the geometric operation (the spin on site ``k``
  moves to site ``perm[k]``).
* Bonds are nearest-neighbour pairs ``(i, j)`` with ``i < j`` sorted
  lexicographically; ``J`` defaults to 1 on every bond.

The clusters are the ones of the paper's benchmarks (Section 4, Table 1) and of
its built-in providers (Section 3): icosahedron, dodecahedron and
icosidodecahedron with I_h (order 120), cuboctahedron with O_h (order 48), and
periodic L x L square tori with translations x C4v.  Small graphs (dimer,
rings, complete graphs) serve closed-form checks.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0


@dataclass
class Cluster:
    name: str
    N: int
    bonds: np.ndarray            # (nbonds, 2) int32, i < j
    gens: np.ndarray             # (ngens, N) int32 permutation arrays
    J: np.ndarray = None         # (nbonds,) float64
    group_order: int = 0         # expected |G| (documentation / tests)
    coords: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        self.bonds = np.asarray(self.bonds, dtype=np.int32).reshape(-1, 2)
        self.gens = np.asarray(self.gens, dtype=np.int32).reshape(-1, self.N)
        if self.J is None:
            self.J = np.ones(len(self.bonds), dtype=np.float64)
        self.J = np.asarray(self.J, dtype=np.float64)

    @property
    def nbonds(self) -> int:
        return len(self.bonds)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _cyclic(v):
    x, y, z = v
    return [(x, y, z), (y, z, x), (z, x, y)]


def _sorted_sites(pts):
    pts = np.asarray(pts, dtype=np.float64)
    key = np.round(pts, 6)
    order = sorted(range(len(pts)), key=lambda i: tuple(key[i]))
    return pts[order]


def _nn_bonds(pts, tol=1e-6):
    n = len(pts)
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
    dmin = np.min(d[~np.eye(n, dtype=bool)])
    bonds = [(i, j) for i in range(n) for j in range(i + 1, n) if abs(d[i, j] - dmin) < tol]
    return np.array(bonds, dtype=np.int32)


def _rot(axis, angle):
    u = np.asarray(axis, dtype=np.float64)
    u = u / np.linalg.norm(u)
    c, s = np.cos(angle), np.sin(angle)
    ux = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return c * np.eye(3) + s * ux + (1 - c) * np.outer(u, u)


def _site_perm(pts, R, tol=1e-6):
    img = pts @ R.T
    perm = np.empty(len(pts), dtype=np.int32)
    for k, p in enumerate(img):
        dist = np.linalg.norm(pts - p, axis=1)
        j = int(np.argmin(dist))
        if dist[j] > tol:
            raise ValueError("operation does not map the cluster onto itself")
        perm[k] = j
    if len(set(perm.tolist())) != len(pts):
        raise ValueError("not a permutation")
    return perm


def _icosahedron_vertices():
    pts = []
    for a in (-1.0, 1.0):
        for b in (-PHI, PHI):
            pts += _cyclic((0.0, a, b))
    return _sorted_sites(pts)


def _ih_generators(pts):
    """C5 about a vertex axis of the icosahedron, C3 about a face axis, inversion."""
    ico = _icosahedron_vertices()
    v = ico[0]
    # a face of the icosahedron: three mutually adjacent vertices
    b = _nn_bonds(ico)
    adj = {i: set() for i in range(12)}
    for i, j in b:
        adj[i].add(j)
        adj[j].add(i)
    face = None
    for i, j in b:
        common = sorted(adj[i] & adj[j])
        if common:
            face = (i, j, common[0])
            break
    fc = ico[list(face)].mean(axis=0)
    g5 = _site_perm(pts, _rot(v, 2 * np.pi / 5))
    g3 = _site_perm(pts, _rot(fc, 2 * np.pi / 3))
    gi = _site_perm(pts, -np.eye(3))
    return np.stack([g5, g3, gi])


# ----------------------------------------------------------------------------
# cluster providers
# ----------------------------------------------------------------------------

def icosahedron() -> Cluster:
    pts = _icosahedron_vertices()
    return Cluster("icosahedron", 12, _nn_bonds(pts), _ih_generators(pts), group_order=120, coords=pts)


def dodecahedron() -> Cluster:
    ico = _icosahedron_vertices()
    b = _nn_bonds(ico)
    adj = {i: set() for i in range(12)}
    for i, j in b:
        adj[i].add(j)
        adj[j].add(i)
    faces = set()
    for i, j in b:
        for k in adj[i] & adj[j]:
            faces.add(tuple(sorted((i, j, k))))
    pts = _sorted_sites([ico[list(f)].mean(axis=0) for f in sorted(faces)])
    return Cluster("dodecahedron", 20, _nn_bonds(pts), _ih_generators(pts), group_order=120, coords=pts)


def icosidodecahedron() -> Cluster:
    ico = _icosahedron_vertices()
    b = _nn_bonds(ico)
    pts = _sorted_sites([(ico[i] + ico[j]) / 2 for i, j in b])
    return Cluster("icosidodecahedron", 30, _nn_bonds(pts), _ih_generators(pts), group_order=120, coords=pts)


def cuboctahedron() -> Cluster:
    pts = []
    for a in (-1.0, 1.0):
        for b in (-1.0, 1.0):
            pts += _cyclic((a, b, 0.0))
    pts = _sorted_sites(pts)
    g4 = _site_perm(pts, _rot((0, 0, 1), np.pi / 2))
    g3 = _site_perm(pts, _rot((1, 1, 1), 2 * np.pi / 3))
    gi = _site_perm(pts, -np.eye(3))
    return Cluster("cuboctahedron", 12, _nn_bonds(pts), np.stack([g4, g3, gi]), group_order=48, coords=pts)


def square_torus(L: int, translations_only: bool = False) -> Cluster:
    """Periodic L x L square lattice; site (x, y) has index x * L + y.

    Generators: unit translations T_x, T_y; for the full space group also the
    90-degree rotation C4 about site 0 and the mirror x -> -x.
    """
    N = L * L

    def idx(x, y):
        return (x % L) * L + (y % L)

    bonds = set()
    for x in range(L):
        for y in range(L):
            for dx, dy in ((1, 0), (0, 1)):
                i, j = idx(x, y), idx(x + dx, y + dy)
                bonds.add((min(i, j), max(i, j)))
    bonds = np.array(sorted(bonds), dtype=np.int32)

    def perm_of(f):
        p = np.empty(N, dtype=np.int32)
        for x in range(L):
            for y in range(L):
                p[idx(x, y)] = idx(*f(x, y))
        return p

    gens = [perm_of(lambda x, y: (x + 1, y)), perm_of(lambda x, y: (x, y + 1))]
    order = N
    if not translations_only:
        gens += [perm_of(lambda x, y: (-y, x)), perm_of(lambda x, y: (-x, y))]
        order = 8 * N
    name = f"square{L}x{L}" + ("_T" if translations_only else "")
    return Cluster(name, N, bonds, np.stack(gens), group_order=order)


def ring(N: int, dihedral: bool = True) -> Cluster:
    bonds = np.array(sorted((min(i, (i + 1) % N), max(i, (i + 1) % N)) for i in range(N)), dtype=np.int32)
    if N == 2:
        bonds = np.array([[0, 1]], dtype=np.int32)
    gens = [np.array([(k + 1) % N for k in range(N)], dtype=np.int32)]
    if dihedral and N > 2:
        gens.append(np.array([(-k) % N for k in range(N)], dtype=np.int32))
    order = 2 * N if (dihedral and N > 2) else N
    return Cluster(f"ring{N}" + ("" if dihedral else "_C"), N, bonds, np.stack(gens), group_order=order)


def dimer() -> Cluster:
    return Cluster("dimer", 2, np.array([[0, 1]]), np.array([[1, 0]]), group_order=2)


def complete_graph(N: int) -> Cluster:
    bonds = np.array(list(itertools.combinations(range(N), 2)), dtype=np.int32)
    cyc = np.array([(k + 1) % N for k in range(N)], dtype=np.int32)
    swap = np.arange(N, dtype=np.int32)
    swap[0], swap[1] = 1, 0
    order = 1
    for k in range(2, N + 1):
        order *= k
    return Cluster(f"K{N}", N, bonds, np.stack([cyc, swap]), group_order=order)


def petersen() -> Cluster:
    """Petersen graph: sites are the 2-subsets of {0..4} (lexicographic), bonds
    join disjoint subsets (15 bonds, 3 per site); its automorphism group is S5
    (order 120, irreps of dimension 1, 1, 4, 4, 5, 5, 6), generated by the
    transposition (0 1) and the 5-cycle (0 1 2 3 4) acting on the subsets."""
    subsets = list(itertools.combinations(range(5), 2))
    index = {s: k for k, s in enumerate(subsets)}
    bonds = np.array([(a, b) for a in range(10) for b in range(a + 1, 10)
                      if not set(subsets[a]) & set(subsets[b])], dtype=np.int32)

    def perm_of(p):
        return np.array([index[tuple(sorted((p[i], p[j])))] for i, j in subsets], dtype=np.int32)

    gens = np.stack([perm_of([1, 0, 2, 3, 4]), perm_of([1, 2, 3, 4, 0])])
    return Cluster("petersen", 10, bonds, gens, group_order=120)


def _qmul(p, q):
    a1, b1, c1, d1 = p
    a2, b2, c2, d2 = q
    return (a1 * a2 - b1 * b2 - c1 * c2 - d1 * d2, a1 * b2 + b1 * a2 + c1 * d2 - d1 * c2,
            a1 * c2 - b1 * d2 + c1 * a2 + d1 * b2, a1 * d2 + b1 * c2 - c1 * b2 + d1 * a2)


def dicyclic(n: int) -> Cluster:
    """Dicyclic group Dic_n (order 4n; Dic_2 is the quaternion group Q8) as
    unit quaternions generated by a = exp(i pi / n) and x = j, acting on its 4n
    elements (the sites) by left multiplication.  Bonds: the Cayley graph of
    right multiplication by a and by x, which left multiplication preserves.
    Its two-dimensional irreps on which a^n = -1 acts are quaternionic."""
    gen_q = [(np.cos(np.pi / n), np.sin(np.pi / n), 0.0, 0.0), (0.0, 0.0, 1.0, 0.0)]
    elems = [(1.0, 0.0, 0.0, 0.0)]

    def find(q):
        for k, e in enumerate(elems):
            if max(abs(u - v) for u, v in zip(e, q)) < 1e-9:
                return k
        return -1

    k = 0
    while k < len(elems):
        for g in gen_q:
            q = _qmul(elems[k], g)
            if find(q) < 0:
                elems.append(q)
        k += 1
    N = len(elems)
    gens = [np.array([find(_qmul(g, e)) for e in elems], dtype=np.int32) for g in gen_q]
    bonds = set()
    for g in gen_q:
        for i, e in enumerate(elems):
            j = find(_qmul(e, g))
            if i != j:
                bonds.add((min(i, j), max(i, j)))
    return Cluster(f"dic{n}", N, np.array(sorted(bonds), dtype=np.int32), np.stack(gens), group_order=4 * n)


BUILTIN = {
    "icosahedron": icosahedron,
    "dodecahedron": dodecahedron,
    "icosidodecahedron": icosidodecahedron,
    "cuboctahedron": cuboctahedron,
    "square4": lambda: square_torus(4),
    "square6": lambda: square_torus(6),
    "dimer": dimer,
    "petersen": petersen,
}


def get(name: str) -> Cluster:
    if name in BUILTIN:
        return BUILTIN[name]()
    if name.startswith("ring"):
        if name.endswith("_C"):      # cyclic group only (translations of the ring)
            return ring(int(name[4:-2]), dihedral=False)
        return ring(int(name[4:]))
    if name.startswith("dic"):
        return dicyclic(int(name[3:]))
    if name.startswith("K"):
        return complete_graph(int(name[1:]))
    if name.startswith("square") and "x" in name:
        L = int(name[6:].split("x")[0])
        return square_torus(L, translations_only=name.endswith("_T"))
    raise KeyError(name)
