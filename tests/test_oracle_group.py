"""Oracle pins: group closure and irreps (paper Section 3) against mathematics."""
import numpy as np
import pytest

from conftest import golden
from oracle import group, irreps
from synth import clusters

PHI = (1 + 5 ** 0.5) / 2


@pytest.fixture(scope="module")
def ih():
    cl = clusters.icosahedron()
    G = group.close(cl.gens, cl.N)
    return cl, G, irreps.compute_irreps(G)


@pytest.mark.parametrize("name,order", [
    ("icosahedron", 120), ("dodecahedron", 120), ("icosidodecahedron", 120),
    ("cuboctahedron", 48), ("square4", 128), ("square6", 288), ("ring6", 12),
    ("dimer", 2), ("K4", 24), ("petersen", 120)])
def test_group_order_and_bond_invariance(name, order):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    assert G.order == order
    assert np.array_equal(G.perms[0], np.arange(cl.N))             # identity first
    assert all(tuple(G.perms[i]) < tuple(G.perms[i + 1]) for i in range(G.order - 1))
    bonds = {tuple(sorted(b)) for b in cl.bonds.tolist()}
    for p in G.perms:
        assert {tuple(sorted((p[i], p[j]))) for i, j in bonds} == bonds


def test_product_convention(ih):
    cl, G, _ = ih
    rng = np.random.default_rng(1)
    for _ in range(50):
        a, b = rng.integers(0, G.order, 2)
        # pi_{ab}(k) = pi_a(pi_b(k))
        assert np.array_equal(G.perms[G.mul[a, b]], G.perms[a][G.perms[b]])
        assert G.mul[a, G.inv[a]] == 0


def test_ih_classes_and_cycle_types():
    """I_h: 10 classes of sizes 1,1,12,12,12,12,15,15,20,20; cycle types on the polyhedra."""
    expect = {
        "icosahedron": {(1, (1,) * 12), (12, (1, 1, 5, 5)), (20, (3, 3, 3, 3)), (15, (2,) * 6),
                        (1, (2,) * 6), (12, (2, 10)), (20, (6, 6)), (15, (1, 1, 1, 1, 2, 2, 2, 2))},
        "dodecahedron": {(1, (1,) * 20), (12, (5,) * 4), (20, (1, 1) + (3,) * 6), (15, (2,) * 10),
                         (1, (2,) * 10), (12, (10, 10)), (20, (2, 6, 6, 6)), (15, (1,) * 4 + (2,) * 8)},
        "icosidodecahedron": {(1, (1,) * 30), (12, (5,) * 6), (20, (3,) * 10), (15, (1, 1) + (2,) * 14),
                              (1, (2,) * 15), (12, (10,) * 3), (20, (6,) * 5), (15, (1,) * 4 + (2,) * 13)},
    }
    for name, exp in expect.items():
        cl = clusters.get(name)
        G = group.close(cl.gens, cl.N)
        sizes = sorted(len(c) for c in G.classes)
        assert sizes == [1, 1, 12, 12, 12, 12, 15, 15, 20, 20]
        got = {(len(c), group.cycle_type(G.perms[c[0]])) for c in G.classes}
        assert got == exp, name


@pytest.mark.parametrize("name", ["icosahedron", "cuboctahedron", "square4", "ring6", "K4", "petersen"])
def test_irreps_invariants(name):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    assert len(irs) == len(G.classes)
    assert sum(ir.dim ** 2 for ir in irs) == G.order
    assert irreps.check_irreps(G, irs) < 1e-12
    # trivial irrep first
    assert irs[0].dim == 1 and np.allclose(irs[0].rho, 1.0)
    # column orthogonality of the character table
    X = np.array([ir.chars for ir in irs])          # (n_irreps, |G|)
    gram = X.conj().T @ X
    for a in range(0, G.order, 7):
        for b in range(0, G.order, 5):
            same = G.class_of[a] == G.class_of[b]
            csize = len(G.classes[G.class_of[a]])
            assert abs(gram[a, b] - (G.order / csize if same else 0.0)) < 1e-9


def test_ih_dims_sum_and_indicators(ih):
    _, G, irs = ih
    dims = [ir.dim for ir in irs]
    assert dims == [1, 1, 3, 3, 3, 3, 4, 4, 5, 5]
    assert sum(dims) == 32                     # Section 2.3: (32/120) D_M
    assert all(ir.indicator == 1 and ir.is_real for ir in irs)


def test_ih_rotation_character_table(ih):
    """Restricted to proper rotations, the 10 I_h irreps give the textbook table of I twice."""
    _, G, irs = ih
    cl = clusters.icosahedron()
    coords = cl.coords

    def kind(p):
        # classify by the geometric operation: det and rotation angle
        src = coords
        dst = coords[p]
        R, *_ = np.linalg.lstsq(src, dst, rcond=None)
        R = R.T
        det = np.linalg.det(R)
        Rp = R * det
        ang = np.degrees(np.arccos(np.clip((np.trace(Rp) - 1) / 2, -1, 1)))
        return int(round(det)), int(round(ang))

    tok = {"phi": PHI, "omphi": 1 - PHI}
    table = {r[0]: [float(tok.get(x, x)) for x in r[1:]] for r in golden("ih_rotation_characters.txt")}
    angles = [0, 72, 144, 120, 180]
    found = []
    for ir in irs:
        row = []
        for ang in angles:
            idx = [g for g in range(G.order) if kind(G.perms[g]) == (1, ang)]
            vals = ir.chars[idx].real
            assert np.ptp(vals) < 1e-9
            row.append(vals[0])
        found.append(row)
    for row in found:
        assert any(np.allclose(row, t, atol=1e-9) for t in table.values())
    for t in table.values():
        assert sum(np.allclose(row, t, atol=1e-9) for row in found) == 2    # g and u


def test_oh_dims():
    cl = clusters.cuboctahedron()
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    assert sorted(ir.dim for ir in irs) == [1, 1, 1, 1, 2, 2, 3, 3, 3, 3]
    assert all(ir.indicator == 1 for ir in irs)


def test_petersen_group_is_s5():
    """The Petersen graph's automorphism group is S5: irreps of dimension
    1, 1, 4, 4, 5, 5, 6 (the partitions of 5), all of real type, and the
    6-dimensional one has character 0 on transpositions (hook partition)."""
    cl = clusters.get("petersen")
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    assert [ir.dim for ir in irs] == [1, 1, 4, 4, 5, 5, 6]
    assert all(ir.indicator == 1 for ir in irs)
    # the transposition (0 1) is the first generator: chi_6 = 0 there
    t = next(i for i, p in enumerate(G.perms) if np.array_equal(p, cl.gens[0]))
    assert abs(irs[6].chars[t]) < 1e-12


def test_square_lattice_group_5x8_has_28_irreps():
    """Section 4.3: the 5x8 lattice space group (C2v with translations), order 160, 28 irreps."""
    G = group.close(_square5x8_gens(), 40)
    irs = irreps.compute_irreps(G)
    assert G.order == 160
    assert len(irs) == 28
    assert sum(ir.dim ** 2 for ir in irs) == 160


def _square5x8_gens():
    Lx, Ly = 5, 8

    def idx(x, y):
        return (x % Lx) * Ly + (y % Ly)

    def perm(f):
        p = np.empty(Lx * Ly, dtype=np.int64)
        for x in range(Lx):
            for y in range(Ly):
                p[idx(x, y)] = idx(*f(x, y))
        return p

    return np.stack([perm(lambda x, y: (x + 1, y)), perm(lambda x, y: (x, y + 1)),
                     perm(lambda x, y: (-x, y)), perm(lambda x, y: (x, -y))])


def test_bad_generator_rejected():
    with pytest.raises(ValueError):
        group.close(np.array([[0, 0, 1]]), 3)
