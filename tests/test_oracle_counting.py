"""Oracle pins: sector and block dimensions (Section 2.1, Eq. 13, Tables 1-2)."""
from math import comb

import numpy as np
import pytest

from conftest import golden
from oracle import basis, counting, group, irreps
from synth import clusters


def test_table1_sector_dims():
    for name, N, two_s, dfull, d0 in golden("table1_sector_dims.txt"):
        N, two_s = int(N), int(two_s)
        assert (two_s + 1) ** N == int(dfull), name
        assert counting.sector_dim(N, two_s, 0) == int(d0), name


def test_sector_dim_closed_forms():
    for N in range(1, 31):
        for k in range(N + 1):
            assert counting.sector_dim(N, 1, 2 * k - N) == comb(N, k)
    # spin 1, N = 3: coefficient of x^3 in (1+x+x^2)^3 = 7
    assert counting.sector_dim(3, 2, 0) == 7
    # sum over all M equals the full Hilbert space
    for N, two_s in [(12, 3), (7, 2), (20, 3)]:
        tot = sum(counting.sector_dim(N, two_s, tm) for tm in range(-N * two_s, N * two_s + 1, 2))
        assert tot == (two_s + 1) ** N


def test_enumeration_matches_count():
    from oracle import sector
    for N, two_s, two_M in [(12, 1, 0), (12, 1, 4), (8, 3, 2), (7, 2, 1 * 0), (6, 6, 2)]:
        labs = sector.enumerate_sector(N, two_s, two_M)
        assert len(labs) == counting.sector_dim(N, two_s, two_M)
        dig = sector.digits(labs, N, two_s + 1)
        assert np.all(dig.sum(axis=1) * 2 - N * two_s == two_M)
        assert np.all(np.diff(labs) > 0)


@pytest.fixture(scope="module")
def dodeca():
    cl = clusters.dodecahedron()
    G = group.close(cl.gens, cl.N)
    return cl, G, irreps.compute_irreps(G)


def test_table2_block_dims(dodeca):
    """The character formula reproduces every printed Table 2 dimension (s=3/2, M=0)."""
    cl, G, irs = dodeca
    dims = counting.block_dims_by_characters(G, irs, 3, 0)
    # the third generator is the geometric inversion x -> -x
    inv = int(np.nonzero((G.perms == cl.gens[2]).all(axis=1))[0][0])
    rows = golden("table2_dodeca_s32_blocks.txt")
    got = sorted((ir.dim, int(round(ir.chars[inv].real / ir.dim)), D) for ir, D in zip(irs, dims))
    want = sorted((int(d), int(p), int(D)) for _, d, D, p in rows)
    assert got == want
    assert sum(ir.dim * D for ir, D in zip(irs, dims)) == counting.sector_dim(20, 3, 0)
    # Section 2.3: total iterated dimension ~ (32/120) D_M
    assert abs(sum(dims) / counting.sector_dim(20, 3, 0) - 0.27) < 0.005


def test_enumerated_block_dims_equal_character_formula(dodeca):
    """n_Gamma from stabilizers (enumeration) vs the character formula: two independent routes."""
    cl, G, irs = dodeca
    for two_M in (0, 6, 14):
        sec = basis.sector_reps(G, cl.N, 1, two_M)
        by_chars = counting.block_dims_by_characters(G, irs, 1, two_M)
        by_enum = [basis.build_block(G, ir, sec, with_psi=False).D for ir in irs]
        assert by_enum == by_chars
        assert sum(ir.dim * D for ir, D in zip(irs, by_enum)) == len(sec.labels)
    # orbit count = A_g block dimension (Burnside)
    sec0 = basis.sector_reps(G, cl.N, 1, 0)
    assert len(sec0.reps) == 1648


def test_square5x8_largest_parity_block():
    """Section 4.3: a spin-flip-resolved M=0 block of the 5x8 lattice with d=4 has 1,723,070,831 rows.

    Under G x Z2 the block dimension of Gamma^{+/-} is
    (1/(2|G|)) sum_g chi(g)^* [F(g) +/- F(g*flip)], F(g*flip) counting M=0 states
    with a_{pi(k)} = 1 - a_k (even cycles only, two choices each).  The printed
    number is one parity half of the largest d=4 irrep (the paper does not say
    which sign convention labels it); both halves must add up to the G-only block.
    """
    from test_oracle_group import _square5x8_gens
    G = group.close(_square5x8_gens(), 40)
    irs = irreps.compute_irreps(G)
    F = np.array([counting.fixed_count(p, 1, 0) for p in G.perms], dtype=np.float64)
    Ff = np.array([0 if any(L % 2 for L in group.cycle_type(p)) else 2 ** len(group.cycle_type(p))
                   for p in G.perms], dtype=np.float64)
    halves = {}
    for i, ir in enumerate(irs):
        Dg = int(round(np.sum(np.conj(ir.chars) * F).real / G.order))
        hp = int(round(np.sum(np.conj(ir.chars) * (F + Ff)).real / (2 * G.order)))
        hm = int(round(np.sum(np.conj(ir.chars) * (F - Ff)).real / (2 * G.order)))
        assert hp + hm == Dg
        halves[i] = (ir.dim, Dg, hp, hm)
    top = max(halves.values(), key=lambda t: t[1])
    assert top[0] == 4 and 1723070831 in top[2:]


def test_icosidodecahedron_m0_dims():
    cl = clusters.icosidodecahedron()
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    dims = counting.block_dims_by_characters(G, irs, 1, 0)
    assert max(dims) == 6465762 and min(dims) == 1291834
    assert dims[0] == 1295266
    assert sum(ir.dim * D for ir, D in zip(irs, dims)) == comb(30, 15)
    assert sum(dims) == 41364764
