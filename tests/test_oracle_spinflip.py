"""Oracle pins for the spin-flip resolution of M = 0 (G x Z2).

What fixes it independently of the oracle's own code:
* the dimer closed form: the m = 0 triplet is even under both the site swap
  and the flip (E = +1/4), the singlet odd under both (E = -3/4);
* F commutes with H_0 and with every generator (plain matrix identities);
* the Gamma^+ and Gamma^- blocks split the Gamma block: their spectra, pooled,
  are the Gamma block's spectrum, and their dimensions add up;
* the dimensions from enumeration equal the character formula over G x Z2,
  including an integer spin (odd cycles of U(g)F fix the middle digit);
* the irreps of G x Z2 pass the homomorphism and great-orthogonality checks.
"""
import numpy as np
import pytest

from oracle import basis, counting, group, hv, irreps, sector, spinflip
from synth import clusters


def _setup(name):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    return cl, G, irs, spinflip.FlipGroup(G), spinflip.flip_irreps(irs)


def test_dimer_closed_form():
    cl, G, irs, G2, irs2 = _setup("dimer")
    sec = basis.sector_reps(G2, 2, 1, 0)
    H = sector.hamiltonian(sec.labels, 2, 1, cl.bonds, cl.J)
    spec = []
    for gi, ir in enumerate(irs2):
        B = basis.build_block(G2, ir, sec)
        spec.append(np.linalg.eigvalsh(hv.block_matrix(B, H)) if B.D else np.zeros(0))
    # order: A1+, A1-, A2+, A2- (A1 symmetric, A2 antisymmetric under the swap)
    assert [len(x) for x in spec] == [1, 0, 0, 1]
    assert abs(spec[0][0] - 0.25) < 1e-14 and abs(spec[3][0] + 0.75) < 1e-14


@pytest.mark.parametrize("name,two_s", [("icosahedron", 1), ("ring6", 1), ("ring6", 2), ("square4", 1),
                                        ("cuboctahedron", 1), ("K4", 3)])
def test_flip_commutes_and_blocks_split(name, two_s):
    cl, G, irs, G2, irs2 = _setup(name)
    d = two_s + 1
    sec = basis.sector_reps(G, cl.N, two_s, 0)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J).toarray()
    fl = np.searchsorted(sec.labels, spinflip.flip_labels(sec.labels, cl.N, d))
    assert np.array_equal(sec.labels[fl], spinflip.flip_labels(sec.labels, cl.N, d))   # F maps M=0 onto itself
    Pf = np.eye(len(fl))[fl]
    assert np.allclose(Pf @ H, H @ Pf, atol=1e-13)
    sec2 = basis.sector_reps(G2, cl.N, two_s, 0)
    dims2 = counting.block_dims_by_characters(G2, irs2, two_s, 0)
    dims1 = counting.block_dims_by_characters(G, irs, two_s, 0)
    for gi, ir in enumerate(irs):
        B = basis.build_block(G, ir, sec)
        spec = np.linalg.eigvalsh(hv.block_matrix(B, H)) if B.D else np.zeros(0)
        parts = []
        for q in (0, 1):
            B2 = basis.build_block(G2, irs2[2 * gi + q], sec2)
            assert B2.D == dims2[2 * gi + q]
            if B2.D:
                M = hv.block_matrix(B2, H)
                assert np.allclose(M, M.T, atol=1e-12)
                parts.append(np.linalg.eigvalsh(M))
        assert dims2[2 * gi] + dims2[2 * gi + 1] == dims1[gi] == B.D
        pooled = np.sort(np.concatenate(parts)) if parts else np.zeros(0)
        assert len(pooled) == len(spec)
        assert np.max(np.abs(pooled - spec), initial=0.0) < 1e-11 * max(1.0, np.max(np.abs(spec), initial=1.0))


def test_flip_irreps_are_irreps():
    cl, G, irs, G2, irs2 = _setup("cuboctahedron")
    assert sum(ir.dim ** 2 for ir in irs2) == G2.order
    assert irreps.check_irreps(G2, irs2) < 1e-10


def test_flip_group_orbit_search_matches_brute_force():
    cl, G, irs, G2, irs2 = _setup("icosahedron")
    sec2 = basis.sector_reps(G2, cl.N, 1, 0)
    for a in sec2.labels[::37]:
        orbit = [int(x) for x in basis.apply_all(G, np.array([a]), cl.N, 2)[0]]
        orbit += [int(x) for x in spinflip.flip_labels(np.array(orbit), cl.N, 2)]
        r, h = basis.canonicalize(G2, np.array([a]), cl.N, 2)
        assert r[0] == min(orbit)
        assert basis.apply_all(G2, np.array([a]), cl.N, 2)[0][h[0]] == r[0]
