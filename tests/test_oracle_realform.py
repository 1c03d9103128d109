"""Pins of the real forms of complex- and quaternionic-type irreps (oracle/realform.py).

Checked against what the mathematics fixes, independently of the module:

* every real form is an orthogonal homomorphism; its rows satisfy the
  orthogonality the block construction uses; a realified pair has character
  2 Re chi, indicator 0 and a two-dimensional real commutant (irreducible over
  the reals, not absolutely irreducible); a realified quaternionic irrep has
  character 2 chi, indicator -2 and a four-dimensional commutant; a real-type
  irrep has a one-dimensional commutant;
* for the cyclic group C_N the real forms are the closed-form rotations by
  2 pi k m / N (characters 2 cos), plus the trivial and (N even) sign irreps;
* completeness: sum over real forms of weight x dim = |G|;
* the block of a realified pair or quaternionic irrep has, by exact
  diagonalization, the spectrum of the complex-arithmetic block of Gamma
  (built from the complex irrep) with every eigenvalue twice, and twice its
  dimension; a quaternionic Gamma block has its levels in pairs;
* the union over real forms of weight copies of each block spectrum is the
  spectrum of the whole sector (full exact diagonalization of the sector),
  and the block dimensions equal the character formula.
"""
import numpy as np
import pytest

from oracle import basis, counting, group, irreps, realform, sector
from synth import clusters

GROUPS = ["ring5_C", "ring8_C", "square3x3_T", "ring6", "icosahedron", "dic2", "dic3", "dic5"]


def _group(name):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    return cl, G, irreps.compute_irreps(G)


@pytest.mark.parametrize("name", GROUPS)
def test_real_forms_are_real_orthogonal_representations(name):
    cl, G, irs = _group(name)
    n = G.order
    forms = realform.real_forms(G, irs)
    assert sum(f.weight * f.irrep.dim for f in forms) == n
    for f in forms:
        rho = f.irrep.rho
        dim = f.irrep.dim
        assert not np.iscomplexobj(rho)
        assert np.allclose(np.einsum("gji,gjk->gik", rho, rho), np.eye(dim), atol=1e-12)
        assert np.allclose(np.einsum("gij,hjk->ghik", rho, rho), rho[G.mul], atol=1e-12)
        # (dim/|G|) sum_g rho[a, m] rho[a, m'] = delta(m, m') for every row a
        for a in range(dim):
            M = rho[:, a, :].T @ rho[:, a, :] * dim / n
            assert np.allclose(M, np.eye(dim), atol=1e-12)
        chi = np.trace(rho, axis1=1, axis2=2)
        nu = chi[G.mul[np.arange(n), np.arange(n)]].sum() / n
        # real commutant: X with rho(g) X = X rho(g) for all g
        A = np.concatenate([np.kron(rho[g], np.eye(dim)) - np.kron(np.eye(dim), rho[g].T) for g in range(n)])
        null = dim * dim - np.linalg.matrix_rank(A, tol=1e-9)
        if f.kind == "complex pair":
            assert f.weight * 2 == dim and abs(nu) < 1e-9 and null == 2
            assert abs(np.dot(chi, chi) / n - 2.0) < 1e-9
        elif f.kind == "quaternionic":
            assert f.weight * 4 == dim and abs(nu + 2) < 1e-9 and null == 4
            assert abs(np.dot(chi, chi) / n - 4.0) < 1e-9
        else:
            assert f.weight == dim and abs(nu - 1) < 1e-9 and null == 1


@pytest.mark.parametrize("N", [5, 6, 8])
def test_cyclic_real_forms_closed_form(N):
    cl, G, irs = _group(f"ring{N}_C")
    forms = realform.real_forms(G, irs)
    m = G.perms[:, 0]                       # element c^m sends site 0 to site m
    want = [np.ones(N)] + ([np.cos(np.pi * m)] if N % 2 == 0 else [])
    want += [2 * np.cos(2 * np.pi * k * m / N) for k in range(1, (N - 1) // 2 + 1)]
    got = [f.irrep.chars.real for f in forms]
    assert len(got) == len(want)
    for w in want:
        assert sum(np.allclose(g, w, atol=1e-12) for g in got) == 1
    assert sum(f.kind == "complex pair" for f in forms) == (N - 1) // 2


CASES = [("ring8_C", 1, 0), ("ring8_C", 1, 2), ("square3x3_T", 1, 1), ("ring6_C", 2, 0), ("ring5_C", 3, 1),
         ("dic2", 2, 0), ("dic2", 1, 2), ("dic3", 1, 0), ("dic3", 1, 2)]


def _hblock(Bk, H):
    P = Bk.Psi
    return (P.conj().T @ H @ P).toarray()


@pytest.mark.parametrize("name,two_s,two_M", CASES)
def test_realified_block_is_doubled_complex_block(name, two_s, two_M):
    cl, G, irs = _group(name)
    sec = basis.sector_reps(G, cl.N, two_s, two_M)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    pairs = 0
    for ir in irs:
        if ir.indicator not in (0, -1):
            continue
        BR = basis.build_block(G, realform.realify(ir), sec)
        BC = basis.build_block(G, ir, sec)
        assert BR.D == 2 * BC.D
        if BC.D == 0:
            continue
        pairs += 1
        P = BR.Psi.toarray()
        assert np.allclose(P.T @ P, np.eye(BR.D), atol=1e-12)
        eR = np.linalg.eigvalsh(_hblock(BR, H))
        eC = np.linalg.eigvalsh(_hblock(BC, H))
        assert np.allclose(eR, np.sort(np.concatenate([eC, eC])), atol=1e-10)
        if ir.indicator == -1:
            assert np.allclose(eC[0::2], eC[1::2], atol=1e-10)
    assert pairs > 0


@pytest.mark.parametrize("name,two_s,two_M", CASES)
def test_weighted_real_form_spectra_make_the_sector_spectrum(name, two_s, two_M):
    cl, G, irs = _group(name)
    sec = basis.sector_reps(G, cl.N, two_s, two_M)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    full = np.linalg.eigvalsh(H.toarray())
    forms = realform.real_forms(G, irs)
    parts = []
    dims = counting.block_dims_by_characters(G, [f.irrep for f in forms], two_s, two_M)
    for f, dchar in zip(forms, dims):
        B = basis.build_block(G, f.irrep, sec)
        assert B.D == dchar
        if B.D:
            e = np.linalg.eigvalsh(_hblock(B, H))
            parts += [e] * f.weight
    assert sum(len(p) for p in parts) == len(full)
    assert np.allclose(np.sort(np.concatenate(parts)), full, atol=1e-10)


def test_real_type_groups_are_unchanged():
    cl, G, irs = _group("icosahedron")
    forms = realform.real_forms(G, irs)
    assert [f.irrep.dim for f in forms] == [ir.dim for ir in irs]
    assert all(f.kind == "real" and f.irrep is ir for f, ir in zip(forms, irs))
