"""Oracle pins: symmetry-adapted basis and H action (Sections 2.3-2.4, Eq. 12, Section 4.1)."""
import numpy as np
import pytest

from oracle import basis, counting, group, hv, irreps, sector
from synth import clusters


def _setup(name, two_s=1):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    return cl, G, irreps.compute_irreps(G)


def _block_spectra(cl, G, irs, two_s, two_M, alpha=0):
    sec = basis.sector_reps(G, cl.N, two_s, two_M)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    spec = {}
    for gi, ir in enumerate(irs):
        B = basis.build_block(G, ir, sec, alpha=min(alpha, ir.dim - 1))
        spec[gi] = np.linalg.eigvalsh(hv.block_matrix(B, H)) if B.D else np.zeros(0)
    return sec, H, spec


@pytest.mark.parametrize("name,two_s", [("icosahedron", 1), ("cuboctahedron", 1), ("ring6", 1),
                                        ("ring6", 2), ("ring5", 1), ("square4", 1), ("K4", 3),
                                        ("petersen", 1), ("petersen", 2)])
def test_union_of_block_spectra_is_sector_spectrum(name, two_s):
    """Section 4.1: every block against the dense reference of the full M sector."""
    cl, G, irs = _setup(name)
    Mmax = cl.N * two_s
    twoMs = range(Mmax % 2, Mmax + 1, 2)
    if name == "square4":
        twoMs = [8, 10, 12]          # keep the dense reference small
    for two_M in twoMs:
        sec, H, spec = _block_spectra(cl, G, irs, two_s, two_M)
        full = np.linalg.eigvalsh(H.toarray())
        union = np.sort(np.concatenate([np.repeat(spec[g], irs[g].dim) for g in spec]))
        assert len(union) == len(full)
        assert np.max(np.abs(union - full)) < 1e-11 * max(1.0, np.max(np.abs(full)))


def test_psi_orthonormal_and_rows_identical():
    """Eq. (12) columns are orthonormal; the block is the same matrix for every partner row."""
    cl, G, irs = _setup("icosahedron")
    for two_M in (0, 2):
        sec = basis.sector_reps(G, cl.N, 1, two_M)
        H = sector.hamiltonian(sec.labels, cl.N, 1, cl.bonds, cl.J)
        for ir in irs:
            mats = []
            for a in range(ir.dim):
                B = basis.build_block(G, ir, sec, alpha=a)
                if B.D == 0:
                    continue
                P = B.Psi
                assert np.abs((P.conj().T @ P).toarray() - np.eye(B.D)).max() < 1e-13
                mats.append(hv.block_matrix(B, H))
            for m in mats[1:]:
                assert np.abs(m - mats[0]).max() < 1e-13
        # distinct irreps / rows are mutually orthogonal subspaces
        cols = [basis.build_block(G, ir, sec, alpha=a).Psi for ir in irs for a in range(ir.dim)]
        allpsi = np.hstack([c.toarray() for c in cols])
        assert allpsi.shape[1] == len(sec.labels)
        assert np.abs(allpsi.T @ allpsi - np.eye(allpsi.shape[1])).max() < 1e-12


def test_hamiltonian_commutes_with_generators():
    for name, two_s in [("icosahedron", 1), ("dodecahedron", 1), ("cuboctahedron", 3), ("square4", 1)]:
        cl = clusters.get(name)
        two_M = (cl.N * two_s) % 2 + (8 if name == "dodecahedron" else 2)
        labs = sector.enumerate_sector(cl.N, two_s, two_M)
        H = sector.hamiltonian(labs, cl.N, two_s, cl.bonds, cl.J)
        for gen in cl.gens:
            img = sector.permute_labels(labs, gen, cl.N, two_s + 1)
            pos = np.searchsorted(labs, img)
            assert np.array_equal(labs[pos], img)
            import scipy.sparse as sp
            U = sp.csr_matrix((np.ones(len(labs)), (pos, np.arange(len(labs)))), shape=H.shape)
            assert abs(H @ U - U @ H).max() < 1e-13


def _all_levels(cl, two_s):
    out = []
    for two_M in range(-cl.N * two_s, cl.N * two_s + 1, 2):
        labs = sector.enumerate_sector(cl.N, two_s, two_M)
        if len(labs):
            out += list(np.linalg.eigvalsh(sector.hamiltonian(labs, cl.N, two_s, cl.bonds, cl.J).toarray()))
    return np.sort(out)


def _multiplet_levels(S_values, energy, degeneracy_of):
    lv = []
    for S, m in S_values:
        lv += [energy(S)] * ((2 * S + 1) * m)
    return np.sort(lv)


def test_closed_forms():
    """Dimer, 4-ring and complete graphs: H = (J/2)[S_tot^2 - sum of fixed spins^2]."""
    # dimer, spins s: E_S = (J/2)[S(S+1) - 2 s(s+1)], S = 0..2s
    for two_s in (1, 2, 3):
        s = two_s / 2
        want = []
        for S2 in range(0, 2 * two_s + 1, 2):
            S = S2 / 2
            want += [0.5 * (S * (S + 1) - 2 * s * (s + 1))] * int(2 * S + 1)
        got = _all_levels(clusters.dimer(), two_s)
        assert np.allclose(got, np.sort(want), atol=1e-12)
    # 4-ring s=1/2: -2 (x1), -1 (x3), 0 (x7), +1 (x5)
    got = _all_levels(clusters.ring(4), 1)
    want = np.sort([-2.0] + [-1.0] * 3 + [0.0] * 7 + [1.0] * 5)
    assert np.allclose(got, want, atol=1e-12)
    # K3 s=1/2: S=1/2 (x2 multiplets) at -3/4, S=3/2 at +3/4
    got = _all_levels(clusters.complete_graph(3), 1)
    want = np.sort([-0.75] * 4 + [0.75] * 4)
    assert np.allclose(got, want, atol=1e-12)
    # K4 s=1/2: S=0 (x2) at -3/2, S=1 (x3) at -1/2, S=2 (x1) at +3/2
    got = _all_levels(clusters.complete_graph(4), 1)
    want = np.sort([-1.5] * 2 + [-0.5] * 9 + [1.5] * 5)
    assert np.allclose(got, want, atol=1e-12)


def test_closed_forms_through_blocks():
    """The same closed forms reached through the symmetry-adapted blocks."""
    cl, G, irs = _setup("ring4")
    allv = []
    for two_M in (0, 2, 4):
        _, _, spec = _block_spectra(cl, G, irs, 1, two_M)
        mult = 1 if two_M == 0 else 2
        for g, ev in spec.items():
            allv += list(np.repeat(ev, irs[g].dim * mult))
    want = np.sort([-2.0] + [-1.0] * 3 + [0.0] * 7 + [1.0] * 5)
    assert np.allclose(np.sort(allv), want, atol=1e-12)


def test_multiplets_nest_across_M():
    """A level of spin S appears in every |M| <= S: spec(M+1, Gamma) is contained in spec(M, Gamma)."""
    cl, G, irs = _setup("icosahedron")
    prev = None
    for two_M in range(12, -1, -2):
        _, _, spec = _block_spectra(cl, G, irs, 1, two_M)
        if prev is not None:
            for g in spec:
                big, small = spec[g], prev[g]
                assert len(big) >= len(small)
                for e in small:
                    assert np.min(np.abs(big - e)) < 1e-10
        prev = spec


def test_sampled_rows_match_explicit_apply():
    cl, G, irs = _setup("dodecahedron")
    sec = basis.sector_reps(G, cl.N, 1, 4)
    H = sector.hamiltonian(sec.labels, cl.N, 1, cl.bonds, cl.J)
    rng = np.random.default_rng(3)
    for gi in (0, 3, 8):
        ir = irs[gi]
        B = basis.build_block(G, ir, sec)
        X = rng.standard_normal((B.D, 2))
        Y = hv.apply(B, H, X)
        rep_pos = {int(r): i for i, r in enumerate(sec.reps)}

        def xfun(r, n):
            i = rep_pos[r]
            return X[B.offsets[i]:B.offsets[i] + n]

        pick = [i for i in rng.choice(len(sec.reps), 12, replace=False) if B.n_rep[i] > 0]
        rows = hv.sampled_rows(G, ir, 0, cl.N, 1, cl.bonds, cl.J, sec.reps[pick], xfun, 2)
        for i, y in zip(pick, rows):
            assert np.abs(y - Y[B.offsets[i]:B.offsets[i] + B.n_rep[i]]).max() < 1e-12


def test_free_orbit_counts():
    """Orbits of full length carry n_Gamma = d_Gamma (Section 2.3)."""
    cl, G, irs = _setup("dodecahedron")
    sec = basis.sector_reps(G, cl.N, 1, 0)
    free = [i for i, s in enumerate(sec.stab_sets) if len(s) == 1]
    assert free
    for ir in irs:
        B = basis.build_block(G, ir, sec, with_psi=False)
        for i in free:
            assert B.n_stab[i] == ir.dim
            assert np.allclose(B.V_stab[i], np.eye(ir.dim))


def _image_loop(label, perm, N, d, flip):
    """Label of U(g) F^f |a> by loops over sites: digit k moves to site perm[k]."""
    dig = []
    x = int(label)
    for _ in range(N):
        x, r = divmod(x, d)
        dig.append(r)
    if flip:
        dig = [d - 1 - a for a in dig]
    new = [0] * N
    for k in range(N):
        new[perm[k]] = dig[k]
    return sum(a * d ** k for k, a in enumerate(new))


@pytest.mark.parametrize("name,two_s,flip", [("icosahedron", 1, False), ("cuboctahedron", 2, False),
                                             ("icosahedron", 1, True), ("ring6", 3, False)])
def test_connecting_element_is_smallest_minimiser(name, two_s, flip):
    """The connecting element h of a label a is the smallest group index among
    all g with U(g) a = min O(a) (the reading of the choice the paper leaves
    free, Section 2.4): every g applied by loops over sites, the minimisers
    collected, and their count equal to the stabilizer order of the
    representative.  Labels with non-trivial stabilizers, where several
    minimisers tie, are sampled on purpose."""
    from oracle import spinflip
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    GG = spinflip.FlipGroup(G) if flip else G
    d = two_s + 1
    rng = np.random.default_rng(5)
    ties = 0
    twoMs = [0] if flip else range((cl.N * two_s) % 2, cl.N * two_s + 1, 2)
    for two_M in twoMs:
        labels = sector.enumerate_sector(cl.N, two_s, two_M)
        sec = basis.sector_reps(GG, cl.N, two_s, two_M)
        # representatives with non-trivial stabilizers and a few members of their orbits
        big = [int(r) for r, s in zip(sec.reps, sec.stab_id) if len(sec.stab_sets[s]) > 1]
        picks = set(rng.choice(labels, size=min(len(labels), 12), replace=False).tolist())
        for r in big[:6]:
            orbit = basis.apply_all(GG, np.array([r]), cl.N, d)[0]
            picks.update(int(x) for x in rng.choice(orbit, size=3))
        picks = sorted(picks)
        rep, h = basis.canonicalize(GG, np.array(picks, dtype=np.int64), cl.N, d)
        for a, r0, h0 in zip(picks, rep, h):
            imgs = [_image_loop(a, G.perms[g % G.order], cl.N, d, g >= G.order) for g in range(GG.order)]
            m = min(imgs)
            mins = [g for g, x in enumerate(imgs) if x == m]
            assert r0 == m and h0 == mins[0], (a, r0, h0, mins[:4])
            ridx = int(np.searchsorted(sec.reps, m))
            assert len(mins) == len(sec.stab_sets[sec.stab_id[ridx]])
            ties += len(mins) > 1
    assert ties >= 5
