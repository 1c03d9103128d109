"""Oracle pins: FTLM stage (Section 2.2, Eqs. 4-7 and 14; Section 4.1 high-T checks)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, ftlm, group, hv, irreps, sector
from synth import clusters


def test_splitmix64_published_values():
    """SplitMix64 seeded with 1234567: the published first five outputs."""
    assert ftlm.splitmix64_stream(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    # the vectorised stream agrees with the scalar definition
    key = ftlm.chain_key(7, 2, 3, 1, 5)
    assert [int(x) for x in ftlm._stream_np(key, 4)] == ftlm.splitmix64_stream(key, 4)


def test_start_vectors():
    v = ftlm.start_vector(1000, 11, 0, 2, 0, 3, "rademacher")
    assert np.allclose(np.abs(v), 1 / np.sqrt(1000))
    assert abs(np.linalg.norm(v) - 1) < 1e-15
    g = ftlm.start_vector(200000, 11, 0, 2, 0, 3, "gaussian") * np.sqrt(200000)
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1) < 0.01
    # different chains differ, same key repeats
    a = ftlm.start_vector(64, 1, 0, 0, 0, 0)
    b = ftlm.start_vector(64, 1, 0, 0, 0, 1)
    assert not np.array_equal(a, b)
    assert np.array_equal(a, ftlm.start_vector(64, 1, 0, 0, 0, 0))


@pytest.fixture(scope="module")
def ico():
    cl = clusters.icosahedron()
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    secs, Hs = {}, {}
    for two_M in range(0, 13, 2):
        secs[two_M] = basis.sector_reps(G, cl.N, 1, two_M)
        Hs[two_M] = sector.hamiltonian(secs[two_M].labels, cl.N, 1, cl.bonds, cl.J)
    return cl, G, irs, secs, Hs


def test_krylov_exhaustion_equals_exact_trace_element(ico):
    """With n = Krylov dimension, sum_k w_k e^{-b theta_k} = <r|e^{-bH}|r> (Eq. 4 element)."""
    cl, G, irs, secs, Hs = ico
    for gi in (0, 8, 9):
        B = basis.build_block(G, irs[gi], secs[0])
        Hb = hv.block_matrix(B, Hs[0])
        r = ftlm.start_vector(B.D, 5, 0, gi, 0, 0, "gaussian")
        a, b = ftlm.lanczos(lambda x: Hb @ x, r, 100)
        th, w = ftlm.ritz(a, b)
        assert abs(w.sum() - 1) < 1e-13
        ev, U = np.linalg.eigh(Hb)
        assert th.min() >= ev.min() - 1e-10 and th.max() <= ev.max() + 1e-10
        for beta in (0.1, 1.0, 5.0):
            exact = r @ (U @ (np.exp(-beta * ev) * (U.T @ r)))
            approx = np.sum(w * np.exp(-beta * th))
            assert abs(approx - exact) < 1e-10 * exact


def test_breakdown_stops_early():
    # start vector inside a 2-dimensional invariant subspace of a diagonal matrix
    d = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    v = np.array([1.0, 1.0, 0.0, 0.0, 0.0]) / np.sqrt(2)
    a, b = ftlm.lanczos(lambda x: d * x, v, 5)
    assert len(a) == 2
    th, w = ftlm.ritz(a, b)
    assert np.allclose(th, [1, 2]) and np.allclose(w, [0.5, 0.5])


def _ftlm_blocks(ico, R, steps, seed=1, dist="rademacher"):
    cl, G, irs, secs, Hs = ico
    blocks = []
    for two_M, sec in secs.items():
        for gi, ir in enumerate(irs):
            B = basis.build_block(G, ir, sec)
            if B.D == 0:
                continue
            Hb = hv.block_matrix(B, Hs[two_M])
            ths, ws = [], []
            for c in range(R):
                r = ftlm.start_vector(B.D, seed, two_M, gi, 0, c, dist)
                th, w = ftlm.ritz(*ftlm.lanczos(lambda x: Hb @ x, r, steps))
                ths.append(th)
                ws.append(w)
            blocks.append(ftlm.BlockRitz(two_M, ir.dim, B.D, ths, ws))
    return blocks


def test_high_temperature_limits(ico):
    """Z(T->inf) = (2s+1)^N; T chi / g^2 -> N s(s+1)/3 (Section 4.1); E/C sane."""
    blocks = _ftlm_blocks(ico, R=2, steps=30)
    T = np.array([1e8, 1e10])
    E, C, chi, lnZ = ftlm.observables(blocks, T, g=2.0, with_logZ=True)
    assert np.allclose(np.exp(lnZ), 2.0 ** 12, rtol=1e-7)
    assert np.allclose(T * chi / 4.0, 12 * 0.5 * 1.5 / 3, rtol=1e-7)


def test_ftlm_vs_full_ed(ico):
    """Icosahedron s=1/2: FTLM with R=32 (all blocks small) against full ED thermodynamics.

    Statistical check (trace-estimator error ~ 1/sqrt(R D)); the seed is fixed.
    """
    cl, G, irs, secs, Hs = ico
    blocks = _ftlm_blocks(ico, R=32, steps=60, seed=3, dist="gaussian")
    spectra = {m: np.linalg.eigvalsh(Hs[m].toarray()) for m in secs}
    T = np.geomspace(0.05, 10, 50)
    E, C, chi = ftlm.observables(blocks, T)
    Ee, Ce, chie = ftlm.ed_observables(spectra, T)
    # ground state exact (every block's Krylov space reaches its lowest level)
    assert abs(min(th.min() for b in blocks for th in b.thetas) - min(s.min() for s in spectra.values())) < 1e-10
    hot = T >= 0.5
    assert np.max(np.abs(E - Ee)[hot] / np.abs(Ee[hot]).max()) < 0.01
    assert np.max(np.abs(C - Ce)[hot]) / Ce.max() < 0.02
    assert np.max(np.abs(chi - chie)[hot]) / chie.max() < 0.08


def test_dimer_ftlm_exact():
    """Dimer: FTLM equals the closed form when the start vectors span each block.

    For s=1/2 every (M, Gamma) block is one-dimensional, so any single start
    vector gives the exact trace; for s=3/2 the blocks have dimension <= 2 and
    the R = D unit vectors are used as start vectors (Eq. 4 is then exact).
    """
    cl = clusters.dimer()
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    for two_s in (1, 3):
        blocks, spectra = [], {}
        for two_M in range(two_s * 2 % 2, 2 * two_s + 1, 2):
            sec = basis.sector_reps(G, 2, two_s, two_M)
            H = sector.hamiltonian(sec.labels, 2, two_s, cl.bonds, cl.J)
            spectra[two_M] = np.linalg.eigvalsh(H.toarray())
            for gi, ir in enumerate(irs):
                B = basis.build_block(G, ir, sec)
                if B.D == 0:
                    continue
                Hb = hv.block_matrix(B, H)
                if two_s == 1:
                    assert B.D == 1
                    starts = [ftlm.start_vector(1, 9, two_M, gi, 0, 0)]
                else:
                    starts = list(np.eye(B.D))
                ths, ws = zip(*[ftlm.ritz(*ftlm.lanczos(lambda x: Hb @ x, r, 5)) for r in starts])
                blocks.append(ftlm.BlockRitz(two_M, ir.dim, B.D, list(ths), list(ws)))
        T = np.geomspace(0.05, 10, 20)
        got = ftlm.observables(blocks, T)
        s = two_s / 2
        levels = []
        for S2 in range(0, 2 * two_s + 1, 2):
            S = S2 / 2
            levels.append((0.5 * (S * (S + 1) - 2 * s * (s + 1)), S))
        beta = 1 / T
        E0 = min(e for e, _ in levels)
        Z = sum((2 * S + 1) * np.exp(-beta * (e - E0)) for e, S in levels)
        E = sum((2 * S + 1) * e * np.exp(-beta * (e - E0)) for e, S in levels) / Z
        E2 = sum((2 * S + 1) * e * e * np.exp(-beta * (e - E0)) for e, S in levels) / Z
        SzSz = sum(S * (S + 1) * (2 * S + 1) / 3 * np.exp(-beta * (e - E0)) for e, S in levels) / Z
        assert np.allclose(got[0], E, rtol=1e-12, atol=1e-12)
        assert np.allclose(got[1], beta ** 2 * (E2 - E ** 2), rtol=1e-9, atol=1e-12)
        assert np.allclose(got[2], beta * SzSz, rtol=1e-12)


def test_ed_observables_high_T_expansion():
    """C ~ N_B (s(s+1))^2 / (3 T^2) at high T for the Heisenberg model."""
    cl = clusters.icosahedron()
    spectra = {m: np.linalg.eigvalsh(sector.hamiltonian(sector.enumerate_sector(12, 1, m), 12, 1, cl.bonds, cl.J).toarray())
               for m in range(0, 13, 2)}
    T = np.array([200.0])
    _, C, _ = ftlm.ed_observables(spectra, T)
    assert abs(C[0] * T[0] ** 2 / (30 * 0.75 ** 2 / 3) - 1) < 0.02


def test_lanczos_reproduces_a_jacobi_matrix():
    """Started from e_1, the recurrence on a symmetric tridiagonal matrix with
    positive off-diagonal returns exactly its diagonal (alpha) and off-diagonal
    (beta): the Lanczos tridiagonalisation of a Jacobi matrix is the matrix
    itself.  Under an orthogonal similarity Q T Q^T started from Q e_1 the
    coefficients are unchanged.  A dropped term, a wrong sign or a shifted
    index in the recurrence breaks one of these."""
    rng = np.random.default_rng(17)
    n = 12
    diag = rng.standard_normal(n)
    off = rng.uniform(0.5, 2.0, n - 1)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    e1 = np.zeros(n)
    e1[0] = 1.0
    a, b = ftlm.lanczos(lambda x: T @ x, e1, n)
    assert len(a) == n
    assert np.max(np.abs(a - diag)) < 1e-13
    assert np.max(np.abs(b[: n - 1] - off)) < 1e-13
    assert abs(b[n - 1]) < 1e-12              # the Krylov space is exhausted
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ T @ Q.T
    a2, b2 = ftlm.lanczos(lambda x: A @ x, 3.0 * (Q @ e1), n)   # any start norm
    assert np.max(np.abs(a2 - diag)) < 1e-12
    assert np.max(np.abs(b2[: n - 1] - off)) < 1e-12
    # fewer steps: the leading part of the same coefficients
    a3, b3 = ftlm.lanczos(lambda x: A @ x, Q @ e1, 5)
    assert len(a3) == 5 and np.max(np.abs(a3 - diag[:5])) < 1e-12 and np.max(np.abs(b3 - off[:5])) < 1e-12


def test_gaussian_start_values_are_standard_normal():
    """Box-Muller values before normalisation: the standard normal law by a
    Kolmogorov-Smirnov test, with its third and fourth moments (0 and 3)."""
    import scipy.stats as st
    D = 200000
    g = ftlm.start_vector(D, 11, 0, 2, 0, 3, "gaussian")
    # the unit vector times sqrt(D): the raw draws up to their sample RMS (1 +- 0.3%)
    x = g * np.sqrt(D)
    ks = st.kstest(x, "norm")
    assert ks.pvalue > 1e-3, ks
    assert abs(np.mean(x ** 3)) < 0.05
    assert abs(np.mean(x ** 4) - 3.0) < 0.1
