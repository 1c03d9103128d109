"""Pins of the KPM oracle (oracle/kpm.py).

* The moments' definition (eigen-decomposition, cos(n arccos x)) equals the
  three-term Chebyshev recurrence applied to vectors; mu_0 = 1, |mu_n| <= 1.
* Over an orthonormal basis the moments sum to the trace sum_k T_n(x_k).
* Jackson kernel: g_0 = 1 and the closed values for N = 2 and N = 3.
* Quadrature weights: sum_k W_k T_m(x_k) = g_m mu_m for m < N (the discrete
  cosine orthogonality), so sum_k W_k = 1.
* Thermodynamics from exact-trace moments converge to full ED of a ring
  (all M sectors) as the number of moments grows; the T -> infinity energy is
  c + w g_1 mu_1 averaged with the block weights.
"""
import numpy as np
import pytest

from oracle import ftlm as oftlm, kpm, sector
from synth import clusters


def _recurrence(Hb, r, c, w, n):
    r = r / np.linalg.norm(r)
    Ht = (Hb - c * np.eye(len(r))) / w
    t0, t1 = r, Ht @ r
    out = [r @ t0, r @ t1]
    for _ in range(2, n):
        t0, t1 = t1, 2 * Ht @ t1 - t0
        out.append(r @ t1)
    return np.array(out[:n])


def test_moments_definition_matches_recurrence():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40))
    H = A + A.T
    e = np.linalg.eigvalsh(H)
    c, w = 0.5 * (e[0] + e[-1]), 0.51 * (e[-1] - e[0])
    r = rng.standard_normal(40)
    mu = kpm.moments(H, r, c, w, 120)
    assert abs(mu[0] - 1) < 1e-14 and np.all(np.abs(mu) <= 1 + 1e-12)
    assert np.allclose(mu, _recurrence(H, r, c, w, 120), atol=1e-11)


def test_orthonormal_basis_gives_the_trace():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((25, 25))
    H = A + A.T
    e = np.linalg.eigvalsh(H)
    c, w = 0.5 * (e[0] + e[-1]), 0.6 * (e[-1] - e[0])
    tot = sum(kpm.moments(H, np.eye(25)[i], c, w, 30) for i in range(25))
    want = np.cos(np.outer(np.arange(30), np.arccos((e - c) / w))).sum(axis=1)
    assert np.allclose(tot, want, atol=1e-11)


def test_jackson_kernel_values():
    assert np.allclose(kpm.jackson(2), [1.0, 0.5])
    # N = 3: q = pi/4, g_1 = [3 cos q + sin q cot q] / 4, g_2 = [2 cos 2q + sin 2q cot q] / 4
    q = np.pi / 4
    assert np.allclose(kpm.jackson(3), [1.0, (3 * np.cos(q) + np.cos(q)) / 4, (0 + 1.0 / np.tan(q)) / 4])
    g = kpm.jackson(200)
    assert g[0] == 1.0 and np.all(np.diff(g) < 0) and 0 < g[-1] < 1e-3


def test_node_weights_reproduce_damped_moments():
    rng = np.random.default_rng(5)
    N, K = 40, 96
    mu = np.concatenate([[1.0], rng.uniform(-1, 1, N - 1)])
    x, W = kpm.node_weights(mu, K)
    g = kpm.jackson(N)
    for m in range(N):
        assert abs(np.sum(W * np.cos(m * np.arccos(x))) - g[m] * mu[m]) < 1e-13
    assert abs(W.sum() - 1) < 1e-14


def _ring_blocks(N, n_mom):
    cl = clusters.ring(N)
    blocks, spectra = [], {}
    for two_M in range(N % 2, N + 1, 2):
        labels = sector.enumerate_sector(cl.N, 1, two_M)
        H = sector.hamiltonian(labels, cl.N, 1, cl.bonds, cl.J).toarray()
        e = np.linalg.eigvalsh(H)
        spectra[two_M] = e
        D = len(e)
        c = 0.5 * (e[0] + e[-1])
        w = max(0.505 * (e[-1] - e[0]), 1e-3)
        mom = np.array([kpm.moments(H, np.eye(D)[i], c, w, n_mom) for i in range(D)])
        blocks.append(kpm.KpmBlock(two_M, 1, D, mom, c, w))
    return blocks, spectra


def test_thermodynamics_converge_to_exact_diagonalization():
    T = np.geomspace(0.3, 10, 25)
    blocks, spectra = _ring_blocks(10, 400)
    E, C, chi = kpm.observables(blocks, T)
    Ee, Ce, chie = oftlm.ed_observables(spectra, T)
    assert np.max(np.abs(E - Ee)) < 2e-3 * np.max(np.abs(Ee))
    assert np.max(np.abs(C - Ce)) < 2e-3 * np.max(np.abs(Ce))
    assert np.max(np.abs(chi - chie)) < 2e-3 * np.max(np.abs(chie))
    # fewer moments: a broader kernel, a larger error
    b2, _ = _ring_blocks(10, 60)
    E2, C2, _ = kpm.observables(b2, T)
    assert np.max(np.abs(C2 - Ce)) > np.max(np.abs(C - Ce))


def test_high_temperature_energy():
    blocks, spectra = _ring_blocks(8, 50)
    E, _, _, lz = kpm.observables(blocks, np.array([1e12]), with_logZ=True)
    g1 = kpm.jackson(50)[1]
    num = den = 0.0
    for b in blocks:
        mult = 1 if b.two_M == 0 else 2
        mu1 = b.moments.mean(axis=0)[1]
        num += mult * b.D * (b.center + b.half_width * g1 * mu1)
        den += mult * b.D
    assert abs(E[0] - num / den) < 1e-9 * abs(num / den) + 1e-9
    assert abs(np.exp(lz[0]) / 2 ** 8 - 1) < 1e-9
