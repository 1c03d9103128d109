"""GPU tests of the whole-cluster FTLM driver (ftlm_campaign).

* Orchestration: the campaign's E, C, chi, ln Z equal, bit for bit, those of
  the same blocks run one by one through ftlm_run (per-step engine) or
  through ftlm_run_fused (fused engine) and summed by ftlm_observables (same
  library irreps, seeds and chain keys).
* Exact limits of the aggregate, independent of the chains: Z(T -> inf) =
  (2s+1)^N and T chi / g^2 -> N s(s+1)/3.
* With the spin flip at M = 0 (G x Z2) and 48 chains, E(T) agrees with the
  oracle's full exact diagonalization within the stochastic error (2% of the
  curve maximum).
* Chains run one at a time (the plain single-vector path) agree with the
  batched run up to rounding.
"""
import numpy as np
import pytest

from gpu_helpers import lib_group, log
from oracle import ftlm as oftlm
from oracle import sector
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

T_GRID = np.geomspace(0.05, 10, 50)


def _blockwise(name, two_s, R, steps, seed, storage, fused=False):
    cl = clusters.get(name)
    G = lib_group(name)
    n_irr = len(G.irreps()["dims"])
    blocks = []
    for two_M in range((cl.N * two_s) % 2, cl.N * two_s + 1, 2):
        S = P.Sector(cl, G, two_M, two_s=two_s)
        for gi in range(n_irr):
            B = P.Block(S, gi, 0)
            if B.D == 0:
                continue
            if fused:
                (a, b, n), = P.run_fused([dict(block=B, R=R, steps=steps, seed=seed, storage=storage)])
            else:
                a, b, n = B.ftlm(R, steps, seed, storage=storage)
            ths, ws = P.ritz_from_run(a, b, n)
            blocks.append(dict(two_M=two_M, d_gamma=B.d_gamma, D=B.D, thetas=ths, weights=ws))
    return blocks


def test_campaign_equals_blockwise_runs():
    log("[campaign] icosahedron vs block-by-block")
    cl = clusters.get("icosahedron")
    for engine, fused in ((P.ENGINE_STEPS, False), (P.ENGINE_FUSED, True)):
        res = P.campaign(cl, cl.gens, 1, 4, 30, 0x5EED0001, T_GRID, storage=P.F64, engine=engine)
        E, C, chi, lz = P.observables(_blockwise("icosahedron", 1, 4, 30, 0x5EED0001, P.F64, fused), T_GRID)
        assert np.array_equal(res["E"], E) and np.array_equal(res["C"], C)
        assert np.array_equal(res["chi"], chi) and np.array_equal(res["logZ"], lz)
    st = res["stats"]
    assert st["sectors"] == 7 and st["blocks"] + st["empty_blocks"] == 70
    hi = P.campaign(cl, cl.gens, 1, 4, 30, 0x5EED0001, np.array([1e9]), storage=P.F64)
    assert abs(np.exp(hi["logZ"][0]) / 2 ** 12 - 1) < 1e-6
    assert abs(1e9 * hi["chi"][0] / (12 * 0.75 / 3) - 1) < 1e-6


def test_campaign_spin_flip_against_exact_diagonalization():
    log("[campaign] icosahedron with the spin flip vs ED")
    cl = clusters.get("icosahedron")
    res = P.campaign(cl, cl.gens, 1, 48, 40, 11, T_GRID, storage=P.F64, spin_flip=True)
    spectra = {}
    for two_M in range(0, cl.N + 1, 2):
        labels = sector.enumerate_sector(cl.N, 1, two_M)
        H = sector.hamiltonian(labels, cl.N, 1, cl.bonds, cl.J).toarray()
        spectra[two_M] = np.linalg.eigvalsh(H)
    Eed, Ced, chied = oftlm.ed_observables(spectra, T_GRID)
    # stochastic error of the trace estimate, normalised by the curve maximum
    # (the convention of the paper's comparisons with exact results)
    assert np.max(np.abs(res["E"] - Eed)) / np.max(np.abs(Eed)) < 0.02
    hi = P.campaign(cl, cl.gens, 1, 4, 30, 1, np.array([1e9]), storage=P.F64, spin_flip=True)
    assert abs(np.exp(hi["logZ"][0]) / 2 ** 12 - 1) < 1e-6


def test_campaign_single_vector_path_matches_batched():
    log("[campaign] single-vector path")
    cl = clusters.get("dodecahedron")
    a = P.campaign(cl, cl.gens, 1, 6, 40, 3, T_GRID, storage=P.F64, all_M=False, two_M=4)
    b = P.campaign(cl, cl.gens, 1, 6, 40, 3, T_GRID, storage=P.F64, all_M=False, two_M=4, chains_per_run=1)
    assert a["stats"]["work"] == b["stats"]["work"]
    assert np.max(np.abs(a["E"] - b["E"]) / np.abs(a["E"])) < 1e-8
