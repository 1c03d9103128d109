"""GPU parity of the real forms of complex-type irreps (translation groups)
and of quaternionic irreps (dicyclic groups Dic_2 = Q8, Dic_3).

* Blocks built with the oracle's realified irreps (user_rho, trace weight
  dim/2 for a complex pair, dim/4 when quaternionic): dimensions, n_Gamma and offsets bit for bit against the oracle's
  block of the same real form, FP64 H.V within 1e-12 of Psi^T H Psi X, and
  the Lanczos coefficients of the fused and the per-step kernels against the
  oracle's recurrence.
* The whole campaign with the library's own irreps (realified pairs, weight
  dim/2; realified quaternionic irreps, weight dim/4) against the oracle's FTLM estimator run on the same blocks (the
  library's irrep matrices, the same chain keys and start vectors): E, C,
  chi within 1e-9 relative; ln Z(T -> inf) = N ln(2s+1) exactly.
"""
import numpy as np
import pytest

from gpu_helpers import lib_group, log, oracle_weight, rel_err_cols
from oracle import basis, ftlm as oftlm, group, hv, irreps, realform, sector
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

CASES = [("ring8_C", 1, 0), ("square3x3_T", 1, 1), ("ring6_C", 2, 0), ("ring5_C", 3, 1), ("square4x4_T", 1, 0),
         ("dic2", 3, 0), ("dic3", 1, 2), ("dic3", 1, 0)]


def _setup(name, two_s, two_M):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    forms = realform.real_forms(G, irreps.compute_irreps(G))
    sec = basis.sector_reps(G, cl.N, two_s, two_M)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    S = P.Sector(cl, lib_group(name), two_M, two_s=two_s)
    return cl, G, forms, sec, H, S


@pytest.mark.parametrize("name,two_s,two_M", CASES)
def test_realified_blocks_and_hv_fp64(name, two_s, two_M):
    cl, G, forms, sec, H, S = _setup(name, two_s, two_M)
    rng = np.random.default_rng(23)
    pairs = 0
    for k, f in enumerate(forms):
        log(f"[realform] {name} 2s={two_s} 2M={two_M} form {k} ({f.kind})")
        B = basis.build_block(G, f.irrep, sec)
        LB = P.Block(S, k, 0, user_rho=f.irrep.rho, user_rho_weight=f.weight)
        assert LB.D == B.D and LB.trace_weight == f.weight and LB.d_gamma == f.irrep.dim
        ex = LB.export()
        assert np.array_equal(ex["n_gamma"].astype(np.int64), B.n_rep)
        assert np.array_equal(ex["offsets"].astype(np.int64), B.offsets)
        if B.D == 0:
            continue
        pairs += f.kind != "real"
        for nvec in (1, 5):
            X = rng.standard_normal((B.D, nvec))
            Y = LB.apply_H(torch.from_numpy(X).cuda()).cpu().numpy()
            assert rel_err_cols(Y, hv.apply(B, H, X)) <= 1e-12, (k, nvec)
    assert pairs > 0


@pytest.mark.parametrize("name,two_s,two_M", CASES[:4] + CASES[5:7])
def test_realified_block_lanczos_against_oracle(name, two_s, two_M):
    cl, G, forms, sec, H, S = _setup(name, two_s, two_M)
    for k, f in enumerate(forms):
        if f.kind == "real":
            continue
        B = basis.build_block(G, f.irrep, sec)
        if B.D < 2:
            continue
        Hb = hv.block_matrix(B, H)
        LB = P.Block(S, k, 0, user_rho=f.irrep.rho, user_rho_weight=f.weight)
        a0, b0, n0 = LB.ftlm(3, 20, 41)
        (a1, b1, n1), = P.run_fused([dict(block=LB, R=3, steps=20, seed=41)])
        for r in range(3):
            v0 = oftlm.start_vector(B.D, 41, two_M, k, 0, r, "rademacher")
            oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, 20)
            m = min(8, len(oa) - 1)
            sig = np.nonzero(ob[:m] < 1e-6 * np.max(ob[:m]))[0] if m > 0 else []
            m = int(sig[0]) if len(sig) else m
            for a in (a0, a1):
                assert np.max(np.abs(a[r, :m + 1] - oa[:m + 1])) <= 1e-10 * np.max(np.abs(oa)), (k, r)
            for b in (b0, b1):
                assert np.max(np.abs(b[r, :m] - ob[:m])) <= 1e-10 * np.max(np.abs(ob)), (k, r)


@pytest.mark.parametrize("name,two_s", [("ring8_C", 1), ("square3x3_T", 1), ("ring6_C", 2), ("dic2", 2), ("dic3", 1)])
def test_campaign_with_realified_pairs_matches_oracle_ftlm(name, two_s):
    log(f"[realform] campaign {name} 2s={two_s}")
    cl = clusters.get(name)
    LG = lib_group(name)
    G = group.close(cl.gens, cl.N)
    info = LG.irreps()
    T = np.geomspace(0.05, 10, 30)
    R, steps, seed = 6, 25, 0x5EED0007
    res = P.campaign(cl, cl.gens, two_s, R, steps, seed, T, storage=P.F64, engine=P.ENGINE_STEPS)
    fused = P.campaign(cl, cl.gens, two_s, R, steps, seed, T, storage=P.F64, engine=P.ENGINE_FUSED)
    # the oracle's estimator on the same blocks (library irrep matrices) and start vectors
    blocks = []
    Ns2 = cl.N * two_s
    for two_M in range(Ns2 % 2, Ns2 + 1, 2):
        sec = basis.sector_reps(G, cl.N, two_s, two_M)
        H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
        for k in range(len(info["dims"])):
            ir = irreps.Irrep(int(info["dims"][k]), LG.rho(k), None, int(info["indicators"][k]))
            ir.chars = np.trace(ir.rho, axis1=1, axis2=2).astype(complex)
            # the library's matrices enter the oracle only as a choice of basis: checked
            # first to be a real orthogonal representation of the oracle's group (with the
            # character of one of the oracle's real forms, inside oracle_weight below)
            assert np.max(np.abs(np.einsum("gij,hjk->ghik", ir.rho, ir.rho) - ir.rho[G.mul])) < 1e-12
            assert np.max(np.abs(np.einsum("gji,gjk->gik", ir.rho, ir.rho) - np.eye(ir.dim))) < 1e-12
            B = basis.build_block(G, ir, sec)
            if B.D == 0:
                continue
            Hb = hv.block_matrix(B, H)
            ths, ws = [], []
            for r in range(R):
                v0 = oftlm.start_vector(B.D, seed, two_M, k, 0, r, "rademacher")
                th, w = oftlm.ritz(*oftlm.lanczos(lambda x: Hb @ x, v0, steps))
                ths.append(th)
                ws.append(w)
            blocks.append(oftlm.BlockRitz(two_M, oracle_weight(name, ir.rho), B.D, ths, ws))
    E, C, chi, lz = oftlm.observables(blocks, T, with_logZ=True)
    for out in (res, fused):
        for got, want in ((out["E"], E), (out["C"], C), (out["chi"], chi), (out["logZ"], lz)):
            assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
    hi = P.campaign(cl, cl.gens, two_s, R, steps, seed, np.array([1e9]), storage=P.F64)
    assert abs(hi["logZ"][0] - cl.N * np.log(two_s + 1)) < 1e-6
    assert res["stats"]["blocks"] == len(blocks)


@pytest.mark.parametrize("name,two_s", [("ring8_C", 1), ("square4x4_T", 1), ("dic2", 2), ("dic3", 1)])
def test_realified_pairs_with_spin_flip(name, two_s):
    """G x Z2 at M = 0 over real forms: Gamma^+ and Gamma^- of every form
    (complex pairs and quaternionic irreps); a campaign with the flip keeps
    ln Z(T -> inf) = N ln(2s + 1), so the trace weights add up."""
    from oracle import spinflip
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    forms = realform.real_forms(G, irreps.compute_irreps(G))
    G2 = spinflip.FlipGroup(G)
    irs2 = spinflip.flip_irreps([f.irrep for f in forms])
    sec = basis.sector_reps(G2, cl.N, two_s, 0)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    S = P.Sector(cl, lib_group(name), 0, two_s=two_s, spin_flip=True)
    rng = np.random.default_rng(29)
    for gi2, ir2 in enumerate(irs2):
        B = basis.build_block(G2, ir2, sec)
        f = forms[gi2 // 2]
        LB = P.Block(S, gi2, 0, user_rho=f.irrep.rho, user_rho_weight=f.weight)
        assert LB.D == B.D
        if B.D == 0:
            continue
        X = rng.standard_normal((B.D, 3))
        Y = LB.apply_H(torch.from_numpy(X).cuda()).cpu().numpy()
        assert rel_err_cols(Y, hv.apply(B, H, X)) <= 1e-12, gi2
    hi = P.campaign(cl, cl.gens, two_s, 4, 20, 5, np.array([1e9]), storage=P.F64, spin_flip=True)
    assert abs(hi["logZ"][0] - cl.N * np.log(two_s + 1)) < 1e-6
