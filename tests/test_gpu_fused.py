"""GPU parity of the fused small-block Lanczos kernel (ftlm_run_fused).

* Against the oracle: the alpha/beta of every chain equal the oracle's
  Lanczos recurrence on the explicitly projected block matrix (same start
  vectors) over the first steps, where the recurrence has not yet amplified
  rounding, for blocks of irrep dimensions 1-5 and several R.
* Against the per-step kernels (ftlm_run, same keys): step counts equal and
  the first steps' coefficients to rounding (FP64 1e-12; FP32 storage 1e-5,
  since a last-bit change of a stored FP32 element moves later coefficients
  by ~1e-7 relative); one call mixing kernel shapes (R, storage, dimension,
  label width) gives each job the result of that job alone, bit for bit.
  A chain offset (first_chain) reproduces the start vectors of the larger run.
* Edge cases: blocks with D < steps (the chain stops at D), a one-row block,
  an empty block, chain offsets (first_chain), repeated blocks, and rejected
  jobs (R > 32, FP16 storage, on-the-fly sectors).
* Campaign: the fused engine agrees with the per-step engine on E, C, chi to
  rounding and runs every block of a small cluster; the automatic engine
  splits a larger cluster between the two.
"""
import numpy as np
import pytest

from gpu_helpers import lib_group, lib_sector, log, oracle_block, oracle_group, oracle_sector
from oracle import ftlm as oftlm
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

T_GRID = np.geomspace(0.05, 10, 50)


def _lib_block(name, two_s, two_M, gi, hv_mode=0):
    cl, G, irs = oracle_group(name)
    return P.Block(lib_sector(name, two_s, two_M, hv_mode=hv_mode), gi, 0, user_rho=irs[gi].rho)


def _rel(a, b):
    if len(b) == 0:
        return 0.0
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _significant(beta, k):
    """Steps whose coefficients are determined by the block rather than by
    rounding: alpha_0..alpha_m and beta_0..beta_{m-1} with m the first step
    (below k) whose beta has cancelled to 1e-6 of the largest (the Krylov space
    is exhausted; the next vector is rounding noise)."""
    beta = np.asarray(beta[:k])
    small = np.nonzero(beta < 1e-6 * max(np.max(np.abs(beta)), 1e-300))[0] if len(beta) else []
    m = int(small[0]) if len(small) else k
    return min(m + 1, k), m


# (cluster, 2s, 2M, irrep) over irrep dimensions 1..5 and both label widths
ORACLE_CASES = [("icosahedron", 1, 0, 0), ("icosahedron", 1, 2, 8), ("icosahedron", 1, 0, 9),
                ("cuboctahedron", 1, 0, 4), ("ring6", 2, 0, 2), ("K4", 3, 2, 3), ("dodecahedron", 1, 8, 4)]


@pytest.mark.parametrize("name,two_s,two_M,gi", ORACLE_CASES)
@pytest.mark.parametrize("R", [1, 3, 24])
def test_fused_against_oracle(name, two_s, two_M, gi, R):
    log(f"[fused] oracle {name} 2s={two_s} 2M={two_M} irrep {gi} R={R}")
    sec, H = oracle_sector(name, two_s, two_M)
    B = oracle_block(name, two_s, two_M, gi)
    if B.D == 0:
        pytest.skip("empty block")
    Hb = (B.Psi.T @ H @ B.Psi).tocsr()
    LB = _lib_block(name, two_s, two_M, gi)
    assert LB.D == B.D
    steps = 30
    (a, b, n), = P.run_fused([dict(block=LB, R=R, steps=steps, seed=91)])
    for r in range(R):
        v0 = oftlm.start_vector(B.D, 91, two_M, gi, 0, r, "rademacher")
        oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, steps)
        assert n[r] <= min(steps, B.D)
        k = min(12, B.D - 1, len(oa))
        if k > 0:
            ka, kb = _significant(ob, k)
            assert _rel(a[r, :ka], oa[:ka]) < 1e-10, (r, a[r, :ka], oa[:ka])
            assert _rel(b[r, :kb], ob[:kb]) < 1e-10
        else:
            assert abs(a[r, 0] - oa[0]) < 1e-12 * max(abs(oa[0]), 1)


STEPS_CASES = [("icosahedron", 1, 0, 8), ("cuboctahedron", 1, 2, 3), ("dodecahedron", 1, 6, 9),
               ("dodecahedron", 1, 10, 0), ("ring6", 2, 2, 1), ("K4", 3, 0, 4)]


@pytest.mark.parametrize("name,two_s,two_M,gi", STEPS_CASES)
@pytest.mark.parametrize("R,storage", [(1, P.F64), (4, P.F64), (24, P.F64), (32, P.F64), (4, P.F32), (24, P.F32)])
def test_fused_matches_per_step_kernels(name, two_s, two_M, gi, R, storage):
    log(f"[fused] vs ftlm_run {name} 2M={two_M} irrep {gi} R={R} storage={storage}")
    LB = _lib_block(name, two_s, two_M, gi)
    if LB.D == 0:
        pytest.skip("empty block")
    steps = 40
    a0, b0, n0 = LB.ftlm(R, steps, 5, storage=storage)
    (a1, b1, n1), = P.run_fused([dict(block=LB, R=R, steps=steps, seed=5, storage=storage)])
    assert np.array_equal(n0, n1)
    tol = 1e-12 if storage == P.F64 else 1e-5
    for r in range(R):
        ka, kb = _significant(b0[r], min(10, int(n0[r])))
        assert _rel(a1[r, :ka], a0[r, :ka]) < tol, r
        assert _rel(b1[r, :kb], b0[r, :kb]) < tol, r
    # unused tail is zero, as in ftlm_run
    for r in range(R):
        assert not a1[r, n1[r]:].any() and not b1[r, n1[r]:].any()


def test_fused_mixed_batch_equals_single_jobs():
    log("[fused] mixed batch")
    jobs = [dict(block=_lib_block("icosahedron", 1, 0, 9), R=4, steps=30, seed=1),
            dict(block=_lib_block("icosahedron", 1, 0, 9), R=24, steps=30, seed=1, storage=P.F32),
            dict(block=_lib_block("cuboctahedron", 1, 0, 4), R=1, steps=25, seed=2, dist=P.GAUSSIAN),
            dict(block=_lib_block("dodecahedron", 1, 8, 4), R=12, steps=50, seed=3),
            dict(block=_lib_block("K4", 3, 2, 3), R=2, steps=20, seed=4),
            dict(block=_lib_block("icosahedron", 1, 2, 0), R=32, steps=30, seed=5, first_chain=7)]
    together = P.run_fused(jobs)
    again = P.run_fused(jobs)
    for j, (a, b, n), (a2, b2, n2) in zip(jobs, together, again):
        (sa, sb, sn), = P.run_fused([j])
        assert np.array_equal(a, sa) and np.array_equal(b, sb) and np.array_equal(n, sn)
        assert np.array_equal(a, a2) and np.array_equal(b, b2)   # deterministic


def test_fused_first_chain_offsets_keys():
    # chains 4, 5 of a 6-chain job and a 2-chain job starting at chain 4 share
    # their start vectors; the lane layout (and so the summation order) differs
    LB = _lib_block("icosahedron", 1, 0, 9)
    (a, b, n), = P.run_fused([dict(block=LB, R=6, steps=20, seed=8)])
    (a2, b2, n2), = P.run_fused([dict(block=LB, R=2, steps=20, seed=8, first_chain=4)])
    for r in range(2):
        ka, kb = _significant(b[4 + r], 12)
        assert _rel(a2[r, :ka], a[4 + r, :ka]) < 1e-12 and _rel(b2[r, :kb], b[4 + r, :kb]) < 1e-12


def test_fused_short_blocks_stop_at_dimension():
    # blocks with D < steps: the recurrence ends after at most D products
    cl, G, irs = oracle_group("icosahedron")
    for two_M, gi in [(12, 0), (10, 0), (10, 8), (8, 4)]:
        LB = _lib_block("icosahedron", 1, two_M, gi)
        if LB.D == 0:
            continue
        a0, b0, n0 = LB.ftlm(3, 30, 6)
        (a1, b1, n1), = P.run_fused([dict(block=LB, R=3, steps=30, seed=6)])
        assert np.array_equal(n0, n1) and n1.max() <= LB.D
        for r in range(3):
            ka, kb = _significant(b0[r], int(n0[r]))
            assert _rel(a1[r, :ka], a0[r, :ka]) < 1e-12
        if LB.D == 1:
            # one row: alpha = <e|H|e>, beta = 0
            sec, H = oracle_sector("icosahedron", 1, two_M)
            B = oracle_block("icosahedron", 1, two_M, gi)
            Hb = (B.Psi.T @ H @ B.Psi).toarray()
            assert np.allclose(a1[:, 0], Hb[0, 0], rtol=1e-13) and n1.tolist() == [1, 1, 1]


def test_fused_empty_block_and_rejections():
    LB = _lib_block("icosahedron", 1, 12, 9)   # M = 6 holds one state, which has no H_u component
    assert LB.D == 0
    (a, b, n), = P.run_fused([dict(block=LB, R=2, steps=5, seed=1)])
    assert not a.any() and not n.any()
    ok = _lib_block("icosahedron", 1, 0, 9)
    for bad in [dict(block=ok, R=33, steps=5, seed=1), dict(block=ok, R=4, steps=5, seed=1, storage=P.F16),
                dict(block=ok, R=4, steps=0, seed=1)]:
        with pytest.raises(P.FtlmError, match="INVALID_ARG"):
            P.run_fused([bad])
    otf = _lib_block("icosahedron", 1, 0, 9, hv_mode=P.HV_ONTHEFLY)
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        P.run_fused([dict(block=otf, R=4, steps=5, seed=1)])


def test_campaign_fused_engine_matches_per_step_engine():
    log("[fused] campaign engines")
    cl = clusters.get("icosahedron")
    for cpr in (0, 1):
        f = P.campaign(cl, cl.gens, 1, 4, 30, 0x5EED0001, T_GRID, storage=P.F64, chains_per_run=cpr,
                       engine=P.ENGINE_FUSED)
        s = P.campaign(cl, cl.gens, 1, 4, 30, 0x5EED0001, T_GRID, storage=P.F64, chains_per_run=cpr,
                       engine=P.ENGINE_STEPS)
        assert f["stats"]["fused_blocks"] == f["stats"]["blocks"] == s["stats"]["blocks"]
        assert s["stats"]["fused_blocks"] == 0
        # a chain whose Krylov space is exhausted stops when rounding noise
        # falls below the breakdown threshold, which the two summation orders
        # may reach a step apart
        assert abs(f["stats"]["work"] - s["stats"]["work"]) <= 1e-3 * s["stats"]["work"]
        for key in ("E", "C", "chi", "logZ"):
            assert _rel(f[key], s[key]) < 1e-9, key


def test_campaign_auto_engine_splits_by_sector_size():
    log("[fused] campaign auto engine, dodecahedron")
    cl = clusters.get("dodecahedron")
    a = P.campaign(cl, cl.gens, 1, 24, 60, 9, T_GRID, storage=P.F64)
    s = P.campaign(cl, cl.gens, 1, 24, 60, 9, T_GRID, storage=P.F64, engine=P.ENGINE_STEPS)
    assert 0 < a["stats"]["fused_blocks"] < a["stats"]["blocks"]
    assert abs(a["stats"]["work"] - s["stats"]["work"]) <= 1e-3 * s["stats"]["work"]
    for key in ("E", "C", "chi"):
        assert _rel(a[key], s[key]) < 1e-8, key
