"""FTLM observables E, C, chi (paper Eqs. 4-7 and 14) per configuration, with
the error stated per temperature.

* Dodecahedron s=1/2, every M >= 0 sector, all ten I_h irreps, R = 24
  Rademacher chains of 60 steps: the library's blocks (the oracle's irrep
  matrices) against the oracle's FTLM on its explicit blocks with the same
  start vectors, FP64 storage within 1e-9 and FP32 storage within 1e-6
  relative at every temperature of the grid.
* Icosidodecahedron s=1/2, M = 0, all ten irreps, R = 24 Gaussian chains of 60
  steps: FP32 storage against the FP64 path of the library, same keys.  The
  blocks (up to 6.5e6 rows) are beyond the explicit oracle; what is compared
  is the precision of the storage, per temperature (E and C; chi vanishes
  when only M = 0 enters).
* The s=3/2 icosahedron, all M, R = 100, N_L = 100: FP16 against FP32
  storage, the paper's own validation of half-precision storage.
"""
import numpy as np
import pytest

from gpu_helpers import lib_block, log, oracle_block, oracle_group, oracle_sector
from oracle import ftlm as oftlm
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

T_GRID = np.geomspace(0.05, 10, 50)
SEED2 = 0x5EED0002
SEED3 = 0x5EED0003


def _rel(x, ref):
    return np.abs(x - ref) / np.abs(ref)


def _log_per_T(tag, eE, eC, eX):
    log(f"  {tag}: max rel err E {eE.max():.2e} C {eC.max():.2e} chi {eX.max():.2e}")
    for k in range(0, len(T_GRID), 7):
        log(f"    T={T_GRID[k]:.4f} E {eE[k]:.2e} C {eC[k]:.2e} chi {eX[k]:.2e}")


@pytest.fixture(scope="module")
def dodeca_oracle():
    """The oracle's FTLM on every (M >= 0, irrep) block of the s=1/2 dodecahedron."""
    name, two_s, R, steps = "dodecahedron", 1, 24, 60
    cl, G, irs = oracle_group(name)
    blocks, keys = [], []
    log("[observables] oracle FTLM, dodecahedron all sectors")
    for two_M in range(0, cl.N * two_s + 1, 2):
        sec, H = oracle_sector(name, two_s, two_M)
        for gi, ir in enumerate(irs):
            B = oracle_block(name, two_s, two_M, gi)
            if B.D == 0:
                continue
            Hb = (B.Psi.T @ H @ B.Psi).tocsr()
            ths, ws = [], []
            for r in range(R):
                v0 = oftlm.start_vector(B.D, SEED2, two_M, gi, 0, r, "rademacher")
                th, w = oftlm.ritz(*oftlm.lanczos(lambda x: Hb @ x, v0, steps))
                ths.append(th)
                ws.append(w)
            blocks.append(oftlm.BlockRitz(two_M, ir.dim, B.D, ths, ws))
            keys.append((two_M, gi, B.D, ir.dim))
    return blocks, keys


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage,tol", [(0, 1e-9), (1, 1e-6)])
def test_dodecahedron_all_sectors_against_oracle(dodeca_oracle, storage, tol):
    ora_blocks, keys = dodeca_oracle
    log(f"[observables] dodecahedron all sectors, storage {storage}")
    lib_blocks = []
    for (two_M, gi, D, dim), ob in zip(keys, ora_blocks):
        LB = lib_block("dodecahedron", 1, two_M, gi)
        assert LB.D == D
        a, b, n = LB.ftlm(24, 60, SEED2, storage=storage)
        # steps per chain: min(60, D), fewer where a start vector lies in a
        # small invariant subspace (the same breakdown test on both sides; in
        # FP32 storage the rounding keeps beta near 1e-7 of the scale, above
        # the 1e-10 test, so such a chain runs on to min(60, D) with weights
        # of order beta^2 on the extra Ritz values)
        want = [len(t) for t in ob.thetas]
        if storage == P.F64:
            assert [int(x) for x in n] == want, (two_M, gi)
        else:
            assert all(w <= int(x) <= min(60, D) for x, w in zip(n, want)), (two_M, gi)
        ths, ws = P.ritz_from_run(a, b, n)
        lib_blocks.append(dict(two_M=two_M, d_gamma=dim, D=D, thetas=ths, weights=ws))
    assert len(lib_blocks) == 97
    E, C, chi, lz = P.observables(lib_blocks, T_GRID)
    Eo, Co, chio, lzo = oftlm.observables(ora_blocks, T_GRID, with_logZ=True)
    eE, eC, eX = _rel(E, Eo), _rel(C, Co), _rel(chi, chio)
    _log_per_T(f"storage {storage}", eE, eC, eX)
    assert eE.max() <= tol and eC.max() <= tol and eX.max() <= tol
    assert np.max(np.abs(lz - lzo)) <= tol * np.max(np.abs(lzo))


@pytest.mark.timeout(900)
def test_icosidodecahedron_m0_fp32_against_fp64():
    log("[observables] icosidodecahedron M=0, ten irreps, FP32 against FP64")
    cl = clusters.get("icosidodecahedron")
    G = P.Group(cl.N, cl.gens)
    S = P.Sector(cl, G, 0, two_s=1)
    b64, b32 = [], []
    dims = []
    for gi in range(10):
        B = P.Block(S, gi, 0)
        dims.append(B.D)
        for st, out in ((P.F64, b64), (P.F32, b32)):
            a, b, n = B.ftlm(24, 60, SEED3, storage=st, dist=P.GAUSSIAN)
            assert np.all(n == 60)
            ths, ws = P.ritz_from_run(a, b, n)
            out.append(dict(two_M=0, d_gamma=B.trace_weight, D=B.D, thetas=ths, weights=ws))
        del B
    assert sorted(dims) == sorted([1295266, 1291834, 3875366, 3878798, 3875366, 3878798, 5170622, 5170622,
                                   6465762, 6462330])
    E, C, chi, _ = P.observables(b32, T_GRID)
    E0, C0, chi0, _ = P.observables(b64, T_GRID)
    # only M = 0 enters: <M^2> = 0, so chi vanishes identically on both sides
    assert np.all(chi == 0.0) and np.all(chi0 == 0.0)
    eE, eC = _rel(E, E0), _rel(C, C0)
    eX = np.zeros_like(eE)
    _log_per_T("FP32 vs FP64 (chi = 0)", eE, eC, eX)
    e0_32 = min(t.min() for b in b32 for t in b["thetas"])
    e0_64 = min(t.min() for b in b64 for t in b["thetas"])
    log(f"  lowest Ritz value FP64 {e0_64:.10f} FP32 {e0_32:.10f}")
    assert abs(e0_32 - e0_64) <= 1e-6 * abs(e0_64)
    assert eE.max() <= 1e-6 and eC.max() <= 1e-6


@pytest.mark.timeout(600)
def test_fp16_storage_on_the_papers_validation_case():
    """Section 4.2's validation of half-precision storage: the s=3/2
    icosahedron, every M >= 0 sector and irrep, R = 100 chains of N_L = 100
    steps, run twice from the same start vectors: vectors stored in FP32, then
    in FP16.  What the paper states and this test checks, for T >= 0.1:
    the deviation lies inside the backward-error envelope of rounding the
    stored iterates, an operator perturbation of norm u W (u = 2^-11, W the
    spectral width: |dE| <= u W, |dC| <= u W C / T, |dchi| <= u W chi / T),
    and it is much smaller than the random-vector error of the trace estimate
    (here at most 1% of the spread between two independent FP32 runs; the
    paper gives a ratio of about a thousand).  The paper's own run printed
    |dC| = 8e-5 and |dchi| = 1e-4, one realization; ours are logged next to
    it."""
    log("[observables] s=3/2 icosahedron, FP16 against FP32 storage")
    cl = clusters.get("icosahedron")
    T = np.geomspace(0.05, 10, 50)
    r32 = P.campaign(cl, cl.gens, 3, 100, 100, 0x5EED0004, T, storage=P.F32)
    r16 = P.campaign(cl, cl.gens, 3, 100, 100, 0x5EED0004, T, storage=P.F16)
    other = P.campaign(cl, cl.gens, 3, 100, 100, 0x5EED0014, T, storage=P.F32)   # independent chains
    assert r32["stats"]["work"] == r16["stats"]["work"]
    dC = np.abs(r16["C"] - r32["C"])
    dX = np.abs(r16["chi"] - r32["chi"])
    dE = np.abs(r16["E"] - r32["E"])
    for k in range(0, len(T), 5):
        log(f"    T={T[k]:.4f} |dE| {dE[k]:.2e} |dC| {dC[k]:.2e} |dchi| {dX[k]:.2e}  (C {r32['C'][k]:.4f} chi {r32['chi'][k]:.4f})")
    hot = T >= 0.1
    log(f"  T >= 0.1: max |dC| {dC[hot].max():.2e}  max |dchi| {dX[hot].max():.2e}  (the paper's run: 8e-5, 1e-4)")
    # spectral width: each bond's S_i.S_j has eigenvalues in [-s(s+1), s^2],
    # so W <= N_b (s(s+1) + s^2) = N_b s (2s + 1)
    u = 2.0 ** -11
    s_ = 1.5
    W = cl.nbonds * s_ * (2 * s_ + 1)
    assert np.all(dE[hot] <= u * W)
    assert np.all(dC[hot] <= u * W * r32["C"][hot] / T[hot])
    assert np.all(dX[hot] <= u * W * r32["chi"][hot] / T[hot])
    stat_C = np.abs(other["C"] - r32["C"])[hot].max()
    stat_X = np.abs(other["chi"] - r32["chi"])[hot].max()
    log(f"  statistical spread between independent FP32 runs: C {stat_C:.2e} chi {stat_X:.2e}")
    assert dC[hot].max() <= 1e-2 * stat_C and dX[hot].max() <= 1e-2 * stat_X
