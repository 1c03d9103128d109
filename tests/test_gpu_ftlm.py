"""GPU parity of the FTLM stage: batched Lanczos coefficients, Ritz data and E, C, chi.

The oracle draws the same SplitMix64 start vectors with its own generator and
runs its own FP64 Lanczos on Psi^H H Psi.  alpha/beta are compared only over the
first steps (before any Ritz value converges, after which two correct FP64
runs with different summation orders drift apart); the thermal observables
are compared on the whole temperature grid.
"""
import numpy as np
import pytest

from gpu_helpers import lib_block, log, oracle_block, oracle_group, oracle_sector
from oracle import ftlm as oftlm
from oracle import hv
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

T_GRID = np.geomspace(0.05, 10, 50)


def test_lanczos_coefficients_fp64():
    name, two_s, two_M, gi = "dodecahedron", 1, 0, 8
    log(f"[lanczos] {name} irrep {gi}")
    sec, H = oracle_sector(name, two_s, two_M)
    B = oracle_block(name, two_s, two_M, gi)
    LB = lib_block(name, two_s, two_M, gi)
    Hb = (B.Psi.T @ H @ B.Psi).tocsr()
    for dist, dname in ((P.RADEMACHER, "rademacher"), (P.GAUSSIAN, "gaussian")):
        a, b, n = LB.ftlm(3, 40, 99, storage=P.F64, dist=dist)
        assert np.all(n == 40)
        for r in range(3):
            v0 = oftlm.start_vector(B.D, 99, two_M, gi, 0, r, dname)
            oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, 40)
            assert np.max(np.abs(a[r, :15] - oa[:15])) < 1e-10 * np.max(np.abs(oa))
            assert np.max(np.abs(b[r, :15] - ob[:15])) < 1e-10 * np.max(np.abs(ob))
        # deterministic: a second run is bitwise identical
        a2, b2, n2 = LB.ftlm(3, 40, 99, storage=P.F64, dist=dist)
        assert np.array_equal(a, a2) and np.array_equal(b, b2)


def test_small_and_empty_blocks():
    # icosahedron M=5/2... all blocks of 2M=10 have D <= 1; A_u at 2M=6 is empty
    log("[lanczos] tiny blocks")
    for two_M, gi in ((10, 0), (10, 4), (6, 1)):
        B = oracle_block("icosahedron", 1, two_M, gi)
        LB = lib_block("icosahedron", 1, two_M, gi)
        a, b, n = LB.ftlm(2, 30, 5, storage=P.F64)
        assert np.all(n == min(B.D, 30))
        if B.D == 1:
            _, H = oracle_sector("icosahedron", 1, two_M)
            assert np.allclose(a[:, 0], hv.block_matrix(B, H)[0, 0], atol=1e-14)


def _ftlm_all_blocks(name, two_s, R, steps, seed, storage, dist):
    cl, G, irs = oracle_group(name)
    lib_blocks, ora_blocks = [], []
    for two_M in range((cl.N * two_s) % 2, cl.N * two_s + 1, 2):
        sec, H = oracle_sector(name, two_s, two_M)
        for gi, ir in enumerate(irs):
            B = oracle_block(name, two_s, two_M, gi)
            if B.D == 0:
                continue
            LB = lib_block(name, two_s, two_M, gi)
            a, b, n = LB.ftlm(R, steps, seed, storage=storage, dist=dist)
            ths, ws = P.ritz_from_run(a, b, n)
            lib_blocks.append(dict(two_M=two_M, d_gamma=ir.dim, D=B.D, thetas=ths, weights=ws))
            Hb = hv.block_matrix(B, H)
            oth, ow = [], []
            for r in range(R):
                v0 = oftlm.start_vector(B.D, seed, two_M, gi, 0, r, "rademacher" if dist == P.RADEMACHER else "gaussian")
                t, w = oftlm.ritz(*oftlm.lanczos(lambda x: Hb @ x, v0, steps))
                oth.append(t)
                ow.append(w)
            ora_blocks.append(oftlm.BlockRitz(two_M, ir.dim, B.D, oth, ow))
    return lib_blocks, ora_blocks


def _rel(x, ref):
    return np.abs(x - ref) / np.abs(ref)


@pytest.mark.parametrize("storage,tol", [(0, 1e-9), (1, 1e-6)])
def test_observables_icosahedron_all_sectors(storage, tol):
    """Icosahedron s=1/2, all M >= 0, all 10 irreps, R=4 Rademacher, 30 steps (per-T relative error)."""
    log(f"[ftlm] icosahedron storage={storage}")
    lib_blocks, ora_blocks = _ftlm_all_blocks("icosahedron", 1, 4, 30, 0x5EED0001, storage, P.RADEMACHER)
    E, C, chi, lz = P.observables(lib_blocks, T_GRID)
    Eo, Co, chio, lzo = oftlm.observables(ora_blocks, T_GRID, with_logZ=True)
    eE, eC, eX = _rel(E, Eo), _rel(C, Co), _rel(chi, chio)
    log(f"  max rel err E {eE.max():.2e} C {eC.max():.2e} chi {eX.max():.2e}")
    assert eE.max() < tol and eC.max() < tol and eX.max() < tol
    # exact high-temperature limits of the aggregate (Section 4.1)
    E2, C2, chi2, lz2 = P.observables(lib_blocks, np.array([1e9]))
    assert abs(np.exp(lz2[0]) / 2 ** 12 - 1) < 1e-6
    assert abs(1e9 * chi2[0] / (12 * 0.75 / 3) - 1) < 1e-6


def test_observables_icosahedron_fp16_storage():
    """FP16 vector storage (FP64 arithmetic, per-chain power-of-two scale): the
    error of E, C, chi against the FP64 oracle, per temperature."""
    log("[ftlm] icosahedron storage=f16")
    lib_blocks, ora_blocks = _ftlm_all_blocks("icosahedron", 1, 4, 30, 0x5EED0001, P.F16, P.RADEMACHER)
    E, C, chi, lz = P.observables(lib_blocks, T_GRID)
    Eo, Co, chio, lzo = oftlm.observables(ora_blocks, T_GRID, with_logZ=True)
    eE, eC, eX = _rel(E, Eo), _rel(C, Co), _rel(chi, chio)
    for k in range(0, len(T_GRID), 7):
        log(f"  T={T_GRID[k]:.3f} rel err E {eE[k]:.2e} C {eC[k]:.2e} chi {eX[k]:.2e}")
    log(f"  max rel err E {eE.max():.2e} C {eC.max():.2e} chi {eX.max():.2e}")
    # Bound from the arithmetic: each stored element carries a relative error of
    # at most u = 2^-11, which moves Ritz values by ~ u W (W = spectral width);
    # E moves by that much, and the Boltzmann weights of C and chi by a relative
    # u W / T.
    u = 2.0 ** -11
    th = np.concatenate([np.concatenate(b.thetas) for b in ora_blocks])
    W = th.max() - th.min()
    assert np.all(np.abs(E - Eo) <= u * W)
    assert np.all(eC <= u * W / T_GRID) and np.all(eX <= u * W / T_GRID)


def test_padded_layout_against_oracle_and_block_layout():
    """The padded vector layout (d_Gamma rows per representative, read without
    the target's row offset) gives the oracle's coefficients; forced on a
    block where it adds padding rows, with FP64 and FP32 storage."""
    name, two_s, two_M, gi = "dodecahedron", 1, 0, 8
    log("[lanczos] padded layout")
    sec, H = oracle_sector(name, two_s, two_M)
    B = oracle_block(name, two_s, two_M, gi)
    Hb = (B.Psi.T @ H @ B.Psi).tocsr()
    _, _, irs = oracle_group(name)
    S = lib_block(name, two_s, two_M, gi).sector
    LP = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_PADDED)
    LB = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_BLOCK)
    assert S.n_reps * 5 > LP.D          # the padded layout has zero rows here
    a, b, n, info = LP.ftlm(3, 40, 99, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_PADDED and info["rows"] == S.n_reps * 5 and info["hv_launches"] == 40
    assert info["hv_ms"] > 0
    for r in range(3):
        v0 = oftlm.start_vector(B.D, 99, two_M, gi, 0, r, "rademacher")
        oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, 40)
        assert np.max(np.abs(a[r, :15] - oa[:15])) < 1e-10 * np.max(np.abs(oa))
        assert np.max(np.abs(b[r, :15] - ob[:15])) < 1e-10 * np.max(np.abs(ob))
    a1, b1, n1, info1 = LB.ftlm(3, 40, 99, storage=P.F64, info=True)
    assert info1["layout"] == P.LAYOUT_BLOCK and info1["rows"] == LB.D
    assert np.max(np.abs(a[:, :15] - a1[:, :15])) < 1e-12 * np.max(np.abs(a1))
    # FP32 storage: the stored rows are the same numbers, only FP64 reduction order differs
    a32, b32, _ = LP.ftlm(3, 30, 7, storage=P.F32)
    a32b, b32b, _ = LB.ftlm(3, 30, 7, storage=P.F32)
    assert np.max(np.abs(a32[:, :15] - a32b[:, :15])) < 1e-6 * np.max(np.abs(a32b))
    assert np.max(np.abs(b32[:, :15] - b32b[:, :15])) < 1e-6 * np.max(np.abs(b32b))


@pytest.mark.parametrize("R", [6, 8, 24])
def test_adjacent_column_kernel_against_oracle(R):
    """Padded rows with d_Gamma equal to its dimension bucket and R filling the
    column tiles (R = 6: 2 lanes x 3 columns, 8: 4 x 2, 24: 8 x 3) take the
    kernel whose lanes hold adjacent columns.  Irrep dimensions 1, 3, 4 and 5:
    coefficients of every chain equal the block layout's (the interleaved
    kernel) and, for two chains, the oracle's Lanczos on the explicit block;
    FP32 and FP16 storage against the block layout at their rounding level."""
    name, two_s, two_M = "dodecahedron", 1, 0
    _, _, irs = oracle_group(name)
    sec, H = oracle_sector(name, two_s, two_M)
    S = lib_block(name, two_s, two_M, 8).sector
    seen = set()
    for gi, ir in enumerate(irs):
        d = ir.rho.shape[1]
        if d in seen or d not in (1, 3, 4, 5):
            continue
        seen.add(d)
        log(f"[lanczos] adjacent columns R={R} irrep {gi} (d={d})")
        LP = P.Block(S, gi, 0, user_rho=ir.rho, layout=P.LAYOUT_PADDED)
        LB = P.Block(S, gi, 0, user_rho=ir.rho, layout=P.LAYOUT_BLOCK)
        if LP.D == 0:
            continue
        a, b, n, info = LP.ftlm(R, 24, 31, storage=P.F64, info=True)
        assert info["layout"] == P.LAYOUT_PADDED
        a1, b1, n1 = LB.ftlm(R, 24, 31, storage=P.F64)
        k = int(min(n.min(), n1.min(), 12))
        assert np.max(np.abs(a[:, :k] - a1[:, :k])) < 1e-12 * np.max(np.abs(a1[:, :k]))
        assert np.max(np.abs(b[:, :k] - b1[:, :k])) < 1e-12 * np.max(np.abs(b1[:, :k]))
        B = oracle_block(name, two_s, two_M, gi)
        Hb = (B.Psi.T @ H @ B.Psi).tocsr()
        for r in (0, R - 1):
            v0 = oftlm.start_vector(B.D, 31, two_M, gi, 0, r, "rademacher")
            oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, 24)
            kk = min(k, len(oa))
            assert np.max(np.abs(a[r, :kk] - oa[:kk])) < 1e-10 * np.max(np.abs(oa[:kk]))
        # FP32 storage on the same layout: the stored rows round the same way
        a32, _, _ = LP.ftlm(R, 12, 31, storage=P.F32)
        a32b, _, _ = LB.ftlm(R, 12, 31, storage=P.F32)
        assert np.max(np.abs(a32[:, :8] - a32b[:, :8])) < 1e-5 * np.max(np.abs(a32b[:, :8]))
        # FP16 storage: a column taken from the wrong chain would differ at the percent level
        a16, _, _ = LP.ftlm(R, 8, 31, storage=P.F16)
        a16b, _, _ = LB.ftlm(R, 8, 31, storage=P.F16)
        assert np.max(np.abs(a16[:, :6] - a16b[:, :6])) < 1e-3 * np.max(np.abs(a16b[:, :6]))
    assert seen == {1, 3, 4, 5}


@pytest.mark.timeout(600)
def test_auto_layout_at_scale_matches_block_layout():
    """On the icosidodecahedron H_g block (D = 6,465,762) AUTO picks the padded
    layout (0.16% extra rows); its FP64 coefficients agree with the block
    layout's over the first steps, and so do those of the benchmark's
    configuration (24 Gaussian chains, FP32 storage) to FP32 rounding."""
    log("[lanczos] auto layout at scale")
    cl = clusters.get("icosidodecahedron")
    G = P.Group(cl.N, cl.gens)
    S = P.Sector(cl, G, 0, two_s=1)
    BA = P.Block(S, 8, 0)
    BB = P.Block(S, 8, 0, layout=P.LAYOUT_BLOCK)
    a, b, n, info = BA.ftlm(4, 20, 3, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_PADDED and info["rows"] == 1295266 * 5
    a1, b1, n1, info1 = BB.ftlm(4, 20, 3, storage=P.F64, info=True)
    assert info1["layout"] == P.LAYOUT_BLOCK and info1["rows"] == 6465762
    assert np.max(np.abs(a - a1)) < 1e-11 * np.max(np.abs(a1))
    assert np.max(np.abs(b - b1)) < 1e-11 * np.max(np.abs(b1))
    # the benchmark's launch configuration: 24 Gaussian chains in FP32 storage
    # (padded rows, adjacent columns per lane) against the block layout
    log("[lanczos] bench configuration, padded against block rows")
    a, b, n, info = BA.ftlm(24, 6, 0x5EED0003, storage=P.F32, dist=P.GAUSSIAN, info=True)
    a1, b1, n1, info1 = BB.ftlm(24, 6, 0x5EED0003, storage=P.F32, dist=P.GAUSSIAN, info=True)
    assert info["layout"] == P.LAYOUT_PADDED and info1["layout"] == P.LAYOUT_BLOCK
    assert np.max(np.abs(a - a1)) < 1e-6 * np.max(np.abs(a1))
    assert np.max(np.abs(b - b1)) < 1e-6 * np.max(np.abs(b1))


def test_graph_replayed_steps_equal_direct_launches():
    """On a non-default stream the Lanczos steps run as replays of one captured
    two-step graph; on the default stream (and when timing is requested) the
    kernels are launched directly.  Every graph run, with other device work and
    synchronizations between them, gives the direct run's coefficients bit for bit."""
    log("[lanczos] graph replays")
    s = torch.cuda.Stream()
    for name, two_s, two_M, gi, R, steps, st in (("dodecahedron", 1, 0, 8, 5, 41, P.F64),
                                                 ("icosahedron", 1, 0, 8, 3, 30, P.F32),
                                                 ("cuboctahedron", 3, 2, 7, 4, 37, P.F32)):
        LB = lib_block(name, two_s, two_M, gi)
        a0, b0, n0 = LB.ftlm(R, steps, 123, storage=st)                      # default stream: direct
        a1, b1, n1, info = LB.ftlm(R, steps, 123, storage=st, stream=s, info=True)  # timed: direct
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1)
        for rep in range(3):
            a2, b2, n2 = LB.ftlm(R, steps, 123, storage=st, stream=s)          # graph replays
            assert np.array_equal(n0, n2) and np.array_equal(a0, a2) and np.array_equal(b0, b2), (name, rep)
            X = torch.randn((LB.D, 3), dtype=torch.float64, device="cuda")
            LB.apply_H(X)                                                    # other work in between
            torch.cuda.synchronize()
