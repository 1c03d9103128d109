"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Integer data (representatives, stabilizer ids, orbit search, lookup, n_Gamma,
offsets) must be bit-exact; FP64 H.V within 1e-12 relative (per column,
infinity norm); FP32 H.V within 2e-7 relative of the oracle applied to the
same FP32-rounded input (FP32 is a storage format: the kernel forms products
and sums in FP64 and rounds once on the store).
"""
import numpy as np
import pytest

from gpu_helpers import lib_block, lib_group, lib_sector, log, oracle_block, oracle_group, oracle_sector, rel_err_cols
from oracle import basis, hv
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

CASES = [  # (cluster, 2s, 2M)
    ("icosahedron", 1, 0), ("icosahedron", 1, 4), ("icosahedron", 1, 10), ("icosahedron", 1, 12),
    ("dodecahedron", 1, 0), ("dodecahedron", 1, 6),
    ("cuboctahedron", 1, 0), ("cuboctahedron", 3, 2),
    ("ring6", 1, 0), ("ring6", 2, 0), ("ring6", 2, 2),
    ("K4", 3, 0), ("dimer", 1, 0), ("square4", 1, 4), ("icosahedron", 3, 6),
]
# labels wider than 32 bits (64-bit words, 10, 12 and 16 four-bit chunks)
WIDE = [("square6x6", 1, 30), ("square6x6", 1, 28), ("dodecahedron", 3, 54), ("ring44", 1, 40), ("ring60", 1, 56)]
CASES += WIDE


@pytest.mark.parametrize("name,two_s,two_M", CASES)
def test_sector_tables_bit_exact(name, two_s, two_M):
    log(f"[sector] {name} 2s={two_s} 2M={two_M}")
    sec, _ = oracle_sector(name, two_s, two_M)
    S = lib_sector(name, two_s, two_M)
    assert S.D_M == len(sec.labels)
    assert S.n_reps == len(sec.reps)
    reps, sid, ssz = S.export()
    assert np.array_equal(reps.astype(np.int64), sec.reps)
    assert np.array_equal(sid.astype(np.int64), sec.stab_id)
    assert [len(s) for s in sec.stab_sets] == list(ssz)


@pytest.mark.parametrize("name,two_s,two_M", CASES[:10] + WIDE)
def test_orbit_search_and_lookup_bit_exact(name, two_s, two_M):
    log(f"[canon] {name} 2s={two_s} 2M={two_M}")
    cl, G, _ = oracle_group(name)
    sec, _ = oracle_sector(name, two_s, two_M)
    S = lib_sector(name, two_s, two_M)
    rng = np.random.default_rng(7)
    labs = sec.labels if len(sec.labels) <= 4000 else rng.choice(sec.labels, 4000, replace=False)
    # add out-of-sector labels (other digit sum) to check the -1 index
    d = two_s + 1
    other = np.array([0, d ** cl.N - 1], dtype=np.int64)
    labs = np.concatenate([labs, other])
    rep, h, idx = S.canonicalize(torch.from_numpy(labs.astype(np.int64)).cuda())
    rep, h, idx = rep.cpu().numpy(), h.cpu().numpy(), idx.cpu().numpy()
    orep, oh = basis.canonicalize(G, labs[:-2], cl.N, d)
    assert np.array_equal(rep[:-2], orep)
    assert np.array_equal(h[:-2], oh)
    assert np.array_equal(idx[:-2], np.searchsorted(sec.reps, orep))
    insector = [np.sum(np.array([(x // d ** k) % d for k in range(cl.N)])) * 2 - cl.N * two_s == two_M for x in other]
    for k, ok in enumerate(insector):
        if not ok:
            assert idx[-2 + k] == -1


@pytest.mark.parametrize("name,two_s,two_M", [c for c in CASES if c[0] != "square4"])
def test_block_data_and_hv_fp64(name, two_s, two_M):
    cl, G, irs = oracle_group(name)
    sec, H = oracle_sector(name, two_s, two_M)
    rng = np.random.default_rng(11)
    for gi, ir in enumerate(irs):
        log(f"[hv64] {name} 2s={two_s} 2M={two_M} irrep={gi}")
        B = oracle_block(name, two_s, two_M, gi)
        LB = lib_block(name, two_s, two_M, gi)
        assert LB.D == B.D
        ex = LB.export()
        assert np.array_equal(ex["n_gamma"].astype(np.int64), B.n_rep)
        assert np.array_equal(ex["offsets"].astype(np.int64), B.offsets)
        assert np.allclose(ex["L"], B.L_rep)
        if B.D == 0:
            X = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
            LB.apply_H(X)        # no-op on an empty block
            continue
        for nvec in (1, 3):
            X = rng.standard_normal((B.D, nvec))
            Y = LB.apply_H(torch.from_numpy(X).cuda()).cpu().numpy()
            Yref = hv.apply(B, H, X)
            assert rel_err_cols(Y, Yref) <= 1e-12, (gi, nvec)


@pytest.mark.parametrize("name,two_s,two_M,gi", [("dodecahedron", 1, 0, 8), ("icosahedron", 1, 0, 9),
                                                 ("cuboctahedron", 3, 2, 7), ("square6x6", 1, 28, 26),
                                                 ("ring60", 1, 56, 10)])
def test_hv_batched_fp32_and_modes(name, two_s, two_M, gi):
    """nvec up to 70 (two vector tiles), FP32 storage, on-the-fly mode; batched == single bitwise."""
    log(f"[hv-batch] {name} 2s={two_s} 2M={two_M} irrep={gi}")
    sec, H = oracle_sector(name, two_s, two_M)
    B = oracle_block(name, two_s, two_M, gi)
    LB = lib_block(name, two_s, two_M, gi)
    LO = lib_block(name, two_s, two_M, gi, hv_mode=P.HV_ONTHEFLY)
    assert LO.hv_mode == P.HV_ONTHEFLY and LB.hv_mode == P.HV_ENTRIES
    assert LB.hv_stats()["entry_bytes"] == 8
    # compact 6-byte entries (when |G| and the flip ids fit 15 bits): same flips, same order
    try:
        LC = lib_block(name, two_s, two_M, gi, entry_format=P.ENTRIES_COMPACT)
        assert LC.hv_stats()["entry_bytes"] == 6
    except P.FtlmError as e:
        assert e.name == "UNSUPPORTED" and name == "square6x6", e
        LC = None
    rng = np.random.default_rng(5)
    # the on-the-fly kernel keeps the irrep matrices in LDS (48 KiB for the
    # small tables); larger ones (8x8 matrices of a group of order 288) are
    # refused with UNSUPPORTED instead of running from global memory
    otf_fits = LB.group_order * LB.d_gamma ** 2 * 8 <= 40 * 1024
    for nvec in (2, 24, 70):
        X = rng.standard_normal((B.D, nvec))
        Xt = torch.from_numpy(X).cuda()
        Y = LB.apply_H(Xt)
        if LC is not None:
            assert torch.equal(LC.apply_H(Xt), Y)
        if otf_fits:
            Yo = LO.apply_H(Xt)
            assert torch.equal(Y, Yo)                    # same flips, same order
        else:
            with pytest.raises(P.FtlmError, match="UNSUPPORTED"):
                LO.apply_H(Xt)
        assert rel_err_cols(Y.cpu().numpy(), hv.apply(B, H, X)) <= 1e-12
        # batched equals one column at a time, bitwise
        for v in (0, nvec - 1):
            Yv = LB.apply_H(Xt[:, v:v + 1].contiguous())
            assert torch.equal(Yv[:, 0], Y[:, v])
        X32 = X.astype(np.float32)
        Y32 = LB.apply_H(torch.from_numpy(X32).cuda()).cpu().numpy()
        assert rel_err_cols(Y32, hv.apply(B, H, X32.astype(np.float64))) <= 2e-7
        # FP16 storage: one rounding of the FP64 result, |err| <= (2^-11 + 2^-24) |y|
        X16 = X.astype(np.float16)
        Y16 = LB.apply_H(torch.from_numpy(X16).cuda())
        assert rel_err_cols(Y16.cpu().numpy(), hv.apply(B, H, X16.astype(np.float64))) <= 2.0 ** -11 + 2.0 ** -24
        if otf_fits:
            assert torch.equal(LO.apply_H(torch.from_numpy(X16).cuda()), Y16)
    # repeated launches are bitwise identical
    X = torch.from_numpy(rng.standard_normal((B.D, 24))).cuda()
    Y1 = LB.apply_H(X)
    Y2 = LB.apply_H(X)
    assert torch.equal(Y1, Y2)


def test_hv_rows_identical_for_every_partner_row():
    """Section 2.3: the block matrix does not depend on the partner row."""
    name, two_s, two_M, gi = "icosahedron", 1, 2, 8
    log(f"[rows] {name}")
    rng = np.random.default_rng(2)
    B0 = lib_block(name, two_s, two_M, gi, row=0)
    X = torch.from_numpy(rng.standard_normal((B0.D, 4))).cuda()
    Y0 = B0.apply_H(X)
    for row in range(1, 5):
        Br = lib_block(name, two_s, two_M, gi, row=row)
        assert Br.row == row
        assert torch.equal(Br.apply_H(X), Y0)


def test_library_irreps_give_same_block_spectrum():
    """Without user_rho the library's own irreps give a similar matrix: same spectrum."""
    name, two_s, two_M = "icosahedron", 1, 0
    log(f"[own-irreps] {name}")
    _, G, irs = oracle_group(name)
    sec, H = oracle_sector(name, two_s, two_M)
    S = lib_sector(name, two_s, two_M)
    for gi in range(len(irs)):
        B = oracle_block(name, two_s, two_M, gi)
        LB = P.Block(S, gi, 0)
        M = LB.apply_H(torch.eye(LB.D, dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.allclose(M, M.T, atol=1e-12)
        ev = np.linalg.eigvalsh(M)
        evo = np.linalg.eigvalsh(hv.block_matrix(B, H))
        assert np.max(np.abs(ev - evo)) < 1e-11


def test_block_errors():
    S = lib_sector("icosahedron", 1, 0)
    with pytest.raises(P.FtlmError) as e:
        P.Block(S, 10, 0)
    assert e.value.name == "IRREP_OUT_OF_RANGE"
    with pytest.raises(P.FtlmError) as e:
        P.Block(S, 8, 5)
    assert e.value.name == "ROW_OUT_OF_RANGE"
    bad = np.tile(np.eye(2), (120, 1, 1))
    bad[5] = [[0, 1], [1, 0]]
    with pytest.raises(P.FtlmError) as e:
        P.Block(S, 0, 0, user_rho=bad)
    assert e.value.name == "BAD_RHO"
    cl = clusters.icosahedron()
    G = lib_group("icosahedron")
    broken = cl.bonds.copy()
    broken[0] = [0, 5] if tuple(broken[0]) != (0, 5) else [0, 6]
    with pytest.raises(P.FtlmError) as e:
        P.Sector(clusters.Cluster("x", 12, broken, cl.gens), G, 0, two_s=1)
    assert e.value.name == "BONDS_NOT_INVARIANT"


def test_torus_block_with_stabilizer_matrices_outside_lds():
    """The 6x6 torus at 2M = 24 has 133 stabilizer types.  With a
    4-dimensional irrep of its order-288 group, rho^T (37 KiB) and the small
    tables are staged in LDS while the V_S matrices (17 KiB more) are read
    through the caches, in the block-row kernel and in the dense-gather
    kernel of padded rows alike.  Sampled output rows, half of them of
    representatives with a non-trivial stabilizer, against the oracle's
    row-by-row evaluation (FP64, 24 vectors, label-keyed input); the padded
    launch against the block-row one."""
    from synth.vectors import label_keyed_values
    name, two_M, nvec, seed = "square6x6", 24, 24, 0x5EED0031
    cl, G, irs = oracle_group(name)
    gi = next(k for k, ir in enumerate(irs) if ir.dim == 4)
    S = lib_sector(name, 1, two_M)
    log(f"[parity] {name} 2M={two_M} irrep {gi} (d=4): {S.n_reps} reps, {S.n_stab} stabilizer types")
    assert S.n_stab * 16 * 8 + 288 * 16 * 8 > 48 * 1024          # V_S does not fit next to rho^T
    B = P.Block(S, gi, 0, user_rho=irs[gi].rho)
    ex = B.export()
    reps, counts, offs = ex["reps"], ex["n_gamma"].astype(np.int64), ex["offsets"].astype(np.int64)
    _, sid, ssz = S.export()
    X = np.zeros((B.D, nvec))
    Xp = np.zeros((len(reps) * 4, nvec))
    vv = np.arange(nvec, dtype=np.uint64)[None, :]
    for i in np.nonzero(counts)[0]:
        vals = label_keyed_values(seed, reps[i], np.arange(counts[i], dtype=np.uint64)[:, None], vv)
        X[offs[i]:offs[i] + counts[i]] = vals
        Xp[4 * i:4 * i + counts[i]] = vals
    Y = B.apply_H(torch.from_numpy(X).cuda()).cpu().numpy()
    Yp, info = B.apply_H_ex(torch.from_numpy(Xp).cuda(), layout=P.LAYOUT_PADDED)
    assert info["adjacent_columns"] == 1
    Yp = Yp.cpu().numpy()
    Yu = np.concatenate([Yp[4 * i:4 * i + counts[i]] for i in np.nonzero(counts)[0]])
    assert rel_err_cols(Yu, Y) <= 1e-12
    rng = np.random.default_rng(31)
    active = np.nonzero(counts)[0]
    nontriv = active[ssz[sid[active]] > 1]
    assert len(nontriv) >= 6
    pick = np.concatenate([rng.choice(active, 6, replace=False), rng.choice(nontriv, 6, replace=False)])

    def xfun(rlab, n):
        return label_keyed_values(seed, np.uint64(rlab), np.arange(n, dtype=np.uint64)[:, None], vv)

    rows = hv.sampled_rows(G, irs[gi], 0, cl.N, 1, cl.bonds, cl.J, reps[pick].astype(np.int64), xfun, nvec)
    scale = max(np.abs(y).max() for y in rows)
    for i, yref in zip(pick, rows):
        got = Y[offs[i]:offs[i] + counts[i]]
        assert np.max(np.abs(got - yref)) <= 1e-12 * scale, (i, np.max(np.abs(got - yref)) / scale)
