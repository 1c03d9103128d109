"""Full-size parity on the s=1/2 icosidodecahedron, M=0 (D_M = 155,117,520).

The representative table is checked without a CPU enumeration: strictly
increasing, every label in the sector, a random sample verified as orbit minima
by the oracle's brute-force search, stabilizer sizes of the sample equal to the
oracle's, and the count equal to the oracle's character-formula A_g dimension;
together these pin the table.  The H_g block (D = 6,465,762) is applied in the
launch configuration the benchmark times (24 vectors, FP32 storage) and in
FP64, to inputs whose values depend only on (representative label, k, column);
sampled output rows are compared with the oracle's row-by-row evaluation.
"""
from math import comb

import numpy as np
import pytest

from gpu_helpers import log
from oracle import basis, counting, group, hv, irreps
from synth import clusters
from synth.vectors import label_keyed_values, label_keyed_values_torch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

SEED = 0x5EED0003


@pytest.fixture(scope="module")
def icosid():
    cl = clusters.icosidodecahedron()
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    LG = P.Group(cl.N, cl.gens)
    log("[scale] building the M=0 sector on the GPU")
    S = P.Sector(cl, LG, 0, two_s=1)
    return cl, G, irs, S


def test_representative_table_at_scale(icosid):
    cl, G, irs, S = icosid
    assert S.D_M == comb(30, 15)
    dims = counting.block_dims_by_characters(G, irs, 1, 0)
    assert S.n_reps == dims[0] == 1295266
    reps, sid, ssz = S.export()
    r = reps.astype(np.int64)
    assert np.all(np.diff(r) > 0)
    pc = np.zeros(len(r), dtype=np.int64)
    x = r.copy()
    for _ in range(30):
        pc += x & 1
        x >>= 1
    assert np.all(pc == 15)
    rng = np.random.default_rng(1)
    pick = rng.choice(len(r), 3000, replace=False)
    canon, h = basis.canonicalize(G, r[pick], cl.N, 2)
    assert np.array_equal(canon, r[pick])
    for i in pick[:300]:
        assert ssz[sid[i]] == len(basis.stabilizer(G, int(r[i]), cl.N, 2))


def _label_keyed(reps, counts, nvec, dtype):
    """X[row, v] = label_keyed_values(SEED, rep label, k, v), built in chunks of representatives."""
    out = np.empty((int(counts.sum()), nvec), dtype=dtype)
    pos = 0
    vv = np.arange(nvec, dtype=np.uint64)[None, :]
    for s in range(0, len(reps), 200000):
        lab = np.repeat(reps[s:s + 200000], counts[s:s + 200000])
        c = counts[s:s + 200000]
        kk = np.arange(len(lab), dtype=np.int64) - np.repeat(np.cumsum(c) - c, c)
        out[pos:pos + len(lab)] = label_keyed_values(SEED, lab[:, None], kk[:, None].astype(np.uint64), vv)
        pos += len(lab)
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("nvec,storage", [(24, "f32"), (2, "f64")])
def test_hg_block_sampled_rows(icosid, nvec, storage):
    cl, G, irs, S = icosid
    gi = 8
    ir = irs[gi]
    log(f"[scale] H_g block nvec={nvec} {storage}")
    B = P.Block(S, gi, 0, user_rho=ir.rho)
    assert B.D == 6465762
    ex = B.export()
    reps = ex["reps"]
    counts = ex["n_gamma"].astype(np.int64)
    dt = np.float32 if storage == "f32" else np.float64
    X = _label_keyed(reps, counts, nvec, dt)
    Xt = torch.from_numpy(X).cuda()
    Y = B.apply_H(Xt).cpu().numpy()
    del Xt
    rng = np.random.default_rng(2)
    active = np.nonzero(counts)[0]
    pick = rng.choice(active, 24, replace=False)

    def xfun(rlab, n):
        vals = label_keyed_values(SEED, np.full((n, 1), rlab, dtype=np.uint64),
                                  np.arange(n, dtype=np.uint64)[:, None], np.arange(nvec, dtype=np.uint64)[None, :])
        return vals.astype(dt).astype(np.float64)

    rows = hv.sampled_rows(G, ir, 0, cl.N, 1, cl.bonds, cl.J, reps[pick].astype(np.int64), xfun, nvec)
    scale = max(np.abs(y).max() for y in rows)
    tol = 2e-7 if storage == "f32" else 1e-12
    for i, yref in zip(pick, rows):
        o = int(ex["offsets"][i])
        got = Y[o:o + counts[i]].astype(np.float64)
        assert np.max(np.abs(got - yref)) <= tol * scale, (i, np.max(np.abs(got - yref)) / scale)


@pytest.mark.timeout(900)
def test_hg_bench_launch_sampled_rows(icosid):
    """The launch the benchmark times, element by element at full size: padded
    rows, 24 FP32 columns, 8 lanes x 3 adjacent columns per representative,
    the Lanczos epilogue Y <- s H X - b Y.  Sampled representatives include
    the first and last, those at workgroup boundaries (32 representatives
    per workgroup) and at the grid stride (8192 workgroups x 32), and random
    ones; each sampled output row is checked against the oracle's row-by-row
    evaluation of s Psi^H H Psi X - b Y0, and the padding rows stay zero.
    The FP64 sums X . Y equal a float64 sum of the returned Y."""
    cl, G, irs, S = icosid
    gi, nvec, d = 8, 24, 5
    ir = irs[gi]
    B = P.Block(S, gi, 0, user_rho=ir.rho)
    reps = B.export()["reps"]
    n_reps = len(reps)
    log("[scale] bench launch: padded input on the device")
    lab = torch.from_numpy(reps.view(np.int64)).cuda()
    v = torch.arange(nvec, dtype=torch.int64, device="cuda")[None, :]
    Xp = torch.zeros((n_reps * d, nvec), dtype=torch.float32, device="cuda")
    Y0 = torch.zeros_like(Xp)
    # rows k >= n_Gamma(i) are the layout's padding and stay zero (the oracle's rows below
    # have its own n_Gamma, so a different count fails the comparison)
    ng = torch.from_numpy(B.export()["n_gamma"].astype(np.int64)).cuda()
    for k in range(d):
        live = ng > k
        vals = label_keyed_values_torch(SEED, lab[:, None], torch.full_like(lab, k)[:, None], v)
        vals0 = label_keyed_values_torch(SEED + 1, lab[:, None], torch.full_like(lab, k)[:, None], v)
        Xp[k::d] = torch.where(live[:, None], vals, 0.0).to(torch.float32)
        Y0[k::d] = torch.where(live[:, None], vals0, 0.0).to(torch.float32)
    rng = np.random.default_rng(8)
    sb = np.stack([rng.uniform(0.5, 2.0, nvec), rng.uniform(-1.0, 1.0, nvec)], axis=1)
    scale = torch.from_numpy(sb).cuda()
    dots = torch.zeros(nvec, dtype=torch.float64, device="cuda")
    Y, info = B.apply_H_ex(Xp, Y0.clone(), layout=P.LAYOUT_PADDED, lanes=8, scale=scale, dots=dots)
    torch.cuda.synchronize()
    assert info["adjacent_columns"] == 1 and info["lanes_used"] == 8
    want = (Xp.double() * Y.double()).sum(0)
    assert torch.allclose(dots, want, rtol=1e-10, atol=0)
    stride = 8192 * 32
    edges = [0, 1, 31, 32, 33, 63, 64, stride - 1, stride, stride + 1, 2 * stride - 1, 2 * stride,
             4 * stride, n_reps - 33, n_reps - 32, n_reps - 2, n_reps - 1]
    pick = np.unique(np.concatenate([edges, rng.choice(n_reps, 12, replace=False)]))
    ngh = ng.cpu().numpy()
    pick = pick[ngh[pick] > 0]
    Yh = Y.cpu().numpy()
    Y0h = Y0.cpu().numpy()
    del Xp, Y, Y0

    def xfun(rlab, n):
        vals = label_keyed_values(SEED, np.full((n, 1), rlab, dtype=np.uint64),
                                  np.arange(n, dtype=np.uint64)[:, None], np.arange(nvec, dtype=np.uint64)[None, :])
        return vals.astype(np.float32).astype(np.float64)

    log(f"[scale] bench launch: {len(pick)} sampled representatives against the oracle")
    rows = hv.sampled_rows(G, ir, 0, cl.N, 1, cl.bonds, cl.J, reps[pick].astype(np.int64), xfun, nvec)
    ref = [sb[:, 0] * y - sb[:, 1] * Y0h[i * d:i * d + len(y)].astype(np.float64) for i, y in zip(pick, rows)]
    scl = max(np.abs(r).max() for r in ref)
    for i, yref in zip(pick, ref):
        n = len(yref)
        got = Yh[i * d:i * d + n].astype(np.float64)
        assert np.max(np.abs(got - yref)) <= 2e-7 * scl, (i, np.max(np.abs(got - yref)) / scl)
        assert not np.any(Yh[i * d + n:(i + 1) * d]), i
