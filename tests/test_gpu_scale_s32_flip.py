"""Full-size parity of the spin-flip resolution on the s=3/2 dodecahedron, M=0.

The M = 0 sector (D_M = 86,981,744,944) resolved by G x Z2: the representative
count and the H_g^+ block dimension (1,812,277,727; with H_g^- it adds up to
the G-only H_g block) from the oracle's character formula over G x Z2,
sampled representatives verified as G x Z2 orbit minima by brute force, and
sampled rows of H.V on H_g^+ (2 vectors, FP32 storage) against the oracle's
row-by-row evaluation on a label-keyed input generated on the device.  Runs in
a module of its own so that the G-only sector of the other full-size module
is freed first.
"""
import gc

import numpy as np
import pytest

from gpu_helpers import log
from oracle import basis, counting, group, hv, irreps
from synth import clusters
from synth.vectors import label_keyed_values, label_keyed_values_torch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

SEED = 0x5EED0005
NVEC = 2


@pytest.fixture(scope="module")
def dodeca32():
    gc.collect()
    torch.cuda.empty_cache()
    cl = clusters.get("dodecahedron")
    G = group.close(cl.gens, cl.N)
    irs = irreps.compute_irreps(G)
    return cl, G, irs, None


@pytest.mark.timeout(900)
def test_spin_flip_sector_and_hg_plus_rows_s32(dodeca32):
    """The same M = 0 sector resolved by the spin flip (G x Z2): representative
    count and H_g^+ dimension from the character formula over G x Z2, sampled
    orbit minima, and sampled rows of H.V on H_g^+ against the oracle."""
    from oracle import spinflip
    cl, G, irs, _ = dodeca32
    G2 = spinflip.FlipGroup(G)
    irs2 = spinflip.flip_irreps(irs)
    dims2 = counting.block_dims_by_characters(G2, irs2, 3, 0)
    LG = P.Group(cl.N, cl.gens)
    log("[scale32] building the spin-flip M=0 sector")
    SZ = P.Sector(cl, LG, 0, two_s=3, spin_flip=True)
    assert SZ.n_reps == dims2[0]
    gi2 = 16                                               # H_g^+
    B = P.Block(SZ, gi2, 0, user_rho=irs[8].rho)
    assert B.D == dims2[gi2] and dims2[16] + dims2[17] == 3624380734
    ex = B.export()
    reps = ex["reps"]
    counts = ex["n_gamma"].astype(np.int64)
    offsets = ex["offsets"].astype(np.int64)
    del ex
    rng = np.random.default_rng(6)
    pick = rng.choice(len(reps), 1000, replace=False)
    canon, _ = basis.canonicalize(G2, reps[pick].astype(np.int64), cl.N, 4)
    assert np.array_equal(canon, reps[pick].astype(np.int64))
    X = torch.empty((B.D, NVEC), dtype=torch.float32, device="cuda")
    v = torch.arange(NVEC, dtype=torch.int64, device="cuda")[None, :]
    step = 20_000_000
    for s in range(0, len(reps), step):
        lab = torch.from_numpy(reps[s:s + step].view(np.int64)).cuda()
        c = torch.from_numpy(counts[s:s + step]).cuda()
        rows = torch.repeat_interleave(lab, c)
        first = torch.repeat_interleave(torch.cumsum(c, 0) - c, c)
        kk = torch.arange(rows.numel(), dtype=torch.int64, device="cuda") - first
        o = int(offsets[s])
        X[o:o + rows.numel()] = label_keyed_values_torch(SEED, rows[:, None], kk[:, None], v).to(torch.float32)
        del lab, c, rows, first, kk
    Y = B.apply_H(X)
    torch.cuda.synchronize()
    del X
    active = np.nonzero(counts)[0]
    pick = rng.choice(active, 12, replace=False)

    def xfun(rlab, n):
        vals = label_keyed_values(SEED, np.full((n, 1), rlab, dtype=np.uint64),
                                  np.arange(n, dtype=np.uint64)[:, None], np.arange(NVEC, dtype=np.uint64)[None, :])
        return vals.astype(np.float32).astype(np.float64)

    rows_ref = hv.sampled_rows(G2, irs2[gi2], 0, cl.N, 3, cl.bonds, cl.J, reps[pick].astype(np.int64), xfun, NVEC)
    scale = max(np.abs(y).max() for y in rows_ref)
    for i, yref in zip(pick, rows_ref):
        o = int(offsets[i])
        got = Y[o:o + counts[i]].double().cpu().numpy()
        assert np.max(np.abs(got - yref)) <= 2e-7 * scale, (i, np.max(np.abs(got - yref)) / scale)
    del Y, B, SZ
