"""The allocation-free H.V entry point (ftlm_apply_H_ex_noalloc) against the
allocating one (ftlm_apply_H_ex): two calls in a row on one GPU, the second
with a smaller input, each equal bit for bit (the same kernels and the same
fixed summation order; only where the partial sums live differs), and a
call that would need more than the static scratch is refused."""
import numpy as np
import pytest

from gpu_helpers import lib_block, log, oracle_group

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")


def _pair(LB, nvec, tdt, layout, seed):
    rows = LB.D_pad if layout == P.LAYOUT_PADDED else LB.D
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.rand((rows, nvec), generator=g, dtype=torch.float64).to(tdt).cuda()
    Y0 = torch.rand((rows, nvec), generator=g, dtype=torch.float64).to(tdt).cuda()
    if layout == P.LAYOUT_PADDED:
        # padding rows (k >= n_Gamma of a representative) hold zeros in X
        ex = LB.export()
        d = LB.d_gamma
        keep = np.zeros(rows, dtype=bool)
        for i, n in enumerate(ex["n_gamma"]):
            keep[i * d:i * d + int(n)] = True
        m = torch.from_numpy(keep).cuda()[:, None]
        X = X * m
        Y0 = Y0 * m
    sb = torch.rand((nvec, 2), generator=g, dtype=torch.float64).cuda() + 0.5
    outs = []
    for noalloc in (False, True):
        Y = Y0.clone()
        dots = torch.full((nvec,), np.nan, dtype=torch.float64, device="cuda")
        Y, info = LB.apply_H_ex(X, Y, layout=layout, scale=sb, dots=dots, shift=0.25, noalloc=noalloc)
        torch.cuda.synchronize()
        outs.append((Y.cpu(), dots.cpu(), info))
    return outs


def test_noalloc_equals_allocating_entry_point_twice():
    log("[noalloc] two calls, the second smaller")
    big = lib_block("dodecahedron", 1, 0, 8)                    # 1648 representatives, d = 5
    (Ya, da, ia), (Yb, db, ib) = _pair(big, 24, torch.float32, P.LAYOUT_PADDED, 1)
    assert ia == ib and ia["adjacent_columns"] == 1
    assert torch.equal(Ya, Yb) and torch.equal(da, db)
    assert torch.isfinite(da).all()
    small = lib_block("icosahedron", 1, 0, 8)                   # 18 representatives
    (Ya, da, ia), (Yb, db, ib) = _pair(small, 6, torch.float64, P.LAYOUT_BLOCK, 2)
    assert ia == ib
    assert torch.equal(Ya, Yb) and torch.equal(da, db)
    assert torch.isfinite(da).all()


def test_noalloc_refuses_more_than_its_scratch():
    LB = lib_block("dodecahedron", 1, 0, 8)
    nvec = 2048                                                  # 412 workgroups x 2048 > 8192 x 64
    X = torch.zeros((LB.D, nvec), dtype=torch.float64, device="cuda")
    sb = torch.ones((nvec, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        LB.apply_H_ex(X, torch.zeros_like(X), layout=P.LAYOUT_BLOCK, scale=sb, noalloc=True)
    # without the epilogue there is no scratch: the same call is fine
    LB.apply_H_ex(X, torch.zeros_like(X), layout=P.LAYOUT_BLOCK, noalloc=True)
