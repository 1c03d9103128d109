"""Element-wise parity of the H.V launches that the Lanczos run makes.

``ftlm_apply_H_ex`` exposes the padded row layout (d_Gamma rows per
representative) and the fused first half of a Lanczos step, so the kernel
instantiation that ``ftlm_run`` uses on large blocks (lanes holding adjacent
columns, the dense gather, the epilogue) can be compared with the oracle's
Psi^H H Psi X row by row (paper Eq. 15, Section 3).  Inputs are seeded; the
oracle's own offsets and n_Gamma place block rows in the padded layout, so no
value read from the library enters the reference.  Tolerances per column:
FP64 1e-12, FP32 2e-7 (one rounding of an FP64 result, against the oracle
applied to the FP32-rounded input), FP16 2^-11 + 2^-24.
"""
import numpy as np
import pytest

from gpu_helpers import log, oracle_block, oracle_group, oracle_sector, rel_err_cols
from oracle import hv
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

# one (cluster, 2s, 2M, irrep) per kernel dimension bucket 1..6
BUCKETS = [("dodecahedron", 1, 0, 0), ("cuboctahedron", 2, 0, 4), ("dodecahedron", 1, 0, 2),
           ("dodecahedron", 1, 0, 6), ("dodecahedron", 1, 0, 8), ("petersen", 3, 0, 6)]
TOL = {P.F64: 1e-12, P.F32: 2e-7, P.F16: 2.0 ** -11 + 2.0 ** -24}
NP = {P.F64: np.float64, P.F32: np.float32, P.F16: np.float16}
TT = {P.F64: torch.float64, P.F32: torch.float32, P.F16: torch.float16}


def _blocks(name, two_s, two_M, gi):
    _, _, irs = oracle_group(name)
    B = oracle_block(name, two_s, two_M, gi)
    sec, H = oracle_sector(name, two_s, two_M)
    cl = clusters.get(name)
    LG = P.Group(cl.N, cl.gens)
    S = P.Sector(cl, LG, two_M, two_s=two_s)
    LB = P.Block(S, gi, 0, user_rho=irs[gi].rho)
    assert LB.D == B.D and LB.n_reps == len(sec.reps) and LB.d_gamma == irs[gi].dim
    return B, H, LB, (LG, S)


def _to_padded(B, X):
    """Padded rows from block rows, placed by the oracle's offsets and n_Gamma."""
    d = B.irrep.dim
    n_reps = len(B.sec.reps)
    Xp = np.zeros((n_reps * d, X.shape[1]), dtype=X.dtype)
    for i in np.nonzero(B.n_rep)[0]:
        o, n = int(B.offsets[i]), int(B.n_rep[i])
        Xp[i * d:i * d + n] = X[o:o + n]
    return Xp


def _from_padded(B, Yp):
    d = B.irrep.dim
    rows = np.concatenate([np.arange(i * d, i * d + int(B.n_rep[i])) for i in np.nonzero(B.n_rep)[0]])
    pad_rows = np.setdiff1d(np.arange(Yp.shape[0]), rows)
    return Yp[rows], Yp[pad_rows]


@pytest.mark.parametrize("bucket", range(6))
def test_padded_adjacent_column_kernel_against_oracle(bucket):
    """Every dimension bucket 1..6, R = 6, 8, 24 (column tiles of 2x3, 4x2 and
    8x3 lanes x columns), FP64, FP32 and FP16: the launch takes the kernel with
    adjacent columns per lane, and every row equals the oracle's."""
    name, two_s, two_M, gi = BUCKETS[bucket]
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    log(f"[hv_ex] {name} 2s={two_s} irrep {gi} (d={B.irrep.dim}) D={B.D} reps={len(B.sec.reps)}")
    rng = np.random.default_rng(100 + bucket)
    for nvec in (6, 8, 24):
        X64 = rng.uniform(-1, 1, (B.D, nvec))
        for dt in (P.F64, P.F32, P.F16):
            X = X64.astype(NP[dt])
            Xp = torch.from_numpy(_to_padded(B, X)).cuda()
            Y, info = LB.apply_H_ex(Xp, layout=P.LAYOUT_PADDED)
            assert info["adjacent_columns"] == 1, (nvec, dt, info)
            got, pad = _from_padded(B, Y.cpu().numpy())
            ref = hv.apply(B, H, X.astype(np.float64))
            err = rel_err_cols(got.astype(np.float64), ref)
            assert err <= TOL[dt], (nvec, dt, err)
            assert not np.any(pad), "padding rows of Y were written"
            # the block-row layout of the same launch gives the same numbers
            Yb, infob = LB.apply_H_ex(torch.from_numpy(X).cuda(), layout=P.LAYOUT_BLOCK)
            assert infob["adjacent_columns"] == 0
            assert rel_err_cols(Yb.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


@pytest.mark.parametrize("bucket", range(6))
def test_paired_rows_kernel_against_oracle(bucket):
    """Two vectors on two lanes per representative (one column each), the
    launch shape of the largest blocks' Lanczos runs: the gather loads both
    columns of a row at once and the lanes swap halves.  Every dimension
    bucket, FP64, FP32 and FP16, plain and with the Lanczos epilogue, against
    the oracle; an input that starts one element past a two-element boundary
    takes the row-by-row gather instead and gives the same bits."""
    name, two_s, two_M, gi = BUCKETS[bucket]
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    rng = np.random.default_rng(300 + bucket)
    nvec = 2
    for dt in (P.F64, P.F32, P.F16):
        X = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
        Xh = _to_padded(B, X)
        Xp = torch.from_numpy(Xh).cuda()
        Y, info = LB.apply_H_ex(Xp, layout=P.LAYOUT_PADDED, lanes=2)
        assert info["lanes_used"] == 2 and info["adjacent_columns"] == 1, info
        got, pad = _from_padded(B, Y.cpu().numpy())
        ref = hv.apply(B, H, X.astype(np.float64))
        assert rel_err_cols(got.astype(np.float64), ref) <= TOL[dt], dt
        assert not np.any(pad)
        # the same rows one element off the two-element boundary
        buf = torch.zeros(Xh.size + 1, dtype=TT[dt], device="cuda")
        Xo = buf[1:].view(Xh.shape)
        Xo.copy_(Xp)
        assert Xo.data_ptr() % (2 * Xo.element_size()) != 0
        Yo, info_o = LB.apply_H_ex(Xo, layout=P.LAYOUT_PADDED, lanes=2)
        assert info_o["lanes_used"] == 2
        assert torch.equal(Yo, Y), dt
        if dt == P.F16:
            continue
        # the epilogue: Y <- s H X - b Y0 and the sums X . Y
        Y0 = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
        sb = np.array([[1.25, 0.0], [0.75, -0.5]])
        Yp = torch.from_numpy(_to_padded(B, Y0)).cuda()
        dots = torch.full((nvec,), np.nan, dtype=torch.float64, device="cuda")
        Ye, info_e = LB.apply_H_ex(Xp, Yp, layout=P.LAYOUT_PADDED, lanes=2,
                                   scale=torch.from_numpy(sb).cuda(), dots=dots)
        assert info_e["adjacent_columns"] == 1
        gote, pade = _from_padded(B, Ye.cpu().numpy())
        refe = sb[:, 0] * ref - sb[:, 1] * Y0.astype(np.float64)
        assert rel_err_cols(gote.astype(np.float64), refe) <= TOL[dt], dt
        assert not np.any(pade)
        X64 = X.astype(np.float64)
        want = np.sum(X64 * gote.astype(np.float64), axis=0)
        assert np.all(np.abs(dots.cpu().numpy() - want) <= 1e-12 * np.sum(np.abs(X64 * gote.astype(np.float64)), axis=0))


@pytest.mark.parametrize("bucket", range(6))
def test_lanczos_epilogue_against_oracle(bucket):
    """The fused first half of a Lanczos step, Y <- s (H - e) X - b Y with the
    FP64 sums X . Y, in the padded layout with adjacent columns: every element
    against s (Psi^H H Psi X - e X) - b Y0 from the oracle, the sums against
    the same sums over the returned Y; one column with b = 0 (the first step)
    equals the plain product times s."""
    name, two_s, two_M, gi = BUCKETS[bucket]
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    rng = np.random.default_rng(200 + bucket)
    nvec = 24
    for dt in (P.F64, P.F32):
        for shift in (0.0, 0.75):
            X = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
            Y0 = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
            sb = np.stack([rng.uniform(0.5, 2.0, nvec), rng.uniform(-1.0, 1.0, nvec)], axis=1)
            sb[0, 1] = 0.0
            Xp = torch.from_numpy(_to_padded(B, X)).cuda()
            Yp = torch.from_numpy(_to_padded(B, Y0)).cuda()
            scale = torch.from_numpy(np.ascontiguousarray(sb)).cuda()
            dots = torch.full((nvec,), np.nan, dtype=torch.float64, device="cuda")
            Y, info = LB.apply_H_ex(Xp, Yp, layout=P.LAYOUT_PADDED, scale=scale, dots=dots, shift=shift)
            assert info["adjacent_columns"] == 1
            got, pad = _from_padded(B, Y.cpu().numpy())
            X64 = X.astype(np.float64)
            ref = sb[:, 0] * (hv.apply(B, H, X64) - shift * X64) - sb[:, 1] * Y0.astype(np.float64)
            assert rel_err_cols(got.astype(np.float64), ref) <= TOL[dt], (dt, shift)
            assert not np.any(pad)
            want = np.sum(X64 * got.astype(np.float64), axis=0)
            d = dots.cpu().numpy()
            assert np.all(np.abs(d - want) <= 1e-12 * np.sum(np.abs(X64 * got.astype(np.float64)), axis=0))
            # b = 0: s times the plain product, bitwise where s = 1 would be
            plain, _ = LB.apply_H_ex(torch.from_numpy(X).cuda(), layout=P.LAYOUT_BLOCK, shift=shift)
            p0 = plain.cpu().numpy()[:, 0].astype(np.float64) * sb[0, 0]
            assert np.max(np.abs(got[:, 0].astype(np.float64) - p0)) <= TOL[dt] * np.max(np.abs(p0)) * 2


def test_options_and_errors():
    B, H, LB, keep = _blocks("dodecahedron", 1, 0, 8)
    X = torch.zeros((LB.D_pad, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        LB.apply_H_ex(X, layout=7)
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        LB.apply_H_ex(X, layout=P.LAYOUT_PADDED, lanes=3)
    dots = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        LB.apply_H_ex(X, layout=P.LAYOUT_PADDED, dots=dots)
    # every lane layout gives the same numbers (each output element is one lane's fixed-order sum)
    rng = np.random.default_rng(3)
    Xb = rng.uniform(-1, 1, (B.D, 5))
    Xp = torch.from_numpy(_to_padded(B, Xb)).cuda()
    ref = None
    for lanes in (1, 2, 4, 8, 16, 32, 64):
        Y, info = LB.apply_H_ex(Xp, layout=P.LAYOUT_PADDED, lanes=lanes)
        assert info["lanes_used"] == lanes
        y = Y.cpu().numpy()
        if ref is None:
            ref = y
            assert rel_err_cols(_from_padded(B, y)[0], hv.apply(B, H, Xb)) <= 1e-12
        assert np.array_equal(y, ref), lanes
    # AUTO takes the layout of ftlm_run: block rows for this small block
    Y, info = LB.apply_H_ex(torch.from_numpy(Xb).cuda(), layout=P.LAYOUT_AUTO)
    assert rel_err_cols(Y.cpu().numpy(), hv.apply(B, H, Xb)) <= 1e-12


def test_empty_block_zeroes_dots():
    _, _, irs = oracle_group("icosahedron")
    cl = clusters.get("icosahedron")
    S = P.Sector(cl, P.Group(cl.N, cl.gens), 6, two_s=1)
    LB = P.Block(S, 1, 0, user_rho=irs[1].rho)          # A_u at 2M = 6 is empty
    assert LB.D == 0
    X = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    dots = torch.full((2,), 5.0, dtype=torch.float64, device="cuda")
    scale = torch.ones((2, 2), dtype=torch.float64, device="cuda")
    LB.apply_H_ex(X, torch.zeros_like(X), layout=P.LAYOUT_BLOCK, scale=scale, dots=dots)
    assert np.array_equal(dots.cpu().numpy(), [0.0, 0.0])


def _packed_rows(n_reps, d, row_bytes):
    """The packed layout as the ABI documents it: rows of representative i and
    the total row count (p = (128 / row_bytes) // d per 128-byte line when
    2 <= p and p d < 128 / row_bytes, else d rows per representative)."""
    L = 128 // row_bytes if 128 % row_bytes == 0 else 0
    p = L // d if L else 0
    if p >= 2 and p * d < L:
        start = (np.arange(n_reps) // p) * L + (np.arange(n_reps) % p) * d
        return start, -(-n_reps // p) * L, True
    return np.arange(n_reps) * d, n_reps * d, False


def _to_layout(B, X, start, rows):
    Xp = np.zeros((rows, X.shape[1]), dtype=X.dtype)
    for i in np.nonzero(B.n_rep)[0]:
        o, n = int(B.offsets[i]), int(B.n_rep[i])
        Xp[start[i]:start[i] + n] = X[o:o + n]
    return Xp


@pytest.mark.parametrize("bucket", range(6))
def test_packed_layout_against_oracle(bucket):
    """The packed row layout (no representative straddles a 128-byte line),
    for every dimension bucket and row sizes of 4, 8 and 16 bytes: every
    output row equals the oracle's, and the rows between representatives and
    the padding rows are not written."""
    name, two_s, two_M, gi = BUCKETS[bucket]
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    rng = np.random.default_rng(300 + bucket)
    d = B.irrep.dim
    n_reps = len(B.sec.reps)
    seen_packed = False
    for nvec, dt in ((1, P.F32), (2, P.F32), (4, P.F32), (1, P.F64), (2, P.F64), (2, P.F16), (8, P.F16)):
        elem = {P.F64: 8, P.F32: 4, P.F16: 2}[dt]
        start, rows, packed = _packed_rows(n_reps, d, nvec * elem)
        seen_packed |= packed
        X = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
        Xp = torch.from_numpy(_to_layout(B, X, start, rows)).cuda()
        Y, info = LB.apply_H_ex(Xp, layout=P.LAYOUT_PACKED)
        Yh = Y.cpu().numpy()
        ref = hv.apply(B, H, X.astype(np.float64))
        got = np.concatenate([Yh[start[i]:start[i] + int(B.n_rep[i])] for i in np.nonzero(B.n_rep)[0]])
        assert rel_err_cols(got.astype(np.float64), ref) <= TOL[dt], (nvec, dt)
        written = np.zeros(rows, dtype=bool)
        for i in np.nonzero(B.n_rep)[0]:
            written[start[i]:start[i] + int(B.n_rep[i])] = True
        assert not np.any(Yh[~written]), (nvec, dt)
    # d = 1, 2, 4 divide every power-of-two line, where packing is the padded layout itself
    assert seen_packed or d in (1, 2, 4)


def test_packed_lanczos_and_kpm_match_block_rows():
    """Lanczos chains and KPM moments in the packed layout (one FP64 chain: 8-byte rows,
    3 representatives of d = 5 to a 16-row line) equal those in block rows up to
    the order of the FP64 reductions; two FP32 chains the same to FP32 rounding."""
    name, two_s, two_M, gi = "dodecahedron", 1, 0, 8
    _, _, irs = oracle_group(name)
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    S = LB.sector
    LK = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_PACKED)
    LBl = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_BLOCK)
    n_reps = len(B.sec.reps)
    a, b, n, info = LK.ftlm(1, 40, 5, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_PACKED and info["rows"] == -(-n_reps // 3) * 16
    a1, b1, n1 = LBl.ftlm(1, 40, 5, storage=P.F64)
    assert np.max(np.abs(a[:, :15] - a1[:, :15])) < 1e-12 * np.max(np.abs(a1))
    assert np.max(np.abs(b[:, :15] - b1[:, :15])) < 1e-12 * np.max(np.abs(b1))
    a, b, n, info = LK.ftlm(2, 30, 6, storage=P.F32, info=True)
    assert info["layout"] == P.LAYOUT_PACKED and info["rows"] == -(-n_reps // 3) * 16
    a1, b1, n1 = LBl.ftlm(2, 30, 6, storage=P.F32)
    assert np.max(np.abs(a[:, :15] - a1[:, :15])) < 1e-6 * np.max(np.abs(a1))
    # R = 3 FP64: 24-byte rows do not divide a line: plain padded rows
    _, _, _, info = LK.ftlm(3, 10, 6, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_PADDED
    m = LK.kpm(1, 41, 9, 0.5, 20.0)
    m1 = LBl.kpm(1, 41, 9, 0.5, 20.0)
    assert np.max(np.abs(m - m1)) < 1e-12


def _aligned_rows(n_reps, d, row_bytes):
    """Start rows of the aligned layout (include/ftlm.h): S rows per
    representative, S the smallest power of two >= d, when the row size is a
    power of two, S > d and S * row_bytes <= 128; plain padded rows otherwise."""
    S = 1
    while S < d:
        S *= 2
    if row_bytes & (row_bytes - 1) == 0 and S > d and S * row_bytes <= 128:
        return np.arange(n_reps) * S, n_reps * S, True
    return np.arange(n_reps) * d, n_reps * d, False


@pytest.mark.parametrize("bucket", range(6))
def test_aligned_layout_against_oracle(bucket):
    """The aligned row layout (each representative's rows in one power-of-two
    block of at most 128 bytes) for every dimension bucket and row sizes of 2
    to 32 bytes, the two-vector launches included (paired-row gather): every
    output row equals the oracle's, and the padding rows are not written."""
    name, two_s, two_M, gi = BUCKETS[bucket]
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    rng = np.random.default_rng(400 + bucket)
    d = B.irrep.dim
    n_reps = len(B.sec.reps)
    seen = False
    for nvec, dt in ((1, P.F32), (2, P.F32), (4, P.F32), (8, P.F32), (1, P.F64), (2, P.F64), (2, P.F16),
                     (3, P.F32)):
        elem = {P.F64: 8, P.F32: 4, P.F16: 2}[dt]
        start, rows, aligned = _aligned_rows(n_reps, d, nvec * elem)
        seen |= aligned
        X = rng.uniform(-1, 1, (B.D, nvec)).astype(NP[dt])
        Xp = torch.from_numpy(_to_layout(B, X, start, rows)).cuda()
        Y, info = LB.apply_H_ex(Xp, layout=P.LAYOUT_ALIGNED)
        Yh = Y.cpu().numpy()
        ref = hv.apply(B, H, X.astype(np.float64))
        got = np.concatenate([Yh[start[i]:start[i] + int(B.n_rep[i])] for i in np.nonzero(B.n_rep)[0]])
        assert rel_err_cols(got.astype(np.float64), ref) <= TOL[dt], (nvec, dt)
        written = np.zeros(rows, dtype=bool)
        for i in np.nonzero(B.n_rep)[0]:
            written[start[i]:start[i] + int(B.n_rep[i])] = True
        assert not np.any(Yh[~written]), (nvec, dt)
    # d = 1, 2, 4 are powers of two already: aligned rows are the padded rows
    assert seen or d in (1, 2, 4)


def test_aligned_lanczos_and_kpm_match_block_rows():
    """Lanczos chains and KPM moments in the aligned layout (d = 5: 8 rows per
    representative) equal those in block rows up to the order of the FP64
    reductions (one FP64 chain, four FP32 chains) or FP32 rounding (two FP32
    chains: the paired-row gather); rows that would pass 128 bytes fall back
    to padded rows."""
    name, two_s, two_M, gi = "dodecahedron", 1, 0, 8
    _, _, irs = oracle_group(name)
    B, H, LB, keep = _blocks(name, two_s, two_M, gi)
    S = LB.sector
    LA = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_ALIGNED)
    LBl = P.Block(S, gi, 0, user_rho=irs[gi].rho, layout=P.LAYOUT_BLOCK)
    n_reps = len(B.sec.reps)
    a, b, n, info = LA.ftlm(1, 40, 5, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_ALIGNED and info["rows"] == n_reps * 8
    a1, b1, n1 = LBl.ftlm(1, 40, 5, storage=P.F64)
    assert np.max(np.abs(a[:, :15] - a1[:, :15])) < 1e-12 * np.max(np.abs(a1))
    assert np.max(np.abs(b[:, :15] - b1[:, :15])) < 1e-12 * np.max(np.abs(b1))
    for R in (2, 4):
        a, b, n, info = LA.ftlm(R, 30, 6, storage=P.F32, info=True)
        assert info["layout"] == P.LAYOUT_ALIGNED and info["rows"] == n_reps * 8
        a1, b1, n1 = LBl.ftlm(R, 30, 6, storage=P.F32)
        assert np.max(np.abs(a[:, :15] - a1[:, :15])) < 1e-6 * np.max(np.abs(a1)), R
        assert np.max(np.abs(b[:, :15] - b1[:, :15])) < 1e-6 * np.max(np.abs(b1)), R
    # 4 FP64 vectors: 32-byte rows, 8 of them pass 128 bytes: plain padded rows
    _, _, _, info = LA.ftlm(4, 10, 6, storage=P.F64, info=True)
    assert info["layout"] == P.LAYOUT_PADDED
    m = LA.kpm(1, 41, 9, 0.5, 20.0)
    m1 = LBl.kpm(1, 41, 9, 0.5, 20.0)
    assert np.max(np.abs(m - m1)) < 1e-12
