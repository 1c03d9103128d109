"""Checkpointed Lanczos runs (ftlm_run_begin / advance / save / load /
finish): a run interrupted after some steps, written to a file, freed and
rebuilt from the file gives the coefficients of one uninterrupted ftlm_run
call bit for bit, in every storage type and row layout; a checkpoint is
refused by another block.  Also the autotuner cache on the device: a tuned
lane layout saved to a file and loaded back is used again, and only for the
architecture it was tuned on."""
import numpy as np
import pytest

from gpu_helpers import lib_block, lib_sector, log, oracle_group

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")


@pytest.mark.parametrize("case", range(6))
def test_interrupted_run_resumes_bitwise(tmp_path, case):
    name, gi, R, steps, stor, layout, cut = [
        ("dodecahedron", 8, 5, 41, P.F64, P.LAYOUT_BLOCK, 13),
        ("dodecahedron", 8, 6, 30, P.F32, P.LAYOUT_PADDED, 14),     # padded rows, adjacent columns
        ("icosahedron", 8, 3, 30, P.F16, P.LAYOUT_BLOCK, 7),
        ("dodecahedron", 2, 24, 60, P.F32, P.LAYOUT_PADDED, 1),
        ("dodecahedron", 8, 2, 40, P.F32, P.LAYOUT_PACKED, 17),     # 3 representatives per 128-byte line
        ("dodecahedron", 8, 2, 40, P.F32, P.LAYOUT_ALIGNED, 9),     # 8 rows (64 bytes) per representative
    ][case]
    log(f"[checkpoint] {name} irrep {gi} R={R} storage {stor} layout {layout} cut at {cut}")
    _, _, irs = oracle_group(name)
    B = P.Block(lib_sector(name, 1, 0), gi, 0, user_rho=irs[gi].rho, layout=layout)
    a0, b0, n0 = B.ftlm(R, steps, 77, storage=stor)
    s = torch.cuda.Stream()
    run = P.LanczosRunState.begin(B, R, steps, 77, storage=stor, stream=s)
    assert run.advance(cut) == cut
    path = tmp_path / "run.ckpt"
    path.write_bytes(b"an earlier file")   # replaced as a whole
    run.save(path)
    assert not (tmp_path / "run.ckpt.part").exists()
    run.close()
    torch.cuda.synchronize()
    X = torch.randn((B.D, 2), dtype=torch.float64, device="cuda")
    B.apply_H(X)                          # other device work in between
    run2 = P.LanczosRunState.load(B, path, R, steps, stream=s)
    a, b, n = run2.finish()
    run2.close()
    assert np.array_equal(n, n0) and np.array_equal(a, a0) and np.array_equal(b, b0)
    # the same run without interruption, through the staged calls
    run3 = P.LanczosRunState.begin(B, R, steps, 77, storage=stor, stream=s)
    a3, b3, n3 = run3.finish()
    run3.close()
    assert np.array_equal(a3, a0) and np.array_equal(b3, b0)


def test_checkpoint_refused_by_another_block(tmp_path):
    _, _, irs = oracle_group("dodecahedron")
    S = lib_sector("dodecahedron", 1, 0)
    B = P.Block(S, 8, 0, user_rho=irs[8].rho)
    run = P.LanczosRunState.begin(B, 2, 20, 5)
    run.advance(3)
    run.save(tmp_path / "a.ckpt")
    run.close()
    other = P.Block(S, 6, 0, user_rho=irs[6].rho)
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        P.LanczosRunState.load(other, tmp_path / "a.ckpt", 2, 20)
    (tmp_path / "b.ckpt").write_bytes(b"not a checkpoint")
    with pytest.raises(P.FtlmError, match="INVALID_ARG"):
        P.LanczosRunState.load(B, tmp_path / "b.ckpt", 2, 20)


def test_autotune_cache_saved_and_loaded_on_the_device(tmp_path):
    B = lib_block("dodecahedron", 1, 0, 8)
    nvec = 6
    X = torch.randn((B.D, nvec), dtype=torch.float64, device="cuda")
    sb = torch.ones((nvec, 2), dtype=torch.float64, device="cuda")
    P.autotune_clear()
    _, info0 = B.apply_H_ex(X, layout=P.LAYOUT_AUTO, scale=sb)     # the Lanczos run's launch, untuned
    best, ms, tried = B.autotune(nvec, P.F64)
    assert best in tried and ms > 0
    arch = P.device_arch()
    assert arch.startswith("gfx")
    path = tmp_path / "tune.txt"
    n = P.autotune_save(path)
    assert n >= 2 and all(line.startswith(arch + " ") for line in path.read_text().split("\n")[:-1])
    P.autotune_clear()
    _, info = B.apply_H_ex(X, layout=P.LAYOUT_AUTO, scale=sb)
    assert info["lanes_used"] == info0["lanes_used"]
    assert P.autotune_load(path, "gfx000:not-this-device") == 0
    assert P.autotune_load(path, arch) == n
    _, info = B.apply_H_ex(X, layout=P.LAYOUT_AUTO, scale=sb)
    assert info["lanes_used"] == best
    P.autotune_clear()
