"""Host-side checks of the benchmark script (no GPU): the one-GPU refusal and
the byte model behind the roofline figure."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_byte_model_block_and_padded_rows():
    # 10 connections, 8 of them to active targets (3 of those with a
    # non-trivial stabilizer), 30 gathered rows; D = 20 rows, 6 representatives
    # of which 5 are active; 4 vectors of 4 bytes; 6-byte compact entries
    st = dict(connections=10, active_connections=8, gathered_rows=30, nontrivial_targets=3, n_active=5,
              entry_bytes=6)
    D, n_reps, nvec, b = 20, 6, 4, 4
    gathered = 30 * nvec * b
    entries = 6 * 10
    per_rep = 32 * 5 + 8 * 1
    block = gathered + entries + 8 * 10 + 2 * D * nvec * b + per_rep
    assert bench.algorithmic_bytes(st, D, n_reps, nvec, b) == block
    # padded rows: 2-byte stabilizer ids for non-trivial and inactive targets
    # instead of the 8-byte metadata word; the epilogue reads q_{j-1} too
    padded = gathered + entries + 2 * (3 + 2) + 3 * D * nvec * b + per_rep
    assert bench.algorithmic_bytes(st, D, n_reps, nvec, b, pad=True, epilogue=True) == padded


def test_workload_irreps_exist_and_match_their_descriptions():
    # every single-sector workload names an irrep of G (or of G x Z2 when it
    # resolves the spin flip, index 2i + q for irrep i of G and parity q) and
    # its roofline irrep; H blocks of I_h have dimension 5
    from oracle import group as ogroup
    from oracle import irreps as oirreps
    from oracle import spinflip
    from synth import clusters

    for name, wl in bench.WORKLOADS.items():
        if wl.get("campaign"):
            continue
        cl = clusters.get(wl["cluster"])
        irs = oirreps.compute_irreps(ogroup.close(cl.gens, cl.N))
        n = 2 * len(irs) if wl.get("flip") else len(irs)
        gi = bench.roofline_irrep(wl)
        assert 0 <= gi < n, name
        if wl["irrep"] != "all":
            assert wl["irrep"] == gi, name
        base = irs[gi // 2] if wl.get("flip") else irs[gi]
        if wl.get("flip"):
            assert spinflip.flip_irreps(irs)[gi].dim == base.dim, name
        if "H_g" in wl["desc"] or gi == 8:
            assert base.dim == 5, name
