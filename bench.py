#!/usr/bin/env python
"""Benchmark of the symmetry-adapted FTLM hot path on one MI355X.

One step = one complete FTLM job: group closure and irreps, sector tables
(representatives, stabilizers, lookup, entry table), and for every block of
the workload its block data and R batched Lanczos chains (one H.V launch per
step for all chains), then Ritz data and the thermal sums on 50 temperatures
over all blocks.  Default workload: the s=1/2 icosidodecahedron, M=0, all ten
I_h irreps (41,364,764 rows), R = 24 Gaussian chains per block, 60 steps,
FP32 vector storage with FP64 reductions.

value = sum over blocks of D * (H.V products of all chains) / step time, in
basis elements x vectors per second.  The roofline object describes the H.V
kernel on the largest block (H_g, D = 6,465,762) inside the timed runs (HIP
events on the launch stream).  After the timed region: the same job in FP64
storage (error of E, C, chi per temperature), the serving mix through the
job server (closed burst for capacity, then a time-bounded Poisson stream:
p50/p99 latency), and the CPU baseline (the FP64 oracle on sampled output
rows of the H_g block, one worker process per host core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    # name: cluster, 2s, 2M, irrep index (library order; "all" = every irrep of
    # the sector, with the roofline measured on roofline_irrep), R, steps, dist, storage
    "icosidodecahedron_M0": dict(cluster="icosidodecahedron", two_s=1, two_M=0, irrep="all", roofline_irrep=8,
                                 R=24, steps=60, dist="gaussian", storage="f32",
                                 desc="s=1/2 Heisenberg icosidodecahedron (N=30, 60 bonds), I_h, M=0 "
                                      "(D_M=155,117,520), all 10 irreps row 1 (blocks 1,291,834..6,465,762, "
                                      "41,364,764 rows); R=24 Gaussian chains per block, 60 Lanczos steps, FP32 "
                                      "storage, FP64 reductions, eigensolve and thermal sums at 50 T",
                                 context=dict(paper="Section 4.3's workstation-scale example: the same ten-irrep "
                                                    "M=0 sweep (as 20 Z2-parity blocks, 8 vectors per launch) in "
                                                    "96.5 s end to end (the paper's workstation GPU is an RTX 4000 "
                                                    "SFF Ada); another machine and a wall time, not a target",
                                              paper_s=96.5, paper_elem_vec_per_s=41364764 * 24 * 60 / 96.5)),
    "icosidodecahedron_Hg": dict(cluster="icosidodecahedron", two_s=1, two_M=0, irrep=8, R=24, steps=60,
                                 dist="gaussian", storage="f32",
                                 desc="s=1/2 Heisenberg icosidodecahedron (N=30, 60 bonds), I_h, M=0, "
                                      "irrep H_g row 1 (D=6,465,762); R=24 Gaussian chains, 60 Lanczos steps, "
                                      "FP32 storage, FP64 reductions"),
    "dodecahedron_s32_Hg": dict(cluster="dodecahedron", two_s=3, two_M=0, irrep=8, R=2, steps=60,
                                dist="rademacher", storage="f32", fp64_check=False, otf_timing=False,
                                desc="s=3/2 Heisenberg dodecahedron (N=20, 30 bonds, 40-bit labels), I_h, M=0 "
                                     "(D_M=86,981,744,944), irrep H_g row 1 (D=3,624,380,734); R=2 Rademacher chains, "
                                     "60 Lanczos steps, FP32 storage, FP64 reductions"),
    "icosidodecahedron_Hg_f16": dict(cluster="icosidodecahedron", two_s=1, two_M=0, irrep=8, R=24, steps=60,
                                     dist="gaussian", storage="f16",
                                     desc="s=1/2 Heisenberg icosidodecahedron (N=30, 60 bonds), I_h, M=0, irrep H_g "
                                          "row 1 (D=6,465,762); R=24 Gaussian chains, 60 Lanczos steps, FP16 storage "
                                          "with a per-chain power-of-two scale, FP64 arithmetic and reductions"),
    "dodecahedron_s32_Hg_f16": dict(cluster="dodecahedron", two_s=3, two_M=0, irrep=8, R=2, steps=60,
                                    dist="rademacher", storage="f16", fp64_check=False, otf_timing=False,
                                    desc="s=3/2 Heisenberg dodecahedron (N=20, 30 bonds, 40-bit labels), I_h, M=0, "
                                         "irrep H_g row 1 (D=3,624,380,734); R=2 Rademacher chains, 60 Lanczos steps, "
                                         "FP16 storage with a per-chain power-of-two scale, FP64 arithmetic"),
    "dodecahedron_s32_Hg_flip": dict(cluster="dodecahedron", two_s=3, two_M=0, irrep=16, R=2, steps=60,
                                     dist="rademacher", storage="f32", fp64_check=False, otf_timing=False, flip=True,
                                     desc="s=3/2 Heisenberg dodecahedron, M=0 resolved by G x Z2 (I_h x spin "
                                          "flip), irrep H_g^+ row 1 (D=1,812,277,727); R=2 Rademacher chains, 60 "
                                          "Lanczos steps, FP32 storage, FP64 reductions"),
    "icosahedron_all": dict(cluster="icosahedron", two_s=1, R=4, steps=30, dist="rademacher", storage="f64",
                            campaign=True, chains_per_run=1,
                            desc="s=1/2 Heisenberg icosahedron (N=12), I_h, all M >= 0 sectors, all 10 irreps, row 1; "
                                 "R=4 Rademacher chains run one at a time (plain single-vector FP64 path), 30 "
                                 "Lanczos steps; E, C, chi at 50 T in [0.05, 10]"),
    "dodecahedron_all": dict(cluster="dodecahedron", two_s=1, R=24, steps=60, dist="rademacher", storage="f64",
                             campaign=True, chains_per_run=0,
                             desc="s=1/2 Heisenberg dodecahedron (N=20), I_h, all M >= 0 sectors, all irreps, row 1; "
                                  "R=24 Rademacher chains batched in one H.V launch per step, 60 Lanczos steps, "
                                  "FP64; E, C, chi at 50 T"),
    "icosidodecahedron_all": dict(cluster="icosidodecahedron", two_s=1, R=24, steps=60, dist="gaussian",
                                  storage="f32", campaign=True, chains_per_run=0, alt_paths=False,
                                  cpu_baseline=False,
                                  roofline_note="the blocks' H.V launches are those of the default workload "
                                                "(its roofline line); no separate roofline for the campaign",
                                  desc="s=1/2 Heisenberg icosidodecahedron (N=30), I_h, all M >= 0 sectors, all "
                                       "10 irreps, row 1; R=24 Gaussian chains batched in one H.V launch per step, "
                                       "60 Lanczos steps, FP32 storage, FP64 reductions; E, C, chi at 50 T",
                                  context=dict(paper="Table 3: the same run (R=24, N_L=60, all M >= 0 sectors) in "
                                                     "91.5 s FP32 and 81.1 s FP16 end to end on one B200, 433.4 s "
                                                     "FP32 on the RTX 4000 SFF Ada workstation; other machines, "
                                                     "not a target",
                                               paper_b200_fp32_s=91.5, paper_b200_fp16_s=81.1,
                                               paper_workstation_fp32_s=433.4)),
    "icosidodecahedron_all_f16": dict(cluster="icosidodecahedron", two_s=1, R=24, steps=60, dist="gaussian",
                                      storage="f16", campaign=True, chains_per_run=0, alt_paths=False,
                                      cpu_baseline=False,
                                      roofline_note="no separate roofline for the campaign",
                                      desc="s=1/2 Heisenberg icosidodecahedron (N=30), I_h, all M >= 0 sectors, "
                                           "all 10 irreps, row 1; R=24 Gaussian chains batched, 60 Lanczos steps, "
                                           "FP16 storage with a per-chain power-of-two scale, FP64 arithmetic; "
                                           "E, C, chi at 50 T"),
    "dodecahedron_Hg": dict(cluster="dodecahedron", two_s=1, two_M=0, irrep=8, R=24, steps=60, dist="rademacher",
                            storage="f64",
                            desc="s=1/2 dodecahedron (N=20), I_h, M=0, irrep H_g (D=7,800); R=24 Rademacher, "
                                 "60 steps, FP64"),
}


def algorithmic_bytes(stats, D, n_reps, nvec, elem, pad=False, epilogue=False):
    """Bytes one H.V launch must move (no cache reuse credited).

    Per connection (flip of an active output representative): the stored
    entry (stats["entry_bytes"]), and the target's 8-byte metadata word in the
    block row layout, or in the padded layout its 2-byte stabilizer id when
    the entry does not mark the stabilizer trivial (inactive targets never
    have a trivial stabilizer); per active connection the gathered X rows
    (n_Gamma(target) * nvec * elem).  Per block row: X read once (diagonal)
    and Y written, plus the previous Lanczos vector read in the Lanczos
    epilogue.  Per active output representative: label, metadata, row pointer
    and diagonal energy (32 bytes); per inactive one its metadata word.
    """
    conn = stats["connections"]
    inact = conn - stats["active_connections"]
    eb = stats.get("entry_bytes", 8)
    target = 2 * (stats.get("nontrivial_targets", 0) + inact) if pad else 8 * conn
    vec = (3 if epilogue else 2) * D * nvec * elem
    return (stats["gathered_rows"] * nvec * elem + eb * conn + target + vec
            + 32 * stats["n_active"] + 8 * (n_reps - stats["n_active"]))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores():
    """Cores this process may use: its affinity set, capped at the 16 threads
    the GPU machine grants one GPU (OMP_NUM_THREADS there)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    return max(1, min(n, cap, 16))


def _single_thread_env():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _oracle_rows_worker(wl, seconds, seed):
    """One worker of the CPU baseline: FP64 oracle H.v (nvec = 1) on random
    output representatives of the block for `seconds`; returns (rows, reps)."""
    import numpy as np

    from oracle import basis as obasis
    from oracle import group as ogroup
    from oracle import hv as ohv
    from oracle import irreps as oirreps
    from synth import clusters
    from synth.vectors import label_keyed_values

    cl = clusters.get(wl["cluster"])
    G = ogroup.close(cl.gens, cl.N)
    irs = oirreps.compute_irreps(G)
    if wl.get("flip"):
        from oracle import spinflip
        G, irs = spinflip.FlipGroup(G), spinflip.flip_irreps(irs)
    ir = irs[wl["irrep"]]
    d = wl["two_s"] + 1
    rng = np.random.default_rng(seed)
    A = (cl.N * wl["two_s"] + wl["two_M"]) // 2

    def xfun(r, n):
        return label_keyed_values(5, np.full(n, r, dtype=np.uint64), np.arange(n, dtype=np.uint64),
                                  np.zeros(n, np.uint64))[:, None]

    rows = reps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        if d == 2:
            bits = rng.choice(cl.N, A, replace=False)
            lab = int(np.sum(2 ** bits.astype(np.int64)))
        else:
            while True:  # a uniform state of the sector: digits with sum A, by rejection
                dig = rng.integers(0, d, cl.N)
                if dig.sum() == A:
                    break
            lab = int(sum(int(a) * d ** k for k, a in enumerate(dig)))
        p, _ = obasis.canonicalize(G, np.array([lab]), cl.N, d)
        out = ohv.sampled_rows(G, ir, 0, cl.N, wl["two_s"], cl.bonds, cl.J, [int(p[0])], xfun, 1)
        rows += out[0].shape[0]
        reps += 1
    return rows, reps, time.perf_counter() - t0


def cpu_baseline(wl, seconds):
    """FP64 oracle H.v (nvec = 1) on sampled output rows of the block, one
    single-threaded worker process per host core (spawned: no GPU state is
    inherited)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    cores = _host_cores()
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn"),
                                initializer=_single_thread_env) as ex:
        futs = [ex.submit(_oracle_rows_worker, wl, seconds, 17 + k) for k in range(cores)]
        res = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    rows = sum(r[0] for r in res)
    reps = sum(r[1] for r in res)
    busy = max(r[2] for r in res)
    per_core = sum(r[0] / r[2] for r in res) / cores
    return dict(value=rows / busy, unit="basis-elems*vecs/s", cores=cores, kind="oracle",
                per_core=per_core, cpu_model=_cpu_model(), os_cpu_count=os.cpu_count(),
                sample=f"{reps} random output representatives of the irrep-{wl['irrep']} block ({rows} rows, nvec=1, "
                       f"FP64), {cores} single-threaded worker processes x {seconds:.0f} s of Python/NumPy "
                       f"({wall:.1f} s with start-up)")


SERVE_CLUSTERS = ("icosahedron", "cuboctahedron", "dodecahedron", "square4x4", "square6x6")
SERVE_DESC = ("Poisson stream of FTLM jobs drawn uniformly from the s=1/2 icosahedron (I_h), cuboctahedron "
              "(O_h), dodecahedron (I_h), 4x4 and 6x6 square tori (translations x C4v, orders 128, 288); "
              "uniform 2M >= 0, irrep, row; R uniform in 4..24; 60 steps; FP64 or FP32 storage; Rademacher")


def draw_jobs(rng, n, groups, clusters, names=SERVE_CLUSTERS):
    """Seeded job descriptions of the serving mix (clusters drawn from names)."""
    jobs = []
    for _ in range(n):
        name = names[rng.integers(len(names))]
        cl = clusters.get(name)
        dims = groups[name]
        gi = int(rng.integers(len(dims)))
        jobs.append(dict(cluster=name, two_M=int(2 * rng.integers(cl.N // 2 + 1)), irrep=gi,
                         row=int(rng.integers(dims[gi])), R=int(rng.integers(4, 25)), steps=60,
                         seed=int(rng.integers(1 << 62)), storage=("f64", "f32")[int(rng.integers(2))]))
    return jobs


def serve(P, np, n_warm, n_jobs, rate, budget_gb, max_active, seed=0x5EED0100, log_path=None, load=0.8,
          poisson_jobs=None, time_bound_s=None, engine=0, names=SERVE_CLUSTERS):
    """Warm-up burst, a closed burst (capacity), then an open Poisson stream (latency).

    The closed burst submits n_jobs at once; its throughput is the capacity
    estimate, and the Poisson stream offers load x capacity (or the given rate)
    for poisson_jobs arrivals (default n_jobs), cut short when the arrivals
    would pass time_bound_s (the count is reported).  A job's latency runs
    from its submission to its coefficients on the host: queueing, table
    builds on a cold cache and the Lanczos run are all inside.
    """
    from synth import clusters
    groups = {n: list(P.Group(clusters.get(n).N, clusters.get(n).gens).irreps()["dims"]) for n in names}
    srv = P.Server(int(budget_gb * (1 << 30)), max_active=max_active)
    F = {"f64": P.F64, "f32": P.F32}
    records = []

    def submit(j):
        cl = clusters.get(j["cluster"])
        return srv.submit(cl, cl.gens, j["two_M"], j["irrep"], j["row"], j["R"], j["steps"], j["seed"],
                          storage=F[j["storage"]], dist=P.RADEMACHER, two_s=1, engine=engine)

    def run(phase, jobs, arrivals):
        t0 = time.perf_counter()
        ids = []
        for j, ta in zip(jobs, arrivals):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            ids.append(submit(j))
        res = [srv.wait(i) for i in ids]
        for r, j in zip(res, jobs):
            if r[0]["status"] != 0:
                raise RuntimeError(f"serving job failed: {j} -> {r[0]}")
            records.append(dict(phase=phase, **j, D=int(r[0]["D"]), d_gamma=int(r[0]["d_gamma"]),
                                submit=r[0]["submit_s"], start=r[0]["start_s"], end=r[0]["end_s"],
                                engine=int(r[0]["engine"])))
        span = max(r[0]["end_s"] for r in res) - min(r[0]["submit_s"] for r in res)
        lat = np.array([r[0]["end_s"] - r[0]["submit_s"] for r in res]) * 1e3
        wait = np.array([r[0]["start_s"] - r[0]["submit_s"] for r in res]) * 1e3
        work = sum(int(r[0]["D"]) * int(r[3].sum()) for r in res)
        print(f"[serve] {phase}: {len(jobs)} jobs in {span:.2f} s, p50 {np.percentile(lat, 50):.1f} ms, "
              f"p99 {np.percentile(lat, 99):.1f} ms", file=sys.stderr, flush=True)
        return dict(jobs=len(jobs), span_s=span, jobs_per_s=len(jobs) / span, elem_vec_per_s=work / span,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    max_ms=float(lat.max()), queue_p50_ms=float(np.percentile(wait, 50)),
                    queue_p99_ms=float(np.percentile(wait, 99)))

    # each phase draws from a generator of its own, so a phase's jobs do not
    # depend on the sizes of the others (runs stay comparable)
    t = time.perf_counter()
    run("warm", draw_jobs(np.random.default_rng(seed + 1), n_warm, groups, clusters, names), [0.0] * n_warm)
    warm_s = time.perf_counter() - t
    burst = run("burst", draw_jobs(np.random.default_rng(seed + 2), n_jobs, groups, clusters, names), [0.0] * n_jobs)
    lam = rate if rate else load * burst["jobs_per_s"]
    n_p = poisson_jobs or n_jobs
    arrivals = np.cumsum(np.random.default_rng(seed + 3).exponential(1.0 / lam, n_p))
    if time_bound_s:
        arrivals = arrivals[arrivals <= time_bound_s]
    stream = run("poisson", draw_jobs(np.random.default_rng(seed + 4), n_p, groups, clusters, names)[:len(arrivals)],
                 arrivals)
    stats = srv.stats()
    srv.close()
    if log_path:
        with open(log_path, "w") as f:
            for r in records:
                f.write(json.dumps(r) + "\n")
    return dict(workload=SERVE_DESC if names == SERVE_CLUSTERS else "serving mix restricted to " + ", ".join(names),
                warmup_jobs=n_warm, warmup_s=warm_s, max_active=max_active,
                engine={0: "auto", 1: "steps", 2: "fused"}[engine],
                budget_gb=budget_gb, closed_burst=burst,
                poisson=dict(rate_jobs_per_s=lam, offered_jobs=n_p, time_bound_s=time_bound_s, **stream),
                engines=dict(fused=sum(r["engine"] == P.ENGINE_FUSED for r in records),
                             steps=sum(r["engine"] == P.ENGINE_STEPS for r in records)),
                resident_bytes_after=stats["used_bytes"])


def oracle_campaign_rate(wl, seconds):
    """FP64 oracle FTLM over the cluster's blocks (explicit basis, SciPy Lanczos), block by block
    until the time budget is spent: basis elements x products per second."""
    import numpy as np

    from oracle import basis as obasis
    from oracle import ftlm as oftlm
    from oracle import group as ogroup
    from oracle import hv as ohv
    from oracle import irreps as oirreps
    from oracle import sector as osector
    from synth import clusters

    cl = clusters.get(wl["cluster"])
    G = ogroup.close(cl.gens, cl.N)
    irs = oirreps.compute_irreps(G)
    two_s = wl["two_s"]
    work, blocks = 0, 0
    t0 = time.perf_counter()
    for two_M in range((cl.N * two_s) % 2, cl.N * two_s + 1, 2):
        sec = obasis.sector_reps(G, cl.N, two_s, two_M)
        H = osector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
        for gi, ir in enumerate(irs):
            B = obasis.build_block(G, ir, sec)
            if B.D == 0:
                continue
            Hb = ohv.block_matrix(B, H)
            for r in range(wl["R"]):
                v0 = oftlm.start_vector(B.D, 1, two_M, gi, 0, r, "rademacher")
                a, b = oftlm.lanczos(lambda x: Hb @ x, v0, wl["steps"])
                work += B.D * len(a)
            blocks += 1
            if time.perf_counter() - t0 > seconds:
                break
        if time.perf_counter() - t0 > seconds:
            break
    el = time.perf_counter() - t0
    return dict(value=work / el, unit="basis-elems*vecs/s", cores=1, kind="oracle",
                sample=f"{blocks} blocks of the campaign (explicit basis, dense block matrix, one chain at a time), "
                       f"{el:.1f} s single-threaded Python/NumPy")


def bench_campaign(P, np, wl, cl, args):
    """Whole-cluster FTLM: every M >= 0 sector and irrep block, thermal sums."""
    T = np.geomspace(0.05, 10, 50)
    storage = {"f64": P.F64, "f32": P.F32, "f16": P.F16}[wl["storage"]]
    dist = P.GAUSSIAN if wl["dist"] == "gaussian" else P.RADEMACHER

    engine = {"auto": P.ENGINE_AUTO, "steps": P.ENGINE_STEPS, "fused": P.ENGINE_FUSED}[args.engine]

    def run(seed, cpr, eng=engine):
        return P.campaign(cl, cl.gens, wl["two_s"], wl["R"], wl["steps"], seed, T, storage=storage, dist=dist,
                          chains_per_run=cpr, engine=eng)

    for w in range(args.warmup):
        run(0x5EED0001 + 100 + w, wl["chains_per_run"])
    t0 = time.perf_counter()
    recs = [run(0x5EED0001 + k, wl["chains_per_run"]) for k in range(args.steps)]
    wall = time.perf_counter() - t0
    work = sum(r["stats"]["work"] for r in recs)
    st = recs[0]["stats"]
    progress(f"campaign: {wall / args.steps:.3f} s per run")
    engine_fields, single_fields = None, None
    if wl.get("alt_paths", True):
        other = 1 if wl["chains_per_run"] == 0 else 0          # the other path, for the speedup figure
        t1 = time.perf_counter()
        alt = run(0x5EED0001, other)
        alt_s = time.perf_counter() - t1
        # the same campaign with the per-step kernels only (no fused small-block kernel)
        run(0x5EED0001, wl["chains_per_run"], P.ENGINE_STEPS)
        t2 = time.perf_counter()
        per_step = run(0x5EED0001, wl["chains_per_run"], P.ENGINE_STEPS)
        per_step_s = time.perf_counter() - t2
        engine_fields = {"name": args.engine, "fused_blocks": st["fused_blocks"],
                         "per_step_engine_elem_vec_per_s": per_step["stats"]["work"] / per_step_s,
                         "speedup_over_per_step_engine": (work / wall) / (per_step["stats"]["work"] / per_step_s)}
        single_fields = {"this_path": "single-vector" if wl["chains_per_run"] == 1 else "batched",
                         "other_path_elem_vec_per_s": alt["stats"]["work"] / alt_s,
                         "speedup_batched_over_single":
                             (work / wall) / (alt["stats"]["work"] / alt_s) if other == 1
                             else (alt["stats"]["work"] / alt_s) / (work / wall)}
    cpu = None if args.no_cpu_baseline or not wl.get("cpu_baseline", True) else \
        oracle_campaign_rate(wl, args.cpu_seconds)
    return {
        "metric": "FTLM campaign basis-elems x vecs/s (all M >= 0 sectors and irreps, thermal sums)",
        "value": work / wall, "unit": "basis-elems*vecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": wl["storage"],
        "data": "synthetic (cluster geometry + seeded SplitMix64 start vectors)",
        "config": {"workload": wl["desc"], "sectors": st["sectors"], "blocks": st["blocks"], "rows": st["rows"],
                   "R": wl["R"], "lanczos_steps": wl["steps"], "parallelism": "single GPU"},
        "roofline": None,
        "roofline_note": wl.get("roofline_note", "every block is cache-resident (largest few MB), so an HBM "
                                                 "roofline does not bound it"),
        "cpu_baseline": cpu,
        "context": dict(wl["context"], this_run_s=wall / args.steps) if "context" in wl else None,
        "breakdown_s": {k: st[k] for k in ("seconds_build", "seconds_lanczos", "seconds_thermo", "seconds_total")},
        "engine": engine_fields,
        "single_vs_batched": single_fields,
        "E_T0.05": float(recs[0]["E"][0]), "E_T10": float(recs[0]["E"][-1]),
    }


def progress(msg):
    """One line per finished phase on stderr (long runs stay visibly alive)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="icosidodecahedron_M0", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hv-reps", type=int, default=20)
    ap.add_argument("--layout", default="auto", choices=["auto", "block", "padded", "packed", "aligned"],
                    help="rows of the Lanczos vectors inside ftlm_run (auto: the library's choice)")
    ap.add_argument("--engine", default="auto", choices=["auto", "steps", "fused"],
                    help="campaign workloads: Lanczos engine (fused small-block kernel, per-step kernels, or automatic)")
    ap.add_argument("--profile-hv", action="store_true",
                    help="counter run: one 1 GiB copy (calibration) and 5 H.V launches, then exit")
    ap.add_argument("--hv-blocks", action="store_true",
                    help="in-run H.V of every block of the workload (20 Lanczos steps each, HIP events, byte model): "
                         "one JSON line per block, then exit")
    ap.add_argument("--serve", action="store_true", help="run the job-server benchmark (serving mix) instead")
    ap.add_argument("--serve-jobs", type=int, default=100, help="jobs of the closed burst (capacity)")
    ap.add_argument("--serve-warm", type=int, default=40)
    ap.add_argument("--serve-poisson-jobs", type=int, default=500, help="arrivals of the Poisson stream")
    ap.add_argument("--serve-seconds", type=float, default=100.0,
                    help="the Poisson stream's arrivals stop after this many seconds")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving phase of the default workload")
    ap.add_argument("--serve-clusters", default=",".join(SERVE_CLUSTERS),
                    help="comma-separated clusters of the serving mix (default: the five of the mix)")
    ap.add_argument("--serve-engine", default="auto", choices=["auto", "steps"],
                    help="auto: small jobs admitted together run as fused batches; steps: per-step kernels only")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="Poisson rate in jobs/s (0: 0.8 x burst rate)")
    ap.add_argument("--serve-active", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-log", default=None, help="write one JSON record per job to this file")
    # 16 hardware queues give each server stream a queue of its own, so a short
    # job's kernels do not wait behind a long job's queued steps (serving mix:
    # short-job run p90 56 ms against 330-390 ms with the default 4 queues)
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues per process (GPU_MAX_HW_QUEUES, read when HIP starts, at most 32); "
                         "0 keeps the runtime's default")
    args = ap.parse_args()
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (sharding across GPUs is not implemented), "
                                   "so --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_17429_amd as P
    from synth import clusters

    if args.serve:
        torch.cuda.set_device(0)
        res = serve(P, np, args.serve_warm, args.serve_jobs, args.serve_rate, args.serve_budget_gb,
                    args.serve_active, log_path=args.serve_log, poisson_jobs=args.serve_poisson_jobs,
                    time_bound_s=args.serve_seconds, engine={"auto": 0, "steps": 1}[args.serve_engine],
                    names=tuple(args.serve_clusters.split(",")))
        p = res["poisson"]
        print(json.dumps({"metric": "FTLM job latency under a Poisson stream (serving mix)", "value": p["p50_ms"],
                          "unit": "ms (p50)", "n_gpus": 1, "higher_is_better": False, "dtype": "f64/f32",
                          "data": "synthetic", "config": {"workload": SERVE_DESC}, "p99_ms": p["p99_ms"],
                          "serving": res}), flush=True)
        return

    wl = WORKLOADS[args.workload]
    cl = clusters.get(wl["cluster"])
    layout = {"auto": P.LAYOUT_AUTO, "block": P.LAYOUT_BLOCK, "padded": P.LAYOUT_PADDED,
              "packed": P.LAYOUT_PACKED, "aligned": P.LAYOUT_ALIGNED}[args.layout]
    LAYOUT_NAMES = {P.LAYOUT_BLOCK: "block", P.LAYOUT_PADDED: "padded", P.LAYOUT_PACKED: "packed",
                    P.LAYOUT_ALIGNED: "aligned"}
    if wl.get("campaign"):
        torch.cuda.set_device(0)
        print(json.dumps(bench_campaign(P, np, wl, cl, args)), flush=True)
        return
    storage = {"f64": P.F64, "f32": P.F32, "f16": P.F16}[wl["storage"]]
    dist = P.GAUSSIAN if wl["dist"] == "gaussian" else P.RADEMACHER
    T = np.geomspace(0.05, 10, 50)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    rirrep = roofline_irrep(wl)

    def job(seed, st=storage):
        """One whole job: group, sector, every block of the workload (R chains
        each, per-block HIP-event timing of the H.V launches), Ritz data and the
        thermal sums over all blocks."""
        t0 = time.perf_counter()
        G = P.Group(cl.N, cl.gens)
        S = P.Sector(cl, G, wl["two_M"], two_s=wl["two_s"], spin_flip=wl.get("flip", False))
        t1 = time.perf_counter()
        irreps = list(range(G.n_irreps)) if wl["irrep"] == "all" else [wl["irrep"]]
        runs, hv = [], None
        for gi in irreps:
            B = P.Block(S, gi, 0, layout=layout)
            if B.D == 0:
                continue
            a, b, n, info = B.ftlm(wl["R"], wl["steps"], seed, storage=st, dist=dist, stream=stream, info=True)
            runs.append((B.D, B.trace_weight, a, b, n))
            if gi == rirrep:
                hv = dict(info, D=B.D)
            del B
        t2 = time.perf_counter()
        blocks = []
        for D, wt, a, b, n in runs:
            ths, ws = P.ritz_from_run(a, b, n)
            blocks.append(dict(two_M=wl["two_M"], d_gamma=wt, D=D, thetas=ths, weights=ws))
        E, C, chi, lz = P.observables(blocks, T)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return dict(work=sum(D * int(n.sum()) for D, _, _, _, n in runs), rows=sum(r[0] for r in runs),
                    blocks=len(runs), build=t1 - t0, lanczos=t2 - t1, thermo=t3 - t2, total=t3 - t0,
                    E0=float(min(t.min() for bl in blocks for t in bl["thetas"])),
                    Emax=float(max(t.max() for bl in blocks for t in bl["thetas"])),
                    hv_ms=hv["hv_ms"], hv_launches=hv["hv_launches"], layout=hv["layout"], hv_D=hv["D"],
                    E=E, C=C, chi=chi)

    def tune_all():
        """Autotune the H.V lane layout once per irrep dimension bucket of the
        workload (cached process-wide; untimed)."""
        G0 = P.Group(cl.N, cl.gens)
        S0 = P.Sector(cl, G0, wl["two_M"], two_s=wl["two_s"], spin_flip=wl.get("flip", False))
        irreps = list(range(G0.n_irreps)) if wl["irrep"] == "all" else [wl["irrep"]]
        # with spin flip the irrep index counts the irreps of G x Z2, so the
        # dimension buckets of G do not apply: tune every listed block
        dims = None if wl.get("flip") else G0.irreps()["dims"]
        seen, out = set(), None
        for gi in irreps:
            if dims is not None:
                if dims[gi] in seen and gi != rirrep:
                    continue
                seen.add(dims[gi])
            B0 = P.Block(S0, gi, 0, layout=layout)
            if B0.D == 0:
                continue
            t = B0.autotune(wl["R"], storage, stream=stream)
            if gi == rirrep:
                out = t
        return out, S0, G0

    if args.profile_hv:
        tuned, S0, G0 = tune_all()
        B0 = P.Block(S0, rirrep, 0, layout=layout)
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                     # calibration: reads and writes 1 GiB
        del src, dst
        torch.cuda.synchronize()
        # the H.V launches the counters see are those of 5 Lanczos steps
        _, _, _, info = B0.ftlm(wl["R"], 5, 0x5EED0003, storage=storage, dist=dist, stream=stream, info=True)
        torch.cuda.synchronize()
        st = B0.hv_stats()
        elem = {P.F64: 8, P.F32: 4, P.F16: 2}[storage]
        pad = info["layout"] in (P.LAYOUT_PADDED, P.LAYOUT_PACKED, P.LAYOUT_ALIGNED)
        print(json.dumps({"copy_bytes": 1 << 30, "hv_launches": info["hv_launches"], "lanes_per_rep": tuned[0],
                          "layout": LAYOUT_NAMES[info["layout"]], "nvec": wl["R"], "elem_bytes": elem,
                          "rows": info["rows"], "avg_launch_ms": info["hv_ms"] / max(info["hv_launches"], 1),
                          "algorithmic_bytes_per_launch": algorithmic_bytes(st, B0.D, S0.n_reps, wl["R"], elem,
                                                                            pad=pad, epilogue=True),
                          "stats": st}), flush=True)
        return

    if args.hv_blocks:
        # every block of the workload: lanes from the autotuner, then the
        # H.V launches of a 20-step run timed on the run's stream
        G1 = P.Group(cl.N, cl.gens)
        S1 = P.Sector(cl, G1, wl["two_M"], two_s=wl["two_s"], spin_flip=wl.get("flip", False))
        n_ir = 2 * G1.n_irreps if wl.get("flip") else G1.n_irreps
        elem = {P.F64: 8, P.F32: 4, P.F16: 2}[storage]
        for gi in (range(n_ir) if wl["irrep"] == "all" else [wl["irrep"]]):
            B1 = P.Block(S1, gi, 0, layout=layout)
            if B1.D == 0:
                continue
            t = B1.autotune(wl["R"], storage, stream=stream)
            _, _, _, info = B1.ftlm(wl["R"], 20, 0x5EED0003, storage=storage, dist=dist, stream=stream, info=True)
            torch.cuda.synchronize()
            ms = info["hv_ms"] / max(info["hv_launches"], 1)
            ab = algorithmic_bytes(B1.hv_stats(), B1.D, S1.n_reps, wl["R"], elem,
                                   pad=info["layout"] != P.LAYOUT_BLOCK, epilogue=True)
            print(json.dumps({"irrep": gi, "d_gamma": B1.d_gamma, "D": B1.D, "lanes_per_rep": t[0],
                              "layout": LAYOUT_NAMES[info["layout"]], "avg_launch_ms": ms,
                              "algorithmic_bytes_per_launch": ab, "achieved_GBs": ab / ms / 1e6,
                              "frac": ab / ms / 1e6 / PEAK_HBM_GBS}), flush=True)
            del B1
        return

    tuned, S0, G0 = tune_all()
    del S0, G0
    progress(f"tuned: {tuned[0]} lanes per representative on the roofline block")
    for w in range(args.warmup):
        job(0x5EED0003 + 1000 + w)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(job(0x5EED0003 + k))
        progress(f"step {k + 1}/{args.steps}: {recs[-1]['total'] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    work = sum(r["work"] for r in recs)
    value = work / wall
    lat = np.array([r["total"] for r in recs]) * 1e3

    # ---- H.V kernel alone on the roofline block: nvec = R, storage dtype, HIP events on the launch stream
    G = P.Group(cl.N, cl.gens)
    S = P.Sector(cl, G, wl["two_M"], two_s=wl["two_s"], spin_flip=wl.get("flip", False))
    B = P.Block(S, rirrep, 0, layout=layout)
    gorder, hv_D = B.group_order, B.D
    tdt = {P.F64: torch.float64, P.F32: torch.float32, P.F16: torch.float16}[storage]
    elem = {P.F64: 8, P.F32: 4, P.F16: 2}[storage]
    X = torch.randn((B.D, wl["R"]), dtype=tdt, device=dev)
    Y = torch.empty_like(X)
    for _ in range(3):
        B.apply_H(X, Y, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.hv_reps):
        B.apply_H(X, Y, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    hv_ms = ev0.elapsed_time(ev1) / args.hv_reps
    stats = B.hv_stats()
    # roofline: the H.V launches of the timed runs on the roofline block (HIP events on the run's stream)
    pad = recs[0]["layout"] in (P.LAYOUT_PADDED, P.LAYOUT_PACKED, P.LAYOUT_ALIGNED)
    lz_launches = sum(r["hv_launches"] for r in recs)
    lz_hv_ms = sum(r["hv_ms"] for r in recs) / max(lz_launches, 1)
    balg = algorithmic_bytes(stats, B.D, S.n_reps, wl["R"], elem, pad=pad, epilogue=True)
    achieved = balg / (lz_hv_ms * 1e-3) / 1e9
    bmin = 3 * B.D * wl["R"] * elem + 32 * stats["n_active"] + 8 * (S.n_reps - stats["n_active"])
    balg_apply = algorithmic_bytes(stats, B.D, S.n_reps, wl["R"], elem)
    # plain single-vector FP64 H.V for the speedup figure
    del X, Y
    X1 = torch.randn((B.D, 1), dtype=torch.float64, device=dev)
    Y1 = torch.empty_like(X1)
    B.apply_H(X1, Y1, stream=stream)
    ev0.record(stream)
    for _ in range(5):
        B.apply_H(X1, Y1, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    hv1_ms = ev0.elapsed_time(ev1) / 5
    del X1, Y1
    # the on-the-fly H.V (flips canonicalised and looked up inside the kernel,
    # no entry table) on the same block, nvec = R, block rows
    otf = None
    if wl.get("otf_timing", True):
        So = P.Sector(cl, G, wl["two_M"], hv_mode=P.HV_ONTHEFLY, two_s=wl["two_s"], spin_flip=wl.get("flip", False))
        Bo = P.Block(So, rirrep, 0)
        Xo = torch.randn((Bo.D, wl["R"]), dtype=tdt, device=dev)
        Yo = torch.empty_like(Xo)
        Bo.apply_H(Xo, Yo, stream=stream)
        ev0.record(stream)
        for _ in range(3):
            Bo.apply_H(Xo, Yo, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        otf_ms = ev0.elapsed_time(ev1) / 3
        otf = {"ms": otf_ms, "elem_vec_per_s": Bo.D * wl["R"] / (otf_ms * 1e-3), "vs_entries": otf_ms / hv_ms,
               "sector_device_bytes": So.device_bytes}
        del Xo, Yo, Bo, So
    torch.cuda.empty_cache()        # the library allocates the runs below itself

    progress(f"H.V alone: {hv_ms:.3f} ms (nvec {wl['R']}), single FP64 {hv1_ms:.3f} ms"
             + (f", on the fly {otf['ms']:.3f} ms" if otf else ""))
    # the second workload on the same H.V: KPM moments (2 per product) for the
    # same R start vectors, window from the Ritz values widened by 5%
    kpm = None
    if storage in (P.F64, P.F32):
        lo, hi = recs[0]["E0"], recs[0]["Emax"]
        kc, kw = 0.5 * (lo + hi), 0.525 * (hi - lo)
        n_mom = 2 * wl["steps"] + 1
        B.kpm(wl["R"], 3, 1, kc, kw, storage=storage, dist=dist, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.kpm(wl["R"], n_mom, 0x5EED0003, kc, kw, storage=storage, dist=dist, stream=stream)
        torch.cuda.synchronize()
        kt = time.perf_counter() - t0
        progress(f"KPM: {n_mom} moments in {kt:.2f} s")
        kpm = {"moments": n_mom, "hv_products": wl["steps"], "seconds": kt,
               "elem_vec_per_s": B.D * wl["R"] * wl["steps"] / kt, "center": kc, "half_width": kw}
    del B, S, G
    torch.cuda.empty_cache()

    # the error of the observables of the storage precision against the FP64
    # path: the first timed job again in FP64 (same keys), per temperature
    # (not for the s=3/2 dodecahedron, whose FP64 vectors do not fit next to its tables)
    obs_err = None
    if storage != P.F64 and wl.get("fp64_check", True):
        progress("FP64 rerun of the first job")
        r64 = job(0x5EED0003, P.F64)
        # chi vanishes identically when only M = 0 enters: compare it absolutely then
        keys = [k for k in ("E", "C", "chi") if np.all(np.abs(r64[k]) > 0)]
        rel = {k: np.abs(recs[0][k] - r64[k]) / np.abs(r64[k]) for k in keys}
        obs_err = {"reference": "the same job with FP64 storage (same chains and keys)",
                   "max_rel": {k: float(v.max()) for k, v in rel.items()},
                   "per_T": {f"{T[i]:.4g}": {k: float(rel[k][i]) for k in rel} for i in range(0, len(T), 7)},
                   "E0_fp64": r64["E0"], "E0_storage": recs[0]["E0"]}
        for k in ("E", "C", "chi"):
            if k not in rel:
                obs_err[f"max_abs_{k}"] = float(np.max(np.abs(recs[0][k] - r64[k])))

    # HBM bytes per launch from the committed counter summary, valid only while
    # the kernel source is the one the counters were taken on
    from paper_2607_17429_amd.profiling import hv_source_sha
    traffic = None
    tp = os.path.join(ROOT, "profiles", f"hv_traffic_{args.workload}.json")
    if os.path.exists(tp):
        tj = json.load(open(tp))
        if tj.get("source_sha") == hv_source_sha():
            traffic = tj.get("bytes_per_launch")

    serving = None
    if not args.no_serve and wl is WORKLOADS["icosidodecahedron_M0"]:
        serving = serve(P, np, args.serve_warm, args.serve_jobs, args.serve_rate, args.serve_budget_gb,
                        args.serve_active, log_path=args.serve_log, poisson_jobs=args.serve_poisson_jobs,
                        time_bound_s=args.serve_seconds, engine={"auto": 0, "steps": 1}[args.serve_engine],
                    names=tuple(args.serve_clusters.split(",")))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(dict(wl, irrep=rirrep), args.cpu_seconds)

    out = {
        "metric": "sym-adapted H.V basis-elems x vecs/s (whole FTLM job), % HBM roofline of H.V; job p50/p99 latency",
        "value": value,
        "unit": "basis-elems*vecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["storage"],
        "data": "synthetic (cluster geometry + seeded SplitMix64 start vectors)",
        "config": {"workload": wl["desc"], "blocks": recs[0]["blocks"], "rows": recs[0]["rows"], "R": wl["R"],
                   "lanczos_steps": wl["steps"], "roofline_block": f"irrep {rirrep} (D={hv_D})",
                   "group_order": gorder, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": f"k_hv inside ftlm_run on the irrep-{rirrep} block (entry-table mode, Lanczos epilogue, "
                               + LAYOUT_NAMES[recs[0]["layout"]] + " rows)",
                     "algorithmic_bytes_per_launch": balg, "avg_launch_ms": lz_hv_ms, "launches": lz_launches,
                     "nvec": wl["R"],
                     # X read once (every row), Y written, the previous vector read by the
                     # epilogue, per-representative data streamed once: no gather re-reads
                     "compulsory_bytes_per_launch": bmin,
                     "compulsory_frac": bmin / (lz_hv_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "cpu_baseline": cpu,
        "speedup_vs_oracle": value / cpu["value"] if cpu else None,
        "context": dict(wl["context"], this_job_s=float(np.mean([r["total"] for r in recs]))) if "context" in wl else None,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "of": "whole jobs of this workload (the timed steps)"},
        "breakdown_ms": {k: float(np.mean([r[k] for r in recs]) * 1e3) for k in ("build", "lanczos", "thermo")},
        "hv": {"apply_H_ms": hv_ms, "apply_H_GBs": balg_apply / (hv_ms * 1e-3) / 1e9,
               "batched_elem_vec_per_s": hv_D * wl["R"] / (hv_ms * 1e-3),
               "single_fp64_elem_vec_per_s": hv_D / (hv1_ms * 1e-3), "single_fp64_ms": hv1_ms,
               "speedup_batched_over_single_fp64": (hv_D * wl["R"] / (hv_ms * 1e-3)) / (hv_D / (hv1_ms * 1e-3)),
               "connections": stats["connections"], "active_connections": stats["active_connections"],
               "on_the_fly": otf},
        "observables_vs_fp64": obs_err,
        "serving": serving,
        "kpm": kpm,
        "E0": recs[0]["E0"],
        "autotune": {"lanes_per_rep": tuned[0], "ms": tuned[1], "tried_ms": tuned[2]} if tuned else None,
    }
    print(json.dumps(out), flush=True)


def roofline_irrep(wl):
    return wl["roofline_irrep"] if wl["irrep"] == "all" else wl["irrep"]


if __name__ == "__main__":
    main()
