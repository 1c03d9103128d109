"""GPU tests of the continuous-batching job server (include/ftlm_server.h).

A job's Lanczos coefficients must not depend on what else runs: every job of a
mixed batch (several clusters, M sectors, irreps, rows, R, storage types and
start-vector distributions, admitted up to four at a time and overlapping on
the device) is compared bit for bit with the same block run alone through
ftlm_run, or through ftlm_run_fused for the jobs the server ran in the fused
small-block kernel (the engine each job reports); both engines are also forced
on the whole mix.  The standalone path is itself compared with the oracle in
test_gpu_ftlm.py; one server job is also checked against the oracle here.
Admission by memory budget, cancellation and failing jobs are covered too.
"""
import numpy as np
import pytest

from gpu_helpers import lib_group, lib_sector, log, oracle_block, oracle_sector
from oracle import ftlm as oftlm
from synth import clusters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2607_17429_amd")

# (cluster, 2M, irrep, row, R, steps, seed, storage, dist)
MIX = [
    ("icosahedron", 0, 0, 0, 4, 40, 11, "f64", "rad"),
    ("icosahedron", 2, 8, 2, 6, 30, 12, "f32", "gau"),
    ("dodecahedron", 0, 8, 1, 8, 50, 13, "f32", "rad"),
    ("dodecahedron", 2, 3, 0, 5, 60, 14, "f64", "gau"),
    ("cuboctahedron", 0, 9, 2, 3, 40, 15, "f64", "rad"),
    ("cuboctahedron", 4, 4, 1, 7, 25, 16, "f32", "rad"),
    ("square4x4", 0, 0, 0, 4, 40, 17, "f64", "rad"),
    ("square4x4", 2, 10, 1, 9, 35, 18, "f32", "gau"),
    ("ring12", 0, 2, 0, 2, 30, 19, "f64", "rad"),
    ("dodecahedron", 0, 8, 4, 24, 60, 20, "f32", "gau"),
    ("icosahedron", 0, 0, 0, 4, 40, 11, "f64", "rad"),   # repeat of the first job
    ("dodecahedron", 4, 9, 0, 3, 45, 21, "f64", "rad"),
]

ST = {"f64": None, "f32": None}
DI = {"rad": None, "gau": None}


def _enums():
    ST.update(f64=P.F64, f32=P.F32)
    DI.update(rad=P.RADEMACHER, gau=P.GAUSSIAN)


def _valid(job):
    name, two_M, gi, row = job[:4]
    dims = lib_group(name).irreps()["dims"]
    return gi < len(dims) and row < dims[gi]


def _standalone(job, engine=None):
    """The same block alone: ftlm_run, or ftlm_run_fused for jobs the server
    ran in the fused small-block kernel."""
    name, two_M, gi, row, R, steps, seed, st, di = job
    B = P.Block(lib_sector(name, 1, two_M), gi, row)
    if engine == P.ENGINE_FUSED:
        (a, b, n), = P.run_fused([dict(block=B, R=R, steps=steps, seed=seed, storage=ST[st], dist=DI[di])])
        return a, b, n
    return B.ftlm(R, steps, seed, storage=ST[st], dist=DI[di])


def _submit(srv, job, engine=0):
    name, two_M, gi, row, R, steps, seed, st, di = job
    cl = clusters.get(name)
    return srv.submit(cl, cl.gens, two_M, gi, row, R, steps, seed, storage=ST[st], dist=DI[di], two_s=1,
                      engine=engine)


def test_mixed_jobs_match_standalone_bitwise():
    _enums()
    for job in MIX:
        assert _valid(job), job
    log("[server] mixed batch of %d jobs, max_active=4" % len(MIX))
    srv = P.Server(8 << 30, max_active=4)
    ids = [_submit(srv, job) for job in MIX]
    results = [srv.wait(i) for i in ids]
    srv.close()
    engines = []
    for job, (res, a, b, n) in zip(MIX, results):
        assert res["status"] == 0, (job, res)
        assert res["submit_s"] <= res["start_s"] <= res["end_s"]
        engines.append(res["engine"])
        a0, b0, n0 = _standalone(job, res["engine"])
        assert np.array_equal(n, n0), job
        assert np.array_equal(a, a0), job
        assert np.array_equal(b, b0), job
    # the repeated job gives the same numbers when it takes the same engine
    if engines[0] == engines[10]:
        assert np.array_equal(results[0][1], results[10][1])
    # submitted together, the small jobs were batched into the fused kernel
    # and the large ones ran the per-step kernels
    assert P.ENGINE_FUSED in engines and P.ENGINE_STEPS in engines


def test_lone_small_job_runs_per_step_kernels():
    """A small job admitted alone takes the per-step kernels (faster for one
    job); its coefficients equal ftlm_run's bit for bit."""
    _enums()
    job = ("icosahedron", 0, 8, 1, 4, 40, 77, "f64", "rad")
    srv = P.Server(1 << 30, max_active=4)
    res, a, b, n = srv.wait(_submit(srv, job))
    srv.close()
    assert res["status"] == 0 and res["engine"] == P.ENGINE_STEPS
    a0, b0, n0 = _standalone(job, P.ENGINE_STEPS)
    assert np.array_equal(a, a0) and np.array_equal(b, b0) and np.array_equal(n, n0)


def test_large_job_is_not_starved_by_small_ones():
    """A job that does not fit next to running jobs is overtaken by at most 64
    later jobs; then nothing behind it is admitted until it is.  The budget is
    set so that the large job fits only when no other job runs (the admission
    estimate of the server, restated here), and a stream of 300 small jobs
    queues behind it while a long job holds memory."""
    _enums()
    log("[server] starvation bound")
    dodec, ico = clusters.get("dodecahedron"), clusters.get("icosahedron")
    G = lib_group("dodecahedron")
    Gi = lib_group("icosahedron")
    # resident sector bytes (entry tables, as the server builds them)
    s_dod = P.Sector(dodec, G, 0, two_s=1, hv_mode=P.HV_ENTRIES)
    s_ico = P.Sector(ico, Gi, 0, two_s=1, hv_mode=P.HV_ENTRIES)
    used0 = s_dod.device_bytes + s_ico.device_bytes
    # the server's estimate for (dodecahedron M=0, H_g, R=32, 20 steps, FP64)
    n_reps, dg, R, steps = s_dod.n_reps, 5, 32, 20
    big_est = n_reps * 16 + 2 * n_reps * dg * R * 8 + 8192 * R * 8 + R * steps * 16 + (1 << 20)
    del s_dod, s_ico
    srv = P.Server(used0 + big_est + (64 << 10), max_active=4)
    # warm both sectors
    for cl, gi in ((dodec, 0), (ico, 0)):
        r, *_ = srv.wait(srv.submit(cl, cl.gens, 0, gi, 0, 2, 5, 1, storage=P.F64, two_s=1))
        assert r["status"] == 0
    assert srv.stats()["used_bytes"] == used0
    hold = srv.submit(dodec, dodec.gens, 0, 8, 0, 4, 3000, 2, storage=P.F64, two_s=1)   # long, holds memory
    big = srv.submit(dodec, dodec.gens, 0, 8, 0, R, steps, 3, storage=P.F64, two_s=1)
    smalls = [srv.submit(ico, ico.gens, 0, 0, 0, 4, 60, 100 + k, storage=P.F64, two_s=1) for k in range(300)]
    rb, *_ = srv.wait(big)
    rs = [srv.wait(i)[0] for i in smalls]
    rh, *_ = srv.wait(hold)
    srv.close()
    assert rb["status"] == 0 and rh["status"] == 0 and all(r["status"] == 0 for r in rs)
    before = sum(r["start_s"] < rb["start_s"] for r in rs)
    log(f"  small jobs admitted before the large one: {before}")
    assert 1 <= before <= 64
    assert rb["start_s"] >= rh["submit_s"]


@pytest.mark.parametrize("engine", ["steps", "fused"])
def test_forced_engine_matches_standalone_bitwise(engine):
    _enums()
    eng = P.ENGINE_STEPS if engine == "steps" else P.ENGINE_FUSED
    jobs = [j for j in MIX if j[4] <= 32 and not (j[0] == "dodecahedron" and j[1] == 0 and engine == "fused")]
    srv = P.Server(8 << 30, max_active=4)
    ids = [_submit(srv, job, eng) for job in jobs]
    results = [srv.wait(i) for i in ids]
    srv.close()
    for job, (res, a, b, n) in zip(jobs, results):
        assert res["status"] == 0 and res["engine"] == eng, (job, res)
        a0, b0, n0 = _standalone(job, eng)
        assert np.array_equal(n, n0) and np.array_equal(a, a0) and np.array_equal(b, b0), job


def test_forced_fused_engine_rejects_unfit_jobs():
    _enums()
    cl = clusters.get("icosahedron")
    srv = P.Server(1 << 30, max_active=2)
    jid = srv.submit(cl, cl.gens, 0, 0, 0, 40, 20, 1, storage=P.F64, two_s=1, engine=P.ENGINE_FUSED)  # R > 32
    res, a, *_ = srv.wait(jid)
    assert res["error"] == "INVALID_ARG" and a is None
    srv.close()


def test_server_job_against_oracle():
    _enums()
    # a one-dimensional irrep (A_g): its matrices are its characters, so the
    # library's block basis is the oracle's and the runs agree up to rounding
    name, two_M, gi = "dodecahedron", 0, 0
    assert lib_group(name).irreps()["dims"][gi] == 1
    srv = P.Server(1 << 30, max_active=2)
    cl = clusters.get(name)
    jid = srv.submit(cl, cl.gens, two_M, gi, 0, 3, 40, 99, storage=P.F64, dist=P.RADEMACHER, two_s=1)
    res, a, b, n = srv.wait(jid)
    srv.close()
    assert res["status"] == 0 and res["d_gamma"] == 1
    sec, H = oracle_sector(name, 1, two_M)
    B = oracle_block(name, 1, two_M, gi)
    assert res["D"] == B.D
    Hb = (B.Psi.T @ H @ B.Psi).tocsr()
    for r in range(3):
        v0 = oftlm.start_vector(B.D, 99, two_M, gi, 0, r, "rademacher")
        oa, ob = oftlm.lanczos(lambda x: Hb @ x, v0, 40)
        assert np.max(np.abs(a[r, :15] - oa[:15])) < 1e-10 * np.max(np.abs(oa))
        assert np.max(np.abs(b[r, :15] - ob[:15])) < 1e-10 * np.max(np.abs(ob))


def test_budget_cancel_and_failures():
    _enums()
    log("[server] budget / cancel / failing jobs")
    cl = clusters.get("dodecahedron")
    # a budget below any footprint: the job fails with OUT_OF_MEMORY, the server keeps going
    srv = P.Server(1 << 16, max_active=2)
    jid = srv.submit(cl, cl.gens, 0, 8, 0, 4, 20, 1, storage=P.F64, two_s=1)
    res, a, *_ = srv.wait(jid)
    assert res["error"] == "OUT_OF_MEMORY" and a is None
    srv.close()

    srv = P.Server(2 << 30, max_active=1)
    bad_irrep = srv.submit(cl, cl.gens, 0, 99, 0, 4, 20, 1, two_s=1)
    bad_row = srv.submit(cl, cl.gens, 0, 8, 7, 4, 20, 1, two_s=1)
    big = srv.submit(cl, cl.gens, 0, 8, 0, 32, 200, 2, storage=P.F64, two_s=1)
    queued = [srv.submit(cl, cl.gens, 2, 3, 0, 4, 30, 3 + k, two_s=1) for k in range(4)]
    srv.cancel(queued[1])
    out = {k: srv.wait(j) for k, j in [("bad_irrep", bad_irrep), ("bad_row", bad_row), ("big", big)]}
    assert out["bad_irrep"][0]["error"] == "IRREP_OUT_OF_RANGE"
    assert out["bad_row"][0]["error"] == "ROW_OUT_OF_RANGE"
    assert out["big"][0]["status"] == 0
    rq = [srv.wait(j) for j in queued]
    assert rq[1][0]["error"] == "CANCELLED"
    for k in (0, 2, 3):
        assert rq[k][0]["status"] == 0
        job = ("dodecahedron", 2, 3, 0, 4, 30, 3 + k, "f64", "rad")
        a0, b0, n0 = _standalone(job, rq[k][0]["engine"])
        assert np.array_equal(rq[k][1], a0) and np.array_equal(rq[k][2], b0)
    st = srv.stats()
    assert st["running"] == 0 and st["queued"] == 0
    assert st["used_bytes"] > 0          # the cached sectors stay resident
    with pytest.raises(P.FtlmError):
        srv.wait(big)                    # already released
    srv.close()


def test_free_with_jobs_in_flight():
    _enums()
    cl = clusters.get("icosahedron")
    srv = P.Server(1 << 30, max_active=2)
    for k in range(6):
        srv.submit(cl, cl.gens, 0, 0, 0, 4, 30, k, two_s=1)
    srv.close()                          # cancels queued jobs, drains running ones


def test_long_job_fed_in_chunks_matches_standalone():
    """A job whose steps are fed to the device in several chunks (the H_g block
    of the icosidodecahedron, D = 6,465,762) next to small jobs gives the same
    coefficients, bit for bit, as one ftlm_run call."""
    _enums()
    log("[server] chunked long job")
    big = ("icosidodecahedron", 0, 8, 0, 8, 20, 31, "f32", "gau")
    small = [("icosahedron", 0, 8, 1, 4, 40, 32 + k, "f64", "rad") for k in range(6)]
    srv = P.Server(16 << 30, max_active=4)
    ids = [_submit(srv, big)] + [_submit(srv, j) for j in small]
    res = [srv.wait(i) for i in ids]
    srv.close()
    assert res[0][0]["D"] == 6465762
    for job, (r, a, b, n) in zip([big] + small, res):
        assert r["status"] == 0, (job, r)
        a0, b0, n0 = _standalone(job, r["engine"])
        assert np.array_equal(n, n0) and np.array_equal(a, a0) and np.array_equal(b, b0), job


def test_long_step_jobs_leave_slots_to_short_ones():
    """With max_active = 3, jobs with long steps (the icosidodecahedron H_g
    block, about 2 ms of estimated device time per step) take at most one
    slot: the second one starts only after the first has ended, while short
    jobs submitted behind both run meanwhile.  Every result equals the same
    run alone, bit for bit."""
    _enums()
    log("[server] slots for short jobs")
    long_jobs = [("icosidodecahedron", 0, 8, 0, 8, 200, 41 + k, "f32", "gau") for k in range(2)]
    short = [("icosahedron", 0, 8, 1, 4, 40, 50 + k, "f64", "rad") for k in range(30)]
    srv = P.Server(16 << 30, max_active=3)
    ids = [_submit(srv, j) for j in long_jobs] + [_submit(srv, j) for j in short]
    res = [srv.wait(i) for i in ids]
    srv.close()
    (r0, *_), (r1, *_) = res[0], res[1]
    assert r0["status"] == 0 and r1["status"] == 0
    assert r1["start_s"] >= r0["end_s"], (r0, r1)
    during = sum(r[0]["start_s"] < r0["end_s"] for r in res[2:])
    log(f"  short jobs started while the first long job ran: {during} of {len(short)}")
    assert during >= 1
    for job, (r, a, b, n) in zip(long_jobs + short, res):
        assert r["status"] == 0, (job, r)
        a0, b0, n0 = _standalone(job, r["engine"])
        assert np.array_equal(n, n0) and np.array_equal(a, a0) and np.array_equal(b, b0), job
