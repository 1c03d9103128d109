"""Python face of the continuous-batching job server (include/ftlm_server.h)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import F64, RADEMACHER, check, lib


class Server:
    """Admits FTLM block jobs by device footprint; jobs overlap on the GPU."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 8):
        h = C.c_void_p()
        check(lib().ftlm_server_create(int(hbm_budget_bytes), int(max_active), C.byref(h)))
        self._h = h
        self._free = lib().ftlm_server_free
        self._keep = {}

    def submit(self, cluster, gens, two_M, irrep, row, R, steps, seed, storage=F64, dist=RADEMACHER, two_s=None,
               engine=0):
        cl = L.make_cluster(cluster.N, two_s if two_s is not None else getattr(cluster, "two_s", 1),
                            cluster.bonds, cluster.J)
        g = np.ascontiguousarray(np.asarray(gens, dtype=np.int32).reshape(-1, cluster.N))
        d = L.JobDesc(cl, g.ctypes.data_as(L.I32P), len(g), int(two_M), int(irrep), int(row), int(R), int(steps),
                      C.c_uint64(seed), int(storage), int(dist), int(engine), 0)
        jid = C.c_int64()
        check(lib().ftlm_server_submit(self._h, C.byref(d), C.byref(jid)))   # arrays are copied
        self._keep[jid.value] = (R, steps)
        return jid.value

    def poll(self, jid) -> bool:
        done = C.c_int32()
        check(lib().ftlm_server_poll(self._h, C.c_int64(jid), C.byref(done)))
        return bool(done.value)

    def wait(self, jid):
        """-> (result dict, alpha, beta, nsteps); raises FtlmError for a failed job."""
        if jid not in self._keep:
            raise L.FtlmError(-1, f"unknown or already released job id {jid}")
        R, steps = self._keep.pop(jid)
        res = L.JobResult()
        alpha = np.zeros((R, steps))
        beta = np.zeros((R, steps))
        ns = np.zeros(R, np.int32)
        rc = lib().ftlm_server_wait(self._h, C.c_int64(jid), C.byref(res), alpha.ctypes.data_as(L.F64P),
                                    beta.ctypes.data_as(L.F64P), ns.ctypes.data_as(L.I32P))
        out = {f: getattr(res, f) for f, _ in L.JobResult._fields_}
        if rc != 0:
            out["error"] = L.STATUS.get(rc, rc)
            msg = lib().ftlm_last_error()
            out["message"] = msg.decode() if msg else ""
            return out, None, None, None
        return out, alpha, beta, ns

    def cancel(self, jid):
        check(lib().ftlm_server_cancel(self._h, C.c_int64(jid)))

    def stats(self):
        u, r, q = C.c_int64(), C.c_int32(), C.c_int32()
        check(lib().ftlm_server_stats(self._h, C.byref(u), C.byref(r), C.byref(q)))
        return dict(used_bytes=u.value, running=r.value, queued=q.value)

    def close(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()
