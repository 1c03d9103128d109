"""Python face of the C ABI: the same calls, with numpy / torch arguments.

Device arrays are torch CUDA tensors (PyTorch supplies device memory and the
stream); every computation happens in ``libftlm.so``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import F16, F32, F64, GAUSSIAN, HV_AUTO, HV_ENTRIES, HV_ONTHEFLY, RADEMACHER, FtlmError, check, lib


class Group:
    """Closure of site-permutation generators and its real irreps."""

    def __init__(self, N, gens):
        gens = np.ascontiguousarray(np.asarray(gens, dtype=np.int32).reshape(-1, N))
        h = C.c_void_p()
        check(lib().ftlm_group_create(int(N), gens.ctypes.data_as(L.I32P), len(gens), C.byref(h)))
        self._h = h
        self._free = lib().ftlm_group_free
        o, ni, nc, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().ftlm_group_info(h, C.byref(o), C.byref(ni), C.byref(nc), C.byref(n)))
        self.order, self.n_irreps, self.n_classes, self.N = o.value, ni.value, nc.value, n.value

    def __del__(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def elements(self):
        out = np.empty((self.order, self.N), dtype=np.int32)
        check(lib().ftlm_group_elements(self._h, out.ctypes.data_as(L.I32P)))
        return out

    def irreps(self):
        n = self.n_irreps
        dims = np.empty(n, np.int32)
        ind = np.empty(n, np.int32)
        weights = np.empty(n, np.int32)
        chars = np.empty((n, self.n_classes))
        cls = np.empty(self.order, np.int32)
        res = C.c_double()
        check(lib().ftlm_group_irreps(self._h, dims.ctypes.data_as(L.I32P), ind.ctypes.data_as(L.I32P),
                                      weights.ctypes.data_as(L.I32P), chars.ctypes.data_as(L.F64P),
                                      cls.ctypes.data_as(L.I32P), C.byref(res)))
        return dict(dims=dims, indicators=ind, weights=weights, chars=chars, class_of=cls, residual=res.value)

    def rho(self, irrep):
        d = int(self.irreps()["dims"][irrep])
        out = np.empty((self.order, d, d))
        check(lib().ftlm_group_rho(self._h, int(irrep), out.ctypes.data_as(L.F64P)))
        return out


class Sector:
    """Irrep-independent tables of one M sector (built on the GPU)."""

    def __init__(self, cluster, group: Group, two_M, hv_mode=HV_AUTO, hbm_limit=0, two_s=None, entry_format=0,
                 spin_flip=False):
        cl = L.make_cluster(cluster.N, two_s if two_s is not None else cluster.two_s, cluster.bonds, cluster.J) \
            if not isinstance(cluster, L.Cluster) else cluster
        self._cl = cl
        self.group = group
        opts = L.make_opts(hv_mode=hv_mode, hbm_limit=hbm_limit, entry_format=entry_format, spin_flip=spin_flip)
        h = C.c_void_p()
        check(lib().ftlm_sector_create(C.byref(cl), group._h, int(two_M), C.byref(opts), C.byref(h)))
        self._h = h
        self._free = lib().ftlm_sector_free
        self.two_M = int(two_M)
        info = L.SectorInfo()
        check(lib().ftlm_sector_info_get(h, C.byref(info)))
        self.D_M, self.n_reps, self.n_entries = info.D_M, info.n_reps, info.n_entries
        self.n_stab, self.label_bits, self.device_bytes = info.n_stab, info.label_bits, info.device_bytes

    def __del__(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def export(self):
        reps = np.empty(self.n_reps, np.uint64)
        sid = np.empty(self.n_reps, np.uint16)
        ssz = np.empty(max(self.n_stab, 1), np.int32)
        check(lib().ftlm_sector_export(self._h, reps.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       sid.ctypes.data_as(C.POINTER(C.c_uint16)), ssz.ctypes.data_as(L.I32P)))
        return reps, sid, ssz[: self.n_stab]

    def canonicalize(self, labels, stream=None):
        """labels: torch uint64/int64 CUDA tensor -> (rep, h, index) CUDA tensors."""
        import torch
        labels = labels.contiguous()
        n = labels.numel()
        rep = torch.empty(n, dtype=torch.int64, device=labels.device)
        h = torch.empty(n, dtype=torch.int32, device=labels.device)
        idx = torch.empty(n, dtype=torch.int64, device=labels.device)
        check(lib().ftlm_sector_canonicalize(self._h, C.c_void_p(labels.data_ptr()), n, C.c_void_p(rep.data_ptr()),
                                             C.c_void_p(h.data_ptr()), C.c_void_p(idx.data_ptr()),
                                             L.stream_handle(stream)))
        return rep, h, idx


class Block:
    """One (M, Gamma, row) block; owns device tables, shares the sector's."""

    def __init__(self, sector: Sector, irrep, row=0, user_rho=None, hbm_limit=0, layout=0, user_rho_weight=0):
        self.sector = sector
        opts = L.make_opts(user_rho=user_rho, hbm_limit=hbm_limit, layout=layout, user_rho_weight=user_rho_weight)
        h = C.c_void_p()
        check(lib().ftlm_block_create(sector._h, int(irrep), int(row), C.byref(opts), C.byref(h)))
        self._h = h
        self._free = lib().ftlm_block_free
        self._load_info()

    @classmethod
    def build(cls, cluster, gens, two_M, irrep, row=0, user_rho=None, hv_mode=HV_AUTO, two_s=None):
        """One call: group + sector + block (ftlm_build_block)."""
        self = cls.__new__(cls)
        self.sector = None
        cl = L.make_cluster(cluster.N, two_s if two_s is not None else getattr(cluster, "two_s", 1), cluster.bonds,
                            cluster.J)
        gens = np.ascontiguousarray(np.asarray(gens, dtype=np.int32).reshape(-1, cluster.N))
        opts = L.make_opts(hv_mode=hv_mode, user_rho=user_rho)
        h = C.c_void_p()
        check(lib().ftlm_build_block(C.byref(cl), gens.ctypes.data_as(L.I32P), len(gens), int(two_M), int(irrep),
                                     int(row), C.byref(opts), C.byref(h)))
        self._h = h
        self._free = lib().ftlm_block_free
        self._load_info()
        return self

    def _load_info(self):
        info = L.BlockInfo()
        check(lib().ftlm_block_info_get(self._h, C.byref(info)))
        for f, _ in L.BlockInfo._fields_:
            setattr(self, f, getattr(info, f))

    def __del__(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def export(self):
        n = self.n_reps
        reps = np.empty(n, np.uint64)
        sid = np.empty(n, np.uint16)
        ng = np.empty(n, np.uint8)
        norms = np.empty(n, np.float64)
        offs = np.empty(n, np.uint64)
        check(lib().ftlm_block_export(self._h, reps.ctypes.data_as(C.POINTER(C.c_uint64)),
                                      sid.ctypes.data_as(C.POINTER(C.c_uint16)),
                                      ng.ctypes.data_as(C.POINTER(C.c_uint8)), norms.ctypes.data_as(L.F64P),
                                      offs.ctypes.data_as(C.POINTER(C.c_uint64))))
        return dict(reps=reps, stab_id=sid, n_gamma=ng, L=norms, offsets=offs)

    def hv_stats(self):
        st = L.HvStats()
        check(lib().ftlm_block_hv_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in L.HvStats._fields_}

    def autotune(self, nvec, dtype=F32, stream=None):
        """Time every H.V lane layout for nvec columns; the fastest is cached process-wide."""
        best = C.c_int32()
        best_ms = C.c_double()
        tried = np.zeros(8, np.int32)
        tried_ms = np.zeros(8)
        n = C.c_int32()
        check(lib().ftlm_block_autotune(self._h, int(nvec), int(dtype), L.stream_handle(stream), C.byref(best),
                                        C.byref(best_ms), tried.ctypes.data_as(L.I32P), tried_ms.ctypes.data_as(L.F64P),
                                        C.byref(n)))
        return best.value, best_ms.value, dict(zip(tried[: n.value].tolist(), tried_ms[: n.value].tolist()))

    def apply_H(self, X, Y=None, stream=None):
        """Y = H X for a (D, nvec) torch CUDA tensor (float64, float32 or float16 storage)."""
        import torch
        if X.dim() == 1:
            X = X[:, None]
        assert X.shape[0] == self.D and X.is_cuda
        if Y is None:
            Y = torch.empty_like(X)
        dtype = {torch.float64: F64, torch.float32: F32, torch.float16: F16}[X.dtype]
        assert Y.dtype == X.dtype
        assert X.stride(1) == 1 and Y.stride(1) == 1 and X.stride(0) == Y.stride(0)
        check(lib().ftlm_apply_H(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), X.shape[1],
                                 X.stride(0), dtype, L.stream_handle(stream)))
        return Y

    @property
    def D_pad(self):
        """Rows of the padded layout: n_reps * d_Gamma."""
        return self.n_reps * self.d_gamma

    def apply_H_ex(self, X, Y=None, layout=0, lanes=0, scale=None, dots=None, shift=0.0, stream=None,
                   noalloc=False):
        """ftlm_apply_H_ex on (rows, nvec) torch CUDA tensors: rows = D (LAYOUT_BLOCK) or
        n_reps * d_Gamma (LAYOUT_PADDED), packed or aligned rows (LAYOUT_PACKED,
        LAYOUT_ALIGNED; see include/ftlm.h); AUTO = the layout ftlm_run takes.  scale:
        float64 CUDA tensor (nvec, 2) of (s, b) pairs, Y <- s (H - shift) X - b Y;
        dots: float64 CUDA tensor (nvec,) receiving sum_rows X * Y.  noalloc: the
        entry point whose scratch is a static device array (ftlm_apply_H_ex_noalloc).
        Returns Y and the launch's (lanes_used, adjacent_columns)."""
        import torch
        if X.dim() == 1:
            X = X[:, None]
        assert X.is_cuda
        if Y is None:
            Y = torch.zeros_like(X)
        dtype = {torch.float64: F64, torch.float32: F32, torch.float16: F16}[X.dtype]
        assert Y.dtype == X.dtype and Y.shape == X.shape
        assert X.stride(1) == 1 and Y.stride(1) == 1 and X.stride(0) == Y.stride(0)
        o = L.HvOpts()
        o.layout = int(layout)
        o.lanes = int(lanes)
        if scale is not None:
            assert scale.dtype == torch.float64 and scale.is_cuda and scale.is_contiguous()
            assert scale.numel() == 2 * X.shape[1]
            o.scale = scale.data_ptr()
        if dots is not None:
            assert dots.dtype == torch.float64 and dots.is_cuda and dots.numel() >= X.shape[1]
            o.dots = dots.data_ptr()
        o.shift = float(shift)
        fn = lib().ftlm_apply_H_ex_noalloc if noalloc else lib().ftlm_apply_H_ex
        check(fn(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), X.shape[1], X.stride(0), dtype,
                 C.byref(o), L.stream_handle(stream)))
        return Y, dict(lanes_used=o.lanes_used, adjacent_columns=o.adjacent_columns)

    def kpm(self, R, n_moments, seed, center, half_width, storage=F64, dist=RADEMACHER, stream=None):
        """Chebyshev moments (ftlm_kpm): R x n_moments."""
        mom = np.zeros((R, n_moments))
        check(lib().ftlm_kpm(self._h, int(R), int(n_moments), C.c_uint64(seed), int(storage), int(dist),
                             float(center), float(half_width), mom.ctypes.data_as(L.F64P),
                             L.stream_handle(stream) if stream is not None else None))
        return mom

    def ftlm(self, R, steps, seed, storage=F64, dist=RADEMACHER, stream=None, info=False):
        """Batched Lanczos: returns alpha, beta (R x steps) and nsteps (R).

        With info=True also a dict (layout, hv_launches, rows, hv_ms) from ftlm_run_ex."""
        alpha = np.zeros((R, steps))
        beta = np.zeros((R, steps))
        ns = np.zeros(R, np.int32)
        ri = L.RunInfo()
        check(lib().ftlm_run_ex(self._h, int(R), int(steps), C.c_uint64(seed), int(storage), int(dist),
                                alpha.ctypes.data_as(L.F64P), beta.ctypes.data_as(L.F64P), ns.ctypes.data_as(L.I32P),
                                L.stream_handle(stream) if stream is not None else None,
                                C.byref(ri) if info else None))
        if info:
            return alpha, beta, ns, {f: getattr(ri, f) for f, _ in L.RunInfo._fields_}
        return alpha, beta, ns


class LanczosRunState:
    """ftlm_run in stages with checkpoints (ftlm_run_begin / advance / save / load / finish)."""

    def __init__(self, block, handle, R, steps):
        self.block, self._h, self.R, self.steps = block, handle, R, steps
        self._free = lib().ftlm_run_state_free

    @classmethod
    def begin(cls, block, R, steps, seed, storage=F64, dist=RADEMACHER, stream=None):
        h = C.c_void_p()
        check(lib().ftlm_run_begin(block._h, int(R), int(steps), C.c_uint64(seed), int(storage), int(dist),
                                   L.stream_handle(stream) if stream is not None else None, C.byref(h)))
        return cls(block, h, int(R), int(steps))

    @classmethod
    def load(cls, block, path, R, steps, stream=None):
        """R and steps size the outputs of finish(); they must be the saved run's."""
        h = C.c_void_p()
        check(lib().ftlm_run_load(block._h, str(path).encode(),
                                  L.stream_handle(stream) if stream is not None else None, C.byref(h)))
        return cls(block, h, int(R), int(steps))

    def advance(self, n):
        done = C.c_int32()
        check(lib().ftlm_run_advance(self._h, int(n), C.byref(done)))
        return done.value

    def save(self, path):
        check(lib().ftlm_run_save(self._h, str(path).encode()))

    def finish(self):
        alpha = np.zeros((self.R, self.steps))
        beta = np.zeros((self.R, self.steps))
        ns = np.zeros(self.R, np.int32)
        check(lib().ftlm_run_finish(self._h, alpha.ctypes.data_as(L.F64P), beta.ctypes.data_as(L.F64P),
                                    ns.ctypes.data_as(L.I32P)))
        return alpha, beta, ns

    def close(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def run_fused(jobs, stream=None):
    """ftlm_run_fused: the fused small-block Lanczos kernel over many jobs.

    jobs: sequence of dicts with keys block, R, steps, seed and optionally
    storage (F64), dist (RADEMACHER), first_chain (0).  Returns one
    (alpha, beta, nsteps) triple per job, as Block.ftlm does."""
    out = []
    arr = (L.FusedJob * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        R, steps = int(j["R"]), int(j["steps"])
        alpha = np.zeros((R, steps))
        beta = np.zeros((R, steps))
        ns = np.zeros(R, np.int32)
        out.append((alpha, beta, ns))
        arr[i] = L.FusedJob(j["block"]._h, R, steps, C.c_uint64(j["seed"]), int(j.get("storage", F64)),
                            int(j.get("dist", RADEMACHER)), int(j.get("first_chain", 0)), 0,
                            alpha.ctypes.data_as(L.F64P), beta.ctypes.data_as(L.F64P), ns.ctypes.data_as(L.I32P))
    check(lib().ftlm_run_fused(arr, len(jobs), L.stream_handle(stream) if stream is not None else None))
    return out


def device_arch():
    """Architecture name of the current device (the autotuner keys carry it)."""
    buf = C.create_string_buffer(256)
    check(lib().ftlm_device_arch(buf, 256))
    return buf.value.decode()


def autotune_save(path, arch=None):
    """Write the autotuner's cached choices of `arch` (None: all) to path; returns their number."""
    n = C.c_int32()
    check(lib().ftlm_autotune_save(str(path).encode(), arch.encode() if arch else None, C.byref(n)))
    return n.value


def autotune_load(path, arch=None):
    """Add the choices of `arch` (None: all) from path to the cache; returns their number."""
    n = C.c_int32()
    check(lib().ftlm_autotune_load(str(path).encode(), arch.encode() if arch else None, C.byref(n)))
    return n.value


def autotune_clear():
    check(lib().ftlm_autotune_clear())


def kpm_observables(blocks, T, g=1.0, n_nodes=0):
    """ftlm_kpm_observables: blocks are dicts (two_M, d_gamma, D, moments (R x M), center, half_width)
    -> E, C, chi, logZ on T."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    arr = (L.KpmBlock * len(blocks))()
    keep = []
    for i, b in enumerate(blocks):
        m = np.ascontiguousarray(np.atleast_2d(b["moments"]), dtype=np.float64)
        keep.append(m)
        arr[i] = L.KpmBlock(int(b["two_M"]), int(b["d_gamma"]), int(b["D"]), m.shape[0], m.shape[1],
                            float(b["center"]), float(b["half_width"]), m.ctypes.data_as(L.F64P))
    nT = len(T)
    E, Cv, chi, lz = np.empty(nT), np.empty(nT), np.empty(nT), np.empty(nT)
    check(lib().ftlm_kpm_observables(arr, len(blocks), T.ctypes.data_as(L.F64P), nT, float(g), int(n_nodes),
                                     E.ctypes.data_as(L.F64P), Cv.ctypes.data_as(L.F64P), chi.ctypes.data_as(L.F64P),
                                     lz.ctypes.data_as(L.F64P)))
    return E, Cv, chi, lz


def tridiag_ritz(alpha, beta):
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    n = len(alpha)
    th = np.empty(n)
    w = np.empty(n)
    check(lib().ftlm_tridiag_ritz(alpha.ctypes.data_as(L.F64P), beta.ctypes.data_as(L.F64P), n,
                                  th.ctypes.data_as(L.F64P), w.ctypes.data_as(L.F64P)))
    return th, w


def ritz_from_run(alpha, beta, nsteps):
    """Per chain Ritz values/weights (lists of arrays) from ftlm() output."""
    ths, ws = [], []
    for r in range(len(nsteps)):
        n = int(nsteps[r])
        th, w = tridiag_ritz(alpha[r, :n], beta[r, : max(n - 1, 0)] if n > 1 else np.zeros(1))
        ths.append(th)
        ws.append(w)
    return ths, ws


def observables(blocks, T, g=1.0):
    """blocks: list of dicts (two_M, d_gamma, D, thetas, weights) -> E, C, chi, logZ."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    arr = (L.Ritz * len(blocks))()
    keep = []
    for i, b in enumerate(blocks):
        R = len(b["thetas"])
        ld = max([len(t) for t in b["thetas"]] + [1])
        th = np.zeros((R, ld))
        w = np.zeros((R, ld))
        ns = np.zeros(R, np.int32)
        for r, (t, ww) in enumerate(zip(b["thetas"], b["weights"])):
            th[r, : len(t)] = t
            w[r, : len(t)] = ww
            ns[r] = len(t)
        keep += [th, w, ns]
        arr[i] = L.Ritz(int(b["two_M"]), int(b["d_gamma"]), int(b["D"]), R, ld, ns.ctypes.data_as(L.I32P),
                        th.ctypes.data_as(L.F64P), w.ctypes.data_as(L.F64P))
    nT = len(T)
    E, Cv, chi, lz = np.empty(nT), np.empty(nT), np.empty(nT), np.empty(nT)
    check(lib().ftlm_observables(arr, len(blocks), T.ctypes.data_as(L.F64P), nT, float(g), E.ctypes.data_as(L.F64P),
                                 Cv.ctypes.data_as(L.F64P), chi.ctypes.data_as(L.F64P), lz.ctypes.data_as(L.F64P)))
    return E, Cv, chi, lz


def campaign(cluster, gens, two_s, R, steps, seed, T, storage=F64, dist=RADEMACHER, all_M=True, two_M=0,
             spin_flip=False, chains_per_run=0, g=1.0, engine=0, fused_max_rounds=0):
    """Whole-cluster FTLM (ftlm_campaign): E, C, chi, logZ on T and the run statistics.

    engine: ENGINE_AUTO (fused small-block kernel for sectors of few
    representatives, per-step kernels otherwise), ENGINE_STEPS or ENGINE_FUSED."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    cl = L.make_cluster(cluster.N, two_s, cluster.bonds, cluster.J)
    gens = np.ascontiguousarray(np.asarray(gens, dtype=np.int32).reshape(-1, cluster.N))
    o = L.CampaignOpts(int(R), int(steps), C.c_uint64(seed), int(storage), int(dist), 1 if all_M else 0,
                       int(two_M), 1 if spin_flip else 0, int(chains_per_run), float(g), int(engine),
                       int(fused_max_rounds))
    out = [np.empty(len(T)) for _ in range(4)]
    st = L.CampaignStats()
    check(lib().ftlm_campaign(C.byref(cl), gens.ctypes.data_as(L.I32P), len(gens), C.byref(o),
                              T.ctypes.data_as(L.F64P), len(T), *[x.ctypes.data_as(L.F64P) for x in out],
                              C.byref(st)))
    E, Cv, chi, logZ = out
    return dict(E=E, C=Cv, chi=chi, logZ=logZ, stats={f: getattr(st, f) for f, _ in L.CampaignStats._fields_})


__all__ = ["Group", "Sector", "Block", "LanczosRunState", "run_fused", "campaign", "tridiag_ritz", "ritz_from_run",
           "observables", "kpm_observables", "device_arch", "autotune_save", "autotune_load", "autotune_clear",
           "FtlmError", "F32", "F64", "RADEMACHER", "GAUSSIAN", "HV_AUTO", "HV_ENTRIES", "HV_ONTHEFLY"]
