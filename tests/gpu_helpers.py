"""Shared setup for the GPU parity tests: oracle objects and library objects for
the same (cluster, spin, M, irrep), with the oracle's irrep matrices passed to
the library (irreps are unique only up to a change of basis)."""
import functools
import sys

import numpy as np

from oracle import basis, group, hv, irreps, sector
from synth import clusters


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@functools.lru_cache(maxsize=None)
def oracle_group(name):
    cl = clusters.get(name)
    G = group.close(cl.gens, cl.N)
    return cl, G, irreps.compute_irreps(G)


@functools.lru_cache(maxsize=None)
def oracle_sector(name, two_s, two_M):
    cl, G, irs = oracle_group(name)
    sec = basis.sector_reps(G, cl.N, two_s, two_M)
    H = sector.hamiltonian(sec.labels, cl.N, two_s, cl.bonds, cl.J)
    return sec, H


@functools.lru_cache(maxsize=None)
def oracle_block(name, two_s, two_M, gi, alpha=0):
    cl, G, irs = oracle_group(name)
    sec, H = oracle_sector(name, two_s, two_M)
    return basis.build_block(G, irs[gi], sec, alpha=alpha)


_lib_groups = {}
_lib_sectors = {}


def lib_group(name):
    import paper_2607_17429_amd as P
    if name not in _lib_groups:
        cl = clusters.get(name)
        _lib_groups[name] = P.Group(cl.N, cl.gens)
    return _lib_groups[name]


def lib_sector(name, two_s, two_M, hv_mode=0, entry_format=0):
    import paper_2607_17429_amd as P
    key = (name, two_s, two_M, hv_mode, entry_format)
    if key not in _lib_sectors:
        cl = clusters.get(name)
        _lib_sectors[key] = P.Sector(cl, lib_group(name), two_M, hv_mode=hv_mode, two_s=two_s,
                                     entry_format=entry_format)
    return _lib_sectors[key]


def lib_block(name, two_s, two_M, gi, row=0, hv_mode=0, entry_format=0):
    import paper_2607_17429_amd as P
    _, _, irs = oracle_group(name)
    return P.Block(lib_sector(name, two_s, two_M, hv_mode, entry_format), gi, row, user_rho=irs[gi].rho)


def rel_err_cols(Y, Yref):
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    num = np.max(np.abs(Y - Yref), axis=0)
    den = np.maximum(np.max(np.abs(Yref), axis=0), 1e-300)
    return np.max(num / den)


@functools.lru_cache(maxsize=None)
def oracle_real_forms(name):
    """The oracle's real forms (with their trace weights) of the cluster's group."""
    from oracle import realform
    cl, G, irs = oracle_group(name)
    return realform.real_forms(G, irs)


def oracle_weight(name, rho):
    """Trace weight of the real form whose character equals that of the
    matrices rho (|G| x d x d, the group's element order): the oracle's rule
    (dim, dim / 2 for a complex pair, dim / 4 for a quaternionic irrep),
    matched by character, never read from the library."""
    ch = np.trace(np.asarray(rho), axis1=1, axis2=2)
    hits = [f.weight for f in oracle_real_forms(name)
            if f.irrep.dim == rho.shape[1] and np.allclose(np.trace(f.irrep.rho, axis1=1, axis2=2).real, ch, atol=1e-8)]
    assert len(hits) == 1, "no unique real form with this character"
    return int(hits[0])
