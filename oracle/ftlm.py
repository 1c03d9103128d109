"""FTLM stage in FP64 (paper Section 2.2, Eqs. 4-7 and 14; Section 3).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle; only tests, the smoke
check and the benchmark's CPU baseline use it.

* Start vectors: a counter-based SplitMix64 stream (Steele, Lea and Flood,
  OOPSLA 2014) per chain, keyed by (seed, 2M, irrep, row, chain); Rademacher
  (sign of the top bit) or Gaussian (Box-Muller on two 53-bit uniforms);
  normalised in FP64.
* Lanczos: the plain three-term recurrence, no reorthogonalisation:
  w = H v_j - beta_j v_{j-1};  alpha_j = <v_j, w>;  w -= alpha_j v_j;
  beta_{j+1} = |w|;  v_{j+1} = w / beta_{j+1}.  n = min(steps, D) products;
  early stop when beta_{j+1} <= 1e-10 * max_{i<=j}(|alpha_i| + beta_i + beta_{i+1}).
* Ritz data: eigenvalues theta_k of the n x n tridiagonal T and weights
  w_k = (first component of the k-th eigenvector)^2, sum_k w_k = 1.
* Thermal sums: Eq. (5) with the multiplicity factor mult_M * d_Gamma of
  Eq. (14), energy moments of Eq. (6), C = beta^2 (<H^2> - <H>^2), and the
  susceptibility of Eq. (7).  Boltzmann factors are shifted by the lowest
  Ritz value over all blocks (exact rewriting; every ratio is unchanged).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import eigh_tridiagonal

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def sm_mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_stream(state: int, count: int):
    """First ``count`` outputs of SplitMix64 started at ``state`` (Python ints)."""
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK
        out.append(sm_mix(state))
    return out


def chain_key(seed: int, two_M: int, irrep: int, row: int, chain: int) -> int:
    h = sm_mix((seed + GAMMA) & MASK)
    for i, x in enumerate((two_M, irrep, row, chain)):
        h = sm_mix(h ^ (((x & MASK) + (i + 2) * GAMMA) & MASK))
    return h


def _stream_np(key: int, count: int) -> np.ndarray:
    j = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + j * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def start_vector(D: int, seed: int, two_M: int, irrep: int, row: int, chain: int, dist: str = "rademacher"):
    key = chain_key(seed, two_M, irrep, row, chain)
    if dist == "rademacher":
        x = _stream_np(key, D)
        v = np.where((x >> np.uint64(63)) != 0, -1.0, 1.0)
    elif dist == "gaussian":
        x = _stream_np(key, 2 * D)
        u1 = ((x[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
        u2 = (x[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        v = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    else:
        raise ValueError(dist)
    return v / np.linalg.norm(v) if D else v


def lanczos(matvec, v0, steps: int):
    """Three-term Lanczos recurrence on unit vectors (Section 2.2), no
    reorthogonalisation.  v_0 = v0 / |v0|; for j = 0, 1, ...:
    w = H v_j - beta_j v_{j-1};  alpha_j = <v_j, w>;  w -= alpha_j v_j;
    beta_{j+1} = |w|;  v_{j+1} = w / beta_{j+1}.
    n = min(steps, D) products; the chain stops early when
    beta_{j+1} <= 1e-10 * max_{i<=j}(|alpha_i| + beta_i + beta_{i+1}).
    Returns alpha_0..alpha_{n-1} and beta_1..beta_n."""
    D = len(v0)
    n_target = min(steps, D)
    alphas, betas = [], []
    if n_target == 0:
        return np.zeros(0), np.zeros(0)
    v = np.array(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta_j = 0.0
    scale = 0.0
    for j in range(n_target):
        w = matvec(v) - beta_j * v_prev
        a = float(np.dot(v, w))
        w = w - a * v
        b = float(np.linalg.norm(w))
        alphas.append(a)
        betas.append(b)
        scale = max(scale, abs(a) + beta_j + b)
        if j + 1 == n_target or b <= 1e-10 * scale:
            break
        v_prev, v, beta_j = v, w / b, b
    return np.array(alphas), np.array(betas)


def ritz(alphas, betas):
    n = len(alphas)
    if n == 0:
        return np.zeros(0), np.zeros(0)
    if n == 1:
        return np.array(alphas, dtype=np.float64), np.ones(1)
    th, U = eigh_tridiagonal(np.asarray(alphas), np.asarray(betas[: n - 1]))
    return th, U[0, :] ** 2


@dataclass
class BlockRitz:
    two_M: int
    d_gamma: int
    D: int
    thetas: list      # per chain: array of Ritz values
    weights: list     # per chain: array of weights

    @property
    def R(self):
        return len(self.thetas)


def observables(blocks, T, g: float = 1.0, with_logZ: bool = False):
    """E, C, chi (Eqs. 5-7, 14) on the temperature grid T (per cluster, k_B = 1).

    With ``with_logZ`` also returns ln Z_FTLM (Eq. 5) = -beta E0 + ln(shifted sum).
    """
    T = np.asarray(T, dtype=np.float64)
    E0 = min(float(np.min(th)) for b in blocks for th in b.thetas if len(th))
    beta = 1.0 / T
    Z = np.zeros_like(T)
    H1 = np.zeros_like(T)
    H2 = np.zeros_like(T)
    ZM = {}
    for b in blocks:
        if b.D == 0 or b.R == 0:
            continue
        mult = 1 if b.two_M == 0 else 2
        fac = mult * b.d_gamma * b.D / b.R
        z = np.zeros_like(T)
        h1 = np.zeros_like(T)
        h2 = np.zeros_like(T)
        for th, w in zip(b.thetas, b.weights):
            sh = np.asarray(th) - E0
            bz = np.exp(-np.outer(beta, sh)) * np.asarray(w)[None, :]
            z += bz.sum(axis=1)
            h1 += (bz * sh[None, :]).sum(axis=1)
            h2 += (bz * sh[None, :] ** 2).sum(axis=1)
        Z += fac * z
        H1 += fac * h1
        H2 += fac * h2
        ZM[b.two_M] = ZM.get(b.two_M, 0.0) + (b.d_gamma * b.D / b.R) * z
    e1 = H1 / Z
    e2 = H2 / Z
    E = E0 + e1
    C = beta ** 2 * (e2 - e1 ** 2)
    num = np.zeros_like(T)
    den = np.zeros_like(T)
    for twoM, z in ZM.items():
        mult = 1 if twoM == 0 else 2
        M = twoM / 2.0
        num += mult * M * M * z
        den += mult * z
    chi = g * g * beta * num / den
    if with_logZ:
        return E, C, chi, np.log(Z) - beta * E0
    return E, C, chi


def ed_observables(sector_spectra, T, g: float = 1.0):
    """Full-ED thermodynamics from {two_M: eigenvalues of H_M} for M >= 0."""
    blocks = [BlockRitz(twoM, 1, len(ev), [np.asarray(ev)], [np.ones(len(ev)) / len(ev)])
              for twoM, ev in sector_spectra.items() if len(ev)]
    return observables(blocks, T, g)
