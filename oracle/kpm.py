"""Kernel polynomial method (KPM) on one symmetry block, in FP64.

TEST INFRASTRUCTURE: part of the CPU oracle; only tests, the smoke check and
the benchmark's CPU baseline use it.

The kernel polynomial method (the paper's Ref. [6]) obtains thermodynamics
from a Chebyshev expansion of the density of states, an alternative to FTLM;
the library runs it on the same symmetry-adapted H.V.  Definitions used here:

* Scaled block Hamiltonian H~ = (H - c) / w, with a centre c and half width w
  that put the block spectrum inside (-1, 1).
* Moments of a normalised start vector r (the FTLM start vectors, same keys):
  mu_n = <r| T_n(H~) |r>, with T_n the Chebyshev polynomials of the first kind,
  T_n(cos t) = cos(n t).  ``moments`` evaluates this definition from the
  eigen-decomposition of the explicit block matrix,
  mu_n = sum_k |<u_k|r>|^2 cos(n arccos e_k), not by a recurrence.
* Jackson kernel g_n for N moments (Weisse, Wellein, Alvermann and Fehske,
  Rev. Mod. Phys. 78, 275 (2006), Eq. (71)):
  g_n = [(N - n + 1) cos(pi n / (N + 1)) + sin(pi n / (N + 1)) cot(pi / (N + 1))] / (N + 1).
* Density of states of a block from the chain-averaged moments, on the K
  Chebyshev nodes x_k = cos(theta_k), theta_k = pi (k + 1/2) / K: the
  Gauss-Chebyshev quadrature weight of node k is
  W_k = (1/K) [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n cos(n theta_k)],
  so that sum_k W_k f(c + w x_k) approximates <r|f(H)|r> averaged over r, and
  sum_k W_k = mu_0 = 1 exactly for K > N.
* Thermodynamics (Eqs. (5)-(7) with Eq. (14)'s weights): node energies
  E_k = c + w x_k; Z = sum_blocks mult_M d_Gamma D sum_k W_k exp(-(E_k - E0)/T),
  E0 the lowest node energy over all blocks (an exact rewriting); E, C, chi
  from the same sums as in ``ftlm.observables``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def moments(Hb: np.ndarray, r: np.ndarray, center: float, half_width: float, n_moments: int) -> np.ndarray:
    """mu_n = <r|T_n((H - c)/w)|r> for n < n_moments, r normalised first."""
    r = np.asarray(r, dtype=np.float64)
    r = r / np.linalg.norm(r)
    e, U = np.linalg.eigh(np.asarray(Hb, dtype=np.float64))
    x = (e - center) / half_width
    if np.any(np.abs(x) >= 1.0):
        raise ValueError("block spectrum outside the scaled interval")
    p = (U.T @ r) ** 2
    n = np.arange(n_moments)
    return np.cos(np.outer(n, np.arccos(x))) @ p


def jackson(N: int) -> np.ndarray:
    n = np.arange(N)
    q = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (N + 1)


def node_weights(mu: np.ndarray, K: int) -> tuple:
    """(x_k, W_k) for the chain-averaged moments mu (length N)."""
    N = len(mu)
    g = jackson(N)
    theta = np.pi * (np.arange(K) + 0.5) / K
    c = g * mu
    W = (c[0] + 2.0 * np.cos(np.outer(theta, np.arange(1, N))) @ c[1:]) / K
    return np.cos(theta), W


@dataclass
class KpmBlock:
    two_M: int
    d_gamma: int          # trace weight
    D: int
    moments: np.ndarray   # (R, N)
    center: float
    half_width: float


def observables(blocks, T, g: float = 1.0, K: int | None = None, with_logZ: bool = False):
    """E, C, chi (and ln Z) on the temperature grid from the blocks' moments."""
    T = np.asarray(T, dtype=np.float64)
    beta = 1.0 / T
    nodes = []
    for b in blocks:
        if b.D == 0:
            continue
        mu = np.asarray(b.moments, dtype=np.float64).mean(axis=0)
        x, W = node_weights(mu, K or 2 * len(mu))
        nodes.append((b, b.center + b.half_width * x, W))
    E0 = min(float(E.min()) for _, E, _ in nodes)
    Z = np.zeros_like(T)
    H1 = np.zeros_like(T)
    H2 = np.zeros_like(T)
    num = np.zeros_like(T)
    for b, E, W in nodes:
        mult = 1 if b.two_M == 0 else 2
        sh = E - E0
        bz = np.exp(-np.outer(beta, sh)) * W[None, :]
        z = bz.sum(axis=1) * b.d_gamma * b.D
        Z += mult * z
        H1 += mult * b.d_gamma * b.D * (bz * sh[None, :]).sum(axis=1)
        H2 += mult * b.d_gamma * b.D * (bz * sh[None, :] ** 2).sum(axis=1)
        num += mult * (b.two_M / 2.0) ** 2 * z
    e1 = H1 / Z
    e2 = H2 / Z
    E = E0 + e1
    C = beta ** 2 * (e2 - e1 ** 2)
    chi = g * g * beta * num / Z
    if with_logZ:
        return E, C, chi, np.log(Z) - beta * E0
    return E, C, chi
