"""Plain FP64 CPU oracle for the symmetry-adapted FTLM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP library:
it has its own group closure (breadth-first, not Dimino), its own irreps, its
own orbit search (brute force over every group element), and it applies the
Hamiltonian through the *explicit* symmetry-adapted basis of Eq. (12)
(Y = Psi^H H_M Psi X) rather than through the closed-form matrix element of
Eq. (15).  Everything is float64 (complex128 where an irrep is complex).

Modules
-------
group     closure, element order, product table, classes (Section 3)
irreps    irreps from the regular representation, real form, checks (Section 3)
counting  sector dimension and character-formula block dimensions (Eq. 13)
sector    M-sector enumeration and sparse H_M from Eqs. (1)-(3)
basis     orbits, representatives, stabilizers, n_Gamma, V_S, explicit Psi
          (Eqs. 8-13)
hv        Y = Psi^H H_M Psi X, also row-sampled for blocks too big to expand
ftlm      SplitMix64 start vectors, FP64 Lanczos, tridiagonal Ritz data,
          thermal sums of Eqs. (4)-(7) and (14), full-ED thermodynamics

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against values the paper prints, closed forms, invariants or brute force,
except the Lanczos coefficients after the first converged Ritz value
(alpha/beta beyond the loss of orthogonality): "parity unpinned" there, and
only the thermal observables built from them are compared.
"""
