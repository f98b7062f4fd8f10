"""CPU FP64 oracle for the LABPSD hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct host implementation of what one LABPSD solve
computes (Cai, Bai, Pask, Sukumar, "Hybrid preconditioning for iterative
diagonalization of ill-conditioned generalized eigenvalue problems in
electronic structure calculations", arXiv:1308.2445).  It exists to check the
GPU path; only the tests, the smoke check and the benchmark's CPU baseline may
import or run it.  It shares no code with the GPU library: it calls NumPy,
SciPy and mpmath only.

Modules
  eigs      the plain definition of the result: lowest eigenpairs of (H, S)
            (eq. ghep), the relative residual Res (eq. res1) and an mpmath route.
  precond   the global preconditioner K = (H - eps_bar S)^{-1} (eq. globalprecond,
            eq. k1p) by a sparse factorisation computed once (eq. ldl).
  minres    MINRES for the local refinement equation (eq. indls, Section 4).
  rr        the Rayleigh-Ritz step on [Psi P] (Section 3, steps 8-9).
  labpsd    the LABPSD outline of Section 3 taken step by step, with the hybrid
            preconditioning scheme and the localisation test.

Every function that has no independent pin says "parity unpinned" in its
docstring; all others are pinned by the CPU tests under tests/.
"""
from . import eigs, precond, minres, rr, labpsd  # noqa: F401
