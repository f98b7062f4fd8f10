"""Global preconditioner K_eps_bar = (H - eps_bar S)^{-1}  (eq. (globalprecond)).

The paper computes a sparse factorisation of H^(loc,1) - eps_bar S once
(eq. (ldl)) and applies P = -K R by substitution (eq. (k1p)).  With no
nonlocal term (H^(nl) = 0) the Sherman-Morrison-Woodbury steps of Section 4
reduce to that plain solve.  With eps_bar below the lowest eigenvalue the
matrix is positive definite, so the factorisation needs no 2x2 pivots.

Here SciPy's SuperLU factors the matrix once with a symmetric fill-reducing
ordering and no numerical pivoting (for an SPD matrix that is the Cholesky
factorisation written as L U with U = D L^T); each apply is one pair of
triangular substitutions.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class GlobalPreconditioner:
    def __init__(self, H, S, eps_bar: float):
        K = (sp.csc_matrix(H) - eps_bar * sp.csc_matrix(S)).tocsc()
        self.eps_bar = float(eps_bar)
        self.K = K
        self.lu = spla.splu(K, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))
        d = self.lu.U.diagonal().real
        if np.any(d <= 0):
            raise np.linalg.LinAlgError("H - eps_bar S is not positive definite")

    def apply(self, R: np.ndarray) -> np.ndarray:
        """P = -(H - eps_bar S)^{-1} R  (eq. (k1p))."""
        R = np.asarray(R, dtype=np.result_type(R, self.K.dtype))
        if R.ndim == 1:
            return -self.lu.solve(R)
        if R.shape[1] == 0:
            return np.zeros_like(R)
        return -self.lu.solve(np.asfortranarray(R))
