"""Rayleigh-Ritz on the search space Z = [Psi P] (Section 3, outline steps 8-9).

Step 8 forms H_R = Z^T H Z and S_R = Z^T S Z from the stored products; step 9
takes the lowest m + m0 eigenpairs (Gamma, W) of the reduced pencil (the paper
calls LAPACK's ZHEGVX).  The reduced S_R is positive definite whenever Z has
full column rank; the conclusions note that a general-purpose code needs a
rank-revealing treatment when it does not, which is the fallback below.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

#: relative eigenvalue floor of the diagonally scaled S_R below which a direction
#: of the search space is treated as linearly dependent and dropped
RANK_TOL = 1e-14


def gram(Z: np.ndarray, ZH: np.ndarray, ZS: np.ndarray):
    """H_R = Z^H (HZ), S_R = Z^H (SZ), each replaced by its Hermitian part (step 8)."""
    HR = Z.conj().T @ ZH
    SR = Z.conj().T @ ZS
    return 0.5 * (HR + HR.conj().T), 0.5 * (SR + SR.conj().T)


def rayleigh_ritz(HR: np.ndarray, SR: np.ndarray, nwant: int):
    """Lowest ``nwant`` eigenpairs (Gamma ascending, W with W^T S_R W = I) of (H_R, S_R).

    Plain route: the symmetric-definite LAPACK driver (step 9).  If S_R is not
    numerically positive definite, the rank-revealing route scales S_R to unit
    diagonal, keeps the eigen-directions of the scaled S_R above RANK_TOL times
    its largest eigenvalue, and solves the reduced standard problem there.
    Returns (Gamma, W, rank_dropped).
    """
    k = HR.shape[0]
    try:
        gam, W = sla.eigh(HR, SR, subset_by_index=[0, nwant - 1])
        return gam, W, 0
    except np.linalg.LinAlgError:
        pass
    d = np.diag(SR).real.copy()
    keep_cols = d > 0
    D = np.zeros(k)
    D[keep_cols] = 1.0 / np.sqrt(d[keep_cols])
    Ss = D[:, None] * SR * D[None, :]
    Hs = D[:, None] * HR * D[None, :]
    lam, Q = np.linalg.eigh(Ss)
    keep = lam > RANK_TOL * lam[-1]
    r = int(keep.sum())
    if r < nwant:
        raise np.linalg.LinAlgError("search space rank %d below the block width %d" % (r, nwant))
    T = Q[:, keep] / np.sqrt(lam[keep])[None, :]
    C = T.conj().T @ Hs @ T
    C = 0.5 * (C + C.conj().T)
    gam, V = np.linalg.eigh(C)
    W = D[:, None] * (T @ V[:, :nwant])
    return gam[:nwant], W, k - r
