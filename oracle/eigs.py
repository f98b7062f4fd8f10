"""The plain definition of the result and of the convergence measure.

* The wanted result is the m lowest eigenpairs (lambda_i, x_i) of the
  Hermitian-definite pencil H x = lambda S x (Section 2, eq. (ghep)), lambda
  ascending, X S-orthonormal.  At the Gamma point the matrices are real; at other
  k-points complex Hermitian, and every transpose below is the conjugate one.
* Res (eq. (res1)) is ||r_i|| / ||H psi_i|| with r_i = H psi_i - eps_i S psi_i.
  The experiments shift H by sigma0 so that H - sigma0 S is positive definite
  (Section 5); the denominator here uses that shifted H, ||(H - sigma0 S) psi_i||,
  while r_i is shift-invariant.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_eigs(H, S, m: int):
    """Lowest m eigenpairs of the dense pencil (H, S) by LAPACK's symmetric-definite
    (real) or Hermitian-definite (complex) driver: the textbook definition of the GHEP
    solution (eq. (ghep))."""
    H = np.asarray(H.toarray() if hasattr(H, "toarray") else H)
    S = np.asarray(S.toarray() if hasattr(S, "toarray") else S)
    lam, X = sla.eigh(H, S, subset_by_index=[0, m - 1])
    return lam, X


def mp_eigs(H, S, dps: int = 40):
    """All eigenvalues of (H, S) in mpmath at ``dps`` digits: Cholesky S = L L^H,
    then the Hermitian eigenvalues of L^{-1} H L^{-H} (real symmetric at the Gamma point,
    complex Hermitian at other k-points).  Independent of LAPACK."""
    import mpmath as mp
    H = np.asarray(H.toarray() if hasattr(H, "toarray") else H)
    S = np.asarray(S.toarray() if hasattr(S, "toarray") else S)
    cplx = np.iscomplexobj(H) or np.iscomplexobj(S)
    with mp.workdps(dps):
        Hm = mp.matrix(H.tolist())
        Sm = mp.matrix(S.tolist())
        Lm = mp.cholesky(Sm)
        Li = mp.inverse(Lm)
        C = Li * Hm * Li.H
        C = (C + C.H) / 2
        ev = mp.eighe(C, eigvals_only=True) if cplx else mp.eigsy(C, eigvals_only=True)
        vals = sorted(float(mp.re(v)) for v in ev)
    return np.array(vals)


def relative_residuals(H, S, lam, X, sigma0: float):
    """Res_i = ||H x_i - lam_i S x_i|| / ||(H - sigma0 S) x_i||  (eq. (res1), shifted H)."""
    HX = H @ X
    SX = S @ X
    R = HX - SX * lam[None, :]
    den = np.linalg.norm(HX - sigma0 * SX, axis=0)
    return np.linalg.norm(R, axis=0) / den


def clusters(lam, sigma0: float, rel_gap: float = 1e-6):
    """Maximal runs of eigenvalues whose neighbour gaps are below
    rel_gap * |lambda - sigma0|; returned as a list of index lists."""
    out = [[0]]
    for i in range(1, len(lam)):
        if abs(lam[i] - lam[i - 1]) < rel_gap * abs(lam[i] - sigma0):
            out[-1].append(i)
        else:
            out.append([i])
    return out


def _s_sines(S, C):
    """Singular values of C in the S norm (ascending), each to about rounding of
    C's entries in absolute terms: the eigenvalues of C^T S C give the squares; the
    ones far below the largest are recomputed from the Gram matrix of their own
    directions, where no large value dilutes them."""
    G = C.conj().T @ (S @ C)
    w, V = np.linalg.eigh(0.5 * (G + G.conj().T))
    w = np.clip(w, 0.0, None)
    small = w < 1e-4 * w.max()
    if small.any() and not small.all():
        w[small] = _s_sines(S, C @ V[:, small]) ** 2
    return np.sqrt(np.sort(w))


def s_principal_angles(S, X, Y):
    """Principal angles between span(X) and span(Y) in the S inner product, ascending.

    Both bases are S-orthonormalised (Qx, Qy).  The cosines are the singular values
    of Qx^T S Qy; the sines are the S-norm singular values of the part of Qy that is
    S-orthogonal to span(Qx), B = Qy - Qx (Qx^T S Qy).  Angles whose sine is below
    1/sqrt(2) are taken from the sine (arccos of a cosine near 1 resolves nothing
    below about 1e-8), the others from the cosine (the sine-cosine rule of Knyazev and
    Argentati, SIAM J. Sci. Comput. 23 (2002)).  Requires dim span(X) <= dim span(Y)."""
    def sorth(A):
        G = A.conj().T @ (S @ A)
        G = 0.5 * (G + G.conj().T)
        w, V = np.linalg.eigh(G)
        return A @ (V / np.sqrt(w)[None, :])
    Qx, Qy = sorth(X), sorth(Y)
    M = Qx.conj().T @ (S @ Qy)
    cos = np.sort(np.clip(np.linalg.svd(M, compute_uv=False), 0.0, 1.0))[::-1]
    sin = np.clip(_s_sines(S, Qy - Qx @ M), 0.0, 1.0)[: cos.shape[0]]
    return np.where(sin < np.sqrt(0.5), np.arcsin(sin), np.arccos(cos))


def shift_invert_eigs(H, S, m: int, sigma: float, tol: float = 1e-13):
    """Lowest m eigenpairs of (H, S) by a library route that shares nothing with LABPSD:
    ARPACK's implicitly restarted Lanczos on the shift-inverted operator
    (H - sigma S)^{-1} S (SciPy ``eigsh`` in shift-invert mode), with sigma below the
    spectrum so that the eigenvalues closest to sigma are the lowest ones (eq. (ghep)).
    (H - sigma S) is factorised once by SuperLU with a symmetric ordering.
    Returns (lambda ascending, X S-orthonormal)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = (sp.csc_matrix(H) - sigma * sp.csc_matrix(S)).tocsc()
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    n = A.shape[0]
    op = spla.LinearOperator((n, n), matvec=lu.solve, dtype=A.dtype)
    ncv = min(n, max(2 * m + 1, m + 64))
    lam, X = spla.eigsh(sp.csr_matrix(H), k=m, M=sp.csr_matrix(S), sigma=sigma, which="LM", OPinv=op,
                        ncv=ncv, tol=tol)
    order = np.argsort(lam)
    return lam[order], X[:, order]


def full_hamiltonian(H_loc, F, G):
    """H = H_loc + H_nl with the nonlocal part in its low-rank form H_nl = F G F^T
    (Section 4, eq. (fgf); real at the Gamma point), as one explicit sparse matrix: the
    plain definition the oracle's solves use.  F: n x k sparse, G: k x k."""
    import scipy.sparse as sp
    Fs = sp.csr_matrix(F)
    Hnl = Fs @ sp.csr_matrix(G) @ Fs.conj().T
    Hnl = 0.5 * (Hnl + Hnl.conj().T)
    return (sp.csr_matrix(H_loc) + Hnl).tocsr()
