"""MINRES for the local refinement equation (Section 4, eq. (indls)).

The local correction solves (H - eps_i S) p = -r_i inexactly, to
||(H - eps_i S) p + r_i|| <= eta ||r_i|| (eq. (approxp)), starting from the
globally preconditioned vector.  H - eps_i S is symmetric indefinite, so the
paper uses MINRES (Paige and Saunders, 1975).

The method below is MINRES written from its definition: Lanczos builds an
orthonormal basis V_k of the Krylov space K_k(A, b) with A V_k = V_{k+1} T_k,
T_k tridiagonal; x_k = V_k y_k minimises ||beta_1 e_1 - T_k y||, which is
solved by Givens rotations applied one column of T_k at a time.  The rotated
right-hand side's last entry is the residual norm ||b - A x_k||, so the stopping
test needs no extra product.
"""
from __future__ import annotations

import math

import numpy as np


def minres(matvec, b: np.ndarray, stop_norm: float, max_iter: int):
    """Approximately solve A x = b from x = 0.

    Stops once the residual norm is <= stop_norm or after max_iter iterations.
    Returns (x, iterations, residual_norms) where residual_norms[k] is the
    recurred ||b - A x_k|| (residual_norms[0] = ||b||).
    """
    n = b.shape[0]
    x = np.zeros(n, dtype=b.dtype)
    beta1 = float(np.linalg.norm(b))
    hist = [beta1]
    if beta1 == 0.0 or beta1 <= stop_norm or max_iter <= 0:
        return x, 0, hist
    v_prev = np.zeros(n, dtype=b.dtype)
    v = b / beta1
    beta = beta1          # beta_k: coupling of v_k to v_{k-1} (beta_1 for the first step)
    # Givens state: the rotation from the previous two columns
    c_prev, s_prev = 1.0, 0.0      # rotation k-1
    c_pp, s_pp = 1.0, 0.0          # rotation k-2
    d_prev = np.zeros(n, dtype=b.dtype)           # direction d_{k-1}
    d_pp = np.zeros(n, dtype=b.dtype)             # direction d_{k-2}
    phibar = beta1
    its = 0
    for k in range(1, max_iter + 1):
        # Lanczos step: A v_k = beta_k v_{k-1} + alpha_k v_k + beta_{k+1} v_{k+1}
        w = matvec(v)
        if k > 1:
            w = w - beta * v_prev
        alpha = float(np.vdot(v, w).real)   # real for a Hermitian A
        w = w - alpha * v
        beta_next = float(np.linalg.norm(w))
        # column k of T_k: (beta_k at row k-1, alpha_k at row k, beta_{k+1} at row k+1)
        # rotation k-2 (identity for k <= 2) maps (0, beta_k) to (eps_k, t1);
        # column 1 has no entry above its diagonal
        eps_k = s_pp * beta if k > 1 else 0.0
        t1 = c_pp * beta if k > 1 else 0.0
        # apply rotation k-1 to (t1, alpha_k) -> (delta_k, gammabar_k)
        delta_k = c_prev * t1 + s_prev * alpha
        gbar = -s_prev * t1 + c_prev * alpha
        # new rotation annihilating beta_{k+1}
        gamma = math.hypot(gbar, beta_next)
        if gamma == 0.0:
            break
        c, s = gbar / gamma, beta_next / gamma
        tau = c * phibar
        phibar = -s * phibar
        # direction and iterate update
        d = (v - delta_k * d_prev - eps_k * d_pp) / gamma
        x = x + tau * d
        its = k
        hist.append(abs(phibar))
        if abs(phibar) <= stop_norm or beta_next == 0.0:
            break
        # shift state
        d_pp, d_prev = d_prev, d
        c_pp, s_pp = c_prev, s_prev
        c_prev, s_prev = c, s
        v_prev = v
        v = w / beta_next
        beta = beta_next
    return x, its, hist
