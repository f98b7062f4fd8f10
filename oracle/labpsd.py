"""LABPSD, the locally accelerated block preconditioned steepest descent method,
taken step by step from the outline in Section 3 with the hybrid preconditioning
scheme of Section 3 and the implementation choices of Sections 4 and 5.

Readings where the paper is silent or garbled (all shared with the GPU solver's
documentation):
  * Res uses the shifted denominator ||(H - sigma0 S) psi|| (Section 5 shifts H
    by sigma0; eq. (res1)).
  * In step 6(b) the refinement residual is delta r_i = (H - eps_i S) p_i + r_i with
    the Ritz value eps_i; with eps_bar, as printed, it would vanish identically
    after an exact global solve.  This is the same as running MINRES on
    eq. (indls) from the start vector p_i (Section 4).
  * Localisation needs the previous iteration's Ritz value; on the first
    iteration of a cold start there is none, so no column is localised there.
    A warm start may pass E0 to serve as that previous value.
  * The stored products Psi_H, Psi_S are updated by recurrence (step 11); they
    are recomputed from H and S every ``refresh_every`` iterations and always
    before convergence is accepted, so that convergence is declared on the true
    residual.
  * A cold start runs one Rayleigh-Ritz step on the start block before the loop.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from .eigs import relative_residuals  # noqa: F401  (re-exported for tests)
from .minres import minres
from .precond import GlobalPreconditioner
from .rr import gram, rayleigh_ritz


@dataclasses.dataclass
class Params:
    nev: int                       # m: wanted eigenpairs
    m0: int                        # guard vectors (Section 3, remark 1)
    tol: float = 1e-8              # tau_eig on Res_max (eq. (resL))
    max_outer: int = 200           # outer BPSD cap
    sigma0: float = 0.0            # shift in the Res denominator (Section 5)
    eps_bar: float = 0.0           # global preconditioner shift (eq. (globalprecond))
    tau1: float = 0.1              # localisation: Res_i <= tau1  (Section 3, remark 4)
    tau2: float = 0.1              # localisation: |eps_i - eps_i^prev| <= tau2 |eps_i^prev|
    eta: float = 0.25              # inexact local solve (eq. (approxp)), Section 5
    max_inner: int = 20            # MINRES cap (Section 5)
    mode: str = "hybrid"           # "hybrid" | "global" | "local"
    refine: str = "minres"         # "minres" (Section 4) | "onestep" (the conclusions' variant)
    refresh_every: int = 10

    @property
    def b(self) -> int:
        return self.nev + self.m0


@dataclasses.dataclass
class IterRecord:
    res: np.ndarray                # Res_i, i < m, at the start of the iteration
    ritz: np.ndarray               # Ritz values E (all b) at the start of the iteration
    unconverged: np.ndarray        # indices U
    localized: np.ndarray          # indices refined by MINRES
    minres_its: np.ndarray         # MINRES iterations per localised column
    rank_dropped: int


@dataclasses.dataclass
class Result:
    lam: np.ndarray
    X: np.ndarray
    E: np.ndarray
    Psi: np.ndarray
    res: np.ndarray
    converged: bool
    outer_iters: int
    minres_iters: int
    history: list
    t_setup: float
    t_solve: float

    @property
    def hp(self) -> float:
        """Outer iterations of this solve (Hp for one GHEP, Section 5.2)."""
        return float(self.outer_iters)

    @property
    def la(self) -> float:
        """MINRES iterations per outer iteration per eigenpair (La, Section 5.2)."""
        m = self.lam.shape[0]
        return self.minres_iters / max(1, self.outer_iters * m)


def residual_block(PsiH, PsiS, E, m: int, sigma0: float):
    """Outline step 4 and eq. (res1): R = Psi_H[:, :m] - Psi_S[:, :m] E[:m] and Res_i."""
    R = PsiH[:, :m] - PsiS[:, :m] * E[None, :m]
    den = np.linalg.norm(PsiH[:, :m] - sigma0 * PsiS[:, :m], axis=0)
    return R, np.linalg.norm(R, axis=0) / den


def localized_columns(U, res, E, E_prev, tau1: float, tau2: float):
    """Section 3, remark 4: pair i is localised if Res_i <= tau1 and its Ritz value
    moved by at most tau2 relative to the previous iteration's."""
    if E_prev is None:
        return np.zeros(0, dtype=np.int64)
    sel = [i for i in U if res[i] <= tau1 and abs(E[i] - E_prev[i]) <= tau2 * abs(E_prev[i])]
    return np.array(sel, dtype=np.int64)


def local_refine(H, S, p, r, eps: float, eta: float, max_inner: int):
    """Outline step 6(b): correct p so that ||(H - eps S) p + r|| <= eta ||r||.

    delta r = (H - eps S) p + r; MINRES on (H - eps S) dp = -delta r from dp = 0,
    stopped at ||delta r + (H - eps S) dp|| <= eta ||r|| (eq. (approxp)); p + dp.
    Returns (p_new, iterations).
    """
    def A(v):
        return H @ v - eps * (S @ v)
    dr = A(p) + r
    target = eta * float(np.linalg.norm(r))
    dp, its, _ = minres(A, -dr, target, max_inner)
    return p + dp, its


def one_step_refine(H, S, p, r, eps: float, eta: float, max_inner: int):
    """The first-order one-step refinement the conclusions propose in place of MINRES:
    p <- p - alpha [(H - eps S) p + r], alpha chosen to minimise the residual norm of
    eq. (idealp), ||(H - eps S) p_new + r||, for that step.  (The printed update has
    '- r_i' inside the bracket, which would minimise ||(H - eps S) p - r||; with eq.
    (idealp)'s right-hand side -r_i the bracket is that equation's residual, + r_i.)
    Each step recomputes rho = (H - eps S) p + r from p; alpha = rho.A rho / ||A rho||^2
    is the minimiser of ||rho - alpha A rho|| over alpha.  Stops when ||rho|| <= eta ||r||
    (eq. (approxp)) or after max_inner steps.  Returns (p_new, steps)."""
    def A(v):
        return H @ v - eps * (S @ v)
    target = eta * float(np.linalg.norm(r))
    p = np.array(p, dtype=np.result_type(p, r), copy=True)
    steps = 0
    for _ in range(max_inner):
        rho = A(p) + r
        if float(np.linalg.norm(rho)) <= target:
            break
        Arho = A(rho)
        den = float(np.vdot(Arho, Arho).real)
        if den == 0.0:
            break
        alpha = np.vdot(Arho, rho) / den     # the minimiser of ||rho - alpha A rho|| (real here)
        p = p - alpha * rho
        steps += 1
    return p, steps


def initial_rr(H, S, X0, b: int):
    """Rayleigh-Ritz on span(X0): the start block becomes S-orthonormal Ritz vectors."""
    XH = H @ X0
    XS = S @ X0
    HR, SR = gram(X0, XH, XS)
    gam, W, _ = rayleigh_ritz(HR, SR, b)
    return gam, X0 @ W, XH @ W, XS @ W


def solve(H, S, params: Params, X0: np.ndarray, E0: np.ndarray | None = None,
          precond: GlobalPreconditioner | None = None) -> Result:
    """Run LABPSD (Section 3 outline) until Res_max <= tol over the first m pairs."""
    m, b = params.nev, params.b
    n = H.shape[0]
    if X0.shape != (n, b):
        raise ValueError("X0 must be n x (nev + m0)")
    t0 = time.perf_counter()
    K = precond if precond is not None else GlobalPreconditioner(H, S, params.eps_bar)
    t1 = time.perf_counter()

    # steps 1-3: start block, products
    E, Psi, PsiH, PsiS = initial_rr(H, S, np.asarray(X0, dtype=np.result_type(X0, H.dtype)), b)
    E_prev = None if E0 is None else np.asarray(E0, dtype=np.float64)[:m].copy()
    fresh = True
    since_refresh = 0
    history = []
    minres_total = 0
    converged = False
    res = None
    outer = 0
    for it in range(1, params.max_outer + 1):
        if since_refresh >= params.refresh_every:
            PsiH, PsiS = H @ Psi, S @ Psi
            fresh, since_refresh = True, 0
        # step 4: residuals and Res
        R, res = residual_block(PsiH, PsiS, E, m, params.sigma0)
        # step 5: convergence on the true residual
        if res.max() <= params.tol:
            if not fresh:
                PsiH, PsiS = H @ Psi, S @ Psi
                fresh, since_refresh = True, 0
                R, res = residual_block(PsiH, PsiS, E, m, params.sigma0)
            if res.max() <= params.tol:
                converged = True
                break
        outer = it
        # step 6: search directions for the unconverged pairs only (remark 3)
        U = np.nonzero(res > params.tol)[0]
        RU = R[:, U]
        loc = localized_columns(U, res, E, E_prev, params.tau1, params.tau2) \
            if params.mode in ("hybrid", "local") else np.zeros(0, dtype=np.int64)
        # 6(a) global preconditioner
        P = K.apply(RU)
        if params.mode == "local":
            # local-only ablation: localised columns start their refinement from zero
            for i in loc:
                P[:, np.searchsorted(U, i)] = 0.0
        # 6(b) local refinement of localised pairs
        its = np.zeros(loc.shape[0], dtype=np.int64)
        refine = one_step_refine if params.refine == "onestep" else local_refine
        for j, i in enumerate(loc):
            c = int(np.searchsorted(U, i))
            P[:, c], its[j] = refine(H, S, P[:, c], R[:, i], float(E[i]), params.eta, params.max_inner)
        minres_total += int(its.sum())
        # step 7: products of P
        PH, PS = H @ P, S @ P
        # steps 8-9: reduced pencil and its lowest b pairs
        Z = np.hstack([Psi, P])
        ZH = np.hstack([PsiH, PH])
        ZS = np.hstack([PsiS, PS])
        HR, SR = gram(Z, ZH, ZS)
        gam, W, dropped = rayleigh_ritz(HR, SR, b)
        history.append(IterRecord(res=res.copy(), ritz=E.copy(), unconverged=U, localized=loc,
                                  minres_its=its, rank_dropped=dropped))
        # steps 10-11: block update
        Psi, PsiH, PsiS = Z @ W, ZH @ W, ZS @ W
        E_prev = E[:m].copy()
        E = gam
        fresh = False
        since_refresh += 1
    t2 = time.perf_counter()
    return Result(lam=E[:m].copy(), X=Psi[:, :m].copy(), E=E.copy(), Psi=Psi, res=res,
                  converged=converged, outer_iters=outer, minres_iters=minres_total,
                  history=history, t_setup=t1 - t0, t_solve=t2 - t1)
