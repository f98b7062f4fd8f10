"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import pufe
from oracle import eigs, labpsd, minres, precond, rr


@pytest.fixture(scope="module")
def tiny():
    # 4^3 mesh, one atom: about a hundred dofs, small enough for mpmath
    return pufe.generate(4.0, 4, 1, 3)


@pytest.fixture(scope="module")
def c1():
    return pufe.workload("c1", 0)


# ------------------------------------------------------------------ result definition

def test_dense_eigs_match_mpmath(tiny):
    lam, X = eigs.dense_eigs(tiny.H(), tiny.S(), 6)
    mp = eigs.mp_eigs(tiny.H(), tiny.S(), dps=40)[:6]
    assert np.max(np.abs(lam - mp) / np.abs(mp - tiny.sigma0)) < 1e-12
    S = tiny.S().toarray()
    assert np.abs(X.T @ S @ X - np.eye(6)).max() < 1e-12


def test_residual_definition_and_backward_error(c1):
    H, S = c1.H(), c1.S()
    lam, X = eigs.dense_eigs(H, S, 4)
    res = eigs.relative_residuals(H, S, lam, X, c1.sigma0)
    assert res.max() < 1e-12
    # a perturbed pair: footnote of Section 2, a rank-one Delta H makes it exact
    rng = np.random.default_rng(0)
    x = X[:, 0] + 1e-3 * rng.standard_normal(c1.n)
    e = float(x @ (H @ x)) / float(x @ (S @ x))
    r = H @ x - e * (S @ x)
    dH = -np.outer(r, x) / float(x @ x)
    assert np.abs((H.toarray() + dH) @ x - e * (S @ x)).max() < 1e-12 * np.abs(r).max() + 1e-15
    assert abs(np.linalg.norm(dH, 2) - np.linalg.norm(r) / np.linalg.norm(x)) < 1e-12
    # Res with sigma0 = 0 is the paper's bound on the relative backward error
    res_unshifted = eigs.relative_residuals(H, S, np.array([e]), x[:, None], 0.0)[0]
    rel_be = np.linalg.norm(dH, 2) / np.linalg.norm(H.toarray(), 2)
    assert rel_be <= res_unshifted * (1 + 1e-12)


def test_residual_block_matches_definition(c1):
    rng = np.random.default_rng(1)
    Psi = rng.standard_normal((c1.n, 6))
    E = np.sort(rng.standard_normal(6))
    H, S = c1.H(), c1.S()
    R, res = labpsd.residual_block(H @ Psi, S @ Psi, E, 4, c1.sigma0)
    for i in range(4):
        ri = H @ Psi[:, i] - E[i] * (S @ Psi[:, i])
        assert np.allclose(R[:, i], ri, rtol=0, atol=1e-13)
        den = np.linalg.norm(H @ Psi[:, i] - c1.sigma0 * (S @ Psi[:, i]))
        assert abs(res[i] - np.linalg.norm(ri) / den) < 1e-14
    assert R.shape[1] == 4       # only the first m columns (step 4)


# ------------------------------------------------------------------ global preconditioner

def test_global_preconditioner_is_shifted_inverse(c1):
    H, S = c1.H(), c1.S()
    K = precond.GlobalPreconditioner(H, S, c1.eps_bar)
    rng = np.random.default_rng(2)
    R = rng.standard_normal((c1.n, 5))
    P = K.apply(R)
    A = (H - c1.eps_bar * S).toarray()
    back = np.linalg.norm(A @ P + R) / np.linalg.norm(R)
    assert back < 1e-12
    assert np.allclose(P, -np.linalg.solve(A, R), rtol=1e-10, atol=1e-12)


def test_global_preconditioner_rejects_shift_above_spectrum(c1):
    lam, _ = eigs.dense_eigs(c1.H(), c1.S(), 2)
    with pytest.raises(np.linalg.LinAlgError):
        precond.GlobalPreconditioner(c1.H(), c1.S(), 0.5 * (lam[0] + lam[1]))


# ------------------------------------------------------------------ MINRES

def _krylov_lsq(A, b, k):
    """x_k = argmin over K_k(A, b) of ||b - A x|| by brute force (dense least squares)."""
    n = b.shape[0]
    Q = np.zeros((n, k))
    q = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):                         # full reorthogonalisation
            q = q - Q[:, :j] @ (Q[:, :j].T @ q)
        q = q / np.linalg.norm(q)
        Q[:, j] = q
        q = A @ q
    y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    return Q @ y


def test_minres_iterates_are_krylov_minimisers(c1):
    H, S = c1.H().toarray(), c1.S().toarray()
    lam, _ = eigs.dense_eigs(H, S, 6)
    A = H - 0.5 * (lam[2] + lam[3]) * S                # symmetric indefinite
    rng = np.random.default_rng(3)
    b = rng.standard_normal(c1.n)
    for k in range(1, 7):
        x, its, hist = minres.minres(lambda v: A @ v, b, 0.0, k)
        assert its == k
        xr = _krylov_lsq(A, b, k)
        assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)
        # the recurred residual norm is the true one, and it never increases
        assert abs(hist[-1] - np.linalg.norm(b - A @ x)) <= 1e-9 * np.linalg.norm(b)
        assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_minres_stops_at_requested_norm(c1):
    A = (c1.H() - 0.3 * c1.S()).toarray()
    rng = np.random.default_rng(4)
    b = rng.standard_normal(c1.n)
    target = 0.25 * np.linalg.norm(b)
    x, its, hist = minres.minres(lambda v: A @ v, b, target, 50)
    assert np.linalg.norm(b - A @ x) <= target * (1 + 1e-8)
    assert its >= 1 and hist[-2] > target            # it did not stop early


def test_local_refine_meets_eq_approxp(c1):
    H, S = c1.H(), c1.S()
    lam, X = eigs.dense_eigs(H, S, 4)
    rng = np.random.default_rng(5)
    psi = X[:, 1] + 1e-2 * rng.standard_normal(c1.n)
    e = float(psi @ (H @ psi)) / float(psi @ (S @ psi))
    r = H @ psi - e * (S @ psi)
    K = precond.GlobalPreconditioner(H, S, c1.eps_bar)
    p0 = K.apply(r)
    p, its = labpsd.local_refine(H, S, p0, r, e, 0.25, 20)
    assert np.linalg.norm(H @ p - e * (S @ p) + r) <= 0.25 * np.linalg.norm(r) * (1 + 1e-8)


# ------------------------------------------------------------------ Rayleigh-Ritz

def test_rayleigh_ritz_closed_form():
    rng = np.random.default_rng(6)
    k, b = 12, 5
    B = rng.standard_normal((k, k)) + 3 * np.eye(k)
    theta = np.sort(rng.standard_normal(k))
    perm = rng.permutation(k)
    HR = B.T @ np.diag(theta[perm]) @ B             # eigenpairs: B w = e_j, value theta_j
    SR = B.T @ B
    gam, W, dropped = rr.rayleigh_ritz(HR, SR, b)
    assert dropped == 0
    assert np.allclose(gam, theta[:b], rtol=0, atol=1e-12)
    assert np.abs(W.T @ SR @ W - np.eye(b)).max() < 1e-11
    assert np.abs(W.T @ HR @ W - np.diag(gam)).max() < 1e-11
    BW = B @ W                                        # columns are signed unit vectors
    for j in range(b):
        col = np.abs(BW[:, j])
        assert abs(col.max() - 1) < 1e-10 and np.sort(col)[-2] < 1e-10


def test_rayleigh_ritz_rank_revealing_fallback(c1):
    H, S = c1.H(), c1.S()
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((c1.n, 8))
    Zd = np.hstack([Z, Z[:, :2]])                   # two exactly repeated columns
    HR, SR = rr.gram(Zd, H @ Zd, S @ Zd)
    gam_d, W_d, dropped = rr.rayleigh_ritz(HR, SR, 6)
    HR0, SR0 = rr.gram(Z, H @ Z, S @ Z)
    gam0, _, _ = rr.rayleigh_ritz(HR0, SR0, 6)
    assert dropped >= 2
    assert np.allclose(gam_d, gam0, rtol=1e-9, atol=1e-12)
    assert np.abs(W_d.T @ SR @ W_d - np.eye(6)).max() < 1e-8


# ------------------------------------------------------------------ full LABPSD

def _solve(P, nev, tol=1e-8, mode="hybrid", seed=0):
    m0 = pufe.guard_vectors(nev)
    prm = labpsd.Params(nev=nev, m0=m0, tol=tol, sigma0=P.sigma0, eps_bar=P.eps_bar, mode=mode)
    return labpsd.solve(P.H(), P.S(), prm, pufe.start_block(P.n, nev + m0, seed))


def test_labpsd_matches_dense_c1(c1):
    res = _solve(c1, 4, tol=1e-12)
    assert res.converged
    lam, X = eigs.dense_eigs(c1.H(), c1.S(), 4)
    assert np.max(np.abs(res.lam - lam) / np.abs(lam - c1.sigma0)) < 1e-12
    S = c1.S()
    for cl in eigs.clusters(lam, c1.sigma0):
        ang = eigs.s_principal_angles(S, res.X[:, cl], X[:, cl])
        assert ang.max() < 1e-7
    assert res.res.max() <= 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_labpsd_matches_mpmath_tiny(tiny, seed):
    res = _solve(tiny, 5, tol=1e-11, seed=seed)
    assert res.converged
    mp = eigs.mp_eigs(tiny.H(), tiny.S(), dps=40)[:5]
    assert np.max(np.abs(res.lam - mp) / np.abs(mp - tiny.sigma0)) < 1e-11


def test_labpsd_free_particle_shell():
    # V = 0, no atoms: the lowest shell 1 + 6 is known in closed form
    P = pufe.generate(6.0, 12, 0, 0)
    P.eps_bar = -0.1
    P.sigma0 = -1.0
    res = _solve(P, 7, tol=1e-10)
    assert res.converged
    ref = pufe.free_particle_eigs(12, 6.0, 7)
    assert np.max(np.abs(res.lam - ref) / np.abs(ref - P.sigma0)) < 1e-10


def test_labpsd_iteration_invariants(c1):
    H, S = c1.H(), c1.S()
    m, m0 = 4, 4
    prm = labpsd.Params(nev=m, m0=m0, tol=1e-12, sigma0=c1.sigma0, eps_bar=c1.eps_bar)
    res = labpsd.solve(H, S, prm, pufe.start_block(c1.n, m + m0, 0))
    exact = sla.eigh(H.toarray(), S.toarray(), eigvals_only=True)[: m + m0]
    ritz = [h.ritz for h in res.history] + [res.E]
    for a, b_ in zip(ritz[:-1], ritz[1:]):
        # span(Psi) is inside span([Psi P]): Ritz values never increase (Section 3)
        assert np.all(b_ <= a + 1e-12 * np.abs(a - c1.sigma0))
    for e in ritz:
        # Courant-Fischer: the i-th Ritz value bounds the i-th eigenvalue from above
        assert np.all(e >= exact - 1e-12 * np.abs(exact - c1.sigma0))
    Psi = res.Psi
    assert np.abs(Psi.T @ (S @ Psi) - np.eye(m + m0)).max() < 1e-10
    assert np.abs(Psi.T @ (H @ Psi) - np.diag(res.E)).max() < 1e-9


def test_galerkin_condition_after_rr(c1):
    H, S = c1.H(), c1.S()
    rng = np.random.default_rng(8)
    Z = rng.standard_normal((c1.n, 10))
    HR, SR = rr.gram(Z, H @ Z, S @ Z)
    gam, W, _ = rr.rayleigh_ritz(HR, SR, 6)
    Psi = Z @ W
    Rg = H @ Psi - (S @ Psi) * gam[None, :]
    assert np.abs(Z.T @ Rg).max() < 1e-10 * np.abs(Z).max() * np.abs(Rg).max() * c1.n + 1e-10


def test_global_only_mode_still_converges_c1(c1):
    res = _solve(c1, 4, tol=1e-8, mode="global")
    assert res.converged
    assert res.minres_iters == 0
