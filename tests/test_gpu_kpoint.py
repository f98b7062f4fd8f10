"""GPU tests of the complex Hermitian (k-point) variant, solved through the real embedding:
the Bloch free-particle closed form, the 250-dof k-point cell against dense and mpmath
eigenvalues and eigenvectors, the 16k-dof k-point cell against the stored oracle LABPSD and
ARPACK eigenvalues, the Gamma point against the real solver, and an SCF-like H update."""
import json
import os

import numpy as np
import pytest

import pufe
from oracle import eigs as oeig

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KF = (0.12, -0.24, 0.37)


def _lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1308_2445_amd as lp
    return lp


def _rel(a, b, s0):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b) - s0)


@pytest.fixture(scope="module")
def ctx():
    import torch
    c = _lp().Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _hermitian(ctx, P, coords=True):
    lp = _lp()
    pr = lp.Problem.from_pencil(ctx, P)
    assert isinstance(pr, lp.HermitianProblem)
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P) if coords else None)
    return pr


def _check_pairs(P, out, tol):
    H, S = P.H(), P.S()
    X = out.X
    m = X.shape[1]
    assert np.abs(X.conj().T @ (S @ X) - np.eye(m)).max() < 1e-10
    res = oeig.relative_residuals(H, S, out.lam, X, P.sigma0)
    assert res.max() <= 10 * tol


@pytest.mark.parametrize("precision", [0, 1])
def test_bloch_free_particle(ctx, precision):
    P = pufe.generate(6.0, 12, 0, 0, kpoint=KF)
    P.eps_bar, P.sigma0 = -0.1, -1.0
    pr = _hermitian(ctx, P)
    out = pr.solve(9, 4, None, tol=1e-10, sigma0=P.sigma0, precision=precision, seed=5)
    assert out.converged, out.stats
    ref = pufe.free_particle_eigs(12, 6.0, 9, kpoint=KF)
    assert _rel(out.lam, ref, P.sigma0).max() < 1e-10
    _check_pairs(P, out, 1e-10)
    pr.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_c1k_matches_dense_and_mpmath(ctx, precision):
    P = pufe.workload("c1k", 0)
    pr = _hermitian(ctx, P)
    m = 4
    out = pr.solve(m, 4, pufe.start_block(P.n, 8, 0) + 1j * pufe.start_block(P.n, 8, 1), tol=1e-10,
                   sigma0=P.sigma0, precision=precision)
    assert out.converged, out.stats
    lam, X = oeig.dense_eigs(P.H(), P.S(), m)
    assert _rel(out.lam, lam, P.sigma0).max() < 1e-10
    path = os.path.join(GOLDEN, "c1k_eigs.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        for k in ("lam_mp", "lam_eigsh", "lam"):
            if k in g:
                assert _rel(out.lam, g[k], P.sigma0).max() < 1e-10
    _check_pairs(P, out, 1e-10)
    S = P.S()
    for cl in oeig.clusters(lam, P.sigma0):
        assert oeig.s_principal_angles(S, out.X[:, cl], X[:, cl]).max() < 1e-7
    pr.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_c2k_matches_stored_routes(ctx, precision):
    path = os.path.join(GOLDEN, "c2k_eigs.json")
    if not os.path.exists(path):
        pytest.skip("no stored eigenvalues for the 16k-dof k-point cell")
    with open(path) as f:
        g = json.load(f)
    P = pufe.workload("c2k", 0)
    assert g["n"] == P.n
    pr = _hermitian(ctx, P)
    m, m0 = g["nev"], g["m0"]
    out = pr.solve(m, m0, None, tol=1e-8, sigma0=P.sigma0, precision=precision, seed=2)
    assert out.converged, out.stats
    for ref in (g["lam"], g["lam_eigsh"]):
        assert _rel(out.lam, ref, P.sigma0).max() < 1e-10
    _check_pairs(P, out, 1e-8)
    print("[c2k] precision=%d iters=%d La=%.2f" % (precision, out.stats["outer_iters"], out.stats["la"]))
    pr.close()


def test_gamma_point_equals_the_real_solver(ctx):
    """At k = 0 the Hermitian path (complex arithmetic through the embedding) reproduces
    the real solver's eigenvalues of the same cell."""
    lp = _lp()
    P0 = pufe.workload("c1", 0)
    Pk = pufe.generate(P0.L, P0.ne, len(P0.atoms), 0, kpoint=(0.0, 0.0, 0.0))
    hr = _hermitian(ctx, Pk)
    a = hr.solve(4, 4, None, tol=1e-10, sigma0=P0.sigma0, seed=1)
    pr = lp.Problem.from_pencil(ctx, P0)
    pr.set_global_precond(P0.eps_bar, pufe.dof_coordinates(P0))
    b = pr.solve(4, 4, pufe.start_block(P0.n, 8, 0), tol=1e-10, sigma0=P0.sigma0)
    assert a.converged and b.converged
    assert _rel(a.lam, b.lam, P0.sigma0).max() < 1e-10
    hr.close()
    pr.close()


def test_kpoint_scf_like_update(ctx):
    """The next GHEP of a k-point sequence: new H through the Hermitian update, solved warm
    from the previous complex eigenvectors, matches the dense eigenvalues of the new pencil."""
    P = pufe.workload("c1k", 0)
    pr = _hermitian(ctx, P)
    a = pr.solve(4, 4, None, tol=1e-10, sigma0=P.sigma0, seed=3)
    h2 = P.h_scaled(1.01)
    pr.update_h(h2)
    X0 = np.hstack([a.X, pufe.start_block(P.n, 4, 9) + 0j])
    b = pr.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0, E0=np.concatenate([a.lam, np.zeros(4)]))
    assert b.converged
    import scipy.sparse as sp
    H2 = sp.csr_matrix((h2, P.col, P.rowptr), shape=(P.n, P.n))
    lam, _ = oeig.dense_eigs(H2, P.S(), 4)
    assert _rel(b.lam, lam, P.sigma0).max() < 1e-10
    assert b.stats["outer_iters"] < a.stats["outer_iters"]
    pr.close()
