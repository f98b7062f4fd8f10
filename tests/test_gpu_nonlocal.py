"""GPU parity of the nonlocal term H = H_loc + F G F^T (Section 4, eqs. (k1), (fgf)):
products with the rank-k term fused into the sliced-ELL epilogues, the shifted products of
the refinement, the global apply in its Sherman-Morrison-Woodbury form, MINRES on the full
operator, and whole solves.  The oracle forms H explicitly (oracle.eigs.full_hamiltonian)
and factorises H - eps_bar S as it is, so the SMW identity is checked, not assumed."""
import json
import os

import numpy as np
import pytest

import pufe
from oracle import eigs as oeig
from oracle import labpsd as olab
from oracle import precond as oprec

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(A, dtype=None):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A).T))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy().T.astype(np.float64)


def _rel(a, b, s0):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b) - s0)


@pytest.fixture(scope="module")
def ctx():
    import paper_1308_2445_amd as lp
    torch = _torch()
    c = lp.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module", params=["c1nl", "c2nl"])
def nlprob(request, ctx):
    import paper_1308_2445_amd as lp
    P = pufe.workload(request.param, 0)
    print("\n[case] nonlocal workload=%s n=%d k=%d" % (request.param, P.n, P.F.shape[1]), flush=True)
    pr = lp.Problem.from_pencil(ctx, P)
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
    H = oeig.full_hamiltonian(P.H(), P.F, P.G)
    yield request.param, P, pr, H
    pr.close()


def test_products_include_the_rank_k_term(nlprob):
    import paper_1308_2445_amd as lp
    torch = _torch()
    name, P, pr, H = nlprob
    rng = np.random.default_rng(31)
    S = P.S()
    for w in (1, 9, 40):
        X = rng.standard_normal((P.n, w))
        Xd = dev(X)
        YH, YS = torch.empty_like(Xd), torch.empty_like(Xd)
        lp.labpsd_spmm(pr, Xd, YH, YS)
        torch.cuda.synchronize()
        ref = H @ X
        scale = abs(P.H()) @ np.abs(X) + abs(P.F) @ (np.abs(P.G) @ (abs(P.F.T) @ np.abs(X)))
        assert np.all(np.abs(host(YH) - ref) <= 1e-13 * scale + 1e-300)
        assert np.all(np.abs(host(YS) - S @ X) <= 1e-14 * (abs(S) @ np.abs(X)) + 1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_shifted_products_include_the_rank_k_term(nlprob, precision):
    import paper_1308_2445_amd as lp
    torch = _torch()
    name, P, pr, H = nlprob
    rng = np.random.default_rng(32)
    w = 13
    X = rng.standard_normal((P.n, w))
    sh = P.eps_bar + rng.uniform(0.5, 3.0, w)
    dt = torch.float64 if precision == 0 else torch.float32
    Xd = dev(X, dt)
    Yd = torch.empty_like(Xd)
    lp.labpsd_spmm_shifted(pr, precision, Xd, torch.from_numpy(sh).cuda(), Yd)
    torch.cuda.synchronize()
    Xu = host(Xd)
    ref = H @ Xu - (P.S() @ Xu) * sh[None, :]
    scale = (abs(P.H()) + abs(P.S()) * np.abs(sh).max()) @ np.abs(Xu) + \
        abs(P.F) @ (np.abs(P.G) @ (abs(P.F.T) @ np.abs(Xu)))
    tol = 1e-13 if precision == 0 else 3e-6
    assert np.all(np.abs(host(Yd) - ref) <= tol * scale + 1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_global_apply_in_smw_form(nlprob, precision):
    """P = -(H_loc + F G F^T - eps_bar S)^{-1} R through the factor of H_loc - eps_bar S and
    the SMW correction, against the oracle's factorisation of the full matrix: per column,
    element by element (FP64), and by the backward residual."""
    import paper_1308_2445_amd as lp
    torch = _torch()
    name, P, pr, H = nlprob
    rng = np.random.default_rng(33)
    for p in (7, 130):
        R = rng.standard_normal((P.n, p))
        Pd = torch.empty((p, P.n), dtype=torch.float64, device="cuda")
        lp.labpsd_precond_apply(pr, precision, dev(R), Pd)
        torch.cuda.synchronize()
        got = host(Pd)
        K = oprec.GlobalPreconditioner(H, P.S(), P.eps_bar)
        ref = K.apply(R)
        back = np.linalg.norm(K.K @ got + R, axis=0) / np.linalg.norm(R, axis=0)
        if precision == 0:
            assert back.max() < 1e-10
            colmax = np.abs(ref).max(axis=0)
            assert np.all(np.abs(got - ref) <= 1e-9 * colmax[None, :])
        else:
            assert back.max() < 5e-3


@pytest.mark.parametrize("precision", [0, 1])
def test_minres_on_the_full_operator(nlprob, precision):
    import paper_1308_2445_amd as lp
    torch = _torch()
    name, P, pr, H = nlprob
    S = P.S()
    m = 4 if P.n < 1000 else 8
    m0 = pufe.guard_vectors(m)
    prm = olab.Params(nev=m, m0=m0, tol=1e-14, max_outer=6, sigma0=P.sigma0, eps_bar=P.eps_bar)
    res = olab.solve(H, S, prm, pufe.start_block(P.n, m + m0, 0))
    R, _ = olab.residual_block(H @ res.Psi, S @ res.Psi, res.E, m, P.sigma0)
    K = oprec.GlobalPreconditioner(H, S, P.eps_bar)
    P0 = K.apply(R)
    cols = np.arange(m, dtype=np.int32)
    shifts = res.E[:m].copy()
    eta, cap = 0.25, 20
    Pd = dev(P0)
    its = torch.zeros(m, dtype=torch.int32, device="cuda")
    lp.labpsd_local_refine(pr, precision, dev(R), Pd, torch.from_numpy(cols).cuda(),
                           torch.from_numpy(shifts).cuda(), eta, cap, its)
    torch.cuda.synchronize()
    got = host(Pd)
    for c in range(m):
        pref, itref = olab.local_refine(H, S, P0[:, c], R[:, c], float(shifts[c]), eta, cap)
        a = H @ got[:, c] - shifts[c] * (S @ got[:, c]) + R[:, c]
        rn = np.linalg.norm(R[:, c])
        if precision == 0:
            assert int(its[c].item()) == itref
            assert np.linalg.norm(got[:, c] - pref) <= 1e-9 * np.linalg.norm(pref)
            assert np.linalg.norm(a) <= eta * rn * (1 + 1e-8) or itref == cap
        else:
            assert abs(int(its[c].item()) - itref) <= 2
            assert np.linalg.norm(a) <= 1.5 * eta * rn or int(its[c].item()) == cap


@pytest.mark.parametrize("precision", [0, 1])
def test_nonlocal_solves_match_stored_eigenvalues(nlprob, precision):
    name, P, pr, H = nlprob
    path = os.path.join(GOLDEN, "%s_eigs.json" % name)
    if not os.path.exists(path):
        pytest.skip("no stored eigenvalues for %s" % name)
    with open(path) as f:
        g = json.load(f)
    assert g["n"] == P.n and g["projectors"] == P.F.shape[1]
    m, m0 = g["nev"], g["m0"]
    out = pr.solve(m, m0, pufe.start_block(P.n, m + m0, 0), tol=1e-9, sigma0=P.sigma0, precision=precision)
    assert out.converged, out.stats
    refs = [g[k] for k in ("lam_mp", "lam_dense", "lam", "lam_eigsh") if k in g]
    assert len(refs) >= 2
    for ref in refs:
        assert _rel(out.lam, ref, P.sigma0).max() < 1e-10
    S = P.S()
    assert np.abs(out.X.T @ (S @ out.X) - np.eye(m)).max() < 1e-10
    res = oeig.relative_residuals(H, S, out.lam, out.X, P.sigma0)
    assert res.max() <= 1e-9 * 1.01
    print("[%s] precision=%d iters=%d La=%.2f" % (name, precision, out.stats["outer_iters"], out.stats["la"]))
