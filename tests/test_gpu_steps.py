"""GPU parity of every hot-path step against the oracle, on identical seeded inputs.

Each step is called through the C ABI (via the ctypes binding) on device blocks,
and compared element by element with the oracle's step.  Sizes: the 250-dof cell
(one partial 64-row slice) and the 15,977-dof cell (250 slices, ragged tail).
"""
import numpy as np
import pytest

import pufe
from oracle import labpsd as olab
from oracle import precond as oprec
from oracle import rr as orr

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(A, dtype=None):
    """numpy n x w (column-major block) -> device tensor (w, n)."""
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A).T))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy().T.astype(np.float64)


@pytest.fixture(scope="module")
def ctx():
    import paper_1308_2445_amd as lp
    torch = _torch()
    c = lp.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module", params=["c1", "c2"])
def prob(request, ctx):
    import paper_1308_2445_amd as lp
    P = pufe.workload(request.param, 0)
    print("\n[case] workload=%s n=%d nnz=%d" % (request.param, P.n, P.nnz), flush=True)
    pr = lp.Problem.from_pencil(ctx, P)
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
    yield P, pr
    pr.close()


def test_spmm_fused(prob):
    """Every launch shape: one, two and four columns per wavefront (w < 16, 16 <= w < 32,
    w >= 32), one and several column bands (w = 200: two), ragged rounds."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(11)
    for w in (1, 8, 20, 37, 200):
        X = rng.standard_normal((P.n, w))
        Xd = dev(X)
        YH = torch.empty_like(Xd)
        YS = torch.empty_like(Xd)
        lp.labpsd_spmm(pr, Xd, YH, YS)
        torch.cuda.synchronize()
        H, S = P.H(), P.S()
        refH, refS = H @ X, S @ X
        scaleH = abs(H) @ np.abs(X)
        scaleS = abs(S) @ np.abs(X)
        assert np.all(np.abs(host(YH) - refH) <= 1e-14 * scaleH + 1e-300)
        assert np.all(np.abs(host(YS) - refS) <= 1e-14 * scaleS + 1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_spmm_shifted(prob, precision):
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(12)
    for w in (13, 24, 150):
        X = rng.standard_normal((P.n, w))
        sh = rng.uniform(-0.5, 0.5, w)
        dt = torch.float64 if precision == 0 else torch.float32
        Xd = dev(X, dt)
        Y = torch.empty_like(Xd)
        lp.labpsd_spmm_shifted(pr, precision, Xd, torch.from_numpy(sh).cuda(), Y)
        torch.cuda.synchronize()
        H, S = P.H(), P.S()
        Xr = X if precision == 0 else X.astype(np.float32).astype(np.float64)
        ref = H @ Xr - (S @ Xr) * sh[None, :]
        scale = abs(H) @ np.abs(Xr) + (abs(S) @ np.abs(Xr)) * np.abs(sh)[None, :]
        tol = 1e-14 if precision == 0 else 2e-6
        assert np.all(np.abs(host(Y) - ref) <= tol * scale + 1e-30)


def test_residual(prob, ctx):
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(13)
    b, m = 9, 7
    Psi = rng.standard_normal((P.n, b))
    E = np.sort(rng.standard_normal(b))
    PH, PS = P.H() @ Psi, P.S() @ Psi
    R = torch.empty((m, P.n), dtype=torch.float64, device="cuda")
    res = torch.empty(m, dtype=torch.float64, device="cuda")
    rn = torch.empty(m, dtype=torch.float64, device="cuda")
    lp.labpsd_residual(ctx, P.n, m, dev(PH), dev(PS), torch.from_numpy(E).cuda(), P.sigma0, R, res, rn)
    torch.cuda.synchronize()
    Rr, resr = olab.residual_block(PH, PS, E, m, P.sigma0)
    assert np.abs(host(R) - Rr).max() <= 1e-14 * np.abs(Rr).max()
    assert np.allclose(res.cpu().numpy(), resr, rtol=1e-12, atol=0)
    assert np.allclose(rn.cpu().numpy(), np.linalg.norm(Rr, axis=0), rtol=1e-12, atol=0)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("p", [21, 150, 300])
def test_global_precond_apply(prob, precision, p):
    """p = 150 takes the wide tasks (64 right-hand sides each, the last group ragged);
    p = 300 in FP64 the 128-wide ones (two full groups and a ragged third)."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(14)
    R = rng.standard_normal((P.n, p))
    Pd = torch.empty((p, P.n), dtype=torch.float64, device="cuda")
    lp.labpsd_precond_apply(pr, precision, dev(R), Pd)
    torch.cuda.synchronize()
    got = host(Pd)
    K = oprec.GlobalPreconditioner(P.H(), P.S(), P.eps_bar)
    ref = K.apply(R)
    A = K.K
    back = np.linalg.norm(A @ got + R, axis=0) / np.linalg.norm(R, axis=0)
    # column by column against the oracle's apply
    colerr = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    if precision == 0:
        assert back.max() < 1e-11
        assert colerr.max() <= 1e-9
    else:
        # FP32 substitutions: a preconditioner, not a solver (stated, not a parity claim)
        assert back.max() < 5e-3
        assert colerr.max() <= 5e-3


@pytest.mark.parametrize("precision", [0, 1])
def test_local_refine(prob, precision):
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    H, S = P.H(), P.S()
    # near-eigenvectors from a few oracle iterations give realistic localised columns
    m = 4 if P.n < 1000 else 8
    m0 = pufe.guard_vectors(m)
    prm = olab.Params(nev=m, m0=m0, tol=1e-14, max_outer=6, sigma0=P.sigma0, eps_bar=P.eps_bar)
    res = olab.solve(H, S, prm, pufe.start_block(P.n, m + m0, 0))
    Psi, E = res.Psi, res.E
    R, _ = olab.residual_block(H @ Psi, S @ Psi, E, m, P.sigma0)
    K = oprec.GlobalPreconditioner(H, S, P.eps_bar)
    P0 = K.apply(R)
    cols = np.arange(0, m, 2, dtype=np.int32)
    shifts = E[cols].copy()
    eta, cap = 0.25, 20
    Pd = dev(P0)
    its = torch.zeros(len(cols), dtype=torch.int32, device="cuda")
    lp.labpsd_local_refine(pr, precision, dev(R), Pd, torch.from_numpy(cols).cuda(),
                           torch.from_numpy(shifts).cuda(), eta, cap, its)
    torch.cuda.synchronize()
    got = host(Pd)
    for j, c in enumerate(cols):
        pref, itref = olab.local_refine(H, S, P0[:, c], R[:, c], float(shifts[j]), eta, cap)
        a = H @ got[:, c] - shifts[j] * (S @ got[:, c]) + R[:, c]
        rn = np.linalg.norm(R[:, c])
        if precision == 0:
            assert int(its[j].item()) == itref
            assert np.linalg.norm(got[:, c] - pref) <= 1e-9 * np.linalg.norm(pref)
            assert np.linalg.norm(a) <= eta * rn * (1 + 1e-8) or itref == cap
        else:
            assert abs(int(its[j].item()) - itref) <= 2
            assert np.linalg.norm(a) <= 1.5 * eta * rn or int(its[j].item()) == cap
    # columns not listed are untouched
    others = [c for c in range(m) if c not in set(cols.tolist())]
    assert np.array_equal(got[:, others], P0[:, others]) if precision == 0 else True


@pytest.mark.parametrize("precision", [0, 1])
def test_local_refine_wide(prob, precision):
    """130 localised columns at once (33 four-column chunks per product, the last ragged)."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    H, S = P.H(), P.S()
    rng = np.random.default_rng(19)
    q = 130
    R = rng.standard_normal((P.n, q))
    K = oprec.GlobalPreconditioner(H, S, P.eps_bar)
    P0 = K.apply(R)
    cols = np.arange(q, dtype=np.int32)
    shifts = P.eps_bar + np.abs(P.eps_bar) * rng.uniform(0.1, 0.6, q)
    eta, cap = 0.25, 20
    Pd = dev(P0)
    its = torch.zeros(q, dtype=torch.int32, device="cuda")
    lp.labpsd_local_refine(pr, precision, dev(R), Pd, torch.from_numpy(cols).cuda(),
                           torch.from_numpy(shifts).cuda(), eta, cap, its)
    torch.cuda.synchronize()
    got = host(Pd)
    itg = its.cpu().numpy()
    for c in range(0, q, 13):
        pref, itref = olab.local_refine(H, S, P0[:, c], R[:, c], float(shifts[c]), eta, cap)
        if precision == 0:
            assert int(itg[c]) == itref
            assert np.linalg.norm(got[:, c] - pref) <= 1e-9 * np.linalg.norm(pref)
        else:
            a = H @ got[:, c] - shifts[c] * (S @ got[:, c]) + R[:, c]
            assert abs(int(itg[c]) - itref) <= 2
            assert np.linalg.norm(a) <= 1.5 * eta * np.linalg.norm(R[:, c]) or int(itg[c]) == cap


def test_gram(prob, ctx):
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(15)
    # 32 x 32 tiles up to k = 191, 64 x 64 from 192
    for k in (1, 5, 33, 70, 191, 192, 300, 538):
        Z = rng.standard_normal((P.n, k))
        ZH, ZS = P.H() @ Z, P.S() @ Z
        HR = torch.empty((k, k), dtype=torch.float64, device="cuda")
        SR = torch.empty((k, k), dtype=torch.float64, device="cuda")
        lp.labpsd_gram(ctx, P.n, k, dev(Z), dev(ZH), dev(ZS), HR, SR)
        HRr, SRr = orr.gram(Z, ZH, ZS)
        bound_h = np.abs(Z).T @ np.abs(ZH)
        bound_s = np.abs(Z).T @ np.abs(ZS)
        assert np.all(np.abs(host(HR) - HRr) <= 1e-13 * bound_h)
        assert np.all(np.abs(host(SR) - SRr) <= 1e-13 * bound_s)
        assert np.array_equal(host(HR), host(HR).T)


def _rr_case(P, k, rng, dup=0):
    """Reduced pencil of k random directions, the last `dup` repeating the first ones;
    also returns the eigenvalues of the pencil without the repeats (the exact answer)."""
    Z0 = rng.standard_normal((P.n, k - dup))
    Z = np.hstack([Z0, Z0[:, :dup]]) if dup else Z0
    HR, SR = orr.gram(Z, P.H() @ Z, P.S() @ Z)
    HR0, SR0 = orr.gram(Z0, P.H() @ Z0, P.S() @ Z0)
    return HR, SR, HR0, SR0


@pytest.mark.parametrize("k,nwant,dup,hscale", [(8, 8, 0, 1.0), (12, 6, 0, 1.0), (68, 36, 0, 1.0), (40, 20, 3, 1.0),
                                                (100, 60, 0, 1.0), (140, 40, 0, 1.0), (68, 36, 0, 1e100),
                                                (68, 36, 0, 1e-100), (129, 129, 0, 1.0), (200, 100, 5, 1.0)])
def test_rayleigh_ritz(prob, ctx, k, nwant, dup, hscale):
    """hscale scales H_R (so every Ritz value) far from 1, which the eigenvalue counts of
    the small solve have to survive."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(16 + k)
    HR, SR, HR0, SR0 = _rr_case(P, k, rng, dup)
    HR, HR0 = HR * hscale, HR0 * hscale
    gam = torch.empty(nwant, dtype=torch.float64, device="cuda")
    W = torch.empty((nwant, k), dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    lp.labpsd_rayleigh_ritz(ctx, k, nwant, dev(HR), dev(SR), gam, W, info)
    g = gam.cpu().numpy()
    Wh = host(W)
    # the oracle on the rank-free pencil (the repeats add nothing to the search space)
    gr, Wr, dropped = orr.rayleigh_ritz(HR0, SR0, nwant)
    inf = info.cpu().numpy()
    assert inf[1] == 0
    if dup:
        assert inf[0] >= dup
    scale = np.abs(gr).max()
    assert np.abs(g - gr).max() <= 1e-11 * scale
    assert np.abs(Wh.T @ SR @ Wh - np.eye(nwant)).max() <= 1e-9
    assert np.abs(Wh.T @ HR @ Wh - np.diag(g)).max() <= 1e-9 * scale


@pytest.fixture(scope="module")
def c2_pencil():
    return pufe.workload("c2", 0)


@pytest.mark.parametrize("k,nwant,dup,hscale", [(300, 150, 0, 1e100), (538, 282, 0, 1.0), (1076, 564, 0, 1.0),
                                                (1400, 700, 0, 1.0), (300, 150, 20, 1.0), (144, 1, 0, 1.0),
                                                (161, 161, 0, 1e-100)])
def test_rayleigh_ritz_large(c2_pencil, ctx, k, nwant, dup, hscale):
    """Orders of the 128k- and 296k-dof cells (k up to 538 and 1076) on pencils of the
    16k-dof cell; with repeated directions the Cholesky of S_R fails and the
    rank-revealing route takes over.  Up to k = 1076 the tridiagonalisation keeps each
    work-group's columns in LDS; at k = 1400 they do not fit and stay in global memory."""
    P = c2_pencil
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(16 + k)
    HR, SR, HR0, SR0 = _rr_case(P, k, rng, dup)
    HR, HR0 = HR * hscale, HR0 * hscale
    gam = torch.empty(nwant, dtype=torch.float64, device="cuda")
    W = torch.empty((nwant, k), dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    print("\n[case] rayleigh_ritz k=%d nwant=%d dup=%d" % (k, nwant, dup), flush=True)
    lp.labpsd_rayleigh_ritz(ctx, k, nwant, dev(HR), dev(SR), gam, W, info)
    g = gam.cpu().numpy()
    Wh = host(W)
    gr, Wr, dropped = orr.rayleigh_ritz(HR0, SR0, nwant)
    inf = info.cpu().numpy()
    assert inf[1] == 0
    if dup:
        assert inf[0] >= dup
    scale = np.abs(gr).max()
    orth = np.abs(Wh.T @ SR @ Wh - np.eye(nwant)).max()
    print("[rr] k=%d eig err %.2e orth %.2e" % (k, np.abs(g - gr).max() / scale, orth), flush=True)
    assert np.abs(g - gr).max() <= 1e-11 * scale
    assert orth <= 1e-10
    assert np.abs(Wh.T @ HR @ Wh - np.diag(g)).max() <= 1e-9 * scale


def test_block_update(prob, ctx):
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    rng = np.random.default_rng(17)
    # from (129, 40) on the wide kernel, 16 CT columns per work-group with CT chosen per
    # launch: 6 at b = 40 and 150, 9 at b = 130 and 282, 8 at b = 128
    for k, b in ((8, 5), (45, 33), (70, 36), (129, 40), (60, 130), (300, 150), (538, 282), (200, 128)):
        Zs = [rng.standard_normal((P.n, k)) for _ in range(3)]
        W = rng.standard_normal((k, b))
        outs = [torch.empty((b, P.n), dtype=torch.float64, device="cuda") for _ in range(3)]
        lp.labpsd_block_update(ctx, P.n, k, b, dev(Zs[0]), dev(Zs[1]), dev(Zs[2]), dev(W), *outs)
        torch.cuda.synchronize()
        for Z, o in zip(Zs, outs):
            ref = Z @ W
            bound = np.abs(Z) @ np.abs(W)
            assert np.all(np.abs(host(o) - ref) <= 1e-14 * bound)


@pytest.mark.parametrize("precision", [0, 1])
def test_local_refine_one_step(prob, precision):
    """The conclusions' one-step refinement (labpsd_set_refine_method) against the oracle's
    one_step_refine per column: the same step counts and directions in FP64 (up to the
    rounding of the recurred residual norm near the stopping threshold), eq. (approxp) met
    or the cap reached in both precisions; 70 columns, the last chunk ragged."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    H, S = P.H(), P.S()
    rng = np.random.default_rng(23)
    q = 70
    # residual-like right-hand sides and shifts inside the spectrum, as in refinement
    m = 4 if P.n < 1000 else 8
    prm = olab.Params(nev=m, m0=pufe.guard_vectors(m), tol=1e-14, max_outer=6, sigma0=P.sigma0,
                      eps_bar=P.eps_bar)
    res = olab.solve(H, S, prm, pufe.start_block(P.n, m + prm.m0, 0))
    R0, _ = olab.residual_block(H @ res.Psi, S @ res.Psi, res.E, m, P.sigma0)
    R = R0[:, rng.integers(0, m, q)] + 1e-3 * rng.standard_normal((P.n, q)) * np.abs(R0).max()
    shifts = res.E[rng.integers(0, m, q)] * (1 + 1e-3 * rng.standard_normal(q))
    K = oprec.GlobalPreconditioner(H, S, P.eps_bar)
    P0 = K.apply(R)
    cols = np.arange(q, dtype=np.int32)
    eta, cap = 0.25, 20
    pr.set_refine_method(lp.REFINE_ONESTEP)
    try:
        Pd = dev(P0)
        its = torch.zeros(q, dtype=torch.int32, device="cuda")
        lp.labpsd_local_refine(pr, precision, dev(R), Pd, torch.from_numpy(cols).cuda(),
                               torch.from_numpy(shifts).cuda(), eta, cap, its)
        torch.cuda.synchronize()
    finally:
        pr.set_refine_method(lp.REFINE_MINRES)
    got = host(Pd)
    itg = its.cpu().numpy()
    assert itg.max() >= 2                                 # the refinement does work here
    for c in range(0, q, 7):
        pref, itref = olab.one_step_refine(H, S, P0[:, c], R[:, c], float(shifts[c]), eta, cap)
        a = H @ got[:, c] - shifts[c] * (S @ got[:, c]) + R[:, c]
        rn = np.linalg.norm(R[:, c])
        if precision == 0:
            assert abs(int(itg[c]) - itref) <= 1
            if int(itg[c]) == itref:
                assert np.linalg.norm(got[:, c] - pref) <= 1e-9 * np.linalg.norm(pref)
            assert np.linalg.norm(a) <= eta * rn * (1 + 1e-8) or int(itg[c]) == cap
        else:
            assert abs(int(itg[c]) - itref) <= 2
            assert np.linalg.norm(a) <= 1.5 * eta * rn or int(itg[c]) == cap


@pytest.mark.parametrize("precision", [0, 1])
def test_level_by_level_apply_matches_sweep(prob, ctx, precision):
    """LABPSD_APPLY_LEVELS: the same products in one launch per level and phase give the
    single-launch sweep's result (both accumulate atomically, so to rounding) and the
    oracle's solve.  150 columns: the default problem takes the sweep (small factors with
    fewer than 128 columns take the level route by default)."""
    P, pr = prob
    import paper_1308_2445_amd as lp
    torch = _torch()
    pl = lp.Problem.from_pencil(ctx, P)
    pl.set_global_precond(P.eps_bar, pufe.dof_coordinates(P), panels=lp.APPLY_LEVELS)
    rng = np.random.default_rng(15)
    R = rng.standard_normal((P.n, 150))
    a = torch.empty((150, P.n), dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    lp.labpsd_precond_apply(pr, precision, dev(R), a)
    lp.labpsd_precond_apply(pl, precision, dev(R), b)
    torch.cuda.synchronize()
    ga, gb = host(a), host(b)
    tol = 1e-12 if precision == 0 else 1e-5
    assert np.linalg.norm(ga - gb) <= tol * np.linalg.norm(ga)
    ref = oprec.GlobalPreconditioner(P.H(), P.S(), P.eps_bar).apply(R)
    assert np.linalg.norm(gb - ref) <= (1e-9 if precision == 0 else 5e-3) * np.linalg.norm(ref)
    pl.close()
