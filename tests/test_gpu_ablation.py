"""GPU tests of the preconditioning variants that Section 5.4 and the conclusions compare:
global-only, local-only and hybrid preconditioning over an SCF-like warm-started sequence,
and a global factor computed in single precision."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import pufe
from oracle import eigs as oeig

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


@pytest.mark.parametrize("panels,precision", [("fp32", 1), ("fp64", 0)])
def test_single_precision_factorisation(ctx, panels, precision):
    """H - eps_bar S factorised in FP32 arithmetic (LABPSD_FACTOR_FP32) still preconditions a
    solve to the stored eigenvalues of the 16k-dof cell at the same tolerance."""
    lp = _lp()
    P = pufe.workload("c2", 0)
    with open(os.path.join(GOLDEN, "c2_eigs.json")) as f:
        g = json.load(f)
    pr = lp.Problem.from_pencil(ctx, P)
    mask = (lp.PANELS_FP32 if panels == "fp32" else lp.PANELS_FP64) | lp.FACTOR_FP32
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P), panels=mask)
    m, m0 = g["nev"], g["m0"]
    out = pr.solve(m, m0, pufe.start_block(P.n, m + m0, 0), tol=1e-8, sigma0=P.sigma0, precision=precision)
    assert out.converged, out.stats
    for ref in (g["lam"], g["lam_eigsh"]):
        assert _rel(out.lam, ref, P.sigma0).max() < 1e-10
    print("[fp32 factor] panels=%s iters=%d La=%.2f" % (panels, out.stats["outer_iters"], out.stats["la"]))
    pr.close()


def test_three_schemes_on_an_scf_like_sequence(ctx):
    """Three warm-started steps of the 250-dof nonlocal cell (amplitudes x 1.01 per step) in
    each scheme: every step converges, the three schemes agree with the dense eigenvalues of
    that step's pencil, global-only never refines and the other two do."""
    lp = _lp()
    P = pufe.workload("c1nl", 0)
    nev, m0 = 4, pufe.guard_vectors(4)
    scales = [1.0, 1.01, 1.0201]
    refs = []
    for sc in scales:
        Hloc = sp.csr_matrix((P.h_scaled(sc), P.col, P.rowptr), shape=(P.n, P.n))
        refs.append(oeig.dense_eigs(oeig.full_hamiltonian(Hloc, P.F, P.G), P.S(), nev)[0])
    for mode, inner in ((lp.GLOBAL_ONLY, 20), (lp.LOCAL_ONLY, 500), (lp.HYBRID, 20)):
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
        srv = lp.Server(ctx, 1 << 40, 1)
        minres = 0
        for j, sc in enumerate(scales):
            pr.set_local_precond(mode=lp.GLOBAL_ONLY if (mode == lp.LOCAL_ONLY and j == 0) else mode,
                                 max_inner=inner)
            rid = srv.submit(pr, nev, m0, X0=pufe.start_block(P.n, nev + m0, 0) if j == 0 else None,
                             h_val=P.h_scaled(sc), tol=1e-10, sigma0=P.sigma0, precision=lp.MIXED)
            r = srv.wait(rid)
            assert r.converged
            assert _rel(r.lam, refs[j], P.sigma0).max() < 1e-10
            minres += r.stats["minres_iters"]
        srv.close()
        pr.close()
        if mode == lp.GLOBAL_ONLY:
            assert minres == 0
        else:
            assert minres > 0
