"""GPU tests of the boundary's input forms: the seeded cold start (X0 = NULL),
device-resident CSR and H values, and the precision mask of the global factor."""
import numpy as np
import pytest

import pufe
from oracle import eigs as oeig

pytestmark = pytest.mark.gpu


def _lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1308_2445_amd as lp
    return lp


@pytest.fixture(scope="module")
def ctx():
    import torch
    c = _lp().Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def c1():
    P = pufe.workload("c1", 0)
    lam, X = oeig.dense_eigs(P.H(), P.S(), 4)
    return P, lam, X


def _rel(a, b, s0):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b) - s0)


def test_seeded_start_is_deterministic_and_correct(ctx, c1):
    """X0 = NULL: the library draws the start block from params.seed.  The same seed gives
    the same start block (the first iteration's residuals agree bit for bit: nothing before
    the first preconditioner apply reduces in a run-dependent order), another seed a
    different start and the same eigenpairs to the tolerance."""
    lp = _lp()
    P, lam, X = c1
    pr = lp.Problem.from_pencil(ctx, P)
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
    print("\n[case] c1 seeded start", flush=True)
    a = pr.solve(4, 4, None, tol=1e-10, sigma0=P.sigma0, seed=7)
    b = pr.solve(4, 4, None, tol=1e-10, sigma0=P.sigma0, seed=7)
    c = pr.solve(4, 4, None, tol=1e-10, sigma0=P.sigma0, seed=8)
    assert a.converged and b.converged and c.converged
    assert np.array_equal(a.res_hist[0], b.res_hist[0])
    assert _rel(a.lam, b.lam, P.sigma0).max() < 1e-12
    assert not np.array_equal(a.res_hist[0], c.res_hist[0])     # a different start block
    for out in (a, c):
        assert _rel(out.lam, lam, P.sigma0).max() < 1e-10
        for cl in oeig.clusters(lam, P.sigma0):
            assert oeig.s_principal_angles(P.S(), out.X[:, cl], X[:, cl]).max() < 1e-6


def test_device_resident_csr_and_h(ctx, c1):
    """A problem created from device arrays, and an H update from a device array, give
    the run of the host-array forms (the same first residuals bit for bit; the global
    apply's atomic accumulation may reorder later sums)."""
    import torch
    lp = _lp()
    P, lam, _ = c1
    host = lp.Problem.from_pencil(ctx, P)
    dev = lp.Problem(ctx, P.n, torch.from_numpy(P.rowptr).cuda(), torch.from_numpy(P.col).cuda(),
                     torch.from_numpy(P.h_val).cuda(), torch.from_numpy(P.s_val).cuda())
    for pr in (host, dev):
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
    X0 = pufe.start_block(P.n, 8, 0)
    a = host.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0)
    b = dev.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0)
    assert np.array_equal(a.res_hist[0], b.res_hist[0])
    assert _rel(a.lam, b.lam, P.sigma0).max() < 1e-12
    # the next GHEP of an SCF-like sequence, H given on the device
    P2 = pufe.generate(P.L, P.ne, 0, 0, atoms=P.atoms, amplitudes=P.amplitudes * 1.01)
    host.update_h(P2.h_val)
    dev.update_h(torch.from_numpy(P2.h_val).cuda())
    a = host.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0)
    b = dev.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0)
    assert np.array_equal(a.res_hist[0], b.res_hist[0])
    lam2, _ = oeig.dense_eigs(P2.H(), P2.S(), 4)
    assert _rel(b.lam, lam2, P.sigma0).max() < 1e-10


def test_precision_mask(ctx, c1):
    """Only the selected factor copies are uploaded: a solve in the other precision is
    refused (ESTATE), the selected one runs; unknown mask bits (16) are rejected."""
    lp = _lp()
    P, lam, _ = c1
    X0 = pufe.start_block(P.n, 8, 0)
    for panels, ok, bad in ((lp.PANELS_FP32, lp.MIXED, lp.FP64), (lp.PANELS_FP64, lp.FP64, lp.MIXED)):
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P), panels=panels)
        out = pr.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0, precision=ok)
        assert out.converged and _rel(out.lam, lam, P.sigma0).max() < 1e-10
        with pytest.raises(lp.LabpsdError) as e:
            pr.solve(4, 4, X0, tol=1e-10, sigma0=P.sigma0, precision=bad)
        assert e.value.code == lp.ESTATE
        pr.close()
    pr = lp.Problem.from_pencil(ctx, P)
    with pytest.raises(lp.LabpsdError) as e:
        pr.set_global_precond(P.eps_bar, None, panels=16)    # no such bit
    assert e.value.code == lp.EINVAL
    pr.close()
