"""Serving (continuous batching) on the GPU: every result is the same alone and in the mix,
admission never exceeds the device budget, warm-started SCF-like chains stay correct."""
import numpy as np
import pytest

import pufe
from oracle import eigs as oeig

pytestmark = pytest.mark.gpu

# (mesh elements per side at h = 0.5, atoms, nev, seed); the two nev = 64 systems reach
# Rayleigh-Ritz orders above 128 (the cooperative many-work-group route), two of them
# at once in the mix
SYSTEMS = [(12, 1, 8, 0), (12, 3, 16, 1), (16, 2, 8, 2), (16, 5, 16, 3), (12, 2, 8, 4), (16, 4, 64, 5),
           (16, 6, 64, 6)]


def _lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1308_2445_amd as lp
    return lp


@pytest.fixture(scope="module")
def pencils():
    out = []
    for ne, na, nev, seed in SYSTEMS:
        P = pufe.generate(ne / 2.0, ne, na, seed)
        out.append((P, nev))
    return out


def _systems(ctx, pencils):
    lp = _lp()
    sys = []
    for P, nev in pencils:
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
        sys.append(pr)
    return sys


def _run(ctx, pencils, slots, budget, precision):
    """Two SCF-like steps per system: a cold start, then H with the potential scaled by
    1.01 warm-started from the first result.  Returns results and run intervals."""
    lp = _lp()
    systems = _systems(ctx, pencils)
    srv = lp.Server(ctx, budget, slots)
    first, second = [], []
    for (P, nev), pr in zip(pencils, systems):
        m0 = pufe.guard_vectors(nev)
        first.append(srv.submit(pr, nev, m0, X0=pufe.start_block(P.n, nev + m0, 7), tol=1e-9,
                                sigma0=P.sigma0, precision=precision))
    for (P, nev), pr in zip(pencils, systems):
        m0 = pufe.guard_vectors(nev)
        second.append(srv.submit(pr, nev, m0, h_val=P.h_scaled(1.01), tol=1e-9, sigma0=P.sigma0,
                                 precision=precision))
    r1 = [srv.wait(r) for r in first]
    r2 = [srv.wait(r) for r in second]
    srv.close()
    for pr in systems:
        pr.close()
    return r1, r2


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_mix(pencils, precision):
    lp = _lp()
    ctx = lp.Context(0)
    big = 1 << 40
    print("\n[case] serving alone (1 slot) precision=%d" % precision, flush=True)
    alone1, alone2 = _run(ctx, pencils, 1, big, precision)
    print("[case] serving mix (4 slots) precision=%d" % precision, flush=True)
    mix1, mix2 = _run(ctx, pencils, 4, big, precision)
    for k, (P, nev) in enumerate(pencils):
        for a, b, hv in ((alone1[k], mix1[k], P.h_val), (alone2[k], mix2[k], P.h_scaled(1.01))):
            assert a.converged and b.converged
            rel = np.abs(a.lam - b.lam) / np.abs(a.lam - P.sigma0)
            assert rel.max() < 1e-10
            # and both are the pencil's eigenvalues
            H = P.H().copy()
            H.data = hv.copy()
            lam, _ = oeig.dense_eigs(H, P.S(), nev) if P.n <= 3000 else (None, None)
            if lam is not None:
                assert (np.abs(b.lam - lam) / np.abs(lam - P.sigma0)).max() < 1e-10
            res = oeig.relative_residuals(H, P.S(), b.lam, b.X, P.sigma0)
            assert res.max() <= 1e-9 * 1.01
    # the warm-started second step needs fewer iterations than the cold first step
    its1 = sum(r.stats["outer_iters"] for r in mix1)
    its2 = sum(r.stats["outer_iters"] for r in mix2)
    assert its2 < its1
    # with four slots the requests did overlap in time
    iv = sorted((r.started, r.finished) for r in mix1 + mix2)
    assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))


def test_admission_respects_budget(pencils):
    lp = _lp()
    ctx = lp.Context(0)
    fps = [lp.solve_footprint(P.n, nev, pufe.guard_vectors(nev), lp.MIXED) for P, nev in pencils]
    budget = int(max(fps) * 1.5)        # at most one big request at a time, sometimes two
    r1, r2 = _run(ctx, pencils, 4, budget, 1)
    rs = r1 + r2
    fp = fps + fps
    events = sorted([(r.started, f) for r, f in zip(rs, fp)] + [(r.finished, -f) for r, f in zip(rs, fp)],
                    key=lambda e: (e[0], e[1]))
    cur = 0
    for _, d in events:
        cur += d
        assert cur <= budget
    assert all(r.converged for r in rs)


def test_budget_too_small_is_rejected(pencils):
    lp = _lp()
    ctx = lp.Context(0)
    P, nev = pencils[0]
    pr = _systems(ctx, pencils[:1])[0]
    srv = lp.Server(ctx, 1024, 2)
    with pytest.raises(lp.LabpsdError) as e:
        srv.submit(pr, nev, 4, X0=pufe.start_block(P.n, nev + 4, 0), sigma0=P.sigma0)
    assert e.value.code == lp.ENOMEM
    with pytest.raises(lp.LabpsdError) as e:
        srv2 = lp.Server(ctx, 1 << 40, 1)
        rid = srv2.submit(pr, nev, 4, sigma0=P.sigma0)     # warm start with nothing resident
        srv2.wait(rid)
    assert e.value.code == lp.EINVAL
