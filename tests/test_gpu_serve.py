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


def test_server_memory_within_budget(pencils):
    """Seven systems, three slots, two SCF-like steps each, a budget of 1.5 of the largest
    request's footprint.  The server's ledger (slot workspaces kept between requests and
    the systems' resident blocks) never exceeds the budget, and the device memory the
    stream took (hipMemGetInfo before the server and after the stream) stays within the
    budget up to allocation rounding."""
    import torch
    lp = _lp()
    ctx = lp.Context(0)
    fps = [lp.solve_footprint(P.n, nev, pufe.guard_vectors(nev), lp.MIXED) for P, nev in pencils]
    budget = int(max(fps) * 1.5)
    systems = _systems(ctx, pencils)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = lp.Server(ctx, budget, 3)
    first, second = [], []
    for (P, nev), pr in zip(pencils, systems):
        m0 = pufe.guard_vectors(nev)
        first.append(srv.submit(pr, nev, m0, X0=pufe.start_block(P.n, nev + m0, 7), tol=1e-9,
                                sigma0=P.sigma0, precision=lp.MIXED))
    for (P, nev), pr in zip(pencils, systems):
        m0 = pufe.guard_vectors(nev)
        second.append(srv.submit(pr, nev, m0, h_val=P.h_scaled(1.01), tol=1e-9, sigma0=P.sigma0,
                                 precision=lp.MIXED))
    rs = [srv.wait(r) for r in first + second]
    mem = srv.memory()
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    # device allocations round up to 2 MiB pages: the slots' three arenas, the resident
    # blocks and the factors' sweep counters
    slack = 2 * 1024 * 1024 * (3 * 3 + 2 * len(systems))
    print("[serve] budget %.1f MB, ledger held %.1f MB peak %.1f MB, device memory taken %.1f MB"
          % (budget / 1e6, mem["held"] / 1e6, mem["peak"] / 1e6, used / 1e6), flush=True)
    assert all(r.converged for r in rs)
    assert mem["peak"] <= budget
    assert used <= budget + slack
    # the resident blocks are all charged and stay charged
    assert mem["held"] >= sum(P.n * (nev + pufe.guard_vectors(nev)) * 8 for P, nev in pencils)
    srv.close()
    for pr in systems:
        pr.close()
    ctx.close()


def test_resident_blocks_can_crowd_out_a_request(pencils):
    """One slot, a budget just above the largest request's own footprint: after the five
    small systems have left their resident blocks, the large request no longer fits even
    with the slot's workspace given back, and it finishes with ENOMEM instead of waiting
    forever; the small ones converge."""
    lp = _lp()
    ctx = lp.Context(0)
    small, big = pencils[:5], pencils[5]
    fp_big = lp.solve_footprint(big[0].n, big[1], pufe.guard_vectors(big[1]), lp.MIXED)
    systems = _systems(ctx, small + [big])
    srv = lp.Server(ctx, fp_big + 4096, 1)
    rids = []
    for (P, nev), pr in zip(small + [big], systems):
        m0 = pufe.guard_vectors(nev)
        rids.append(srv.submit(pr, nev, m0, X0=pufe.start_block(P.n, nev + m0, 3), tol=1e-9, sigma0=P.sigma0,
                               precision=lp.MIXED))
    for rid in rids[:-1]:
        assert srv.wait(rid).converged
    with pytest.raises(lp.LabpsdError) as e:
        srv.wait(rids[-1])
    assert e.value.code == lp.ENOMEM
    assert srv.memory()["peak"] <= fp_big + 4096
    srv.close()
    for pr in systems:
        pr.close()
    ctx.close()


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
