"""Pins of the synthetic PUFE-shaped input generator (CPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import pufe


def test_symmetric_and_shared_pattern():
    P = pufe.workload("c1", 0)
    H, S = P.H(), P.S()
    assert abs(H - H.T).max() == 0.0
    assert abs(S - S.T).max() == 0.0
    # one pattern: sorted, unique columns per row, structurally symmetric
    for i in range(P.n):
        c = P.col[P.rowptr[i]:P.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    pat = (abs(H) + abs(S) + (H != 0) + (S != 0)).tocsr()
    assert (pat != pat.T).nnz == 0


def test_free_particle_closed_form():
    # no atoms: the pencil is the periodic trilinear Laplacian, separable in closed form
    for ne, L in [(6, 6.0), (8, 4.0), (5, 7.5)]:
        P = pufe.generate(L, ne, 0, 0)
        w = sla.eigh(P.H().toarray(), P.S().toarray(), eigvals_only=True)
        ref = pufe.free_particle_eigs(ne, L, P.n)
        assert np.max(np.abs(w - ref)) < 1e-11 * max(1.0, ref.max())


def test_partition_of_unity_integrals():
    P = pufe.workload("c1", 0)
    std = np.nonzero(P.dof_atom < 0)[0]
    S = P.S().tocsr()
    # the hat functions sum to one, so the standard block of S integrates 1 over the cell
    assert abs(S[std][:, std].sum() - P.L ** 3) < 1e-10 * P.L ** 3
    # with the potential switched off the gradient of the partition of unity is zero:
    # H applied to the standard-dof indicator vanishes on every row (enriched rows too)
    P0 = pufe.generate(P.L, P.ne, 0, 0, atoms=P.atoms, amplitudes=np.zeros(1))
    one = np.zeros(P0.n)
    one[P0.dof_atom < 0] = 1.0
    assert np.abs(P0.H() @ one).max() < 1e-12


def test_definite_and_shift_below_spectrum():
    P = pufe.workload("c1", 0)
    H, S = P.H().toarray(), P.S().toarray()
    sla.cholesky(S)                                   # S positive definite
    lam = sla.eigh(H, S, eigvals_only=True)
    assert lam[0] > P.v_min                           # positive Gauss weights: lambda > min V
    sla.cholesky(H - P.eps_bar * S)                   # global shift gives an SPD matrix
    sla.cholesky(H - P.sigma0 * S)


def test_dof_counts_match_workloads():
    assert pufe.count_dofs(6.0, 6, 1, 0) < 300
    n2 = pufe.count_dofs(12.0, 24, 8, 0)
    assert 14000 < n2 < 17000
    n3 = pufe.count_dofs(24.0, 48, 64, 0)
    assert 115000 < n3 < 135000
    n5 = pufe.count_dofs(32.0, 64, 128, 0)
    assert 280000 < n5 < 310000
    assert pufe.workload("c1", 0).n == pufe.count_dofs(6.0, 6, 1, 0)


def test_seeded_reproducible():
    a = pufe.generate(6.0, 6, 2, 5)
    b = pufe.generate(6.0, 6, 2, 5)
    assert np.array_equal(a.h_val, b.h_val) and np.array_equal(a.col, b.col)
    assert np.array_equal(pufe.start_block(50, 4, 3), pufe.start_block(50, 4, 3))
    c = pufe.generate(6.0, 6, 2, 6)
    assert not np.array_equal(a.atoms, c.atoms)


def test_atoms_respect_separation():
    at = pufe.place_atoms(64, 24.0, 0)
    d = at[:, None, :] - at[None, :, :]
    d -= 24.0 * np.round(d / 24.0)
    r = np.linalg.norm(d, axis=2) + np.eye(64) * 10
    assert r.min() >= 1.5


@pytest.mark.parametrize("seed", [0, 1])
def test_enrichment_makes_s_ill_conditioned(seed):
    P = pufe.workload("c1", seed)
    P0 = pufe.generate(6.0, 6, 0, 0)
    c = np.linalg.cond(P.S().toarray())
    c0 = np.linalg.cond(P0.S().toarray())
    assert c > 100 * c0          # enrichment raises cond(S) sharply (Table 1 trend)
