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


# ------------------------------------------------------------------ nonlocal projectors

def test_projector_partition_of_unity_and_symmetry():
    """The standard hats sum to one at every point (partition of unity), so summing an
    s projector's column over the standard dofs gives the quadrature of beta_s itself,
    which at h = 0.5 matches the closed form of the Gaussian cut at radius Rc,
    (2 pi rc^2)^(3/2) [erf(x / sqrt 2) - sqrt(2 / pi) x exp(-x^2 / 2)] with x = Rc / rc
    (the chi distribution's CDF), to 1e-6 (the cut runs through elements); the p
    projectors are odd about the atom, so their sums vanish.  G is diagonal and positive
    (s, p x 3 per atom), and F >= 0 in every s column."""
    import math
    from pufe.generate import PROJ_RC, PROJ_CUT, PROJ_ENERGY
    P = pufe.workload("c2nl", 0)
    F, G = P.F, P.G
    assert F.shape == (P.n, 4 * len(P.atoms))
    std = P.dof_atom < 0
    sums = np.asarray(F[std].sum(axis=0)).ravel()
    x = math.sqrt(2.0 * math.log(1.0 / PROJ_CUT))
    closed = (2 * math.pi * PROJ_RC ** 2) ** 1.5 * (math.erf(x / math.sqrt(2.0))
                                                   - math.sqrt(2.0 / math.pi) * x * math.exp(-x * x / 2))
    assert np.abs(sums[0::4] - closed).max() < 1e-6 * closed
    for l in (1, 2, 3):
        assert np.abs(sums[l::4]).max() < 1e-6 * closed
    assert np.allclose(np.diag(G)[0::4], PROJ_ENERGY[0]) and np.allclose(np.diag(G)[1::4], PROJ_ENERGY[1])
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0
    Fs = F[:, 0::4]
    assert Fs.data.min() >= 0.0


def test_nonlocal_term_raises_the_spectrum():
    """G is positive semidefinite, so H_loc + F G F^T >= H_loc and every eigenvalue rises
    (Weyl); eps_bar stays below lambda_1 of both pencils."""
    import scipy.linalg as sla
    from oracle import eigs
    P = pufe.workload("c1nl", 0)
    H = eigs.full_hamiltonian(P.H(), P.F, P.G)
    assert abs(H - H.T).max() == 0.0
    l0 = sla.eigh(P.H().toarray(), P.S().toarray(), eigvals_only=True)
    l1 = sla.eigh(H.toarray(), P.S().toarray(), eigvals_only=True)
    assert np.all(l1 >= l0 - 1e-12 * np.abs(l0).max())
    assert P.eps_bar < l0[0] <= l1[0]


# ------------------------------------------------------------------ k-points (Bloch-periodic pencils)

KF = (0.12, -0.24, 0.37)


def test_kpoint_pencil_is_hermitian_and_reduces_to_gamma():
    """At a k-point H and S are complex Hermitian with S positive definite; at k = 0 (and at
    any integer k, a reciprocal lattice vector) the phases are one and the pencil is the
    real one; k and -k give complex-conjugate pencils (time reversal)."""
    G = pufe.generate(6.0, 6, 1, 0)
    P = pufe.generate(6.0, 6, 1, 0, kpoint=KF)
    assert np.iscomplexobj(P.h_val) and np.abs(P.h_val.imag).max() > 1e-3
    H, S = P.H().toarray(), P.S().toarray()
    assert np.abs(H - H.conj().T).max() == 0.0 and np.abs(S - S.conj().T).max() == 0.0
    assert np.linalg.eigvalsh(S).min() > 0
    for k in ((0.0, 0.0, 0.0), (1.0, -1.0, 2.0)):
        Q = pufe.generate(6.0, 6, 1, 0, kpoint=k)
        assert np.array_equal(Q.col, G.col)
        assert np.abs(Q.h_val - G.h_val).max() < 1e-14 and np.abs(Q.s_val - G.s_val).max() < 1e-14
    M = pufe.generate(6.0, 6, 1, 0, kpoint=tuple(-x for x in KF))
    assert np.abs(M.h_val - np.conj(P.h_val)).max() < 1e-15


def test_kpoint_free_particle_closed_form():
    """V = 0, no enrichment, Bloch-periodic at k: the spectrum is separable with wave
    numbers 2 pi (j + k_d) / ne per dimension; dense LAPACK and the oracle's LABPSD (complex
    Hermitian arithmetic) reproduce it, which pins the phase convention of the assembly."""
    from oracle import eigs, labpsd
    P = pufe.generate(4.0, 8, 0, 0, kpoint=KF)
    ref = pufe.free_particle_eigs(8, 4.0, 7, kpoint=KF)
    lam, _ = eigs.dense_eigs(P.H(), P.S(), 7)
    assert np.abs(lam - ref).max() < 1e-12
    prm = labpsd.Params(nev=7, m0=4, tol=1e-11, sigma0=-1.0, eps_bar=-0.1)
    res = labpsd.solve(P.H(), P.S(), prm, pufe.start_block(P.n, 11, 0) + 1j * pufe.start_block(P.n, 11, 1))
    assert res.converged
    assert np.max(np.abs(res.lam - ref) / np.abs(ref + 1.0)) < 1e-11
    S = P.S()
    assert np.abs(res.X.conj().T @ (S @ res.X) - np.eye(7)).max() < 1e-10
