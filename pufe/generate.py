"""Seeded synthetic PUFE-shaped generalized eigenproblems (inputs only).

This module builds the sparse pencil (H, S) that the solver and the oracle both
consume.  It holds none of the eigensolver's arithmetic: it is the
discretisation that produces the input matrices, and the random draws
(atom positions, cold-start blocks) that the solver treats as given data.

Construction (the stand-in for the paper's PUFE Hamiltonian and overlap
matrices, Section 2, eq. (ghep), and the cubic-cell setting of Section 5):

* periodic cube of side ``L`` meshed with ``ne**3`` trilinear hexahedra,
  h = L / ne, one finite-element node per mesh vertex (ne**3 nodes);
* effective potential  V(r) = -4 * sum_atoms sum_images exp(-|r - R|^2 / (2 * 0.5^2));
* partition-of-unity enrichment: every FE node lying within 2 bohr of an atom
  (nearest periodic image) carries one extra basis function, its hat function
  times g(r) = exp(-alpha |r - R*|^2) with R* the atom image nearest that node;
* H_ij = 1/2 int grad(phi_i).grad(phi_j) + int V phi_i phi_j,
  S_ij = int phi_i phi_j, with 3^3 Gauss points per element, or 4^3 Gauss
  points for every integral of an element that has an enriched node.

Degrees of freedom are numbered node-major: each node's standard function
first, then its enriched functions in atom order.  H and S share one sparsity
pattern (as the paper notes for PUFE, Section 4 footnote on eq. (k1)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

ENRICH_RADIUS = 2.0          # bohr: node-within-radius enrichment rule
ENRICH_ALPHA = 1.0           # g(r) = exp(-alpha |r - R|^2)
V_DEPTH = 4.0                # V = -V_DEPTH * exp(-|r - R|^2 / (2 * V_WIDTH^2))
V_WIDTH = 0.5
MIN_SEP = 1.5                # minimum atom separation (minimum image), bohr
V_CUTOFF = 5.5               # potential terms beyond this distance are < 1e-26


@dataclasses.dataclass
class Problem:
    """A sparse symmetric-definite pencil (H, S) with one shared CSR pattern."""
    n: int
    rowptr: np.ndarray       # int64[n+1]
    col: np.ndarray          # int32[nnz], sorted within each row
    h_val: np.ndarray        # float64[nnz]
    s_val: np.ndarray        # float64[nnz]
    v_min: float             # minimum of V over all quadrature points
    sigma0: float            # shift making H - sigma0 S positive definite
    eps_bar: float           # default global preconditioner shift (below lambda_1)
    L: float
    ne: int
    atoms: np.ndarray        # (natoms, 3)
    amplitudes: np.ndarray   # (natoms,) potential depth multipliers (SCF-like drift)
    dof_node: np.ndarray     # int64[n] host node of every dof
    dof_atom: np.ndarray     # int64[n] enrichment atom (-1 for standard dofs)
    seed: int
    k_val: np.ndarray | None = None   # kinetic part 1/2 int grad.grad on the pattern (h_val - k_val is V)
    alpha: float = ENRICH_ALPHA       # enrichment exponent the pencil was built with
    F: object = None                  # nonlocal projectors (n x k CSC) or None
    G: np.ndarray | None = None       # their k x k coupling
    kpoint: np.ndarray | None = None  # reduced k-point of a Bloch-periodic (complex) pencil

    def h_scaled(self, scale: float) -> np.ndarray:
        """H values with every potential amplitude multiplied by ``scale``."""
        return self.k_val + scale * (self.h_val - self.k_val)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def H(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.h_val, self.col, self.rowptr), shape=(self.n, self.n))

    def S(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.s_val, self.col, self.rowptr), shape=(self.n, self.n))


def _gauss01(npts: int):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def _quad3d(npts: int):
    x, w = _gauss01(npts)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), W


# local node a = ax + 2 ay + 4 az at offsets (ax, ay, az) in {0,1}^3
_LOCAL_OFF = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)


def _shape(xi: np.ndarray):
    """Trilinear shape functions and reference gradients at points xi (nq,3)."""
    nq = xi.shape[0]
    N = np.empty((nq, 8))
    dN = np.empty((nq, 8, 3))
    for a in range(8):
        o = _LOCAL_OFF[a]
        f = [np.where(o[d] == 1, xi[:, d], 1.0 - xi[:, d]) for d in range(3)]
        g = [np.where(o[d] == 1, 1.0, -1.0) * np.ones(nq) for d in range(3)]
        N[:, a] = f[0] * f[1] * f[2]
        dN[:, a, 0] = g[0] * f[1] * f[2]
        dN[:, a, 1] = f[0] * g[1] * f[2]
        dN[:, a, 2] = f[0] * f[1] * g[2]
    return N, dN


def place_atoms(natoms: int, L: float, seed: int, min_sep: float = MIN_SEP) -> np.ndarray:
    """Uniform positions in [0,L)^3, rejecting any closer than min_sep (minimum image)."""
    rng = np.random.default_rng(seed)
    atoms = []
    tries = 0
    while len(atoms) < natoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place atoms with the requested separation")
        p = rng.uniform(0.0, L, size=3)
        ok = True
        for q in atoms:
            d = p - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < min_sep:
                ok = False
                break
        if ok:
            atoms.append(p)
    return np.array(atoms, dtype=np.float64).reshape(natoms, 3)


def _potential_at(elem_ijk: np.ndarray, xi: np.ndarray, h: float,
                  ne: int, atoms: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """V at quadrature points xi of the listed elements, all periodic images within cutoff.

    Returns an array (len(elem_ijk), nq).
    """
    nel = elem_ijk.shape[0]
    nq = xi.shape[0]
    V = np.zeros((nel, nq))
    # element id -> row in elem_ijk
    lookup = -np.ones(ne ** 3, dtype=np.int64)
    eid = elem_ijk[:, 0] + ne * (elem_ijk[:, 1] + ne * elem_ijk[:, 2])
    lookup[eid] = np.arange(nel)
    reach = int(math.ceil(V_CUTOFF / h)) + 1
    inv2w2 = 1.0 / (2.0 * V_WIDTH * V_WIDTH)
    for a in range(atoms.shape[0]):
        R = atoms[a]
        base = np.floor(R / h).astype(np.int64)
        rngs = [np.arange(base[d] - reach, base[d] + reach + 1) for d in range(3)]
        I, J, K = np.meshgrid(*rngs, indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        # unwrapped element origin minus atom -> displacement of quadrature points
        org = np.stack([I, J, K], axis=1) * h - R            # (nb,3)
        cen = org + 0.5 * h
        keep = np.linalg.norm(cen, axis=1) <= V_CUTOFF + h
        I, J, K, org = I[keep], J[keep], K[keep], org[keep]
        phys = (I % ne) + ne * ((J % ne) + ne * (K % ne))
        rows = lookup[phys]
        sel = rows >= 0
        if not np.any(sel):
            continue
        rows, org = rows[sel], org[sel]
        d = org[:, None, :] + h * xi[None, :, :]              # (nb,nq,3)
        contrib = -V_DEPTH * amps[a] * np.exp(-inv2w2 * np.einsum("bqd,bqd->bq", d, d))
        np.add.at(V, rows, contrib)
    return V


def generate(L: float, ne: int, natoms: int, seed: int, *, amplitudes=None,
             atoms: np.ndarray | None = None, alpha: float = ENRICH_ALPHA, kpoint=None) -> Problem:
    """Assemble the PUFE-shaped pencil for a periodic cube (see module docstring).

    alpha is the exponent of the enrichment g(r) = exp(-alpha |r - R|^2).  The named
    workloads use 1.0; a smaller alpha makes g flatter over a node's support, so each
    enriched function approaches a multiple of its hat function and S approaches
    singularity (cond(S) grows roughly like 1/alpha^2), the regime of Section 2's
    Table 1 where enrichment drives cond(S) to 1e8 and beyond.

    kpoint (three reduced coordinates k_f, the wave vector 2 pi k_f / L) assembles the
    Bloch-periodic pencil of that k-point (Section 2's k-point sampling): a basis function
    that an element reaches through the periodic boundary with lattice translation T L
    carries the phase exp(2 pi i k_f . T), so element entry (a, b) is multiplied by
    exp(2 pi i k_f . (T_b - T_a)) and H, S become complex Hermitian.  None (or the Gamma
    point, where every phase is one) gives the real pencil of the same construction."""
    kf = None if kpoint is None else np.asarray(kpoint, dtype=np.float64).reshape(3)
    h = L / ne
    nnode = ne ** 3
    if atoms is None:
        atoms = place_atoms(natoms, L, seed) if natoms > 0 else np.zeros((0, 3))
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 3)
    natoms = atoms.shape[0]
    amps = np.ones(natoms) if amplitudes is None else np.asarray(amplitudes, dtype=np.float64)

    # ---- enrichment: (node, atom) pairs with node within ENRICH_RADIUS of the atom
    pairs_node, pairs_atom = [], []
    reachn = int(math.ceil(ENRICH_RADIUS / h)) + 1
    for a in range(natoms):
        R = atoms[a]
        base = np.round(R / h).astype(np.int64)
        rngs = [np.arange(base[d] - reachn, base[d] + reachn + 1) for d in range(3)]
        I, J, K = np.meshgrid(*rngs, indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        nid = (I % ne) + ne * ((J % ne) + ne * (K % ne))
        nid = np.unique(nid)
        ii, jj, kk = nid % ne, (nid // ne) % ne, nid // (ne * ne)
        d = np.stack([ii, jj, kk], axis=1) * h - R
        d -= L * np.round(d / L)
        dist = np.linalg.norm(d, axis=1)
        nid = nid[dist <= ENRICH_RADIUS]
        pairs_node.append(nid)
        pairs_atom.append(np.full(nid.shape[0], a, dtype=np.int64))
    if natoms:
        pn = np.concatenate(pairs_node)
        pa = np.concatenate(pairs_atom)
    else:
        pn = np.zeros(0, dtype=np.int64)
        pa = np.zeros(0, dtype=np.int64)
    order = np.lexsort((pa, pn))
    pn, pa = pn[order], pa[order]
    nenr_node = np.bincount(pn, minlength=nnode)
    # node-major dof numbering
    first_dof = np.zeros(nnode + 1, dtype=np.int64)
    first_dof[1:] = np.cumsum(1 + nenr_node)
    n = int(first_dof[-1])
    # dof of enriched pair = first_dof[node] + 1 + rank within node
    rank = np.arange(pn.shape[0]) - np.searchsorted(pn, pn, side="left")
    pair_dof = first_dof[pn] + 1 + rank
    dof_node = np.repeat(np.arange(nnode), 1 + nenr_node)
    dof_atom = -np.ones(n, dtype=np.int64)
    dof_atom[pair_dof] = pa
    max_enr = int(nenr_node.max()) if nnode else 0

    # ---- elements
    ee = np.arange(ne ** 3)
    E = np.stack([ee % ne, (ee // ne) % ne, ee // (ne * ne)], axis=1)     # element ijk
    enodes = np.empty((ne ** 3, 8), dtype=np.int64)
    for a in range(8):
        o = _LOCAL_OFF[a]
        enodes[:, a] = ((E[:, 0] + o[0]) % ne) + ne * (((E[:, 1] + o[1]) % ne) + ne * ((E[:, 2] + o[2]) % ne))
    enr_elem = nenr_node[enodes].sum(axis=1) > 0
    # Bloch phases of the element-local nodes (k-point cells): T = wraps of E + offset
    if kf is not None:
        wraps = (E[:, None, :] + _LOCAL_OFF[None, :, :]) // ne                 # (nel, 8, 3)
        node_phase = np.exp(2j * np.pi * np.einsum("ead,d->ea", wraps, kf))   # (nel, 8)

    rows_all, cols_all, hv_all, sv_all, kv_all = [], [], [], [], []
    vmin = np.inf

    # ---- standard elements: 3^3 Gauss, 8 trilinear functions
    xi3, w3 = _quad3d(3)
    N3, dN3 = _shape(xi3)
    Kref = 0.5 * np.einsum("q,qad,qbd->ab", w3, dN3, dN3) * h        # 1/2 int grad.grad (h^3 / h^2)
    Mref = np.einsum("q,qa,qb->ab", w3, N3, N3) * h ** 3
    std = np.nonzero(~enr_elem)[0]
    chunk = 65536
    for c0 in range(0, std.shape[0], chunk):
        els = std[c0:c0 + chunk]
        Vq = _potential_at(E[els], xi3, h, ne, atoms, amps)
        if Vq.size:
            vmin = min(vmin, float(Vq.min()))
        Vloc = np.einsum("eq,q,qa,qb->eab", Vq, w3 * h ** 3, N3, N3)
        Hloc = Kref[None] + Vloc
        Sloc = np.broadcast_to(Mref, Hloc.shape)
        dofs = first_dof[enodes[els]]                                   # (e,8)
        rows_all.append(np.repeat(dofs, 8, axis=1).ravel())
        cols_all.append(np.tile(dofs, (1, 8)).ravel())
        Kl = np.broadcast_to(Kref, Hloc.shape)
        if kf is not None:
            ph = node_phase[els]
            pab = np.conj(ph)[:, :, None] * ph[:, None, :]
            Hloc, Sloc, Kl = Hloc * pab, Sloc * pab, Kl * pab
        hv_all.append(Hloc.reshape(-1))
        kv_all.append(np.ascontiguousarray(Kl).reshape(-1))
        sv_all.append(np.ascontiguousarray(Sloc).reshape(-1))

    # ---- enriched elements: 4^3 Gauss, 8 hats plus the enriched functions of their nodes
    xi4, w4 = _quad3d(4)
    N4, dN4 = _shape(xi4)
    enr = np.nonzero(enr_elem)[0]
    F = 8 + 8 * max_enr
    echunk = 4096
    for c0 in range(0, enr.shape[0], echunk):
        els = enr[c0:c0 + echunk]
        ne_c = els.shape[0]
        Vq = _potential_at(E[els], xi4, h, ne, atoms, amps)
        if Vq.size:
            vmin = min(vmin, float(Vq.min()))
        nq = xi4.shape[0]
        phi = np.zeros((ne_c, nq, F))
        grad = np.zeros((ne_c, nq, F, 3))
        dof = np.zeros((ne_c, F), dtype=np.int64)
        valid = np.zeros((ne_c, F), dtype=bool)
        phi[:, :, :8] = N4[None]
        grad[:, :, :8, :] = dN4[None] / h
        nodes = enodes[els]
        dof[:, :8] = first_dof[nodes]
        valid[:, :8] = True
        org = E[els] * h                                                # unwrapped element origin
        rq = org[:, None, :] + h * xi4[None, :, :]                      # (e,nq,3)
        slot = 8
        slot_node = list(range(8))
        for a in range(8):
            nd = nodes[:, a]
            xnode = org + _LOCAL_OFF[a] * h                             # (e,3) local node position
            for r in range(max_enr):
                has = nenr_node[nd] > r
                if not np.any(has):
                    continue
                pdof = first_dof[nd] + 1 + r
                at = np.where(has, dof_atom[np.where(has, pdof, 0)], 0)
                dd = xnode - atoms[at]
                dd -= L * np.round(dd / L)
                Rstar = xnode - dd                                      # nearest image to the node
                u = rq - Rstar[:, None, :]                              # (e,nq,3)
                g = np.exp(-alpha * np.einsum("eqd,eqd->eq", u, u))
                dg = -2.0 * alpha * u * g[..., None]
                m = has[:, None]
                phi[:, :, slot] = np.where(m, N4[None, :, a] * g, 0.0)
                gr = g[..., None] * (dN4[None, :, a, :] / h) + N4[None, :, a, None] * dg
                grad[:, :, slot, :] = np.where(m[..., None], gr, 0.0)
                dof[:, slot] = np.where(has, pdof, 0)
                valid[:, slot] = has
                slot_node.append(a)
                slot += 1
        wq = w4 * h ** 3
        Kloc = 0.5 * np.einsum("q,eqfd,eqgd->efg", wq, grad, grad, optimize=True)
        Hloc = Kloc + np.einsum("q,eq,eqf,eqg->efg", wq, Vq, phi, phi, optimize=True)
        Sloc = np.einsum("q,eqf,eqg->efg", wq, phi, phi, optimize=True)
        if kf is not None:
            ph = node_phase[els][:, slot_node]                          # (e, used slots)
            ns = ph.shape[1]
            pab = np.ones((ne_c, F, F), dtype=np.complex128)
            pab[:, :ns, :ns] = np.conj(ph)[:, :, None] * ph[:, None, :]
            Hloc, Sloc, Kloc = Hloc * pab, Sloc * pab, Kloc * pab
        vv = valid[:, :, None] & valid[:, None, :]
        R_ = np.repeat(dof[:, :, None], F, axis=2)
        C_ = np.repeat(dof[:, None, :], F, axis=1)
        rows_all.append(R_[vv])
        cols_all.append(C_[vv])
        hv_all.append(Hloc[vv])
        kv_all.append(Kloc[vv])
        sv_all.append(Sloc[vv])

    rows = np.concatenate(rows_all)
    cols = np.concatenate(cols_all)
    Hc = sp.coo_matrix((np.concatenate(hv_all), (rows, cols)), shape=(n, n)).tocsr()
    Sc = sp.coo_matrix((np.concatenate(sv_all), (rows, cols)), shape=(n, n)).tocsr()
    Kc = sp.coo_matrix((np.concatenate(kv_all), (rows, cols)), shape=(n, n)).tocsr()
    # exact (Hermitian) symmetry: duplicate summation order may differ between (i,j) and (j,i)
    if kf is None:
        Kc = ((Kc + Kc.T) * 0.5).tocsr()
        Hc = ((Hc + Hc.T) * 0.5).tocsr()
        Sc = ((Sc + Sc.T) * 0.5).tocsr()
    else:
        Kc = ((Kc + Kc.conj().T) * 0.5).tocsr()
        Hc = ((Hc + Hc.conj().T) * 0.5).tocsr()
        Sc = ((Sc + Sc.conj().T) * 0.5).tocsr()
    # one shared pattern: union of both patterns, explicit zeros kept
    pat = (abs(Hc) + abs(Sc)).tocsr()
    pat.sort_indices()
    Hc = _on_pattern(Hc, pat)
    Sc = _on_pattern(Sc, pat)
    Kc = _on_pattern(Kc, pat)
    if not np.isfinite(vmin):
        vmin = 0.0
    return Problem(n=n, rowptr=pat.indptr.astype(np.int64), col=pat.indices.astype(np.int32),
                   h_val=Hc, s_val=Sc, v_min=vmin, sigma0=vmin - 1.0, eps_bar=vmin - 0.1,
                   L=float(L), ne=int(ne), atoms=atoms, amplitudes=amps, dof_node=dof_node,
                   dof_atom=dof_atom, seed=int(seed), k_val=Kc, alpha=float(alpha), kpoint=kf)


# ------------------------------------------------------------------ nonlocal projectors

PROJ_RC = 0.35               # bohr: projector width, beta(r) ~ exp(-|r - R|^2 / (2 rc^2))
PROJ_CUT = 1e-6              # projectors are cut where beta_s falls below this (r = 5.26 rc)
PROJ_ENERGY = (4.0, 2.0)     # hartree: G entries of the s and p projectors


def nonlocal_projectors(P: Problem, per_atom: int = 4, rc: float = PROJ_RC,
                        energies=PROJ_ENERGY):
    """The low-rank nonlocal term H_nl = F G F^T of a separable (Kleinman-Bylander-like)
    pseudopotential for the cell of P (Section 4, eq. (fgf)): per atom an s projector
    beta_s = exp(-d^2 / (2 rc^2)) and, with per_atom = 4, three p projectors
    beta_x = (d_x / rc) beta_s, ...  (d = r minus the nearest image of the atom), cut off
    where beta_s < PROJ_CUT (a core radius of 5.26 rc) or at half the cell.  F[i, c] = integral of phi_i beta_c over the
    cell by 4^3 Gauss points per element, phi_i the basis function of dof i (hat, or hat
    times the enrichment g); G = diag(energies[s], energies[p] x 3) per atom.
    Returns (F as an n x k CSC matrix, G as a k x k dense array), k = per_atom * atoms."""
    assert per_atom in (1, 4)
    ne, L = P.ne, P.L
    h = L / ne
    natoms = P.atoms.shape[0]
    n = P.n
    # dof numbering: first dof of every node, then its enriched dofs in atom order
    first_dof = np.zeros(ne ** 3 + 1, dtype=np.int64)
    np.add.at(first_dof, P.dof_node + 1, 1)
    first_dof = np.cumsum(first_dof)
    cut = min(rc * math.sqrt(2.0 * math.log(1.0 / PROJ_CUT)), 0.5 * L)
    xi, w = _quad3d(4)
    N, _ = _shape(xi)
    rows_all, cols_all, vals_all = [], [], []
    reach = int(math.ceil(cut / h)) + 1
    for a in range(natoms):
        R = P.atoms[a]
        base = np.floor(R / h).astype(np.int64)
        rng_ = np.arange(-reach, reach + 1)
        I, J, K = np.meshgrid(base[0] + rng_, base[1] + rng_, base[2] + rng_, indexing="ij")
        org = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) * h      # unwrapped element origins
        # keep elements with a point within the cut-off
        cen = org + 0.5 * h
        keep = np.linalg.norm(cen - R, axis=1) <= cut + 0.5 * math.sqrt(3.0) * h
        org = org[keep]
        eijk = np.round(org / h).astype(np.int64) % ne
        xq = org[:, None, :] + h * xi[None, :, :]                           # (e, nq, 3)
        d = xq - R
        d -= L * np.round(d / L)
        r2 = np.einsum("eqd,eqd->eq", d, d)
        bs = np.exp(-r2 / (2.0 * rc * rc)) * (r2 <= cut * cut)
        betas = [bs] if per_atom == 1 else [bs, d[..., 0] / rc * bs, d[..., 1] / rc * bs, d[..., 2] / rc * bs]
        wq = w * h ** 3
        for loc in range(8):
            o = _LOCAL_OFF[loc]
            nd = ((eijk[:, 0] + o[0]) % ne) + ne * (((eijk[:, 1] + o[1]) % ne) + ne * ((eijk[:, 2] + o[2]) % ne))
            xnode = org + o * h
            # the hat function of the node, then its enriched functions
            funcs = [(first_dof[nd], N[None, :, loc] * np.ones((org.shape[0], 1)))]
            nen = first_dof[nd + 1] - first_dof[nd] - 1
            for rr in range(int(nen.max()) if nen.size else 0):
                has = nen > rr
                pdof = np.where(has, first_dof[nd] + 1 + rr, 0)
                at = np.where(has, P.dof_atom[pdof], 0)
                dd = xnode - P.atoms[at]
                dd -= L * np.round(dd / L)
                u = xq - (xnode - dd)[:, None, :]
                g = np.exp(-P.alpha * np.einsum("eqd,eqd->eq", u, u))
                funcs.append((np.where(has, pdof, -1), N[None, :, loc] * g * has[:, None]))
            for dof, phi in funcs:
                for l, be in enumerate(betas):
                    v = np.einsum("q,eq,eq->e", wq, phi, be)
                    ok = (dof >= 0) & (v != 0.0)
                    rows_all.append(dof[ok])
                    cols_all.append(np.full(int(ok.sum()), a * per_atom + l, dtype=np.int64))
                    vals_all.append(v[ok])
    k = natoms * per_atom
    F = sp.coo_matrix((np.concatenate(vals_all) if vals_all else np.zeros(0),
                       (np.concatenate(rows_all) if rows_all else np.zeros(0, dtype=np.int64),
                        np.concatenate(cols_all) if cols_all else np.zeros(0, dtype=np.int64))),
                      shape=(n, k)).tocsc()
    F.sum_duplicates()
    F.sort_indices()
    g = [energies[0]] + ([energies[1]] * 3 if per_atom == 4 else [])
    G = np.diag(np.tile(np.asarray(g, dtype=np.float64), natoms))
    return F, G


def _on_pattern(A: sp.csr_matrix, pat: sp.csr_matrix) -> np.ndarray:
    """Values of A laid out on the CSR pattern ``pat`` (zeros where A has none)."""
    A = A.tocsr()
    A.sort_indices()
    out = np.zeros(pat.indices.shape[0], dtype=A.dtype)
    # both sorted per row: merge by row-wise search
    n = pat.shape[0]
    prow = np.repeat(np.arange(n), np.diff(pat.indptr))
    arow = np.repeat(np.arange(n), np.diff(A.indptr))
    pkey = prow.astype(np.int64) * n + pat.indices
    akey = arow.astype(np.int64) * n + A.indices
    pos = np.searchsorted(pkey, akey)
    out[pos] = A.data
    return out


def dof_coordinates(P: Problem) -> np.ndarray:
    """Position (x, y, z) of every dof's host node, row-major n x 3 (for orderings)."""
    ne = P.ne
    h = P.L / ne
    nd = P.dof_node
    return np.ascontiguousarray(np.stack([nd % ne, (nd // ne) % ne, nd // (ne * ne)], axis=1) * h,
                                dtype=np.float64)


def count_dofs(L: float, ne: int, natoms: int, seed: int) -> int:
    """Number of dofs the construction gives, without assembling (nodes + enriched pairs)."""
    h = L / ne
    atoms = place_atoms(natoms, L, seed) if natoms > 0 else np.zeros((0, 3))
    g = np.arange(ne) * h
    total = ne ** 3
    for a in range(atoms.shape[0]):
        d = [g - atoms[a, k] for k in range(3)]
        d = [x - L * np.round(x / L) for x in d]
        r2 = d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2
        total += int(np.count_nonzero(r2 <= ENRICH_RADIUS ** 2))
    return total


# ------------------------------------------------------------------ named workloads

#: The five workload shapes: (L, ne, natoms, nev).  Serving draws its own.
WORKLOADS = {
    "c1": dict(L=6.0, ne=6, natoms=1, nev=4),
    "c2": dict(L=12.0, ne=24, natoms=8, nev=32),
    "c3": dict(L=24.0, ne=48, natoms=64, nev=256),
    "c5": dict(L=32.0, ne=64, natoms=128, nev=512),
    # the 250- and 16k-dof cells with flat enrichments: cond(S) above 1e8
    "c1i": dict(L=6.0, ne=6, natoms=1, nev=4, alpha=1e-3),
    "c2i": dict(L=12.0, ne=24, natoms=8, nev=32, alpha=1e-2),
    # the 250- and 16k-dof cells with a nonlocal term H_nl = F G F^T of four projectors per atom
    "c1nl": dict(L=6.0, ne=6, natoms=1, nev=4, projectors=4),
    "c2nl": dict(L=12.0, ne=24, natoms=8, nev=32, projectors=4),
    # the paper's second k-point, k_f = (0.12, -0.24, 0.37): complex Hermitian pencils
    "c1k": dict(L=6.0, ne=6, natoms=1, nev=4, kpoint=(0.12, -0.24, 0.37)),
    "c2k": dict(L=12.0, ne=24, natoms=8, nev=32, kpoint=(0.12, -0.24, 0.37)),
}


def guard_vectors(nev: int) -> int:
    """Number of extra guard vectors m0 carried beside the nev wanted ones."""
    return max(int(math.ceil(nev / 10.0)), 4)


def workload(name: str, seed: int = 0, **kw) -> Problem:
    """The named cell's pencil; for cells with a nonlocal term its projectors are attached as
    P.F (n x k CSC) and P.G (k x k), and P.h_val stays the local part."""
    w = WORKLOADS[name]
    if "alpha" in w:
        kw.setdefault("alpha", w["alpha"])
    if "kpoint" in w:
        kw.setdefault("kpoint", w["kpoint"])
    P = generate(w["L"], w["ne"], w["natoms"], seed, **kw)
    if w.get("projectors"):
        P.F, P.G = nonlocal_projectors(P, w["projectors"])
    return P


def start_block(n: int, b: int, seed: int) -> np.ndarray:
    """Cold-start block: i.i.d. standard normal n x b, column-major (Fortran) order."""
    rng = np.random.default_rng(seed + 1000)
    return np.asfortranarray(rng.standard_normal((n, b)))


def free_particle_eigs(ne: int, L: float, count: int, kpoint=None) -> np.ndarray:
    """Exact spectrum of the assembled trilinear pencil with V = 0 and no enrichment.

    Separable: per dimension the 1-D linear-element pencil on a periodic ring has
    K_1 = (2 - 2cos t)/h and M_1 = h (4 + 2cos t)/6 at wavenumber t = 2 pi j / ne
    (t = 2 pi (j + k_d) / ne for the Bloch-periodic pencil of reduced k-point k);
    the 3-D stiffness is sum_d K_d prod_{e!=d} M_e and the mass prod_d M_d,
    so lambda = 1/2 sum_d K_d / M_d.
    """
    h = L / ne
    kf = np.zeros(3) if kpoint is None else np.asarray(kpoint, dtype=np.float64)
    rs = []
    for d in range(3):
        t = 2.0 * np.pi * (np.arange(ne) + kf[d]) / ne
        k1 = (2.0 - 2.0 * np.cos(t)) / h
        m1 = h * (4.0 + 2.0 * np.cos(t)) / 6.0
        rs.append(k1 / m1)
    lam = 0.5 * (rs[0][:, None, None] + rs[1][None, :, None] + rs[2][None, None, :])
    return np.sort(lam.ravel())[:count]
