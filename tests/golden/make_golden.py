"""Write the stored oracle results the GPU parity tests compare against.

Calls only the oracle (and the shared input generator).  Run from the repo root:
    python tests/golden/make_golden.py [c1 c2 c1i c2i ...]  # oracle LABPSD (+ dense, mpmath, eigsh)
    python tests/golden/make_golden.py --eigsh c3 c5        # add / write the eigsh route only

Every file records two routes where they are affordable: the oracle's own LABPSD
run (``lam``, tol 1e-11) and ARPACK shift-invert Lanczos (``lam_eigsh``,
oracle.eigs.shift_invert_eigs), plus the dense LAPACK solve (``lam_dense``) for
n <= 3000 and mpmath at 40 digits (``lam_mp``) for n <= 300.  c1i and c2i are the
250- and 16k-dof cells with flat enrichments (cond(S) about 2.5e8 and 2.3e8).  The 296k-dof cell has the eigsh route only: the oracle's LABPSD run
there is many hours long.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pufe  # noqa: E402
from oracle import eigs, labpsd  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(P):
    h = hashlib.sha256()
    for a in (P.rowptr, P.col, P.h_val, P.s_val):
        h.update(np.ascontiguousarray(a).tobytes())
    if P.F is not None:
        for a in (P.F.indptr, P.F.indices, P.F.data, P.G):
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def path_of(name):
    return os.path.join(HERE, "%s_eigs.json" % name)


def hamiltonian(P):
    """The full H of the cell: the local part, plus F G F^T where the cell has projectors."""
    return P.H() if P.F is None else eigs.full_hamiltonian(P.H(), P.F, P.G)


def add_eigsh(P, out, m):
    """ARPACK shift-invert route at sigma = eps_bar (below lambda_1); a few pairs past m
    are computed so the m-th value is not at the edge of the Krylov window."""
    t = time.perf_counter()
    extra = max(8, m // 16)
    lam, _ = eigs.shift_invert_eigs(hamiltonian(P), P.S(), m + extra, P.eps_bar)
    out["lam_eigsh"] = lam[:m].tolist()
    out["lam_eigsh_next"] = lam[m:].tolist()
    out["eigsh_route"] = ("scipy eigsh shift-invert (ARPACK Lanczos on (H - eps_bar S)^-1 S, SuperLU MMD "
                          "ordering), %d pairs, tol 1e-13, %.0f s" % (m + extra, time.perf_counter() - t))


def main(names):
    for name in names:
        P = pufe.workload(name, 0)
        w = pufe.WORKLOADS[name]
        m = w["nev"]
        m0 = pufe.guard_vectors(m)
        prm = labpsd.Params(nev=m, m0=m0, tol=1e-11, sigma0=P.sigma0, eps_bar=P.eps_bar)
        H = hamiltonian(P)
        res = labpsd.solve(H, P.S(), prm, pufe.start_block(P.n, m + m0, 0))
        out = dict(workload=name, seed=0, n=P.n, nnz=P.nnz, nev=m, m0=m0, sha256=digest(P),
                   sigma0=P.sigma0, eps_bar=P.eps_bar, tol=1e-11, converged=bool(res.converged),
                   lam=res.lam.tolist(), res=res.res.tolist(), outer_iters=res.outer_iters,
                   route="oracle.labpsd.solve (tol 1e-11, cold start seed 0)")
        if P.n <= 3000:
            lam, _ = eigs.dense_eigs(H, P.S(), m)
            out["lam_dense"] = lam.tolist()
        if P.n <= 300:
            # mpmath at 40 digits: exact to far below FP64 rounding, whatever cond(S)
            out["lam_mp"] = eigs.mp_eigs(H, P.S(), dps=40)[:m].tolist()
        if P.F is not None:
            out["projectors"] = int(P.F.shape[1])
            out["f_nnz"] = int(P.F.nnz)
        if "alpha" in w:
            out["alpha"] = w["alpha"]
        add_eigsh(P, out, m)
        with open(path_of(name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "converged", res.converged, "iters", res.outer_iters, flush=True)


def main_eigsh(names):
    for name in names:
        P = pufe.workload(name, 0)
        m = pufe.WORKLOADS[name]["nev"]
        if os.path.exists(path_of(name)):
            with open(path_of(name)) as f:
                out = json.load(f)
            assert out["sha256"] == digest(P), "stored file belongs to another pencil"
        else:
            out = dict(workload=name, seed=0, n=P.n, nnz=P.nnz, nev=m, m0=pufe.guard_vectors(m),
                       sha256=digest(P), sigma0=P.sigma0, eps_bar=P.eps_bar)
        add_eigsh(P, out, m)
        with open(path_of(name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, out["eigsh_route"], flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--eigsh":
        main_eigsh(args[1:])
    else:
        main(args or ["c1", "c2"])
