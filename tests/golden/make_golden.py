"""Write the stored oracle results the GPU parity tests compare against.

Calls only the oracle (and the shared input generator).  Run from the repo root:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

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
    return h.hexdigest()


def main(names):
    for name in names:
        P = pufe.workload(name, 0)
        w = pufe.WORKLOADS[name]
        m = w["nev"]
        m0 = pufe.guard_vectors(m)
        prm = labpsd.Params(nev=m, m0=m0, tol=1e-11, sigma0=P.sigma0, eps_bar=P.eps_bar)
        res = labpsd.solve(P.H(), P.S(), prm, pufe.start_block(P.n, m + m0, 0))
        out = dict(workload=name, seed=0, n=P.n, nnz=P.nnz, nev=m, m0=m0, sha256=digest(P),
                   sigma0=P.sigma0, eps_bar=P.eps_bar, tol=1e-11, converged=bool(res.converged),
                   lam=res.lam.tolist(), res=res.res.tolist(), outer_iters=res.outer_iters,
                   route="oracle.labpsd.solve (tol 1e-11, cold start seed 0)")
        if P.n <= 3000:
            lam, _ = eigs.dense_eigs(P.H(), P.S(), m)
            out["lam_dense"] = lam.tolist()
        with open(os.path.join(HERE, "%s_eigs.json" % name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "converged", res.converged, "iters", res.outer_iters)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
