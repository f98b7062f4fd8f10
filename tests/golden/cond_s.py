"""cond(S) of the workloads' overlap matrices, reported beside the measurements.

The extreme eigenvalues of S come from Lanczos (SciPy's eigsh: the largest, then the
smallest algebraic one with a wide Krylov space; on the 16k-dof cell this matches
shift-invert about zero to five digits).  Input only: no part of the solver is used.
Run from the repo root:
    python tests/golden/cond_s.py c1 c2 c3 c5
"""
import json
import os
import sys
import time

import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pufe  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "cond_s.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        P = pufe.workload(name, 0)
        S = P.S().tocsr()
        t = time.perf_counter()
        lmax = float(spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0])
        if name.endswith("i"):
            # the ill-conditioned cells: plain Lanczos cannot resolve lambda_min; shift-invert
            # about zero (SuperLU of S) does
            lmin = float(spla.eigsh(S.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False,
                                    tol=1e-10)[0])
        else:
            lmin = float(spla.eigsh(S, k=1, which="SA", return_eigenvectors=False, tol=1e-4, ncv=200,
                                    maxiter=50000)[0])
        data[name] = dict(n=P.n, lambda_max=lmax, lambda_min=lmin, cond=lmax / lmin,
                          seconds=time.perf_counter() - t)
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
