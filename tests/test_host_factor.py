"""CPU tests of the host side of the global preconditioner (the nested-dissection ordering
and the multifrontal supernodal Cholesky of H - eps_bar S, eq. (ldl)), through a small C++
driver (tests/factor_harness.cpp) built with g++ against the library's factor.cpp, once
plainly and once under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import pufe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_2445_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "factor_harness.cpp")


def _build(tmpdir, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = os.path.join(str(tmpdir), "factor_harness" + ("_san" if sanitize else ""))
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    subprocess.run([gxx, "-std=c++17", *flags, "-I", CSRC, HARNESS, os.path.join(CSRC, "factor.cpp"),
                    "-o", exe, "-lpthread"], check=True)
    return exe


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("fh"), False)


@pytest.fixture(scope="module")
def harness_san(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("fhs"), True)


def _run(exe, tmpdir, K, coords, b, single=False):
    K = sp.csr_matrix(K)
    K.sort_indices()
    n = K.shape[0]
    inp = os.path.join(str(tmpdir), "in.bin")
    out = os.path.join(str(tmpdir), "out.bin")
    with open(inp, "wb") as f:
        np.array([n, K.nnz, coords is not None, int(single)], dtype=np.int64).tofile(f)
        K.indptr.astype(np.int64).tofile(f)
        K.indices.astype(np.int32).tofile(f)
        K.data.astype(np.float64).tofile(f)
        if coords is not None:
            np.ascontiguousarray(coords, dtype=np.float64).tofile(f)
        np.asarray(b, dtype=np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", LABPSD_HOST_THREADS="4")
    subprocess.run([exe, inp, out], check=True, env=env)
    raw = np.fromfile(out, dtype=np.int64, count=5)
    x = np.fromfile(out, dtype=np.float64, offset=40)
    return dict(status=int(raw[0]), nsn=int(raw[1]), perm_ok=bool(raw[2]), sym_ok=bool(raw[3]),
                lev_ok=bool(raw[4])), x


def _shifted(P, eps):
    return (P.H() - eps * P.S()).tocsr()


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("use_coords", [True, False])
def test_factor_solves_and_structure(harness, tmp_path, name, use_coords):
    """The ordering is a permutation, the factor's symbolic pattern contains K's, the tree
    is ordered, and the factor solves K x = b to 1e-11 against SciPy's sparse solve (with
    coordinate bisection and with the graph's level-structure bisection)."""
    P = pufe.workload(name, 0)
    K = _shifted(P, P.eps_bar)
    b = np.random.default_rng(41).standard_normal(P.n)
    info, x = _run(harness, tmp_path, K, pufe.dof_coordinates(P) if use_coords else None, b)
    assert info["status"] == 0 and info["perm_ok"] and info["sym_ok"] and info["lev_ok"]
    assert info["nsn"] > (1 if P.n > 1000 else 0)
    ref = spla.spsolve(K.tocsc(), b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    assert np.linalg.norm(K @ x - b) <= 1e-11 * np.linalg.norm(b)


def test_factor_matches_dense_cholesky(harness, tmp_path):
    """The factor applied to the identity gives K^{-1}, which equals the inverse from
    numpy's dense Cholesky factor (L L^T = K) column by column."""
    P = pufe.workload("c1", 0)
    K = _shifted(P, P.eps_bar)
    L = np.linalg.cholesky(K.toarray())
    Kinv = np.linalg.inv(L).T @ np.linalg.inv(L)
    for j in (0, 17, P.n - 1):
        e = np.zeros(P.n)
        e[j] = 1.0
        _, x = _run(harness, tmp_path, K, pufe.dof_coordinates(P), e)
        assert np.abs(x - Kinv[:, j]).max() <= 1e-10 * np.abs(Kinv).max()


def test_single_precision_factorisation(harness, tmp_path):
    """The FP32 numeric factorisation solves to single-precision accuracy only (and is still a
    usable preconditioner: K x close to b)."""
    P = pufe.workload("c2", 0)
    K = _shifted(P, P.eps_bar)
    b = np.random.default_rng(42).standard_normal(P.n)
    info, x = _run(harness, tmp_path, K, pufe.dof_coordinates(P), b, single=True)
    assert info["status"] == 0
    rel = np.linalg.norm(K @ x - b) / np.linalg.norm(b)
    assert 1e-9 < rel < 1e-3


def test_shift_above_the_spectrum_is_not_positive_definite(harness, tmp_path):
    import scipy.linalg as sla
    P = pufe.workload("c1", 0)
    lam = sla.eigh(P.H().toarray(), P.S().toarray(), eigvals_only=True)
    K = _shifted(P, 0.5 * (lam[1] + lam[2]))
    info, _ = _run(harness, tmp_path, K, pufe.dof_coordinates(P), np.ones(P.n))
    assert info["status"] == -4


@pytest.mark.parametrize("name", ["c1", "c2i"])
def test_factor_under_address_and_ub_sanitizers(harness_san, tmp_path, name):
    """The same driver built with -fsanitize=address,undefined: no invalid access, leak or
    undefined behaviour in the ordering, the factorisation (threaded) and the solve."""
    P = pufe.workload(name, 0)
    K = _shifted(P, P.eps_bar)
    b = np.random.default_rng(43).standard_normal(P.n)
    for coords in (pufe.dof_coordinates(P), None):
        info, x = _run(harness_san, tmp_path, K, coords, b)
        assert info["status"] == 0 and info["perm_ok"] and info["sym_ok"]
        # normwise backward error (the 16k-dof flat-enrichment K is itself ill-conditioned)
        knorm = spla.norm(K, 1)
        assert np.linalg.norm(K @ x - b, 1) <= 1e-13 * (knorm * np.linalg.norm(x, 1) + np.linalg.norm(b, 1))


def test_hermitian_host_pieces(tmp_path):
    """The host pieces of the k-point variant (hermitian.cpp), built with g++ under
    AddressSanitizer and UBSan: cyclic Jacobi on seeded random Hermitian matrices (and one
    with a fivefold eigenvalue) gives A V = V diag and unitary V to 1e-13; the real
    embedding is symmetric and maps A x to R(A) R(x)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "hermitian_harness")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-I", CSRC, os.path.join(ROOT, "tests", "hermitian_harness.cpp"),
                    os.path.join(CSRC, "hermitian.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    jac = [l.split() for l in out if l.startswith("jacobi")]
    assert len(jac) == 5
    for _, n, res, orth in jac:
        assert float(res) < 1e-13 and float(orth) < 1e-13, (n, res, orth)
    emb = [l.split() for l in out if l.startswith("embed")][0]
    assert emb[1] == "1" and float(emb[2]) < 1e-14
