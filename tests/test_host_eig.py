"""The library's host eigensolvers (dense symmetric QR, tridiagonal QR and
inverse iteration), built with g++ from the library sources and checked
against numpy on random and clustered matrices."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_05215_amd", "csrc")


@pytest.fixture(scope="module")
def lib():
    out = os.path.join(tempfile.mkdtemp(), "libhosteig.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                    os.path.join(CSRC, "host_eig.cpp"),
                    os.path.join(ROOT, "tests", "native", "host_eig_shim.cpp"), "-o", out],
                   check=True)
    L = C.CDLL(out)
    dp = C.POINTER(C.c_double)
    L.t_sym_eig.argtypes = [C.c_int, dp, dp, dp]
    L.t_tridiag_eig.argtypes = [C.c_int, dp, dp, dp, dp]
    L.t_tridiag_eigvecs.argtypes = [C.c_int, dp, dp, C.c_int, dp, dp]
    L.t_tridiag_eigvecs.restype = None
    L.t_arrow_eig_sel.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, C.c_double, dp]
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tridiag(rng, m, clusters=False):
    if clusters:
        # block-diagonal copies of one tridiagonal: every eigenvalue repeated
        k = m // 2
        d0 = rng.standard_normal(k)
        e0 = rng.standard_normal(k - 1)
        d = np.concatenate([d0, d0])
        e = np.concatenate([e0, [0.0], e0])
        return d, e
    return rng.standard_normal(m), rng.standard_normal(m - 1)


@pytest.mark.parametrize("m", [1, 2, 7, 60])
def test_sym_eig_matches_numpy(lib, m):
    rng = np.random.default_rng(m)
    M = rng.standard_normal((m, m))
    M = (M + M.T) / 2
    A = np.asfortranarray(M.copy())
    w = np.empty(m)
    V = np.empty((m, m), order="F")
    lib.t_sym_eig(m, _p(A), _p(w), _p(V))
    assert np.abs(w - np.linalg.eigvalsh(M)).max() <= 1e-12 * max(1, np.abs(w).max())
    assert np.abs(M @ V - V * w).max() <= 1e-11
    assert np.abs(V.T @ V - np.eye(m)).max() <= 1e-12


@pytest.mark.parametrize("m,clusters", [(50, False), (400, False), (300, True)])
def test_tridiag_eig_and_inverse_iteration(lib, m, clusters):
    rng = np.random.default_rng(m + clusters)
    d, e = _tridiag(rng, m, clusters)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ref = np.linalg.eigvalsh(T)
    w = np.empty(m)
    lib.t_tridiag_eig(m, _p(d.copy()), _p(np.concatenate([e, [0.0]])), _p(w), None)
    assert np.abs(w - ref).max() <= 1e-12 * np.abs(ref).max()
    # eigenvectors of the upper third of the spectrum
    sel = w[2 * m // 3:].copy()
    Z = np.empty((len(sel), m))
    lib.t_tridiag_eigvecs(m, _p(d), _p(np.concatenate([e, [0.0]])), len(sel), _p(sel), _p(Z))
    Z = Z.T
    assert np.abs(T @ Z - Z * sel).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(Z.T @ Z - np.eye(len(sel))).max() <= 1e-10


@pytest.mark.parametrize("m,kind", [(300, "arrow"), (200, "clustered")])
def test_arrowhead_selected_vectors_large_and_clustered(lib, m, kind):
    """Eigenvalues of all, eigenvectors of the top ones only, of a thick-restart
    T (an arrowhead block then a tridiagonal; clustered: every Ritz value of the
    block repeated, as for multiple eigenvalues) through the reduced form."""
    rng = np.random.default_rng(m)
    l = m // 3
    th = np.sort(rng.uniform(0.5, 1.0, l))
    if kind == "clustered":
        th[1::2] = th[0::2][: len(th[1::2])]
    s = rng.standard_normal(l) * 1e-3
    al = rng.uniform(-1, 1, m - l)
    be = rng.uniform(0.1, 0.5, m - l - 1)
    M = np.zeros((m, m))
    M[np.arange(l), np.arange(l)] = th
    M[:l, l] = M[l, :l] = s
    M[np.arange(l, m), np.arange(l, m)] = al
    M[np.arange(l, m - 1), np.arange(l + 1, m)] = be
    M[np.arange(l + 1, m), np.arange(l, m - 1)] = be
    ref = np.linalg.eigvalsh(M)
    thr = float(np.quantile(ref, 0.7))
    w = np.empty(m)
    V = np.zeros((m, m))
    k = lib.t_arrow_eig_sel(m, l, _p(th), _p(s), _p(al), _p(be), _p(w), thr, _p(V))
    assert k == int((ref >= thr).sum())
    assert np.abs(w - ref).max() <= 1e-12 * np.abs(ref).max()
    Z = V[:k].T
    sel = w[m - k:]
    assert np.abs(M @ Z - Z * sel).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(Z.T @ Z - np.eye(k)).max() <= 1e-10


@pytest.mark.parametrize("k,l,seed", [(60, 25, 0), (90, 60, 1), (40, 39, 2), (30, 1, 3),
                                      (12, 11, 4), (200, 120, 5), (3, 1, 6)])
def test_arrowhead_form_matches_dense(lib, k, l, seed):
    """Thick-restart matrix (diagonal block with an arrow into index l, then
    tridiagonal): eigenvalues and the selected eigenvectors through the
    reduction of the arrowhead block equal a dense eigensolve; the eigenvectors
    are orthonormal and satisfy T y = theta y."""
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(0.3, 1.0, l))[::-1].copy()
    s = rng.standard_normal(l) * 1e-2 * rng.uniform(0, 1, l) ** 3
    al = rng.uniform(-0.2, 0.4, k - l)
    be = rng.uniform(0.05, 0.3, max(k - l - 1, 1))
    T = np.zeros((k, k))
    T[np.arange(l), np.arange(l)] = th
    T[l, :l] = T[:l, l] = s
    for r in range(l, k):
        T[r, r] = al[r - l]
        if r + 1 < k:
            T[r, r + 1] = T[r + 1, r] = be[r - l]
    ref = np.linalg.eigvalsh(T)
    thr = float(np.quantile(ref, 0.7))
    w = np.empty(k)
    V = np.zeros((k, k))
    nsel = lib.t_arrow_eig_sel(k, l, _p(th), _p(s), _p(al), _p(be), _p(w), thr, _p(V))
    assert np.abs(w - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert nsel == int((ref >= thr).sum())
    Y = V.reshape(k, k)[:nsel].T          # column-major k x nsel
    lam = w[k - nsel:]
    assert np.abs(Y.T @ Y - np.eye(nsel)).max() <= 1e-10
    assert np.abs(T @ Y - Y * lam).max() <= 1e-11
