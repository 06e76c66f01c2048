"""ORACLE -- test infrastructure only.

ctypes binding of the plain C reference implementation in ``evsl_oracle.c``
(EVSL paper, arXiv:1802.05215). Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this package; the HIP library and its
Python binding never do.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "evsl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DAMP_NONE, DAMP_SIGMA, DAMP_JACKSON = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP on row loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _setup(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class LanOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("max_its", C.c_int), ("ncycle", C.c_int), ("tol", C.c_double),
                ("seed", C.c_uint64), ("nev_cap", C.c_int)]


class SiOpts(C.Structure):
    _fields_ = [("block", C.c_int), ("max_its", C.c_int), ("tol", C.c_double),
                ("seed", C.c_uint64), ("nev_cap", C.c_int)]


class LanStats(C.Structure):
    _fields_ = [("nev", C.c_int), ("niter", C.c_int), ("nmv", C.c_int), ("nrestart", C.c_int),
                ("status", C.c_int)]


def _setup(L):
    L.or_splitmix64.restype = C.c_uint64
    L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.or_uniform01.restype = C.c_double
    L.or_uniform01.argtypes = [C.c_uint64, C.c_uint64]
    L.or_spmv.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp]
    L.or_damping.argtypes = [C.c_int, C.c_int, _dp]
    L.or_cheb_series.restype = C.c_double
    L.or_cheb_series.argtypes = [C.c_int, _dp, C.c_double]
    L.or_find_pol.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_int,
                              C.POINTER(C.c_int), _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int)]
    L.or_filter_apply.argtypes = [C.c_int64, _ip, _ip, _dp, C.c_double, C.c_double, C.c_int,
                                  _dp, C.c_int, _dp, _dp]
    L.or_rademacher.argtypes = [C.c_uint64, C.c_int64, C.c_int, _dp]
    L.or_kpm_moments.argtypes = [C.c_int64, _ip, _ip, _dp, C.c_double, C.c_double, C.c_int,
                                 C.c_int, _dp, _dp]
    L.or_kpm_count.restype = C.c_double
    L.or_kpm_count.argtypes = [C.c_int, _dp, C.c_int, C.c_double, C.c_double, C.c_double,
                               C.c_double]
    L.or_slicer.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_int, C.c_int, _dp]
    L.or_jacobi_eig.argtypes = [C.c_int, _dp, _dp, _dp]
    L.or_lanczos_bounds.argtypes = [C.c_int64, _ip, _ip, _dp, C.c_int, C.c_uint64, _dp, _dp]
    L.or_lanczos_start.argtypes = [C.c_uint64, C.c_int64, C.c_int64, _dp]
    L.or_filtered_lanczos.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, C.c_int, _dp, C.c_double,
                                      C.POINTER(LanOpts), _dp, _dp, _dp, C.POINTER(LanStats)]
    L.or_filtered_lanczos_nr.argtypes = L.or_filtered_lanczos.argtypes
    L.or_lspol.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, _dp]
    L.or_cg_solve.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp]
    L.or_lanczos_bounds_gen.argtypes = [C.c_int64, _ip, _ip, _dp, _ip, _ip, _dp, C.c_int,
                                        C.c_uint64, _dp, _dp]
    L.or_filtered_lanczos_gen.argtypes = [C.c_int64, _ip, _ip, _dp, _ip, _ip, _dp, _dp, C.c_int, _dp,
                                          C.c_double, C.POINTER(LanOpts), _dp, _dp, _dp,
                                          C.POINTER(LanStats)]
    L.or_filtered_lanczos_gen_tr.argtypes = L.or_filtered_lanczos_gen.argtypes
    L.or_lanczos_dos.argtypes = [C.c_int64, _ip, _ip, _dp, C.c_int, C.c_int, C.c_uint64, _dp, _dp,
                                 _ip]
    L.or_lanczos_count.argtypes = [_dp, _dp, _ip, C.c_int, C.c_int, C.c_int64, C.c_double,
                                   C.c_double, C.c_double]
    L.or_lanczos_count.restype = C.c_double
    L.or_lanczos_slicer.argtypes = [_dp, _dp, _ip, C.c_int, C.c_int, C.c_int64, C.c_double,
                                    C.c_double, C.c_double, C.c_int, C.c_int, _dp]
    L.or_filtered_subspace.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, C.c_int, _dp, C.c_double,
                                       C.POINTER(SiOpts), _dp, _dp, _dp, C.POINTER(LanStats)]


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _csr(A):
    return (C.c_int64(A.n), _i(np.ascontiguousarray(A.row_ptr, np.int32)),
            _i(np.ascontiguousarray(A.col, np.int32)), _d(_f64(A.val)))


def splitmix64(seed, i):
    return lib().or_splitmix64(seed, i)


def spmv(A, x):
    x = _f64(x)
    y = np.empty(A.n)
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    lib().or_spmv(A.n, _i(rp), _i(ci), _d(va), _d(x), _d(y))
    return y


def damping(kind, k):
    g = np.empty(k + 1)
    if lib().or_damping(kind, k, _d(g)) != 0:
        raise ValueError("bad damping")
    return g


def cheb_series(coef, t):
    coef = _f64(coef)
    return lib().or_cheb_series(len(coef) - 1, _d(coef), float(t))


def find_pol(intv, damping=DAMP_SIGMA, tau=0.8, tau_ext=0.4, max_deg=10000):
    """Returns dict(deg, gamma, bar, cc, dd, coef, boundary, status)."""
    iv = _f64(intv)
    coef = np.zeros(max_deg + 1)
    deg = C.c_int()
    bnd = C.c_int()
    gamma, bar, cc, dd = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    rc = lib().or_find_pol(_d(iv), damping, tau, tau_ext, max_deg, C.byref(deg), C.byref(gamma),
                           C.byref(bar), C.byref(cc), C.byref(dd), _d(coef), C.byref(bnd))
    if rc < 0:
        raise ValueError("find_pol: invalid interval")
    return dict(deg=deg.value, gamma=gamma.value, bar=bar.value, cc=cc.value, dd=dd.value,
                coef=coef[:deg.value + 1].copy(), boundary=bnd.value, status=rc)


def filter_apply(A, cc, dd, coef, V):
    V = _f64(V)
    nvec = 1 if V.ndim == 1 else V.shape[1]
    Y = np.empty_like(V)
    coef = _f64(coef)
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    lib().or_filter_apply(A.n, _i(rp), _i(ci), _d(va), cc, dd, len(coef) - 1, _d(coef), nvec,
                          _d(V), _d(Y))
    return Y


def rademacher(seed, n, nvec):
    V = np.empty((n, nvec))
    lib().or_rademacher(seed, n, nvec, _d(V))
    return V


def kpm_moments(A, lmin, lmax, K, V):
    V = _f64(V)
    nvec = 1 if V.ndim == 1 else V.shape[1]
    mom = np.empty(K + 1)
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    lib().or_kpm_moments(A.n, _i(rp), _i(ci), _d(va), lmin, lmax, K, nvec, _d(V), _d(mom))
    return mom


def kpm_count(mom, damping, lmin, lmax, x0, x1):
    mom = _f64(mom)
    return lib().or_kpm_count(len(mom) - 1, _d(mom), damping, lmin, lmax, x0, x1)


def slicer(mom, damping, intv, nslices, npts=2000):
    mom = _f64(mom)
    iv = _f64(intv)
    sli = np.empty(nslices + 1)
    if lib().or_slicer(len(mom) - 1, _d(mom), damping, _d(iv), nslices, npts, _d(sli)) != 0:
        raise ValueError("slicer failed")
    return sli


def jacobi_eig(A):
    m = A.shape[0]
    a = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    w = np.empty(m)
    V = np.empty((m, m), order="F")
    lib().or_jacobi_eig(m, a.ctypes.data_as(_dp), _d(w), V.ctypes.data_as(_dp))
    return w, V


def lanczos_bounds(A, nsteps=80, seed=3):
    lo, hi = C.c_double(), C.c_double()
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    if lib().or_lanczos_bounds(A.n, _i(rp), _i(ci), _d(va), nsteps, seed, C.byref(lo),
                               C.byref(hi)) != 0:
        raise ValueError("bounds failed")
    return lo.value, hi.value


def lanczos_start(seed, n, restart=0):
    x = np.empty(n)
    lib().or_lanczos_start(seed, n, restart, _d(x))
    return x


def filtered_lanczos(A, intv, pol, m=None, max_its=None, ncycle=30, tol=1e-10, seed=2,
                     nev_cap=None, nev_est=None):
    """Algorithm alg:FiltLanTR on one slice. Returns (lam, Y (n x nev), res, stats)."""
    if nev_est is None:
        nev_est = 50
    if m is None:
        m = max(3 * int(nev_est) + 30, 60)
    if max_its is None:
        max_its = max(20 * m, 2000)
    if nev_cap is None:
        nev_cap = max(4 * int(nev_est) + 40, 100)
    n = A.n
    iv = _f64(intv)
    coef = _f64(pol["coef"])
    lam = np.empty(nev_cap)
    res = np.empty(nev_cap)
    Y = np.empty((nev_cap, n))       # column-major n x nev_cap == row-major nev_cap x n
    opts = LanOpts(m, max_its, ncycle, tol, seed, nev_cap)
    st = LanStats()
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    rc = lib().or_filtered_lanczos(n, _i(rp), _i(ci), _d(va), _d(iv), len(coef) - 1, _d(coef),
                                   pol["bar"], C.byref(opts), _d(lam), _d(res), _d(Y),
                                   C.byref(st))
    if rc != 0:
        raise ValueError("filtered_lanczos: invalid arguments")
    k = st.nev
    stats = dict(nev=k, niter=st.niter, nmv=st.nmv, nrestart=st.nrestart, status=st.status)
    return lam[:k].copy(), Y[:k].T.copy(), res[:k].copy(), stats


def filtered_lanczos_nr(A, intv, pol, m=None, ncycle=30, tol=1e-10, seed=2, nev_cap=None,
                        nev_est=None):
    """Filtered non-restart Lanczos on one slice (at most m steps). Returns
    (lam, Y (n x nev), res, stats) as filtered_lanczos."""
    if nev_est is None:
        nev_est = 50
    if m is None:
        m = max(5 * int(nev_est) + 200, 400)
    if nev_cap is None:
        nev_cap = max(2 * int(nev_est) + 40, 100)
    n = A.n
    iv = _f64(intv)
    coef = _f64(pol["coef"])
    lam = np.empty(nev_cap)
    res = np.empty(nev_cap)
    Y = np.empty((nev_cap, n))
    opts = LanOpts(m, m, ncycle, tol, seed, nev_cap)
    st = LanStats()
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    rc = lib().or_filtered_lanczos_nr(n, _i(rp), _i(ci), _d(va), _d(iv), len(coef) - 1, _d(coef),
                                      pol["bar"], C.byref(opts), _d(lam), _d(res), _d(Y),
                                      C.byref(st))
    if rc != 0:
        raise ValueError("filtered_lanczos_nr: invalid arguments")
    k = st.nev
    stats = dict(nev=k, niter=st.niter, nmv=st.nmv, nrestart=st.nrestart, status=st.status)
    return lam[:k].copy(), Y[:k].T.copy(), res[:k].copy(), stats


def filtered_subspace(A, intv, pol, block=None, max_its=200, tol=1e-10, seed=2, nev_cap=None,
                      nev_est=None):
    """Filtered subspace iteration on one slice with a block of `block`
    vectors (default 3 nev_est + 8). Returns (lam, Y (n x nev), res, stats)."""
    if nev_est is None:
        nev_est = 50
    if block is None:
        block = 3 * int(nev_est) + 8
    block = min(block, A.n)
    if nev_cap is None:
        nev_cap = block
    n = A.n
    iv = _f64(intv)
    coef = _f64(pol["coef"])
    lam = np.empty(nev_cap)
    res = np.empty(nev_cap)
    Y = np.empty((nev_cap, n))
    opts = SiOpts(block, max_its, tol, seed, nev_cap)
    st = LanStats()
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    rc = lib().or_filtered_subspace(n, _i(rp), _i(ci), _d(va), _d(iv), len(coef) - 1, _d(coef),
                                    pol["bar"], C.byref(opts), _d(lam), _d(res), _d(Y),
                                    C.byref(st))
    if rc != 0:
        raise ValueError("filtered_subspace: invalid arguments")
    k = st.nev
    stats = dict(nev=k, niter=st.niter, nmv=st.nmv, status=st.status)
    return lam[:k].copy(), Y[:k].T.copy(), res[:k].copy(), stats


def lanczos_dos(A, m, nvec, seed=1):
    """Lanczos DOS quadrature: (nodes, weights, dims), nodes/weights nvec x m."""
    rp, ci, va = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                  _f64(A.val))
    nodes = np.zeros((nvec, m))
    weights = np.zeros((nvec, m))
    dims = np.zeros(nvec, np.int32)
    if lib().or_lanczos_dos(A.n, _i(rp), _i(ci), _d(va), m, nvec, seed, _d(nodes), _d(weights),
                            _i(dims)) != 0:
        raise ValueError("lanczos_dos: invalid arguments")
    return nodes, weights, dims


def lanczos_count(q, n, sigma, x0, x1):
    nodes, weights, dims = q
    nvec, m = nodes.shape
    return lib().or_lanczos_count(_d(nodes), _d(weights), _i(dims), nvec, m, n, sigma, x0, x1)


def lanczos_slicer(q, n, sigma, xi, eta, nslices, npts=2000):
    nodes, weights, dims = q
    nvec, m = nodes.shape
    sli = np.empty(nslices + 1)
    if lib().or_lanczos_slicer(_d(nodes), _d(weights), _i(dims), nvec, m, n, sigma, xi, eta,
                               nslices, npts, _d(sli)) != 0:
        raise ValueError("lanczos_slicer failed")
    return sli


def _csr(A):
    return (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
            _f64(A.val))


def lspol(kind, lo, hi, deg):
    """Chebyshev coefficients of 1/t (kind 0) or 1/sqrt(t) (kind 1) on [lo, hi]."""
    coef = np.zeros(deg + 1)
    if lib().or_lspol(kind, lo, hi, deg, _d(coef)) != 0:
        raise ValueError("lspol: invalid arguments")
    return coef


def cg_solve(B, r):
    rp, ci, vb = _csr(B)
    r = _f64(r)
    x = np.empty_like(r)
    lib().or_cg_solve(B.n, _i(rp), _i(ci), _d(vb), _d(r), _d(x))
    return x


def lanczos_bounds_gen(A, B, nsteps=80, seed=3):
    ra, ca, va = _csr(A)
    rb, cb, vb = _csr(B)
    lo, hi = C.c_double(), C.c_double()
    lib().or_lanczos_bounds_gen(A.n, _i(ra), _i(ca), _d(va), _i(rb), _i(cb), _d(vb), nsteps, seed,
                                C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def filtered_lanczos_gen(A, B, intv, pol, m=None, ncycle=30, tol=1e-10, seed=2, nev_cap=None,
                         nev_est=None):
    """Filtered non-restart Lanczos for the pencil (A, B). Returns (lam, Y (n x nev,
    B-orthonormal), res, stats)."""
    if nev_est is None:
        nev_est = 50
    if m is None:
        m = max(5 * int(nev_est) + 200, 400)
    if nev_cap is None:
        nev_cap = max(2 * int(nev_est) + 40, 100)
    n = A.n
    ra, ca, va = _csr(A)
    rb, cb, vb = _csr(B)
    iv = _f64(intv)
    coef = _f64(pol["coef"])
    lam, res = np.empty(nev_cap), np.empty(nev_cap)
    Y = np.empty((nev_cap, n))
    opts = LanOpts(m, m, ncycle, tol, seed, nev_cap)
    st = LanStats()
    rc = lib().or_filtered_lanczos_gen(n, _i(ra), _i(ca), _d(va), _i(rb), _i(cb), _d(vb), _d(iv),
                                       len(coef) - 1, _d(coef), pol["bar"], C.byref(opts), _d(lam),
                                       _d(res), _d(Y), C.byref(st))
    if rc != 0:
        raise ValueError("filtered_lanczos_gen: invalid arguments")
    k = st.nev
    stats = dict(nev=k, niter=st.niter, nmv=st.nmv, status=st.status)
    return lam[:k].copy(), Y[:k].T.copy(), res[:k].copy(), stats


def filtered_lanczos_gen_tr(A, B, intv, pol, m=None, max_its=None, ncycle=30, tol=1e-10, seed=2,
                            nev_cap=None, nev_est=None):
    """Filtered thick-restart Lanczos for the pencil (A, B) (Algorithm
    alg:FiltLanTR in the B-inner product). Returns (lam, Y (n x nev,
    B-orthonormal), res, stats)."""
    if nev_est is None:
        nev_est = 50
    if m is None:
        m = max(3 * int(nev_est) + 30, 60)
    if max_its is None:
        max_its = max(20 * m, 2000)
    if nev_cap is None:
        nev_cap = max(4 * int(nev_est) + 40, 100)
    n = A.n
    ra, ca, va = _csr(A)
    rb, cb, vb = _csr(B)
    iv = _f64(intv)
    coef = _f64(pol["coef"])
    lam, res = np.empty(nev_cap), np.empty(nev_cap)
    Y = np.empty((nev_cap, n))
    opts = LanOpts(m, max_its, ncycle, tol, seed, nev_cap)
    st = LanStats()
    rc = lib().or_filtered_lanczos_gen_tr(n, _i(ra), _i(ca), _d(va), _i(rb), _i(cb), _d(vb),
                                          _d(iv), len(coef) - 1, _d(coef), pol["bar"],
                                          C.byref(opts), _d(lam), _d(res), _d(Y), C.byref(st))
    if rc != 0:
        raise ValueError("filtered_lanczos_gen_tr: invalid arguments")
    k = st.nev
    stats = dict(nev=k, niter=st.niter, nmv=st.nmv, nrestart=st.nrestart, status=st.status)
    return lam[:k].copy(), Y[:k].T.copy(), res[:k].copy(), stats
