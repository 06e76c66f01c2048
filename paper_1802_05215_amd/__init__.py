"""Python binding of libevsl_mi355 (polynomial-filtered spectrum slicing,
EVSL, arXiv:1802.05215) for MI355X.

This module only marshals arguments to the C-ABI declared in
include/evsl_mi355.h: every step of the computation runs in the HIP library.
PyTorch supplies device memory and the stream. Importing the module does not
need a GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libevsl_mi355.so")

EVSL_OK, EVSL_EINVAL, EVSL_ENOMEM, EVSL_EHIP, EVSL_EDEGREE, EVSL_ENOCONV, EVSL_ESPECTRUM, \
    EVSL_ENOTIMPL, EVSL_ESCRATCH = range(9)
EVSL_NOALLOC_SCRATCH_BYTES = 64 << 20
EVSL_F64, EVSL_F32 = 0, 1
EVSL_LAN_TR, EVSL_LAN_NR = 0, 1
DAMP_NONE, DAMP_SIGMA, DAMP_JACKSON = 0, 1, 2

# every entry point declared in include/evsl_mi355.h
EXPORTS = [
    "evsl_create", "evsl_destroy", "evsl_last_hip_error", "evsl_strerror",
    "evsl_spectrum_bounds", "evsl_kpm_dos", "evsl_slice_spectrum", "evsl_kpm_count",
    "evsl_cheb_coeffs", "evsl_filter_apply", "evsl_filtered_lanczos",
    "evsl_filtered_lanczos_batch", "evsl_eigs_get_vectors", "evsl_eigs_free",
    "evsl_filter_stats", "evsl_reset_stats", "evsl_set_timing", "evsl_set_spmv_variant",
    "evsl_set_block_variant", "evsl_autotune", "evsl_set_group_width", "evsl_copy_probe",
    "evsl_gram", "evsl_mem_stats", "evsl_filtered_subspace", "evsl_filtered_subspace_batch",
    "evsl_set_graphs", "evsl_lanczos_dos", "evsl_lanczos_count", "evsl_slice_spectrum_lanczos",
    "evsl_lspol", "evsl_spectrum_bounds_gen", "evsl_filtered_lanczos_gen",
    "evsl_set_block_schedule", "evsl_get_block_schedule", "evsl_autotune_schedule",
    "evsl_filter_apply_noalloc",
]


class EvslError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = _lib().evsl_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")


class CsrT(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("dtype", C.c_int)]


class PolT(C.Structure):
    _fields_ = [("deg", C.c_int), ("boundary", C.c_int), ("gamma", C.c_double),
                ("cc", C.c_double), ("dd", C.c_double), ("bar", C.c_double),
                ("coef", C.POINTER(C.c_double)), ("cap", C.c_int)]


class LanOptsT(C.Structure):
    _fields_ = [("m", C.c_int), ("max_its", C.c_int), ("ncycle", C.c_int), ("tol", C.c_double),
                ("seed", C.c_uint64), ("nev_est", C.c_int), ("nev_cap", C.c_int),
                ("prec", C.c_int), ("val32", C.c_void_p), ("tol_lo", C.c_double),
                ("polish", C.c_int), ("polish_div", C.c_int), ("method", C.c_int),
                ("reserved", C.c_int)]


class SiOptsT(C.Structure):
    _fields_ = [("block", C.c_int), ("max_its", C.c_int), ("tol", C.c_double),
                ("seed", C.c_uint64), ("nev_est", C.c_int), ("reserved", C.c_int * 3)]


class EigsT(C.Structure):
    _fields_ = [("nev", C.c_int), ("lam", C.POINTER(C.c_double)), ("res", C.POINTER(C.c_double)),
                ("Y", C.c_void_p), ("niter", C.c_int), ("nmv", C.c_int), ("nrestart", C.c_int),
                ("npolish", C.c_int), ("status", C.c_int), ("north2", C.c_int),
                ("t_mv", C.c_double), ("t_orth", C.c_double),
                ("t_ritz", C.c_double), ("t_tot", C.c_double)]


_LIB = None
_dp = C.POINTER(C.c_double)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libevsl_mi355.so not built ({LIB_PATH}); run "
                              "`python -m paper_1802_05215_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.evsl_strerror.restype = C.c_char_p
        L.evsl_strerror.argtypes = [C.c_int]
        L.evsl_create.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]
        L.evsl_destroy.argtypes = [C.c_void_p]
        L.evsl_last_hip_error.argtypes = [C.c_void_p]
        L.evsl_spectrum_bounds.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, C.c_uint64, _dp, _dp]
        L.evsl_kpm_dos.argtypes = [C.c_void_p, C.POINTER(CsrT), _dp, C.c_int, C.c_int, C.c_uint64,
                                   C.c_int, _dp, _dp]
        L.evsl_slice_spectrum.argtypes = [_dp, C.c_int, C.c_int, _dp, C.c_int, C.c_int, _dp]
        L.evsl_kpm_count.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                     C.c_double, _dp]
        L.evsl_cheb_coeffs.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(PolT)]
        L.evsl_filter_apply.argtypes = [C.c_void_p, C.POINTER(CsrT), C.POINTER(PolT), C.c_int,
                                        C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_int, C.c_int]
        L.evsl_filter_apply_noalloc.argtypes = L.evsl_filter_apply.argtypes
        L.evsl_filtered_lanczos.argtypes = [C.c_void_p, C.POINTER(CsrT), _dp, C.POINTER(PolT),
                                            C.POINTER(LanOptsT), C.POINTER(EigsT)]
        L.evsl_filtered_lanczos_batch.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, _dp,
                                                  C.POINTER(PolT), C.POINTER(LanOptsT),
                                                  C.POINTER(EigsT)]
        L.evsl_eigs_get_vectors.argtypes = [C.c_void_p, C.POINTER(EigsT), C.c_int64, C.c_void_p,
                                            C.c_int64]
        L.evsl_eigs_free.argtypes = [C.c_void_p, C.POINTER(EigsT)]
        L.evsl_eigs_free.restype = None
        L.evsl_filter_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _dp, _dp]
        L.evsl_reset_stats.argtypes = [C.c_void_p]
        L.evsl_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.evsl_set_graphs.argtypes = [C.c_void_p, C.c_int]
        _ip = C.POINTER(C.c_int)
        L.evsl_lspol.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, _dp]
        L.evsl_spectrum_bounds_gen.argtypes = [C.c_void_p, C.POINTER(CsrT), C.POINTER(CsrT), _dp,
                                               C.c_int, C.c_int, C.c_uint64, _dp, _dp]
        L.evsl_filtered_lanczos_gen.argtypes = [C.c_void_p, C.POINTER(CsrT), C.POINTER(CsrT), _dp,
                                                C.c_int, _dp, C.POINTER(PolT),
                                                C.POINTER(LanOptsT), C.POINTER(EigsT)]
        L.evsl_lanczos_dos.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, C.c_int, C.c_uint64,
                                       _dp, _dp, _ip]
        L.evsl_lanczos_count.argtypes = [_dp, _dp, _ip, C.c_int, C.c_int, C.c_int64, C.c_double,
                                         C.c_double, C.c_double, _dp]
        L.evsl_slice_spectrum_lanczos.argtypes = [_dp, _dp, _ip, C.c_int, C.c_int, C.c_int64,
                                                  C.c_double, C.c_double, C.c_double, C.c_int,
                                                  C.c_int, _dp]
        L.evsl_set_spmv_variant.argtypes = [C.c_void_p, C.c_int]
        L.evsl_set_block_variant.argtypes = [C.c_int]
        L.evsl_autotune.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, C.c_int,
                                    C.POINTER(C.c_int), _dp]
        L.evsl_set_group_width.argtypes = [C.c_void_p, C.c_int]
        L.evsl_set_block_schedule.argtypes = [C.c_void_p] + [C.c_int] * 6
        L.evsl_get_block_schedule.argtypes = [C.c_void_p] + [_ip] * 6
        L.evsl_autotune_schedule.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, C.c_int, _dp]
        L.evsl_copy_probe.argtypes = [C.c_void_p, C.c_int64, C.c_int, _dp]
        L.evsl_filtered_subspace.argtypes = [C.c_void_p, C.POINTER(CsrT), _dp, C.POINTER(PolT),
                                             C.POINTER(SiOptsT), C.POINTER(EigsT)]
        L.evsl_filtered_subspace_batch.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_int, _dp,
                                                   C.POINTER(PolT), C.POINTER(SiOptsT),
                                                   C.POINTER(EigsT)]
        L.evsl_mem_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.c_int]
        L.evsl_gram.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_void_p, C.c_int64,
                                C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]
        _LIB = L
    return _LIB


def load():
    """Load the native library (raises ImportError when it is not built)."""
    return _lib()


def evsl_set_block_variant(v):
    _chk(_lib().evsl_set_block_variant(int(v)), "evsl_set_block_variant")


def _chk(rc, where, ok=(EVSL_OK,)):
    if rc not in ok:
        raise EvslError(rc, where)
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a):
    return a.ctypes.data_as(_dp)


# ------------------------------------------------------------------ context / matrices
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AllocT(C.Structure):
    """evsl_alloc_t: a device allocator given to evsl_create."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


def make_allocator(alloc, free):
    """evsl_alloc_t from two Python callables: alloc(nbytes, stream) -> device
    address (int) or 0 when it cannot; free(ptr, stream). The returned object
    keeps the callbacks alive; pass it to Ctx(alloc=...)."""
    a = ALLOC_FN(lambda user, nbytes, stream: alloc(int(nbytes), stream) or None)
    f = FREE_FN(lambda user, ptr, stream: free(ptr, stream))
    t = AllocT(a, f, None)
    t._keep = (a, f)
    return t


class Ctx:
    """evsl_ctx_t bound to a torch (HIP) stream; `alloc` an evsl_alloc_t from
    make_allocator (None: the library's hipMalloc)."""

    def __init__(self, stream=None, alloc=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.alloc = alloc
        self.h = C.c_void_p()
        _chk(_lib().evsl_create(C.byref(self.h), C.c_void_p(stream.cuda_stream),
                                C.byref(alloc) if alloc is not None else None), "evsl_create")

    def close(self):
        if self.h:
            _lib().evsl_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def filter_stats(self):
        n = C.c_int64()
        s, b = C.c_double(), C.c_double()
        _chk(_lib().evsl_filter_stats(self.h, C.byref(n), C.byref(s), C.byref(b)), "filter_stats")
        return dict(launches=n.value, seconds=s.value, bytes=b.value)

    def reset_stats(self):
        _chk(_lib().evsl_reset_stats(self.h), "reset_stats")

    def set_timing(self, on):
        _chk(_lib().evsl_set_timing(self.h, int(bool(on))), "set_timing")

    def set_graphs(self, on):
        _chk(_lib().evsl_set_graphs(self.h, int(bool(on))), "set_graphs")

    def set_spmv_variant(self, v):
        _chk(_lib().evsl_set_spmv_variant(self.h, int(v)), "set_spmv_variant")

    def set_group_width(self, g):
        _chk(_lib().evsl_set_group_width(self.h, int(g)), "set_group_width")

    def set_block_schedule(self, map, chunk_cols=0, group=1, lane_cols=0, rows_per_wg=0,
                           lds_staging=1):
        _chk(_lib().evsl_set_block_schedule(self.h, int(map), int(chunk_cols), int(group),
                                            int(lane_cols), int(rows_per_wg), int(lds_staging)),
             "evsl_set_block_schedule")

    def block_schedule(self):
        """(map, chunk columns, row-block run, columns per lane, rows per
        workgroup, LDS staging) of the block filter schedule."""
        v = [C.c_int() for _ in range(6)]
        _chk(_lib().evsl_get_block_schedule(self.h, *[C.byref(x) for x in v]),
             "evsl_get_block_schedule")
        return tuple(x.value for x in v)

    def mem_stats(self, reset_peak=False):
        """(bytes held now, peak bytes) of the context's device allocations."""
        cur, peak = C.c_int64(), C.c_int64()
        _chk(_lib().evsl_mem_stats(self.h, C.byref(cur), C.byref(peak), int(bool(reset_peak))),
             "evsl_mem_stats")
        return cur.value, peak.value


def evsl_copy_probe(ctx, nbytes, reps=20):
    """Seconds per launch of a plain copy of nbytes (read nbytes + write nbytes)."""
    t = C.c_double()
    _chk(_lib().evsl_copy_probe(ctx.h, int(nbytes), int(reps), C.byref(t)), "evsl_copy_probe")
    return t.value


def evsl_autotune(ctx, A, max_cols, prec=EVSL_F64):
    """Returns (group width, microseconds per column-step)."""
    g = C.c_int()
    us = C.c_double()
    _chk(_lib().evsl_autotune(ctx.h, C.byref(A.t), int(max_cols), int(prec), C.byref(g),
                              C.byref(us)), "evsl_autotune")
    return g.value, us.value


def evsl_autotune_schedule(ctx, A, ncols, prec=EVSL_F64):
    """Picks the block filter schedule for ncols columns on A (kept in ctx);
    returns ctx.block_schedule() followed by the ms per degree step."""
    ms = C.c_double()
    _chk(_lib().evsl_autotune_schedule(ctx.h, C.byref(A.t), int(ncols), int(prec), C.byref(ms)),
         "evsl_autotune_schedule")
    return ctx.block_schedule() + (ms.value,)


class DeviceCsr:
    """CSR matrix resident on the device (torch tensors) + its evsl_csr_t."""

    def __init__(self, row_ptr, col, val, n):
        self.row_ptr, self.col, self.val, self.n = row_ptr, col, val, int(n)
        import torch
        dt = EVSL_F64 if val.dtype == torch.float64 else EVSL_F32
        self.t = CsrT(self.n, int(col.numel()), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                      dt)

    @property
    def nnz(self):
        return int(self.col.numel())

    @classmethod
    def from_host(cls, A, device="cuda", dtype=None):
        import torch
        dtype = dtype or torch.float64
        rp = torch.as_tensor(np.ascontiguousarray(A.row_ptr, np.int32)).to(device)
        ci = torch.as_tensor(np.ascontiguousarray(A.col, np.int32)).to(device)
        va = torch.as_tensor(np.ascontiguousarray(A.val, np.float64)).to(device=device, dtype=dtype)
        return cls(rp, ci, va, A.n)

    def with_values(self, val):
        return DeviceCsr(self.row_ptr, self.col, val, self.n)


# ------------------------------------------------------------------ entry points
def evsl_spectrum_bounds(ctx, A, nsteps=80, seed=3):
    lo, hi = C.c_double(), C.c_double()
    _chk(_lib().evsl_spectrum_bounds(ctx.h, C.byref(A.t), nsteps, seed, C.byref(lo), C.byref(hi)),
         "evsl_spectrum_bounds")
    return lo.value, hi.value


def evsl_kpm_dos(ctx, A, intv, degree, nvec, seed=1, damping=DAMP_JACKSON):
    iv = _f64(intv)
    mom = np.empty(degree + 1)
    est = C.c_double()
    _chk(_lib().evsl_kpm_dos(ctx.h, C.byref(A.t), _dptr(iv), degree, nvec, seed, damping,
                             _dptr(mom), C.byref(est)), "evsl_kpm_dos")
    return mom, est.value


def evsl_slice_spectrum(moments, damping, intv, nslices, npts=2000):
    mom, iv = _f64(moments), _f64(intv)
    sli = np.empty(nslices + 1)
    _chk(_lib().evsl_slice_spectrum(_dptr(mom), len(mom) - 1, damping, _dptr(iv), nslices, npts,
                                    _dptr(sli)), "evsl_slice_spectrum")
    return sli


def evsl_kpm_count(moments, damping, lmin, lmax, x0, x1):
    mom = _f64(moments)
    out = C.c_double()
    _chk(_lib().evsl_kpm_count(_dptr(mom), len(mom) - 1, damping, lmin, lmax, x0, x1,
                               C.byref(out)), "evsl_kpm_count")
    return out.value


def evsl_lanczos_dos(ctx, A, msteps, nvec, seed=1):
    """Lanczos DOS quadrature: (nodes, weights, dims), nodes/weights nvec x msteps."""
    nodes = np.zeros((nvec, msteps))
    weights = np.zeros((nvec, msteps))
    dims = np.zeros(nvec, np.int32)
    _chk(_lib().evsl_lanczos_dos(ctx.h, C.byref(A.t), msteps, nvec, seed, _dptr(nodes),
                                 _dptr(weights), dims.ctypes.data_as(C.POINTER(C.c_int))),
         "evsl_lanczos_dos")
    return nodes, weights, dims


def evsl_lanczos_count(q, n, sigma, x0, x1):
    nodes, weights, dims = (np.ascontiguousarray(q[0], np.float64),
                            np.ascontiguousarray(q[1], np.float64),
                            np.ascontiguousarray(q[2], np.int32))
    out = C.c_double()
    _chk(_lib().evsl_lanczos_count(_dptr(nodes), _dptr(weights),
                                   dims.ctypes.data_as(C.POINTER(C.c_int)), nodes.shape[0],
                                   nodes.shape[1], int(n), sigma, x0, x1, C.byref(out)),
         "evsl_lanczos_count")
    return out.value


def evsl_slice_spectrum_lanczos(q, n, sigma, xi, eta, nslices, npts=2000):
    nodes, weights, dims = (np.ascontiguousarray(q[0], np.float64),
                            np.ascontiguousarray(q[1], np.float64),
                            np.ascontiguousarray(q[2], np.int32))
    sli = np.empty(nslices + 1)
    _chk(_lib().evsl_slice_spectrum_lanczos(_dptr(nodes), _dptr(weights),
                                            dims.ctypes.data_as(C.POINTER(C.c_int)),
                                            nodes.shape[0], nodes.shape[1], int(n), sigma, xi, eta,
                                            nslices, npts, _dptr(sli)),
         "evsl_slice_spectrum_lanczos")
    return sli


class Pol:
    """A polynomial filter (evsl_pol_t with its host coefficient buffer)."""

    def __init__(self, max_deg):
        self.buf = np.zeros(max_deg + 1)
        self.t = PolT(0, 0, 0.0, 0.0, 0.0, 0.0, _dptr(self.buf), max_deg + 1)
        self.status = EVSL_OK

    deg = property(lambda s: s.t.deg)
    boundary = property(lambda s: s.t.boundary)
    gamma = property(lambda s: s.t.gamma)
    cc = property(lambda s: s.t.cc)
    dd = property(lambda s: s.t.dd)
    bar = property(lambda s: s.t.bar)

    @property
    def coef(self):
        return self.buf[:self.t.deg + 1].copy()


def evsl_cheb_coeffs(intv, damping=DAMP_JACKSON, tau=0.8, tau_ext=0.4, max_deg=10000):
    iv = _f64(intv)
    p = Pol(max_deg)
    p.status = _chk(_lib().evsl_cheb_coeffs(_dptr(iv), damping, tau, tau_ext, max_deg,
                                            C.byref(p.t)), "evsl_cheb_coeffs",
                    ok=(EVSL_OK, EVSL_EDEGREE))
    return p


def _filter_call(fn, name, ctx, A, pols, col_group, V, Y, prec):
    import torch
    if prec is None:
        prec = EVSL_F64 if V.dtype == torch.float64 else EVSL_F32
    ncols = 1 if V.dim() == 1 else V.shape[1]
    ldv = 1 if V.dim() == 1 else V.stride(0)
    arr = (PolT * len(pols))(*[p.t for p in pols])
    cg = np.ascontiguousarray(col_group, dtype=np.int32)
    _chk(fn(ctx.h, C.byref(A.t), arr, len(pols), cg.ctypes.data_as(C.POINTER(C.c_int32)),
            C.c_void_p(V.data_ptr()), C.c_void_p(Y.data_ptr()), ldv, ncols, prec), name)


def evsl_filter_apply(ctx, A, pols, col_group, V, Y, prec=None):
    """Y = p(A-hat) V for row-major torch tensors V, Y (n x ncols, contiguous)."""
    _filter_call(_lib().evsl_filter_apply, "evsl_filter_apply", ctx, A, pols, col_group, V, Y,
                 prec)


def evsl_filter_apply_noalloc(ctx, A, pols, col_group, V, Y, prec=None):
    """evsl_filter_apply with its scratch in the library's static device array
    (no device allocation); EvslError(EVSL_ESCRATCH) when it does not fit."""
    _filter_call(_lib().evsl_filter_apply_noalloc, "evsl_filter_apply_noalloc", ctx, A, pols,
                 col_group, V, Y, prec)


def lan_opts(m=0, max_its=0, ncycle=0, tol=1e-8, seed=2, nev_est=0, nev_cap=0, prec=EVSL_F64,
             val32=None, tol_lo=0.0, polish=0, polish_div=0, method=0):
    return LanOptsT(m, max_its, ncycle, tol, seed, nev_est, nev_cap, prec,
                    C.c_void_p(val32.data_ptr() if val32 is not None else 0), tol_lo, polish,
                    polish_div, method, 0)


def evsl_gram(ctx, X, Y, C_out):
    """C_out (p x q, column-major torch view) = X^T Y for column-major torch
    views X (n x p) and Y (n x q) (i.e. tensors whose transposes are contiguous)."""
    n, p = X.shape
    q = Y.shape[1]
    _chk(_lib().evsl_gram(ctx.h, n, p, q, C.c_void_p(X.data_ptr()), X.stride(1),
                          C.c_void_p(Y.data_ptr()), Y.stride(1), C.c_void_p(C_out.data_ptr()),
                          C_out.stride(1)), "evsl_gram")


def _take(ctx, out, n, device):
    """Copy a library-owned result into numpy/torch objects and free it."""
    import torch
    k = out.nev
    lam = np.ctypeslib.as_array(out.lam, shape=(k,)).copy() if k else np.empty(0)
    res = np.ctypeslib.as_array(out.res, shape=(k,)).copy() if k else np.empty(0)
    Yt = torch.empty((k, n), dtype=torch.float64, device=device)
    if k:
        _chk(_lib().evsl_eigs_get_vectors(ctx.h, C.byref(out), n, C.c_void_p(Yt.data_ptr()), n),
             "evsl_eigs_get_vectors")
        torch.cuda.current_stream().synchronize()
    stats = dict(nev=k, niter=out.niter, nmv=out.nmv, nrestart=out.nrestart, npolish=out.npolish,
                 north2=out.north2, status=out.status,
                 t_mv=out.t_mv, t_orth=out.t_orth, t_ritz=out.t_ritz, t_tot=out.t_tot)
    _lib().evsl_eigs_free(ctx.h, C.byref(out))
    return lam, Yt.T, res, stats


def evsl_filtered_lanczos(ctx, A, intv, pol, opts=None):
    """Returns (lam ascending, Y (n x nev torch view), res, stats)."""
    iv = _f64(intv)
    out = EigsT()
    opts = opts or lan_opts()
    _chk(_lib().evsl_filtered_lanczos(ctx.h, C.byref(A.t), _dptr(iv), C.byref(pol.t),
                                      C.byref(opts), C.byref(out)), "evsl_filtered_lanczos",
         ok=(EVSL_OK, EVSL_ENOCONV))
    return _take(ctx, out, A.n, A.val.device)


def evsl_filtered_lanczos_batch(ctx, A, intvs, pols, opts_list):
    ns = len(pols)
    iv = _f64(np.asarray(intvs).reshape(-1))
    parr = (PolT * ns)(*[p.t for p in pols])
    oarr = (LanOptsT * ns)(*opts_list)
    outs = (EigsT * ns)()
    _chk(_lib().evsl_filtered_lanczos_batch(ctx.h, C.byref(A.t), ns, _dptr(iv), parr, oarr, outs),
         "evsl_filtered_lanczos_batch", ok=(EVSL_OK, EVSL_ENOCONV))
    return [_take(ctx, outs[q], A.n, A.val.device) for q in range(ns)]


def si_opts(block=0, max_its=0, tol=1e-8, seed=2, nev_est=0):
    return SiOptsT(block, max_its, tol, seed, nev_est, (C.c_int * 3)())


def evsl_filtered_subspace(ctx, A, intv, pol, opts=None):
    """Filtered subspace iteration on one slice: (lam, Y, res, stats)."""
    iv = _f64(intv)
    out = EigsT()
    opts = opts or si_opts()
    _chk(_lib().evsl_filtered_subspace(ctx.h, C.byref(A.t), _dptr(iv), C.byref(pol.t),
                                       C.byref(opts), C.byref(out)), "evsl_filtered_subspace",
         ok=(EVSL_OK, EVSL_ENOCONV))
    return _take(ctx, out, A.n, A.val.device)


def evsl_filtered_subspace_batch(ctx, A, intvs, pols, opts_list):
    ns = len(pols)
    iv = _f64(np.asarray(intvs).reshape(-1))
    parr = (PolT * ns)(*[p.t for p in pols])
    oarr = (SiOptsT * ns)(*opts_list)
    outs = (EigsT * ns)()
    _chk(_lib().evsl_filtered_subspace_batch(ctx.h, C.byref(A.t), ns, _dptr(iv), parr, oarr, outs),
         "evsl_filtered_subspace_batch", ok=(EVSL_OK, EVSL_ENOCONV))
    return [_take(ctx, outs[q], A.n, A.val.device) for q in range(ns)]


def evsl_lspol(kind, lo, hi, deg):
    """Chebyshev coefficients of the least-squares fit of 1/t (kind 0) or
    1/sqrt(t) (kind 1) on [lo, hi]."""
    coef = np.zeros(deg + 1)
    _chk(_lib().evsl_lspol(kind, lo, hi, deg, _dptr(coef)), "evsl_lspol")
    return coef


def evsl_spectrum_bounds_gen(ctx, A, B, bbounds, bdeg, nsteps=80, seed=3):
    bb = _f64(bbounds)
    lo, hi = C.c_double(), C.c_double()
    _chk(_lib().evsl_spectrum_bounds_gen(ctx.h, C.byref(A.t), C.byref(B.t), _dptr(bb), bdeg,
                                         nsteps, seed, C.byref(lo), C.byref(hi)),
         "evsl_spectrum_bounds_gen")
    return lo.value, hi.value


def evsl_filtered_lanczos_gen(ctx, A, B, bbounds, bdeg, intv, pol, opts=None):
    """Filtered Lanczos for (A, B), non-restart by default or thick restart
    (opts.method = EVSL_LAN_TR): (lam, Y (B-orthonormal), res, stats)."""
    bb = _f64(bbounds)
    iv = _f64(intv)
    out = EigsT()
    opts = opts or lan_opts(method=EVSL_LAN_NR)
    _chk(_lib().evsl_filtered_lanczos_gen(ctx.h, C.byref(A.t), C.byref(B.t), _dptr(bb), bdeg,
                                          _dptr(iv), C.byref(pol.t), C.byref(opts), C.byref(out)),
         "evsl_filtered_lanczos_gen", ok=(EVSL_OK, EVSL_ENOCONV))
    return _take(ctx, out, A.n, A.val.device)
