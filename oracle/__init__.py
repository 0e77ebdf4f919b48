"""Python access to the plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It loads ``liboracle.so`` (plain C, built by gcc from
``oracle.c``) through ctypes and shares nothing with the GPU library.
Every function names the passage of the paper it follows; the C source
holds the arithmetic.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, NOT_CONVERGED, EINVAL, ENOMEM, BREAKDOWN = 0, 1, -1, -2, -4

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_c_i64, _c_int, _c_dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double


def lib():
    """Load liboracle.so, building it with gcc only if it is not there."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _LIB = _configure(ctypes.CDLL(path))
    return _LIB


def load_timing_build(path):
    """A timing build of the oracle (oracle/build.py build_timing), for the
    benchmark's CPU baseline: the same functions, passed as `library=`."""
    return _configure(ctypes.CDLL(path))


def _configure(L):
    """Declare the C signatures on a loaded build of oracle.c."""
    L.orc_num_threads.restype = _c_int
    L.orc_num_threads.argtypes = []
    L.orc_num_rows.restype = _c_i64
    L.orc_num_rows.argtypes = [_c_int] * 3
    L.orc_count_nnz.restype = _c_i64
    L.orc_count_nnz.argtypes = [_c_int] * 3
    L.orc_boundary.restype = None
    L.orc_boundary.argtypes = [_c_int] * 3 + [ctypes.c_void_p, ctypes.c_void_p, _u8p, _f64p]
    L.orc_element_matrix.restype = None
    L.orc_element_matrix.argtypes = [_c_dbl] * 3 + [_f64p]
    L.orc_assemble.restype = _c_int
    L.orc_assemble.argtypes = [_c_int] * 3 + [ctypes.c_void_p, ctypes.c_void_p, _c_int,
                                              _i64p, _i32p, _f64p, _f64p]
    L.orc_assemble_rows.restype = _c_int
    L.orc_assemble_rows.argtypes = [_c_int] * 3 + [ctypes.c_void_p, ctypes.c_void_p, _c_i64, _i64p,
                                                   _i32p, _f64p, _i32p, _f64p]
    L.orc_csr_spmv.restype = None
    L.orc_csr_spmv.argtypes = [_c_i64, _i64p, _i32p, _f64p, _f64p, _f64p]
    L.orc_bcrsvar_count.restype = _c_i64
    L.orc_bcrsvar_count.argtypes = [_c_i64, _i64p, _i32p]
    L.orc_bcrsvar_build.restype = None
    L.orc_bcrsvar_build.argtypes = [_c_i64, _i64p, _i32p, _i32p, _i64p, _i64p]
    for fn in (L.orc_bcrsvar_spmv, L.orc_bcrsvar_spmv_switch):
        fn.restype = None
        fn.argtypes = [_c_i64, _i64p, _i32p, _i64p, _f64p, _f64p, _f64p]
    L.orc_bcrs13_build.restype = _c_i64
    L.orc_bcrs13_build.argtypes = [_c_i64, _i64p, _i32p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_bcrs13_spmv.restype = None
    L.orc_bcrs13_spmv.argtypes = [_c_i64, _i64p, _i32p, _f64p, _f64p, _f64p]
    L.orc_cg.restype = _c_int
    L.orc_cg.argtypes = [_c_i64, _i64p, _i32p, _f64p, _f64p, _f64p, _c_dbl, _c_int,
                         ctypes.POINTER(_c_int), ctypes.POINTER(_c_dbl),
                         ctypes.POINTER(_c_dbl), ctypes.c_void_p]
    L.orc_cg_single_reduction.restype = _c_int
    L.orc_cg_single_reduction.argtypes = L.orc_cg.argtypes
    L.orc_cg_jacobi.restype = _c_int
    L.orc_cg_jacobi.argtypes = L.orc_cg.argtypes
    L.orc_cg_mixed.restype = _c_int
    L.orc_cg_mixed.argtypes = [_c_i64, _i64p, _i32p, _f64p, _f64p, _f64p, _c_dbl, _c_dbl,
                               _c_int, _c_int, ctypes.POINTER(_c_int),
                               ctypes.POINTER(_c_int), ctypes.POINTER(_c_dbl)]
    L.orc_cg_mixed_keep.restype = _c_int
    L.orc_cg_mixed_keep.argtypes = [_c_i64, _i64p, _i32p, _f64p, _f64p, _f64p, _c_dbl, _c_dbl,
                                    _c_int, _c_int, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_c_int),
                                    ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_dbl)]
    L.orc_analytic_u.restype = _c_dbl
    L.orc_analytic_u.argtypes = [_c_dbl, _c_dbl, _c_dbl, _c_int]
    return L


def _opt(a, dtype):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class CSR:
    """CRS matrix of Sec. 3.1 (val, col, ptr with ptr[m] = nnz) plus b."""

    def __init__(self, ptr, col, val, b):
        self.ptr, self.col, self.val, self.b = ptr, col, val, b

    @property
    def m(self):
        return len(self.ptr) - 1

    @property
    def nnz(self):
        return int(self.ptr[-1])

    def dense(self):
        A = np.zeros((self.m, self.m))
        rows = np.repeat(np.arange(self.m), np.diff(self.ptr))
        A[rows, self.col] = self.val
        return A


def num_rows(Nx, Ny, Nz):
    """Nodes of the Nx x Ny x Nz box mesh (Sec. 1 problem statement)."""
    return int(lib().orc_num_rows(Nx, Ny, Nz))


def count_nnz(Nx, Ny, Nz):
    """Stored entries from running the Fig 3.6 neighbour loop."""
    return int(lib().orc_count_nnz(Nx, Ny, Nz))


def boundary(Nx, Ny, Nz, face_vals=None, node_g=None):
    """Dirichlet flag and value per node (Sec. 1 boundary conditions)."""
    m = num_rows(Nx, Ny, Nz)
    fv, fvp = _opt(face_vals, np.float64)
    ng, ngp = _opt(node_g, np.float64)
    d = np.zeros(m, np.uint8)
    g = np.zeros(m, np.float64)
    lib().orc_boundary(Nx, Ny, Nz, fvp, ngp, d, g)
    return d.astype(bool), g


def element_matrix(hx, hy, hz):
    """8x8 trilinear brick stiffness by 2x2x2 Gauss quadrature (Sec. 1)."""
    K = np.zeros(64)
    lib().orc_element_matrix(hx, hy, hz, K)
    return K.reshape(8, 8)


def assemble(Nx, Ny, Nz, face_vals=None, node_g=None, apply_bc=True):
    """CRS matrix and right-hand side (Sec. 1 assembly, Figs 3.6/3.7)."""
    m = num_rows(Nx, Ny, Nz)
    nnz = count_nnz(Nx, Ny, Nz)
    ptr = np.zeros(m + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    b = np.zeros(m, np.float64)
    fv, fvp = _opt(face_vals, np.float64)
    ng, ngp = _opt(node_g, np.float64)
    st = lib().orc_assemble(Nx, Ny, Nz, fvp, ngp, int(bool(apply_bc)), ptr, col, val, b)
    if st != OK:
        raise ValueError(f"orc_assemble failed with status {st}")
    return CSR(ptr, col, val, b)


def assemble_rows(Nx, Ny, Nz, rows, face_vals=None, node_g=None):
    """Selected rows of the assembled system, built one at a time (same
    arithmetic as assemble()).  Returns a list of (cols, vals) and b[rows]."""
    rows = np.ascontiguousarray(rows, np.int64)
    n = len(rows)
    cols = np.zeros(27 * n, np.int32)
    vals = np.zeros(27 * n, np.float64)
    cnt = np.zeros(n, np.int32)
    b = np.zeros(n, np.float64)
    fv, fvp = _opt(face_vals, np.float64)
    ng, ngp = _opt(node_g, np.float64)
    st = lib().orc_assemble_rows(Nx, Ny, Nz, fvp, ngp, n, rows, cols, vals, cnt, b)
    if st != OK:
        raise ValueError(f"orc_assemble_rows failed with status {st}")
    out = [(cols[27 * r:27 * r + cnt[r]].copy(), vals[27 * r:27 * r + cnt[r]].copy()) for r in range(n)]
    return out, b


def csr_spmv(A, x, library=None):
    """y = A x over CRS, summed in ascending column order (Fig 3.1).
    library: a timing build (load_timing_build) instead of the oracle's own."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(A.m)
    (library or lib()).orc_csr_spmv(A.m, A.ptr, A.col, A.val, x, y)
    return y


def bcrsvar(A):
    """1xn variable BCRS of Sec. 3.1: (jas, offsets, ptr); val is A.val."""
    L = lib()
    nns = int(L.orc_bcrsvar_count(A.m, A.ptr, A.col))
    jas = np.zeros(nns, np.int32)
    offs = np.zeros(nns + 1, np.int64)
    bptr = np.zeros(A.m + 1, np.int64)
    L.orc_bcrsvar_build(A.m, A.ptr, A.col, jas, offs, bptr)
    return jas, offs, bptr


def bcrsvar_spmv(A, fmt, x, switch=False):
    """BCRS SpMV of Fig 3.2, or its length-switch form of Fig 3.3."""
    jas, offs, bptr = fmt
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(A.m)
    fn = lib().orc_bcrsvar_spmv_switch if switch else lib().orc_bcrsvar_spmv
    fn(A.m, bptr, jas, offs, A.val, x, y)
    return y


def bcrs13(A):
    """Fixed 1x3 zero-padded blocks (segment format with n = 3): (bptr, bcol, bval)."""
    L = lib()
    nb = int(L.orc_bcrs13_build(A.m, A.ptr, A.col, None, None, None, None))
    bptr = np.zeros(A.m + 1, np.int64)
    bcol = np.zeros(nb, np.int32)
    bval = np.zeros(3 * nb, np.float64)
    v = np.ascontiguousarray(A.val)
    L.orc_bcrs13_build(A.m, A.ptr, A.col, v.ctypes.data_as(ctypes.c_void_p),
                       bptr.ctypes.data_as(ctypes.c_void_p), bcol.ctypes.data_as(ctypes.c_void_p),
                       bval.ctypes.data_as(ctypes.c_void_p))
    return bptr, bcol, bval


def bcrs13_spmv(A, fmt, x, library=None):
    """y = A x over the 1x3 blocks of bcrs13(A), each block's three products
    in column order (Figs 3.2/3.3 with n = 3).  library: a timing build
    (load_timing_build) instead of the oracle's own."""
    bptr, bcol, bval = fmt
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(A.m)
    (library or lib()).orc_bcrs13_spmv(A.m, bptr, bcol, bval, x, y)
    return y


def cg(A, b=None, x0=None, tol=1e-8, max_iter=200, history=False, library=None):
    """Unpreconditioned CG (Sec. 1 CG module).  Returns a dict with x,
    status, iterations, recurrence and true relative residuals and, when
    asked, the residual history ||r_k||/||b||, k = 0..iterations.  library:
    a timing build (load_timing_build) instead of the oracle's own."""
    b = A.b if b is None else np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.m) if x0 is None else np.array(x0, np.float64, copy=True)
    its, rr, rt = _c_int(0), _c_dbl(0), _c_dbl(0)
    hist = np.zeros(max_iter + 1) if history else None
    hp = hist.ctypes.data_as(ctypes.c_void_p) if history else None
    st = (library or lib()).orc_cg(A.m, A.ptr, A.col, A.val, b, x, tol, max_iter,
                      ctypes.byref(its), ctypes.byref(rr), ctypes.byref(rt), hp)
    out = dict(x=x, status=st, iterations=its.value, rel_res_rec=rr.value, rel_res_true=rt.value)
    if history:
        out["history"] = hist[: its.value + 1]
    return out


def cg_single_reduction(A, b=None, x0=None, tol=1e-8, max_iter=200, history=False):
    """Single-reduction (Chronopoulos-Gear) CG: both dot products of an
    iteration taken after its one SpMV.  Same outputs as cg()."""
    b = A.b if b is None else np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.m) if x0 is None else np.array(x0, np.float64, copy=True)
    its, rr, rt = _c_int(0), _c_dbl(0), _c_dbl(0)
    hist = np.zeros(max_iter + 1) if history else None
    hp = hist.ctypes.data_as(ctypes.c_void_p) if history else None
    st = lib().orc_cg_single_reduction(A.m, A.ptr, A.col, A.val, b, x, tol, max_iter,
                                       ctypes.byref(its), ctypes.byref(rr), ctypes.byref(rt), hp)
    out = dict(x=x, status=st, iterations=its.value, rel_res_rec=rr.value, rel_res_true=rt.value)
    if history:
        out["history"] = hist[: its.value + 1]
    return out


def cg_jacobi(A, b=None, x0=None, tol=1e-8, max_iter=200, history=False):
    """Jacobi-preconditioned CG (M = diag(A)), stopping on ||r||/||b|| as
    cg() does.  Same outputs as cg()."""
    b = A.b if b is None else np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.m) if x0 is None else np.array(x0, np.float64, copy=True)
    its, rr, rt = _c_int(0), _c_dbl(0), _c_dbl(0)
    hist = np.zeros(max_iter + 1) if history else None
    hp = hist.ctypes.data_as(ctypes.c_void_p) if history else None
    st = lib().orc_cg_jacobi(A.m, A.ptr, A.col, A.val, b, x, tol, max_iter,
                             ctypes.byref(its), ctypes.byref(rr), ctypes.byref(rt), hp)
    out = dict(x=x, status=st, iterations=its.value, rel_res_rec=rr.value, rel_res_true=rt.value)
    if history:
        out["history"] = hist[: its.value + 1]
    return out


def cg_mixed(A, b=None, x0=None, tol=1e-10, inner_tol=1e-4, max_outer=50, max_inner=500,
             keep_direction=False, inner_f32=True, emulated=False, safeguards=False):
    """FP32-inner CG inside FP64 iterative refinement (mixed-precision
    extension).  keep_direction: the inner CG goes on from its last direction
    after each refinement step (orc_cg_mixed_keep); inner_f32=False runs the
    inner steps in FP64; emulated forces orc_cg_mixed_keep (FP32 emulated in
    FP64 arithmetic) for the restarting form too; safeguards adds the
    last-step inner tolerance and the FP64 CG fallback on stagnation
    (orc_cg_mixed_keep's adaptive and fallback)."""
    b = A.b if b is None else np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.m) if x0 is None else np.array(x0, np.float64, copy=True)
    outer, inner, fb, rt = _c_int(0), _c_int(0), _c_int(0), _c_dbl(0)
    if keep_direction or not inner_f32 or emulated or safeguards:
        sg = int(bool(safeguards))
        st = lib().orc_cg_mixed_keep(A.m, A.ptr, A.col, A.val, b, x, tol, inner_tol, max_outer, max_inner,
                                     int(bool(keep_direction)), int(bool(inner_f32)), sg, sg,
                                     ctypes.byref(outer), ctypes.byref(inner), ctypes.byref(fb), ctypes.byref(rt))
    else:
        st = lib().orc_cg_mixed(A.m, A.ptr, A.col, A.val, b, x, tol, inner_tol, max_outer, max_inner,
                                ctypes.byref(outer), ctypes.byref(inner), ctypes.byref(rt))
    return dict(x=x, status=st, outer=outer.value, inner_iterations=inner.value,
                fallback_iterations=fb.value, rel_res_true=rt.value)


def analytic_u(x, y, z, max_pq=4001):
    """Series solution for u=1 on x=1, 0 elsewhere (Sec. 1 verification)."""
    return float(lib().orc_analytic_u(float(x), float(y), float(z), int(max_pq)))
