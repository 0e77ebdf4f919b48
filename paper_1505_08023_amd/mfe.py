"""Thin Python layer over the C ABI: PyTorch supplies device memory and the stream.

Nothing here computes: every step runs in the HIP kernels of libmfe.so.  The
classes only turn torch tensors into device pointers and status codes into
exceptions.
"""
import atexit
import contextlib
import ctypes
import sys
import weakref

import torch

from . import _lib
from ._lib import (MFE_BCRS13, MFE_CSR, MFE_F32, MFE_F64, MFE_NOT_CONVERGED, MFE_OK, MFE_EBREAKDOWN,
                   check, mfe_cg_stats)

FORMATS = {"csr": MFE_CSR, "bcrs13": MFE_BCRS13}


def _fmt(fmt):
    return FORMATS[fmt] if isinstance(fmt, str) else int(fmt)


def _ptr(t, dtype, n=None, name="tensor"):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


_LIVE = weakref.WeakSet()  # contexts and problems still holding library objects


@atexit.register
def _close_all():
    """Release library objects while torch (which owns their memory) is alive."""
    objs = list(_LIVE)
    for o in objs:
        if isinstance(o, (Problem, Batch, Net)):
            o.close()
    for o in objs:
        if isinstance(o, Context):
            o.close()


@contextlib.contextmanager
def _on(ctx):
    """Order library work on ctx.stream after the caller's current stream, and
    the caller's later work after it (the library stream is non-blocking)."""
    cur = torch.cuda.current_stream(ctx.device)
    same = cur == ctx.stream
    if not same:
        ctx.stream.wait_stream(cur)
    with torch.cuda.stream(ctx.stream):
        yield
    if not same:
        cur.wait_stream(ctx.stream)


class _TorchAllocator:
    """Device memory for the library's own storage, taken from torch's caching allocator."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.alloc_cb = _lib.mfe_alloc_fn(self._alloc)
        self.free_cb = _lib.mfe_free_fn(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


class Context:
    """One device and one stream.  All work of its problems is ordered on `stream`."""

    def __init__(self, device=0, stream=None, torch_memory=True):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._allocator = _TorchAllocator(self.device) if torch_memory else None
        h = ctypes.c_void_p()
        a = self._allocator
        check(self.lib.mfe_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                      a.alloc_cb if a else _lib.mfe_alloc_fn(),
                                      a.free_cb if a else _lib.mfe_free_fn(), None, ctypes.byref(h)),
              "mfe_ctx_create")
        self.handle = h
        self.problems = weakref.WeakSet()
        _LIVE.add(self)

    def dot(self, x, y):
        n = x.numel()
        out = ctypes.c_double()
        with _on(self):
            check(self.lib.mfe_dot(self.handle, n, _ptr(x, torch.float64, n, "x"),
                                   _ptr(y, torch.float64, n, "y"), ctypes.byref(out)), "mfe_dot")
        return out.value

    def stream_probe(self, kind, src, dst, events=None):
        """Bandwidth probe (mfe_stream_probe): kind "copy" writes src into dst,
        kind "read" reads src and writes per-workgroup sums to dst (>= 4096
        doubles).  events = (before, after) torch.cuda.Event pair recorded
        around the kernel on the library's stream."""
        n = src.numel()
        k = {"copy": 0, "read": 1}[kind]
        ev = (None, None)
        if events is not None:
            for e in events:  # materialise the HIP event handles on this stream
                if not e.cuda_event:
                    e.record(self.stream)
            ev = (ctypes.c_void_p(events[0].cuda_event), ctypes.c_void_p(events[1].cuda_event))
        if dst.numel() < (n if k == 0 else 4096):
            raise ValueError("dst too small for the probe")
        with _on(self):
            check(self.lib.mfe_stream_probe(self.handle, k, n, _ptr(src, torch.float64, n, "src"),
                                            _ptr(dst, torch.float64, None, "dst"), ev[0], ev[1]),
                  "mfe_stream_probe")

    def prolong(self, xc, coarse, factor, bnd=None, xf=None):
        """Trilinear prolongation of nodal values xc of the coarse (Nx, Ny, Nz)
        element mesh to the mesh refined factor times (mfe_prolong_trilinear);
        bnd: values for the fine boundary nodes (e.g. the fine problem's b)."""
        Nx, Ny, Nz = coarse
        mc = (Nx + 1) * (Ny + 1) * (Nz + 1)
        mf = (Nx * factor + 1) * (Ny * factor + 1) * (Nz * factor + 1)
        if xf is None:
            with _on(self):
                xf = torch.empty(mf, dtype=torch.float64, device=self.device)
        with _on(self):
            check(self.lib.mfe_prolong_trilinear(self.handle, Nx, Ny, Nz, _ptr(xc, torch.float64, mc, "xc"), factor,
                                                 _ptr(bnd, torch.float64, mf, "bnd"), _ptr(xf, torch.float64, mf, "xf")),
                  "mfe_prolong_trilinear")
        return xf

    def close(self):
        if self.handle:
            for p in list(self.problems):
                p.close()
            self.stream.synchronize()
            self.lib.mfe_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """An assembled system A x = b held by the library (CSR, optionally 1x3 BCRS, FP64/FP32)."""

    def __init__(self, ctx, handle, mesh=None):
        self.ctx, self.handle, self.mesh = ctx, handle, mesh
        m, nnz, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(ctx.lib.mfe_problem_info(handle, ctypes.byref(m), ctypes.byref(nnz), ctypes.byref(nb)),
              "mfe_problem_info")
        self.m, self.nnz, self.nblocks = m.value, nnz.value, nb.value
        v = [ctypes.c_int64() for _ in range(4)]
        check(ctx.lib.mfe_problem_bcrs13_layout(handle, *[ctypes.byref(t) for t in v]), "mfe_problem_bcrs13_layout")
        # 1x3 BCRS storage: slices, slot rows, slices with descriptor-formed
        # column indices and their real blocks (zeros without 1x3 BCRS)
        self.b13_layout = dict(zip(("slices", "slots", "compressed_slices", "compressed_blocks"),
                                   (t.value for t in v)))
        v = [ctypes.c_int64() for _ in range(3)]
        check(ctx.lib.mfe_problem_csr_layout(handle, *[ctypes.byref(t) for t in v]), "mfe_problem_csr_layout")
        # CRS wavefront tiles: rows per tile, tiles, tiles with descriptor-formed column indices
        self.csr_layout = dict(zip(("tile_rows", "tiles", "compressed_tiles"), (t.value for t in v)))
        v = [ctypes.c_int64() for _ in range(4)]
        check(ctx.lib.mfe_problem_csr_groups(handle, *[ctypes.byref(t) for t in v]), "mfe_problem_csr_groups")
        # CRS group walk of a mesh problem (zeros: the tiles above are walked)
        self.csr_layout.update(zip(("items", "groups", "group_rows", "other_rows"), (t.value for t in v)))
        ctx.problems.add(self)
        _LIVE.add(self)

    @classmethod
    def mesh(cls, ctx, Nx, Ny, Nz, face_vals=None, node_g=None, formats=("csr", "bcrs13"),
             precisions=("f64",)):
        fl = 0
        for f in formats:
            fl |= _fmt(f)
        pr = 0
        for p in precisions:
            pr |= {"f64": MFE_F64, "f32": MFE_F32}[p]
        fv = None
        if face_vals is not None:
            fv = (ctypes.c_double * 6)(*[float(v) for v in face_vals])
        m = (Nx + 1) * (Ny + 1) * (Nz + 1)
        h = ctypes.c_void_p()
        with _on(ctx):
            check(ctx.lib.mfe_problem_create(ctx.handle, Nx, Ny, Nz, fv, _ptr(node_g, torch.float64, m, "node_g"),
                                             fl, pr, ctypes.byref(h)), "mfe_problem_create")
        return cls(ctx, h, mesh=(Nx, Ny, Nz))

    @classmethod
    def from_csr(cls, ctx, ptr, col, val, b=None, formats=("csr",), precisions=("f64",)):
        fl = 0
        for f in formats:
            fl |= _fmt(f)
        pr = 0
        for p in precisions:
            pr |= {"f64": MFE_F64, "f32": MFE_F32}[p]
        m = ptr.numel() - 1
        h = ctypes.c_void_p()
        with _on(ctx):
            check(ctx.lib.mfe_problem_from_csr(ctx.handle, m, _ptr(ptr, torch.int32, None, "ptr"),
                                               _ptr(col, torch.int32, None, "col"),
                                               _ptr(val, torch.float64, None, "val"),
                                               _ptr(b, torch.float64, m, "b"), fl, pr, ctypes.byref(h)),
                  "mfe_problem_from_csr")
        return cls(ctx, h)

    @classmethod
    def from_csr_host(cls, ctx, ptr, col, val, b=None, formats=("csr",), precisions=("f64",)):
        """A generic CRS problem from host (numpy) arrays (mfe_problem_from_csr_host)."""
        import numpy as np
        fl = 0
        for f in formats:
            fl |= _fmt(f)
        pr = 0
        for p in precisions:
            pr |= {"f64": MFE_F64, "f32": MFE_F32}[p]
        ptr = np.ascontiguousarray(ptr, dtype=np.int32)
        m = ptr.size - 1
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        if col.size < ptr[-1] or val.size < ptr[-1]:
            raise ValueError("col and val must hold ptr[m] entries")
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        if bb is not None and bb.size != m:
            raise ValueError(f"b must have {m} entries")
        h = ctypes.c_void_p()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        with _on(ctx):
            check(ctx.lib.mfe_problem_from_csr_host(ctx.handle, m, vp(ptr), vp(col), vp(val),
                                                    vp(bb) if bb is not None else None, fl, pr, ctypes.byref(h)),
                  "mfe_problem_from_csr_host")
        return cls(ctx, h)

    def export_csr_host(self):
        """(ptr, col, val, b) as numpy arrays (mfe_problem_export_csr_host)."""
        import numpy as np
        ptr = np.empty(self.m + 1, np.int32)
        col = np.empty(self.nnz, np.int32)
        val = np.empty(self.nnz, np.float64)
        b = np.empty(self.m, np.float64)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_problem_export_csr_host(self.handle, vp(ptr), vp(col), vp(val), vp(b)),
                  "mfe_problem_export_csr_host")
        return ptr, col, val, b

    def rhs(self, b=None):
        """The right-hand side b (mfe_rhs) into a device tensor."""
        if b is None:
            with _on(self.ctx):
                b = torch.empty(self.m, dtype=torch.float64, device=self.ctx.device)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_rhs(self.handle, _ptr(b, torch.float64, self.m, "b")), "mfe_rhs")
        return b

    # -- data out -------------------------------------------------------------------------
    def export_csr(self):
        d = self.ctx.device
        ptr = torch.empty(self.m + 1, dtype=torch.int32, device=d)
        col = torch.empty(self.nnz, dtype=torch.int32, device=d)
        val = torch.empty(self.nnz, dtype=torch.float64, device=d)
        b = torch.empty(self.m, dtype=torch.float64, device=d)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_problem_export_csr(self.handle, _ptr(ptr, torch.int32), _ptr(col, torch.int32),
                                                      _ptr(val, torch.float64), _ptr(b, torch.float64)),
                  "mfe_problem_export_csr")
        self.ctx.stream.synchronize()
        return ptr, col, val, b

    def export_bcrs13(self):
        d = self.ctx.device
        bptr = torch.empty(self.m + 1, dtype=torch.int32, device=d)
        bcol = torch.empty(self.nblocks, dtype=torch.int32, device=d)
        bval = torch.empty(3 * self.nblocks, dtype=torch.float64, device=d)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_problem_export_bcrs13(self.handle, _ptr(bptr, torch.int32),
                                                         _ptr(bcol, torch.int32), _ptr(bval, torch.float64)),
                  "mfe_problem_export_bcrs13")
        self.ctx.stream.synchronize()
        return bptr, bcol, bval

    def set_bc(self, face_vals=None, node_g=None):
        fv = None if face_vals is None else (ctypes.c_double * 6)(*[float(v) for v in face_vals])
        with _on(self.ctx):
            check(self.ctx.lib.mfe_problem_set_bc(self.handle, fv, _ptr(node_g, torch.float64, self.m, "node_g")),
                  "mfe_problem_set_bc")

    # -- operations -----------------------------------------------------------------------
    def spmv(self, x, y=None, fmt="bcrs13"):
        if y is None:
            y = torch.empty_like(x)
        if x.dtype == torch.float32:
            fn, dt, name = self.ctx.lib.mfe_spmv_f32, torch.float32, "mfe_spmv_f32"
        else:
            fn, dt, name = self.ctx.lib.mfe_spmv, torch.float64, "mfe_spmv"
        with _on(self.ctx):
            check(fn(self.handle, _fmt(fmt), _ptr(x, dt, self.m, "x"), _ptr(y, dt, self.m, "y")), name)
        return y

    def spmv_dot(self, p, q=None, pq=None, fmt="bcrs13", events=None):
        """q = A p and p.q (into the device scalar pq) by the fused CG kernel,
        in FP64, or in FP32 (mfe_spmv_dot_f32) when p is a float32 tensor.
        events = (before, after) torch.cuda.Event pair recorded around the kernel."""
        f32 = p.dtype == torch.float32
        dt = torch.float32 if f32 else torch.float64
        if q is None:
            q = torch.empty_like(p)
        if pq is None:
            pq = torch.zeros(1, dtype=torch.float64, device=p.device)
        ev = (None, None)
        if events is not None:
            for e in events:  # materialise the HIP event handles on this stream
                if not e.cuda_event:
                    e.record(self.ctx.stream)
            ev = (ctypes.c_void_p(events[0].cuda_event), ctypes.c_void_p(events[1].cuda_event))
        name = "mfe_spmv_dot_f32" if f32 else "mfe_spmv_dot"
        with _on(self.ctx):
            check(getattr(self.ctx.lib, name)(self.handle, _fmt(fmt), _ptr(p, dt, self.m, "p"), _ptr(q, dt, self.m, "q"),
                                              _ptr(pq, torch.float64, 1, "pq"), ev[0], ev[1]), name)
        return q, pq

    def spmv_dot_noalloc(self, p, q, pq, fmt="bcrs13"):
        """q = A p and p.q into the device scalar pq (FP64) through
        mfe_spmv_dot_noalloc, which allocates no device memory: the caller
        passes every output."""
        with _on(self.ctx):
            check(self.ctx.lib.mfe_spmv_dot_noalloc(self.handle, _fmt(fmt), _ptr(p, torch.float64, self.m, "p"),
                                                    _ptr(q, torch.float64, self.m, "q"),
                                                    _ptr(pq, torch.float64, 1, "pq")), "mfe_spmv_dot_noalloc")
        return q, pq

    def cg(self, x=None, tol=1e-8, max_iter=200, fmt="bcrs13", history=False, raise_on_breakdown=True,
           warm=False, variant="cg"):
        """Unpreconditioned CG from x (zero if None).  warm=True: x is a guess
        that the solve replaces by zero when ||b - A x|| >= ||b||
        (mfe_cg_warm).  variant="single_reduction": the Chronopoulos-Gear
        form with one reduction point per iteration
        (mfe_cg_single_reduction); variant="jacobi": diagonally
        preconditioned (mfe_cg_jacobi).  Returns (x, stats dict)."""
        d = self.ctx.device
        if x is None:
            with _on(self.ctx):
                x = torch.zeros(self.m, dtype=torch.float64, device=d)
        hist = torch.zeros(max_iter + 1, dtype=torch.float64, device=d) if history else None
        st = mfe_cg_stats()
        names = {"cg": "mfe_cg_warm" if warm else "mfe_cg", "single_reduction": "mfe_cg_single_reduction",
                 "jacobi": "mfe_cg_jacobi"}
        if variant not in names or (warm and variant != "cg"):
            raise ValueError(f"unsupported CG variant {variant!r} (warm={warm})")
        name = names[variant]
        with _on(self.ctx):
            rc = getattr(self.ctx.lib, name)(self.handle, _fmt(fmt), _ptr(x, torch.float64, self.m, "x"),
                                             float(tol), int(max_iter), _ptr(hist, torch.float64),
                                             ctypes.byref(st))
        ok = (MFE_OK, MFE_NOT_CONVERGED) + (() if raise_on_breakdown else (MFE_EBREAKDOWN,))
        check(rc, name, ok)
        out = st.as_dict()
        if history:
            out["history"] = hist[: st.iterations + 1].cpu()
        return x, out

    def verify_series(self, x, x_max=0.75, want_u=False):
        """Nodal error against the series solution of the paper's problem at
        the nodes with x-coordinate <= x_max (mfe_verify_series).  Returns
        dict(max_err, rms_err, count[, u])."""
        u = None
        if want_u:
            with _on(self.ctx):
                u = torch.empty(self.m, dtype=torch.float64, device=self.ctx.device)
        mx, rms, cnt = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        with _on(self.ctx):
            check(self.ctx.lib.mfe_verify_series(self.handle, _ptr(x, torch.float64, self.m, "x"), float(x_max),
                                                 _ptr(u, torch.float64), ctypes.byref(mx), ctypes.byref(rms),
                                                 ctypes.byref(cnt)), "mfe_verify_series")
        out = dict(max_err=mx.value, rms_err=rms.value, count=cnt.value)
        if want_u:
            out["u"] = u
        return out

    def cg_mixed(self, x=None, tol=1e-10, inner_tol=1e-4, max_outer=50, max_inner=2000, fmt="bcrs13",
                 warm=False, keep_direction=False):
        """FP32-inner CG inside FP64 iterative refinement from x (zero if
        None); warm=True rejects a guess no closer than zero
        (mfe_cg_mixed_warm); keep_direction=True lets the inner CG go on
        from its last direction after each refinement step
        (mfe_cg_mixed_ex).  Returns (x, stats dict)."""
        d = self.ctx.device
        if x is None:
            with _on(self.ctx):
                x = torch.zeros(self.m, dtype=torch.float64, device=d)
        st = mfe_cg_stats()
        xp = _ptr(x, torch.float64, self.m, "x")
        with _on(self.ctx):
            if keep_direction:
                name = "mfe_cg_mixed_ex"
                flags = (_lib.MFE_MIXED_WARM if warm else 0) | _lib.MFE_MIXED_KEEP_DIRECTION
                rc = self.ctx.lib.mfe_cg_mixed_ex(self.handle, _fmt(fmt), xp, float(tol), float(inner_tol),
                                                  int(max_outer), int(max_inner), flags, ctypes.byref(st))
            else:
                name = "mfe_cg_mixed_warm" if warm else "mfe_cg_mixed"
                rc = getattr(self.ctx.lib, name)(self.handle, _fmt(fmt), xp, float(tol), float(inner_tol),
                                                 int(max_outer), int(max_inner), ctypes.byref(st))
        check(rc, name, (MFE_OK, MFE_NOT_CONVERGED))
        return x, st.as_dict()

    def close(self):
        if self.handle and self.ctx.handle:
            self.ctx.lib.mfe_problem_destroy(self.handle)
        self.handle = None


class Batch:
    """Many box meshes solved together (block-diagonal storage, per-system CG)."""

    def __init__(self, ctx, sizes, face_vals=None, formats=("csr", "bcrs13"), precisions=("f64",)):
        import numpy as np
        self.ctx = ctx
        sizes = np.ascontiguousarray(sizes, dtype=np.int32).reshape(-1, 3)
        self.nsys = sizes.shape[0]
        fv = None
        if face_vals is not None:
            fv = np.ascontiguousarray(face_vals, dtype=np.float64).reshape(self.nsys, 6)
        fl = 0
        for f in formats:
            fl |= _fmt(f)
        pr = 0
        for p in precisions:
            pr |= {"f64": MFE_F64, "f32": MFE_F32}[p]
        h = ctypes.c_void_p()
        with _on(ctx):
            check(ctx.lib.mfe_batch_create(ctx.handle, self.nsys, sizes.ctypes.data_as(ctypes.c_void_p),
                                           fv.ctypes.data_as(ctypes.c_void_p) if fv is not None else None,
                                           fl, pr, ctypes.byref(h)), "mfe_batch_create")
        self._attach(h)

    @classmethod
    def from_problems(cls, ctx, problems, formats=("csr", "bcrs13"), precisions=("f64",)):
        """A batch of existing problems, copied (mfe_batch_from_problems)."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.nsys = len(problems)
        fl = 0
        for f in formats:
            fl |= _fmt(f)
        pr = 0
        for p in precisions:
            pr |= {"f64": MFE_F64, "f32": MFE_F32}[p]
        arr = (ctypes.c_void_p * self.nsys)(*[p.handle.value for p in problems])
        h = ctypes.c_void_p()
        with _on(ctx):
            check(ctx.lib.mfe_batch_from_problems(ctx.handle, self.nsys, ctypes.cast(arr, ctypes.c_void_p), fl, pr,
                                                  ctypes.byref(h)), "mfe_batch_from_problems")
        self._attach(h)
        return self

    def _attach(self, h):
        import numpy as np
        ctx = self.ctx
        self.handle = h
        m, nnz = ctypes.c_int64(), ctypes.c_int64()
        offs = np.zeros(self.nsys + 1, dtype=np.int64)
        check(ctx.lib.mfe_batch_info(h, ctypes.byref(m), ctypes.byref(nnz), offs.ctypes.data_as(ctypes.c_void_p)),
              "mfe_batch_info")
        self.m, self.nnz, self.row_offsets = m.value, nnz.value, offs
        v = [ctypes.c_int64() for _ in range(4)]
        check(ctx.lib.mfe_batch_bcrs13_layout(h, *[ctypes.byref(t) for t in v]), "mfe_batch_bcrs13_layout")
        self.b13_layout = dict(zip(("slices", "slots", "compressed_slices", "compressed_blocks"),
                                   (t.value for t in v)))
        ctx.problems.add(self)
        _LIVE.add(self)

    def export_csr(self):
        d = self.ctx.device
        ptr = torch.empty(self.m + 1, dtype=torch.int32, device=d)
        col = torch.empty(self.nnz, dtype=torch.int32, device=d)
        val = torch.empty(self.nnz, dtype=torch.float64, device=d)
        b = torch.empty(self.m, dtype=torch.float64, device=d)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_batch_export_csr(self.handle, _ptr(ptr, torch.int32), _ptr(col, torch.int32),
                                                    _ptr(val, torch.float64), _ptr(b, torch.float64)),
                  "mfe_batch_export_csr")
        self.ctx.stream.synchronize()
        return ptr, col, val, b

    def set_bc(self, face_vals=None, node_g=None):
        import numpy as np
        fv = None if face_vals is None else np.ascontiguousarray(face_vals, dtype=np.float64).reshape(self.nsys, 6)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_batch_set_bc(self.handle, fv.ctypes.data_as(ctypes.c_void_p) if fv is not None else None,
                                                _ptr(node_g, torch.float64, self.m, "node_g")), "mfe_batch_set_bc")

    def autotune(self, fmt="bcrs13"):
        lanes, factor = ctypes.c_int(), ctypes.c_int()
        with _on(self.ctx):
            check(self.ctx.lib.mfe_batch_autotune(self.handle, _fmt(fmt), ctypes.byref(lanes), ctypes.byref(factor)),
                  "mfe_batch_autotune")
        return lanes.value, factor.value

    def _stats(self):
        return (mfe_cg_stats * self.nsys)()

    def cg(self, x=None, tol=1e-8, max_iter=5000, fmt="bcrs13"):
        if x is None:
            with _on(self.ctx):
                x = torch.zeros(self.m, dtype=torch.float64, device=self.ctx.device)
        st = self._stats()
        with _on(self.ctx):
            rc = self.ctx.lib.mfe_batch_cg(self.handle, _fmt(fmt), _ptr(x, torch.float64, self.m, "x"), float(tol),
                                           int(max_iter), ctypes.cast(st, ctypes.c_void_p))
        check(rc, "mfe_batch_cg", (MFE_OK, MFE_NOT_CONVERGED))
        return x, [s.as_dict() for s in st]

    def cg_mixed(self, x=None, tol=1e-8, inner_tol=1e-4, max_outer=50, max_inner=2000, fmt="bcrs13",
                 keep_direction=False):
        if x is None:
            with _on(self.ctx):
                x = torch.zeros(self.m, dtype=torch.float64, device=self.ctx.device)
        st = self._stats()
        flags = _lib.MFE_MIXED_KEEP_DIRECTION if keep_direction else 0
        with _on(self.ctx):
            rc = self.ctx.lib.mfe_batch_cg_mixed_ex(self.handle, _fmt(fmt), _ptr(x, torch.float64, self.m, "x"),
                                                    float(tol), float(inner_tol), int(max_outer), int(max_inner),
                                                    flags, ctypes.cast(st, ctypes.c_void_p))
        check(rc, "mfe_batch_cg_mixed_ex", (MFE_OK, MFE_NOT_CONVERGED))
        return x, [s.as_dict() for s in st]

    def close(self):
        if self.handle and self.ctx.handle:
            self.ctx.lib.mfe_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def cg_batched(ctx, problems, xs=None, tol=1e-8, max_iter=5000, fmt="bcrs13", mixed=False):
    """One batched solve of existing problems (mfe_cg_batched): xs is a list
    of FP64 device vectors (x0 in, solution out; zeros if None).  Returns
    (xs, list of stats dicts)."""
    n = len(problems)
    if xs is None:
        with _on(ctx):
            xs = [torch.zeros(p.m, dtype=torch.float64, device=ctx.device) for p in problems]
    ptrs = (ctypes.c_void_p * n)(*[_ptr(x, torch.float64, p.m, "x").value for x, p in zip(xs, problems)])
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    st = (mfe_cg_stats * n)()
    with _on(ctx):
        rc = ctx.lib.mfe_cg_batched(ctx.handle, n, ctypes.cast(hs, ctypes.c_void_p), _fmt(fmt),
                                    ctypes.cast(ptrs, ctypes.c_void_p), float(tol), int(max_iter), int(bool(mixed)),
                                    ctypes.cast(st, ctypes.c_void_p))
    check(rc, "mfe_cg_batched", (MFE_OK, MFE_NOT_CONVERGED))
    return xs, [s.as_dict() for s in st]


CONV_MODES = {"s1": 0, "s2": 1, "t2": 2}


def conv3d(ctx, mode, x, w, bias=None, relu=False, out32=False):
    """One 3x3x3 convolution on the matrix cores.  x: bf16 CUDA tensor
    [batch, G, G, G, cin]; w: FP32 array-like [cout, 27, cin]."""
    import numpy as np
    if x.dtype != torch.bfloat16 or not x.is_contiguous() or x.dim() != 5:
        raise ValueError("x must be a contiguous bf16 tensor [batch, G, G, G, cin]")
    b, G, cin = x.shape[0], x.shape[1], x.shape[4]
    w = np.ascontiguousarray(w, dtype=np.float32)
    cout = w.shape[0]
    Go = {"s1": G, "s2": (G - 1) // 2 + 1, "t2": 2 * (G - 1) + 1}[mode]
    y = torch.empty((b, Go, Go, Go, cout), dtype=torch.bfloat16, device=x.device)
    y32 = torch.empty((b, Go, Go, Go, cout), dtype=torch.float32, device=x.device) if out32 else None
    bh = None if bias is None else np.ascontiguousarray(bias, dtype=np.float32)
    with _on(ctx):
        check(ctx.lib.mfe_conv3d_bf16(ctx.handle, CONV_MODES[mode], b, G, cin, ctypes.c_void_p(x.data_ptr()), cout,
                                      w.ctypes.data_as(ctypes.c_void_p),
                                      bh.ctypes.data_as(ctypes.c_void_p) if bh is not None else None, int(relu),
                                      ctypes.c_void_p(y.data_ptr()),
                                      ctypes.c_void_p(y32.data_ptr()) if y32 is not None else None), "mfe_conv3d_bf16")
    return (y, y32) if out32 else y


def conv3d_dgrad(ctx, mode, gy, w, G_in, gx=None, accumulate=False, out32=False):
    """Input gradient of conv3d(mode) on a G_in grid for output gradient gy
    (bf16 [batch, Go, Go, Go, cout]); w: FP32 [cout, 27, cin].  Returns gx
    (bf16 [batch, G_in, G_in, G_in, cin]; with accumulate, gx += the
    gradient) and, when asked, the FP32 sum before rounding."""
    import numpy as np
    if gy.dtype != torch.bfloat16 or not gy.is_contiguous() or gy.dim() != 5:
        raise ValueError("gy must be a contiguous bf16 tensor [batch, Go, Go, Go, cout]")
    w = np.ascontiguousarray(w, dtype=np.float32)
    b, cout, cin = gy.shape[0], gy.shape[4], w.shape[2]
    if gx is None:
        if accumulate:
            raise ValueError("accumulate needs gx")
        gx = torch.empty((b, G_in, G_in, G_in, cin), dtype=torch.bfloat16, device=gy.device)
    elif tuple(gx.shape) != (b, G_in, G_in, G_in, cin) or gx.dtype != torch.bfloat16 or not gx.is_contiguous():
        raise ValueError("gx must be a contiguous bf16 tensor [batch, G_in, G_in, G_in, cin]")
    gx32 = torch.empty((b, G_in, G_in, G_in, cin), dtype=torch.float32, device=gy.device) if out32 else None
    with _on(ctx):
        check(ctx.lib.mfe_conv3d_dgrad_bf16(ctx.handle, CONV_MODES[mode], b, G_in, cin, ctypes.c_void_p(gy.data_ptr()),
                                            cout, w.ctypes.data_as(ctypes.c_void_p), int(bool(accumulate)),
                                            ctypes.c_void_p(gx.data_ptr()),
                                            ctypes.c_void_p(gx32.data_ptr()) if gx32 is not None else None),
              "mfe_conv3d_dgrad_bf16")
    return (gx, gx32) if out32 else gx


def conv3d_wgrad(ctx, mode, x, gy):
    """Weight gradient [cout, 27, cin] (numpy FP32) of conv3d(mode, x) for output gradient gy."""
    import numpy as np
    b, G, cin = x.shape[0], x.shape[1], x.shape[4]
    cout = gy.shape[4]
    dw = np.zeros((cout, 27, cin), dtype=np.float32)
    with _on(ctx):
        check(ctx.lib.mfe_conv3d_wgrad_bf16(ctx.handle, CONV_MODES[mode], b, G, cin, ctypes.c_void_p(x.data_ptr()),
                                            cout, ctypes.c_void_p(gy.data_ptr()), dw.ctypes.data_as(ctypes.c_void_p)),
              "mfe_conv3d_wgrad_bf16")
    return dw


class Net:
    """The encoder-decoder that predicts the CG initial guess (include/mfe.h)."""

    def __init__(self, ctx, G, batch_max):
        self.ctx, self.G, self.batch_max = ctx, G, batch_max
        h = ctypes.c_void_p()
        with _on(ctx):
            check(ctx.lib.mfe_net_create(ctx.handle, G, batch_max, ctypes.byref(h)), "mfe_net_create")
        self.handle = h
        n = ctypes.c_int64()
        check(ctx.lib.mfe_net_num_params(h, ctypes.byref(n)), "mfe_net_num_params")
        self.nparams = n.value
        ctx.problems.add(self)
        _LIVE.add(self)

    def set_params(self, flat):
        import numpy as np
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.nparams
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_set_params(self.handle, flat.ctypes.data_as(ctypes.c_void_p)),
                  "mfe_net_set_params")

    def get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)),
                  "mfe_net_get_params")
        return out

    def forward(self, g):
        b = g.numel() // self.G ** 3
        pred = torch.empty(g.numel(), dtype=torch.float32, device=g.device)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_forward(self.handle, b, _ptr(g, torch.float64), _ptr(pred, torch.float32)),
                  "mfe_net_forward")
        return pred

    def loss_grad(self, g, target, want_grad=False, energy=None, fmt="bcrs13"):
        """Forward, loss and backward (the gradient is kept for adam_step).
        energy=None: mean squared error over interior nodes; energy=a Problem
        (the (G-1)^3 mesh): the error's energy norm e^T A e per interior node."""
        import numpy as np
        b = g.numel() // self.G ** 3
        loss = ctypes.c_double()
        grad = np.zeros(self.nparams, dtype=np.float32) if want_grad else None
        gp = grad.ctypes.data_as(ctypes.c_void_p) if want_grad else None
        with _on(self.ctx):
            if energy is None:
                check(self.ctx.lib.mfe_net_loss_grad(self.handle, b, _ptr(g, torch.float64),
                                                     _ptr(target, torch.float64), ctypes.byref(loss), gp),
                      "mfe_net_loss_grad")
            else:
                check(self.ctx.lib.mfe_net_loss_grad_energy(self.handle, energy.handle, FORMATS[fmt], b,
                                                            _ptr(g, torch.float64), _ptr(target, torch.float64),
                                                            ctypes.byref(loss), gp),
                      "mfe_net_loss_grad_energy")
        return (loss.value, grad) if want_grad else loss.value

    def set_grad(self, flat):
        """Replace the gradient the next adam_step applies (FP32, natural layout)."""
        import numpy as np
        g = np.ascontiguousarray(flat, dtype=np.float32)
        if g.size != self.nparams:
            raise ValueError(f"expected {self.nparams} gradient entries, got {g.size}")
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_set_grad(self.handle, g.ctypes.data_as(ctypes.c_void_p)), "mfe_net_set_grad")

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_adam_step(self.handle, lr, beta1, beta2, eps), "mfe_net_adam_step")

    def predict_x0(self, g, x0=None):
        n = self.G ** 3
        if x0 is None:
            x0 = torch.empty_like(g)
        with _on(self.ctx):
            check(self.ctx.lib.mfe_net_predict_x0(self.handle, _ptr(g, torch.float64, n, "g"),
                                                  _ptr(x0, torch.float64, n, "x0")), "mfe_net_predict_x0")
        return x0

    def close(self):
        if self.handle and self.ctx.handle:
            self.ctx.lib.mfe_net_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
