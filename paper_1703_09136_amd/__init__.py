"""Python binding of the MI355X layered-media heterogeneous FMM (libhfmm.so).

Argument marshalling only: every stage of the matvec runs in the HIP library.
PyTorch provides device memory and the current stream. The library must have
been built (``python -m paper_1703_09136_amd.build``); nothing here falls back
to another implementation.

Entry points mirror the C interface (include/hfmm.h):
  Plan(k, interfaces, points, tol, ...)   -> hfmm_plan
  Plan.apply(q)                           -> hfmm_apply          (u = A q)
  Plan.apply_adjoint(v, q, grad_xy)       -> hfmm_apply_adjoint  (w = A^H v, source-coordinate gradient)
  Plan.info()                             -> hfmm_plan_info
  hfmm_apply_autograd(q, plan, points)    -> autograd: forward A q, backward A^H g and d/d points
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfmm.so")

HFMM_OK = 0
STATUS_NAMES = {0: "HFMM_OK", 1: "HFMM_ERR_INVALID_ARG", 2: "HFMM_ERR_DOMAIN", 3: "HFMM_ERR_UNSUPPORTED",
                4: "HFMM_ERR_NO_MEMORY", 5: "HFMM_ERR_DEVICE", 6: "HFMM_ERR_ACCURACY"}

# every symbol declared in include/hfmm.h
EXPORTS = ("hfmm_default_options", "hfmm_plan", "hfmm_apply", "hfmm_apply_adjoint", "hfmm_plan_info",
           "hfmm_profile_enable", "hfmm_profile_read", "hfmm_stage_name",
           "hfmm_destroy", "hfmm_status_string", "hfmm_last_error_message",
           "hfmm_plan_batch", "hfmm_apply_batch", "hfmm_batch_graph", "hfmm_batch_plan", "hfmm_batch_destroy",
           "hfmm_apply_noalloc", "hfmm_tree_build", "hfmm_tree_counts", "hfmm_tree_copy", "hfmm_tree_destroy",
           "hfmm_bie_solve", "hfmm_transmit", "hfmm_transmit_up", "hfmm_middle_scattered")
NSTAGES = 9
HFMM_FP64, HFMM_FP32, HFMM_BF16 = 0, 1, 2
HFMM_SELF_SCATTERED, HFMM_SELF_NONE = 0, 1
HFMM_TREE_GPU, HFMM_TREE_HOST = 0, 1

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("self_term", ctypes.c_int32), ("interface_refine", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("leaf_kb", ctypes.c_double), ("top_level", ctypes.c_int32), ("max_nrhs", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("order", ctypes.c_int32), ("impedance", ctypes.c_double),
                ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


_TORCH_DELETE = None


def _torch_alloc(nbytes, ctx):
    """Device memory for the library from torch's caching allocator (current
    device and stream); NULL (None) makes the library report HFMM_ERR_NO_MEMORY."""
    global _TORCH_DELETE
    import torch
    _TORCH_DELETE = torch.cuda.caching_allocator_delete
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
    except Exception:
        return None


def _torch_free(ptr, ctx):
    # at interpreter exit torch may be torn down before the last plan: the
    # memory then goes with the process
    if ptr and _TORCH_DELETE is not None:
        try:
            _TORCH_DELETE(int(ptr))
        except Exception:
            pass


# kept for the life of the module: the library holds these function pointers
_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)


class Info(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("order", ctypes.c_int32 * 32), ("boxes", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64), ("image_pairs", ctypes.c_int64),
                ("p2p_pairs", ctypes.c_int64), ("interface_pairs", ctypes.c_int64),
                ("image_tables", ctypes.c_int64), ("flops_m2l", ctypes.c_double),
                ("flops_updown", ctypes.c_double), ("flops_p2p", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("p2p_evals", ctypes.c_int64),
                ("top_level", ctypes.c_int32), ("m2l_tile", ctypes.c_int32),
                ("interface_nodes", ctypes.c_int32), ("interface_leaf_pairs", ctypes.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "order"}
        d["order"] = [int(self.order[i]) for i in range(self.levels)]
        return d


class HFMMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load libhfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError("libhfmm.so is not built: run python -m paper_1703_09136_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.hfmm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.hfmm_default_options.restype = None
    lib.hfmm_plan.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), i64, vp, dbl,
                              ctypes.POINTER(Options), vp]
    lib.hfmm_plan.restype = ctypes.c_int
    lib.hfmm_apply.argtypes = [vp, vp, vp, i32, vp]
    lib.hfmm_apply.restype = ctypes.c_int
    lib.hfmm_apply_noalloc.argtypes = [vp, vp, vp, i32, vp]
    lib.hfmm_apply_noalloc.restype = ctypes.c_int
    lib.hfmm_apply_adjoint.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.hfmm_apply_adjoint.restype = ctypes.c_int
    lib.hfmm_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.hfmm_plan_info.restype = ctypes.c_int
    lib.hfmm_profile_enable.argtypes = [vp, i32]
    lib.hfmm_profile_enable.restype = ctypes.c_int
    lib.hfmm_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.hfmm_profile_read.restype = ctypes.c_int
    lib.hfmm_stage_name.argtypes = [i32]
    lib.hfmm_stage_name.restype = ctypes.c_char_p
    lib.hfmm_destroy.argtypes = [vp]
    lib.hfmm_destroy.restype = None
    lib.hfmm_tree_build.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(dbl), ctypes.POINTER(dbl), i64, vp,
                                    ctypes.POINTER(Options), i32, vp]
    lib.hfmm_tree_build.restype = ctypes.c_int
    lib.hfmm_tree_counts.argtypes = [vp, ctypes.POINTER(i64)]
    lib.hfmm_tree_counts.restype = ctypes.c_int
    lib.hfmm_tree_copy.argtypes = [vp, ctypes.POINTER(dbl), vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hfmm_tree_copy.restype = ctypes.c_int
    lib.hfmm_tree_destroy.argtypes = [vp]
    lib.hfmm_tree_destroy.restype = None
    lib.hfmm_bie_solve.argtypes = [vp, vp, vp, vp, dbl, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
    lib.hfmm_bie_solve.restype = ctypes.c_int
    lib.hfmm_transmit.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), i64, vp, vp, i32, i64, vp, vp, dbl,
                                  vp]
    lib.hfmm_transmit.restype = ctypes.c_int
    lib.hfmm_transmit_up.argtypes = lib.hfmm_transmit.argtypes
    lib.hfmm_transmit_up.restype = ctypes.c_int
    lib.hfmm_middle_scattered.argtypes = [ctypes.POINTER(dbl), ctypes.POINTER(dbl), i64, vp, vp, i32, i64, vp, vp,
                                          dbl, vp]
    lib.hfmm_middle_scattered.restype = ctypes.c_int
    lib.hfmm_status_string.argtypes = [ctypes.c_int]
    lib.hfmm_status_string.restype = ctypes.c_char_p
    lib.hfmm_last_error_message.argtypes = []
    lib.hfmm_last_error_message.restype = ctypes.c_char_p
    pp = ctypes.POINTER(vp)
    lib.hfmm_plan_batch.argtypes = [pp, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i64), pp,
                                    dbl, ctypes.POINTER(Options), vp]
    lib.hfmm_plan_batch.restype = ctypes.c_int
    lib.hfmm_apply_batch.argtypes = [vp, pp, pp, i32, vp]
    lib.hfmm_apply_batch.restype = ctypes.c_int
    lib.hfmm_batch_graph.argtypes = [vp, i32]
    lib.hfmm_batch_graph.restype = ctypes.c_int
    lib.hfmm_batch_plan.argtypes = [vp, i32, pp]
    lib.hfmm_batch_plan.restype = ctypes.c_int
    lib.hfmm_batch_destroy.argtypes = [vp]
    lib.hfmm_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(status):
    if status != HFMM_OK:
        raise HFMMError(status, _lib.hfmm_last_error_message().decode())


def default_options(torch_allocator=False, **kw) -> Options:
    """hfmm_default_options with the given fields changed; torch_allocator
    routes the plan's device memory through torch's caching allocator."""
    lib = load()
    o = Options()
    lib.hfmm_default_options(ctypes.byref(o))
    kinds = dict(Options._fields_)
    for key, val in kw.items():
        if key not in kinds or key in ("alloc", "free", "alloc_ctx", "struct_size"):
            raise TypeError("unknown option %r" % key)
        setattr(o, key, float(val) if kinds[key] is ctypes.c_double else int(val))
    if torch_allocator:
        o.alloc = _TORCH_ALLOC
        o.free = _TORCH_FREE
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _stream_obj(stream):
    import torch
    return stream if stream is not None else torch.cuda.current_stream()


def _as_rhs(t, n, name, device=None):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128):
        raise TypeError("%s must be a complex128 CUDA tensor" % name)
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, the plan on %s" % (name, t.device, device))
    if t.dim() == 1:
        t2 = t.reshape(1, -1)
    elif t.dim() == 2:
        t2 = t
    else:
        raise ValueError("%s must have shape (n,) or (nrhs, n)" % name)
    if t2.shape[1] != n or t2.shape[0] < 1:
        raise ValueError("%s must have shape (nrhs, %d)" % (name, n))
    # a lazily conjugated or negated view holds the unconjugated values in memory
    return t2.resolve_conj().resolve_neg().contiguous()


def _check_out(out, q2, name):
    """An output buffer must match the right-hand sides exactly and not overlap them."""
    import torch
    if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()):
        raise TypeError("%s must be a contiguous complex128 CUDA tensor" % name)
    if out.is_conj() or out.is_neg():
        raise TypeError("%s must not be a conjugated or negated view" % name)
    if out.device != q2.device or tuple(out.shape) not in ((q2.shape[0], q2.shape[1]),) + \
            (((q2.shape[1],),) if q2.shape[0] == 1 else ()):
        raise ValueError("%s must have shape %s on %s" % (name, tuple(q2.shape), q2.device))
    a0, a1 = out.data_ptr(), out.data_ptr() + out.numel() * 16
    b0, b1 = q2.data_ptr(), q2.data_ptr() + q2.numel() * 16
    if a0 < b1 and b0 < a1:
        raise ValueError("%s overlaps the right-hand sides" % name)


def build_tree(k, interfaces, points, builder=HFMM_TREE_GPU, stream=None, **options):
    """The quadtree and interaction lists hfmm_plan builds for these points
    (hfmm_tree_build): a dict of numpy arrays (frame, keys, perm, boxes as
    (nboxes, 12) int32 rows, lev_begin, and the pair lists fv, iv, fu, iu as
    (m, 2) int32) plus the counts. builder: HFMM_TREE_GPU or HFMM_TREE_HOST."""
    import numpy as np
    import torch
    lib = load()
    if not (points.is_cuda and points.dtype == torch.float64 and points.dim() == 2 and points.shape[1] == 2):
        raise TypeError("points must be a float64 CUDA tensor of shape (n, 2)")
    pts = points.contiguous()
    kk = (ctypes.c_double * 1)(float(k[0]))
    ii = (ctypes.c_double * 1)(float(interfaces[0]))
    opts = default_options(**options)
    h = ctypes.c_void_p()
    _check(lib.hfmm_tree_build(ctypes.byref(h), kk, ii, int(pts.shape[0]), ctypes.c_void_p(pts.data_ptr()),
                               ctypes.byref(opts), int(builder), _stream_ptr(stream)))
    try:
        c = (ctypes.c_int64 * 8)()
        _check(lib.hfmm_tree_counts(h, c))
        n, nb, nlev, top, nfv, niv, nfu, niu = (int(v) for v in c)
        out = {"n": n, "boxes_count": nb, "levels": nlev, "top": top,
               "frame": np.zeros(3), "keys": np.zeros(n, np.uint64), "perm": np.zeros(n, np.int32),
               "boxes": np.zeros((nb, 12), np.int32), "lev_begin": np.zeros(nlev + 1, np.int32),
               "fv": np.zeros((nfv, 2), np.int32), "iv": np.zeros((niv, 2), np.int32),
               "fu": np.zeros((nfu, 2), np.int32), "iu": np.zeros((niu, 2), np.int32)}
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
        _check(lib.hfmm_tree_copy(h, out["frame"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ptr(out["keys"]),
                                  ptr(out["perm"]), ptr(out["boxes"]), ptr(out["lev_begin"]), ptr(out["fv"]),
                                  ptr(out["iv"]), ptr(out["fu"]), ptr(out["iu"])))
    finally:
        lib.hfmm_tree_destroy(h)
    return out


def transmit(k, interfaces, src, q, tgt, tol=1e-10, stream=None, up=False):
    """The field below the top interface of top-layer sources (hfmm_transmit):
    u[r, t] = sum_s q[r, s] G(tgt_t, src_s), the middle- and bottom-layer fields
    of Section 2.3; with up=True the reverse pairs, sources below and targets
    in the top layer (hfmm_transmit_up). src, tgt: float64 CUDA tensors (n, 2);
    q: complex128 CUDA, (ns,) or (nrhs, ns). Returns (nt,) or (nrhs, nt)."""
    import torch
    lib = load()
    for name, p in (("src", src), ("tgt", tgt)):
        if not (p.is_cuda and p.dtype == torch.float64 and p.dim() == 2 and p.shape[1] == 2):
            raise TypeError("%s must be a float64 CUDA tensor of shape (n, 2)" % name)
    s2, t2 = src.contiguous(), tgt.contiguous()
    ns, nt = int(s2.shape[0]), int(t2.shape[0])
    q2 = _as_rhs(q, ns, "q", s2.device)
    if t2.device != s2.device:
        raise ValueError("tgt is on %s, src on %s" % (t2.device, s2.device))
    u = torch.empty((q2.shape[0], nt), dtype=torch.complex128, device=s2.device)
    kk = (ctypes.c_double * len(k))(*[float(v) for v in k])
    ii = (ctypes.c_double * max(1, len(interfaces)))(*([float(v) for v in interfaces] or [0.0]))
    fn = lib.hfmm_transmit_up if up else lib.hfmm_transmit
    _check(fn(len(k), kk, ii, ns, ctypes.c_void_p(s2.data_ptr()), ctypes.c_void_p(q2.data_ptr()),
              int(q2.shape[0]), nt, ctypes.c_void_p(t2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
              float(tol), _stream_ptr(stream)))
    return u[0] if q.dim() == 1 else u


def middle_scattered(k, interfaces, src, q, tgt, tol=1e-10, stream=None):
    """The middle layer's scattered field of middle-layer sources
    (hfmm_middle_scattered): u[r, t] = sum_s q[r, s] G^s_22(tgt_t, src_s), three
    layers. src, tgt: float64 CUDA tensors (n, 2); q: complex128 CUDA, (ns,) or
    (nrhs, ns). Returns (nt,) or (nrhs, nt)."""
    import torch
    lib = load()
    if len(k) != 3 or len(interfaces) != 2:
        raise ValueError("the middle layer needs three wavenumbers and two interfaces")
    for name, p in (("src", src), ("tgt", tgt)):
        if not (p.is_cuda and p.dtype == torch.float64 and p.dim() == 2 and p.shape[1] == 2):
            raise TypeError("%s must be a float64 CUDA tensor of shape (n, 2)" % name)
    s2, t2 = src.contiguous(), tgt.contiguous()
    ns, nt = int(s2.shape[0]), int(t2.shape[0])
    q2 = _as_rhs(q, ns, "q", s2.device)
    if t2.device != s2.device:
        raise ValueError("tgt is on %s, src on %s" % (t2.device, s2.device))
    u = torch.empty((q2.shape[0], nt), dtype=torch.complex128, device=s2.device)
    kk = (ctypes.c_double * 3)(*[float(v) for v in k])
    ii = (ctypes.c_double * 2)(*[float(v) for v in interfaces])
    _check(lib.hfmm_middle_scattered(kk, ii, ns, ctypes.c_void_p(s2.data_ptr()), ctypes.c_void_p(q2.data_ptr()),
                                     int(q2.shape[0]), nt, ctypes.c_void_p(t2.data_ptr()),
                                     ctypes.c_void_p(u.data_ptr()), float(tol), _stream_ptr(stream)))
    return u[0] if q.dim() == 1 else u


class Plan:
    """A plan of the heterogeneous FMM for fixed points and medium (hfmm_plan)."""

    def __init__(self, k, interfaces, points, tol=1e-8, stream=None, torch_allocator=True, **options):
        import torch
        lib = load()
        k = [float(v) for v in k]
        interfaces = [float(v) for v in interfaces]
        if not (points.is_cuda and points.dtype == torch.float64 and points.dim() == 2 and points.shape[1] == 2):
            raise TypeError("points must be a float64 CUDA tensor of shape (n, 2)")
        pts = points.contiguous()
        self.n = int(pts.shape[0])
        self.k = tuple(k)
        self.interfaces = tuple(interfaces)
        kk = (ctypes.c_double * len(k))(*k)
        ii = (ctypes.c_double * max(1, len(interfaces)))(*(interfaces or [0.0]))
        opts = default_options(torch_allocator=torch_allocator, **options)
        self.device = pts.device
        h = ctypes.c_void_p()
        _check(lib.hfmm_plan(ctypes.byref(h), len(k), kk, ii, self.n, ctypes.c_void_p(pts.data_ptr()),
                             float(tol), ctypes.byref(opts), _stream_ptr(stream)))
        self._h = h
        self._lib = lib

    def apply(self, q, out=None, stream=None):
        """u = A q for q of shape (n,) or (nrhs, n), complex128 on the GPU."""
        import torch
        q2 = _as_rhs(q, self.n, "q", self.device)
        if out is not None:
            _check_out(out, q2, "out")
        u = out if out is not None else torch.empty_like(q2)
        _check(self._lib.hfmm_apply(self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                    q2.shape[0], _stream_ptr(stream)))
        return u.reshape(q.shape) if out is None else u

    def apply_noalloc(self, q, out, stream=None):
        """u = A q into ``out`` with the library's fixed workspace (hfmm_apply_noalloc)."""
        q2 = _as_rhs(q, self.n, "q", self.device)
        _check_out(out, q2, "out")
        _check(self._lib.hfmm_apply_noalloc(self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            q2.shape[0], _stream_ptr(stream)))
        return out

    def apply_adjoint(self, v, q=None, grad_xy=False, stream=None):
        """w = A^H v; with grad_xy also the source-coordinate gradient (see hfmm.h)."""
        import torch
        v2 = _as_rhs(v, self.n, "v", self.device)
        if grad_xy and q is None:
            raise ValueError("grad_xy needs q")
        w = torch.empty_like(v2)
        # the contiguous copy of q must outlive the call (the library reads it
        # asynchronously on the stream)
        q2 = _as_rhs(q, self.n, "q", self.device) if q is not None else None
        if q2 is not None and q2.shape != v2.shape:
            raise ValueError("q and v must have the same shape")
        qp = ctypes.c_void_p(q2.data_ptr()) if q2 is not None else None
        g = torch.zeros((self.n, 2), dtype=torch.float64, device=v2.device) if grad_xy else None
        _check(self._lib.hfmm_apply_adjoint(self._h, ctypes.c_void_p(v2.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                            v2.shape[0], qp, ctypes.c_void_p(g.data_ptr()) if g is not None else None,
                                            _stream_ptr(stream)))
        if q2 is not None and q2.data_ptr() != q.data_ptr():
            # a temporary copy: keep it until the work on the stream has read it
            q2.record_stream(_stream_obj(stream))
        w = w.reshape(v.shape)
        return (w, g) if grad_xy else w

    def info(self) -> dict:
        inf = Info()
        _check(self._lib.hfmm_plan_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def bie_solve(self, w, f, phi=None, tol=1e-10, restart=50, max_iter=1000, stream=None):
        """GMRES for (A W + D) phi = f, the Nystrom single-layer system on the
        plan's nodes with trapezoidal weights w (hfmm_bie_solve); returns
        (phi, matvecs, relative residual)."""
        import torch
        f2 = _as_rhs(f, self.n, "f", self.device)
        if f2.shape[0] != 1:
            raise ValueError("one right-hand side")
        if not (w.is_cuda and w.dtype == torch.float64 and w.numel() == self.n and w.device == self.device):
            raise TypeError("w must be a float64 CUDA tensor of n weights on the plan's device")
        w2 = w.contiguous()
        x = torch.zeros_like(f2) if phi is None else _as_rhs(phi, self.n, "phi", self.device).clone()
        it = ctypes.c_int32()
        res = ctypes.c_double()
        _check(self._lib.hfmm_bie_solve(self._h, ctypes.c_void_p(w2.data_ptr()), ctypes.c_void_p(f2.data_ptr()),
                                        ctypes.c_void_p(x.data_ptr()), float(tol), int(restart), int(max_iter),
                                        ctypes.byref(it), ctypes.byref(res), _stream_ptr(stream)))
        return x[0], int(it.value), float(res.value)

    def profile(self, enable=True):
        """Record HIP events between the stages of every apply (hfmm_profile_enable)."""
        _check(self._lib.hfmm_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """Accumulated milliseconds per stage and the number of applies (hfmm_profile_read)."""
        ms = (ctypes.c_double * NSTAGES)()
        cnt = ctypes.c_int32()
        _check(self._lib.hfmm_profile_read(self._h, ms, ctypes.byref(cnt)))
        names = [self._lib.hfmm_stage_name(i).decode() for i in range(NSTAGES)]
        return dict(zip(names, list(ms))), cnt.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hfmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent geometries in one medium, applied together (hfmm_plan_batch).

    ``points`` is a list of float64 CUDA tensors (n_g, 2). apply() takes a list
    of complex128 right-hand sides (nrhs, n_g) and returns the list of results.
    graph(True) makes repeated applies with the same tensors replay a captured
    HIP graph; that needs a stream other than the legacy null stream."""

    def __init__(self, k, interfaces, points, tol=1e-8, stream=None, torch_allocator=True, **options):
        import torch
        lib = load()
        k = [float(v) for v in k]
        interfaces = [float(v) for v in interfaces]
        pts = []
        for p in points:
            if not (p.is_cuda and p.dtype == torch.float64 and p.dim() == 2 and p.shape[1] == 2):
                raise TypeError("points must be float64 CUDA tensors of shape (n, 2)")
            pts.append(p.contiguous())
        self._pts = pts
        self.ns = [int(p.shape[0]) for p in pts]
        G = len(pts)
        kk = (ctypes.c_double * len(k))(*k)
        ii = (ctypes.c_double * max(1, len(interfaces)))(*(interfaces or [0.0]))
        nn = (ctypes.c_int64 * G)(*self.ns)
        pp = (ctypes.c_void_p * G)(*[p.data_ptr() for p in pts])
        opts = default_options(torch_allocator=torch_allocator, **options)
        h = ctypes.c_void_p()
        _check(lib.hfmm_plan_batch(ctypes.byref(h), G, len(k), kk, ii, nn, pp, float(tol), ctypes.byref(opts),
                                   _stream_ptr(stream)))
        self._h = h
        self._lib = lib

    def __len__(self):
        return len(self.ns)

    def graph(self, enable=True):
        _check(self._lib.hfmm_batch_graph(self._h, 1 if enable else 0))

    def apply(self, qs, outs=None, stream=None):
        import torch
        G = len(self.ns)
        if len(qs) != G:
            raise ValueError("one right-hand side tensor per geometry")
        q2 = [_as_rhs(q, n, "q", p.device) for q, n, p in zip(qs, self.ns, self._pts)]
        nrhs = q2[0].shape[0]
        if any(q.shape[0] != nrhs for q in q2):
            raise ValueError("every geometry needs the same number of right-hand sides")
        if outs is not None:
            if len(outs) != G:
                raise ValueError("one output tensor per geometry")
            for o, q in zip(outs, q2):
                _check_out(o, q, "outs[g]")
        us = outs if outs is not None else [torch.empty_like(q) for q in q2]
        qa = (ctypes.c_void_p * G)(*[q.data_ptr() for q in q2])
        ua = (ctypes.c_void_p * G)(*[u.data_ptr() for u in us])
        _check(self._lib.hfmm_apply_batch(self._h, qa, ua, nrhs, _stream_ptr(stream)))
        return us

    def info(self, g):
        h = ctypes.c_void_p()
        _check(self._lib.hfmm_batch_plan(self._h, int(g), ctypes.byref(h)))
        inf = Info()
        _check(self._lib.hfmm_plan_info(h, ctypes.byref(inf)))
        return inf.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hfmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class HFMMApply(torch.autograd.Function):
        """u = A(points) q with the hand-written adjoint as its backward:
        grad_q = A^H grad_u and, when ``points`` requires grad, the gradient in
        the source coordinates (targets held fixed) from hfmm_apply_adjoint.
        The plan's tree stays frozen; ``points`` is the tensor the plan was built
        from (it only carries the autograd edge)."""

        @staticmethod
        def forward(ctx, q, points, plan):
            ctx.plan = plan
            ctx.save_for_backward(q)
            return plan.apply(q)

        @staticmethod
        def backward(ctx, g):
            (q,) = ctx.saved_tensors
            if ctx.needs_input_grad[1]:
                w, gxy = ctx.plan.apply_adjoint(g.contiguous(), q=q.detach(), grad_xy=True)
                return w, gxy, None
            return ctx.plan.apply_adjoint(g.contiguous()), None, None

    return HFMMApply


def hfmm_apply_autograd(q, plan, points=None):
    """u = plan.apply(q) differentiable in q and, if ``points`` (the plan's
    points, [n][2] float64) requires grad, in the source coordinates."""
    return _autograd().apply(q, points, plan)
