"""Python binding of libfc2t2.so: argument marshalling over ctypes, torch for device memory.

Every step of the computation runs in the HIP library; this module only checks shapes,
allocates outputs and workspaces with torch, and passes raw device pointers and torch's
current stream.  It raises if the library has not been built: there is no fallback.

Names follow the C-ABI (fc2t2.h) without the ``fc2t2_`` prefix, as methods of ``Plan``.
The autograd wrappers ``Explicit``, ``RayIntegral`` and ``RayRoot`` give the layers of the
paper's sections 4, 6.1 and 5 with their hand-written backward passes.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfc2t2.so")

KERNELS = {"gaussian": 0, "imq": 1, "poly": 2}
M2L_PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x2": 3, "bf16x3": 4, "separable": 5, "f16x3": 6,
            "f32_mfma": 7}
FIT = {"taylor": 0, "lsq": 0x100}   # M2L tensor: derivatives, or least-squares fit (section 3.1)
IO = {"f32": 0, "f64": 1}
OP = {"expand": 0, "eval_backward": 1, "expand_backward": 2, "ray_integral_backward": 3,
      "ray_root_backward": 4, "eval_sorted": 5, "ray_volume_backward": 6, "bin_points": 7}
VOLUME_STOP_DEPTH = 4.5   # the volume walk ends after the first cell exiting deeper than this
ROOT_SAVED = 12
ROOT_SMOOTH, ROOT_FACE, ROOT_GRAZING = 0, 1, 2   # kind of a ray-root hit, saved[:, 10]

_lib = None


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double)]


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("param", ctypes.c_double), ("n_coef", ctypes.c_int),
                ("coef", ctypes.POINTER(ctypes.c_double))]


class FC2T2Error(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    """Load libfc2t2.so (torch is imported first so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FC2T2Error("libfc2t2.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.fc2t2_status_string.restype = ctypes.c_char_p
    L.fc2t2_status_string.argtypes = [i32]
    L.fc2t2_multi_indices.restype = i32
    L.fc2t2_multi_indices.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int)]
    L.fc2t2_supported.restype = i32
    L.fc2t2_supported.argtypes = [i32, i32]
    L.fc2t2_plan_create.restype = i32
    L.fc2t2_plan_create.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Kernel), i32, i32, i32,
                                    i32, vp, ctypes.POINTER(vp)]
    L.fc2t2_plan_destroy.restype = i32
    L.fc2t2_plan_destroy.argtypes = [vp]
    for name in ("fc2t2_plan_P", "fc2t2_plan_P_pad", "fc2t2_plan_levels"):
        getattr(L, name).restype = i32
        getattr(L, name).argtypes = [vp]
    L.fc2t2_out_of_domain.restype = i32
    L.fc2t2_out_of_domain.argtypes = [vp, ctypes.POINTER(i64), i32, vp]
    L.fc2t2_grazing_roots.restype = i32
    L.fc2t2_grazing_roots.argtypes = [vp, ctypes.POINTER(i64), i32, vp]
    L.fc2t2_sort_failures.restype = i32
    L.fc2t2_sort_failures.argtypes = [vp, ctypes.POINTER(i64), i32, vp]
    L.fc2t2_debug_sort_fault.restype = None
    L.fc2t2_debug_sort_fault.argtypes = [i32]
    L.fc2t2_debug_root_cascade.restype = None
    L.fc2t2_debug_root_cascade.argtypes = [i32]
    L.fc2t2_local_numel.restype = sz
    L.fc2t2_local_numel.argtypes = [vp]
    L.fc2t2_workspace_size.restype = sz
    L.fc2t2_workspace_size.argtypes = [vp, i32, i64]
    L.fc2t2_expand.restype = i32
    L.fc2t2_expand.argtypes = [vp, vp, vp, i64, vp, vp, sz, vp]
    L.fc2t2_eval.restype = i32
    L.fc2t2_eval.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.fc2t2_eval_sorted.restype = i32
    L.fc2t2_eval_sorted.argtypes = [vp, vp, vp, i64, vp, vp, sz, vp]
    L.fc2t2_sort_queries.restype = i32
    L.fc2t2_sort_queries.argtypes = [vp, vp, i64, vp, sz, vp]
    L.fc2t2_eval_presorted.restype = i32
    L.fc2t2_eval_presorted.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    L.fc2t2_eval_backward_sorted.restype = i32
    L.fc2t2_eval_backward_sorted.argtypes = [vp, vp, i64, vp, vp, vp, vp, sz, i32, vp]
    L.fc2t2_eval_backward.restype = i32
    L.fc2t2_eval_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    L.fc2t2_expand_backward.restype = i32
    L.fc2t2_expand_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.fc2t2_eval_backward_ex.restype = i32
    L.fc2t2_eval_backward_ex.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, i32, vp]
    L.fc2t2_expand_backward_ex.restype = i32
    L.fc2t2_expand_backward_ex.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, sz, i32, vp]
    L.fc2t2_ray_integral.restype = i32
    L.fc2t2_ray_integral.argtypes = [vp, vp, vp, vp, dbl, dbl, i64, vp, vp]
    L.fc2t2_ray_integral_backward.restype = i32
    L.fc2t2_ray_integral_backward.argtypes = [vp, vp, vp, dbl, dbl, i64, vp, vp, vp, sz, vp]
    L.fc2t2_ray_root.restype = i32
    L.fc2t2_ray_root.argtypes = [vp, vp, vp, vp, dbl, dbl, i64, dbl, vp, vp, vp, vp, vp]
    L.fc2t2_ray_root_at.restype = i32
    L.fc2t2_ray_root_at.argtypes = [vp, vp, vp, vp, dbl, dbl, i64, vp, vp, vp, vp, vp, vp]
    L.fc2t2_bin_points.restype = i32
    L.fc2t2_bin_points.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fc2t2_ray_volume.restype = i32
    L.fc2t2_ray_volume.argtypes = [vp, vp, vp, vp, dbl, dbl, i64, vp, vp, vp, vp]
    L.fc2t2_ray_volume_backward.restype = i32
    L.fc2t2_ray_volume_backward.argtypes = [vp, vp, vp, vp, dbl, dbl, i64, vp, vp, vp, vp, sz, vp]
    L.fc2t2_m2l.restype = i32
    L.fc2t2_m2l.argtypes = [vp, i32, i32, vp, vp, i32, vp]
    L.fc2t2_level_numel.restype = sz
    L.fc2t2_level_numel.argtypes = [vp, i32]
    L.fc2t2_ray_root_backward.restype = i32
    L.fc2t2_ray_root_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    L.fc2t2_ray_root_backward_noalloc.restype = i32
    L.fc2t2_ray_root_backward_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.fc2t2_stage_timing.restype = i32
    L.fc2t2_stage_timing.argtypes = [vp, ctypes.c_uint32]
    L.fc2t2_stage_time.restype = i32
    L.fc2t2_stage_time.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        raise FC2T2Error("%s failed: %s (status %d)" % (what, lib().fc2t2_status_string(status).decode(), status))


def multi_indices(dim: int, K: int):
    """The library's multi-index order as a list of tuples."""
    L = lib()
    P = L.fc2t2_multi_indices(dim, K, None)
    if P < 0:
        raise FC2T2Error("bad dim/K")
    buf = (ctypes.c_int * (P * dim))()
    L.fc2t2_multi_indices(dim, K, buf)
    return [tuple(buf[i * dim:(i + 1) * dim]) for i in range(P)]


# Pipeline stages that fc2t2_stage_timing can bracket with events (enum fc2t2_stage order).
STAGES = ("sort", "p2m", "shift_up", "m2l", "shift_down", "l2p", "l2p_T", "m2l_T", "p2m_T", "ray", "ray_T",
          "qgrad")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A grid, a kernel psi and an order K (the paper's initialize(func, levels, rho))."""

    def __init__(self, dim: int, n: int, lo: float, hi: float, kernel: str, param: float = 0.0,
                 K: int = 4, m2l: str = "f32", io: str = "f32", channels: int = 1,
                 coef: Optional[Sequence[float]] = None, device=None, fit: str = "taylor"):
        L = lib()
        self.fit = fit
        self.dim, self.n, self.lo, self.hi, self.K = dim, n, float(lo), float(hi), K
        self.kernel, self.param, self.m2l_prec, self.io, self.C = kernel, float(param), m2l, io, channels
        self.dtype = torch.float64 if io == "f64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        g = _Grid(dim, n, self.lo, self.hi)
        if coef is not None:
            arr = (ctypes.c_double * len(coef))(*[float(c) for c in coef])
            self._coef = arr
            k = _Kernel(KERNELS[kernel], self.param, len(coef), ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
        else:
            k = _Kernel(KERNELS[kernel], self.param, 0, None)
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.fc2t2_plan_create(ctypes.byref(g), ctypes.byref(k), K, M2L_PREC[m2l] | FIT[fit], IO[io],
                                       channels, _stream(), ctypes.byref(out)), "fc2t2_plan_create")
        self.handle = out
        self.P = L.fc2t2_plan_P(out)
        self.P_pad = L.fc2t2_plan_P_pad(out)
        self.levels = L.fc2t2_plan_levels(out)
        self.h = (self.hi - self.lo) / n

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.fc2t2_plan_destroy(h)
            self.handle = None

    # ------------------------------------------------------------------ helpers
    def _t(self, x: torch.Tensor, shape, name: str) -> torch.Tensor:
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise FC2T2Error("%s must be a CUDA tensor" % name)
        if x.dtype != self.dtype:
            raise FC2T2Error("%s must be %s" % (name, self.dtype))
        if tuple(x.shape) != tuple(shape):
            raise FC2T2Error("%s has shape %s, expected %s" % (name, tuple(x.shape), tuple(shape)))
        return x.contiguous()

    def local_shape(self):
        return (self.C, self.n ** self.dim, self.P_pad)

    def new_local(self) -> torch.Tensor:
        return torch.zeros(self.local_shape(), dtype=self.dtype, device=self.device)

    def workspace(self, op: str, count: int) -> torch.Tensor:
        nbytes = lib().fc2t2_workspace_size(self.handle, OP[op], int(count))
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def level_shape(self, level: int):
        return (self.C, (self.n >> level) ** self.dim, self.P_pad)

    def stage_timing(self, stages=()):
        """Time the named stages (see STAGES) with events on the launch stream from now on."""
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
        _check(lib().fc2t2_stage_timing(self.handle, mask), "fc2t2_stage_timing")

    def stage_time(self, stage: str):
        """(milliseconds, calls) recorded for a stage since the last read; clears them."""
        ms, calls = ctypes.c_double(0.0), ctypes.c_int64(0)
        _check(lib().fc2t2_stage_time(self.handle, STAGES.index(stage), ctypes.byref(ms), ctypes.byref(calls)),
               "fc2t2_stage_time")
        return ms.value, calls.value

    def m2l(self, level: int, src: torch.Tensor, out: torch.Tensor, transpose: bool = False,
            accumulate: bool = False):
        """One M2L (or M2L^T) launch at a level between caller-owned grids of that level."""
        shp = self.level_shape(level)
        src = self._t(src, shp, "in")
        assert out.is_contiguous() and tuple(out.shape) == shp and out.dtype == self.dtype
        _check(lib().fc2t2_m2l(self.handle, level, int(transpose), _ptr(src), _ptr(out), int(accumulate),
                               _stream()), "fc2t2_m2l")

    # ------------------------------------------------------------------ C-ABI calls
    def expand(self, p: torch.Tensor, w: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        N = p.shape[0]
        p = self._t(p, (N, self.dim), "p")
        w = self._t(w, (N, self.C), "w")
        Lt = self.new_local() if out is None else self._t(out, self.local_shape(), "L")
        ws = self.workspace("expand", N)
        _check(lib().fc2t2_expand(self.handle, _ptr(p), _ptr(w), N, _ptr(Lt), _ptr(ws), ws.numel(),
                                  _stream()), "fc2t2_expand")
        self._debug_domain("sources")
        return Lt

    def eval(self, Lt: torch.Tensor, q: torch.Tensor, grad: bool = False, hess: bool = False):
        M = q.shape[0]
        q = self._t(q, (M, self.dim), "q")
        Lt = self._t(Lt, self.local_shape(), "L")
        y = torch.empty((M, self.C), dtype=self.dtype, device=self.device)
        g = torch.empty((M, self.C, self.dim), dtype=self.dtype, device=self.device) if grad or hess else None
        nh = self.dim * (self.dim + 1) // 2
        hs = torch.empty((M, self.C, nh), dtype=self.dtype, device=self.device) if hess else None
        _check(lib().fc2t2_eval(self.handle, _ptr(Lt), _ptr(q), M, _ptr(y), _ptr(g), _ptr(hs), _stream()),
               "fc2t2_eval")
        self._debug_domain("queries")
        return y, g, hs

    @property
    def sorted_queries(self) -> bool:
        """Whether eval_sorted / eval_backward_sorted apply (FP32 IO, one channel)."""
        return self.io == "f32" and self.C == 1

    def eval_sorted(self, Lt: torch.Tensor, q: torch.Tensor, ws: Optional[torch.Tensor] = None):
        """y at the queries taken in cell order; returns (y, ws), ws holding the sorted queries for
        eval_backward_sorted."""
        M = q.shape[0]
        q = self._t(q, (M, self.dim), "q")
        Lt = self._t(Lt, self.local_shape(), "L")
        if ws is None:
            ws = self.workspace("eval_sorted", M)
        y = torch.empty((M, self.C), dtype=self.dtype, device=self.device)
        _check(lib().fc2t2_eval_sorted(self.handle, _ptr(Lt), _ptr(q), M, _ptr(y), _ptr(ws), ws.numel(), _stream()),
               "fc2t2_eval_sorted")
        self._debug_domain("queries")
        return y, ws

    def sort_queries(self, q: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """First half of eval_sorted: the queries binned and sorted by cell into ws (returned), on
        the current stream.  eval_presorted then evaluates from ws; a caller can run this on a
        side stream while the expansion is built."""
        M = q.shape[0]
        q = self._t(q, (M, self.dim), "q")
        if ws is None:
            ws = self.workspace("eval_sorted", M)
        _check(lib().fc2t2_sort_queries(self.handle, _ptr(q), M, _ptr(ws), ws.numel(), _stream()),
               "fc2t2_sort_queries")
        return ws

    def eval_presorted(self, Lt: torch.Tensor, M: int, ws: torch.Tensor) -> torch.Tensor:
        """Second half of eval_sorted: y [M] (input order) from the records sort_queries left in ws
        (ordered after it on the device)."""
        Lt = self._t(Lt, self.local_shape(), "L")
        y = torch.empty((M, self.C), dtype=self.dtype, device=self.device)
        _check(lib().fc2t2_eval_presorted(self.handle, _ptr(Lt), M, _ptr(y), _ptr(ws), ws.numel(), _stream()),
               "fc2t2_eval_presorted")
        self._debug_domain("queries")
        return y

    def eval_backward_sorted(self, Lt, M: int, gy, ws, gL: torch.Tensor, gq: Optional[torch.Tensor] = None,
                             accumulate: bool = True):
        """gL, gq += (accumulate) or = (otherwise) the cotangents of L and q, from the sorted queries
        an eval_sorted call left in ws."""
        gy = self._t(gy, (M, self.C), "gy")
        assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        if gq is not None:
            assert gq.is_contiguous() and tuple(gq.shape) == (M, self.dim) and gq.dtype == self.dtype
        _check(lib().fc2t2_eval_backward_sorted(self.handle, _ptr(Lt), M, _ptr(gy), _ptr(gL), _ptr(gq), _ptr(ws),
                                                ws.numel(), 1 if accumulate else 0, _stream()),
               "fc2t2_eval_backward_sorted")

    def out_of_domain(self, reset: bool = False) -> int:
        """Points outside [lo, hi]^dim met by expand (sources) and eval (queries) since the plan was
        made or last reset; they were binned into the nearest boundary cell.  Synchronises."""
        c = ctypes.c_int64(0)
        _check(lib().fc2t2_out_of_domain(self.handle, ctypes.byref(c), 1 if reset else 0, _stream()),
               "fc2t2_out_of_domain")
        return int(c.value)

    def grazing_roots(self, reset: bool = False) -> int:
        """Ray roots classified as grazing (the ray tangent to the level set; their backward
        inserts only the surface-gradient term) since the plan was made or last reset.
        Synchronises."""
        c = ctypes.c_int64(0)
        _check(lib().fc2t2_grazing_roots(self.handle, ctypes.byref(c), 1 if reset else 0, _stream()),
               "fc2t2_grazing_roots")
        return int(c.value)

    def sort_failures(self, reset: bool = False) -> int:
        """Sorts by cell whose look-back gave up on this plan since it was made or last reset (the
        outputs of the calls since then are not valid).  Synchronises."""
        c = ctypes.c_int64(0)
        _check(lib().fc2t2_sort_failures(self.handle, ctypes.byref(c), 1 if reset else 0, _stream()),
               "fc2t2_sort_failures")
        return int(c.value)

    @staticmethod
    def root_kind(saved: torch.Tensor) -> torch.Tensor:
        """Kind of each ray-root hit (ROOT_SMOOTH, ROOT_FACE, ROOT_GRAZING) from the saved record."""
        return saved[:, 10].to(torch.int32)

    def _debug_domain(self, what: str):
        # debug mode (FC2T2_DEBUG=1): fail on points outside the domain and on failed sorts, at the
        # call that met them
        if os.environ.get("FC2T2_DEBUG", "0") not in ("", "0"):
            n = self.out_of_domain(reset=True)
            if n:
                raise FC2T2Error("%d %s outside the domain [%g, %g]^%d (binned into boundary cells)"
                                 % (n, what, self.lo, self.hi, self.dim))
            f = self.sort_failures(reset=True)
            if f:
                raise FC2T2Error("%d sort(s) by cell failed (look-back gave up); outputs are not valid" % f)

    def eval_backward(self, Lt, q, gy, gL: Optional[torch.Tensor] = None, gq: Optional[torch.Tensor] = None,
                      accumulate: bool = True):
        """gL, gq += (accumulate) or = (otherwise) the cotangents of L and q."""
        M = q.shape[0]
        q = self._t(q, (M, self.dim), "q")
        gy = self._t(gy, (M, self.C), "gy")
        if gL is not None:
            assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        if gq is not None:
            assert gq.is_contiguous() and tuple(gq.shape) == (M, self.dim) and gq.dtype == self.dtype
        ws = self.workspace("eval_backward", M) if gL is not None else None
        _check(lib().fc2t2_eval_backward_ex(self.handle, _ptr(Lt), _ptr(q), M, _ptr(gy), _ptr(gL), _ptr(gq),
                                            _ptr(ws), 0 if ws is None else ws.numel(), 1 if accumulate else 0,
                                            _stream()), "fc2t2_eval_backward_ex")

    def expand_backward(self, gL, p, w, gp: Optional[torch.Tensor] = None, gw: Optional[torch.Tensor] = None,
                        accumulate: bool = True):
        """gp, gw += (accumulate) or = (otherwise) the cotangents of p and w."""
        N = p.shape[0]
        p = self._t(p, (N, self.dim), "p")
        w = self._t(w, (N, self.C), "w")
        gL = self._t(gL, self.local_shape(), "gL")
        if gp is not None:
            assert gp.is_contiguous() and tuple(gp.shape) == (N, self.dim) and gp.dtype == self.dtype
        if gw is not None:
            assert gw.is_contiguous() and tuple(gw.shape) == (N, self.C) and gw.dtype == self.dtype
        ws = self.workspace("expand_backward", N)
        _check(lib().fc2t2_expand_backward_ex(self.handle, _ptr(gL), _ptr(p), _ptr(w), N, _ptr(gp), _ptr(gw),
                                              _ptr(ws), ws.numel(), 1 if accumulate else 0, _stream()),
               "fc2t2_expand_backward_ex")

    def ray_integral(self, Lt, o, r, t0: float, t1: float) -> torch.Tensor:
        R = o.shape[0]
        o = self._t(o, (R, 3), "o")
        r = self._t(r, (R, 3), "r")
        Lt = self._t(Lt, self.local_shape(), "L")
        y = torch.empty((R, self.C), dtype=self.dtype, device=self.device)
        _check(lib().fc2t2_ray_integral(self.handle, _ptr(Lt), _ptr(o), _ptr(r), float(t0), float(t1), R,
                                        _ptr(y), _stream()), "fc2t2_ray_integral")
        return y

    def ray_integral_backward(self, o, r, t0: float, t1: float, gy, gL):
        R = o.shape[0]
        o = self._t(o, (R, 3), "o")
        r = self._t(r, (R, 3), "r")
        gy = self._t(gy, (R, self.C), "gy")
        assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        ws = self.workspace("ray_integral_backward", R)
        _check(lib().fc2t2_ray_integral_backward(self.handle, _ptr(o), _ptr(r), float(t0), float(t1), R,
                                                 _ptr(gy), _ptr(gL), _ptr(ws), ws.numel(), _stream()),
               "fc2t2_ray_integral_backward")

    def bin_points(self, x, extra=None, with_payload: bool = False):
        """Stable sort of points by finest cell: (keys_sorted [N], perm [N], starts [G + 1]) as
        int32 views of the library's uint32 outputs, plus the sorted payload with with_payload
        (coordinates [N, dim], or [N, dim + 1] with extra [N] appended)."""
        N = x.shape[0]
        x = self._t(x, (N, self.dim), "x")
        if extra is not None:
            extra = self._t(extra, (N,), "extra")
            with_payload = True
        keys = torch.empty(N, dtype=torch.int32, device=self.device)
        perm = torch.empty(N, dtype=torch.int32, device=self.device)
        starts = torch.empty(self.n ** self.dim + 1, dtype=torch.int32, device=self.device)
        pay = None
        if with_payload:
            pay = torch.empty((N, self.dim + (1 if extra is not None else 0)), dtype=self.dtype, device=self.device)
        ws = self.workspace("bin_points", N)
        _check(lib().fc2t2_bin_points(self.handle, _ptr(x), N, _ptr(extra), _ptr(keys), _ptr(perm), _ptr(starts),
                                      _ptr(pay), _ptr(ws), ws.numel(), _stream()), "fc2t2_bin_points")
        return (keys, perm, starts, pay) if with_payload else (keys, perm, starts)

    @staticmethod
    def _bg(bg):
        """Background colour as a host array of 3 doubles (None: black)."""
        if bg is None:
            return None
        vals = [float(v) for v in bg]
        assert len(vals) == 3, "bg has three components"
        return (ctypes.c_double * 3)(*vals)

    def ray_volume(self, Lt, o, r, t0: float, t1: float, bg=None, with_trans: bool = False):
        """Volumetric rendering (four channels: density, R, G, B): colour y [R, 3], and the exit
        transmittance [R] as well with with_trans."""
        R = o.shape[0]
        o = self._t(o, (R, 3), "o")
        r = self._t(r, (R, 3), "r")
        Lt = self._t(Lt, self.local_shape(), "L")
        y = torch.empty((R, 3), dtype=self.dtype, device=self.device)
        tr = torch.empty(R, dtype=self.dtype, device=self.device) if with_trans else None
        _check(lib().fc2t2_ray_volume(self.handle, _ptr(Lt), _ptr(o), _ptr(r), float(t0), float(t1), R,
                                      self._bg(bg), _ptr(y), _ptr(tr), _stream()), "fc2t2_ray_volume")
        return (y, tr) if with_trans else y

    def ray_volume_backward(self, Lt, o, r, t0: float, t1: float, gy, gL, bg=None):
        """gL += the cotangent of the four channels of Lt from colour cotangents gy [R, 3]."""
        R = o.shape[0]
        o = self._t(o, (R, 3), "o")
        r = self._t(r, (R, 3), "r")
        Lt = self._t(Lt, self.local_shape(), "L")
        gy = self._t(gy, (R, 3), "gy")
        assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        ws = self.workspace("ray_volume_backward", R)
        _check(lib().fc2t2_ray_volume_backward(self.handle, _ptr(Lt), _ptr(o), _ptr(r), float(t0), float(t1), R,
                                               self._bg(bg), _ptr(gy), _ptr(gL), _ptr(ws), ws.numel(), _stream()),
               "fc2t2_ray_volume_backward")

    def ray_root(self, Lt, o, r, t0: float, t1: float, level_frac: float = 0.5,
                 tau: Optional[torch.Tensor] = None):
        """First upward crossing of level_frac * max f along each ray, or of the given per-ray
        levels tau [R] (fc2t2_ray_root_at)."""
        R = o.shape[0]
        o = self._t(o, (R, 3), "o")
        r = self._t(r, (R, 3), "r")
        Lt = self._t(Lt, self.local_shape(), "L")
        t = torch.empty(R, dtype=self.dtype, device=self.device)
        normal = torch.empty((R, 3), dtype=self.dtype, device=self.device)
        hit = torch.empty(R, dtype=torch.int32, device=self.device)
        saved = torch.empty((R, ROOT_SAVED), dtype=self.dtype, device=self.device)
        if tau is None:
            _check(lib().fc2t2_ray_root(self.handle, _ptr(Lt), _ptr(o), _ptr(r), float(t0), float(t1), R,
                                        float(level_frac), _ptr(t), _ptr(normal), _ptr(hit), _ptr(saved),
                                        _stream()), "fc2t2_ray_root")
        else:
            tau = self._t(tau, (R,), "tau")
            _check(lib().fc2t2_ray_root_at(self.handle, _ptr(Lt), _ptr(o), _ptr(r), float(t0), float(t1), R,
                                           _ptr(tau), _ptr(t), _ptr(normal), _ptr(hit), _ptr(saved), _stream()),
                   "fc2t2_ray_root_at")
        return t, normal, hit, saved

    def ray_root_backward(self, saved, hit, gt, gn, gL):
        R = saved.shape[0]
        saved = self._t(saved, (R, ROOT_SAVED), "saved")
        assert hit.dtype == torch.int32 and hit.is_contiguous()
        if gt is not None:
            gt = self._t(gt, (R,), "gt")
        if gn is not None:
            gn = self._t(gn, (R, 3), "gn")
        assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        ws = self.workspace("ray_root_backward", R)
        _check(lib().fc2t2_ray_root_backward(self.handle, _ptr(saved), _ptr(hit), R, _ptr(gt), _ptr(gn),
                                             _ptr(gL), _ptr(ws), ws.numel(), _stream()),
               "fc2t2_ray_root_backward")

    def ray_root_backward_noalloc(self, saved, hit, gt, gn, gL):
        """ray_root_backward with the library's fixed device scratch (no workspace, nothing
        allocated by the call); calls on one GPU must not overlap in time."""
        R = saved.shape[0]
        saved = self._t(saved, (R, ROOT_SAVED), "saved")
        assert hit.dtype == torch.int32 and hit.is_contiguous()
        if gt is not None:
            gt = self._t(gt, (R,), "gt")
        if gn is not None:
            gn = self._t(gn, (R, 3), "gn")
        assert gL.is_contiguous() and tuple(gL.shape) == self.local_shape() and gL.dtype == self.dtype
        _check(lib().fc2t2_ray_root_backward_noalloc(self.handle, _ptr(saved), _ptr(hit), R, _ptr(gt), _ptr(gn),
                                                     _ptr(gL), _stream()), "fc2t2_ray_root_backward_noalloc")


# ---------------------------------------------------------------------------- autograd

_side_streams = {}


def _side_stream(device) -> "torch.cuda.Stream":
    """A second stream per device (default priority) for work that overlaps the current
    stream's."""
    key = torch.device(device).index
    if key not in _side_streams:
        _side_streams[key] = torch.cuda.Stream(device=device)
    return _side_streams[key]


class Explicit(torch.autograd.Function):
    """y = f(q; p, w) (section 4) with the backward of section 4.1."""

    @staticmethod
    def forward(ctx, plan: Plan, p, w, q):
        if plan.sorted_queries:
            # queries sorted once, in the forward, on a side stream while the expansion is built;
            # the backward reuses the sorted records
            ws = plan.workspace("eval_sorted", q.shape[0])
            main = torch.cuda.current_stream()
            side = _side_stream(q.device)
            side.wait_stream(main)
            with torch.cuda.stream(side):
                plan.sort_queries(q, ws)
            Lt = plan.expand(p, w)
            main.wait_stream(side)
            y = plan.eval_presorted(Lt, q.shape[0], ws)
        else:
            Lt = plan.expand(p, w)
            (y, _, _), ws = plan.eval(Lt, q), None
        ctx.plan, ctx.ws = plan, ws
        ctx.save_for_backward(p, w, q, Lt)
        return y

    @staticmethod
    def backward(ctx, gy):
        plan = ctx.plan
        p, w, q, Lt = ctx.saved_tensors
        gy = gy.contiguous()
        need_p, need_w, need_q = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        # fresh buffers, written (not accumulated) by the library
        gq = torch.empty_like(q) if need_q else None
        gp = torch.empty_like(p) if need_p else None
        gw = torch.empty_like(w) if need_w else None
        gL = torch.empty(plan.local_shape(), dtype=plan.dtype, device=q.device) if (need_p or need_w) else None
        if ctx.ws is not None and gL is not None:
            plan.eval_backward_sorted(Lt, q.shape[0], gy, ctx.ws, gL, gq, accumulate=False)
        else:
            plan.eval_backward(Lt, q, gy, gL, gq, accumulate=False)
        ctx.ws = None
        if gL is not None:
            plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
        return None, gp, gw, gq


class RayIntegral(torch.autograd.Function):
    """y_r = integral of f(o_r + t r_r) over t in [t0, t1] (section 6.1) and its backward
    by ray insertion (section 6.2.1)."""

    @staticmethod
    def forward(ctx, plan: Plan, p, w, o, r, t0: float, t1: float):
        Lt = plan.expand(p, w)
        y = plan.ray_integral(Lt, o, r, t0, t1)
        ctx.plan, ctx.t0, ctx.t1 = plan, t0, t1
        ctx.save_for_backward(p, w, o, r)
        return y

    @staticmethod
    def backward(ctx, gy):
        plan = ctx.plan
        p, w, o, r = ctx.saved_tensors
        gL = plan.new_local()
        plan.ray_integral_backward(o, r, ctx.t0, ctx.t1, gy.contiguous(), gL)
        gp = torch.empty_like(p) if ctx.needs_input_grad[1] else None
        gw = torch.empty_like(w) if ctx.needs_input_grad[2] else None
        plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
        return None, gp, gw, None, None, None, None


class RayVolume(torch.autograd.Function):
    """Colour of each ray through the density and colour fields of one four-channel expansion
    (section 6.1.2: channel 0 the density, channels 1..3 R, G, B), with the backward of
    section 6.2.2 as the exact derivative of the forward.  Keeping the density non-negative
    (e.g. non-negative density weights) is the caller's part."""

    @staticmethod
    def forward(ctx, plan: Plan, p, w, o, r, t0: float, t1: float, bg=None):
        Lt = plan.expand(p, w)
        y = plan.ray_volume(Lt, o, r, t0, t1, bg)
        ctx.plan, ctx.t0, ctx.t1, ctx.bg = plan, t0, t1, bg
        ctx.save_for_backward(p, w, o, r, Lt)
        return y

    @staticmethod
    def backward(ctx, gy):
        plan = ctx.plan
        p, w, o, r, Lt = ctx.saved_tensors
        gL = plan.new_local()
        plan.ray_volume_backward(Lt, o, r, ctx.t0, ctx.t1, gy.contiguous(), gL, ctx.bg)
        gp = torch.empty_like(p) if ctx.needs_input_grad[1] else None
        gw = torch.empty_like(w) if ctx.needs_input_grad[2] else None
        plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
        return None, gp, gw, None, None, None, None, None


class RayRoot(torch.autograd.Function):
    """(t*, grad f(q*)) of the first level crossing along each ray (section 5.1), with the
    implicit-function-theorem backward of section 5.2.  The level is level_frac * max f along
    the ray, or the given per-ray levels tau; either way it is held fixed in the backward."""

    @staticmethod
    def forward(ctx, plan: Plan, p, w, o, r, t0: float, t1: float, level_frac: float = 0.5, tau=None):
        Lt = plan.expand(p, w)
        t, normal, hit, saved = plan.ray_root(Lt, o, r, t0, t1, level_frac, tau)
        ctx.plan = plan
        ctx.save_for_backward(p, w, saved, hit)
        ctx.mark_non_differentiable(hit)
        return t, normal, hit

    @staticmethod
    def backward(ctx, gt, gn, _ghit):
        plan = ctx.plan
        p, w, saved, hit = ctx.saved_tensors
        gL = plan.new_local()
        plan.ray_root_backward(saved, hit, None if gt is None else gt.contiguous(),
                               None if gn is None else gn.contiguous(), gL)
        gp = torch.empty_like(p) if ctx.needs_input_grad[1] else None
        gw = torch.empty_like(w) if ctx.needs_input_grad[2] else None
        plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
        return None, gp, gw, None, None, None, None, None, None
