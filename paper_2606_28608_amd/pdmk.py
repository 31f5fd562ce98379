"""Python binding of libpdmk (include/pdmk.h): argument marshalling only.

Every step of the evaluation runs in the HIP library; PyTorch provides device
memory and the stream.  If libpdmk.so is missing the functions raise: there is
no fallback implementation.

    from paper_2606_28608_amd import pdmk
    pot = pdmk.pdmk_eval(L, src, q, eps=1e-6)            # targets = sources
    pot, grad = pdmk.pdmk_eval(L, src, q, eps=1e-6, grad=True)
    plan = pdmk.Plan(L, dim=3, eps=1e-6); pot = plan.eval(src, q)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdmk.so")

PDMK_PREC_FP64 = 0
PDMK_PREC_MIXED = 1
PDMK_WANT_GRAD = 1
PDMK_ALLOW_NONNEUTRAL = 2
PDMK_DETERMINISTIC = 4
PDMK_VECTOR_PLANE_WAVES = 8
PDMK_ONE_STREAM = 16
PDMK_BLOCH = 32
PDMK_VIRTUAL_IMAGES = 64
PDMK_BALANCE = 128
PDMK_ALL_PAIRS = 256
PDMK_FP32_RESIDUAL = 1
PDMK_FP32_PROXY = 2
PDMK_FP32_WINDOW = 4
PDMK_BF16_PLANE_WAVES = 8

STATUS = {0: "PDMK_OK", -1: "PDMK_ERR_INVALID_ARG", -2: "PDMK_ERR_SINGULAR_LATTICE",
          -3: "PDMK_ERR_NOT_NEUTRAL", -4: "PDMK_ERR_EPS_RANGE", -5: "PDMK_ERR_NONFINITE",
          -6: "PDMK_ERR_OUT_OF_MEMORY", -7: "PDMK_ERR_HIP", -8: "PDMK_ERR_NO_DEVICE",
          -9: "PDMK_ERR_UNSUPPORTED", -10: "PDMK_ERR_SCRATCH"}


class PdmkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("eps", ctypes.c_double), ("precision", ctypes.c_int),
                ("kappa", ctypes.c_double), ("n_s", ctypes.c_int), ("flags", ctypes.c_uint),
                ("porder", ctypes.c_int), ("npw", ctypes.c_int), ("nufft_w", ctypes.c_int),
                ("sigma", ctypes.c_double), ("fp32_stages", ctypes.c_uint),
                ("bloch", ctypes.c_double * 3)]


class Geometry(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("L_oriented", ctypes.c_double * 9),
                ("Q", ctypes.c_double * 9), ("perm", ctypes.c_int * 3),
                ("volume", ctypes.c_double), ("rc", ctypes.c_double),
                ("nroot", ctypes.c_int * 3), ("origin", ctypes.c_double * 3),
                ("fgrid", ctypes.c_int * 3), ("fgrid_paper", ctypes.c_int * 3),
                ("n_shifts", ctypes.c_int), ("c", ctypes.c_double),
                ("w0_zero_rc", ctypes.c_double), ("porder", ctypes.c_int),
                ("npw", ctypes.c_int), ("nufft_w", ctypes.c_int), ("n_s", ctypes.c_int),
                ("nufft_beta", ctypes.c_double), ("kappa", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_trg", ctypes.c_int64),
                ("n_images", ctypes.c_int64), ("n_levels", ctypes.c_int),
                ("n_boxes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("n_nonleaf", ctypes.c_int64), ("n_direct_pairs", ctypes.c_int64),
                ("n_pw_pairs", ctypes.c_int64), ("t_build_ms", ctypes.c_double),
                ("t_near_ms", ctypes.c_double), ("t_far_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("t_direct_ms", ctypes.c_double),
                ("t_pw_ms", ctypes.c_double), ("t_proxy_ms", ctypes.c_double),
                ("n_support_pairs", ctypes.c_int64), ("series_len", ctypes.c_int),
                ("t_call_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("n_pwout_boxes", ctypes.c_int64), ("n_pwin_boxes", ctypes.c_int64),
                ("t_pwout_ms", ctypes.c_double), ("t_pwin_ms", ctypes.c_double),
                ("t_pwtr_ms", ctypes.c_double), ("n_staged_pairs", ctypes.c_int64),
                ("t_spread_ms", ctypes.c_double), ("t_fft_ms", ctypes.c_double),
                ("t_interp_ms", ctypes.c_double), ("n_forced_splits", ctypes.c_int64),
                ("balance_rounds", ctypes.c_int), ("pairs_once", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelInfo(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("c0_over_psi0", ctypes.c_double), ("w0_zero", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def lib():
    """Load libpdmk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libpdmk bind to that one, so the process has one runtime.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpdmk.so is not built (run paper_2606_28608_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.pdmk_default_opts.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(Opts)]
        L.pdmk_eval.argtypes = [ctypes.POINTER(Opts), _dp, ctypes.c_int64, _vp, _vp,
                                ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.pdmk_plan_create.argtypes = [ctypes.POINTER(Opts), _dp, ctypes.POINTER(_vp)]
        L.pdmk_plan_eval.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp,
                                     _vp]
        L.pdmk_plan_adjoint.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp]
        L.pdmk_batch_create.argtypes = [ctypes.POINTER(Opts), ctypes.c_int, _dp, ctypes.c_int,
                                        ctypes.POINTER(_vp)]
        L.pdmk_batch_eval.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), _vp, _vp, _vp, _vp,
                                      _vp]
        L.pdmk_batch_destroy.argtypes = [_vp]
        L.pdmk_batch_destroy.restype = None
        L.pdmk_batch_stats.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(Stats)]
        L.pdmk_batch_bind.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), _vp, _vp, _vp, _vp,
                                      _vp]
        L.pdmk_batch_execute.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.pdmk_batch_status.argtypes = [_vp]
        L.pdmk_batch_tune.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), _vp, _vp, ctypes.c_int,
                                      _dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp, _dp,
                                      ctypes.POINTER(ctypes.c_int)]
        L.pdmk_plan_tune.argtypes = [ctypes.POINTER(Opts), _dp, ctypes.c_int, _dp,
                                     ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int64,
                                     _vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _dp, _dp,
                                     ctypes.POINTER(ctypes.c_int)]
        L.pdmk_plan_eval_bloch.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp,
                                           _vp, _vp]
        L.pdmk_plan_eval_parts.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp,
                                           _vp, _vp, _vp]
        L.pdmk_plan_eval_noalloc.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp,
                                             _vp, _vp, _vp]
        L.pdmk_plan_bind.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp,
                                     _vp]
        L.pdmk_plan_execute.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.pdmk_plan_status.argtypes = [_vp]
        L.pdmk_plan_unbind.argtypes = [_vp]
        L.pdmk_plan_unbind.restype = None
        L.pdmk_plan_destroy.argtypes = [_vp]
        L.pdmk_plan_destroy.restype = None
        L.pdmk_plan_geometry.argtypes = [_vp, ctypes.POINTER(Geometry)]
        L.pdmk_geometry_get.argtypes = [ctypes.POINTER(Opts), _dp, ctypes.POINTER(Geometry)]
        L.pdmk_plan_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
        L.pdmk_kernel_info_get.argtypes = [ctypes.c_int, ctypes.c_double,
                                           ctypes.POINTER(KernelInfo)]
        L.pdmk_kernel_eval_residual.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_int64, _dp, _dp]
        L.pdmk_kernel_eval_w0hat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int64, _dp, _dp]
        L.pdmk_status_string.argtypes = [ctypes.c_int]
        L.pdmk_status_string.restype = ctypes.c_char_p
        L.pdmk_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise PdmkError(code, lib().pdmk_last_error().decode())


def default_opts(dim, eps, precision="fp64", grad=False, allow_nonneutral=False,
                 deterministic=False, vector_plane_waves=False, one_stream=False, bloch=None,
                 virtual_images=False, balance=False, all_pairs=False, **over):
    """pdmk_opts for (dim, eps) with the defaults of pdmk_default_opts; keyword
    arguments set flags (grad, allow_nonneutral, deterministic,
    vector_plane_waves, one_stream, bloch = Bloch vector, virtual_images, balance,
    all_pairs) or
    override fields (kappa, n_s, porder, npw, nufft_w,
    sigma, fp32_stages)."""
    o = Opts()
    _check(lib().pdmk_default_opts(int(dim), float(eps), ctypes.byref(o)))
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    o.precision = PDMK_PREC_MIXED if precision == "mixed" else PDMK_PREC_FP64
    o.flags = ((PDMK_WANT_GRAD if grad else 0) | (PDMK_ALLOW_NONNEUTRAL if allow_nonneutral else 0)
               | (PDMK_DETERMINISTIC if deterministic else 0)
               | (PDMK_VECTOR_PLANE_WAVES if vector_plane_waves else 0)
               | (PDMK_ONE_STREAM if one_stream else 0)
               | (PDMK_BLOCH if bloch is not None else 0)
               | (PDMK_VIRTUAL_IMAGES if virtual_images else 0)
               | (PDMK_BALANCE if balance else 0)
               | (PDMK_ALL_PAIRS if all_pairs else 0))
    if bloch is not None:
        b = [float(v) for v in bloch]
        if len(b) != dim:
            raise ValueError("the Bloch vector needs %d components" % dim)
        for i, v in enumerate(b):
            o.bloch[i] = v
    for k, v in over.items():
        if v is not None:
            setattr(o, k, v)
    return o


def _lattice(L, dim):
    L = np.asarray(L, dtype=np.float64)
    if L.shape != (dim, dim):
        raise ValueError("L must be %dx%d with lattice vectors as columns" % (dim, dim))
    return np.asfortranarray(L).ravel(order="F").copy()


def tune(L, src, q, eps=1e-6, precision="fp64", candidates=None, trials=2, trg=None,
         dim=None, **over):
    """Runtime planning (pdmk_plan_tune): times each (kappa, n_s) candidate on
    this input and returns (kappa, n_s, {(kappa, n_s): ms}).  Default
    candidates: kappa in {3, 4, 6} with the default leaf capacity times
    {1, 1.5, 2, 2.5} (with residual pairs evaluated once, leaves larger than
    the paper's table pay off)."""
    import torch
    L = np.asarray(L, dtype=np.float64)
    dim = dim or L.shape[0]
    o = default_opts(dim, eps, precision, **over)
    if candidates is None:
        base = o.n_s
        candidates = [(k, int(round(base * f))) for k in (3.0, 4.0, 6.0)
                      for f in (1.0, 1.5, 2.0, 2.5)]
    kap = np.array([float(c[0]) for c in candidates], dtype=np.float64)
    nss = (ctypes.c_int * len(candidates))(*[int(c[1]) for c in candidates])
    src = _dev(src, torch)
    q = _dev(q, torch)
    n = src.shape[0]
    if trg is not None:
        trg = _dev(trg, torch)
        m = trg.shape[0]
    else:
        m = n
    pot = torch.empty(m, dtype=torch.float64, device=src.device)
    times = np.zeros(len(candidates), dtype=np.float64)
    bk = ctypes.c_double(0.0)
    bn = ctypes.c_int(0)
    Lf = _lattice(L, dim)
    _check(lib().pdmk_plan_tune(ctypes.byref(o), Lf.ctypes.data_as(_dp), len(candidates),
                                kap.ctypes.data_as(_dp), nss, int(trials), n,
                                ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                m, ctypes.c_void_p(trg.data_ptr()) if trg is not None else None,
                                ctypes.c_void_p(pot.data_ptr()),
                                _stream(torch), times.ctypes.data_as(_dp), ctypes.byref(bk), ctypes.byref(bn)))
    table = {(float(c[0]), int(c[1])): float(t) for c, t in zip(candidates, times)}
    return bk.value, bn.value, table


def geometry(L, dim=None, eps=1e-6, **over):
    """Host-only planning quantities for (L, eps) (no device needed)."""
    L = np.asarray(L, dtype=np.float64)
    dim = dim or L.shape[0]
    o = default_opts(dim, eps, **over)
    g = Geometry()
    Lf = _lattice(L, dim)
    _check(lib().pdmk_geometry_get(ctypes.byref(o), Lf.ctypes.data_as(_dp), ctypes.byref(g)))
    return g


def kernel_info(dim, eps):
    k = KernelInfo()
    _check(lib().pdmk_kernel_info_get(int(dim), float(eps), ctypes.byref(k)))
    return k


def residual(dim, eps, h, r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.empty_like(r)
    _check(lib().pdmk_kernel_eval_residual(int(dim), float(eps), float(h), r.size,
                                           r.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
    return out


def w0hat(dim, eps, rc, k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    out = np.empty_like(k)
    _check(lib().pdmk_kernel_eval_w0hat(int(dim), float(eps), float(rc), k.size,
                                        k.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
    return out


def _dev(t, torch, dim=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a torch tensor on the GPU")
    t = t.to(torch.float64).contiguous()
    return t


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A pdmk_plan: host tables and geometry for one (L, options) pair."""

    def __init__(self, L, dim=None, eps=1e-6, precision="fp64", grad=False,
                 allow_nonneutral=False, **over):
        L = np.asarray(L, dtype=np.float64)
        self.dim = dim or L.shape[0]
        self.opts = default_opts(self.dim, eps, precision, grad, allow_nonneutral, **over)
        self.eps = float(eps)
        self.want_grad = grad
        self._h = _vp()
        Lf = _lattice(L, self.dim)
        _check(lib().pdmk_plan_create(ctypes.byref(self.opts), Lf.ctypes.data_as(_dp),
                                      ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pdmk_plan_destroy(h)
            self._h = None

    def eval(self, src, q, trg=None, out=None, want_grad=None):
        """Potential at the targets (the sources when trg is None); with
        gradients when the plan was made with grad=True or want_grad is set
        (then returns (pot, grad))."""
        import torch
        wg = self.want_grad if want_grad is None else bool(want_grad)
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if src.shape != (n, self.dim) or q.shape != (n,):
            raise ValueError("src must be (N, dim) and q (N,)")
        if trg is not None:
            trg = _dev(trg, torch)
            m = trg.shape[0]
        else:
            m = n
        pot = torch.empty(m, dtype=torch.float64, device=src.device) if out is None else out
        grad = torch.empty((m, self.dim), dtype=torch.float64, device=src.device) \
            if wg else None
        if m == 0:   # an empty target array has no address (NULL means the sources)
            return (pot, grad) if wg else pot
        _check(lib().pdmk_plan_eval(self._h, n, ctypes.c_void_p(src.data_ptr()),
                                    ctypes.c_void_p(q.data_ptr()), m,
                                    ctypes.c_void_p(trg.data_ptr()) if trg is not None else None,
                                    ctypes.c_void_p(pot.data_ptr()),
                                    ctypes.c_void_p(grad.data_ptr()) if grad is not None else None,
                                    _stream(torch)))
        return (pot, grad) if wg else pot

    def eval_bloch(self, src, q, trg=None):
        """pdmk_plan_eval_bloch (plan made with bloch=beta): complex potential
        (torch.complex128) at the targets (the sources when trg is None)."""
        import torch
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if src.shape != (n, self.dim) or q.shape != (n,):
            raise ValueError("src must be (N, dim) and q (N,)")
        trg = _dev(trg, torch) if trg is not None else None
        m = trg.shape[0] if trg is not None else n
        out = torch.empty((m, 2), dtype=torch.float64, device=src.device)
        if m == 0:   # an empty target array has no address (NULL means the sources)
            return torch.view_as_complex(out)
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_eval_bloch(self._h, n, vp(src), vp(q), m, vp(trg), vp(out),
                                          _stream(torch)))
        return torch.view_as_complex(out)

    def eval_parts(self, src, q, trg=None):
        """pdmk_plan_eval_parts: (near, far) halves of the potential."""
        import torch
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        trg = _dev(trg, torch) if trg is not None else None
        m = trg.shape[0] if trg is not None else n
        near = torch.empty(m, dtype=torch.float64, device=src.device)
        far = torch.empty(m, dtype=torch.float64, device=src.device)
        if m == 0:   # an empty target array has no address (NULL means the sources)
            return near, far
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_eval_parts(self._h, n, vp(src), vp(q), m, vp(trg), vp(near),
                                          vp(far), _stream(torch)))
        return near, far

    def eval_noalloc(self, src, q, pot, grad=None, trg=None):
        """pdmk_plan_eval_noalloc: eval() into caller-provided outputs, with the
        library's fixed device scratch as workspace (no device allocation)."""
        import torch
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if src.shape != (n, self.dim) or q.shape != (n,):
            raise ValueError("src must be (N, dim) and q (N,)")
        trg = _dev(trg, torch) if trg is not None else None
        m = trg.shape[0] if trg is not None else n
        if pot.shape != (m,) or pot.dtype != torch.float64 or not pot.is_contiguous():
            raise ValueError("pot must be a contiguous float64 tensor of the target count")
        if grad is not None and (grad.shape != (m, self.dim) or grad.dtype != torch.float64
                                 or not grad.is_contiguous()):
            raise ValueError("grad must be a contiguous float64 (M, dim) tensor")
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_eval_noalloc(self._h, n, vp(src), vp(q), m, vp(trg), vp(pot),
                                            vp(grad), _stream(torch)))

    def bind(self, src, q, trg=None, want_grad=None):
        """pdmk_plan_bind: a full evaluation that keeps the tree for execute().
        Returns what eval() returns."""
        import torch
        wg = self.want_grad if want_grad is None else bool(want_grad)
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if src.shape != (n, self.dim) or q.shape != (n,):
            raise ValueError("src must be (N, dim) and q (N,)")
        trg = _dev(trg, torch) if trg is not None else None
        m = trg.shape[0] if trg is not None else n
        pot = torch.empty(m, dtype=torch.float64, device=src.device)
        grad = torch.empty((m, self.dim), dtype=torch.float64, device=src.device) if wg else None
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_bind(self._h, n, vp(src), vp(q), m, vp(trg), vp(pot), vp(grad),
                                    _stream(torch)))
        self._bound = (n, m)
        return (pot, grad) if wg else pot

    def execute(self, q, src=None, trg=None, out=None, grad_out=None, want_grad=None):
        """pdmk_plan_execute on the kept tree: charges q, optionally moved
        positions src / trg (frozen tree).  Enqueues only; status() waits and
        reports device-detected input errors."""
        import torch
        if getattr(self, "_bound", None) is None:
            raise ValueError("bind() first")
        n, m = self._bound
        wg = self.want_grad if want_grad is None else bool(want_grad)
        q = _dev(q, torch)
        if q.shape != (n,):
            raise ValueError("q must have the bound source count")
        if src is not None:
            src = _dev(src, torch)
            if src.shape != (n, self.dim):
                raise ValueError("src must have the bound shape")
        if trg is not None:
            trg = _dev(trg, torch)
            if trg.shape != (m, self.dim):
                raise ValueError("trg must have the bound shape")
        pot = torch.empty(m, dtype=torch.float64, device=q.device) if out is None else out
        grad = None
        if wg:
            grad = torch.empty((m, self.dim), dtype=torch.float64, device=q.device) \
                if grad_out is None else grad_out
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_execute(self._h, vp(src), vp(trg), vp(q), vp(pot), vp(grad),
                                       _stream(torch)))
        return (pot, grad) if wg else pot

    def status(self):
        """pdmk_plan_status: waits for the last execute; raises its error."""
        _check(lib().pdmk_plan_status(self._h))

    def unbind(self):
        lib().pdmk_plan_unbind(self._h)
        self._bound = None

    def adjoint(self, src, q, g, trg=None, grad_phi=None, want_dq=True, want_dsrc=True,
                want_dtrg=False):
        """pdmk_plan_adjoint: returns (dq, dsrc, dtrg) for dl/dPhi = g (entries
        not asked for are None).  grad_phi is the forward gradient."""
        import torch
        src = _dev(src, torch)
        q = _dev(q, torch)
        g = _dev(g, torch)
        n = src.shape[0]
        if trg is not None:
            trg = _dev(trg, torch)
        m = trg.shape[0] if trg is not None else n
        if g.shape != (m,):
            raise ValueError("g must have one entry per target")
        if grad_phi is not None:
            grad_phi = _dev(grad_phi, torch)
        dev = src.device
        dq = torch.empty(n, dtype=torch.float64, device=dev) if want_dq else None
        ds = torch.empty((n, self.dim), dtype=torch.float64, device=dev) if want_dsrc else None
        dt = torch.empty((m, self.dim), dtype=torch.float64, device=dev) \
            if (want_dtrg and trg is not None) else None
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_plan_adjoint(self._h, n, vp(src), vp(q), m, vp(trg), vp(g),
                                       vp(grad_phi), vp(dq), vp(ds), vp(dt), _stream(torch)))
        return dq, ds, dt

    def geometry(self):
        g = Geometry()
        _check(lib().pdmk_plan_geometry(self._h, ctypes.byref(g)))
        return g

    def stats(self):
        s = Stats()
        _check(lib().pdmk_plan_stats(self._h, ctypes.byref(s)))
        return s.as_dict()


def pdmk_eval(L, src, q, trg=None, eps=1e-6, precision="fp64", grad=False,
              allow_nonneutral=False, **over):
    """One evaluation through pdmk_eval (plan created and destroyed inside)."""
    import torch
    L = np.asarray(L, dtype=np.float64)
    dim = L.shape[0]
    o = default_opts(dim, eps, precision, grad, allow_nonneutral, **over)
    src = _dev(src, torch)
    q = _dev(q, torch)
    n = src.shape[0]
    m = trg.shape[0] if trg is not None else n
    if trg is not None:
        trg = _dev(trg, torch)
    pot = torch.empty(m, dtype=torch.float64, device=src.device)
    g = torch.empty((m, dim), dtype=torch.float64, device=src.device) if grad else None
    if m == 0:   # an empty target array has no address (NULL means the sources)
        return (pot, g) if grad else pot
    Lf = _lattice(L, dim)
    _check(lib().pdmk_eval(ctypes.byref(o), Lf.ctypes.data_as(_dp), n,
                           ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(q.data_ptr()), m,
                           ctypes.c_void_p(trg.data_ptr()) if trg is not None else None,
                           ctypes.c_void_p(pot.data_ptr()),
                           ctypes.c_void_p(g.data_ptr()) if g is not None else None,
                           _stream(torch)))
    return (pot, g) if grad else pot


class Batch:
    """A pdmk_batch: one plan per system (lattices Ls, shape (n_sys, d, d),
    columns = lattice vectors), evaluated by concurrent workers."""

    def __init__(self, Ls, eps=1e-6, precision="fp64", grad=False, allow_nonneutral=False,
                 workers=0, **over):
        Ls = np.asarray(Ls, dtype=np.float64)
        self.n_sys, self.dim = Ls.shape[0], Ls.shape[1]
        self.opts = default_opts(self.dim, eps, precision, grad, allow_nonneutral, **over)
        self.want_grad = grad
        Lf = np.ascontiguousarray(np.stack([_lattice(L, self.dim) for L in Ls]))
        self._h = _vp()
        _check(lib().pdmk_batch_create(ctypes.byref(self.opts), self.n_sys,
                                       Lf.ctypes.data_as(_dp), int(workers),
                                       ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pdmk_batch_destroy(h)
            self._h = None

    def eval(self, offsets, src, q):
        """offsets: host int array (n_sys + 1); src (N, d), q (N,) on the GPU."""
        import torch
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if off.shape != (self.n_sys + 1,):
            raise ValueError("offsets must have n_sys + 1 entries")
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if off[-1] != n or q.shape != (n,):
            raise ValueError("offsets do not match the arrays")
        pot = torch.empty(n, dtype=torch.float64, device=src.device)
        grad = torch.empty((n, self.dim), dtype=torch.float64, device=src.device) \
            if self.want_grad else None
        _check(lib().pdmk_batch_eval(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(q.data_ptr()),
                                     ctypes.c_void_p(pot.data_ptr()),
                                     ctypes.c_void_p(grad.data_ptr()) if grad is not None
                                     else None, _stream(torch)))
        return (pot, grad) if self.want_grad else pot

    def stats(self, sys):
        s = Stats()
        _check(lib().pdmk_batch_stats(self._h, int(sys), ctypes.byref(s)))
        return s.as_dict()

    def bind(self, offsets, src, q):
        """pdmk_batch_bind: one evaluation that keeps every system's tree;
        returns the potentials (and gradients with grad=True)."""
        import torch
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if off.shape != (self.n_sys + 1,):
            raise ValueError("offsets must have n_sys + 1 entries")
        src = _dev(src, torch)
        q = _dev(q, torch)
        n = src.shape[0]
        if off[-1] != n or q.shape != (n,):
            raise ValueError("offsets do not match the arrays")
        pot = torch.empty(n, dtype=torch.float64, device=src.device)
        grad = torch.empty((n, self.dim), dtype=torch.float64, device=src.device) \
            if self.want_grad else None
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_batch_bind(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     vp(src), vp(q), vp(pot), vp(grad), _stream(torch)))
        self._bound_n = n
        return (pot, grad) if self.want_grad else pot

    def execute(self, q, out=None, grad_out=None):
        """pdmk_batch_execute: new charges on the kept trees (enqueues only;
        status() waits and reports device-detected input errors)."""
        import torch
        n = getattr(self, "_bound_n", None)
        if n is None:
            raise ValueError("bind() first")
        q = _dev(q, torch)
        if q.shape != (n,):
            raise ValueError("q must have the bound size")
        pot = torch.empty(n, dtype=torch.float64, device=q.device) if out is None else out
        grad = None
        if self.want_grad:
            grad = torch.empty((n, self.dim), dtype=torch.float64, device=q.device) \
                if grad_out is None else grad_out
        vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        _check(lib().pdmk_batch_execute(self._h, vp(q), vp(pot), vp(grad), _stream(torch)))
        return (pot, grad) if self.want_grad else pot

    def status(self):
        _check(lib().pdmk_batch_status(self._h))

    def tune(self, offsets, src, q, candidates=None, trials=2):
        """Batch autotuner (pdmk_batch_tune): per size class floor(log2 n), times
        each (kappa, n_s) candidate on a sample of the class evaluated
        concurrently by the batch's workers and re-plans the class with the
        fastest.  Default candidates: kappa in {2, 3} with the default leaf
        capacity times 2^0 .. 2^9 (small cells run fastest on shallow trees).  Returns host arrays of each
        system's (kappa, n_s) after tuning."""
        import torch
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if off.shape != (self.n_sys + 1,):
            raise ValueError("offsets must have n_sys + 1 entries")
        src = _dev(src, torch)
        q = _dev(q, torch)
        if off[-1] != src.shape[0] or q.shape != (src.shape[0],):
            raise ValueError("offsets do not match the arrays")
        if candidates is None:
            base = self.opts.n_s
            candidates = [(k, base * f) for k in (2.0, 3.0) for f in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)]
        kap = np.array([float(c[0]) for c in candidates], dtype=np.float64)
        nss = (ctypes.c_int * len(candidates))(*[int(c[1]) for c in candidates])
        k_out = np.zeros(self.n_sys, dtype=np.float64)
        n_out = np.zeros(self.n_sys, dtype=np.int32)
        _check(lib().pdmk_batch_tune(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(q.data_ptr()), len(candidates),
                                     kap.ctypes.data_as(_dp), nss, int(trials), _stream(torch),
                                     k_out.ctypes.data_as(_dp),
                                     n_out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return k_out, n_out


def _autograd_fn():
    import torch

    class _PeriodicPotentialFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, src, q, trg, plan):
            need_pos = src.requires_grad or (trg is not None and trg.requires_grad)
            if need_pos:
                pot, gphi = plan.eval(src.detach(), q.detach(),
                                      trg.detach() if trg is not None else None, want_grad=True)
            else:
                pot, gphi = plan.eval(src.detach(), q.detach(),
                                      trg.detach() if trg is not None else None,
                                      want_grad=False), None
            ctx.plan = plan
            ctx.has_trg = trg is not None
            ctx.save_for_backward(src.detach(), q.detach(),
                                  trg.detach() if trg is not None else None, gphi)
            return pot

        @staticmethod
        def backward(ctx, gout):
            src, q, trg, gphi = ctx.saved_tensors
            want_dq = ctx.needs_input_grad[1]
            want_ds = ctx.needs_input_grad[0]
            want_dt = ctx.has_trg and ctx.needs_input_grad[2]
            dq, ds, dt = ctx.plan.adjoint(src, q, gout.contiguous(), trg=trg, grad_phi=gphi,
                                          want_dq=want_dq, want_dsrc=want_ds,
                                          want_dtrg=want_dt)
            return ds, dq, dt, None

    return _PeriodicPotentialFn


_FN = None


def periodic_potential(plan, src, q, trg=None):
    """Differentiable potential (torch.autograd): Phi at the targets (the
    sources when trg is None) for the plan's lattice and accuracy.  Gradients
    flow to src, q and trg through pdmk_plan_adjoint; the forward computes
    grad Phi only when a position requires grad.

    Position gradients need a plan made with grad=True (PDMK_WANT_GRAD): that
    flag widens the far-field window so that grad Phi meets the plan's
    accuracy; a plan without it raises ValueError when a position requires
    grad.  Charge gradients work with any plan."""
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    need_pos = src.requires_grad or (trg is not None and trg.requires_grad)
    if need_pos and not plan.want_grad:
        raise ValueError("position gradients need a plan made with grad=True "
                         "(PDMK_WANT_GRAD widens the far-field window for accurate gradients)")
    return _FN.apply(src, q, trg, plan)
