"""Python binding of libfftpim.so (the C ABI in include/fftpim.h).

Argument marshalling only: every step of the apply runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  Importing
this module does not build anything; if the shared library is missing every
call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfftpim.so")

F64, F32, F32_FARBF16, F32_FARBF16X3 = 0, 1, 2, 3
REAL, COMPLEX = 0, 1
SELF_IMAGES, SELF_EXCLUDE = 0, 1
ORDER_USER, ORDER_PLAN = 0, 1
PART_NEAR_GRID, PART_NEAR_CORR, PART_FAR, PART_ALL = 1, 2, 4, 7

STATUS = {
    0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_CELL", 3: "NOT_NEUTRAL", 4: "WOOD_ANOMALY",
    5: "UNSUPPORTED", 6: "NO_MEMORY", 7: "DEVICE", 8: "UNIMPLEMENTED", 9: "SCRATCH_LIMIT",
}

# the entry points declared in include/fftpim.h
EXPORTS = (
    "fftpim_default_params", "fftpim_plan", "fftpim_apply", "fftpim_apply_adjoint",
    "fftpim_apply_pair", "fftpim_apply_parts", "fftpim_get_permutation", "fftpim_plan_info", "fftpim_last_status",
    "fftpim_destroy", "fftpim_error_string", "fftpim_eval_pgf", "fftpim_stage_times", "fftpim_eval_pgf_self",
    "fftpim_apply_pair_noalloc", "fftpim_grad_positions", "fftpim_autotune", "fftpim_batch_create",
    "fftpim_batch_apply", "fftpim_batch_destroy",
)
STAGES = ("pack", "near_spread", "near_fft", "near_interp", "near_corr", "far", "unpack")


class FFTPIMError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__("%s failed: %s (%d)" % (where, self.name, code))


class Problem(ctypes.Structure):
    _fields_ = [("periodic_dims", ctypes.c_int), ("L", ctypes.c_double * 3), ("k0", ctypes.c_double),
                ("kt", ctypes.c_double * 3), ("has_box", ctypes.c_int), ("box_lo", ctypes.c_double * 3),
                ("box_hi", ctypes.c_double * 3), ("k0_im", ctypes.c_double), ("kt_im", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("near_n", ctypes.c_int * 3), ("near_order", ctypes.c_int), ("corr_radius", ctypes.c_int),
                ("far_n", ctypes.c_int * 3), ("far_order", ctypes.c_int), ("n_images", ctypes.c_int),
                ("precision", ctypes.c_int), ("value_type", ctypes.c_int), ("self_mode", ctypes.c_int),
                ("order_io", ctypes.c_int), ("nrhs_max", ctypes.c_int), ("corr_layout", ctypes.c_int),
                ("max_bytes", ctypes.c_size_t), ("corr_ball", ctypes.c_double), ("far_sum", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_obs", ctypes.c_int64), ("near_n", ctypes.c_int * 3),
                ("near_fft", ctypes.c_int * 3), ("near_cells", ctypes.c_int * 3), ("near_h", ctypes.c_double * 3),
                ("domain_lo", ctypes.c_double * 3), ("domain_hi", ctypes.c_double * 3),
                ("far_n", ctypes.c_int * 3), ("far_cells", ctypes.c_int * 3), ("far_h", ctypes.c_double * 3),
                ("corr_nnz", ctypes.c_int64), ("corr_sym_values", ctypes.c_int64), ("corr_csr_nnz", ctypes.c_int64),
                ("corr_tile_values", ctypes.c_int64),
                ("corr_value_bytes", ctypes.c_int), ("corr_layout_used", ctypes.c_int),
                ("device_bytes", ctypes.c_int64), ("nplanes_max", ctypes.c_int),
                ("plan_seconds", ctypes.c_double), ("far_fft", ctypes.c_int * 3)]


class TuneReport(ctypes.Structure):
    _fields_ = [("predicted_rel_err", ctypes.c_double), ("predicted_ms", ctypes.c_double),
                ("predicted_corr_nnz", ctypes.c_int64), ("candidates", ctypes.c_int)]


_lib = None


def lib():
    """Load libfftpim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfftpim.so is not built; run `python -m paper_2312_02376_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.fftpim_default_params.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params)]
        L.fftpim_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Problem), ctypes.POINTER(Params), i64, vp,
                                  i64, vp, vp]
        L.fftpim_apply.argtypes = [vp, vp, vp, ci, vp]
        L.fftpim_apply_adjoint.argtypes = [vp, vp, vp, ci, vp]
        L.fftpim_apply_pair.argtypes = [vp, vp, vp, vp, vp, ci, vp]
        L.fftpim_apply_pair_noalloc.argtypes = [vp, vp, vp, vp, vp, ci, vp]
        L.fftpim_grad_positions.argtypes = [vp, vp, vp, ci, vp, vp]
        L.fftpim_apply_parts.argtypes = [vp, ci, ci, vp, vp, ci, vp]
        L.fftpim_get_permutation.argtypes = [vp, ci, vp]
        L.fftpim_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.fftpim_last_status.argtypes = [vp]
        L.fftpim_destroy.argtypes = [vp]
        L.fftpim_error_string.argtypes = [ci]
        L.fftpim_error_string.restype = ctypes.c_char_p
        L.fftpim_eval_pgf.argtypes = [ctypes.POINTER(Problem), i64, vp, vp]
        L.fftpim_stage_times.argtypes = [vp, ci, vp, vp]
        L.fftpim_eval_pgf_self.argtypes = [ctypes.POINTER(Problem), vp]
        L.fftpim_autotune.argtypes = [ctypes.POINTER(Problem), i64, vp, ctypes.c_double, ci, ci,
                                      ctypes.POINTER(Params), ctypes.POINTER(TuneReport)]
        L.fftpim_batch_create.argtypes = [ctypes.POINTER(vp), vp, ci, ci, ci]
        L.fftpim_batch_apply.argtypes = [vp, vp, vp, vp, ci, vp]
        L.fftpim_batch_destroy.argtypes = [vp]
        for name in EXPORTS:
            if name != "fftpim_error_string":
                getattr(L, name).restype = ci
        _lib = L
    return _lib


def _check(code, where):
    if code != 0:
        raise FFTPIMError(code, where)


def make_problem(periodic_dims, L, k0=0.0, kt=(0.0, 0.0, 0.0), box=None):
    pr = Problem()
    pr.periodic_dims = int(periodic_dims)
    Lv = list(np.broadcast_to(np.asarray(L, float), (3,))) if np.ndim(L) == 0 else list(L) + [1.0] * (3 - len(L))
    for c in range(3):
        pr.L[c] = float(Lv[c])
        k = complex(kt[c]) if c < len(kt) else 0j
        pr.kt[c] = k.real
        pr.kt_im[c] = k.imag
    pr.k0 = complex(k0).real
    pr.k0_im = complex(k0).imag
    if box is not None:
        pr.has_box = 1
        for c in range(3):
            pr.box_lo[c] = float(box[0][c])
            pr.box_hi[c] = float(box[1][c])
    return pr


def eval_pgf(r, periodic_dims, L, k0=0.0, kt=(0.0, 0.0, 0.0)):
    """The library's host evaluator of G^p (used for the far-zone table) at
    host points r (n, 3); returns complex128 (n,).  No GPU is touched."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1, 3))
    out = np.empty((r.shape[0], 2))
    pr = make_problem(periodic_dims, L, k0, kt)
    _check(lib().fftpim_eval_pgf(ctypes.byref(pr), r.shape[0], r.ctypes.data, out.ctypes.data), "fftpim_eval_pgf")
    return out[:, 0] + 1j * out[:, 1]


def eval_pgf_self(periodic_dims, L, k0=0.0, kt=(0.0, 0.0, 0.0)):
    """The library's lim_{r->0}[G^p(r) - G0(r)] (host only)."""
    out = np.empty(2)
    pr = make_problem(periodic_dims, L, k0, kt)
    _check(lib().fftpim_eval_pgf_self(ctypes.byref(pr), out.ctypes.data), "fftpim_eval_pgf_self")
    return complex(out[0], out[1])


def _overlap(a, b):
    """True when the memory spans of two dense tensors intersect."""
    if a.device != b.device:
        return False
    a0, b0 = a.data_ptr(), b.data_ptr()
    a1 = a0 + a.numel() * a.element_size()
    b1 = b0 + b.numel() * b.element_size()
    return a0 < b1 and b0 < a1


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """An FFT-PIM plan over coinciding sources and observers.

    positions: torch CUDA float64 tensor (N, 3) in the zeroth cell.
    The remaining arguments map one-to-one onto fftpim_problem_t and
    fftpim_params_t (include/fftpim.h); precision is "f64", "f32",
    "f32_farbf16" (FP32 with a bfloat16-input far grid sum) or
    "f32_farbf16x3" (the same with split three-product bfloat16 terms);
    far_sum is "auto", "direct" or "fft" (the far grid sum of Eq. (8)).
    """

    def __init__(self, positions, periodic_dims, L, k0=0.0, kt=(0.0, 0.0, 0.0), near_n=(16, 16, 16),
                 near_order=4, corr_radius=6, far_n=(16, 16, 16), far_order=7, n_images=1, precision="f64",
                 value_type="complex", order="user", nrhs_max=1, box=None, self_mode="images",
                 corr_layout="auto", max_bytes=0, corr_ball=0.0, far_sum="auto", observers=None, stream=None):
        import torch
        if not (isinstance(positions, torch.Tensor) and positions.is_cuda and positions.dtype == torch.float64):
            raise TypeError("positions must be a CUDA float64 tensor of shape (N, 3)")
        pos = positions.contiguous()
        self.N = int(pos.shape[0])
        obs = None
        if observers is not None:
            if not (isinstance(observers, torch.Tensor) and observers.is_cuda and observers.dtype == torch.float64):
                raise TypeError("observers must be a CUDA float64 tensor of shape (M, 3)")
            obs = observers.contiguous()
        self.M = self.N if obs is None else int(obs.shape[0])
        self.problem = make_problem(periodic_dims, L, k0, kt, box)
        pm = Params()
        for c in range(3):
            pm.near_n[c] = int(np.broadcast_to(near_n, (3,))[c])
            pm.far_n[c] = int(np.broadcast_to(far_n, (3,))[c])
        pm.near_order = int(near_order)
        pm.corr_radius = int(corr_radius)
        pm.far_order = int(far_order)
        pm.n_images = int(n_images)
        pm.precision = {"f64": F64, "f32": F32, "f32_farbf16": F32_FARBF16,
                        "f32_farbf16x3": F32_FARBF16X3}[precision]
        pm.value_type = {"real": REAL, "complex": COMPLEX}[value_type]
        pm.self_mode = {"images": SELF_IMAGES, "exclude": SELF_EXCLUDE}[self_mode]
        pm.order_io = {"user": ORDER_USER, "plan": ORDER_PLAN}[order]
        pm.nrhs_max = int(nrhs_max)
        pm.corr_layout = {"auto": 0, "csr": 1, "sym": 2, "tile": 3}[corr_layout]
        pm.max_bytes = int(max_bytes)
        pm.corr_ball = float(corr_ball)
        pm.far_sum = {"auto": 0, "direct": 1, "fft": 2}[far_sum]
        self.params = pm
        self.precision = precision
        self.value_type = value_type
        if precision == "f64":
            self.dtype = torch.float64 if value_type == "real" else torch.complex128
        else:
            self.dtype = torch.float32 if value_type == "real" else torch.complex64
        self.device = pos.device
        h = ctypes.c_void_p()
        _check(lib().fftpim_plan(ctypes.byref(h), ctypes.byref(self.problem), ctypes.byref(pm), self.N,
                                 ctypes.c_void_p(pos.data_ptr()), 0 if obs is None else self.M,
                                 None if obs is None else ctypes.c_void_p(obs.data_ptr()), _stream_handle(stream)),
               "fftpim_plan")
        self._h = h

    def _io(self, x, out, adjoint=False):
        """Checks an input of the sources (observers when adjoint) and an
        output of the observers (sources when adjoint)."""
        import torch
        n_in, n_out = (self.M, self.N) if adjoint else (self.N, self.M)
        if not isinstance(x, torch.Tensor) or x.dtype != self.dtype or x.device != self.device:
            raise TypeError("expected a %s tensor on %s" % (self.dtype, self.device))
        squeeze = x.dim() == 1
        x2 = x.reshape(1, -1) if squeeze else x
        if x2.shape[1] != n_in:
            raise ValueError("expected %d points, got %d" % (n_in, x2.shape[1]))
        x2 = x2.contiguous()
        if out is None:
            out = torch.empty((x2.shape[0], n_out), dtype=x2.dtype, device=x2.device)
        else:
            # the library writes nrhs x N elements through out's pointer:
            # accept only a tensor that holds exactly that, densely
            if not isinstance(out, torch.Tensor) or out.dtype != self.dtype:
                raise TypeError("out must be a %s tensor" % self.dtype)
            if out.device != self.device:
                raise ValueError("out is on %s, the plan on %s" % (out.device, self.device))
            o2 = out.reshape(1, -1) if (squeeze and out.dim() == 1) else out
            want = (x2.shape[0], n_out)
            if tuple(o2.shape) != want:
                raise ValueError("out has shape %s, expected %s" % (tuple(out.shape),
                                                                   (n_out,) if squeeze else want))
            if not out.is_contiguous():
                raise ValueError("out must be contiguous")
            if _overlap(out, x2):
                raise ValueError("out must not overlap the input")
            out = o2
        return x2, out, squeeze

    def apply(self, q, out=None, stream=None):
        """u = A q, q of shape (nrhs, N) or (N,)."""
        q2, out, sq = self._io(q, out)
        _check(lib().fftpim_apply(self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  q2.shape[0], _stream_handle(stream)), "fftpim_apply")
        return out[0] if sq else out

    def adjoint(self, v, out=None, stream=None):
        """w = A^H v (mean removed for the neutral static case)."""
        v2, out, sq = self._io(v, out, adjoint=True)
        _check(lib().fftpim_apply_adjoint(self._h, ctypes.c_void_p(v2.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          v2.shape[0], _stream_handle(stream)), "fftpim_apply_adjoint")
        return out[0] if sq else out

    def apply_pair(self, q, v, out_u=None, out_w=None, stream=None):
        """(A q, A^H v) in one call; q and v of the same shape."""
        q2, out_u, sq = self._io(q, out_u)
        v2, out_w, _ = self._io(v, out_w)
        if v2.shape != q2.shape:
            raise ValueError("q and v must have the same shape")
        if _overlap(out_u, out_w) or _overlap(out_u, v2) or _overlap(out_w, q2):
            raise ValueError("out_u and out_w must not overlap each other or the inputs")
        _check(lib().fftpim_apply_pair(self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(out_u.data_ptr()),
                                       ctypes.c_void_p(v2.data_ptr()), ctypes.c_void_p(out_w.data_ptr()),
                                       q2.shape[0], _stream_handle(stream)), "fftpim_apply_pair")
        return (out_u[0], out_w[0]) if sq else (out_u, out_w)

    def apply_pair_noalloc(self, q, v, out_u, out_w, stream=None):
        """apply_pair through the entry point that allocates nothing: the
        outputs must be given, and the pair's work arrays come from the
        library's fixed per-device array."""
        if out_u is None or out_w is None:
            raise ValueError("apply_pair_noalloc needs out_u and out_w")
        q2, out_u, sq = self._io(q, out_u)
        v2, out_w, _ = self._io(v, out_w)
        if v2.shape != q2.shape:
            raise ValueError("q and v must have the same shape")
        if _overlap(out_u, out_w) or _overlap(out_u, v2) or _overlap(out_w, q2):
            raise ValueError("out_u and out_w must not overlap each other or the inputs")
        _check(lib().fftpim_apply_pair_noalloc(self._h, ctypes.c_void_p(q2.data_ptr()),
                                               ctypes.c_void_p(out_u.data_ptr()), ctypes.c_void_p(v2.data_ptr()),
                                               ctypes.c_void_p(out_w.data_ptr()), q2.shape[0],
                                               _stream_handle(stream)), "fftpim_apply_pair_noalloc")
        return (out_u[0], out_w[0]) if sq else (out_u, out_w)

    def grad_positions(self, q, g, out=None, stream=None):
        """dL/dr (N, 3) float64 for L = Re sum conj(g) (A q) (real values:
        sum g (A q)), q and g of shape (nrhs, N) or (N,)."""
        import torch
        q2 = self._in(q)
        g2 = self._in(g)
        if g2.shape != q2.shape:
            raise ValueError("q and g must have the same shape")
        if out is None:
            out = torch.empty((self.N, 3), dtype=torch.float64, device=self.device)
        elif (out.dtype != torch.float64 or out.device != self.device or tuple(out.shape) != (self.N, 3)
              or not out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 (N, 3) tensor on the plan's device")
        _check(lib().fftpim_grad_positions(self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(g2.data_ptr()),
                                           q2.shape[0], ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "fftpim_grad_positions")
        return out

    def _in(self, x):
        x2, _, _ = self._io(x, None)
        return x2

    def apply_parts(self, q, parts, adjoint=False, out=None, stream=None):
        q2, out, sq = self._io(q, out, adjoint=adjoint)
        _check(lib().fftpim_apply_parts(self._h, int(parts), 1 if adjoint else 0, ctypes.c_void_p(q2.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), q2.shape[0], _stream_handle(stream)),
               "fftpim_apply_parts")
        return out[0] if sq else out

    def permutation(self, observers=False):
        """Plan-order position -> caller index, of the sources or (with
        observers=True) of the observers."""
        import torch
        n = self.M if observers else self.N
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        _check(lib().fftpim_get_permutation(self._h, 1 if observers else 0, ctypes.c_void_p(perm.data_ptr())),
               "fftpim_get_permutation")
        return perm

    def info(self):
        inf = Info()
        _check(lib().fftpim_plan_info(self._h, ctypes.byref(inf)), "fftpim_plan_info")
        return {f: (list(getattr(inf, f)) if hasattr(getattr(inf, f), "__len__") else getattr(inf, f))
                for f, _ in Info._fields_}

    def stage_times(self, enable):
        """Start (enable=True) or stop per-stage HIP-event timing; returns
        {stage: (total_ms, launches)} accumulated since timing was started."""
        ms = np.zeros(len(STAGES))
        calls = np.zeros(len(STAGES), dtype=np.int64)
        _check(lib().fftpim_stage_times(self._h, 1 if enable else 0, ms.ctypes.data, calls.ctypes.data),
               "fftpim_stage_times")
        return {s: (float(ms[i]), int(calls[i])) for i, s in enumerate(STAGES)}

    def last_status(self):
        return int(lib().fftpim_last_status(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().fftpim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class FFTPIMFunction(torch.autograd.Function):
        """u = A q with dL/dq = A^H dL/du: the backward pass is the library's
        conjugate-transpose apply (for a real loss of complex u, PyTorch's
        gradient convention makes the gradient of q exactly A^H times the
        gradient of u; for real static kernels A^H = A^T).  When positions
        are given and require a gradient, the backward pass also returns
        dL/dr from fftpim_grad_positions (the plan must have been made from
        those positions)."""

        @staticmethod
        def forward(ctx, q, positions, plan):
            ctx.plan = plan
            ctx.save_for_backward(q)
            return plan.apply(q)

        @staticmethod
        def backward(ctx, gu):
            (q,) = ctx.saved_tensors
            gu = gu.contiguous()
            gq = ctx.plan.adjoint(gu) if ctx.needs_input_grad[0] else None
            gpos = None
            if ctx.needs_input_grad[1]:
                gpos = ctx.plan.grad_positions(q.detach().contiguous(), gu)
            return gq, gpos, None

    return FFTPIMFunction


_FN = None


def apply_autograd(plan, q, positions=None):
    """Differentiable u = A q for a Plan: gradients with respect to the
    amplitudes q and, when `positions` (the tensor the plan was made from)
    requires a gradient, with respect to the positions."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(q, positions, plan)


_PRECISIONS = {"f64": F64, "f32": F32, "f32_farbf16": F32_FARBF16, "f32_farbf16x3": F32_FARBF16X3}


def autotune(positions, periodic_dims, L, target, k0=0.0, kt=(0.0, 0.0, 0.0), precision="f64", nrhs=1,
             value_type="complex", box=None):
    """fftpim_autotune: the cost-model parameter choice for a target relative
    error.  Returns (kwargs for Plan, report dict)."""
    import torch
    if not (isinstance(positions, torch.Tensor) and positions.is_cuda and positions.dtype == torch.float64):
        raise TypeError("positions must be a CUDA float64 tensor of shape (N, 3)")
    pos = positions.contiguous()
    pr = make_problem(periodic_dims, L, k0, kt, box)
    pm = Params()
    _check(lib().fftpim_default_params(ctypes.byref(pr), ctypes.byref(pm)), "fftpim_default_params")
    pm.value_type = {"real": REAL, "complex": COMPLEX}[value_type]
    rep = TuneReport()
    _check(lib().fftpim_autotune(ctypes.byref(pr), int(pos.shape[0]), ctypes.c_void_p(pos.data_ptr()), float(target),
                                 _PRECISIONS[precision], int(nrhs), ctypes.byref(pm), ctypes.byref(rep)),
           "fftpim_autotune")
    kw = dict(near_n=tuple(pm.near_n), near_order=pm.near_order, corr_radius=pm.corr_radius,
              corr_ball=pm.corr_ball, far_n=tuple(pm.far_n), far_order=pm.far_order, n_images=pm.n_images,
              precision=precision, value_type=value_type, nrhs_max=max(1, pm.nrhs_max))
    report = {f: getattr(rep, f) for f, _ in TuneReport._fields_}
    return kw, report


class Batch:
    """fftpim_batch_*: several plans applied together (the plans are not
    owned and must outlive the batch)."""

    def __init__(self, plans, lanes=4, graph=False):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().fftpim_batch_create(ctypes.byref(h), arr, len(self.plans), int(lanes), 1 if graph else 0),
               "fftpim_batch_create")
        self._h = h

    def apply(self, xs, outs=None, adjoint=False, stream=None):
        import torch
        if len(xs) != len(self.plans):
            raise ValueError("one input per cell")
        ins, os_, nr = [], [], []
        made = []
        for c, (pl, x) in enumerate(zip(self.plans, xs)):
            x2, out, squeeze = pl._io(x, None if outs is None else outs[c])
            made.append((x2, out, squeeze))
            ins.append(x2.data_ptr())
            os_.append(out.data_ptr())
            nr.append(int(x2.shape[0]))
        n = len(self.plans)
        ia = (ctypes.c_void_p * n)(*ins)
        oa = (ctypes.c_void_p * n)(*os_)
        ra = (ctypes.c_int * n)(*nr)
        _check(lib().fftpim_batch_apply(self._h, ia, oa, ra, 1 if adjoint else 0, _stream_handle(stream)),
               "fftpim_batch_apply")
        self._keep = made  # inputs stay alive until the caller synchronises
        return [o.reshape(-1) if sq else o for (_, o, sq) in made]

    def close(self):
        if getattr(self, "_h", None):
            lib().fftpim_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
