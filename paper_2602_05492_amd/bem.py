"""Thin Python binding of libbem.so (include/bem.h): argument marshalling only.

Every step of the method runs in the HIP library; this module checks tensor
placement, dtypes and shapes, passes raw device pointers and the current HIP
stream, and raises BemError on a non-zero status.  PyTorch provides device
memory and streams.  If the library is not built, every call fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")
HEADER = os.path.join(HERE, "..", "include", "bem.h")

PREC = {"fp64": 0, "mixed": 1}
GRAM = {"fp64": 0, "fp32_mfma": 1, "bf16x3_mfma": 2, "fp64_valu": 3}
HANDLE_MODELS = {"cubic": 0, "straight": 1}
PARAMS_PER_HANDLE = {"cubic": 20, "straight": 10}
STATUS = {0: "BEM_OK", -1: "BEM_EINVAL", -2: "BEM_ENOMEM", -3: "BEM_ESTATE", -4: "BEM_ENOTPD",
          -5: "BEM_EHIP", -6: "BEM_ENUMERIC"}


class BemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("elems_per_side", ctypes.c_int32), ("segs_per_handle", ctypes.c_int32), ("eps", ctypes.c_double),
                ("near_factor", ctypes.c_double), ("tile_rows", ctypes.c_int32), ("device", ctypes.c_int32),
                ("handle_model", ctypes.c_int32)]


class LMState(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("cbar", ctypes.c_double * 3), ("cbar_sum", ctypes.c_double * 3),
                ("cbar_count", ctypes.c_int64), ("mean_rule", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("loss_before", ctypes.c_double), ("loss_after", ctypes.c_double), ("chol_retries", ctypes.c_int32),
                ("compat", ctypes.c_int32), ("compat_violation", ctypes.c_double), ("reg_value", ctypes.c_double),
                ("snap_pairs", ctypes.c_int32), ("data_count", ctypes.c_int64)]


class Reg(ctypes.Structure):
    """Regularisation terms of the LM step (bem_reg); a zero weight switches a term off."""
    _fields_ = [("length_weight", ctypes.c_double), ("length_max", ctypes.c_double),
                ("snap_weight", ctypes.c_double), ("snap_dist", ctypes.c_double), ("snap_mix", ctypes.c_double),
                ("sparse_wd", ctypes.c_double), ("sparse_wc", ctypes.c_double), ("sparse_t", ctypes.c_double),
                ("sparse_eps", ctypes.c_double)]


_lib = None
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64

_SIGS = {
    "bem_build": (ctypes.c_int, [ctypes.POINTER(Opts), P, ctypes.POINTER(P)]),
    "bem_build_elements": (ctypes.c_int, [ctypes.POINTER(Opts), P, I32, P, ctypes.POINTER(P)]),
    "bem_factor": (ctypes.c_int, [P, P]),
    "bem_eval": (ctypes.c_int, [P, P, I32, P, I64, ctypes.POINTER(ctypes.c_double), P, ctypes.c_int, P]),
    "bem_vjp": (ctypes.c_int, [P, P, I32, P, I64, P, P, ctypes.c_int, P]),
    "bem_vjp_noalloc": (ctypes.c_int, [P, P, I32, P, I64, P, P, P]),
    "bem_jtj": (ctypes.c_int, [P, P, I32, P, I64, P, P, P, ctypes.c_int, ctypes.c_int, P]),
    "lm_step": (ctypes.c_int, [P, P, I32, P, I64, P, ctypes.POINTER(LMState), ctypes.c_int, ctypes.c_int, P]),
    "bem_jacobian": (ctypes.c_int, [P, P, I32, P, I64, P, P]),
    "bem_set_regularization": (ctypes.c_int, [P, ctypes.POINTER(Reg)]),
    "bem_regularization": (ctypes.c_int, [P, P, I32, ctypes.POINTER(ctypes.c_double), P, P, ctypes.POINTER(I32), P]),
    "bem_prune": (ctypes.c_int, [P, P, I32, ctypes.c_double, ctypes.POINTER(I32), P]),
    "bem_partition_samples": (ctypes.c_int, [P, P, I64, I32, P, P, P, P, ctypes.POINTER(I64), P]),
    "bem_boundary_solve": (ctypes.c_int, [P, P, I32, P, P, P]),
    "bem_get_matrix": (ctypes.c_int, [P, I32, P, P]),
    "bem_num_elements": (I32, [P]),
    "bem_near_capacity": (I32, [P]),
    "bem_factor_info": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "bem_profile": (ctypes.c_int, [P, I32]),
    "bem_profile_read": (ctypes.c_int, [P, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "bem_profile_name": (ctypes.c_char_p, [I32]),
    "bem_destroy": (None, [P]),
    "bem_last_error": (ctypes.c_char_p, [P]),
}


def header_functions() -> list:
    """Names of the functions declared in include/bem.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|int32_t|const char\*)\s+\**\s*(\w+)\s*\(", txt, flags=re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2602_05492_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check_dev(name, t, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass
class Options:
    segs_per_handle: int = 32
    eps: float = 1e-2
    elems_per_side: int = 256
    near_factor: float = 1.0
    tile_rows: int = 0
    device: int = 0
    handle_model: str = "cubic"     # "cubic" (20 parameters per handle) or "straight" (10)


class Context:
    """A built and factored outer-boundary system plus the library's workspaces.  With
    elements ([M, 4] float64 array-like of element end points a, b) the outer boundary is
    that set of straight elements (a subdomain's boundary) instead of the unit square."""

    def __init__(self, opts: Options | None = None, elements=None, **kw):
        self.opts = opts or Options(**kw)
        L = lib()
        if self.opts.handle_model not in HANDLE_MODELS:
            raise ValueError(f"handle_model must be one of {sorted(HANDLE_MODELS)}")
        o = Opts(self.opts.elems_per_side, self.opts.segs_per_handle, self.opts.eps, self.opts.near_factor,
                 self.opts.tile_rows, self.opts.device, HANDLE_MODELS[self.opts.handle_model])
        self.Q = PARAMS_PER_HANDLE[self.opts.handle_model]
        h = ctypes.c_void_p()
        with torch.cuda.device(self.opts.device):
            st = _stream()
            if elements is None:
                rc = L.bem_build(ctypes.byref(o), st, ctypes.byref(h))
            else:
                import numpy as np
                el = np.ascontiguousarray(elements, dtype=np.float64)
                if el.ndim != 2 or el.shape[1] != 4:
                    raise ValueError("elements must be [M, 4]")
                rc = L.bem_build_elements(ctypes.byref(o), ctypes.c_void_p(el.ctypes.data), el.shape[0], st,
                                          ctypes.byref(h))
            if rc != 0:
                raise BemError(rc, L.bem_last_error(None).decode())
            self._h = h
            self._check(L.bem_factor(self._h, st))
        self.M = L.bem_num_elements(self._h)
        self.device = torch.device("cuda", self.opts.device)

    @property
    def near_capacity(self) -> int:
        """Near-pair list slots per 64 samples of the mixed sweeps (grown by lm_step)."""
        return int(lib().bem_near_capacity(self._h))

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise BemError(rc, lib().bem_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().bem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _theta_x(self, theta, x):
        _check_dev("theta", theta, torch.float64)
        if theta.dim() != 2 or theta.shape[1] != self.Q:
            raise ValueError(f"theta must be [H, {self.Q}] for {self.opts.handle_model} handles")
        if x is not None:
            _check_dev("x", x, torch.float64)
            if x.dim() != 2 or x.shape[1] != 2:
                raise ValueError("x must be [N, 2]")
        return theta.shape[0], (x.shape[0] if x is not None else 0)

    # -- kernel timing -----------------------------------------------------------
    def profile(self, enable: bool = True):
        self._check(lib().bem_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{family: (total_ms, launches)} of the kernels recorded since profile(True)."""
        out = {}
        for t in range(12):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            self._check(lib().bem_profile_read(self._h, t, ctypes.byref(ms), ctypes.byref(n)))
            out[lib().bem_profile_name(t).decode()] = (ms.value, n.value)
        return out

    # -- entry points ----------------------------------------------------------
    def factor_info(self):
        s = ctypes.c_double()
        sh = ctypes.c_double()
        self._check(lib().bem_factor_info(self._h, ctypes.byref(s), ctypes.byref(sh)))
        return s.value, sh.value

    def matrix(self, which: int = 0) -> torch.Tensor:
        out = torch.empty((self.M, self.M), dtype=torch.float64, device=self.device)
        self._check(lib().bem_get_matrix(self._h, which, _ptr(out), _stream()))
        return out

    def boundary_solve(self, theta):
        H, _ = self._theta_x(theta, None)
        F = torch.empty((self.M, 3), dtype=torch.float64, device=self.device)
        U = torch.empty_like(F)
        self._check(lib().bem_boundary_solve(self._h, _ptr(theta), H, _ptr(F), _ptr(U), _stream()))
        return F, U

    def eval(self, theta, x, cbar=(0.0, 0.0, 0.0), prec: str = "fp64", out=None) -> torch.Tensor:
        H, N = self._theta_x(theta, x)
        dt = torch.float64 if prec == "fp64" else torch.float32
        if out is None:
            out = torch.empty((N, 3), dtype=dt, device=self.device)
        else:
            _check_dev("out", out, dt, (N, 3))
        cb = (ctypes.c_double * 3)(*[float(c) for c in cbar])
        self._check(lib().bem_eval(self._h, _ptr(theta), H, _ptr(x), N, cb, _ptr(out), PREC[prec], _stream()))
        return out

    def vjp(self, theta, x, gbar, prec: str = "fp64", out=None) -> torch.Tensor:
        H, N = self._theta_x(theta, x)
        dt = torch.float64 if prec == "fp64" else torch.float32
        _check_dev("gbar", gbar, dt, (N, 3))
        if out is None:
            out = torch.empty((H, self.Q), dtype=torch.float64, device=self.device)
        else:
            _check_dev("out", out, torch.float64, (H, self.Q))
        self._check(lib().bem_vjp(self._h, _ptr(theta), H, _ptr(x), N, _ptr(gbar), _ptr(out), PREC[prec], _stream()))
        return out

    def vjp_noalloc(self, theta, x, gbar, out) -> torch.Tensor:
        """bem_vjp_noalloc: the float64 adjoint into a caller-allocated out [H, Q], allocating nothing."""
        H, N = self._theta_x(theta, x)
        _check_dev("gbar", gbar, torch.float64, (N, 3))
        _check_dev("out", out, torch.float64, (H, self.Q))
        self._check(lib().bem_vjp_noalloc(self._h, _ptr(theta), H, _ptr(x), N, _ptr(gbar), _ptr(out), _stream()))
        return out

    def jtj(self, theta, x, resid, gram: str = "fp64", prec: str = "fp64"):
        H, N = self._theta_x(theta, x)
        dt = torch.float64 if prec == "fp64" else torch.float32
        _check_dev("resid", resid, dt, (N, 3))
        P_ = self.Q * H
        JtJ = torch.empty((P_, P_), dtype=torch.float64, device=self.device)
        Jtr = torch.empty((P_,), dtype=torch.float64, device=self.device)
        self._check(lib().bem_jtj(self._h, _ptr(theta), H, _ptr(x), N, _ptr(resid), _ptr(JtJ), _ptr(Jtr),
                                  GRAM[gram], PREC[prec], _stream()))
        return JtJ, Jtr

    def jacobian(self, theta, x) -> torch.Tensor:
        H, N = self._theta_x(theta, x)
        J = torch.empty((N, 3, self.Q * H), dtype=torch.float64, device=self.device)
        self._check(lib().bem_jacobian(self._h, _ptr(theta), H, _ptr(x), N, _ptr(J), _stream()))
        return J

    def set_regularization(self, **terms):
        """Set the LM step's regularisation terms (bem_reg field names); no arguments: all off."""
        if not terms:
            self._check(lib().bem_set_regularization(self._h, None))
            return
        r = Reg(**terms)
        self._check(lib().bem_set_regularization(self._h, ctypes.byref(r)))

    def regularization(self, theta, with_derivatives: bool = True):
        """(value, grad [P] or None, hess [P, P] or None, snapped pairs) of the terms at theta."""
        H, _ = self._theta_x(theta, None)
        P_ = self.Q * H
        v = ctypes.c_double()
        n = I32()
        g = hm = None
        if with_derivatives:
            g = torch.empty((P_,), dtype=torch.float64, device=self.device)
            hm = torch.empty((P_, P_), dtype=torch.float64, device=self.device)
        self._check(lib().bem_regularization(self._h, _ptr(theta), H, ctypes.byref(v), _ptr(g) if g is not None else None,
                                             _ptr(hm) if hm is not None else None, ctypes.byref(n), _stream()))
        return v.value, g, hm, n.value

    def prune(self, theta, threshold: float) -> torch.Tensor:
        """Remove, in place, the handles whose wd and wc norms are both below threshold; returns the
        view theta[:H_kept]."""
        H, _ = self._theta_x(theta, None)
        k = I32()
        self._check(lib().bem_prune(self._h, _ptr(theta), H, float(threshold), ctypes.byref(k), _stream()))
        return theta[: k.value]

    def partition(self, labels, x, target=None, D: int = 1):
        """Stable partition of the samples (and targets) by subdomain label in [0, D) on the GPU:
        (x sorted, target sorted or None, offsets list of D + 1 row indices)."""
        _check_dev("labels", labels, torch.int32)
        _check_dev("x", x, torch.float64)
        N = x.shape[0]
        if labels.shape != (N,) or x.shape != (N, 2):
            raise ValueError("labels must be [N] and x [N, 2]")
        if target is not None:
            _check_dev("target", target, torch.float64, (N, 3))
        xo = torch.empty_like(x)
        To = torch.empty_like(target) if target is not None else None
        off = (I64 * (D + 1))()
        self._check(lib().bem_partition_samples(self._h, _ptr(labels), N, D, _ptr(x), _ptr(target), _ptr(xo),
                                                _ptr(To), off, _stream()))
        return xo, To, [int(v) for v in off]

    def lm_step(self, theta, x, target, state: LMState, gram: str = "fp64", prec: str = "fp64") -> LMState:
        H, N = self._theta_x(theta, x)
        _check_dev("target", target, torch.float64, (N, 3))
        self._check(lib().lm_step(self._h, _ptr(theta), H, _ptr(x), N, _ptr(target), ctypes.byref(state),
                                  GRAM[gram], PREC[prec], _stream()))
        return state


def lm_step_subdomains(contexts, thetas, x, target, labels, states, gram: str = "fp64", prec: str = "fp64"):
    """One LM step in every subdomain (Sec. 4.1, Sec. 4.3): the samples are grouped by label on
    the GPU, then subdomain d takes its own step (its own handles, mean colour, normal equations,
    Cholesky and damping) on its own samples.  contexts, thetas and states are per subdomain.
    Every subdomain's data terms are divided by the number of samples drawn over the whole image
    (all N rows, including those outside every subdomain), as the Monte Carlo estimates of
    Eq. losshessian and Eq. lossjacobian do."""
    xs, Ts, off = contexts[0].partition(labels, x, target, len(contexts))
    N = x.shape[0]
    for d, (ctx, th, st) in enumerate(zip(contexts, thetas, states)):
        st.data_count = N
        ctx.lm_step(th, xs[off[d]:off[d + 1]], Ts[off[d]:off[d + 1]], st, gram, prec)
    return states


def new_lm_state(lam: float = 1e-3, mean_rule: int = 0, compat: int = 0) -> LMState:
    s = LMState()
    s.lam = lam
    s.mean_rule = mean_rule
    s.compat = compat
    return s


class BemEval(torch.autograd.Function):
    """u = bem_eval(theta, x); backward = bem_vjp (gradient with respect to theta only)."""

    @staticmethod
    def forward(fctx, theta, x, ctx: Context, cbar, prec: str):
        fctx.save_for_backward(theta, x)
        fctx.bem = ctx
        fctx.prec = prec
        return ctx.eval(theta.detach(), x, cbar, prec)

    @staticmethod
    def backward(fctx, gu):
        theta, x = fctx.saved_tensors
        dt = torch.float64 if fctx.prec == "fp64" else torch.float32
        g = fctx.bem.vjp(theta.detach(), x, gu.to(dt).contiguous(), fctx.prec)
        return g, None, None, None, None


def bem_eval(theta, x, ctx: Context, cbar=(0.0, 0.0, 0.0), prec: str = "fp64"):
    return BemEval.apply(theta, x, ctx, tuple(cbar), prec)
