"""Shared helpers of the GPU tests: contexts, device copies, error metrics."""
import functools
import sys

import numpy as np


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@functools.lru_cache(maxsize=None)
def ctx_for(S: int, eps: float = 1e-2, per_side: int = 256, near_factor: float = 1.0, tile_rows: int = 0,
            handle_model: str = "cubic"):
    from paper_2602_05492_amd import bem as B
    return B.Context(segs_per_handle=S, eps=eps, elems_per_side=per_side, near_factor=near_factor,
                     tile_rows=tile_rows, handle_model=handle_model)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_err(got, ref):
    """max |got - ref| / max(1, max |ref|)"""
    return float(np.abs(got - ref).max() / max(1.0, np.abs(ref).max())) if np.size(ref) else 0.0


def mixed_step_tol(JtJ, lam, extra=None):
    """Bar on max|delta - delta_oracle| / max|delta_oracle| for a mixed-precision LM step.

    The mixed path differs from the oracle by float32 rounding (u = 2^-24) in the features, the
    residuals and the Gram's accumulation, a relative perturbation of the damped normal equations
    (lam D + H) delta = g that the diagonally scaled system amplifies by its condition number
    kappa.  The measured step errors are 1.2e-7 kappa to 1.5e-7 kappa (about 2 u kappa: 1.1e-5 at
    kappa = 84, 8.7e-4 at kappa = 7.7e3); the bar is 10 u kappa.  JtJ is the oracle's
    (1/N) sum J^T J at the step's parameters, extra an added Hessian (regularisation terms)."""
    H = np.asarray(JtJ, dtype=np.float64) + (0.0 if extra is None else extra)
    d = np.diag(H).copy()
    d = np.maximum(d, 1e-12 * max(d.max(), 1e-300))      # the damping D = diag of the whole Hessian
    Hd = H + lam * np.diag(d)
    s = 1.0 / np.sqrt(np.diag(Hd))
    kappa = float(np.linalg.cond(Hd * s[:, None] * s[None, :]))
    return 10.0 * kappa * 2.0 ** -24
