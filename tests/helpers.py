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
