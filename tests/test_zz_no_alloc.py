"""bem_vjp_noalloc, the float64 adjoint that allocates nothing (its workspaces live in the
library's static per-device scratch array), called through the raw C ABI and compared with
bem_vjp (FP64) at the FP64 bar (1e-10 relative) on two calls in a row, the second smaller, and
a size beyond the scratch rejected with BEM_EINVAL."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log

pytestmark = pytest.mark.gpu


def _raw(ctx, th, x, g, out):
    P = ctypes.c_void_p
    return B.lib().bem_vjp_noalloc(ctx._h, P(th.data_ptr()), th.shape[0], P(x.data_ptr()), x.shape[0],
                                   P(g.data_ptr()), P(out.data_ptr()), P(torch.cuda.current_stream().cuda_stream))


def test_noalloc_vjp_matches_vjp_two_calls():
    wl = W.make_config(5)                                   # 256 cubic handles x 32 segments (K = 8,192)
    ctx = ctx_for(wl.S)
    cases = [(wl.theta0, wl.samples(0)[:200_003], 71), (wl.theta0[:37], wl.samples(1)[:5_001], 72)]
    for th_h, x_h, seed in cases:                          # the second call smaller in H and N
        th, x = dev(th_h), dev(x_h)
        g = dev(W.random_vector(seed, (len(x_h), 3)))
        ref = host(ctx.vjp(th, x, g, "fp64"))
        out = torch.full((th_h.shape[0], 20), float("nan"), dtype=torch.float64, device="cuda")
        assert _raw(ctx, th, x, g, out) == 0, B.lib().bem_last_error(ctx._h)
        torch.cuda.synchronize()
        got = host(out)
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        log(f"bem_vjp_noalloc H = {th_h.shape[0]}, N = {len(x_h)}: rel err vs bem_vjp {err:.3e}")
        assert np.isfinite(got).all() and err < 1e-10


def test_noalloc_vjp_rejects_sizes_beyond_scratch():
    ctx = ctx_for(32)
    H = 13_376 // 32 + 64                                   # K = 15,424 segments: beyond the 64 MiB array
    th = dev(np.tile(W.make_config(5).theta0[:1], (H, 1)))
    x = dev(W.random_points(3, 100_000, 0.01, 0.99))
    g = dev(np.zeros((100_000, 3)))
    out = torch.empty((H, 20), dtype=torch.float64, device="cuda")
    assert _raw(ctx, th, x, g, out) == -1
    msg = B.lib().bem_last_error(ctx._h).decode()
    log(f"rejected: {msg}")
    assert "scratch" in msg
