"""GPU forward path (bem_build, bem_factor, bem_eval, bem_boundary_solve) against the FP64 oracle.

Bars: FP64 path within 1e-10 relative; mixed path within 1e-4 absolute in colour.
Workloads are the seeded tiny / medium / near-singular / LM-sized handle sets.
"""
import numpy as np
import pytest

import oracle as O
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def test_matrix_and_pseudo_inverse_match_oracle():
    ctx = ctx_for(32)
    bnd = O.boundary(256)
    A = host(ctx.matrix(0))
    assert np.abs(A - bnd.A).max() <= 1e-15 * np.abs(bnd.A).max()
    Ap = host(ctx.matrix(1))
    err = np.abs(Ap - bnd.Apinv).max() / np.abs(bnd.Apinv).max()
    log("pinv rel err", err)
    assert err < 1e-11
    sig, shift = ctx.factor_info()
    s = np.linalg.svd(bnd.A, compute_uv=False)
    assert abs(sig - s[-1]) < 1e-8 * s[-1]
    assert s[-2] <= shift <= s[0]


def test_boundary_rhs_and_values_tiny():
    wl = W.make_config(1)
    ctx = ctx_for(wl.S)
    F, U = ctx.boundary_solve(dev(wl.theta_true))
    bnd = O.boundary(256)
    Fo = O.boundary_rhs(wl.theta_true, wl.S, wl.eps, bnd)
    Uo = bnd.Apinv @ Fo
    assert np.abs(host(F) - Fo).max() < 1e-13 * np.abs(Fo).max()
    assert np.abs(host(U) - Uo).max() < 1e-11 * np.abs(Uo).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_eval_tiny_full(prec):
    wl = W.make_config(1)
    ctx = ctx_for(wl.S)
    x = wl.samples(0)
    u = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, prec))
    uo = O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps)
    err = np.abs(u - uo).max()
    log(prec, "tiny max abs err", err)
    assert err < (FP64_TOL * max(1, np.abs(uo).max()) if prec == "fp64" else MIXED_TOL)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_eval_medium_subsample(prec):
    wl = W.make_config(2)
    ctx = ctx_for(wl.S)
    x = wl.samples(0)
    idx = wl.subsample(3000)
    u = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, prec))
    uo = O.evaluate(wl.theta_true, x[idx], wl.cbar_true, wl.S, wl.eps)
    err = np.abs(u[idx] - uo).max()
    log(prec, "medium max abs err", err)
    assert err < (FP64_TOL * max(1, np.abs(uo).max()) if prec == "fp64" else MIXED_TOL)


def test_eval_near_singular_mixed():
    """10% of the samples within 1e-3 of a segment: mixed error, split near / far."""
    wl = W.make_config(3)
    ctx = ctx_for(wl.S)
    x = wl.samples(0)
    n_near = int(round(0.1 * wl.N))
    idx_far = wl.subsample(600, wl.N - n_near)
    idx_near = (wl.N - n_near) + wl.subsample(600, n_near, step=1)
    idx = np.concatenate([idx_far, idx_near])
    u = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, "mixed"))
    u64 = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, "fp64"))
    uo = O.evaluate(wl.theta_true, x[idx], wl.cbar_true, wl.S, wl.eps)
    e_far = np.abs(u[idx_far] - uo[:600]).max()
    e_near = np.abs(u[idx_near] - uo[600:]).max()
    log(f"near-singular workload: mixed err far {e_far:.3e} near {e_near:.3e}; "
        f"fp64 err {np.abs(u64[idx] - uo).max():.3e}; mixed vs fp64 over all N {np.abs(u - u64).max():.3e}")
    assert max(e_far, e_near) < MIXED_TOL
    assert np.abs(u64[idx] - uo).max() < FP64_TOL * max(1, np.abs(uo).max())
    assert np.abs(u - u64).max() < MIXED_TOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_eval_lm_workload_full_size_sampled(prec):
    """Full-size LM workload (256 handles x 32 segments, 2,097,152 samples): sampled outputs vs the oracle."""
    wl = W.make_config(5)
    ctx = ctx_for(wl.S)
    x = wl.samples(0)
    u = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, prec))
    idx = wl.subsample(96)
    idx = np.concatenate([idx, [0, wl.N - 1]])
    uo = O.evaluate(wl.theta_true, x[idx], wl.cbar_true, wl.S, wl.eps)
    err = np.abs(u[idx] - uo).max()
    log(prec, "LM workload sampled max abs err", err)
    assert np.isfinite(u).all()
    assert err < (FP64_TOL * max(1, np.abs(uo).max()) if prec == "fp64" else MIXED_TOL)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_edge_cases(prec):
    ctx = ctx_for(8)
    theta = W.random_handles(21, 3)
    # empty sample set
    out = ctx.eval(dev(theta), dev(np.zeros((0, 2))), (0.1, 0.2, 0.3), prec)
    assert out.shape == (0, 3)
    # no handles: u = cbar
    x = W.random_points(21, 1000)
    u = host(ctx.eval(dev(np.zeros((0, 20))), dev(x), (0.1, 0.2, 0.3), prec))
    assert np.allclose(u, [0.1, 0.2, 0.3], atol=1e-7 if prec == "mixed" else 0)
    # ragged N, samples hugging the outer boundary, a zero-length handle
    th = theta.copy()
    th[1, :8] = np.tile(th[1, :2], 4)
    xb = np.array([[1e-7, 0.5], [0.5, 1 - 1e-7], [1 - 1e-6, 1e-6], [0.3, 2e-7]])
    xx = np.concatenate([x[:997], xb])
    u = host(ctx.eval(dev(th), dev(xx), (0.0, 0.0, 0.0), prec))
    uo = O.evaluate(th, xx, np.zeros(3), 8, 1e-2)
    err = np.abs(u - uo).max()
    log(prec, "edge max abs err", err)
    assert err < (FP64_TOL if prec == "fp64" else MIXED_TOL)


def test_fp64_is_deterministic():
    wl = W.make_config(2)
    ctx = ctx_for(wl.S)
    x = dev(wl.samples(0)[:50000])
    th = dev(wl.theta_true)
    a = host(ctx.eval(th, x, wl.cbar_true, "fp64"))
    b = host(ctx.eval(th, x, wl.cbar_true, "fp64"))
    assert np.array_equal(a, b)


def test_call_order_and_argument_errors():
    import ctypes
    import torch
    from paper_2602_05492_amd import bem as B
    L = B.lib()
    o = B.Opts(64, 4, 1e-2, 1.0, 0, 0)
    h = ctypes.c_void_p()
    assert L.bem_build(ctypes.byref(o), None, ctypes.byref(h)) == 0
    th = dev(W.random_handles(1, 2))
    x = dev(W.random_points(1, 10))
    u = torch.empty((10, 3), dtype=torch.float64, device="cuda")
    cb = (ctypes.c_double * 3)(0, 0, 0)
    rc = L.bem_eval(h, th.data_ptr(), 2, x.data_ptr(), 10, cb, u.data_ptr(), 0, None)
    assert rc == -3                                   # not factored yet
    assert b"factor" in L.bem_last_error(h)
    assert L.bem_factor(h, None) == 0
    assert L.bem_eval(h, th.data_ptr(), 2, x.data_ptr(), 10, cb, u.data_ptr(), 7, None) == -1   # bad precision
    assert L.bem_eval(h, th.data_ptr(), -1, x.data_ptr(), 10, cb, u.data_ptr(), 0, None) == -1  # bad H
    assert L.bem_eval(h, th.data_ptr(), 2, x.data_ptr(), 10, cb, u.data_ptr(), 0, None) == 0
    torch.cuda.synchronize()
    L.bem_destroy(h)
