"""GPU LM step with the compatibility condition enforced (Sec. 3.1.2, Sec. 4.3) against
the oracle's constrained step and re-projection.

Bars: FP64 path theta' within 1e-8 (tiny) / 1e-7 (medium) relative to the step, same
accept decision and damping; mixed / split-BF16 within 10 u kappa of the step (helpers.mixed_step_tol); the reported
violation of the condition after the step at rounding level.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu


def _case(config, n, per_side):
    wl = W.make_config(config)
    idx = wl.subsample(n) if config != 1 else np.arange(n)
    x = wl.samples(0)[idx]
    truth = O.reproject(wl.theta_true, wl.S)                        # a compatible ground truth
    T = O.evaluate(truth, x, wl.cbar_true, wl.S, wl.eps, per_side) + wl.spec.sigma * wl.noise(0)[idx]
    return wl, x, T


def _compare(wl, x, T, per_side, lam, gram, prec, tol):
    ctx = ctx_for(wl.S, per_side=per_side)
    st_o = O.LMState(lam=lam, mean_rule=0, compat=True)
    th_o, st_o = O.lm_step(wl.theta0, x, T, st_o, wl.S, wl.eps, per_side)
    th = dev(wl.theta0)
    st = B.new_lm_state(lam, 0, compat=1)
    ctx.lm_step(th, dev(x), dev(T), st, gram, prec)
    d_o = th_o - wl.theta0
    d = host(th) - wl.theta0
    e = float(np.abs(d - d_o).max() / np.abs(d_o).max()) if st_o.accepted else float(np.abs(d).max())
    log(f"compat lm {gram}/{prec}: accepted {st.accepted}/{st_o.accepted}, lambda {st.lam:.1e}/{st_o.lam:.1e}, "
        f"step rel err {e:.3e} (bar {tol:.3e}), violation {st.compat_violation:.2e}")
    assert bool(st.accepted) == bool(st_o.accepted)
    assert st.lam == pytest.approx(st_o.lam)
    assert e < tol
    if st.accepted:
        A = O.compat_vectors(host(th), wl.S)
        flat = host(th).reshape(-1)
        assert np.abs(A.T @ flat).max() <= 1e-12 * (np.abs(A) * np.abs(flat)[:, None]).sum(0).max()
        assert st.compat_violation < 1e-12


def test_compat_step_tiny_fp64():
    wl, x, T = _case(1, 4096, 256)
    _compare(wl, x, T, 256, 1e-1, "fp64", "fp64", 1e-8)


def test_compat_step_tiny_mixed_bf16x3():
    wl, x, T = _case(1, 4096, 256)
    tol = mixed_step_tol(O.normal_equations(wl.theta0, x, np.zeros_like(T), wl.S, wl.eps)[0], 1e-1)
    _compare(wl, x, T, 256, 1e-1, "bf16x3_mfma", "mixed", tol)


def test_compat_step_medium_fp64():
    wl, x, T = _case(2, 2048, 256)
    _compare(wl, x, T, 256, 1e-1, "fp64", "fp64", 1e-7)


def test_compat_flag_is_validated():
    wl = W.make_config(1)
    ctx = ctx_for(wl.S)
    st = B.new_lm_state(1e-3, 0, compat=2)
    x = wl.samples(0)[:64]
    with pytest.raises(B.BemError):
        ctx.lm_step(dev(wl.theta0), dev(x), dev(np.zeros((64, 3))), st, "fp64", "fp64")
