"""GPU near-pair list capacity of the mixed sweeps.  With long handles most of the domain lies
within two handle lengths of many handles, so the near pairs of a 64-sample wavefront exceed
the initial capacity (1,024 slots).  Before lm_step those samples take the inline sweeps (forward,
adjoint, J tiles); lm_step raises the capacity and repeats its sweep; afterwards the listed
path runs.  Every stage against the oracle's straight model, bars as for MIXED elsewhere:
colour within 1e-4 absolute, gradients within 1e-3 relative, split-BF16 J^T J within 1e-4
relative, the LM step within 10 u kappa (helpers.mixed_step_tol) of the oracle's.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu
ST = O.straight
S, EPS = 1, 1e-2


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _long_handles(seed, H, length=0.4):
    rng = np.random.default_rng(np.random.SeedSequence(entropy=9000 + seed))
    c = rng.uniform(0.3, 0.7, size=(H, 2))
    ang = rng.uniform(0, 2 * np.pi, size=H)
    d = 0.5 * length * np.stack([np.cos(ang), np.sin(ang)], 1)
    return np.ascontiguousarray(np.concatenate([c - d, c + d, W.draw_straight_colours(rng, H)], axis=1))


def _max_wave_count(th, x):
    """Largest number of near (sample, handle) pairs over 64-sample wavefronts (float64 test)."""
    a, b = th[:, None, 0:2], th[:, None, 2:4]
    L2 = ((b - a) ** 2).sum(-1)
    near = (((a - x[None]) ** 2).sum(-1) < 4 * L2) & (((b - x[None]) ** 2).sum(-1) < 4 * L2)
    per = near.sum(0)
    per = np.concatenate([per, np.zeros((-len(per)) % 64, int)])
    return int(per.reshape(-1, 64).sum(1).max())


def _check_stage(ctx, th, x, g, r, tag):
    cbar = np.array([0.3, 0.5, 0.7])
    uo = ST.evaluate(th, x, cbar, S, EPS)
    u32 = host(ctx.eval(dev(th), dev(x), cbar, "mixed"))
    go = ST.vjp(th, x, g, S, EPS)
    g32 = host(ctx.vjp(dev(th), dev(x), dev(g, torch.float32), "mixed"))
    Ho, _ = ST.normal_equations(th, x, r, S, EPS)
    JtJ, _ = ctx.jtj(dev(th), dev(x), dev(r, torch.float32), "bf16x3_mfma", "mixed")
    eu, eg, eh = float(np.abs(u32 - uo).max()), _rel(g32, go), _rel(host(JtJ), Ho)
    log(f"{tag}: capacity {ctx.near_capacity}, forward {eu:.2e}, adjoint {eg:.2e}, JtJ {eh:.2e}")
    assert eu < 1e-4 and eg < 1e-3 and eh < 1e-4


def test_capacity_grows_in_lm_step():
    H, N = 40, 3000
    th_true = _long_handles(1, H)
    x = W.random_points(2, N, 0.001, 0.999)
    need = _max_wave_count(th_true, x)
    assert need > 1100, need                   # the case overflows the initial capacity
    ctx = B.Context(segs_per_handle=S, eps=EPS, handle_model="straight", tile_rows=1024)
    assert ctx.near_capacity == 1024
    g = W.random_vector(3, (N, 3))
    r = W.random_vector(4, (N, 3))
    _check_stage(ctx, th_true, x, g, r, "before lm_step (inline near pairs)")
    assert ctx.near_capacity == 1024           # only lm_step raises it

    th0 = th_true.copy()
    rng = np.random.default_rng(5)
    th0[:, :4] += 0.005 * rng.standard_normal((H, 4))
    th0[:, 4:] += 0.05 * rng.standard_normal((H, 6))
    T = ST.evaluate(th_true, x, np.full(3, 0.5), S, EPS) + 0.05 * W.random_vector(6, (N, 3))
    st_o = O.LMState(lam=1e-1, mean_rule=0)
    th_o, st_o = ST.lm_step(th0, x, T, st_o, S, EPS)
    tol = mixed_step_tol(ST.normal_equations(th0, x, np.zeros_like(T), S, EPS)[0], 1e-1)
    th = dev(th0)
    st = B.new_lm_state(1e-1, 0)
    ctx.lm_step(th, dev(x), dev(T), st, "bf16x3_mfma", "mixed")
    d_o, d = th_o - th0, host(th) - th0
    e = _rel(d, d_o) if st_o.accepted else float(np.abs(d).max())
    cap = ctx.near_capacity
    log(f"lm_step: capacity {cap} (largest wavefront count at theta0 {_max_wave_count(th0, x)}), "
        f"accepted {st.accepted}/{st_o.accepted}, loss {st.loss_before:.9e}/{st_o.loss_before:.9e}, step rel err {e:.3e} "
        f"(bar {tol:.3e})")
    assert cap % 256 == 0 and cap >= _max_wave_count(th0, x) - 16
    assert st.loss_before == pytest.approx(st_o.loss_before, rel=1e-5)
    assert bool(st.accepted) == bool(st_o.accepted)
    assert e < tol

    _check_stage(ctx, th_true, x, g, r, "after lm_step (listed near pairs)")
