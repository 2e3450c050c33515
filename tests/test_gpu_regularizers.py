"""GPU regularisation terms (Sec. 4.4: handle length, end point snapping, sparsity), their
place in lm_step, and handle pruning, against the oracle.

Bars: values, gradients and Hessians within 1e-12 relative (float64 on both sides; the
snapping pairs are an integer decision taken with the same float64 formula, so the pair
count must agree exactly); LM steps as in the other LM tests; pruning bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu
RG = O.regularizers

TERMS = dict(length_weight=2.0, length_max=0.12, snap_weight=3.0, snap_dist=0.08, snap_mix=0.6,
             sparse_wd=0.05, sparse_wc=0.02, sparse_t=0.1, sparse_eps=1e-2)


def _straight(seed, H, length=0.15):
    rng = np.random.default_rng(np.random.SeedSequence(entropy=7000 + seed))
    c = rng.uniform(0.2, 0.8, size=(H, 2))
    ang = rng.uniform(0, 2 * np.pi, size=H)
    L = length * rng.uniform(0.5, 1.5, size=H)
    d = 0.5 * L[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    return np.ascontiguousarray(np.concatenate([c - d, c + d, rng.uniform(-0.3, 0.3, size=(H, 6))], axis=1))


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(autouse=True)
def _clear_terms():
    yield
    for model in ("cubic", "straight"):
        for S in (1, 8):
            ctx_for(S, handle_model=model).set_regularization()


@pytest.mark.parametrize("model", ["straight", "cubic"])
def test_terms_match_oracle(model):
    th = _straight(1, 40) if model == "straight" else W.random_handles(2, 24, spread=0.1)
    ctx = ctx_for(1 if model == "straight" else 8, handle_model=model)
    ctx.set_regularization(**TERMS)
    v, g, hm, npairs = ctx.regularization(dev(th))
    Ro, go, Ho, pairs = RG.terms(th, RG.Reg(**TERMS))
    log(f"{model}: R {v:.12e} / {Ro:.12e}, pairs {npairs} / {len(pairs)}")
    assert npairs == len(pairs) and npairs > 0
    assert v == pytest.approx(Ro, rel=1e-12)
    assert _rel(host(g), go) < 1e-12
    assert _rel(host(hm), Ho) < 1e-12
    v2, g2, h2, _ = ctx.regularization(dev(th), with_derivatives=False)
    assert v2 == v and g2 is None and h2 is None


def test_terms_validated():
    ctx = ctx_for(1, handle_model="straight")
    for bad in (dict(length_weight=-1.0), dict(snap_weight=1.0, snap_dist=0.0), dict(snap_weight=1.0, snap_dist=0.1,
                                                                                     snap_mix=1.5),
                dict(sparse_wd=1.0, sparse_t=0.0), dict(sparse_wc=float("nan"), sparse_t=1.0)):
        with pytest.raises(B.BemError):
            ctx.set_regularization(**bad)
    ctx.set_regularization(snap_weight=1.0, snap_dist=0.1, snap_mix=0.5)
    with pytest.raises(B.BemError):
        ctx.regularization(dev(np.zeros((70000, 10))), with_derivatives=False)


@pytest.mark.parametrize("compat", [0, 1])
@pytest.mark.parametrize("gram,prec,tol", [("fp64", "fp64", 1e-8), ("bf16x3_mfma", "mixed", None)])
def test_lm_step_with_terms(compat, gram, prec, tol):
    th_true = _straight(3, 8)
    th0 = th_true.copy()
    rng = np.random.default_rng(4)
    th0[:, :4] += 0.01 * rng.standard_normal((8, 4))
    th0[:, 4:] += 0.1 * rng.standard_normal((8, 6))
    x = W.random_points(5, 4096)
    T = O.straight.evaluate(th_true, x, np.full(3, 0.5), 1, 1e-2) + 0.1 * W.random_vector(6, (4096, 3))
    reg = RG.Reg(**TERMS)
    st_o = O.LMState(lam=1e-1, mean_rule=0, compat=bool(compat))
    th_o, st_o = O.straight.lm_step(th0, x, T, st_o, 1, 1e-2, reg=reg)
    if tol is None:
        tol = mixed_step_tol(O.straight.normal_equations(th0, x, np.zeros_like(T), 1, 1e-2)[0], 1e-1,
                             RG.terms(th0, reg)[2])
    ctx = ctx_for(1, handle_model="straight")
    ctx.set_regularization(**TERMS)
    th = dev(th0)
    st = B.new_lm_state(1e-1, 0, compat=compat)
    ctx.lm_step(th, dev(x), dev(T), st, gram, prec)
    R0 = RG.terms(th0, reg)[0]
    d_o, d = th_o - th0, host(th) - th0
    e = _rel(d, d_o) if st_o.accepted else float(np.abs(d).max())
    log(f"lm+terms {gram}/{prec} compat={compat}: accepted {st.accepted}/{st_o.accepted}, R {st.reg_value:.6e}/{R0:.6e}, "
        f"pairs {st.snap_pairs}, loss {st.loss_before:.9e}/{st_o.loss_before:.9e}, step rel err {e:.3e} (bar {tol:.3e})")
    assert st.reg_value == pytest.approx(R0, rel=1e-12)
    assert st.loss_before == pytest.approx(st_o.loss_before, rel=1e-10 if prec == "fp64" else 1e-5)
    assert bool(st.accepted) == bool(st_o.accepted)
    assert st.lam == pytest.approx(st_o.lam)
    assert e < tol


@pytest.mark.parametrize("model", ["straight", "cubic"])
def test_prune_matches_oracle(model):
    th = _straight(7, 300) if model == "straight" else W.random_handles(8, 300)
    rng = np.random.default_rng(9)
    small = rng.random(300) < 0.3
    th[small, 4 if model == "straight" else 8:] *= 1e-4
    ref = RG.prune(th, 1e-3)
    ctx = ctx_for(1 if model == "straight" else 8, handle_model=model)
    d = dev(th)
    out = ctx.prune(d, 1e-3)
    log(f"prune {model}: {out.shape[0]} of 300 kept (oracle {ref.shape[0]})")
    assert out.shape == ref.shape
    assert np.array_equal(host(out), ref)
    assert ctx.prune(dev(np.zeros((0, th.shape[1]))), 1e-3).shape[0] == 0


def test_paper_workload_step_with_terms():
    """Full paper-native workload (500 handles, 100,000 samples), split-BF16 / mixed, every term on:
    the terms' value at the start against the oracle and a finite, decreasing-or-rejected step."""
    wl = W.make_config(W.PAPER_CONFIG)
    terms = dict(length_weight=1.0, length_max=0.08, snap_weight=1.0, snap_dist=0.02, snap_mix=0.5,
                 sparse_wd=1e-4, sparse_wc=5e-5, sparse_t=0.05, sparse_eps=1e-3)
    ctx = ctx_for(wl.S, handle_model="straight")
    ctx.set_regularization(**terms)
    x = dev(wl.samples(0))
    tht = dev(wl.theta_true)
    T = (ctx.eval(tht, x, wl.cbar_true, "fp64") + wl.spec.sigma * dev(wl.noise(0))).clamp_(max=1.0)
    th = dev(wl.theta0)
    st = B.new_lm_state(wl.lam0, 0)
    ctx.lm_step(th, x, T, st, "bf16x3_mfma", "mixed")
    R0 = RG.value(wl.theta0, RG.Reg(**terms), RG.snap_pairs(wl.theta0, 0.02, 0.5))
    log(f"paper workload + terms: R {st.reg_value:.9e} / {R0:.9e}, pairs {st.snap_pairs}, "
        f"loss {st.loss_before:.6e} -> {st.loss_after:.6e}, accepted {st.accepted}")
    assert st.reg_value == pytest.approx(R0, rel=1e-12)
    assert st.snap_pairs == len(RG.snap_pairs(wl.theta0, 0.02, 0.5))
    assert np.isfinite(host(th)).all()
    assert bool(st.accepted) == (st.loss_after < st.loss_before)
