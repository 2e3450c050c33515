"""Pins of the oracle's regularisation terms (Sec. 4.4: handle length, end point snapping,
sparsity) and handle pruning: central differences of every gradient and Hessian, closed
forms, hand-built snapping configurations, and the LM step with the terms rebuilt from
its definition."""
import numpy as np
import pytest

import oracle as O
from paper_2602_05492_amd import workload as W

RG = O.regularizers


def _straight(seed, H, length=0.2):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, size=(H, 2))
    ang = rng.uniform(0, 2 * np.pi, size=H)
    L = length * rng.uniform(0.5, 1.5, size=H)
    d = 0.5 * L[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    return np.concatenate([c - d, c + d, rng.uniform(-0.3, 0.3, size=(H, 6))], axis=1)


REG = RG.Reg(length_weight=2.0, length_max=0.2, snap_weight=3.0, snap_dist=0.15, snap_mix=0.6,
             sparse_wd=0.05, sparse_wc=0.02, sparse_t=0.1, sparse_eps=1e-2)


def _radial_curvature(th, reg):
    """The left-out part of the sparsity Hessian: f''(s) u u^T per jump vector, with
    f(s) = lam t tanh(s/t), f''(s) = -(2 lam / t) sech^2(s/t) tanh(s/t), u = w/s."""
    H, Q = th.shape
    out = np.zeros((H * Q, H * Q))
    _, _, wd, wc = RG.layout(Q)
    for lam, groups in ((reg.sparse_wd, wd), (reg.sparse_wc, wc)):
        for h in range(H):
            for grp in groups:
                c = [h * Q + k for k in grp]
                w = th[h, list(grp)]
                s = np.sqrt(w @ w + reg.sparse_eps ** 2)
                th_ = np.tanh(s / reg.sparse_t)
                f2 = -2 * lam / reg.sparse_t * (1 - th_ ** 2) * th_
                out[np.ix_(c, c)] += f2 * np.outer(w / s, w / s)
    return out


@pytest.mark.parametrize("kind", ["straight", "cubic"])
def test_gradient_and_hessian_central_differences(kind):
    th = _straight(1, 5) if kind == "straight" else W.random_handles(2, 4, spread=0.12)
    R, g, Hm, pairs = RG.terms(th, REG)
    assert pairs, "the configuration should snap at least one pair"
    assert R > 0
    flat = th.reshape(-1)
    h = 1e-6
    Hfd = np.zeros_like(Hm)
    for p in range(flat.size):
        tp, tm = flat.copy(), flat.copy()
        tp[p] += h
        tm[p] -= h
        Rp, gp, _, _ = RG.terms(tp.reshape(th.shape), REG, pairs)
        Rm, gm, _, _ = RG.terms(tm.reshape(th.shape), REG, pairs)
        assert (Rp - Rm) / (2 * h) == pytest.approx(g[p], rel=1e-6, abs=1e-8), p
        Hfd[:, p] = (gp - gm) / (2 * h)
    # the finite-difference Hessian of the gradient contains the sparsity term's negative radial
    # curvature, which the step's Hessian leaves out
    assert np.allclose(Hfd - _radial_curvature(th, REG), Hm, rtol=1e-5, atol=1e-6)
    assert np.allclose(Hm, Hm.T, atol=1e-14)
    assert np.linalg.eigvalsh(Hm).min() > -1e-12


def test_length_closed_form():
    th = np.array([[0.1, 0.2, 0.1 + 0.3 * 0.6, 0.2 + 0.3 * 0.8, 0, 0, 0, 0, 0, 0]])
    R, g, Hm = RG.length_term(th, 2.0, 0.2)
    assert R == pytest.approx(2.0 * 0.1 ** 2, rel=1e-12)
    assert np.allclose(g[2:4], 2 * 2.0 * 0.1 * np.array([0.6, 0.8]))
    assert np.allclose(g[0:2], -g[2:4])
    R0, g0, H0 = RG.length_term(th, 2.0, 0.35)
    assert R0 == 0.0 and not g0.any() and not H0.any()
    # positive semi-definite for any length above the threshold
    assert np.linalg.eigvalsh(Hm).min() > -1e-14


def test_sparsity_limits():
    th = np.zeros((2, 10))
    th[1, 4:7] = [30.0, -40.0, 0.0]
    R, g, _ = RG.sparsity_term(th, 0.5, 0.0, 0.1, 1e-2)
    # handle 0: w = 0 gives lam t tanh(eps / t) and no gradient; handle 1 saturates at lam t
    assert R == pytest.approx(0.5 * 0.1 * np.tanh(0.1) + 0.5 * 0.1, rel=1e-12)
    assert not g[:10].any()
    assert np.abs(g[10:]).max() < 1e-12


def _seg(a, b):
    return [a[0], a[1], b[0], b[1], 0, 0, 0, 0, 0, 0]


def test_snap_pairs_mutual_best():
    th = np.array([_seg((0.1, 0.5), (0.3, 0.5)),       # end 1 (index 1) near handle 1's start
                   _seg((0.305, 0.5), (0.5, 0.5)),     # collinear continuation (index 2)
                   _seg((0.3, 0.51), (0.3, 0.7))])     # perpendicular, also near (index 4)
    assert RG.snap_pairs(th, 0.05, 0.5) == [(1, 2)]
    # handle 1 moved away: the perpendicular handle becomes handle 0's mutual best
    th2 = th.copy()
    th2[1, :4] = [0.8, 0.8, 0.9, 0.9]
    assert RG.snap_pairs(th2, 0.05, 0.5) == [(1, 4)]
    # nothing within the distance threshold
    assert RG.snap_pairs(th, 0.004, 0.5) == []


def test_snap_direction_decides_with_small_mix():
    th = np.array([_seg((0.1, 0.5), (0.3, 0.5)),
                   _seg((0.302, 0.5), (0.302, 0.7)),   # closer, perpendicular (index 2)
                   _seg((0.31, 0.5), (0.5, 0.5))])     # farther, collinear (index 4)
    assert RG.snap_pairs(th, 0.05, 0.9) == [(1, 2)]     # distance dominates
    assert RG.snap_pairs(th, 0.05, 0.1) == [(1, 4)]     # direction dominates


def test_snap_term_closed_form():
    th = np.array([_seg((0.1, 0.5), (0.3, 0.5)), _seg((0.31, 0.52), (0.5, 0.5))])
    R, g, Hm = RG.snap_term(th, 3.0, [(1, 2)])
    assert R == pytest.approx(3.0 * (0.01 ** 2 + 0.02 ** 2), rel=1e-12)
    assert np.allclose(g[2:4], 6.0 * np.array([-0.01, -0.02]))
    assert np.allclose(g[10:12], -g[2:4])


@pytest.mark.parametrize("compat", [False, True])
def test_lm_step_with_regularizers_from_definition(compat):
    ST = O.straight
    th = _straight(3, 4)
    S, eps, ps = 1, 1e-2, 16
    x = W.random_points(4, 96)
    T = ST.evaluate(_straight(5, 4), x, np.full(3, 0.4), S, eps, ps)
    st = O.LMState(lam=1e-1, mean_rule=1, compat=compat)
    th1, st = ST.lm_step(th, x, T, st, S, eps, ps, reg=REG)
    u0 = ST.evaluate(th, x, np.zeros(3), S, eps, ps)
    cbar = (T - u0).mean(0)
    r = (u0 + cbar - T).reshape(-1)
    Jr = ST.jacobian(th, x, S, eps, ps).reshape(-1, 40)
    R0, gR, HR, pairs = RG.terms(th, REG)
    JtJ, Jtr = Jr.T @ Jr / 96 + HR, Jr.T @ r / 96 + gR
    if compat:
        d = O.constrained_step(JtJ, Jtr, 1e-1, ST.compat_vectors(th, S))
        ref = ST.reproject(th - d.reshape(th.shape), S)
    else:
        ref = th - O.damped_step(JtJ, Jtr, 1e-1).reshape(th.shape)
    assert np.allclose(th1 if st.accepted else ref, ref, rtol=1e-10, atol=1e-12)
    assert st.loss_before == pytest.approx(0.5 * float(r @ r) / 96 + R0, rel=1e-12)
    L1 = O.loss(ST.evaluate(ref, x, cbar, S, eps, ps), T) + RG.value(ref, REG, pairs)
    assert st.loss_after == pytest.approx(L1, rel=1e-12)
    assert st.accepted == (L1 < st.loss_before)


def test_prune():
    th = _straight(6, 5)
    th[1, 4:10] = [1e-4, 0, 0, 0, 2e-4, 0]          # both norms small: removed
    th[3, 4:7] = 0.0                                 # wd zero, wc large: kept
    th[3, 7:10] = [0.5, 0.0, 0.0]
    out = RG.prune(th, 1e-3)
    assert out.shape == (4, 10)
    assert np.array_equal(out, th[[0, 2, 3, 4]])
    cub = W.random_handles(7, 3)
    cub[2, 8:20] = 0.0
    cub[2, 11] = 5e-4
    assert np.array_equal(RG.prune(cub, 1e-3), cub[:2])


@pytest.mark.parametrize("compat", [False, True])
def test_data_count_scales_only_the_data_terms(compat):
    """A subdomain's step divides its data terms by the samples drawn over the whole image, M_H
    (Eq. losshessian, Eq. lossjacobian), and leaves the regularisers (Sec. 4.4) as they are.
    Dividing the whole objective by a constant does not change the LM step or its accept test
    (the step is invariant to a rescaled loss), so the step with data_count = m and weights w
    equals the step with the subdomain's own count and weights w N / m, and its losses are the
    latter's times N / m. A slip that scaled only some of the data terms (loss, gradient or
    Hessian) or also the regularisers breaks the equality."""
    ST = O.straight
    th = _straight(3, 4)
    S, eps, ps = 1, 1e-2, 16
    x = W.random_points(4, 96)
    T = ST.evaluate(_straight(5, 4), x, np.full(3, 0.4), S, eps, ps)
    m = 96 * 7
    k = 96 / m
    scaled = RG.Reg(**{f: (getattr(REG, f) / k if f in ("length_weight", "snap_weight", "sparse_wd", "sparse_wc")
                          else getattr(REG, f)) for f in REG.__dataclass_fields__})
    st_a = O.LMState(lam=1e-1, mean_rule=1, compat=compat, data_count=m)
    th_a, st_a = ST.lm_step(th, x, T, st_a, S, eps, ps, reg=REG)
    st_b = O.LMState(lam=1e-1, mean_rule=1, compat=compat)
    th_b, st_b = ST.lm_step(th, x, T, st_b, S, eps, ps, reg=scaled)
    assert st_a.accepted == st_b.accepted
    assert np.allclose(th_a, th_b, rtol=1e-9, atol=1e-12)
    assert st_a.loss_before == pytest.approx(k * st_b.loss_before, rel=1e-12)
    assert st_a.loss_after == pytest.approx(k * st_b.loss_after, rel=1e-9)
    # without regularisers the step does not depend on data_count at all
    st_c = O.LMState(lam=1e-1, mean_rule=1, compat=compat, data_count=m)
    th_c, _ = ST.lm_step(th, x, T, st_c, S, eps, ps)
    st_d = O.LMState(lam=1e-1, mean_rule=1, compat=compat)
    th_d, _ = ST.lm_step(th, x, T, st_d, S, eps, ps)
    assert np.allclose(th_c, th_d, rtol=1e-9, atol=1e-12)
    with pytest.raises(ValueError):
        ST.lm_step(th, x, T, O.LMState(lam=1e-1, data_count=95), S, eps, ps)
