"""GPU subdomains (Sec. 4.1): outer boundaries made of arbitrary straight elements
(bem_build_elements), the stable partition of samples by subdomain label, and one LM step per
subdomain, against the oracle on the same boundaries.

Bars as for the unit square: FP64 within 1e-10 relative, mixed colour within 1e-4 absolute
and gradients within 1e-3 relative; the boundary matrix within 1e-13; the partition bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import regularizers as RG
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu

L_SHAPE = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.5], [0.5, 0.5], [0.5, 1.0], [0.0, 1.0]])


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _elements(ea, eb):
    return np.concatenate([ea, eb], axis=1)


def _inside_L(x):
    return ~((x[:, 0] > 0.5) & (x[:, 1] > 0.5))


def _L_case(n_per_edge=16, closed=True):
    ea, eb = O.polygon_elements(L_SHAPE if closed else L_SHAPE[:5], n_per_edge, closed=closed)
    th = W.random_handles(41, 4, spread=0.08, centre_lo=0.15, centre_hi=0.35)
    x = W.random_points(42, 6000, 0.001, 0.999)
    x = np.ascontiguousarray(x[_inside_L(x)][:3000])
    return ea, eb, th, x


def test_square_from_elements_is_bit_identical():
    ea, eb = O.square_boundary(32)
    c1 = B.Context(segs_per_handle=8, elems_per_side=32)
    c2 = B.Context(segs_per_handle=8, elements=_elements(ea, eb))
    assert c2.M == 128
    assert torch.equal(c1.matrix(0), c2.matrix(0)) and torch.equal(c1.matrix(1), c2.matrix(1))
    th = dev(W.random_handles(43, 3))
    x = dev(W.random_points(44, 512))
    assert torch.equal(c1.eval(th, x, (0.1, 0.2, 0.3)), c2.eval(th, x, (0.1, 0.2, 0.3)))


@pytest.mark.parametrize("closed", [True, False])
def test_L_shape_forward_adjoint_and_matrix(closed):
    ea, eb, th, x = _L_case(closed=closed)
    bnd = O.boundary_from_elements(ea, eb)
    ctx = B.Context(segs_per_handle=8, elements=_elements(ea, eb))
    eA = _rel(host(ctx.matrix(0)), bnd.A)
    eP = _rel(host(ctx.matrix(1)), bnd.Apinv)
    cbar = np.array([0.2, 0.4, 0.6])
    uo = O.evaluate(th, x, cbar, 8, 1e-2, bnd)
    u64 = host(ctx.eval(dev(th), dev(x), cbar, "fp64"))
    u32 = host(ctx.eval(dev(th), dev(x), cbar, "mixed"))
    g = W.random_vector(45, (len(x), 3))
    go = O.vjp(th, x, g, 8, 1e-2, bnd)
    g64 = host(ctx.vjp(dev(th), dev(x), dev(g), "fp64"))
    g32 = host(ctx.vjp(dev(th), dev(x), dev(g, torch.float32), "mixed"))
    log(f"L-shape closed={closed}: A {eA:.2e}, A+ {eP:.2e}, forward {_rel(u64, uo):.2e} / {np.abs(u32 - uo).max():.2e}, "
        f"adjoint {_rel(g64, go):.2e} / {_rel(g32, go):.2e}")
    assert eA < 1e-13 and eP < 1e-10
    assert _rel(u64, uo) < 1e-10 and np.abs(u32 - uo).max() < 1e-4
    assert _rel(g64, go) < 1e-10 and _rel(g32, go) < 1e-3


def test_L_shape_normal_equations_and_lm_step():
    ea, eb, th, x = _L_case(n_per_edge=12)
    bnd = O.boundary_from_elements(ea, eb)
    ctx = B.Context(segs_per_handle=8, elements=_elements(ea, eb), tile_rows=1024)
    r = W.random_vector(46, (len(x), 3))
    Ho, go = O.normal_equations(th, x, r, 8, 1e-2, bnd)
    JtJ, Jtr = ctx.jtj(dev(th), dev(x), dev(r), "fp64", "fp64")
    assert _rel(host(JtJ), Ho) < 1e-10 and _rel(host(Jtr), go) < 1e-10
    th0 = th + 0.01 * W.random_vector(47, th.shape)
    T = O.evaluate(th, x, np.full(3, 0.5), 8, 1e-2, bnd) + 0.1 * W.random_vector(48, (len(x), 3))
    st_o = O.LMState(lam=1e-1, mean_rule=0)
    th_o, st_o = O.lm_step(th0, x, T, st_o, 8, 1e-2, bnd)
    d = dev(th0)
    st = B.new_lm_state(1e-1, 0)
    ctx.lm_step(d, dev(x), dev(T), st, "fp64", "fp64")
    e = _rel(host(d) - th0, th_o - th0) if st_o.accepted else float(np.abs(host(d) - th0).max())
    log(f"L-shape lm: accepted {st.accepted}/{st_o.accepted}, step rel err {e:.3e}")
    assert bool(st.accepted) == bool(st_o.accepted) and e < 1e-8


def test_L_shape_mixed_lm_step():
    """Mixed precision / split-BF16 LM step on the L-shape (samples visited cell by cell over
    the boundary's bounding box inside lm_step) against the oracle's step."""
    ea, eb, th, x = _L_case(n_per_edge=12)
    bnd = O.boundary_from_elements(ea, eb)
    ctx = B.Context(segs_per_handle=8, elements=_elements(ea, eb), tile_rows=1024)
    th0 = th + 0.01 * W.random_vector(57, th.shape)
    T = O.evaluate(th, x, np.full(3, 0.5), 8, 1e-2, bnd) + 0.1 * W.random_vector(58, (len(x), 3))
    st_o = O.LMState(lam=1e-1, mean_rule=0)
    th_o, st_o = O.lm_step(th0, x, T, st_o, 8, 1e-2, bnd)
    tol = mixed_step_tol(O.normal_equations(th0, x, np.zeros_like(T), 8, 1e-2, bnd)[0], 1e-1)
    d = dev(th0)
    st = B.new_lm_state(1e-1, 0)
    ctx.lm_step(d, dev(x), dev(T), st, "bf16x3_mfma", "mixed")
    e = _rel(host(d) - th0, th_o - th0) if st_o.accepted else float(np.abs(host(d) - th0).max())
    log(f"L-shape mixed lm: accepted {st.accepted}/{st_o.accepted}, loss {st.loss_before:.9e}/{st_o.loss_before:.9e}, "
        f"step rel err {e:.3e} (bar {tol:.3e})")
    assert st.loss_before == pytest.approx(st_o.loss_before, rel=1e-5)
    assert bool(st.accepted) == bool(st_o.accepted)
    assert e < tol


def test_build_elements_validation():
    with pytest.raises(B.BemError):
        B.Context(segs_per_handle=4, elements=np.zeros((1, 4)))
    bad = _elements(*O.polygon_elements(L_SHAPE, 4))
    bad[3, 2:] = bad[3, :2]
    with pytest.raises(B.BemError):
        B.Context(segs_per_handle=4, elements=bad)


@pytest.mark.parametrize("N", [0, 1, 4095, 100_003])
def test_partition_matches_stable_sort(N):
    ctx = B.Context(segs_per_handle=4, elems_per_side=8)
    rng = np.random.default_rng(N + 1)
    D = 5
    labels = rng.integers(-1, D + 1, size=N).astype(np.int32)        # -1 and D are dropped
    x = rng.random((N, 2))
    T = rng.random((N, 3))
    xo, To, off = ctx.partition(dev(labels), dev(x), dev(T), D)
    order = np.concatenate([np.nonzero(labels == d)[0] for d in range(D)]) if N else np.zeros(0, int)
    counts = [int((labels == d).sum()) for d in range(D)]
    assert off == [0] + list(np.cumsum(counts))
    assert np.array_equal(host(xo)[: off[D]], x[order])
    assert np.array_equal(host(To)[: off[D]], T[order])


@pytest.mark.parametrize("with_reg", [False, True])
def test_two_subdomains_lm_step(with_reg):
    """Left and right halves of the unit square as subdomains with their own handles: one
    partitioned call equals the oracle's independent step in each half, whose data terms are
    divided by all samples drawn over the image (10% of them in no subdomain), also with the
    regularisation terms of Sec. 4.4 on, where that normalisation sets their relative weight."""
    halves = [np.array([[0.0, 0.0], [0.5, 0.0], [0.5, 1.0], [0.0, 1.0]]),
              np.array([[0.5, 0.0], [1.0, 0.0], [1.0, 1.0], [0.5, 1.0]])]
    bnds, ctxs, ths, ths0 = [], [], [], []
    for d, poly in enumerate(halves):
        ea, eb = O.polygon_elements(poly, 8)
        bnds.append(O.boundary_from_elements(ea, eb))
        ctxs.append(B.Context(segs_per_handle=8, elements=_elements(ea, eb)))
        lo = 0.1 + 0.5 * d
        th = W.random_handles(50 + d, 2, spread=0.06, centre_lo=lo + 0.05, centre_hi=lo + 0.25)
        th[:, 1:8:2] = np.clip(th[:, 1:8:2], 0.1, 0.9)
        ths.append(th)
        ths0.append(th + 0.01 * W.random_vector(60 + d, th.shape))
    x = W.random_points(70, 5000, 0.001, 0.999)
    labels = (x[:, 0] >= 0.5).astype(np.int32)
    labels[::10] = -1                                   # samples outside both subdomains
    reg = RG.Reg(length_weight=2.0, length_max=0.05, snap_weight=0.0, snap_dist=0.1, snap_mix=0.5,
                 sparse_wd=0.01, sparse_wc=0.005, sparse_t=0.1, sparse_eps=1e-2) if with_reg else None
    if with_reg:
        for c in ctxs:
            c.set_regularization(**{f: getattr(reg, f) for f in reg.__dataclass_fields__})
    T = np.zeros((len(x), 3))
    for d in range(2):
        m = labels == d
        T[m] = O.evaluate(ths[d], x[m], np.full(3, 0.3 + 0.2 * d), 8, 1e-2, bnds[d]) + 0.05 * W.random_vector(80 + d, (m.sum(), 3))
    dth = [dev(t) for t in ths0]
    sts = [B.new_lm_state(1e-1, 0) for _ in range(2)]
    B.lm_step_subdomains(ctxs, dth, dev(x), dev(T), dev(labels), sts, "fp64", "fp64")
    for d in range(2):
        m = labels == d
        st_o = O.LMState(lam=1e-1, mean_rule=0, data_count=len(x))
        th_o, st_o = O.lm_step(ths0[d], x[m], T[m], st_o, 8, 1e-2, bnds[d], reg=reg)
        assert sts[d].loss_before == pytest.approx(st_o.loss_before, rel=1e-10)
        e = _rel(host(dth[d]) - ths0[d], th_o - ths0[d]) if st_o.accepted else float(np.abs(host(dth[d]) - ths0[d]).max())
        log(f"subdomain {d}: {m.sum()} samples, accepted {sts[d].accepted}/{st_o.accepted}, cbar {sts[d].cbar[:]} / "
            f"{st_o.cbar}, step rel err {e:.3e}")
        assert bool(sts[d].accepted) == bool(st_o.accepted)
        assert np.allclose(np.array(sts[d].cbar[:]), st_o.cbar, rtol=1e-12)
        assert e < 1e-8
