"""GPU straight handles (Sec. 3.2 line segments; Sec. 4.1 two end points and constant jumps,
10 parameters per handle) against the oracle's straight model, through the C ABI with
handle_model = straight.

Bars as for cubic handles: FP64 within 1e-10 relative (forward, adjoint, Jacobian, J^T J);
MIXED colour within 1e-4 absolute and gradients within 1e-3 relative; reduced-precision Grams
within 1e-4 relative on J^T J; LM steps as in the cubic LM tests.  The paper-native workload
(500 Sobol-placed handles, one piece each, 100,000 samples) is checked at full size on sampled
rows of the forward pass and on the adjoint of a 1,024-sample subset.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu
ST = O.straight


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _handles(seed, H, length=0.2):
    """Straight handles with crossing allowed: centres in [0.25, 0.75]^2, random directions."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy=5000 + seed))
    c = rng.uniform(0.25, 0.75, size=(H, 2))
    ang = rng.uniform(0, 2 * np.pi, size=H)
    d = 0.5 * length * np.stack([np.cos(ang), np.sin(ang)], 1)
    return np.ascontiguousarray(np.concatenate([c - d, c + d, W.draw_straight_colours(rng, H)], axis=1))


def _points(seed, th, n, near_frac=0.1):
    """Uniform points plus a share within 1e-3 of a handle (the near-singular branch)."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy=6000 + seed))
    nn = int(near_frac * n)
    x = rng.uniform(1e-6, 1.0, size=(n - nn, 2))
    k = rng.integers(0, th.shape[0], nn)
    a, b = th[k, 0:2], th[k, 2:4]
    v = b - a
    nrm = np.stack([v[:, 1], -v[:, 0]], 1) / np.linalg.norm(v, axis=1, keepdims=True)
    xn = a + rng.random(nn)[:, None] * v + rng.uniform(-1e-3, 1e-3, nn)[:, None] * nrm
    return np.ascontiguousarray(np.concatenate([x, xn]))


@pytest.mark.parametrize("S", [1, 4])
def test_forward_and_adjoint_small(S):
    th = _handles(1, 6)
    x = _points(2, th, 3000)
    ctx = ctx_for(S, handle_model="straight")
    cbar = np.array([0.3, 0.5, 0.7])
    uo = ST.evaluate(th, x, cbar, S, 1e-2)
    u64 = host(ctx.eval(dev(th), dev(x), cbar, "fp64"))
    u32 = host(ctx.eval(dev(th), dev(x), cbar, "mixed"))
    e64, e32 = _rel(u64, uo), float(np.abs(u32 - uo).max())
    g = W.random_vector(3, (len(x), 3))
    go = ST.vjp(th, x, g, S, 1e-2)
    g64 = host(ctx.vjp(dev(th), dev(x), dev(g), "fp64"))
    g32 = host(ctx.vjp(dev(th), dev(x), dev(g, torch.float32), "mixed"))
    r64, r32 = _rel(g64, go), _rel(g32, go)
    log(f"straight S={S}: forward fp64 {e64:.2e} mixed abs {e32:.2e}; adjoint fp64 {r64:.2e} mixed {r32:.2e}")
    assert g64.shape == (6, 10)
    assert e64 < 1e-10 and e32 < 1e-4
    assert r64 < 1e-10 and r32 < 1e-3


def test_jacobian_small():
    th = _handles(4, 3)
    x = _points(5, th, 80)
    ctx = ctx_for(2, per_side=64, handle_model="straight")
    J = host(ctx.jacobian(dev(th), dev(x)))
    Jo = ST.jacobian(th, x, 2, 1e-2, 64)
    err = _rel(J, Jo)
    log("straight jacobian rel err", err)
    assert J.shape == (80, 3, 30) and err < 1e-10


@pytest.mark.parametrize("gram,prec,tol", [("fp64", "fp64", 1e-10), ("fp32_mfma", "mixed", 1e-4),
                                           ("bf16x3_mfma", "mixed", 1e-4)])
def test_normal_equations_small(gram, prec, tol):
    """Several sample tiles and a ragged tail (N = 2085, tiles of 640)."""
    th = _handles(6, 8)
    x = _points(7, th, 2085)
    ctx = ctx_for(1, tile_rows=640, handle_model="straight")
    r = W.random_vector(8, (len(x), 3))
    Ho, go = ST.normal_equations(th, x, r, 1, 1e-2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    JtJ, Jtr = ctx.jtj(dev(th), dev(x), dev(r, dt), gram, prec)
    eh, eg = _rel(host(JtJ), Ho), _rel(host(Jtr), go)
    log(f"straight jtj {gram}/{prec}: JtJ {eh:.3e} Jtr {eg:.3e}")
    assert JtJ.shape == (80, 80)
    assert eh < tol and eg < max(tol, 1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("n", [37, 200, 1001])
def test_normal_equations_ragged_tiles(n):
    """Split-BF16 J^T J with one-segment handles on sample counts whose last tile ends inside a
    32-sample block of the blocked tile (37; 1001: tiles of 256 and a last one of 233) or on a
    multiple of 8 that is not one of 32 (200)."""
    th = _handles(14, 8)
    x = _points(15, th, n)
    ctx = ctx_for(1, tile_rows=256, handle_model="straight")
    r = W.random_vector(16, (n, 3))
    Ho, go = ST.normal_equations(th, x, r, 1, 1e-2)
    JtJ, Jtr = ctx.jtj(dev(th), dev(x), dev(r, torch.float32), "bf16x3_mfma", "mixed")
    eh, eg = _rel(host(JtJ), Ho), _rel(host(Jtr), go)
    log(f"straight jtj N={n}: JtJ {eh:.3e} Jtr {eg:.3e}")
    assert eh < 1e-4 and eg < 1e-3


@pytest.mark.parametrize("compat", [0, 1])
@pytest.mark.parametrize("gram,prec,tol", [("fp64", "fp64", 1e-8), ("bf16x3_mfma", "mixed", None)])
def test_lm_step_small(compat, gram, prec, tol):
    th_true = _handles(9, 6)
    th0 = th_true.copy()
    rng = np.random.default_rng(10)
    th0[:, :4] += 0.01 * rng.standard_normal((6, 4))
    th0[:, 4:] += 0.1 * rng.standard_normal((6, 6))
    if compat:
        th_true = ST.reproject(th_true, 1)
    x = _points(11, th_true, 4096, near_frac=0.0)
    T = ST.evaluate(th_true, x, np.full(3, 0.5), 1, 1e-2) + 0.1 * W.random_vector(12, (4096, 3))
    lam = 1e-1
    st_o = O.LMState(lam=lam, mean_rule=0, compat=bool(compat))
    th_o, st_o = ST.lm_step(th0, x, T, st_o, 1, 1e-2)
    if tol is None:
        tol = mixed_step_tol(ST.normal_equations(th0, x, np.zeros_like(T), 1, 1e-2)[0], lam)
    ctx = ctx_for(1, handle_model="straight")
    th = dev(th0)
    st = B.new_lm_state(lam, 0, compat=compat)
    ctx.lm_step(th, dev(x), dev(T), st, gram, prec)
    d_o = th_o - th0
    d = host(th) - th0
    e = _rel(d, d_o) if st_o.accepted else float(np.abs(d).max())
    log(f"straight lm {gram}/{prec} compat={compat}: accepted {st.accepted}/{st_o.accepted}, "
        f"loss {st.loss_before:.9e}/{st_o.loss_before:.9e}, step rel err {e:.3e} (bar {tol:.3e})")
    assert bool(st.accepted) == bool(st_o.accepted)
    assert st.lam == pytest.approx(st_o.lam)
    assert e < tol
    if compat and st.accepted:
        assert st.compat_violation < 1e-12


def test_paper_workload_full_size_sampled():
    """500 Sobol-placed straight handles, S = 1, 100,000 samples (the timed paper-native
    workload): forward at full size on 1,024 sampled rows, and the adjoint of a 1,024-sample
    subset against the oracle."""
    wl = W.make_config(W.PAPER_CONFIG)
    ctx = ctx_for(wl.S, handle_model="straight")
    xh = wl.samples(0)
    x = dev(xh)
    th = dev(wl.theta0)
    u64 = host(ctx.eval(th, x, wl.cbar_true, "fp64"))
    u32 = host(ctx.eval(th, x, wl.cbar_true, "mixed"))
    idx = wl.subsample(1024)
    uo = ST.evaluate(wl.theta0, xh[idx], wl.cbar_true, wl.S, wl.eps)
    e64, e32 = _rel(u64[idx], uo), float(np.abs(u32[idx] - uo).max())
    xs = np.ascontiguousarray(xh[idx])
    g = W.random_vector(13, (1024, 3))
    go = ST.vjp(wl.theta0, xs, g, wl.S, wl.eps)
    g64 = host(ctx.vjp(th, dev(xs), dev(g), "fp64"))
    g32 = host(ctx.vjp(th, dev(xs), dev(g, torch.float32), "mixed"))
    r64, r32 = _rel(g64, go), _rel(g32, go)
    log(f"paper workload: forward fp64 {e64:.2e}, mixed abs {e32:.2e}; adjoint fp64 {r64:.2e}, mixed {r32:.2e}")
    assert e64 < 1e-10 and e32 < 1e-4
    assert r64 < 1e-10 and r32 < 1e-3


def test_paper_workload_full_size_normal_equations_and_step():
    """The paper-native workload at full size (500 straight handles, 100,000 samples in two
    balanced sample tiles): J^T J of the split-BF16 / mixed path element by element against the
    FP64 Gram's J^T J on the same batch (within 1e-4 of the largest entry), and the mixed LM step
    (split-BF16 and FP32 MFMA) from the same start within 1.5e-3 (relative, 2-norm) of the FP64
    step."""
    wl = W.make_config(W.PAPER_CONFIG)
    ctx = ctx_for(wl.S, handle_model="straight")
    x = dev(wl.samples(0))
    th0 = dev(wl.theta0)
    T = ctx.eval(dev(wl.theta_true), x, wl.cbar_true, "fp64") + wl.spec.sigma * dev(wl.noise(0))
    T = T.clamp_(max=wl.spec.target_max)
    r = 0.1 * wl.noise(0)
    H64 = host(ctx.jtj(th0, x, dev(r), "fp64", "fp64")[0])
    scale = np.abs(H64).max()
    for gram in ("bf16x3_mfma", "fp32_mfma"):
        e = float(np.abs(host(ctx.jtj(th0, x, dev(r, torch.float32), gram, "mixed")[0]) - H64).max() / scale)
        log(f"paper workload J^T J {gram}/mixed vs fp64: {e:.3e}")
        assert e < 1e-4
    # the first damping (from 1e-3 up) at which the FP64 step is accepted
    for lam in (1e-3, 1e-2, 1e-1, 1.0, 10.0):
        th = th0.clone()
        st = B.new_lm_state(lam, 0)
        ctx.lm_step(th, x, T, st, "fp64", "fp64")
        if st.accepted:
            break
    assert st.accepted
    d = {"fp64": (th - th0).flatten()}
    for gram in ("bf16x3_mfma", "fp32_mfma"):
        th = th0.clone()
        st = B.new_lm_state(lam, 0)
        ctx.lm_step(th, x, T, st, gram, "mixed")
        assert st.accepted
        d[gram] = (th - th0).flatten()
    e = {g: float(torch.linalg.norm(d[g] - d["fp64"]) / torch.linalg.norm(d["fp64"])) for g in ("bf16x3_mfma", "fp32_mfma")}
    log(f"paper workload LM step direction vs FP64 (lambda {lam:g}): {e}")
    assert e["bf16x3_mfma"] < 1.5e-3 and e["fp32_mfma"] < 1.5e-3


def test_handle_model_validated():
    with pytest.raises(ValueError):
        B.Context(segs_per_handle=1, handle_model="quadratic")
    ctx = ctx_for(1, handle_model="straight")
    with pytest.raises(ValueError):
        ctx.eval(dev(np.zeros((2, 20))), dev(np.full((4, 2), 0.5)))
