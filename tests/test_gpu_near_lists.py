"""Mixed precision with every branch of the near-pair lists: listed pairs, and
wavefronts whose list slice overflows (their samples are flagged and redone
with the near pairs inline).

The mixed path evaluates a pair in float64 when both segment end points lie
within max(2 nf, nf + 1) * L of the sample, nf = near_factor (2 nf * L for the
factors >= 1 used here; a factor of 0.5 takes the radius 1.5 L, which still
contains every sample within 0.5 L of the segment).  near_factor = 1.5 overflows the
slices of most wavefronts of the medium workload (within such a wavefront some
samples' pairs are listed, the rest flagged); near_factor = 60 makes every
pair near, so every slice overflows and every sample takes the flagged path.
Each case is compared with the FP64 oracle at the mixed-precision bars of the
other GPU tests (colour 1e-4 absolute, gradient 1e-3 relative, J^T J 1e-4 and
J^T r 1e-3 relative, LM step 10 u kappa: helpers.mixed_step_tol).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_05492_amd import bem as B
from paper_2602_05492_amd import workload as W
from helpers import ctx_for, dev, host, log, mixed_step_tol

pytestmark = pytest.mark.gpu

SLOTS_PER_WAVE = 1024          # list capacity of one 64-sample wavefront
FACTORS = [1.5, 60.0]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _overflowing_waves(theta, x, S, nf):
    """Fraction of 64-sample wavefronts whose near handle-segment pairs (float64 reading of the
    predicate) exceed one slice; the outer elements only add to the count."""
    t = np.arange(S + 1) / S
    B3 = np.stack([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t ** 2 * (1 - t), t ** 3], 1)
    P = np.einsum("tc,hcd->htd", B3, theta[:, :8].reshape(-1, 4, 2))
    a, b = P[:, :-1].reshape(-1, 2), P[:, 1:].reshape(-1, 2)
    L2 = ((b - a) ** 2).sum(1)
    r2 = (2 * nf) ** 2 * L2
    da = ((a[None] - x[:, None]) ** 2).sum(2)
    db = ((b[None] - x[:, None]) ** 2).sum(2)
    near = (da < r2[None]) & (db < r2[None])
    per_wave = near.sum(1)[: len(x) // 64 * 64].reshape(-1, 64).sum(1)
    return float((per_wave > SLOTS_PER_WAVE).mean())


def _case(n):
    wl = W.make_config(2)
    idx = wl.subsample(n)
    return wl, wl.samples(0)[idx]


@pytest.mark.parametrize("nf", FACTORS)
def test_overflow_is_exercised(nf):
    wl, x = _case(2048)
    frac = _overflowing_waves(wl.theta_true, x, wl.S, nf)
    log(f"near_factor {nf}: {frac:.2f} of the wavefronts overflow")
    assert (0.0 < frac < 1.0) if nf == 1.5 else frac == 1.0


@pytest.mark.parametrize("nf", FACTORS)
def test_eval_mixed_near_lists(nf):
    wl, x = _case(3000)
    ctx = ctx_for(wl.S, near_factor=nf)
    got = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, "mixed"))
    ref = O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps)
    err = float(np.abs(got - ref).max())
    log(f"near_factor {nf}: mixed eval max abs err {err:.3e}")
    assert err < 1e-4


@pytest.mark.parametrize("nf", FACTORS)
def test_vjp_mixed_near_lists(nf):
    wl, x = _case(3000)
    ctx = ctx_for(wl.S, near_factor=nf)
    g = W.random_vector(61, (len(x), 3))
    got = host(ctx.vjp(dev(wl.theta_true), dev(x), dev(g, torch.float32), "mixed"))
    ref = O.vjp(wl.theta_true, x, g, wl.S, wl.eps)
    err = _rel(got, ref)
    log(f"near_factor {nf}: mixed vjp rel err {err:.3e}")
    assert err < 1e-3


@pytest.mark.parametrize("nf", FACTORS)
def test_jtj_mixed_near_lists(nf):
    """Several sample tiles (1024 rows each, the last ragged), so tiles start at non-zero wavefronts."""
    wl, x = _case(3000)
    ctx = ctx_for(wl.S, near_factor=nf, tile_rows=1024)
    r = W.random_vector(62, (len(x), 3))
    Ho, go = O.normal_equations(wl.theta_true, x, r, wl.S, wl.eps)
    for gram in ["bf16x3_mfma", "fp64"]:
        JtJ, Jtr = ctx.jtj(dev(wl.theta_true), dev(x), dev(r, torch.float32), gram, "mixed")
        eh, eg = _rel(host(JtJ), Ho), _rel(host(Jtr), go)
        log(f"near_factor {nf}: jtj {gram}/mixed rel err JtJ {eh:.3e} Jtr {eg:.3e}")
        assert eh < 1e-4 and eg < 1e-3


@pytest.mark.parametrize("nf", FACTORS)
def test_lm_step_mixed_near_lists(nf):
    """lm_step hands the forward sweep's list to the adjoint and the J tiles."""
    wl, x = _case(4096)
    T = O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps) + wl.spec.sigma * W.random_vector(63, (len(x), 3))
    ctx = ctx_for(wl.S, near_factor=nf, tile_rows=1024)
    lam = 1e-1                                          # a damping at which the step is accepted
    st_o = O.LMState(lam=lam, mean_rule=0)
    th_o, st_o = O.lm_step(wl.theta0, x, T, st_o, wl.S, wl.eps)
    tol = mixed_step_tol(O.normal_equations(wl.theta0, x, np.zeros_like(T), wl.S, wl.eps)[0], lam)
    th = dev(wl.theta0)
    st = B.new_lm_state(lam, 0)
    ctx.lm_step(th, dev(x), dev(T), st, "bf16x3_mfma", "mixed")
    assert st_o.accepted
    assert bool(st.accepted) == bool(st_o.accepted)
    assert abs(st.loss_before - st_o.loss_before) <= 1e-4 * st_o.loss_before
    d_o = th_o - wl.theta0
    d = host(th) - wl.theta0
    e = float(np.abs(d - d_o).max() / np.abs(d_o).max()) if st_o.accepted else float(np.abs(d).max())
    log(f"near_factor {nf}: lm step rel err {e:.3e} (bar {tol:.3e}), accepted {st.accepted}")
    assert e < tol


def test_eval_mixed_small_near_factor():
    """near_factor = 0.5 on the near-singular stress samples (10% within 1e-3 of a segment): the
    radius max(2 nf, nf + 1) L = 1.5 L still sends every pair closer than 0.5 L to the float64
    evaluation; colour within the mixed-precision bar of the oracle."""
    wl = W.make_config(3)
    x = wl.samples(0, n=4096)                          # 410 of them within 1e-3 of a segment
    th = wl.theta_true
    ctx = ctx_for(wl.S, near_factor=0.5)
    got = host(ctx.eval(dev(th), dev(x), wl.cbar_true, "mixed"))
    ref = O.evaluate(th, x, wl.cbar_true, wl.S, wl.eps)
    err = float(np.abs(got - ref).max())
    log(f"near_factor 0.5: mixed eval max abs err {err:.3e}")
    assert err < 1e-4


def _boundary_band(n, seed, per_side=256):
    """n samples between 1e-7 and 1e-4 inside the unit square's edges, each within 1e-6 to 1e-2
    element lengths of a junction of two outer elements, ordered along the perimeter so that each
    64-sample wavefront covers a short stretch of one or two edges: its bounding box is small, and
    the wavefront skips the near tests of every other group of outer elements.  There a float32
    value of a single element's double layer is off by up to 3e-2 (the angle it subtends turns
    fast), so a near pair missed by the culling shows in the colour's beta rows of J^T J."""
    rng = np.random.default_rng(seed)
    off = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0) * 10.0 ** rng.uniform(-6.0, -2.0, n)
    s = np.sort(np.mod((rng.integers(0, 4 * per_side, n) + off) / per_side, 4.0))
    d = 10.0 ** rng.uniform(-7.0, -4.0, n)
    side, t = np.floor(s).astype(int), s - np.floor(s)
    x = np.empty((n, 2))
    for k, (px, py) in enumerate([(t, d), (1.0 - d, t), (1.0 - t, 1.0 - d), (d, 1.0 - t)]):
        m = side == k
        x[m, 0], x[m, 1] = px[m], py[m]
    return x


def test_eval_mixed_boundary_band():
    """Samples in the boundary band, wavefronts compact along it: the forward sweep's culled
    element groups; colour within the mixed-precision bar of the oracle."""
    wl = W.make_config(2)
    x = _boundary_band(4096, 71)
    ctx = ctx_for(wl.S)
    got = host(ctx.eval(dev(wl.theta_true), dev(x), wl.cbar_true, "mixed"))
    ref = O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps)
    err = float(np.abs(got - ref).max())
    log(f"boundary band: mixed eval max abs err {err:.3e}")
    assert err < 1e-4


def test_vjp_and_jtj_mixed_boundary_band():
    """The same band through the classification of the adjoint and of the J tiles (element groups
    culled per wavefront there too): every pair of a sample with an outer element within the near
    radius must reach the float64 list for the beta rows of J^T J to meet their bar."""
    wl = W.make_config(2)
    x = _boundary_band(2048, 72)
    ctx = ctx_for(wl.S, tile_rows=1024)
    g = W.random_vector(73, (len(x), 3))
    got = host(ctx.vjp(dev(wl.theta_true), dev(x), dev(g, torch.float32), "mixed"))
    ref = O.vjp(wl.theta_true, x, g, wl.S, wl.eps)
    ev = _rel(got, ref)
    Ho, go = O.normal_equations(wl.theta_true, x, g, wl.S, wl.eps)
    JtJ, Jtr = ctx.jtj(dev(wl.theta_true), dev(x), dev(g, torch.float32), "bf16x3_mfma", "mixed")
    eh, eg = _rel(host(JtJ), Ho), _rel(host(Jtr), go)
    log(f"boundary band: mixed vjp rel err {ev:.3e}, JtJ {eh:.3e}, Jtr {eg:.3e}")
    assert ev < 1e-3 and eh < 1e-4 and eg < 1e-3


def _morton_sorted(x, bits=10):
    """x reordered along a Z curve over a 2^bits grid of the unit square (wavefronts of nearby
    samples)."""
    q = np.clip((x * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(len(x), dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b) | ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return x[np.argsort(key, kind="stable")]


def test_near_singular_compact_wavefronts():
    """Samples within 1e-3 of the handle segments, ordered along a Z curve so that each wavefront's
    box is small and most groups of 32 segments are skipped per wavefront in the forward sweep, the
    classification and the J-tile feature kernel (16 segments per handle).  Every pair nearer than
    the near radius must reach the float64 evaluation, where the float32 forms fail; colour,
    gradient, J^T J and J^T r within the mixed-precision bars of the oracle."""
    wl = W.make_config(2)
    rng = np.random.default_rng(74)
    x = _morton_sorted(W.near_samples(rng, wl.theta_true[:, :8].reshape(-1, 4, 2), wl.S, 4096))
    ctx = ctx_for(wl.S, tile_rows=1024)
    th = dev(wl.theta_true)
    u = host(ctx.eval(th, dev(x), wl.cbar_true, "mixed"))
    eu = float(np.abs(u - O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps)).max())
    g = W.random_vector(75, (len(x), 3))
    ev = _rel(host(ctx.vjp(th, dev(x), dev(g, torch.float32), "mixed")), O.vjp(wl.theta_true, x, g, wl.S, wl.eps))
    Ho, go = O.normal_equations(wl.theta_true, x, g, wl.S, wl.eps)
    JtJ, Jtr = ctx.jtj(th, dev(x), dev(g, torch.float32), "bf16x3_mfma", "mixed")
    eh, eg = _rel(host(JtJ), Ho), _rel(host(Jtr), go)
    log(f"near-singular, compact wavefronts: colour {eu:.3e}, vjp {ev:.3e}, JtJ {eh:.3e}, Jtr {eg:.3e}")
    assert eu < 1e-4 and ev < 1e-3 and eh < 1e-4 and eg < 1e-3
