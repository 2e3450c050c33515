"""Pins of the oracle's compatibility enforcement (Sec. 3.1.2 compatibility condition,
Sec. 4.3 enforcement in the LM step), checked against independent computations:

* the flux int over the handles of w_c by direct trapezoidal integration along the
  polylines (arc length, w_c interpolated between segment end values), against
  a_c . theta from the closed-form coefficients;
* a straight, uniformly parametrised handle: alpha = beta = L / 2;
* the constrained step against the null-space form Z (Z^T Hd Z)^{-1} Z^T g with Z
  an orthonormal basis of {delta : A^T delta = 0} (scipy.linalg.null_space);
* the re-projection: exact feasibility, geometry untouched, minimal (parallel to a_c) change;
* one LM step with the enforcement keeps the parameters feasible.
"""
import numpy as np
import pytest
from scipy.linalg import cho_factor, cho_solve, null_space

import oracle as O
from paper_2602_05492_amd import workload as W


def _flux_by_quadrature(theta, S, n_sub=33):
    """int over the polylines of w_c, trapezoid with n_sub points per segment (exact for the
    piecewise-linear jump, up to rounding)."""
    p = O.handle_vertices(theta, S)
    t = np.arange(S + 1) / S
    out = np.zeros(3)
    for h in range(theta.shape[0]):
        wc_v = (1 - t)[:, None] * theta[h, 14:17] + t[:, None] * theta[h, 17:20]   # at the vertices
        for k in range(S):
            a, b = p[h, k], p[h, k + 1]
            L = np.linalg.norm(b - a)
            if L <= O.DEGENERATE_LENGTH:
                continue
            s = np.linspace(0.0, 1.0, n_sub)
            w = (1 - s)[:, None] * wc_v[k] + s[:, None] * wc_v[k + 1]
            out += np.trapezoid(w, s * L, axis=0)
    return out


def test_compat_vectors_match_direct_integration():
    th = W.random_handles(71, 5)
    S = 7
    A = O.compat_vectors(th, S)
    got = A.T @ th.reshape(-1)
    ref = _flux_by_quadrature(th, S)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    # only the wc columns of theta enter
    assert np.all(A.reshape(5, 20, 3)[:, :14] == 0.0)


def test_compat_straight_handle_closed_form():
    th = np.zeros((1, 20))
    p0, d = np.array([0.2, 0.3]), np.array([0.45, -0.1])
    for j in range(4):                          # evenly spaced collinear control points: B(t) = p0 + t d
        th[0, 2 * j:2 * j + 2] = p0 + d * j / 3.0
    A = O.compat_vectors(th, 16).reshape(20, 3)
    L = np.linalg.norm(d)
    for c in range(3):
        assert A[14 + c, c] == pytest.approx(L / 2, rel=1e-13)
        assert A[17 + c, c] == pytest.approx(L / 2, rel=1e-13)


def test_constrained_step_feasible_and_equals_null_space_form():
    rng = np.random.default_rng(72)
    H, S = 3, 6
    P = 20 * H
    th = W.random_handles(72, H)
    A = O.compat_vectors(th, S)
    B = rng.standard_normal((P, P))
    JtJ = B @ B.T / P + 1e-3 * np.eye(P)
    g = rng.standard_normal(P)
    lam = 1e-2
    delta = O.constrained_step(JtJ, g, lam, A)
    assert np.abs(A.T @ delta).max() <= 1e-12 * np.abs(A).max() * np.abs(delta).max()
    d = np.maximum(np.diag(JtJ), 1e-12 * np.diag(JtJ).max())
    Hd = JtJ + lam * np.diag(d)
    Z = null_space(A.T)
    ref = Z @ np.linalg.solve(Z.T @ Hd @ Z, Z.T @ g)
    assert np.allclose(delta, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    # without constraints it is the plain damped step
    assert np.allclose(O.constrained_step(JtJ, g, lam, np.zeros((P, 3))), cho_solve(cho_factor(Hd, lower=True), g))


def test_reproject_exact_and_minimal():
    th = W.random_handles(73, 4)
    S = 5
    out = O.reproject(th, S)
    A = O.compat_vectors(out, S)
    assert np.abs(A.T @ out.reshape(-1)).max() <= 1e-14 * np.abs(out).max() * np.abs(A).max()
    assert np.all(out[:, :14] == th[:, :14])                      # geometry and wd untouched
    diff = (out - th).reshape(-1)
    for c in range(3):
        idx = np.nonzero(A[:, c])[0]
        a, dc = A[idx, c], diff[idx]
        # the change of channel c is a multiple of a_c (orthogonal projection)
        assert np.abs(dc - a * (dc @ a) / (a @ a)).max() <= 1e-14 * max(np.abs(dc).max(), 1e-300)


def test_lm_step_with_enforcement_stays_feasible():
    wl = W.make_config(1)
    S, eps, ps = 8, 1e-2, 32
    x = wl.samples(0, n=384)
    th0 = O.reproject(wl.theta0, S)
    T = O.evaluate(O.reproject(wl.theta_true, S), x, wl.cbar_true, S, eps, ps) + 0.05 * wl.noise(0)[:384]
    st = O.LMState(lam=1e-1, mean_rule=0, compat=True)
    th1, st = O.lm_step(th0, x, T, st, S, eps, ps)
    assert st.accepted
    A = O.compat_vectors(th1, S)
    assert np.abs(A.T @ th1.reshape(-1)).max() <= 1e-13 * np.abs(th1).max() * np.abs(A).max()
