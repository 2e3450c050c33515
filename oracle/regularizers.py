"""Regularisation terms of the LM step (Sec. 4.4) and handle pruning.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Each term R(theta) enters the step through its analytic gradient and Hessian, added to the
loss Jacobian and the approximate Hessian of Eq. optimstep; the accept test compares the
reconstruction loss plus R.  Terms, for handles with end points E0, E1 (straight: A, B;
cubic: P0, P3) and jump vectors w (straight: wd, wc; cubic: wd0, wd1, wc0, wc1):

  length    mu_l (l - l_max)^2 for every handle with l = |E1 - E0| > l_max, else 0;
  snapping  mu_s |e - e'|^2 for every pair of end points e, e' of different handles that
            are closer than d_snap and are each other's lowest snapping score, the score
            being  mix * |e - e'| / d_snap + (1 - mix) * (1 - |tau . tau'|)  with tau the unit
            chord direction of each handle (ties to the lower end point index; the pairs are
            chosen at the current parameters and kept for the trial point);
  sparsity  lam * t * tanh(sqrt(w . w + eps^2) / t) for every jump vector, lam = lam_d for
            wd and lam_c for wc.

The approximate Hessian of the step must stay positive definite for its Cholesky solve
(Sec. 4.3).  The length and snapping Hessians are positive semi-definite as they are; the
sparsity term saturates, so its curvature along w (the second derivative of the tanh in
s = sqrt(w.w + eps^2)) is negative: that radial part is left out and the term contributes
f'(s)/s (I - u u^T), u = w / s, its curvature across w.

Pruning removes the handles whose wd and wc norms (the larger over both ends for cubic
handles) are both below a threshold.

Pins (tests/test_oracle_regularizers.py): central differences of every gradient and Hessian,
the closed forms below and above the length threshold, the saturation of the sparsity term,
hand-built snapping configurations, and the LM step with the terms rebuilt from its
definition.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Reg:
    length_weight: float = 0.0
    length_max: float = 0.0
    snap_weight: float = 0.0
    snap_dist: float = 0.0
    snap_mix: float = 0.5
    sparse_wd: float = 0.0
    sparse_wc: float = 0.0
    sparse_t: float = 1.0
    sparse_eps: float = 0.0

    def active(self) -> bool:
        return self.length_weight > 0 or self.snap_weight > 0 or self.sparse_wd > 0 or self.sparse_wc > 0


def layout(Q: int):
    """Columns of one handle: (E0 x, E0 y), (E1 x, E1 y), [(wd columns)], [(wc columns)]."""
    if Q == 10:
        return (0, 1), (2, 3), [(4, 5, 6)], [(7, 8, 9)]
    return (0, 1), (6, 7), [(8, 9, 10), (11, 12, 13)], [(14, 15, 16), (17, 18, 19)]


def endpoints(theta) -> np.ndarray:
    """[2H, 2]: end point 2h + j of handle h (j = 0 first, 1 last)."""
    theta = np.asarray(theta, dtype=np.float64)
    e0, e1, _, _ = layout(theta.shape[1])
    out = np.empty((2 * theta.shape[0], 2))
    out[0::2] = theta[:, list(e0)]
    out[1::2] = theta[:, list(e1)]
    return out


def length_term(theta, mu: float, lmax: float):
    """(R, grad [P], Hess [P, P]) of the handle length penalty."""
    theta = np.asarray(theta, dtype=np.float64)
    H, Q = theta.shape
    P = H * Q
    g = np.zeros(P)
    Hm = np.zeros((P, P))
    R = 0.0
    if mu <= 0:
        return R, g, Hm
    e0, e1, _, _ = layout(Q)
    for h in range(H):
        d = theta[h, list(e1)] - theta[h, list(e0)]
        ln = float(np.hypot(*d))
        if ln <= lmax:
            continue
        ex = ln - lmax
        R += mu * ex * ex
        tau = d / ln
        # d l / d E1 = tau, d l / d E0 = -tau;  d^2 l / d E1^2 = (I - tau tau^T) / l
        gl = 2.0 * mu * ex * tau
        Hb = 2.0 * mu * (np.outer(tau, tau) + ex / ln * (np.eye(2) - np.outer(tau, tau)))
        c0 = [h * Q + c for c in e0]
        c1 = [h * Q + c for c in e1]
        g[c1] += gl
        g[c0] -= gl
        Hm[np.ix_(c1, c1)] += Hb
        Hm[np.ix_(c0, c0)] += Hb
        Hm[np.ix_(c0, c1)] -= Hb
        Hm[np.ix_(c1, c0)] -= Hb
    return R, g, Hm


def snap_pairs(theta, dist: float, mix: float) -> list:
    """Mutually best end point pairs (i, j), i < j, end point indices as in endpoints()."""
    theta = np.asarray(theta, dtype=np.float64)
    E = endpoints(theta)
    n = E.shape[0]
    chord = E[1::2] - E[0::2]
    ln = np.sqrt(chord[:, 0] * chord[:, 0] + chord[:, 1] * chord[:, 1])
    tau = np.where(ln[:, None] > 0, chord / np.where(ln > 0, ln, 1.0)[:, None], 0.0)
    best = np.full(n, -1)
    for i in range(n):
        bs = np.inf
        for j in range(n):
            if j // 2 == i // 2:
                continue
            dx, dy = E[i, 0] - E[j, 0], E[i, 1] - E[j, 1]
            d = float(np.sqrt(dx * dx + dy * dy))
            if not d < dist:
                continue
            dot = abs(tau[i // 2, 0] * tau[j // 2, 0] + tau[i // 2, 1] * tau[j // 2, 1])
            s = mix * (d / dist) + (1.0 - mix) * (1.0 - dot)
            if s < bs:
                bs, best[i] = s, j
    return [(i, int(best[i])) for i in range(n) if best[i] > i and best[best[i]] == i]


def snap_term(theta, mu: float, pairs):
    """(R, grad, Hess) of mu |e - e'|^2 over the given end point pairs."""
    theta = np.asarray(theta, dtype=np.float64)
    H, Q = theta.shape
    P = H * Q
    g = np.zeros(P)
    Hm = np.zeros((P, P))
    R = 0.0
    if mu <= 0:
        return R, g, Hm
    e0, e1, _, _ = layout(Q)

    def cols(e):
        return [(e // 2) * Q + c for c in (e0 if e % 2 == 0 else e1)]

    E = endpoints(theta)
    I2 = 2.0 * mu * np.eye(2)
    for i, j in pairs:
        d = E[i] - E[j]
        R += mu * float(d @ d)
        ci, cj = cols(i), cols(j)
        g[ci] += 2.0 * mu * d
        g[cj] -= 2.0 * mu * d
        Hm[np.ix_(ci, ci)] += I2
        Hm[np.ix_(cj, cj)] += I2
        Hm[np.ix_(ci, cj)] -= I2
        Hm[np.ix_(cj, ci)] -= I2
    return R, g, Hm


def sparsity_term(theta, lam_d: float, lam_c: float, t: float, eps: float):
    """(R, grad, Hess) of lam t tanh(sqrt(w.w + eps^2)/t) over every jump vector w (Hessian
    without its negative radial curvature)."""
    theta = np.asarray(theta, dtype=np.float64)
    H, Q = theta.shape
    P = H * Q
    g = np.zeros(P)
    Hm = np.zeros((P, P))
    R = 0.0
    _, _, wd, wc = layout(Q)
    for lam, groups in ((lam_d, wd), (lam_c, wc)):
        if lam <= 0:
            continue
        for h in range(H):
            for grp in groups:
                c = [h * Q + k for k in grp]
                w = theta[h, list(grp)]
                s = float(np.sqrt(w @ w + eps * eps))
                th = np.tanh(s / t)
                sech2 = 1.0 - th * th
                R += lam * t * th
                if s == 0.0:
                    continue
                f1 = lam * sech2                       # d/ds of lam t tanh(s/t) (> 0)
                u = w / s
                g[c] += f1 * u
                Hm[np.ix_(c, c)] += f1 / s * (np.eye(3) - np.outer(u, u))
    return R, g, Hm


def terms(theta, reg: Reg, pairs=None):
    """Total (R, grad, Hess, pairs); snapping pairs chosen at theta unless given."""
    if pairs is None:
        pairs = snap_pairs(theta, reg.snap_dist, reg.snap_mix) if reg.snap_weight > 0 else []
    R1, g1, H1 = length_term(theta, reg.length_weight, reg.length_max)
    R2, g2, H2 = snap_term(theta, reg.snap_weight, pairs)
    R3, g3, H3 = sparsity_term(theta, reg.sparse_wd, reg.sparse_wc, reg.sparse_t, reg.sparse_eps)
    return R1 + R2 + R3, g1 + g2 + g3, H1 + H2 + H3, pairs


def value(theta, reg: Reg, pairs) -> float:
    return terms(theta, reg, pairs)[0]


def prune(theta, threshold: float) -> np.ndarray:
    """Handles kept (in order): those with the wd norm or the wc norm (the larger over the
    handle's ends) at or above the threshold."""
    theta = np.asarray(theta, dtype=np.float64)
    _, _, wd, wc = layout(theta.shape[1])
    nd = np.max([np.linalg.norm(theta[:, list(g)], axis=1) for g in wd], axis=0)
    nc = np.max([np.linalg.norm(theta[:, list(g)], axis=1) for g in wc], axis=0)
    return theta[(nd >= threshold) | (nc >= threshold)].copy()
