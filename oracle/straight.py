"""Straight handles: the paper's own handle representation (Sec. 3.2 restricts handles to
line segments; Sec. 4.1 gives each handle its two end points and colour and derivative
jumps that are constant over the handle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Parameters per handle (10 float64, the column order of every Jacobian here):
  [Ax Ay Bx By | wd RGB | wc RGB]
The handle is the segment A -> B, cut into S equal straight pieces; wd and wc take the same
value at every point of it.

The oracle evaluates a straight handle as the cubic handle of bem_oracle with control points
P_j = A + (j/3)(B - A), j = 0..3, and equal jumps at both ends.  A cubic Bezier curve with
evenly spaced collinear control points is A + t (B - A) (the Bernstein polynomials reproduce
linear functions), so its polyline vertices are A + (k/S)(B - A) and its jumps are constant:
the two handles are the same set of segments with the same densities.  The map
theta20 = theta10 E^T is linear, so every derivative is the cubic one times E (chain rule),
and the compatibility vectors are E^T a_c.

Pins (tests/test_oracle_straight.py): the vertices and jumps of the embedded handle against
the closed form; the field of a one-piece handle against adaptive quadrature of the kernels;
invariance of the field under subdivision (constant densities on a straight segment); central
finite differences of the Jacobian in the 10 parameters; the flux of w_c as |B - A| w_c.
"""
from __future__ import annotations

import numpy as np

from . import bem_oracle as O

PARAMS = 10


def embedding_matrix() -> np.ndarray:
    """E [20, 10]: cubic parameters of one handle from its straight parameters."""
    E = np.zeros((20, PARAMS))
    for j in range(4):
        for d in range(2):
            E[2 * j + d, d] = 1.0 - j / 3.0
            E[2 * j + d, 2 + d] = j / 3.0
    for c in range(3):
        E[8 + c, 4 + c] = E[11 + c, 4 + c] = 1.0        # wd at both ends
        E[14 + c, 7 + c] = E[17 + c, 7 + c] = 1.0       # wc at both ends
    return E


E = embedding_matrix()


def embed(theta) -> np.ndarray:
    """[H, 10] -> the equivalent cubic handles [H, 20]."""
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, PARAMS)
    return theta @ E.T


def evaluate(theta, x, cbar, S: int, eps: float, per_side: int = 256) -> np.ndarray:
    return O.evaluate(embed(theta), x, cbar, S, eps, per_side)


def jacobian(theta, x, S: int, eps: float, per_side: int = 256) -> np.ndarray:
    """du_c/dtheta [n, 3, 10H]."""
    H = np.asarray(theta).shape[0]
    J = O.jacobian(embed(theta), x, S, eps, per_side)
    n = J.shape[0]
    return np.einsum("nchq,qp->nchp", J.reshape(n, 3, H, 20), E).reshape(n, 3, PARAMS * H)


def vjp(theta, x, gbar, S: int, eps: float, per_side: int = 256) -> np.ndarray:
    """sum_x sum_c gbar_c(x) du_c/dtheta(x), [H, 10]."""
    return O.vjp(embed(theta), x, gbar, S, eps, per_side) @ E


def normal_equations(theta, x, resid, S: int, eps: float, per_side: int = 256):
    """(1/N) sum_x J^T J and (1/N) sum_x J^T r in the straight parameters."""
    H = np.asarray(theta).shape[0]
    JtJ, Jtr = O.normal_equations(embed(theta), x, resid, S, eps, per_side)
    JtJ = np.einsum("qp,aqbr,rs->apbs", E, JtJ.reshape(H, 20, H, 20), E).reshape(PARAMS * H, PARAMS * H)
    return JtJ, (Jtr.reshape(H, 20) @ E).reshape(-1)


def compat_vectors(theta, S: int) -> np.ndarray:
    """A [10H, 3] with a_c . theta = int over the handles of w_c (Sec. 3.1.2)."""
    H = np.asarray(theta).shape[0]
    A = O.compat_vectors(embed(theta), S).reshape(H, 20, 3)
    return np.einsum("hqc,qp->hpc", A, E).reshape(PARAMS * H, 3)


def reproject(theta, S: int) -> np.ndarray:
    """Orthogonal projection of the wc parameters onto the compatibility condition (Sec. 4.3)."""
    return O.project_compatible(theta, compat_vectors(theta, S))


STRAIGHT = O.HandleModel(evaluate=evaluate, normal_equations=normal_equations, compat_vectors=compat_vectors,
                         reproject=reproject)


def lm_step(theta, x, T, state: O.LMState, S: int, eps: float, per_side: int = 256, reg=None):
    return O.lm_step(theta, x, T, state, S, eps, per_side, model=STRAIGHT, reg=reg)
