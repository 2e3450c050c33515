"""Plain, slow FP64 CPU oracle of the differential-BEM hot path.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product.  It shares no code with
the HIP library and takes every step in the paper's order, in float64:

  handles -> straight segments            (Sec. 3.2, handles as line segments;
                                            Bezier polylines are the reading here)
  handle term f(x) by exact segment
  integrals of the regularised kernels     (Eq. handleterm, Eq. fundsol, Sec. 3.1.3)
  Galerkin boundary matrix, 3-pt Gauss     (Eq. bie_galerkin)
  truncated-SVD solve (drop smallest s.v.) (Sec. 3.1.3, null space)
  interior evaluation + mean colour        (Sec. 3.1.3, Eq. bie with alpha = 1)
  Jacobian: differential BIE, same matrix  (Eq. diffbie, Sec. 3.2 discretisation)
  normal equations, LM step, damping       (Eq. optimstep, Eq. losshessian,
                                            Eq. lossjacobian, Sec. 4.3)
  compatibility condition: constrained     (Sec. 3.1.2 compatibility, Sec. 4.3
  step and re-projection of w_c             enforcement)

Segment integrals are the antiderivatives of the two kernels evaluated at the
segment ends (exactly the integral the paper approximates by quadrature); the
differences of logarithms and arctangents at the two ends are formed with the
identities log a - log b = log1p((a-b)/b) and atan(p) - atan(q) =
atan2(p-q, 1+pq), which keep relative accuracy for short segments.
Derivatives with respect to segment end points use forward-mode dual numbers
through those same expressions.

Pins (tests/test_oracle_*.py): adaptive quadrature of single segment
integrals; the double-layer identity on closed polygons; Green's third
identity reproducing u = x and u = x^2 - y^2; the single layer of a circle;
matrix row sums and spectrum; jump relations across a handle; the
alpha = 1/2 jump of the outer boundary (the interior formula's limit on each
element equals the solved boundary value, which fixes the size of the
right-hand side against the matrix); the zero-Neumann condition converging
under refinement for compatible handles; central finite differences of every
derivative; exact colour recovery by one Gauss-Newton step; LM invariants.  The paper prints no worked numerical example, so no pin
is a value printed in the paper.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

from . import dual as du
from . import regularizers as rg

TWO_PI = 2.0 * np.pi
FOUR_PI = 4.0 * np.pi
GAUSS3_NODES = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])      # on [-1, 1]
GAUSS3_WEIGHTS = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])
PAIR_CHUNK = 1 << 19                                                 # sample x segment pairs per chunk


# =============================================================================
# handles -> segments
# =============================================================================
def bernstein3(t: np.ndarray) -> np.ndarray:
    """Cubic Bernstein basis [len(t), 4]."""
    t = np.asarray(t, dtype=np.float64)
    s = 1.0 - t
    return np.stack([s ** 3, 3.0 * s * s * t, 3.0 * s * t * t, t ** 3], axis=-1)


def vertex_params(S: int) -> np.ndarray:
    return np.arange(S + 1, dtype=np.float64) / S


def handle_vertices(theta: np.ndarray, S: int) -> np.ndarray:
    """Polyline vertices p_{h,k} = B(k/S) of each handle, [H, S+1, 2]."""
    ctrl = theta[:, :8].reshape(-1, 4, 2)
    return np.einsum("kj,hjc->hkc", bernstein3(vertex_params(S)), ctrl)


def handle_jumps(theta: np.ndarray, S: int):
    """Jumps at the vertices, linear in t between the two handle ends: wd, wc [H, S+1, 3]."""
    t = vertex_params(S)[None, :, None]
    wd = (1.0 - t) * theta[:, None, 8:11] + t * theta[:, None, 11:14]
    wc = (1.0 - t) * theta[:, None, 14:17] + t * theta[:, None, 17:20]
    return wd, wc


def segment_table(theta: np.ndarray, S: int) -> dict:
    """Straight segments a->b of all handles (K = H*S) and the jumps at both ends."""
    p = handle_vertices(theta, S)
    wd, wc = handle_jumps(theta, S)
    return {
        "a": p[:, :-1].reshape(-1, 2), "b": p[:, 1:].reshape(-1, 2),
        "wd_a": wd[:, :-1].reshape(-1, 3), "wd_b": wd[:, 1:].reshape(-1, 3),
        "wc_a": wc[:, :-1].reshape(-1, 3), "wc_b": wc[:, 1:].reshape(-1, 3),
    }


# =============================================================================
# segment integrals of the regularised kernels
# =============================================================================
def segment_moments(x, ax, ay, bx, by, eps: float):
    """Linear-density moments of one straight segment a->b seen from x.

    For the segment z(s) = a + s*tau, s in [0, L], with right normal n, the two
    kernels of the handle term (Eq. handleterm) with r^2 -> r^2 + eps^2 are
        double layer  -dG/dn_z = (1/2pi) n.(z-x) / (r^2+eps^2)
        single layer   G       = -(1/4pi) log(r^2+eps^2)
    and a density linear between its end values w(a), w(b) integrates to
        M_a w(a) + M_b w(b),  M_a = int k (1 - s/L) ds,  M_b = int k s/L ds.
    Returns (Md_a, Md_b, Ms_a, Ms_b), each broadcast to [n, K].
    x is [n, 2] float; ax.. are [K] arrays or Duals.
    """
    with np.errstate(divide="ignore", invalid="ignore"):
        return _segment_moments(x, ax, ay, bx, by, eps)


def _segment_moments(x, ax, ay, bx, by, eps: float):
    X = np.asarray(x, dtype=np.float64)[:, 0:1]
    Y = np.asarray(x, dtype=np.float64)[:, 1:2]
    vx = bx - ax
    vy = by - ay
    L = du.sqrt(vx * vx + vy * vy)
    tx = vx / L
    ty = vy / L
    nx, ny = ty, -tx                                   # right normal of the travel direction
    t0 = (X - ax) * tx + (Y - ay) * ty                 # foot of x along the segment
    h = (ax - X) * nx + (ay - Y) * ny                  # n.(z - x), constant along the segment
    u0 = -t0                                           # u = s - t0 runs from u0 to u1
    u1 = L - t0
    q2 = h * h + eps * eps
    q = du.sqrt(q2)
    r0 = u0 * u0 + q2                                  # |z - x|^2 + eps^2 at the two ends
    r1 = u1 * u1 + q2
    qv = du.value(q)
    r0v = du.value(r0)
    r1v = du.value(r1)
    # lam0 = log r0;  ell = log r1 - log r0 = log1p((r1 - r0)/r0), r1 - r0 = L (u0 + u1).
    # Limits at an end point (eps = 0, x = a or x = b): u log u^2 -> 0, r log r -> 0.
    lam0 = du.log(du.where(r0v > 0, r0, 1.0))
    ell = du.where(r0v > 0,
                   du.where(r1v > 0, du.log1p(L * (u0 + u1) / du.where(r0v > 0, r0, 1.0)), -lam0),
                   du.log(du.where(r1v > 0, r1, 1.0)))
    # Delta = atan(u1/q) - atan(u0/q) = atan2(q L, q^2 + u0 u1)  (q > 0)
    qs = du.where(qv > 0, q, 1.0)
    Delta = du.arctan2(q * L, q2 + u0 * u1)

    # double layer: int h/(u^2+q^2) du = (h/q) atan(u/q);  int u h/(u^2+q^2) du = (h/2) log(u^2+q^2)
    K0d = du.where(qv > 0, h / qs * Delta, 0.0) / TWO_PI       # principal value 0 on the line when eps = 0
    K1d = h * ell / FOUR_PI
    # single layer: int log(u^2+q^2) du = u log(u^2+q^2) - 2u + 2q atan(u/q)
    #   between u0 and u1:  u1 ell + L lam0 - 2L + 2 q Delta
    # int u log(u^2+q^2) du = ((u^2+q^2) log(u^2+q^2) - (u^2+q^2)) / 2
    #   between u0 and u1:  (r1 ell + (r1 - r0)(lam0 - 1)) / 2
    u1ell = du.where(r1v > 0, u1 * ell, 0.0)
    r1ell = du.where(r1v > 0, r1 * ell, 0.0)
    K0s = -(u1ell + L * lam0 - 2.0 * L + 2.0 * q * Delta) / FOUR_PI
    K1s = -0.5 * (r1ell + L * (u0 + u1) * (lam0 - 1.0)) / FOUR_PI

    # s = u + t0:  int k s/L ds = (K1 + t0 K0)/L
    Md_b = (K1d + t0 * K0d) / L
    Ms_b = (K1s + t0 * K0s) / L
    return K0d - Md_b, Md_b, K0s - Ms_b, Ms_b


# A segment shorter than this (in units of the domain width) is degenerate:
# its integral is below ~1e-11 for the regularised kernels and its end-point
# derivative has no limit as the length goes to 0, so it contributes nothing.
DEGENERATE_LENGTH = 1e-12


def _chunks(n: int, k: int):
    step = max(1, PAIR_CHUNK // max(k, 1))
    for s in range(0, n, step):
        yield slice(s, min(n, s + step))


def handle_term(x: np.ndarray, theta: np.ndarray, S: int, eps: float) -> np.ndarray:
    """f(x) of Eq. handleterm summed over all handle segments, [n, 3]."""
    seg = segment_table(theta, S)
    a, b = seg["a"], seg["b"]
    keep = np.hypot(*(b - a).T) > DEGENERATE_LENGTH     # degenerate segments carry no integral
    a, b = a[keep], b[keep]
    w = [seg[k][keep] for k in ("wd_a", "wd_b", "wc_a", "wc_b")]
    out = np.zeros((len(x), 3))
    for sl in _chunks(len(x), len(a)):
        M = segment_moments(x[sl], a[:, 0], a[:, 1], b[:, 0], b[:, 1], eps)
        for Mm, wm in zip(M, w):
            out[sl] += Mm @ wm
    return out


# =============================================================================
# outer boundary (Eq. bie_galerkin) and its truncated-SVD solve
# =============================================================================
def square_boundary(per_side: int):
    """Unit square, counter-clockwise from the origin, per_side equal elements per side."""
    c = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.0, 0.0]])
    t = np.arange(per_side + 1) / per_side
    ea, eb = [], []
    for s in range(4):
        p = c[s][None, :] + t[:, None] * (c[s + 1] - c[s])[None, :]
        ea.append(p[:-1])
        eb.append(p[1:])
    return np.concatenate(ea), np.concatenate(eb)


def gauss_points(ea: np.ndarray, eb: np.ndarray):
    """3-point Gauss points [M,3,2] and weights [M,3] (weights include |Gamma|/2)."""
    mid = 0.5 * (ea + eb)
    half = 0.5 * (eb - ea)
    pts = mid[:, None, :] + GAUSS3_NODES[None, :, None] * half[:, None, :]
    ln = np.hypot(half[:, 0], half[:, 1])
    return pts, GAUSS3_WEIGHTS[None, :] * ln[:, None]


def element_normals(ea: np.ndarray, eb: np.ndarray) -> np.ndarray:
    v = eb - ea
    v = v / np.hypot(v[:, 0], v[:, 1])[:, None]
    return np.stack([v[:, 1], -v[:, 0]], axis=1)         # right normal = outward for a CCW boundary


def dG_dn(x: np.ndarray, y: np.ndarray, ny: np.ndarray) -> np.ndarray:
    """dG/dn_y(x, y) = -(1/2pi) n_y.(y-x)/|y-x|^2 (Eq. fundsol), exact kernel."""
    d = y - x
    return -(ny * d).sum(-1) / (TWO_PI * (d * d).sum(-1))


def assemble_matrix(ea: np.ndarray, eb: np.ndarray) -> np.ndarray:
    """A_ij = delta_ij |Gamma_i|/2 + int_Gi int_Gj dG/dn_y, 3x3 Gauss; the coincident term is zero."""
    M = len(ea)
    pts, wts = gauss_points(ea, eb)
    nrm = element_normals(ea, eb)
    X = pts.reshape(-1, 2)
    Wx = wts.reshape(-1)
    A = np.zeros((M, M))
    rows = np.repeat(np.arange(M), 3)
    for blk in range(0, M, 64):
        j = np.arange(blk, min(M, blk + 64))
        Y = pts[j].reshape(-1, 2)
        Ny = np.repeat(nrm[j], 3, axis=0)
        Wy = wts[j].reshape(-1)
        with np.errstate(divide="ignore", invalid="ignore"):
            K = dG_dn(X[:, None, :], Y[None, :, :], Ny[None, :, :])
        cols = np.repeat(j, 3)
        same = rows[:, None] == cols[None, :]
        K = np.where(same, 0.0, K) * Wx[:, None] * Wy[None, :]
        A[:, j] = K.reshape(M, 3, len(j), 3).sum(axis=(1, 3))
    A[np.arange(M), np.arange(M)] += np.hypot(*(eb - ea).T) / 2.0
    return A


def truncated_pinv(A: np.ndarray) -> np.ndarray:
    """Pseudo-inverse discarding the smallest singular value (Sec. 3.1.3)."""
    U, s, Vt = np.linalg.svd(A)
    return (Vt[:-1].T / s[:-1]) @ U[:, :-1].T


@dataclass
class Boundary:
    ea: np.ndarray
    eb: np.ndarray
    gp: np.ndarray      # Gauss points [M,3,2]
    gw: np.ndarray      # Gauss weights [M,3]
    A: np.ndarray
    Apinv: np.ndarray

    @property
    def M(self) -> int:
        return len(self.ea)


def boundary_from_elements(ea: np.ndarray, eb: np.ndarray) -> Boundary:
    """Galerkin system and truncated pseudo-inverse of any set of straight elements a -> b
    (closed or open, possibly self-intersecting: the subdomain boundaries of Sec. 4.1)."""
    ea = np.ascontiguousarray(ea, dtype=np.float64)
    eb = np.ascontiguousarray(eb, dtype=np.float64)
    gp, gw = gauss_points(ea, eb)
    A = assemble_matrix(ea, eb)
    return Boundary(ea, eb, gp, gw, A, truncated_pinv(A))


@lru_cache(maxsize=8)
def boundary(per_side: int = 256) -> Boundary:
    return boundary_from_elements(*square_boundary(per_side))


def polygon_elements(verts, per_edge: int, closed: bool = True):
    """Elements of a polyline through verts [n, 2] (closed: back to the first vertex), each
    edge cut into per_edge equal elements, in vertex order."""
    v = np.asarray(verts, dtype=np.float64)
    if closed:
        v = np.concatenate([v, v[:1]])
    t = np.arange(per_edge + 1) / per_edge
    ea, eb = [], []
    for k in range(len(v) - 1):
        p = v[k][None, :] + t[:, None] * (v[k + 1] - v[k])[None, :]
        ea.append(p[:-1])
        eb.append(p[1:])
    return np.concatenate(ea), np.concatenate(eb)


def as_boundary(b) -> Boundary:
    """A Boundary, or the unit square with b elements per side."""
    return b if isinstance(b, Boundary) else boundary(b)


def element_weights(x: np.ndarray, bnd: Boundary) -> np.ndarray:
    """beta_j(x) = -int_Gj dG/dn_y dy for interior x: the double layer of unit density, eps = 0."""
    out = np.empty((len(x), bnd.M))
    for sl in _chunks(len(x), bnd.M):
        Md_a, Md_b, _, _ = segment_moments(x[sl], bnd.ea[:, 0], bnd.ea[:, 1], bnd.eb[:, 0], bnd.eb[:, 1], 0.0)
        out[sl] = Md_a + Md_b
    return out


def boundary_rhs(theta: np.ndarray, S: int, eps: float, bnd: Boundary) -> np.ndarray:
    """F_i = int_Gi f(x) dx by 3-point Gauss (right-hand side of Eq. bie_galerkin), [M,3]."""
    f = handle_term(bnd.gp.reshape(-1, 2), theta, S, eps).reshape(bnd.M, 3, 3)
    return (bnd.gw[:, :, None] * f).sum(axis=1)


def boundary_values(theta: np.ndarray, S: int, eps: float, bnd: Boundary) -> np.ndarray:
    return bnd.Apinv @ boundary_rhs(theta, S, eps, bnd)


def evaluate(theta, x, cbar, S: int, eps: float, per_side: int = 256) -> np.ndarray:
    """u(x) = cbar + sum_j beta_j(x) U_j + f(x) (Eq. bie, alpha = 1, plus the domain mean colour)."""
    bnd = as_boundary(per_side)
    U = boundary_values(theta, S, eps, bnd)
    x = np.asarray(x, dtype=np.float64)
    return np.asarray(cbar, dtype=np.float64)[None, :] + element_weights(x, bnd) @ U + handle_term(x, theta, S, eps)


# =============================================================================
# derivatives (differential BIE, Eq. diffbie)
# =============================================================================
def handle_term_jacobian(x: np.ndarray, theta: np.ndarray, S: int, eps: float) -> np.ndarray:
    """df_c/dtheta at x, [n, 3, P], P = 20H, columns in theta's row-major order."""
    H = theta.shape[0]
    seg = segment_table(theta, S)
    a, b = seg["a"], seg["b"]
    K = H * S
    ln = np.hypot(*(b - a).T)
    live = ln > DEGENERATE_LENGTH
    B = bernstein3(vertex_params(S))                     # [S+1, 4]
    tk = vertex_params(S)
    w = [seg[k] for k in ("wd_a", "wd_b", "wc_a", "wc_b")]
    n = len(x)
    J = np.zeros((n, 3, 20 * H))
    ax = du.seed(a[:, 0], 4, 0)
    ay = du.seed(a[:, 1], 4, 1)
    bx = du.seed(b[:, 0], 4, 2)
    by = du.seed(b[:, 1], 4, 3)
    for sl in _chunks(n, K):
        M = segment_moments(x[sl], ax, ay, bx, by, eps)
        Mv = [np.where(live[None, :], m.v, 0.0) for m in M]
        Md = [np.where(live[None, :, None], m.d, 0.0) for m in M]
        m_ = len(x[sl])
        # d f_c / d(a, b) per segment: [m, K, 4, 3]
        dfd = sum(Md[i][:, :, :, None] * w[i][None, :, None, :] for i in range(4))
        dfd = dfd.reshape(m_, H, S, 4, 3)
        gv = np.zeros((m_, H, S + 1, 2, 3))
        gv[:, :, :-1] += dfd[:, :, :, 0:2]
        gv[:, :, 1:] += dfd[:, :, :, 2:4]
        dP = np.einsum("kj,nhkdc->nhjdc", B, gv)                     # [m, H, 4, 2, 3]
        geo = dP.reshape(m_, H, 8, 3).transpose(0, 3, 1, 2)          # [m, 3, H, 8]
        # colour coefficients (channel independent)
        Mv = [m.reshape(m_, H, S) for m in Mv]
        ta = tk[None, None, :-1]
        tb = tk[None, None, 1:]
        e = np.stack([
            (Mv[0] * (1 - ta) + Mv[1] * (1 - tb)).sum(-1),
            (Mv[0] * ta + Mv[1] * tb).sum(-1),
            (Mv[2] * (1 - ta) + Mv[3] * (1 - tb)).sum(-1),
            (Mv[2] * ta + Mv[3] * tb).sum(-1),
        ], axis=-1)                                                  # [m, H, 4]
        Jc = J[sl].reshape(m_, 3, H, 20)
        Jc[:, :, :, :8] = geo
        for c in range(3):
            for mm in range(4):
                Jc[:, c, :, 8 + 3 * mm + c] = e[:, :, mm]
        J[sl] = Jc.reshape(m_, 3, 20 * H)
    return J


def boundary_rhs_jacobian(theta: np.ndarray, S: int, eps: float, bnd: Boundary) -> np.ndarray:
    """dF/dtheta [M, 3, P]."""
    Jf = handle_term_jacobian(bnd.gp.reshape(-1, 2), theta, S, eps).reshape(bnd.M, 3, 3, -1)
    return (bnd.gw[:, :, None, None] * Jf).sum(axis=1)


def boundary_derivative_values(theta, S, eps, bnd: Boundary) -> np.ndarray:
    """Z_c = A^+ dF_c/dtheta: the discretised differential BIE solved per column, [M, 3, P]."""
    dF = boundary_rhs_jacobian(theta, S, eps, bnd)
    return (bnd.Apinv @ dF.reshape(bnd.M, -1)).reshape(dF.shape)


def jacobian(theta, x, S: int, eps: float, per_side: int = 256) -> np.ndarray:
    """du_c/dtheta at x = df_c/dtheta + sum_j beta_j(x) Z_{j,c}, [n, 3, P]."""
    bnd = as_boundary(per_side)
    Z = boundary_derivative_values(theta, S, eps, bnd)
    x = np.asarray(x, dtype=np.float64)
    return handle_term_jacobian(x, theta, S, eps) + np.einsum("nj,jcp->ncp", element_weights(x, bnd), Z)


def vjp(theta, x, gbar, S: int, eps: float, per_side: int = 256, chunk: int = 2048) -> np.ndarray:
    """sum_x sum_c gbar_c(x) du_c/dtheta(x), [H, 20]."""
    bnd = as_boundary(per_side)
    Z = boundary_derivative_values(theta, S, eps, bnd)
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros(theta.size)
    for s in range(0, len(x), chunk):
        xs = x[s:s + chunk]
        Jf = handle_term_jacobian(xs, theta, S, eps)
        g += np.einsum("nc,ncp->p", gbar[s:s + chunk], Jf)
        psi = element_weights(xs, bnd).T @ gbar[s:s + chunk]        # [M, 3]
        g += np.einsum("jc,jcp->p", psi, Z)
    return g.reshape(theta.shape)


def normal_equations(theta, x, resid, S: int, eps: float, per_side: int = 256, chunk: int = 2048):
    """(1/N) sum_x J^T J and (1/N) sum_x J^T r with uniform density p = 1 (Eq. losshessian, Eq. lossjacobian)."""
    bnd = as_boundary(per_side)
    Z = boundary_derivative_values(theta, S, eps, bnd)
    x = np.asarray(x, dtype=np.float64)
    N = len(x)
    P = theta.size
    JtJ = np.zeros((P, P))
    Jtr = np.zeros(P)
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        J = handle_term_jacobian(xs, theta, S, eps) + np.einsum("nj,jcp->ncp", element_weights(xs, bnd), Z)
        Jr = J.reshape(-1, P)
        JtJ += Jr.T @ Jr
        Jtr += Jr.T @ resid[s:s + chunk].reshape(-1)
    return JtJ / N, Jtr / N


# =============================================================================
# Levenberg-Marquardt (Eq. optimstep, Sec. 4.3)
# =============================================================================
@dataclass
class LMState:
    lam: float = 1e-3
    cbar_sum: np.ndarray = None
    cbar_count: int = 0
    mean_rule: int = 0          # 0: running mean of all targets seen; 1: least-squares constant
    accepted: bool = False
    loss_before: float = np.nan
    loss_after: float = np.nan
    cbar: np.ndarray = None
    compat: bool = False        # enforce the compatibility condition (Sec. 4.3)
    chol_retries: int = 0       # damping raises after a failed Cholesky in the last step
    data_count: int = 0         # M_H, the samples drawn over the whole image (0: the step's own)

    def __post_init__(self):
        if self.cbar_sum is None:
            self.cbar_sum = np.zeros(3)
        if self.cbar is None:
            self.cbar = np.zeros(3)


LAMBDA_MIN, LAMBDA_MAX = 1e-12, 1e12


def loss(u: np.ndarray, T: np.ndarray) -> float:
    """Monte Carlo estimate of (1/2) int |u - T|^2 with uniform samples on the unit square."""
    r = u - T
    return 0.5 * float((r * r).sum()) / len(u)


def damped_step(JtJ: np.ndarray, Jtr: np.ndarray, lam: float) -> np.ndarray:
    """delta = (lam D + JtJ)^{-1} Jtr, D = diag(JtJ), by Cholesky."""
    from scipy.linalg import cho_factor, cho_solve
    d = np.diag(JtJ).copy()
    d = np.maximum(d, 1e-12 * max(d.max(), 1e-300))
    Hd = JtJ + lam * np.diag(d)
    return cho_solve(cho_factor(Hd, lower=True), Jtr)


# =============================================================================
# Compatibility condition (Sec. 3.1.2: zero net flux of the normal-derivative
# jump over the handles) and its enforcement in the LM step (Sec. 4.3)
# =============================================================================
def compat_vectors(theta, S: int) -> np.ndarray:
    """Columns a_c (c = RGB) of A [P, 3] with a_c . theta = int over the handles of w_c.

    On a straight segment the jump w_c is linear between its end values, so its
    integral is L (w_c(a) + w_c(b)) / 2; with w_c(t) = (1 - t) wc0 + t wc1 at the
    vertex parameters t_k this sums, per handle, to alpha_h wc0 + beta_h wc1 with
      alpha_h = sum_k L_hk (2 - t_k - t_{k+1}) / 2,   beta_h = sum_k L_hk (t_k + t_{k+1}) / 2.
    Segments not longer than DEGENERATE_LENGTH carry no jump (as in the handle term)."""
    theta = np.asarray(theta, dtype=np.float64)
    H = theta.shape[0]
    p = handle_vertices(theta, S)
    L = np.sqrt(((p[:, 1:] - p[:, :-1]) ** 2).sum(-1))                   # [H, S]
    L = np.where(L > DEGENERATE_LENGTH, L, 0.0)
    t = vertex_params(S)
    alpha = (L * (2.0 - t[:-1] - t[1:]) / 2.0).sum(1)
    beta = (L * (t[:-1] + t[1:]) / 2.0).sum(1)
    A = np.zeros((H, 20, 3))
    for c in range(3):
        A[:, 14 + c, c] = alpha
        A[:, 17 + c, c] = beta
    return A.reshape(H * 20, 3)


def constrained_step(JtJ: np.ndarray, Jtr: np.ndarray, lam: float, A: np.ndarray) -> np.ndarray:
    """The damped step of damped_step restricted to A^T delta = 0 (the projection of the
    approximate Hessian and of the gradient onto the feasible directions for fixed end points):
    the minimiser of delta^T Hd delta / 2 - delta^T Jtr over that subspace, from the KKT system
      [Hd A; A^T 0] [delta; nu] = [Jtr; 0]  ->  delta = Hd^{-1} (Jtr - A nu),
      (A^T Hd^{-1} A) nu = A^T Hd^{-1} Jtr."""
    from scipy.linalg import cho_factor, cho_solve
    d = np.diag(JtJ).copy()
    d = np.maximum(d, 1e-12 * max(d.max(), 1e-300))
    cf = cho_factor(JtJ + lam * np.diag(d), lower=True)
    keep = np.abs(A).sum(0) > 0                     # a channel without handles has no constraint
    A = A[:, keep]
    d0 = cho_solve(cf, Jtr)
    if A.shape[1] == 0:
        return d0
    X = cho_solve(cf, A)
    nu = np.linalg.solve(A.T @ X, A.T @ d0)
    return d0 - X @ nu


def project_compatible(theta, A: np.ndarray) -> np.ndarray:
    """theta minus, per channel c, its component along a_c: the orthogonal projection onto
    a_c . theta = 0 for the given vectors A [P, 3] (their supports are disjoint)."""
    theta = np.asarray(theta, dtype=np.float64).copy()
    flat = theta.reshape(-1)
    for c in range(3):
        a = A[:, c]
        aa = float(a @ a)
        if aa > 0:
            flat -= a * (float(a @ flat) / aa)
    return flat.reshape(theta.shape)


def reproject(theta, S: int) -> np.ndarray:
    """Orthogonal projection of the wc parameters onto a_c(theta) . theta = 0, with a_c taken at
    theta's own end points (the re-projection after each update, Sec. 4.3)."""
    return project_compatible(theta, compat_vectors(theta, S))


@dataclass(frozen=True)
class HandleModel:
    """The operations of one handle parametrisation that an LM step uses."""
    evaluate: object
    normal_equations: object
    compat_vectors: object
    reproject: object


CUBIC = HandleModel(evaluate=evaluate, normal_equations=normal_equations, compat_vectors=compat_vectors,
                    reproject=reproject)


def lm_step(theta, x, T, state: LMState, S: int, eps: float, per_side: int = 256, model: HandleModel = CUBIC,
            reg: rg.Reg | None = None):
    """One damped Gauss-Newton step with accept/reject on the same samples.  Returns (theta', state).
    With regularisation terms (Sec. 4.4) their Hessian and gradient are added to the normal
    equations and their value to the loss on both sides of the accept test."""
    evaluate, normal_equations = model.evaluate, model.normal_equations
    compat_vectors, reproject = model.compat_vectors, model.reproject
    theta = np.asarray(theta, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    state.cbar_sum = state.cbar_sum + T.sum(axis=0)
    state.cbar_count += len(T)
    u0 = evaluate(theta, x, np.zeros(3), S, eps, per_side)           # zero-mean reconstruction
    if state.mean_rule == 0:
        cbar = state.cbar_sum / state.cbar_count
    else:
        cbar = (T - u0).mean(axis=0)
    state.cbar = cbar
    u = u0 + cbar[None, :]
    # the data terms are Monte Carlo estimates over the M_H samples drawn for the whole image
    # (Eq. losshessian, Eq. lossjacobian): a subdomain's step sums its own samples and divides by
    # M_H, so its data terms keep their weight against the regularisers (Sec. 4.4)
    if state.data_count and state.data_count < len(T):
        raise ValueError("data_count must be 0 or at least the number of samples")
    wdat = len(T) / state.data_count if state.data_count else 1.0
    L0 = wdat * loss(u, T)
    JtJ, Jtr = normal_equations(theta, x, u - T, S, eps, per_side)
    JtJ, Jtr = wdat * JtJ, wdat * Jtr
    pairs = None
    if reg is not None and reg.active():
        R0, gR, HR, pairs = rg.terms(theta, reg)
        JtJ, Jtr, L0 = JtJ + HR, Jtr + gR, L0 + R0
    from scipy.linalg import LinAlgError
    state.chol_retries = 0
    while True:                     # a failed Cholesky raises the damping (at most 10 times)
        try:
            if state.compat:
                delta = constrained_step(JtJ, Jtr, state.lam, compat_vectors(theta, S))
            else:
                delta = damped_step(JtJ, Jtr, state.lam)
            break
        except LinAlgError:
            if state.chol_retries >= 10:
                raise
            state.lam = min(state.lam * 10.0, LAMBDA_MAX)
            state.chol_retries += 1
    theta_new = theta - delta.reshape(theta.shape)
    if state.compat:
        theta_new = reproject(theta_new, S)
    L1 = wdat * loss(evaluate(theta_new, x, cbar, S, eps, per_side), T)
    if pairs is not None:
        L1 += rg.value(theta_new, reg, pairs)
    state.loss_before, state.loss_after = L0, L1
    if L1 < L0:
        state.accepted = True
        state.lam = max(state.lam / 10.0, LAMBDA_MIN)
        return theta_new, state
    state.accepted = False
    state.lam = min(state.lam * 10.0, LAMBDA_MAX)
    return theta.copy(), state
