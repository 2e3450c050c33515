"""Seeded synthetic workloads for the differential-BEM hot path.

This module only draws random numbers and arranges them into the arrays the
method consumes: cubic Bezier control points, jump colours, sample positions
and unit Gaussian noise.  It holds none of the method's arithmetic (no
segment integrals, no boundary system, no Jacobians); both the CPU oracle and
the HIP library consume its arrays.

Curves are sampled here in two places, and only to decide *where random draws
go*: rejecting draws whose handles cross (tiny workload), tuning the spread of
crossing handles, and placing stress samples next to a handle.  Nothing the
curve sampling produces is handed to either implementation except sample
positions, which are inputs.

Parameter layout per handle (20 float64, the column order of every Jacobian):
  [P0x P0y P1x P1y P2x P2y P3x P3y | wd0 RGB | wd1 RGB | wc0 RGB | wc1 RGB]
wd = colour jump (left minus right side of the travel direction), wc = jump
of the normal derivative, each given at both ends of the handle and linear in
the curve parameter t (paper Sec. 3.1.1, jump formulation of the handle term).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

# independent random streams of one workload
GEOM, COLOUR, PERTURB, SAMPLES, NOISE, GRID = range(6)

BOX_LO, BOX_HI = 0.15, 0.85       # control points live in this sub-square of the unit domain
EPS_PAPER = 1e-2                  # kernel regularisation used in all of the paper's experiments (Sec. 4, smoothing study)
ELEMS_PER_SIDE = 256              # outer-boundary elements per side: length 1/256 of the width (Sec. 3.1.3)


@dataclass(frozen=True)
class ConfigSpec:
    index: int
    H: int              # handles
    S: int              # straight segments per handle
    N: int              # samples per step
    sigma: float        # target noise per channel
    crossing: bool      # handles may cross (spread tuned to ~20% crossing pairs)
    near_frac: float    # fraction of samples placed within 1e-3 of a handle segment
    lm_iters: int
    name: str
    model: str = "cubic"              # "cubic": 20 parameters per handle; "straight": 10 (Sec. 4.1)
    target_max: float | None = None   # targets clamped to at most this value (Sec. 4.3)

    @property
    def params_per_handle(self) -> int:
        return 20 if self.model == "cubic" else 10


SPECS = {
    1: ConfigSpec(1, 4, 32, 16_384, 0.1, False, 0.0, 1, "tiny FP64: 4 disjoint handles x 32 segments, 16,384 samples"),
    2: ConfigSpec(2, 32, 16, 262_144, 0.2, True, 0.0, 20, "medium FP64: 32 crossing handles x 16 segments, 262,144 samples"),
    3: ConfigSpec(3, 128, 32, 1_048_576, 0.0, True, 0.1, 0, "mixed forward: 128 handles x 32 segments, 1,048,576 samples, 10% near a segment"),
    4: ConfigSpec(4, 256, 32, 4_194_304, 0.3, True, 0.0, 0, "differentiation: 256 handles x 32 segments, 4,194,304 samples"),
    5: ConfigSpec(5, 256, 32, 2_097_152, 0.2, True, 0.0, 50, "LM normal equations: 256 handles x 32 segments, 2,097,152 samples, P=5,120"),
    # the paper's own setting: 500 straight handles placed by a Sobol sequence at 1/20 of the
    # width (Sec. 4.2), 100,000 uniform samples per step, targets clamped at 1 (Sec. 4.3)
    6: ConfigSpec(6, 500, 1, 100_000, 0.1, True, 0.0, 100,
                  "paper-native: 500 straight handles (Sobol placement, length 1/20), 100,000 samples, P=5,000",
                  model="straight", target_max=1.0),
}
PAPER_CONFIG = 6
SOBOL_LENGTH = 1.0 / 20.0         # initial handle length: 1/20 of the image width (Sec. 4.2)


def rng_for(config: int, stream: int, step: int = 0) -> np.random.Generator:
    """Independent generator for (config, stream, step); config i is seeded with i-1."""
    return np.random.default_rng(np.random.SeedSequence(entropy=config - 1, spawn_key=(stream, step)))


# ----------------------------------------------------------------------------
# generator-side curve sampling (placement and rejection only)
# ----------------------------------------------------------------------------
def _curve_points(ctrl: np.ndarray, m: int) -> np.ndarray:
    """Points of cubic Bezier curves at t = k/m, k = 0..m.  ctrl [..., 4, 2] -> [..., m+1, 2]."""
    t = np.linspace(0.0, 1.0, m + 1)
    s = 1.0 - t
    w = np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], axis=-1)      # [m+1, 4]
    return np.einsum("kj,...jc->...kc", w, ctrl)


def _polylines_cross(pa: np.ndarray, pb: np.ndarray) -> bool:
    """True if polyline pa [m+1,2] and polyline pb [n+1,2] properly intersect."""
    a0, a1 = pa[:-1, None, :], pa[1:, None, :]
    b0, b1 = pb[None, :-1, :], pb[None, 1:, :]

    def orient(p, q, r):
        return (q[..., 0] - p[..., 0]) * (r[..., 1] - p[..., 1]) - (q[..., 1] - p[..., 1]) * (r[..., 0] - p[..., 0])

    d1 = orient(b0, b1, a0)
    d2 = orient(b0, b1, a1)
    d3 = orient(a0, a1, b0)
    d4 = orient(a0, a1, b1)
    return bool(np.any((d1 * d2 < 0) & (d3 * d4 < 0)))


def crossing_fraction(ctrl: np.ndarray, S: int) -> float:
    """Fraction of handle pairs whose S-segment polylines cross."""
    pts = _curve_points(ctrl, S)
    H = ctrl.shape[0]
    n = 0
    tot = 0
    for i in range(H):
        for j in range(i + 1, H):
            tot += 1
            n += _polylines_cross(pts[i], pts[j])
    return n / max(tot, 1)


# ----------------------------------------------------------------------------
# geometry draws
# ----------------------------------------------------------------------------
def _disjoint_handles(rng: np.random.Generator, H: int, S: int) -> np.ndarray:
    """Control points uniform in the box, redrawn until no two handle polylines cross."""
    for _ in range(100_000):
        ctrl = rng.uniform(BOX_LO, BOX_HI, size=(H, 4, 2))
        pts = _curve_points(ctrl, S)
        if not any(_polylines_cross(pts[i], pts[j]) for i in range(H) for j in range(i + 1, H)):
            return ctrl
    raise RuntimeError("could not draw non-crossing handles")


def _spread_handles(rng: np.random.Generator, H: int, spread: float) -> np.ndarray:
    centre = rng.uniform(BOX_LO, BOX_HI, size=(H, 1, 2))
    offs = rng.uniform(-1.0, 1.0, size=(H, 4, 2))
    return np.clip(centre + spread * offs, BOX_LO, BOX_HI)


@lru_cache(maxsize=None)
def medium_spread(target: float = 0.20) -> float:
    """Spread s of the medium workload tuned by bisection so ~20% of handle pairs cross."""
    spec = SPECS[2]
    lo, hi = 0.005, 1.0
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        ctrl = _spread_handles(rng_for(2, GEOM), spec.H, mid)
        if crossing_fraction(ctrl, spec.S) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def draw_geometry(config: int) -> np.ndarray:
    spec = SPECS[config]
    rng = rng_for(config, GEOM)
    if not spec.crossing:
        return _disjoint_handles(rng, spec.H, spec.S)
    spread = medium_spread() * np.sqrt(SPECS[2].H / spec.H)
    return _spread_handles(rng, spec.H, spread)


def draw_colours(rng: np.random.Generator, H: int) -> np.ndarray:
    """Jump parameters [H,12] from left/right end colours uniform in [0,1].

    wd = cL - cR (the colour jump, Sec. 3.1.1).  wc = cL + cR - 1: the derivative
    jump has no counterpart in a left/right colour description, so this zero-mean
    map is a chosen reading that exercises the single layer.
    """
    c = rng.uniform(0.0, 1.0, size=(H, 2, 2, 3))      # [handle, end, side(L,R), rgb]
    wd = c[:, :, 0, :] - c[:, :, 1, :]
    wc = c[:, :, 0, :] + c[:, :, 1, :] - 1.0
    return np.concatenate([wd[:, 0], wd[:, 1], wc[:, 0], wc[:, 1]], axis=1)


def sobol_handles(n: int, seed: int, length: float = SOBOL_LENGTH) -> np.ndarray:
    """End points [n, 4] = (A, B) of straight handles placed as in Sec. 4.2.

    A comes from a scrambled Sobol sequence in the unit square (scipy's generator, direction
    numbers of Joe and Kuo); B lies at distance `length` from A in the direction of a third
    Sobol coordinate; B is then snapped into the domain (the unit square, the one subdomain
    here) by clamping, which shortens handles that would leave it.
    """
    from scipy.stats import qmc
    m = max(1, int(np.ceil(np.log2(max(n, 1)))))
    u = qmc.Sobol(d=3, scramble=True, seed=np.random.default_rng(np.random.SeedSequence(entropy=seed))).random_base2(m)[:n]
    a = u[:, :2]
    ang = 2.0 * np.pi * u[:, 2]
    b = np.clip(a + length * np.stack([np.cos(ang), np.sin(ang)], axis=1), 0.0, 1.0)
    return np.concatenate([a, b], axis=1)


def draw_straight_colours(rng: np.random.Generator, H: int) -> np.ndarray:
    """Constant jumps [H, 6] = (wd RGB, wc RGB) from left/right colours uniform in [0,1], with
    the same map as draw_colours (wd = cL - cR, wc = cL + cR - 1)."""
    c = rng.uniform(0.0, 1.0, size=(H, 2, 3))
    return np.concatenate([c[:, 0] - c[:, 1], c[:, 0] + c[:, 1] - 1.0], axis=1)


def pack_theta(ctrl: np.ndarray, colours: np.ndarray) -> np.ndarray:
    H = ctrl.shape[0]
    return np.ascontiguousarray(np.concatenate([ctrl.reshape(H, 8), colours], axis=1), dtype=np.float64)


# ----------------------------------------------------------------------------
# samples and noise
# ----------------------------------------------------------------------------
def uniform_samples(rng: np.random.Generator, n: int) -> np.ndarray:
    """n points uniform in the open unit square (exact boundary values redrawn)."""
    x = rng.random((n, 2))
    bad = (x <= 0.0)
    while bad.any():
        x[bad] = rng.random(int(bad.sum()))
        bad = (x <= 0.0)
    return x


def near_samples(rng: np.random.Generator, ctrl: np.ndarray, S: int, n: int, band: float = 1e-3) -> np.ndarray:
    """n points at signed distance delta, |delta| in [1e-9, band], from random handle segments."""
    pts = _curve_points(ctrl, S)                         # [H, S+1, 2]
    a = pts[:, :-1].reshape(-1, 2)
    b = pts[:, 1:].reshape(-1, 2)
    k = rng.integers(0, a.shape[0], size=n)
    s = rng.random(n)
    delta = rng.uniform(-band, band, size=n)
    small = np.abs(delta) < 1e-9
    delta[small] = np.where(delta[small] < 0, -1e-9, 1e-9)
    v = b[k] - a[k]
    ln = np.linalg.norm(v, axis=1, keepdims=True)
    ln[ln == 0] = 1.0
    nrm = np.stack([v[:, 1], -v[:, 0]], axis=1) / ln
    return a[k] + s[:, None] * v + delta[:, None] * nrm


@dataclass
class Workload:
    spec: ConfigSpec
    theta_true: np.ndarray
    theta0: np.ndarray
    eps: float = EPS_PAPER
    elems_per_side: int = ELEMS_PER_SIDE
    lam0: float = 1e-3
    cbar_true: np.ndarray = field(default_factory=lambda: np.full(3, 0.5))

    @property
    def H(self) -> int:
        return self.spec.H

    @property
    def S(self) -> int:
        return self.spec.S

    @property
    def N(self) -> int:
        return self.spec.N

    @property
    def P(self) -> int:
        return self.spec.params_per_handle * self.spec.H

    def target(self, u_true: np.ndarray, step: int = 0, idx=None) -> np.ndarray:
        """Noisy target from the noise-free reconstruction at the step's samples (rows idx of
        them if given): u_true + sigma * noise, clamped at target_max when the workload sets it."""
        nz = self.noise(step)
        T = u_true + self.spec.sigma * (nz if idx is None else nz[idx])
        return np.minimum(T, self.spec.target_max) if self.spec.target_max is not None else T

    def samples(self, step: int = 0, n: int | None = None) -> np.ndarray:
        n = self.spec.N if n is None else n
        rng = rng_for(self.spec.index, SAMPLES, step)
        n_near = int(round(self.spec.near_frac * n))
        x = uniform_samples(rng, n - n_near)
        if n_near:
            xn = near_samples(rng, self.theta_true[:, :8].reshape(-1, 4, 2), self.spec.S, n_near)
            x = np.concatenate([x, xn], axis=0)
        return np.ascontiguousarray(x)

    def noise(self, step: int = 0, n: int | None = None) -> np.ndarray:
        n = self.spec.N if n is None else n
        return rng_for(self.spec.index, NOISE, step).standard_normal((n, 3))

    def subsample(self, n: int, n_total: int | None = None, step: int = 0) -> np.ndarray:
        """Sorted indices of n distinct samples out of n_total (default N)."""
        n_total = self.spec.N if n_total is None else n_total
        rng = rng_for(self.spec.index, GRID, 1000 + step)
        return np.sort(rng.choice(n_total, size=n, replace=False))


def pixel_grid(res: int = 512) -> np.ndarray:
    c = (np.arange(res) + 0.5) / res
    gx, gy = np.meshgrid(c, c, indexing="xy")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)


@lru_cache(maxsize=None)
def make_config(config: int) -> Workload:
    spec = SPECS[config]
    if spec.model == "straight":
        # ground truth: Sobol-placed handles with random constant jumps; start: another Sobol
        # placement (the initialisation of Sec. 4.2) with small random jumps
        ends = sobol_handles(spec.H, seed=100 * config + GEOM)
        theta_true = np.ascontiguousarray(
            np.concatenate([ends, draw_straight_colours(rng_for(config, COLOUR), spec.H)], axis=1))
        ends0 = sobol_handles(spec.H, seed=100 * config + PERTURB)
        jumps0 = 0.05 * rng_for(config, PERTURB).standard_normal((spec.H, 6))
        theta0 = np.ascontiguousarray(np.concatenate([ends0, jumps0], axis=1))
        return Workload(spec=spec, theta_true=theta_true, theta0=theta0)
    ctrl = draw_geometry(config)
    theta_true = pack_theta(ctrl, draw_colours(rng_for(config, COLOUR), spec.H))
    rng = rng_for(config, PERTURB)
    theta0 = theta_true.copy()
    theta0[:, :8] = np.clip(theta0[:, :8] + rng.normal(0.0, 0.01, size=(spec.H, 8)), BOX_LO, BOX_HI)
    theta0[:, 8:] = theta0[:, 8:] + rng.normal(0.0, 0.1, size=(spec.H, 12))
    return Workload(spec=spec, theta_true=theta_true, theta0=theta0)


def random_handles(seed: int, H: int, spread: float = 0.15, centre_lo: float = 0.25, centre_hi: float = 0.75) -> np.ndarray:
    """Small ad-hoc handle sets for tests: theta [H,20]."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy=1000 + seed))
    centre = rng.uniform(centre_lo, centre_hi, size=(H, 1, 2))
    ctrl = np.clip(centre + spread * rng.uniform(-1, 1, size=(H, 4, 2)), 0.05, 0.95)
    return pack_theta(ctrl, draw_colours(rng, H))


def random_points(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(entropy=2000 + seed))
    x = rng.uniform(lo, hi, size=(n, 2))
    x[x <= 0.0] = 1e-6
    return x


def random_vector(seed: int, shape) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(entropy=3000 + seed))
    return rng.standard_normal(shape)
