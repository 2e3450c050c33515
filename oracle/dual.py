"""Forward-mode dual numbers over numpy arrays (test infrastructure only).

A Dual carries a value array `v` and a derivative array `d` of shape
v.shape + (m,), one slot per seeded input.  Only the operations the oracle's
closed forms use are defined.  Numpy broadcasting applies to both parts.
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    # -- helpers -------------------------------------------------------------
    @staticmethod
    def _parts(x):
        if isinstance(x, Dual):
            return x.v, x.d
        return np.asarray(x, dtype=np.float64), None

    @staticmethod
    def _combine(v, terms):
        d = None
        for dv, coef in terms:
            if dv is None:
                continue
            t = dv * np.asarray(coef)[..., None]
            d = t if d is None else d + t
        if d is None:
            return v
        d = np.broadcast_to(d, np.shape(v) + (d.shape[-1],))
        return Dual(v, d)

    # -- arithmetic ----------------------------------------------------------
    def __add__(self, o):
        ov, od = self._parts(o)
        return self._combine(self.v + ov, [(self.d, 1.0), (od, 1.0)])

    __radd__ = __add__

    def __sub__(self, o):
        ov, od = self._parts(o)
        return self._combine(self.v - ov, [(self.d, 1.0), (od, -1.0)])

    def __rsub__(self, o):
        ov, od = self._parts(o)
        return self._combine(ov - self.v, [(self.d, -1.0), (od, 1.0)])

    def __mul__(self, o):
        ov, od = self._parts(o)
        return self._combine(self.v * ov, [(self.d, ov), (od, self.v)])

    __rmul__ = __mul__

    def __truediv__(self, o):
        ov, od = self._parts(o)
        r = self.v / ov
        return self._combine(r, [(self.d, 1.0 / ov), (od, -r / ov)])

    def __rtruediv__(self, o):
        ov, od = self._parts(o)
        r = ov / self.v
        return self._combine(r, [(self.d, -r / self.v), (od, 1.0 / self.v)])

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __getitem__(self, idx):
        return Dual(self.v[idx], self.d[idx])


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x, dtype=np.float64)


def deriv(x, shape_m):
    """Derivative array of x (zeros if x is a plain array)."""
    if isinstance(x, Dual):
        return x.d
    v = np.asarray(x, dtype=np.float64)
    return np.zeros(v.shape + (shape_m,))


def sqrt(x):
    xv, xd = Dual._parts(x)
    r = np.sqrt(xv)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(r > 0, 0.5 / np.where(r > 0, r, 1.0), 0.0)
    return Dual._combine(r, [(xd, c)])


def log(x):
    xv, xd = Dual._parts(x)
    return Dual._combine(np.log(xv), [(xd, 1.0 / xv)])


def log1p(x):
    xv, xd = Dual._parts(x)
    return Dual._combine(np.log1p(xv), [(xd, 1.0 / (1.0 + xv))])


def arctan2(y, x):
    yv, yd = Dual._parts(y)
    xv, xd = Dual._parts(x)
    den = xv * xv + yv * yv
    with np.errstate(divide="ignore", invalid="ignore"):
        cy = np.where(den > 0, xv / np.where(den > 0, den, 1.0), 0.0)
        cx = np.where(den > 0, -yv / np.where(den > 0, den, 1.0), 0.0)
    return Dual._combine(np.arctan2(yv, xv), [(yd, cy), (xd, cx)])


def where(cond, a, b):
    av, ad = Dual._parts(a)
    bv, bd = Dual._parts(b)
    v = np.where(cond, av, bv)
    if ad is None and bd is None:
        return v
    m = (ad if ad is not None else bd).shape[-1]
    shape = np.shape(v) + (m,)
    ad = np.zeros(shape) if ad is None else np.broadcast_to(ad, shape)
    bd = np.zeros(shape) if bd is None else np.broadcast_to(bd, shape)
    return Dual(v, np.where(np.asarray(cond)[..., None], ad, bd))


def seed(values, m: int, slot: int):
    """Dual with unit derivative in one slot."""
    v = np.asarray(values, dtype=np.float64)
    d = np.zeros(v.shape + (m,))
    d[..., slot] = 1.0
    return Dual(v, d)
