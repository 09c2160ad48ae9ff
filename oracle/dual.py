"""Forward-mode dual numbers over numpy arrays (oracle derivative machinery).

A ``Dual`` carries a value array ``v`` of shape (...) and a derivative array
``d`` of shape (..., K): K directional derivatives propagated by the chain
rule.  Only the operations the projection function needs are provided.
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    @staticmethod
    def variable(v, index, k):
        """Seed: value v with unit derivative in direction ``index`` of k."""
        v = np.asarray(v, dtype=np.float64)
        d = np.zeros(v.shape + (k,))
        d[..., index] = 1.0
        return Dual(v, d)

    @staticmethod
    def const(v, k):
        v = np.asarray(v, dtype=np.float64)
        return Dual(v, np.zeros(v.shape + (k,)))

    # arithmetic -------------------------------------------------------------
    def _lift(self, o):
        if isinstance(o, Dual):
            return o
        o = np.asarray(o, dtype=np.float64)
        return Dual(o, np.zeros(o.shape + (self.d.shape[-1],)))

    def __add__(self, o):
        o = self._lift(o)
        return Dual(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __sub__(self, o):
        o = self._lift(o)
        return Dual(self.v - o.v, self.d - o.d)

    def __rsub__(self, o):
        return self._lift(o) - self

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        o = self._lift(o)
        return Dual(self.v * o.v, self.d * o.v[..., None] + o.d * self.v[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = self._lift(o)
        inv = 1.0 / o.v
        return Dual(self.v * inv,
                    (self.d - o.d * (self.v * inv)[..., None]) * inv[..., None])

    def __rtruediv__(self, o):
        return self._lift(o) / self


def sin(x):
    if isinstance(x, Dual):
        return Dual(np.sin(x.v), x.d * np.cos(x.v)[..., None])
    return np.sin(x)


def cos(x):
    if isinstance(x, Dual):
        return Dual(np.cos(x.v), -x.d * np.sin(x.v)[..., None])
    return np.cos(x)


def sqrt(x):
    if isinstance(x, Dual):
        s = np.sqrt(x.v)
        return Dual(s, x.d * (0.5 / s)[..., None])
    return np.sqrt(x)


def real(x):
    """Real part of a value (dual, complex or real) used only for branching."""
    if isinstance(x, Dual):
        return x.v
    return np.real(x)


def where(mask, a, b):
    """Elementwise select for duals or plain arrays."""
    if isinstance(a, Dual) or isinstance(b, Dual):
        k = a.d.shape[-1] if isinstance(a, Dual) else b.d.shape[-1]
        a = a if isinstance(a, Dual) else Dual.const(np.broadcast_to(a, mask.shape), k)
        b = b if isinstance(b, Dual) else Dual.const(np.broadcast_to(b, mask.shape), k)
        return Dual(np.where(mask, a.v, b.v), np.where(mask[..., None], a.d, b.d))
    return np.where(mask, a, b)
