"""Truncated multivariate Taylor numbers ("jets") for barrier derivatives.

TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Nothing in the product
path may import this package.

A jet carries the coefficients of a function's expansion in up to three
nilpotent infinitesimals e1, e2, e3 (e_i^2 = 0), one coefficient per subset
of {1, 2, 3} (bitmask index 0..7).  Evaluating a barrier f at
z + e1 u + e2 v + e3 w yields, in the coefficient of e1 e2 e3, the third
directional derivative f'''(z)[u, v, w]; lower subsets give the lower
derivatives.  This is how the oracle obtains grad f, Hess f and the
third-order contraction used by the exp/pow corrector (higher-order
correction of the combined step, Sec. 2.2) without hand-derived formulas.
Every coefficient is a numpy array, so one jet evaluates a whole family of
cones at once.
"""
from __future__ import annotations

import math

import numpy as np

_SUBSETS = list(range(8))


class Jet:
    __slots__ = ("c",)

    def __init__(self, c):
        self.c = c  # list of 8 arrays (or scalars)

    @staticmethod
    def const(a):
        a = np.asarray(a, dtype=np.float64)
        return Jet([a] + [np.zeros_like(a) for _ in range(7)])

    @staticmethod
    def seed(a, dirs):
        """a + sum_i e_i * dirs[i] (dirs: dict bit -> array)."""
        a = np.asarray(a, dtype=np.float64)
        c = [a] + [np.zeros_like(a) for _ in range(7)]
        for bit, d in dirs.items():
            c[bit] = c[bit] + np.asarray(d, dtype=np.float64)
        return Jet(c)

    # -- arithmetic --------------------------------------------------------
    def __add__(self, o):
        if not isinstance(o, Jet):
            c = list(self.c)
            c[0] = c[0] + o
            return Jet(c)
        return Jet([a + b for a, b in zip(self.c, o.c)])

    __radd__ = __add__

    def __neg__(self):
        return Jet([-a for a in self.c])

    def __sub__(self, o):
        return self + (-o if isinstance(o, Jet) else -o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if not isinstance(o, Jet):
            return Jet([a * o for a in self.c])
        out = []
        for S in _SUBSETS:
            acc = 0.0
            T = S
            # enumerate all subsets T of S
            while True:
                acc = acc + self.c[T] * o.c[S & ~T]
                if T == 0:
                    break
                T = (T - 1) & S
            out.append(acc)
        return Jet(out)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if not isinstance(o, Jet):
            return Jet([a / o for a in self.c])
        return self * o.apply_fn(lambda a: [1.0 / a, -1.0 / a**2, 2.0 / a**3, -6.0 / a**4])

    def __rtruediv__(self, o):
        return Jet.const(np.broadcast_to(o, self.c[0].shape).astype(np.float64)) / self

    # -- scalar functions via their Taylor series --------------------------
    def apply_fn(self, derivs):
        """g(self) given derivs(a) = [g(a), g'(a), g''(a), g'''(a)]."""
        a = self.c[0]
        g = derivs(a)
        delta = Jet([np.zeros_like(a)] + list(self.c[1:]))
        out = Jet.const(g[0] * np.ones_like(a))
        power = Jet.const(np.ones_like(a))
        for k in range(1, 4):
            power = power * delta
            out = out + power * (g[k] / math.factorial(k))
        return out

    def log(self):
        return self.apply_fn(lambda a: [np.log(a), 1.0 / a, -1.0 / a**2, 2.0 / a**3])

    def exp(self):
        return self.apply_fn(lambda a: [np.exp(a)] * 4)

    def powc(self, p):
        """self ** p for a constant exponent p (array or scalar), self > 0."""
        return self.apply_fn(lambda a: [a**p, p * a**(p - 1), p * (p - 1) * a**(p - 2),
                                        p * (p - 1) * (p - 2) * a**(p - 3)])


def derivatives(f, z, params=None):
    """grad f(z) and Hess f(z) for a family of 3-d cones.

    z: (N, 3).  f(zj, params) takes a list of 3 jets and returns a jet.
    Returns (g (N,3), H (N,3,3)).
    """
    N = z.shape[0]
    g = np.zeros((N, 3))
    H = np.zeros((N, 3, 3))
    for j in range(3):
        for k in range(j, 3):
            zj = []
            for i in range(3):
                d = {}
                if i == j:
                    d[1] = 1.0
                if i == k:
                    d[2] = d.get(2, 0.0) + 1.0
                zj.append(Jet.seed(z[:, i], d))
            val = f(zj, params)
            H[:, j, k] = val.c[3]
            H[:, k, j] = val.c[3]
            if j == k:
                g[:, j] = val.c[1]
    return g, H


def third(f, z, u, v, params=None):
    """The vector T with T_k = f'''(z)[u, v, e_k] for a family of 3-d cones."""
    N = z.shape[0]
    out = np.zeros((N, 3))
    for k in range(3):
        zj = []
        for i in range(3):
            d = {1: u[:, i], 2: v[:, i]}
            if i == k:
                d[4] = 1.0
            zj.append(Jet.seed(z[:, i], d))
        out[:, k] = f(zj, params).c[7]
    return out


def value(f, z, params=None):
    return f([Jet.const(z[:, i]) for i in range(3)], params).c[0]
