"""Forward-mode dual numbers over numpy arrays (oracle; test infrastructure).

The paper builds its Rosenbrock and SDC systems with the exact Jacobian of F
(section 3.3.2, text after equation rb_system).  The oracle obtains that
Jacobian by forward-mode automatic differentiation: every model quantity is a
Dual carrying its value ``v`` (shape (N,), one entry per vertex) and its
gradient ``d`` with respect to the n state variables (shape (n, N)).  Each
operation below applies the textbook derivative rule, so the Jacobian is exact
up to rounding and needs no hand-derived entries.

Model code is written once against the functions ``exp``, ``log``, ``sqrt``,
``expm1``, ``where`` and ``val`` of this module; called with plain float
arrays they return plain arrays, called with Duals they return Duals.
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000.0
    __array_ufunc__ = None  # numpy defers mixed ops to the reflected Dual methods

    def __init__(self, v, d):
        self.v = v
        self.d = d

    # ---- arithmetic -----------------------------------------------------
    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.d + o.d)
        return Dual(self.v + o, self.d)

    __radd__ = __add__

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v - o.v, self.d - o.d)
        return Dual(self.v - o, self.d)

    def __rsub__(self, o):
        return Dual(o - self.v, -self.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.d * o.v + o.d * self.v)
        return Dual(self.v * o, self.d * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            q = self.v / o.v
            return Dual(q, (self.d - o.d * q) / o.v)
        return Dual(self.v / o, self.d / o)

    def __rtruediv__(self, o):
        # o / self, o a constant
        q = o / self.v
        return Dual(q, -self.d * (q / self.v))

    def __pow__(self, p):
        # real constant exponent only
        if isinstance(p, Dual):
            raise TypeError("Dual ** Dual is not used by the models")
        if p == 2:
            return self * self
        if p == 3:
            return self * self * self
        vp = self.v ** p
        return Dual(vp, self.d * (p * self.v ** (p - 1)))

    # elementary functions (dispatched from the module functions below)
    def _exp(self):
        e = np.exp(self.v)
        return Dual(e, self.d * e)

    def _expm1(self):
        return Dual(np.expm1(self.v), self.d * np.exp(self.v))

    def _log(self):
        return Dual(np.log(self.v), self.d / self.v)

    def _sqrt(self):
        s = np.sqrt(self.v)
        return Dual(s, self.d * (0.5 / s))

    @staticmethod
    def _where(cond, a, b):
        shape_n = (a.d if isinstance(a, Dual) else b.d).shape
        av = val(a)
        bv = val(b)
        ad = a.d if isinstance(a, Dual) else np.zeros(shape_n)
        bd = b.d if isinstance(b, Dual) else np.zeros(shape_n)
        return Dual(np.where(cond, av, bv), np.where(cond[None, :], ad, bd))


def val(x):
    """Value part of a Dual, or the array itself."""
    return x.v if isinstance(x, Dual) else x


def exp(x):
    return x._exp() if isinstance(x, Dual) else np.exp(x)


def expm1(x):
    return x._expm1() if isinstance(x, Dual) else np.expm1(x)


def log(x):
    return x._log() if isinstance(x, Dual) else np.log(x)


def sqrt(x):
    return x._sqrt() if isinstance(x, Dual) else np.sqrt(x)


def where(cond, a, b):
    """Pick a where cond else b, elementwise; cond is a boolean array computed
    from values only, so the derivative is that of the branch taken."""
    if isinstance(a, Dual):
        return type(a)._where(cond, a, b)
    if isinstance(b, Dual):
        return type(b)._where(cond, a, b)
    return np.where(cond, a, b)


def seed(X):
    """Turn a state array X (n, N) into a list of n Duals with unit gradients."""
    n, N = X.shape
    out = []
    for i in range(n):
        d = np.zeros((n, N))
        d[i, :] = 1.0
        out.append(Dual(X[i].astype(np.float64), d))
    return out


def split(values, n, N):
    """Collect a list of n model outputs (Duals or constants) into the value
    array F (n, N) and the Jacobian J (N, n, n) with J[v, i, k] = dF_i/dX_k."""
    F = np.empty((n, N))
    J = np.zeros((N, n, n))
    for i, f in enumerate(values):
        if isinstance(f, Dual):
            F[i] = f.v
            J[:, i, :] = f.d.T
        else:
            F[i] = f
    return F, J
