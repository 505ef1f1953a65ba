"""Material constants and loads of the coupled problem.

Oracle module (test infrastructure only).

* Lame constants from (E, nu) as in Table 3 (lame_mode 1 keeps the literal
  mu = E/(1+nu) printed there; lame_mode 0 uses the textbook E/(2(1+nu))).
* kappa_1..3 of Section 2.2, obtained here by inverting eq. (mreform)
  symbolically rather than copying the printed formulas.
* Loads.  For the smooth manufactured solution of Section 4.1 the body forces
  and the fluid source are derived symbolically from the governing equations
  (2.1)-(2.3) with the constitutive relations of Table 1 (gravity off):
      f_P = -div sigma_P(u_P) + alpha grad p
      z   = d/dt (c0 p + alpha div u_P) - div((K/mu_f) grad p)
      f_E = -div sigma_E(u_E)
  sigma_D(u) = lambda_D div u I + 2 mu_D eps(u).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable

import numpy as np
import sympy as sp

from workloads import (Material, Load, Workload, XSPLIT, YSPLIT, CORE,
                       MANUFACTURED, PERIODIC, POINT_SOURCE, PATCH, RAW,
                       PATCH_UX, PATCH_UY, PATCH_P)


def lame(m: Material):
    lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu))
    if m.lame_mode == 1:
        mu = m.E / (1.0 + m.nu)
    else:
        mu = m.E / (2.0 * (1.0 + m.nu))
    return lam, mu


def kappas(m: Material):
    """Solve eq. (mreform) xi = alpha p - lam eps, eta = c0 p + alpha eps for (p, eps).

    Returns (kappa1, kappa2, kappa3) with p = k1 xi + k2 eta and
    eps = k1 eta - k3 xi.
    """
    lam, _ = lame(m)
    p, e, xi, eta = sp.symbols('p e xi eta')
    sol = sp.solve([sp.Eq(xi, m.alpha * p - lam * e), sp.Eq(eta, m.c0 * p + m.alpha * e)],
                   [p, e], dict=True)[0]
    k1 = float(sp.diff(sol[p], xi))
    k2 = float(sp.diff(sol[p], eta))
    k3 = float(-sp.diff(sol[e], xi))
    return k1, k2, k3


@dataclass
class Loads:
    fPx: Callable
    fPy: Callable
    fEx: Callable
    fEy: Callable
    z: Callable
    # exact solution (None for loads without one)
    uPx: Callable = None
    uPy: Callable = None
    uEx: Callable = None
    uEy: Callable = None
    p: Callable = None
    xiP: Callable = None
    xiE: Callable = None
    eta: Callable = None
    # initial data
    u0x_P: Callable = None
    u0y_P: Callable = None
    u0x_E: Callable = None
    u0y_E: Callable = None
    p0: Callable = None
    eta0: Callable = None


def _zero(x, y, t):
    return np.zeros_like(np.asarray(x, dtype=np.float64))


def _lam(expr, x, y, t):
    f = sp.lambdify((x, y, t), expr, 'numpy')

    def g(X, Y, T):
        return np.broadcast_to(np.asarray(f(X, Y, T), dtype=np.float64), np.shape(X)).copy()
    return g


def manufactured_symbolic(w: Workload):
    """Symbolic exact fields of Section 4.1 (or the polynomial patch solution)
    for the layout of ``w``.  The elastic displacement adds the correction of
    Section 4.1 that makes the traction and displacement continuous on the
    interface, rotated to the x-split layout when needed."""
    x, y, t = sp.symbols('x y t', real=True)
    lamP, muP = lame(w.mat_p)
    lamE, muE = lame(w.mat_e)
    a = w.mat_p.alpha
    if w.load.kind == PATCH:
        mono = [1, x, y, x * x, x * y, y * y]
        nq = 6 if w.order_u == 2 else 3
        uP = sp.Matrix([sum(sp.Float(c) * mm for c, mm in zip(PATCH_UX[:nq], mono[:nq])),
                        sum(sp.Float(c) * mm for c, mm in zip(PATCH_UY[:nq], mono[:nq]))])
        p = sp.Float(PATCH_P[0]) + (sp.Float(PATCH_P[1]) * y if w.order_u == 2 else 0)
    else:
        s = sp.sin(2 * sp.pi * x) * sp.sin(2 * sp.pi * y)
        uP = sp.Matrix([s, s])
        p = sp.sin(sp.pi * x) * sp.sin(sp.pi * y)
    if w.layout == XSPLIT:
        uE = uP + sp.Matrix([-a * p * (x - sp.Rational(1, 2)) / (lamP + 2 * muP), 0])
    elif w.layout == YSPLIT:
        uE = uP + sp.Matrix([0, -a * p * (y - sp.Rational(1, 2)) / (lamP + 2 * muP)])
    else:
        raise ValueError("manufactured solution needs a straight interface")
    return x, y, t, uP, uE, p, (lamP, muP, lamE, muE)


def _div(u, x, y):
    return sp.diff(u[0], x) + sp.diff(u[1], y)


def _div_sigma(u, lam, mu, x, y):
    gu = sp.Matrix([[sp.diff(u[0], x), sp.diff(u[0], y)],
                    [sp.diff(u[1], x), sp.diff(u[1], y)]])
    eps = (gu + gu.T) / 2
    sig = lam * _div(u, x, y) * sp.eye(2) + 2 * mu * eps
    return sp.Matrix([sp.diff(sig[0, 0], x) + sp.diff(sig[0, 1], y),
                      sp.diff(sig[1, 0], x) + sp.diff(sig[1, 1], y)])


def make_loads(w: Workload) -> Loads:
    L = w.load
    if L.kind in (MANUFACTURED, PATCH):
        x, y, t, uP, uE, p, (lamP, muP, lamE, muE) = manufactured_symbolic(w)
        mp = w.mat_p
        fP = -_div_sigma(uP, lamP, muP, x, y) + mp.alpha * sp.Matrix([sp.diff(p, x), sp.diff(p, y)])
        fE = -_div_sigma(uE, lamE, muE, x, y)
        kap = mp.K / mp.mu_f
        z = sp.diff(mp.c0 * p + mp.alpha * _div(uP, x, y), t) \
            - kap * (sp.diff(p, x, 2) + sp.diff(p, y, 2))
        xiP = mp.alpha * p - lamP * _div(uP, x, y)
        eta = mp.c0 * p + mp.alpha * _div(uP, x, y)
        xiE = -lamE * _div(uE, x, y)
        f = lambda e: _lam(sp.simplify(e), x, y, t)
        return Loads(fPx=f(fP[0]), fPy=f(fP[1]), fEx=f(fE[0]), fEy=f(fE[1]), z=f(z),
                     uPx=f(uP[0]), uPy=f(uP[1]), uEx=f(uE[0]), uEy=f(uE[1]), p=f(p),
                     xiP=f(xiP), xiE=f(xiE), eta=f(eta),
                     u0x_P=f(uP[0]), u0y_P=f(uP[1]), u0x_E=f(uE[0]), u0y_E=f(uE[1]),
                     p0=f(p), eta0=f(eta))
    if L.kind == PERIODIC:
        A, om, ph = L.amp, L.omega, L.phase

        def fx(x, y, t):
            return A * math.sin(om * t + ph) * np.sin(np.pi * x) * np.sin(np.pi * y)

        def fy(x, y, t):
            return A * math.sin(om * t + ph) * np.cos(np.pi * x) * np.sin(np.pi * y)

        def z(x, y, t):
            return A * math.sin(om * t + ph) * np.sin(np.pi * x) * np.sin(np.pi * y)
        return Loads(fPx=fx, fPy=fy, fEx=fx, fEy=fy, z=z,
                     u0x_P=_zero, u0y_P=_zero, u0x_E=_zero, u0y_E=_zero, p0=_zero, eta0=_zero)
    if L.kind == POINT_SOURCE:
        cx, cy, sg = L.cx, L.cy, L.sigma

        def z(x, y, t):
            r2 = (x - cx) ** 2 + (y - cy) ** 2
            return math.sin(t) * np.exp(-r2 / (2 * sg * sg)) / (2 * np.pi * sg * sg)
        return Loads(fPx=_zero, fPy=_zero, fEx=_zero, fEy=_zero, z=z,
                     u0x_P=_zero, u0y_P=_zero, u0x_E=_zero, u0y_E=_zero, p0=_zero, eta0=_zero)
    if L.kind == RAW:
        # the data are nodal arrays (workloads.raw_arrays); the assembly reads them directly
        return Loads(fPx=_zero, fPy=_zero, fEx=_zero, fEy=_zero, z=_zero)
    raise ValueError(L.kind)
