"""Pins of the oracle's caller-data (RAW) loads: nodal body forces and source, traction
on the sides without displacement Dirichlet data and fluid flux on the poroelastic
edges of the sides without pressure Dirichlet data (the boundary terms <t_P, v_P>,
<t_E, v_E> of eqs. (vf1), (vf4) and <z_w, q> of eq. (vf3)).

Patch test: a polynomial solution that the finite element spaces contain (P2 or P1
displacement, linear pressure, stationary) with its traction sigma~(u, xi) n, its flux
(K/mu_f) grad p . n and its (constant) body force given as nodal data must be
reproduced exactly by the discrete solution, for every mix of Dirichlet, traction
and flux sides.  A wrong edge mass matrix, a traction read on the wrong side, region or
component, or a flux with the wrong sign breaks the exactness.
"""
import numpy as np
import pytest
import sympy as sp

import workloads as W
from oracle.fem import edge_mass, mass
from oracle.monolithic import solve_steps
from oracle.problem import manufactured_symbolic, kappas


def _patch_raw(order_u, ncell, dir_u, dir_p, layout=W.XSPLIT):
    base = W.patch_case(order_u=order_u, ncell=ncell, nsub_x=2, nsub_y=1, nsteps=2)
    base = base.replace(layout=layout)
    x, y, t, uP, uE, p, (lamP, muP, lamE, muE) = manufactured_symbolic(base)
    mp = base.mat_p
    kap = mp.K / mp.mu_f

    def eps(u):
        g = sp.Matrix([[sp.diff(u[0], x), sp.diff(u[0], y)], [sp.diff(u[1], x), sp.diff(u[1], y)]])
        return (g + g.T) / 2

    divP = sp.diff(uP[0], x) + sp.diff(uP[1], y)
    divE = sp.diff(uE[0], x) + sp.diff(uE[1], y)
    xiP = mp.alpha * p - lamP * divP
    xiE = -lamE * divE
    sigP = 2 * muP * eps(uP) - xiP * sp.eye(2)
    sigE = 2 * muE * eps(uE) - xiE * sp.eye(2)
    fP = -sp.Matrix([sp.diff(sigP[0, 0], x) + sp.diff(sigP[0, 1], y), sp.diff(sigP[1, 0], x) + sp.diff(sigP[1, 1], y)])
    fE = -sp.Matrix([sp.diff(sigE[0, 0], x) + sp.diff(sigE[0, 1], y), sp.diff(sigE[1, 0], x) + sp.diff(sigE[1, 1], y)])
    normals = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    mu = order_u * ncell + 1
    n1 = ncell + 1
    su = 1.0 / (order_u * ncell)
    h = 1.0 / ncell
    Xu, Yu = np.meshgrid(np.arange(mu) * su, np.arange(mu) * su, indexing="xy")
    X1, Y1 = np.meshgrid(np.arange(n1) * h, np.arange(n1) * h, indexing="xy")
    ev = lambda e, X, Y: np.broadcast_to(np.asarray(sp.lambdify((x, y), e, "numpy")(X, Y), float), X.shape).ravel()
    raw = {"f_p": np.stack([ev(fP[c], Xu, Yu) for c in range(2)]),
           "f_e": np.stack([ev(fE[c], Xu, Yu) for c in range(2)]),
           "z": np.zeros(n1 * n1),
           "t_side": np.zeros((2, 4, 2, mu)), "zw_side": np.zeros((4, n1)),
           "g_u": np.zeros((2, mu * mu)), "g_p": ev(p, X1, Y1),
           "eta0": ev(mp.c0 * p + mp.alpha * divP, X1, Y1)}
    along_u = np.arange(mu) * su
    along_1 = np.arange(n1) * h
    for sd, (nx, ny) in enumerate(normals):
        if sd < 2:
            xs, ys, xs1, ys1 = np.full(mu, float(sd)), along_u, np.full(n1, float(sd)), along_1
        else:
            xs, ys, xs1, ys1 = along_u, np.full(mu, float(sd - 2)), along_1, np.full(n1, float(sd - 2))
        for r, sig in enumerate((sigP, sigE)):
            tr = sig * sp.Matrix([nx, ny])
            for c in range(2):
                raw["t_side"][r, sd, c] = ev(tr[c], xs, ys)
        raw["zw_side"][sd] = ev(kap * (sp.diff(p, x) * nx + sp.diff(p, y) * ny), xs1, ys1)
    # Dirichlet displacement: u_P where the cell region is poroelastic, u_E elsewhere
    # (the two agree on the interface)
    gP = np.stack([ev(uP[c], Xu, Yu) for c in range(2)])
    gE = np.stack([ev(uE[c], Xu, Yu) for c in range(2)])
    poro = (Xu.ravel() <= 0.5) if layout == W.XSPLIT else (Yu.ravel() <= 0.5)
    raw["g_u"] = np.where(poro[None, :], gP, gE)
    w = base.replace(name=f"rawpatch_p{order_u}_h{ncell}_u{dir_u}_p{dir_p}", load=W.Load(kind=W.RAW, raw_fixed=raw),
                     dirichlet_u=dir_u, dirichlet_p=dir_p)
    exact = {"uP": (gP, Xu), "uE": (gE, Xu), "p": ev(p, X1, Y1), "eta": raw["eta0"]}
    return w, exact


@pytest.mark.parametrize("order_u,ncell,dir_u,dir_p", [
    (2, 4, 0b0101, 0b0001),   # traction on x = 1 and y = 1 (both regions), flux on y = 0 and y = 1
    (2, 6, 0b0001, 0b0001),   # traction on three sides
    (2, 4, 0b1110, 0b1111),   # traction on x = 0 (poroelastic only), no flux side
    (1, 6, 0b0101, 0b0001),
])
def test_raw_patch_with_traction_and_flux_is_exact(order_u, ncell, dir_u, dir_p):
    w, exact = _patch_raw(order_u, ncell, dir_u, dir_p)
    tr = solve_steps(w, nsteps=2)
    S = tr.system
    for x in tr.states:
        lat = S.to_lattice(x)
        for name in ("ux_P", "uy_P", "ux_E", "uy_E"):
            comp = 0 if name[1] == "x" else 1
            ref = exact["uP" if name.endswith("P") else "uE"][0][comp]
            got = lat[name]
            sel = np.isfinite(got)
            assert sel.any()
            assert np.abs(got[sel] - ref[sel]).max() <= 1e-10 * max(1.0, np.abs(ref).max()), name
        for name in ("p", "eta"):
            got = lat[name]
            sel = np.isfinite(got)
            assert np.abs(got[sel] - exact[name][sel]).max() <= 1e-10 * max(1.0, np.abs(exact[name]).max()), name


def test_raw_patch_fails_without_the_boundary_terms():
    """The same data with the traction and the flux dropped is no longer reproduced."""
    w, exact = _patch_raw(2, 4, 0b0101, 0b0001)
    raw = dict(w.load.raw_fixed)
    for key in ("t_side", "zw_side"):
        bad = dict(raw)
        bad[key] = np.zeros_like(raw[key])
        wb = w.replace(load=W.Load(kind=W.RAW, raw_fixed=bad))
        lat = solve_steps(wb, nsteps=1).system.to_lattice(solve_steps(wb, nsteps=1).states[0])
        errs = []
        for name, ref in (("ux_P", exact["uP"][0][0]), ("p", exact["p"])):
            sel = np.isfinite(lat[name])
            errs.append(np.abs(lat[name][sel] - ref[sel]).max())
        assert max(errs) > 1e-6, key


def test_edge_and_element_mass_integrate_polynomials():
    """Closed-form edge masses against Gauss-Legendre quadrature of the traces; element
    masses sum to the area and integrate x exactly."""
    s, wq = np.polynomial.legendre.leggauss(5)
    s = 0.5 * (s + 1)
    wq = 0.5 * wq
    L = 0.3
    for order, psi in ((1, [1 - s, s]), (2, [(1 - s) * (1 - 2 * s), s * (2 * s - 1), 4 * s * (1 - s)])):
        P = np.array(psi)
        ref = L * (P * wq) @ P.T
        assert np.allclose(edge_mass(order, L), ref, rtol=0, atol=1e-15)
    X = np.array([[[0.1, 0.2], [0.7, 0.25], [0.3, 0.9]]])
    area = 0.5 * abs((X[0, 1, 0] - X[0, 0, 0]) * (X[0, 2, 1] - X[0, 0, 1]) - (X[0, 2, 0] - X[0, 0, 0]) * (X[0, 1, 1] - X[0, 0, 1]))
    for order in (1, 2):
        M = mass(order, X)[0]
        assert abs(M.sum() - area) < 1e-15
    # integral of x over the triangle = area * mean of the vertex x's; the nodal values of
    # x for P2 are the vertex and midpoint x's
    xs = X[0, :, 0]
    nod = np.concatenate([xs, [(xs[0] + xs[1]) / 2, (xs[1] + xs[2]) / 2, (xs[2] + xs[0]) / 2]])
    assert abs(mass(2, X)[0].sum(axis=0) @ nod - area * xs.mean()) < 1e-15
