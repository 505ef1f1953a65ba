"""Pins of the decoupled-mass-balance oracle (the Remark after eq. (linalg-system),
Section 2.5): explicit lumped-mass update of the fluid content, momentum balance alone,
pressure from row 3.

Each check ties the module to something other than itself: the polynomial patch solution
(reproduced exactly by the discretisation and stationary in time), the coupled oracle's
own step (whose rows 1, 2, 3, 5, 6, 7 the decoupled momentum and pressure steps must
satisfy), the coupled discrete stationary state, first-order convergence in tau to the
implicit scheme with the same lumped storage term, and closed forms of the lumped mass and
of the fluid stiffness.
"""
import numpy as np
import pytest

import workloads as W
from oracle.decoupled import DecoupledState, DecoupledSystem, solve_steps as dec_steps
from oracle.monolithic import solve_steps as mono_steps


def _rel(a, b):
    sel = ~np.isnan(b)
    s = np.abs(b[sel]).max()
    return np.abs(a[sel] - b[sel]).max() / (s if s > 0 else 1.0)


@pytest.mark.parametrize("order", [1, 2])
def test_patch_solution_is_a_fixed_point(order):
    """The patch solution is stationary and reproduced exactly; from its nodal
    interpolant every decoupled step must return it (to rounding)."""
    w = W.patch_case(order_u=order, ncell=6, nsub_x=2, nsub_y=1, nsteps=3)
    tr = dec_steps(w)
    S = tr.system.S
    for x, t in zip(tr.states, tr.times):
        eu, ep = S.errors(x, t)
        assert eu < 1e-11 and ep < 1e-11, (eu, ep)
        lat = S.to_lattice(x)
        xy = S.mesh.p1_xy(np.arange(S.mesh.n1))
        for nm, fn in (("xiP", S.loads.xiP), ("eta", S.loads.eta), ("p", S.loads.p)):
            sel = ~np.isnan(lat[nm])
            ex = fn(xy[sel, 0], xy[sel, 1], t)
            assert np.abs(lat[nm][sel] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max()), nm


def test_momentum_and_pressure_steps_satisfy_the_coupled_rows():
    """Given the coupled step's eta^n, the decoupled momentum step must return the
    coupled (u, xi) (rows 1, 2, 5, 6, 7 are the same rows) and step (3) the coupled p
    (row 3 holds in the coupled solution)."""
    w = W.plain_fp64_small().replace(ncell=8, order_u=2)
    tr = mono_steps(w, nsteps=2)
    D = DecoupledSystem(w)
    for x_c, t in zip(tr.states, tr.times):
        eta_c = x_c[D.ieta]
        x_d = D.momentum(t, eta_c)
        lat_c, lat_d = D.S.to_lattice(x_c), D.S.to_lattice(x_d)
        for nm in ("ux_P", "uy_P", "ux_E", "uy_E", "xiP", "xiE"):
            assert _rel(lat_d[nm], lat_c[nm]) < 1e-10, nm
        p = D.k1 * x_d[D.ixi] + D.k2 * eta_c
        free = ~D.pdir
        pc = x_c[D.ip]
        assert np.abs(p[free] - pc[free]).max() < 1e-9 * np.abs(pc).max()


def test_momentum_step_breaks_without_the_fluid_coupling():
    """The same check fails if the k1 R_P eta term of row 2 is dropped (planted in a copy
    of the momentum right-hand side: eta taken as zero)."""
    w = W.plain_fp64_small().replace(ncell=8, order_u=2)
    tr = mono_steps(w, nsteps=1)
    D = DecoupledSystem(w)
    x_c, t = tr.states[0], tr.times[0]
    x_d = D.momentum(t, np.zeros(len(D.ieta)))
    lat_c, lat_d = D.S.to_lattice(x_c), D.S.to_lattice(x_d)
    assert _rel(lat_d["xiP"], lat_c["xiP"]) > 1e-3


def _periodic_case(order):
    """A smooth forced problem from the zero state (no start-up transient): the periodic
    load, alpha = 0.5 so that alpha^2 < c0 lambda (the stability condition of the lagged
    pressure Dirichlet nodes)."""
    w = W.plain_fp64_small().replace(ncell=8, order_u=order)
    w.mat_p.alpha = 0.5
    w.load.kind = W.PERIODIC
    w.load.amp = 1.0
    w.load.omega = 2 * np.pi * 20
    w.load.phase = 0.0
    return w


@pytest.mark.parametrize("order", [1, 2])
def test_first_order_in_tau_towards_the_implicit_scheme(order):
    """The decoupled scheme is explicit Euler on the semi-discrete system whose storage term
    uses the lumped mass; against the implicit (backward-Euler) scheme of that same system
    (the coupled oracle with lumped_storage) its error at a fixed time halves with tau."""
    base = _periodic_case(order)
    T = 0.016
    errs = []
    for tau in (2e-3, 1e-3, 5e-4):
        w = base.replace(tau=tau)
        n = int(round(T / tau))
        xd = dec_steps(w, nsteps=n).states[-1]
        trc = mono_steps(w, nsteps=n, lumped_storage=True)
        S = trc.system
        lc, ld = S.to_lattice(trc.states[-1]), S.to_lattice(xd)
        errs.append(max(_rel(ld[nm], lc[nm]) for nm in ("p", "eta", "xiP", "ux_P", "uy_E")))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[2] < 3e-2, errs
    assert 1.7 < r1 < 2.3 and 1.7 < r2 < 2.3, (errs, r1, r2)


def test_discrete_stationary_state_is_a_fixed_point():
    """The stationary solution of the coupled discrete problem (row 4 without the storage
    term) satisfies every step of the decoupled scheme: one step from it returns it."""
    w = W.plain_fp64_small().replace(ncell=8, order_u=2, tau=1e-3)
    D = DecoupledSystem(w)
    S = D.S
    S.factor()
    eta_s = S.initial_eta("steady")
    x1 = S.solve_step(w.tau, eta_s)
    st = DecoupledState(eta=x1[D.ieta].copy(), p=x1[D.ip].copy(), xi=x1[D.ixi].copy())
    x2, _ = D.step(2 * w.tau, st)
    l1, l2 = S.to_lattice(x1), S.to_lattice(x2)
    for nm in ("ux_P", "uy_P", "ux_E", "uy_E", "xiP", "eta", "p", "xiE"):
        assert _rel(l2[nm], l1[nm]) < 1e-11, nm


@pytest.mark.parametrize("layout", [W.XSPLIT, W.YSPLIT])
def test_lumped_mass_totals_the_poroelastic_area(layout):
    w = W.plain_fp64_small().replace(ncell=8, order_u=2, layout=layout)
    D = DecoupledSystem(w)
    assert abs(D.mL.sum() - 0.5) < 1e-13
    assert (D.mL > 0).all()


def test_fluid_stiffness_annihilates_constants_and_interior_linears():
    """A_f (Neumann stiffness of the poroelastic region) maps constants to zero and a
    linear pressure to zero at the nodes whose support lies inside the region."""
    w = W.plain_fp64_small().replace(ncell=8, order_u=1)
    D = DecoupledSystem(w)
    S = D.S
    xy = S.mesh.p1_xy(S.blocks.node['p'])
    one = np.ones(len(xy))
    assert np.abs(D.Af @ one).max() < 1e-13
    lin = 0.3 + 2.0 * xy[:, 0] - 1.5 * xy[:, 1]
    inner = (xy[:, 0] > 1e-12) & (xy[:, 0] < 0.5 - 1e-12) & (xy[:, 1] > 1e-12) & (xy[:, 1] < 1 - 1e-12)
    assert np.abs((D.Af @ lin)[inner]).max() < 1e-12
    assert np.abs((D.Af @ lin)[~inner]).max() > 1e-3  # the boundary rows carry the flux
