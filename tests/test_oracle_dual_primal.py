"""Pins of the dual-primal oracle (primal xi / p and corner DOFs, multipliers on the
remaining u / eta DOFs; the SPD-safe gluing that the Introduction's BDDC / FETI-DP
references suggest for three-field Biot).

Each check ties the module to something other than itself: the monolithic solution of
eq. (linalg-system) (Theorem 3.1's equivalence holds for any gluing that enforces the
same continuity), the multipliers of the dual gluing on the DOFs where both are unique,
the inertia of the two interface operators (the dual gluing's F has one negative
eigenvalue per pressure-side multiplier, the dual-primal F none), the quasi-definite
sign pattern of the primal coarse matrix, and a lattice count of the multipliers.
"""
import numpy as np
import pytest

import workloads as W
from oracle import indexing as ix
from oracle import local as lo
from oracle.dual_primal import DualPrimal
from oracle.monolithic import solve_steps


def _soft(nsx=4, nsy=4, ncell=8, order=2, layout=W.XSPLIT):
    """Moderate materials (nu = 0.3) so that dense checks are well conditioned."""
    return W.nearly_incompressible_scaled(ncell, 4).replace(
        mat_p=W.Material(E=10.0, nu=0.3, c0=0.5, K=0.2), mat_e=W.Material(E=10.0, nu=0.3),
        nsub_x=nsx, nsub_y=nsy, order_u=order, layout=layout)


def _first_step_local(w, L):
    tr = solve_steps(w, nsteps=1)
    S = tr.system
    eta0 = S.initial_eta()
    etamap = dict(zip(8 * S.blocks.node['eta'] + 2, eta0))
    eta_loc = [np.array([etamap.get(c, 0.0) for c in s.codes]) for s in L.spec.subs]
    return tr, lo.local_rhs(w, L, w.tau, eta_loc)


NAMES = {0: 'ux_', 1: 'uy_', 2: 'eta', 3: 'xiP', 4: 'p', 5: 'xiE'}


@pytest.mark.parametrize("nsx,nsy,order,ncell,cut_x", [(4, 4, 2, 8, None), (4, 2, 1, 12, None), (2, 1, 2, 8, None),
                                                       (4, 3, 2, 12, (0, 2, 6, 9, 12))])
def test_dual_primal_numbering(nsx, nsy, order, ncell, cut_x):
    w = _soft(nsx, nsy, ncell, order).replace(coupling="primal", cut_x=cut_x)
    spec = ix.build(w)
    wd = w.replace(coupling="dual")
    dspec = ix.build(wd)
    cx, cy = w.cuts()
    r = 2 if order == 2 else 1
    mu = r * ncell + 1
    owners = {}
    for s in spec.subs:
        for c in s.codes:
            owners.setdefault(c, set()).add(s.sid)
    primal = set(int(c) for c in spec.primal)
    for c, o in owners.items():
        if len(o) < 2:
            continue
        kind, node = c % 8, c // 8
        if kind in (3, 4, 5):
            assert c in primal
        elif c in primal:
            # a U-type primal DOF sits at a corner of the subdomain grid
            if kind == 2:
                i, j = node % (ncell + 1), node // (ncell + 1)
            else:
                I, J = node % mu, node // mu
                assert I % r == 0 and J % r == 0
                i, j = I // r, J // r
            assert i in cx and j in cy
    assert not any(s.floating for s in spec.subs)
    # multiplier rows: exactly the dual gluing's rows of the non-primal codes, same order
    keep = [k for k, c in enumerate(dspec.row_code) if int(c) not in primal]
    assert np.array_equal(spec.row_code, dspec.row_code[keep])
    assert spec.n_lambda == ix.closed_form_n_lambda(w)
    # the two owners of every dual code; the rows annihilate a continuous field
    assert np.all(spec.mult == 2)
    vals = [np.array([np.sin(0.37 * c) for c in s.codes]) for s in spec.subs]
    jump = np.array([sum(sg * vals[s][loc] for s, loc, sg in row) for row in spec.rows])
    assert np.abs(jump).max() == 0.0
    # local order: interior, dual interface, primal interface (categories 0/1, 2, 3)
    for s in spec.subs:
        cats = np.asarray(s.cats)
        assert np.all(np.diff(cats) >= 0)
        for c, cat in zip(s.codes, cats):
            if cat == 3:
                assert c in primal
            elif cat == 2:
                assert c not in primal and len(owners[c]) == 2


@pytest.mark.parametrize("layout,order", [(W.XSPLIT, 2), (W.YSPLIT, 1)])
def test_dual_primal_solution_is_the_monolithic_solution(layout, order):
    w = _soft(4, 4, 8, order, layout).replace(coupling="primal")
    D = DualPrimal(w)
    tr, f = _first_step_local(w, D.L)
    lam, us = D.solve(f)
    lat = tr.system.to_lattice(tr.states[0])
    for s, u in zip(D.spec.subs, us):
        for k, c in enumerate(s.codes):
            node, kind = c // 8, c % 8
            key = NAMES[kind] + (('P' if s.poro else 'E') if kind < 2 else '')
            ref = lat[key][node]
            assert abs(u[k] - ref) <= 1e-9 * max(1.0, abs(ref)), (s.sid, c)


def test_dual_primal_multipliers_equal_the_dual_gluings_on_edge_dofs():
    # On a DOF shared by two subdomains the multiplier is the flux K_s u_s - f_s of one
    # side, fixed by the solution: both gluings must give it (a wrong sign of a B row or
    # a primal row left unsummed fails here).  The 2 x 2 decomposition has no floating
    # subdomain, so the dual gluing's torn system is solved directly.
    w = _soft(2, 2, 8, 2)
    Ld = lo.build_local(w)
    spec = Ld.spec
    ns = [len(s.codes) for s in spec.subs]
    off = np.concatenate([[0], np.cumsum(ns)])
    N, nl = off[-1], spec.n_lambda
    A = np.zeros((N + nl, N + nl))
    for i, K in enumerate(Ld.K):
        A[off[i]:off[i + 1], off[i]:off[i + 1]] = K
    for j, row in enumerate(spec.rows):
        for s, loc, sg in row:
            A[N + j, off[s] + loc] = sg
            A[off[s] + loc, N + j] = sg
    _, f = _first_step_local(w, Ld)
    lam_d = np.linalg.solve(A, np.concatenate(f + [np.zeros(nl)]))[N:]
    wp = w.replace(coupling="primal")
    D = DualPrimal(wp)
    _, fp = _first_step_local(wp, D.L)
    lam_p, _ = D.solve(fp)
    where = {int(c): j for j, c in enumerate(spec.row_code) if spec.mult[j] == 2}
    scale = np.abs(lam_d).max()
    for j, c in enumerate(D.spec.row_code):
        assert abs(lam_p[j] - lam_d[where[int(c)]]) <= 1e-9 * scale, c


@pytest.mark.parametrize("nsx,nsy", [(2, 2), (4, 2)])
def test_operator_inertia_dual_versus_dual_primal(nsx, nsy):
    # Dual gluing (no floating subdomain here, so F = sum_s B_s K_s^{-1} B_s^T): one
    # negative eigenvalue per multiplier of a negative-type field (xi_P, p, xi_E).
    # Dual-primal gluing: F symmetric positive definite.
    w = _soft(nsx, nsy, 8, 2)
    L = lo.build_local(w)
    spec = L.spec
    assert not any(s.floating for s in spec.subs)
    nl = spec.n_lambda
    F = np.zeros((nl, nl))
    for si, (s, K) in enumerate(zip(spec.subs, L.K)):
        B = np.zeros((nl, len(s.codes)))
        for j, row in enumerate(spec.rows):
            for sub, loc, sg in row:
                if sub == si:
                    B[j, loc] += sg
        F += B @ np.linalg.solve(K, B.T)
    ev = np.linalg.eigvalsh(0.5 * (F + F.T))
    n_p = int(np.isin(spec.row_code % 8, (3, 4, 5)).sum())
    assert n_p > 0
    assert int((ev < -1e-12 * np.abs(ev).max()).sum()) == n_p
    D = DualPrimal(w.replace(coupling="primal"))
    Fp = D.operator()
    assert np.abs(Fp - Fp.T).max() <= 1e-12 * np.abs(Fp).max()
    evp = np.linalg.eigvalsh(0.5 * (Fp + Fp.T))
    assert evp.min() > 1e-6 * evp.max()


def test_primal_coarse_matrix_is_quasi_definite_in_the_global_order():
    # The global primal order puts the U-type corners (u, eta) before xi and p: the U block
    # of S_PiPi is positive definite and the Schur complement onto the P-type block negative
    # definite, so S_PiPi has an LDL^T factorisation without pivoting in that order.
    w = _soft(4, 4, 8, 2).replace(coupling="primal")
    D = DualPrimal(w)
    S = D.coarse_matrix()
    assert np.abs(S - S.T).max() <= 1e-10 * np.abs(S).max()
    kinds = D.primal_kinds()
    U = np.isin(kinds, (0, 1, 2))
    first_p = int(np.argmax(~U))
    assert U[:first_p].all() and not U[first_p:].any()
    A = S[np.ix_(U, U)]
    assert np.linalg.eigvalsh(A).min() > 0.0
    Sc = S[np.ix_(~U, ~U)] - S[np.ix_(~U, U)] @ np.linalg.solve(A, S[np.ix_(U, ~U)])
    assert np.linalg.eigvalsh(0.5 * (Sc + Sc.T)).max() < 0.0
