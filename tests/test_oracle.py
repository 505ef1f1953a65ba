"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against a
closed form, a polynomial reproduction property, a brute-force solve, an
invariant, or the convergence orders printed in Tables 4 and 5.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fem, indexing as ix, local as lo
from oracle.mesh import Mesh
from oracle.monolithic import MonolithicSystem, solve_steps, linf_l2_errors
from oracle.problem import kappas, lame

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- quadrature and element matrices ---------------------------------------

def test_radon7_integrates_degree5_monomials_exactly():
    # reference triangle (0,0),(1,0),(0,1): int x^a y^b = a! b! / (a+b+2)!
    X = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    L, w = fem.radon7()
    pts = L @ X[0]
    for a in range(6):
        for b in range(6 - a):
            q = 0.5 * np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(q - exact) < 1e-15, (a, b)


def test_radon7_not_exact_for_degree6():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    L, w = fem.radon7()
    pts = L @ X
    q = 0.5 * np.sum(w * pts[:, 0] ** 6)
    assert abs(q - math.factorial(6) / math.factorial(8)) > 1e-6


def test_p1_mass_and_stiffness_closed_forms():
    h = 0.25
    X = np.array([[[0, 0], [h, 0], [h, h]], [[0, 0], [h, h], [0, h]]], dtype=float)
    em = fem.element_matrices(1, X, mu=1.0, K_over_muf=1.0)
    area = h * h / 2
    mass = area / 12 * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    np.testing.assert_allclose(em['R'][0], mass, rtol=1e-14)
    np.testing.assert_allclose(em['R'][1], mass, rtol=1e-14)
    # Laplacian of the right isosceles triangle with the right angle at vertex 1
    lap = np.array([[0.5, -0.5, 0.0], [-0.5, 1.0, -0.5], [0.0, -0.5, 0.5]])
    np.testing.assert_allclose(em['Af'][0], lap, atol=1e-14)
    lap1 = np.array([[0.5, 0.0, -0.5], [0.0, 0.5, -0.5], [-0.5, -0.5, 1.0]])
    np.testing.assert_allclose(em['Af'][1], lap1, atol=1e-14)


@pytest.mark.parametrize("order", [1, 2])
def test_rigid_modes_in_kernel_of_A_and_divergence_free(order):
    rng = np.random.default_rng(0)
    X = rng.random((5, 3, 2))
    em = fem.element_matrices(order, X, mu=2.5, K_over_muf=1.0)
    L = np.eye(3) if order == 1 else np.array(
        [[1, 0, 0], [0, 1, 0], [0, 0, 1], [.5, .5, 0], [0, .5, .5], [.5, 0, .5]])
    for e in range(5):
        nodes = L @ X[e]
        for mode in range(3):
            r = np.zeros(2 * len(nodes))
            if mode < 2:
                r[mode::2] = 1.0
            else:
                r[0::2] = -nodes[:, 1]
                r[1::2] = nodes[:, 0]
            assert np.abs(em['A'][e] @ r).max() < 1e-12 * np.abs(em['A'][e]).max()
            assert np.abs(em['B'][e] @ r).max() < 1e-13
        # a uniform dilation u = x has eps = I: energy 2 mu * 2 * area
        r = np.zeros(2 * len(nodes))
        r[0::2] = nodes[:, 0]
        r[1::2] = nodes[:, 1]
        area, _ = fem.geometry(X[e:e + 1])
        assert abs(r @ em['A'][e] @ r - 2 * 2.5 * 2 * area[0]) < 1e-12
        # and div u = 2, so -(1, div u) = -2 area summed over the P1 test functions
        assert abs(em['B'][e].sum(axis=0) @ r + 2 * area[0]) < 1e-13


def test_assembled_B_vanishes_on_constants_at_interior_nodes():
    # 1^T B e_j = -int div theta_j = -boundary flux = 0 for an interior node j
    w = W.plain_fp64_small().replace(ncell=4, order_u=2)
    S = MonolithicSystem(w)
    b, o = S.blocks, S.blocks.offsets
    Bp = S.K[o['xiP']:o['xiP'] + b.sizes['xiP'], o['uP']:o['uP'] + b.sizes['uP']].toarray()
    colsum = Bp.sum(axis=0)
    xy = S.mesh.pu_xy(b.node['uP'])
    interior = (xy[:, 0] > 1e-12) & (xy[:, 0] < 0.5 - 1e-12) & (xy[:, 1] > 1e-12) & (xy[:, 1] < 1 - 1e-12)
    assert interior.any()
    assert np.abs(colsum[interior]).max() < 1e-14


def test_kappas_invert_the_multiphysics_map():
    # eq. (mreform): xi = alpha p - lam eps, eta = c0 p + alpha eps
    for m in (W.Material(E=1e4, nu=0.49999, c0=1e-3), W.Material(E=1.0, nu=0.3, c0=1.0, alpha=0.7)):
        k1, k2, k3 = kappas(m)
        lam, _ = lame(m)
        rng = np.random.default_rng(1)
        for _ in range(5):
            xi, eta = rng.standard_normal(2)
            p = k1 * xi + k2 * eta
            eps = k1 * eta - k3 * xi
            assert abs(m.alpha * p - lam * eps - xi) < 1e-9 * max(1, abs(lam * eps))
            assert abs(m.c0 * p + m.alpha * eps - eta) < 1e-12
        den = m.alpha ** 2 + m.c0 * lam
        assert abs(k1 - m.alpha / den) < 1e-15 * abs(k1) + 1e-300


def test_lame_modes():
    m = W.Material(E=1e4, nu=0.2)
    assert lame(m) == pytest.approx((1e4 * 0.2 / (1.2 * 0.6), 1e4 / 2.4))
    m.lame_mode = 1
    assert lame(m)[1] == pytest.approx(1e4 / 1.2)


# --- the global system ------------------------------------------------------

def test_system_matrix_symmetric():
    S = MonolithicSystem(W.nearly_incompressible_scaled(8, 2))
    K = S.K
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()


@pytest.mark.parametrize("order", [1, 2])
def test_patch_test_reproduces_polynomial_solution(order):
    # u in P_k, p linear (P2) or constant (P1): the discrete solution equals the exact one
    w = W.patch_case(order_u=order, ncell=6, nsub_x=2, nsub_y=1, nsteps=3)
    tr = solve_steps(w)
    S = tr.system
    for x, t in zip(tr.states, tr.times):
        eu, ep = S.errors(x, t)
        assert eu < 1e-12 and ep < 1e-12
        lat = S.to_lattice(x)
        xy = S.mesh.p1_xy(np.arange(S.mesh.n1))
        sel = ~np.isnan(lat['xiP'])
        ex = S.loads.xiP(xy[sel, 0], xy[sel, 1], t)
        assert np.abs(lat['xiP'][sel] - ex).max() < 1e-10 * max(1, np.abs(ex).max())


def test_patch_test_breaks_if_a_coupling_sign_flips():
    # the same check catches a wrong sign in one block (planted in a copy of the matrix)
    w = W.patch_case(order_u=2, ncell=4, nsub_x=2, nsub_y=1, nsteps=1)
    S = MonolithicSystem(w)
    b, o = S.blocks, S.blocks.offsets
    K = S.K.tolil()
    r = slice(o['xiP'], o['xiP'] + b.sizes['xiP'])
    c = slice(o['eta'], o['eta'] + b.sizes['eta'])
    K[r, c] = -K[r, c]
    S.K = K.tocsr()
    S.Kff = S.K[S.free][:, S.free].tocsc()
    S.KfD = S.K[S.free][:, S.dir].tocsr()
    S.factor()
    x = S.solve_step(w.tau, S.initial_eta(), refine=0)
    eu, ep = S.errors(x, w.tau)
    assert max(eu, ep) > 1e-6


def test_brute_force_dense_solve_matches():
    w = W.plain_fp64_small().replace(ncell=4, order_u=2)
    S = MonolithicSystem(w)
    S.factor()
    eta = S.initial_eta()
    x = S.solve_step(w.tau, eta)
    f = S.rhs(w.tau, eta)
    xD = S.dirichlet_values(w.tau)
    xd = np.linalg.solve(S.Kff.toarray(), f[S.free] - S.KfD @ xD)
    assert np.abs(x[S.free] - xd).max() <= 1e-10 * np.abs(xd).max()


def _orders(order_u, nu, hs, init="steady"):
    eu, ep = [], []
    for n in hs:
        w = W.paper_table_case(order_u, n, nu, nsteps=2, lame_mode=1)
        a, b = linf_l2_errors(solve_steps(w, init=init))
        eu.append(a)
        ep.append(b)
    hs = np.array(hs, dtype=float)
    r = np.log(hs[1:] / hs[:-1])
    return np.log(np.array(eu[:-1]) / eu[1:]) / r, np.log(np.array(ep[:-1]) / ep[1:]) / r


@pytest.mark.slow
@pytest.mark.parametrize("order_u,nu", [(2, "0.2"), (2, "0.4999"), (1, "0.2"), (1, "0.4999")])
def test_convergence_orders_match_tables_4_and_5(order_u, nu):
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    ref = tab["table4" if order_u == 2 else "table5"][nu]
    ou, op = _orders(order_u, float(nu), [16, 24, 32])
    # finest-pair displacement order within 0.35 of the printed one
    assert abs(ou[-1] - ref["u_order"][-1]) < 0.35, (ou, ref["u_order"])
    # pressure orders inside the range the tables print (1.3 .. 3.1)
    assert np.all((op > 1.3) & (op < 3.1)), op


# --- indexing and the torn system --------------------------------------------

def _xsplit_closed_form(n, nx, ny, order):
    # multipliers of a uniform nx x ny grid, x-split, u and p Dirichlet on the outer boundary
    r = 2 if order == 2 else 1
    per_comp = (nx - 1 + ny - 1) * (r * n - 1) + (nx - 1) * (ny - 1)
    cross = (nx // 2 - 1) * (ny - 1)
    eta = (nx // 2 - 1) * (n + 1) + (ny - 1) * (n // 2 + 1) + cross
    p = (nx // 2 - 1) * (n - 1) + (ny - 1) * (n // 2) + cross
    return 2 * per_comp + 3 * eta + p


@pytest.mark.parametrize("n,nx,ny,order", [(16, 2, 1, 1), (16, 4, 4, 2), (24, 4, 2, 2),
                                            (32, 8, 8, 2), (64, 8, 8, 2)])
def test_n_lambda_closed_form(n, nx, ny, order):
    w = W.nearly_incompressible_scaled(n, nx).replace(nsub_x=nx, nsub_y=ny, order_u=order)
    spec = ix.build(w)
    assert spec.n_lambda == _xsplit_closed_form(n, nx, ny, order)
    assert spec.n_lambda == ix.closed_form_n_lambda(w)


def test_jump_rows_signed_boolean_and_annihilate_continuous_fields():
    w = W.nearly_incompressible_scaled(8, 4)
    spec = ix.build(w)
    rows = spec.rows
    assert np.all(np.sort(rows[:, :, 2], axis=1) == [-1, 1])
    # B applied to a continuous field (value = f(code)) is zero
    vals = [np.array([np.sin(0.37 * c) for c in s.codes]) for s in spec.subs]
    jump = np.array([sum(sg * vals[s][loc] for s, loc, sg in r) for r in rows])
    assert np.abs(jump).max() == 0.0
    # P-E rows put +1 on the poroelastic copy
    for r in rows:
        (s1, _, g1), (s2, _, g2) = r
        if spec.subs[s1].poro != spec.subs[s2].poro:
            assert (g1 if spec.subs[s1].poro else g2) == 1
    # no multiplier on a Dirichlet node: every glued code is a local DOF of both sides
    for r, c in zip(rows, spec.row_code):
        for s, loc, _ in r:
            assert spec.subs[s].codes[loc] == c


def test_torn_system_equals_monolithic_solution():
    # Theorem 3.1: the primal part of the torn saddle-point system is the monolithic solution
    w = W.nearly_incompressible_scaled(8, 4).replace(mat_p=W.Material(E=10.0, nu=0.3, c0=0.5, K=0.2),
                                                      mat_e=W.Material(E=10.0, nu=0.3))
    L = lo.build_local(w)
    spec = L.spec
    ns = [len(s.codes) for s in spec.subs]
    off = np.concatenate([[0], np.cumsum(ns)])
    N = off[-1]
    nl = spec.n_lambda
    A = np.zeros((N + nl, N + nl))
    for i, K in enumerate(L.K):
        A[off[i]:off[i + 1], off[i]:off[i + 1]] = K
    for j, r in enumerate(spec.rows):
        for s, loc, sg in r:
            A[N + j, off[s] + loc] = sg
            A[off[s] + loc, N + j] = sg
    tr = solve_steps(w, nsteps=1)
    S = tr.system
    eta0 = S.initial_eta()
    etamap = dict(zip(8 * S.blocks.node['eta'] + 2, eta0))
    eta_loc = [np.array([etamap.get(c, 0.0) for c in s.codes]) for s in spec.subs]
    f = lo.local_rhs(w, L, w.tau, eta_loc)
    rhs = np.concatenate(f + [np.zeros(nl)])
    x = np.linalg.solve(A, rhs)
    lat = S.to_lattice(tr.states[0])
    names = {0: 'ux_', 1: 'uy_', 2: 'eta', 3: 'xiP', 4: 'p', 5: 'xiE'}
    for i, s in enumerate(spec.subs):
        for k, c in enumerate(s.codes):
            node, kind = c // 8, c % 8
            key = names[kind] + (('P' if s.poro else 'E') if kind < 2 else '')
            ref = lat[key][node]
            assert abs(x[off[i] + k] - ref) <= 1e-9 * max(1.0, abs(ref)), (i, c)


def test_floating_subdomain_kernel_and_generalized_inverse():
    w = W.nearly_incompressible_scaled(16, 4).replace(mat_p=W.Material(E=10.0, nu=0.3, c0=0.5, K=0.2),
                                                       mat_e=W.Material(E=10.0, nu=0.3))
    L = lo.build_local(w)
    nfloat = 0
    for s, K in zip(L.spec.subs, L.K):
        if not s.floating:
            continue
        nfloat += 1
        R = ix.rigid_modes(w, s)
        assert np.abs(K @ R).max() < 1e-12 * np.abs(K).max()
        Kp = lo.generalized_inverse(K, s.cats)
        assert np.abs(K @ Kp @ K - K).max() < 1e-8 * np.abs(K).max()
        assert np.linalg.matrix_rank(K, tol=1e-9 * np.abs(K).max()) == len(s.codes) - 3
    assert nfloat == 4


def test_schur_complement_inverse_is_the_interface_block_of_the_inverse():
    # Block elimination of eq. (reduced-system): with K ordered [I | b], the inverse of the
    # Schur complement S_bb = K_bb - K_bI K_II^{-1} K_Ib is the trailing b x b block of K^{-1}.
    # For a floating subdomain K is singular; removing its fixed DOFs (which sit in b) leaves
    # K_ss nonsingular, the same identity holds for the remaining interface set b', and the
    # rigid-mode traces span the kernel of S_bb.  A swapped I / b index set or a transposed
    # coupling block fails here.
    w = W.nearly_incompressible_scaled(16, 4).replace(mat_p=W.Material(E=10.0, nu=0.3, c0=0.5, K=0.2),
                                                       mat_e=W.Material(E=10.0, nu=0.3))
    L = lo.build_local(w)
    seen = {True: 0, False: 0}
    for s, K in zip(L.spec.subs, L.K):
        cats = np.asarray(s.cats)
        b = np.nonzero(cats >= 2)[0]
        S = lo.schur_bb(K, s.cats)
        assert S.shape == (len(b), len(b))
        assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
        keep = np.nonzero(cats != 4)[0]                 # all DOFs but the fixed ones
        bk = np.nonzero(cats[b] != 4)[0]                # b' inside b
        Kinv = np.linalg.inv(K[np.ix_(keep, keep)])
        pos = {g: i for i, g in enumerate(keep)}
        tail = Kinv[np.ix_([pos[g] for g in b[bk]], [pos[g] for g in b[bk]])]
        Sinv = np.linalg.inv(S[np.ix_(bk, bk)])
        assert np.abs(Sinv - tail).max() <= 1e-9 * np.abs(tail).max(), s.sid
        if s.floating:
            R = ix.rigid_modes(w, s)[b]
            assert np.abs(S @ R).max() <= 1e-10 * np.abs(S).max() * np.abs(R).max()
        seen[bool(s.floating)] += 1
    assert seen[True] > 0 and seen[False] > 0
