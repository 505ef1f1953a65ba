"""Pins of the 3D oracle (d = 3 of Section 2: Kuhn tetrahedra of the unit cube, P2 or P1
displacement and P1 scalars, eq. (linalg-system) with three displacement components).

Each check ties the module to something other than itself: exactness of the collapsed
rule on monomials (closed form a! b! c! / (a + b + c + 3)!), textbook closed forms of the
P1 mass, the P1 stiffness and the integrals of the P2 basis, the six rigid-body modes in
the kernels of A and B, the stationary polynomial solution that the spaces contain
(reproduced to rounding, and lost when a coupling sign flips), and the numbering rules.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import indexing as ix
from oracle.fem3d import Mesh3D, element_matrices, tet_rule, geometry
from oracle.monolithic3d import MonolithicSystem3D, solve_steps, patch_data, patch_exact


def test_collapsed_rule_is_exact_to_degree_5_and_not_6():
    pts, w = tet_rule(4)
    for a, b, c in [(0, 0, 0), (1, 0, 0), (2, 1, 1), (3, 1, 1), (2, 2, 1), (4, 1, 0), (5, 0, 0), (1, 2, 2)]:
        ex = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        q = (w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c).sum()
        assert abs(q - ex) <= 1e-14 * ex, (a, b, c)
    ex = math.factorial(6) / math.factorial(9)
    assert abs((w * pts[:, 0] ** 6).sum() - ex) > 1e-4 * ex


def test_element_closed_forms():
    m = Mesh3D(2, 2)
    em = element_matrices(2, m.X, 1.0, 1.7)
    em1 = element_matrices(1, m.X, 1.0, 1.7)
    vol, g = geometry(m.X)
    assert abs(vol.sum() / 6.0 - 1.0) < 1e-14          # the tetrahedra fill the cube
    for e in range(len(m.X)):
        T = vol[e] / 6.0
        R = T * (np.ones((4, 4)) + np.eye(4)) / 20.0
        assert np.abs(em['R'][e] - R).max() < 1e-15
        assert np.abs(em['Af'][e] - 1.7 * T * g[e] @ g[e].T).max() < 1e-12
        # P2 basis: int phi = -|T| / 20 at the vertices, |T| / 5 at the edge midpoints
        ip = em['M'][e].sum(axis=1)
        assert np.abs(ip[:4] + T / 20.0).max() < 1e-15 and np.abs(ip[4:] - T / 5.0).max() < 1e-15
        assert np.abs(em1['M'][e] - R).max() < 1e-15


@pytest.mark.parametrize("order", [1, 2])
def test_rigid_modes_in_the_kernels_of_A_and_B(order):
    m = Mesh3D(2, order)
    em = element_matrices(order, m.X, 1.3, 1.0)
    X = m.U / float(m.r * m.n)                          # displacement node coordinates
    for e in range(len(m.X)):
        modes = []
        for c in range(3):
            v = np.zeros((X.shape[1], 3))
            v[:, c] = 1.0
            modes.append(v.ravel())
        for i, j in ((0, 1), (0, 2), (1, 2)):
            v = np.zeros((X.shape[1], 3))
            v[:, i] = -X[e][:, j]
            v[:, j] = X[e][:, i]
            modes.append(v.ravel())
        Rm = np.array(modes).T
        assert np.abs(em['A'][e] @ Rm).max() < 1e-13
        assert np.abs(em['B'][e] @ Rm).max() < 1e-15


def _patch(order, ncell=4, nsub=(2, 2, 2)):
    w = W.cube_case(ncell=ncell, order_u=order, nsub=nsub, nsteps=2).replace(dirichlet_p=0x3F)
    kw = {} if order == 2 else {"q": (0.0, 0.0, 0.0)}
    w.load.raw_fixed = patch_data(w, **kw)
    return w, kw


@pytest.mark.parametrize("order", [1, 2])
def test_patch_solution_is_reproduced(order):
    w, kw = _patch(order)
    tr = solve_steps(w)
    ex = patch_exact(w, kw)
    for x in tr.states:
        lat = tr.system.to_lattice(x)
        for k, v in lat.items():
            sel = ~np.isnan(v)
            assert np.abs(v[sel] - ex[k][sel]).max() <= 1e-12 * max(1.0, np.abs(ex[k]).max()), k


def test_patch_breaks_if_a_coupling_sign_flips():
    w, kw = _patch(2)
    S = MonolithicSystem3D(w)
    o, n = S.blocks.offsets, S.blocks.sizes
    K = S.K.tolil()
    u = slice(o['uP'], o['uP'] + n['uP'])
    xi = slice(o['xiP'], o['xiP'] + n['xiP'])
    K[xi, u] = -K[xi, u]
    K[u, xi] = -K[u, xi]
    K = K.tocsr()
    S.Kff = K[S.free][:, S.free].tocsc()
    S.KfD = K[S.free][:, S.dir].tocsr()
    S.factor()
    x = S.solve_step(w.tau, S.initial_eta())
    lat = S.to_lattice(x)
    ex = patch_exact(w, kw)
    sel = ~np.isnan(lat['xiP'])
    assert np.abs(lat['xiP'][sel] - ex['xiP'][sel]).max() > 1e-3 * np.abs(ex['xiP']).max()


@pytest.mark.parametrize("w", [W.cube_case(ncell=4), W.cube_case(ncell=8, nsub=(4, 2, 2)),
                               W.cube_case(ncell=4, order_u=1, nsub=(2, 1, 3))], ids=lambda w: w.name)
def test_3d_numbering_rules(w):
    spec = ix.build(w)
    n, r = w.ncell, (2 if w.order_u == 2 else 1)
    mu, n1 = r * n + 1, n + 1
    cuts = [[(a * n) // k for a in range(k + 1)] for k in (w.nsub_x, w.nsub_y, w.nsub_z)]
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
            if kind == 2:
                ijk = (node % n1, (node // n1) % n1, node // (n1 * n1))
            else:
                IJK = (node % mu, (node // mu) % mu, node // (mu * mu))
                assert all(v % r == 0 for v in IJK)
                ijk = tuple(v // r for v in IJK)
            assert all(v in cut for v, cut in zip(ijk, cuts))
        else:
            assert len(o) in (2, 4)              # a face (two owners) or a grid edge (four)
    assert not any(s.floating for s in spec.subs)
    vals = [np.array([np.sin(0.37 * c) for c in s.codes]) for s in spec.subs]
    jump = np.array([sum(sg * vals[s][loc] for s, loc, sg in row) for row in spec.rows])
    assert np.abs(jump).max() == 0.0
    for row, c in zip(spec.rows, spec.row_code):
        for s, loc, _ in row:
            assert spec.subs[s].codes[loc] == c
