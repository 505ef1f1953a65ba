"""Tetrahedral P1 / P2 elements on the unit cube (the d = 3 case of Section 2: the paper's
domain is a subset of R^d, d = 2, 3).

Oracle module (test infrastructure only).

Mesh: n^3 cubes, each split into the six tetrahedra of the Kuhn triangulation that share
the cube's main diagonal: for a permutation (a, b, c) of the axes the tetrahedron has the
vertices v0 = (i, j, k), v1 = v0 + e_a, v2 = v1 + e_b, v3 = (i + 1, j + 1, k + 1).  All
cubes use the same split, so the mesh is conforming; every edge midpoint lies on the
doubled lattice, which carries the P2 displacement nodes.

Element matrices are integrated with a collapsed Gauss-Legendre rule (the reference
tetrahedron as the image of the unit cube under x = u, y = (1-u) v, z = (1-u)(1-v) w,
Jacobian (1-u)^2 (1-v)), exact for the polynomial degrees that occur here; the forms are
those of Section 2.3: [A]_ij = 2 mu (eps(theta_j), eps(theta_i)), [B]_ij = -(phi_i, div
theta_j), [R]_ij = (phi_i, phi_j), [A_f]_ij = (K/mu_f)(grad phi_j, grad phi_i), and the
scalar P_k mass for the load vectors of nodal data.
"""
from __future__ import annotations

import numpy as np

PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


class Mesh3D:
    """Kuhn tetrahedra of the unit cube with n cubes per side."""

    def __init__(self, n: int, order: int):
        self.n, self.order = n, order
        r = 1 if order == 1 else 2
        self.r = r
        self.mu = r * n + 1          # displacement lattice points per side
        self.n1 = n + 1              # P1 lattice points per side
        self.nu_lat = self.mu ** 3
        self.n1_lat = self.n1 ** 3
        ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        cells = np.stack([ii.T.ravel(), jj.T.ravel(), kk.T.ravel()], axis=1)  # x fastest
        V = np.zeros((len(cells), 6, 4, 3), dtype=np.int64)
        for t, (a, b, c) in enumerate(PERMS):
            e = np.eye(3, dtype=np.int64)
            V[:, t, 0] = cells
            V[:, t, 1] = cells + e[a]
            V[:, t, 2] = cells + e[a] + e[b]
            V[:, t, 3] = cells + 1
        self.V = V.reshape(-1, 4, 3)                   # lattice coordinates of the vertices
        self.cell = np.repeat(np.arange(len(cells)), 6)
        self.X = self.V / float(n)
        n1, mu = self.n1, self.mu
        self.p1 = (self.V[:, :, 2] * n1 + self.V[:, :, 1]) * n1 + self.V[:, :, 0]
        U = r * self.V
        if r == 2:
            mids = np.stack([(U[:, a] + U[:, b]) // 2 for a, b in EDGES], axis=1)
            U = np.concatenate([U, mids], axis=1)
        self.U = U                                     # displacement lattice coordinates
        self.pu = (U[:, :, 2] * mu + U[:, :, 1]) * mu + U[:, :, 0]
        centre = (self.V[:, 0] + 0.5 * (self.V[:, 3] - self.V[:, 0]))
        self.cell_xyz = (cells + 0.5) / n
        self.tet_poro = (cells[self.cell, 0] + 0.5) / n < 0.5
        del centre

    def pu_xyz(self, nodes):
        mu = self.mu
        nodes = np.asarray(nodes)
        return np.stack([nodes % mu, (nodes // mu) % mu, nodes // (mu * mu)], axis=-1) / float(self.r * self.n)

    def p1_xyz(self, nodes):
        n1 = self.n1
        nodes = np.asarray(nodes)
        return np.stack([nodes % n1, (nodes // n1) % n1, nodes // (n1 * n1)], axis=-1) / float(self.n)

    def on_faces_pu(self, nodes, mask):
        return _on_faces(np.asarray(nodes), self.mu, mask)

    def on_faces_p1(self, nodes, mask):
        return _on_faces(np.asarray(nodes), self.n1, mask)


def _on_faces(nodes, m, mask):
    i, j, k = nodes % m, (nodes // m) % m, nodes // (m * m)
    out = np.zeros(nodes.shape, dtype=bool)
    for bit, hit in enumerate((i == 0, i == m - 1, j == 0, j == m - 1, k == 0, k == m - 1)):
        if mask >> bit & 1:
            out |= hit
    return out


def tet_rule(q: int = 4):
    """Collapsed Gauss-Legendre rule on the reference tetrahedron (vertices 0, e1, e2, e3):
    points (q^3, 3), weights summing to 1/6; exact for polynomials of degree <= 2q - 3."""
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for u, wu in zip(x, w):
        for v, wv in zip(x, w):
            for s, ws in zip(x, w):
                pts.append((u, (1 - u) * v, (1 - u) * (1 - v) * s))
                wts.append(wu * wv * ws * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def _basis(order, lam, glam):
    """Values (Q, nloc) and gradients (E, Q, nloc, 3) of the P_order basis from the
    barycentric coordinates lam (Q, 4) and their constant gradients glam (E, 4, 3)."""
    if order == 1:
        val = lam
        grad = np.broadcast_to(glam[:, None], (glam.shape[0], lam.shape[0], 4, 3))
        return val, grad
    vals = [lam[:, i] * (2 * lam[:, i] - 1) for i in range(4)]
    grads = [(4 * lam[:, i] - 1)[None, :, None] * glam[:, None, i, :] for i in range(4)]
    for a, b in EDGES:
        vals.append(4 * lam[:, a] * lam[:, b])
        grads.append(4 * (lam[:, a][None, :, None] * glam[:, None, b, :] + lam[:, b][None, :, None] * glam[:, None, a, :]))
    return np.stack(vals, axis=1), np.stack(grads, axis=2)


def geometry(X):
    """Jacobians of the affine maps of the elements X (E, 4, 3): |det J| (E,) and the
    gradients of the barycentric coordinates (E, 4, 3)."""
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)               # rows: gradients of the reference coordinates
    g = np.empty((len(X), 4, 3))
    g[:, 1:] = Jinv
    g[:, 0] = -Jinv.sum(axis=1)
    return np.abs(det), g


def element_matrices(order: int, X: np.ndarray, mu: float, kappa: float, q: int = 4):
    """Element matrices of the elements X (E, 4, 3).  Displacement DOFs interleaved by node
    (3 a + c for node a, component c).  Returns A (E, 3n, 3n), B (E, 4, 3n), R (E, 4, 4),
    Af (E, 4, 4) and M (E, n, n), the scalar P_order mass."""
    pts, wts = tet_rule(q)
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)
    adet, glam = geometry(X)
    W = adet[:, None] * wts[None, :]                         # (E, Q)
    phi, dphi = _basis(order, lam, glam)                     # (Q, n), (E, Q, n, 3)
    psi, dpsi = _basis(1, lam, glam)
    n = phi.shape[1]
    E = len(X)
    # A[ac, bd] = mu * int (delta_cd grad phi_a . grad phi_b + d_d phi_a d_c phi_b)
    G = np.einsum('eq,eqai,eqbj->eaibj', W, dphi, dphi)      # int d_i phi_a d_j phi_b
    A = np.zeros((E, n, 3, n, 3))
    lap = np.einsum('eaibi->eab', G)
    for c in range(3):
        A[:, :, c, :, c] += mu * lap
    A += mu * np.transpose(G, (0, 1, 4, 3, 2))               # [a, c, b, d] <- G[a, d, b, c]
    A = A.reshape(E, 3 * n, 3 * n)
    # B[i, bd] = - int psi_i d_d phi_b
    B = -np.einsum('eq,qi,eqbd->eibd', W, psi, dphi).reshape(E, 4, 3 * n)
    R = np.einsum('eq,qi,qj->eij', W, psi, psi)
    Af = kappa * np.einsum('eq,eqik,eqjk->eij', W, dpsi, dpsi)
    M = np.einsum('eq,qi,qj->eij', W, phi, phi)
    return {'A': A, 'B': B, 'R': R, 'Af': Af, 'M': M}
