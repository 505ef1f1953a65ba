"""Lagrange P1/P2 elements on affine triangles and their element matrices.

Oracle module (test infrastructure only; see the package docstring).

Element matrices follow the bilinear forms of Section 2.3:
  (aD)  a_D(u, v) = 2 mu_D (eps(u), eps(v))
  (bD)  b_D(v, xi) = -(xi, div v)
  (af)  a_f(p, q) = (1/mu_f) (K grad p, grad q)
and the L2 mass (phi_i, phi_j) that builds the R blocks of eq. (linalg-system).
All integrals are evaluated with the 7-point degree-5 rule of Radon, which is
exact for every product that occurs (polynomial degree <= 4).
"""
from __future__ import annotations

import math

import numpy as np

_S15 = math.sqrt(15.0)


def radon7():
    """Barycentric points (7, 3) and weights (7,) of Radon's degree-5 rule.

    Weights are normalised to sum to one (multiply by the triangle area).
    Points: the centroid, and the two orbits (a, a, 1-2a) with
    a = (6 -+ sqrt 15)/21.
    """
    a1 = (6.0 - _S15) / 21.0
    a2 = (6.0 + _S15) / 21.0
    w0 = 9.0 / 40.0
    w1 = (155.0 - _S15) / 1200.0
    w2 = (155.0 + _S15) / 1200.0
    pts = [(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0)]
    wts = [w0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        pts += [(a, a, b), (a, b, a), (b, a, a)]
        wts += [w, w, w]
    return np.array(pts), np.array(wts)


def geometry(X):
    """Affine geometry of triangles X (E, 3, 2).

    Returns area (E,) and the constant barycentric gradients G (E, 3, 2),
    G[e, i] = grad lambda_i on triangle e.
    """
    X = np.asarray(X, dtype=np.float64)
    x0, x1, x2 = X[:, 0], X[:, 1], X[:, 2]
    d1 = x1 - x0
    d2 = x2 - x0
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    area = 0.5 * np.abs(det)
    # lambda_1 and lambda_2 as functions of x: solve [d1 d2] [l1 l2]^T = x - x0
    inv = np.empty((X.shape[0], 2, 2))
    inv[:, 0, 0] = d2[:, 1] / det
    inv[:, 0, 1] = -d2[:, 0] / det
    inv[:, 1, 0] = -d1[:, 1] / det
    inv[:, 1, 1] = d1[:, 0] / det
    G = np.empty((X.shape[0], 3, 2))
    G[:, 1] = inv[:, 0]
    G[:, 2] = inv[:, 1]
    G[:, 0] = -G[:, 1] - G[:, 2]
    return area, G


def basis(order, L):
    """Values of the P1 or P2 Lagrange basis at barycentric points L (q, 3).

    P2 node order: vertices 0, 1, 2 then edge midpoints (01), (12), (20).
    Returns (q, nb).
    """
    L = np.asarray(L)
    if order == 1:
        return L.copy()
    l0, l1, l2 = L[:, 0], L[:, 1], L[:, 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=1)


def basis_grad(order, L, G):
    """Gradients of the basis at barycentric points L (q, 3) on triangles G (E, 3, 2).

    Returns (E, q, nb, 2).
    """
    L = np.asarray(L)
    E = G.shape[0]
    q = L.shape[0]
    if order == 1:
        return np.broadcast_to(G[:, None, :, :], (E, q, 3, 2)).copy()
    out = np.empty((E, q, 6, 2))
    for i in range(3):
        out[:, :, i, :] = (4 * L[None, :, i, None] - 1) * G[:, None, i, :]
    for k, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
        out[:, :, 3 + k, :] = 4 * (L[None, :, b, None] * G[:, None, a, :]
                                   + L[None, :, a, None] * G[:, None, b, :])
    return out


def element_matrices(order_u, X, mu, K_over_muf):
    """Element matrices on triangles X (E, 3, 2) for one region.

    Returns dict with
      A  (E, 2nu, 2nu): 2 mu (eps(theta_j), eps(theta_i)); DOF (node, comp) -> 2*node+comp
      B  (E, 3, 2nu):   -(phi_k, div theta_j)
      R  (E, 3, 3):     (phi_k, phi_l)
      Af (E, 3, 3):     (K/mu_f) (grad phi_l, grad phi_k)
    """
    L, w = radon7()
    area, G = geometry(X)
    nu = 3 if order_u == 1 else 6
    gu = basis_grad(order_u, L, G)          # (E, q, nu, 2)
    g1 = basis_grad(1, L, G)                # (E, q, 3, 2)
    v1 = basis(1, L)                        # (q, 3)
    wq = w[None, :] * area[:, None]         # (E, q)
    E = X.shape[0]
    # symmetric gradients of vector basis theta_(i,c) = phi_i e_c
    eps = np.zeros((E, len(w), nu, 2, 2, 2))  # [..., node, comp, a, b]
    for c in range(2):
        for a in range(2):
            for b in range(2):
                # eps_ab(phi e_c) = 0.5 (d_a phi delta_bc + d_b phi delta_ac)
                val = 0.0
                if b == c:
                    val = val + 0.5 * gu[..., a]
                if a == c:
                    val = val + 0.5 * gu[..., b]
                eps[:, :, :, c, a, b] = val
    eps = eps.reshape(E, len(w), 2 * nu, 2, 2)
    A = 2.0 * mu * np.einsum('eq,eqiab,eqjab->eij', wq, eps, eps)
    div = eps[..., 0, 0] + eps[..., 1, 1]    # (E, q, 2nu)
    B = -np.einsum('eq,qk,eqj->ekj', wq, v1, div)
    R = np.einsum('eq,qk,ql->ekl', wq, v1, v1)
    Af = K_over_muf * np.einsum('eq,eqkd,eqld->ekl', wq, g1, g1)
    return dict(A=A, B=B, R=R, Af=Af)


def mass(order, X):
    """(phi_j, phi_i) of the P1 or P2 basis on triangles X (E, nb, nb), 7-point rule
    (exact: the integrand has degree <= 4).  With nodal coefficients c of an
    interpolant, mass @ c is its load vector (f_h, phi_i)."""
    L, w = radon7()
    area, _ = geometry(X)
    v = basis(order, L)
    return np.einsum('eq,qi,qj->eij', w[None, :] * area[:, None], v, v)


def edge_mass(order, length):
    """(psi_j, psi_i) over a straight edge of the given length for the traces of the P1
    or P2 basis on it, node order (end a, end b) or (end a, end b, midpoint).  Closed
    form: with s in [0, 1], psi_a = (1-s)(1-2s), psi_b = s(2s-1), psi_m = 4s(1-s)."""
    if order == 1:
        return length / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    return length / 30.0 * np.array([[4.0, -1.0, 2.0], [-1.0, 4.0, 2.0], [2.0, 2.0, 16.0]])


def load_vectors(order_u, X, fx, fy, z, t):
    """Consistent load vectors on triangles X with the 7-point rule.

    fx, fy, z: callables (x, y, t) -> array.  Returns Fu (E, 2nu), Z (E, 3).
    """
    L, w = radon7()
    area, _ = geometry(X)
    pts = np.einsum('qi,eid->eqd', L, X)     # physical quadrature points (E, q, 2)
    x, y = pts[..., 0], pts[..., 1]
    vu = basis(order_u, L)                   # (q, nu)
    v1 = basis(1, L)
    wq = w[None, :] * area[:, None]
    FX = fx(x, y, t) * wq
    FY = fy(x, y, t) * wq
    nu = vu.shape[1]
    Fu = np.empty((X.shape[0], 2 * nu))
    Fu[:, 0::2] = FX @ vu
    Fu[:, 1::2] = FY @ vu
    Z = (z(x, y, t) * wq) @ v1
    return Fu, Z


def interpolate_l2_error(order, X, coef, exact, t):
    """Squared L2 norm of (u_h - exact) over triangles X with the 7-point rule.

    coef: (E, nb) element coefficients of u_h; exact: callable (x, y, t).
    """
    L, w = radon7()
    area, _ = geometry(X)
    pts = np.einsum('qi,eid->eqd', L, X)
    vh = coef @ basis(order, L).T            # (E, q)
    ex = exact(pts[..., 0], pts[..., 1], t)
    return float(np.sum(w[None, :] * area[:, None] * (vh - ex) ** 2))
