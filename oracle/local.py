"""Torn (per-subdomain) form of the discrete system, in the numbering of
``oracle.indexing``.

Oracle module (test infrastructure only).

Sub-assembly: K = sum_s R_s^T K_s R_s, where K_s is the system matrix of eq.
(linalg-system) restricted to the elements of subdomain s (Dirichlet DOFs
removed and lifted).  For a poroelastic subdomain the unknowns are
(u, xi_P, eta, p) and the blocks are those of rows 1-4 of eq. (linalg-system);
for an elastic one (u, xi_E) with rows 5-6.  Gluing with the signed Boolean
maps B_s gives the torn saddle-point system

    K_s u_s + B_s^T lam = f_s,     sum_s B_s u_s = 0,

whose primal part equals the monolithic solution (Theorem 3.1).  The helpers
below build the dense K_s, the local right-hand sides, and the plain-definition
references for the quantities the FETI path derives from them: the interface
Schur complement S_bb = K_bb - K_bI K_II^{-1} K_Ib (eq. (reduced-system)) and
the generalised inverse with the fixed DOFs of a floating subdomain zeroed.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from workloads import Workload
from .mesh import Mesh
from .fem import element_matrices, load_vectors
from .problem import lame, kappas, make_loads
from . import indexing as ix


@dataclass
class LocalSystem:
    spec: ix.IndexSpec
    K: List[np.ndarray]          # dense K_s in local order
    lift_cols: List[np.ndarray]  # per subdomain: list of Dirichlet codes touched
    K_D: List[np.ndarray]        # K_s restricted to (local, Dirichlet-codes) for lifting
    elems: List[np.ndarray]      # triangle ids of each subdomain


def _local_element_codes(w: Workload, m: Mesh, tri: np.ndarray, poro: bool):
    """Codes of the element DOFs in the order of oracle.fem.element_matrices."""
    nloc = 3 if w.order_u == 1 else 6
    pu = m.pu[tri]
    p1 = m.p1[tri]
    ucodes = np.empty((len(tri), 2 * nloc), dtype=np.int64)
    ucodes[:, 0::2] = 8 * pu
    ucodes[:, 1::2] = 8 * pu + 1
    if poro:
        return ucodes, 8 * p1 + 3, 8 * p1 + 2, 8 * p1 + 4
    return ucodes, 8 * p1 + 5, None, None


def build_local(w: Workload) -> LocalSystem:
    spec = ix.build(w)
    m = Mesh(w.ncell, w.order_u, w.layout)
    lamP, muP = lame(w.mat_p)
    lamE, muE = lame(w.mat_e)
    k1, k2, k3 = kappas(w.mat_p)
    Ks, KDs, Dcodes, elems = [], [], [], []
    n = w.ncell
    for s in spec.subs:
        cells = [(j * n + i) for j in range(s.j0, s.j1) for i in range(s.i0, s.i1)]
        tri = np.array(sorted([2 * c for c in cells] + [2 * c + 1 for c in cells]))
        elems.append(tri)
        X = m.X[tri]
        if s.poro:
            em = element_matrices(w.order_u, X, muP, w.mat_p.K / w.mat_p.mu_f)
        else:
            em = element_matrices(w.order_u, X, muE, 1.0)
        uc, xc, ec, pc = _local_element_codes(w, m, tri, s.poro)
        trip = []   # (row codes, col codes, values)

        def add(rc, cc, M, sc=1.0):
            trip.append((np.broadcast_to(rc[:, :, None], M.shape).ravel(),
                         np.broadcast_to(cc[:, None, :], M.shape).ravel(), (sc * M).ravel()))
        add(uc, uc, em['A'])
        add(uc, xc, np.transpose(em['B'], (0, 2, 1)))
        add(xc, uc, em['B'])
        if s.poro:
            add(xc, xc, em['R'], -k3)
            add(xc, ec, em['R'], k1)
            add(ec, xc, em['R'], k1)
            add(ec, ec, em['R'], k2)
            add(ec, pc, em['R'], -1.0)
            add(pc, ec, em['R'], -1.0)
            add(pc, pc, em['Af'], -w.tau)
        else:
            add(xc, xc, em['R'], -1.0 / lamE)
        rc = np.concatenate([t[0] for t in trip])
        cc = np.concatenate([t[1] for t in trip])
        vv = np.concatenate([t[2] for t in trip])
        pos = {c: i for i, c in enumerate(s.codes)}
        # Dirichlet codes = codes that appear in elements but are not local DOFs
        allc = np.unique(np.concatenate([rc, cc]))
        dcodes = np.array([c for c in allc if c not in pos], dtype=np.int64)
        dpos = {c: i for i, c in enumerate(dcodes)}
        ns = len(s.codes)
        K = np.zeros((ns, ns))
        KD = np.zeros((ns, len(dcodes)))
        for r, c, v in zip(rc, cc, vv):
            if r not in pos:
                continue
            if c in pos:
                K[pos[r], pos[c]] += v
            else:
                KD[pos[r], dpos[c]] += v
        Ks.append(K)
        KDs.append(KD)
        Dcodes.append(dcodes)
    return LocalSystem(spec, Ks, Dcodes, KDs, elems)


def local_rhs(w: Workload, L: LocalSystem, t: float, eta_prev_local: List[np.ndarray],
              dirichlet_value=None) -> List[np.ndarray]:
    """f_s of the torn system at time t (rows 1 and 4 of eq. (linalg-system), lifted).

    eta_prev_local: per subdomain, the local eta^{n-1} values (indexed by local
    DOF, entries at non-eta DOFs ignored).
    """
    m = Mesh(w.ncell, w.order_u, w.layout)
    loads = make_loads(w)
    out = []
    for si, s in enumerate(L.spec.subs):
        tri = L.elems[si]
        X = m.X[tri]
        fx, fy = (loads.fPx, loads.fPy) if s.poro else (loads.fEx, loads.fEy)
        Fu, Z = load_vectors(w.order_u, X, fx, fy, loads.z, t)
        pos = {c: i for i, c in enumerate(s.codes)}
        f = np.zeros(len(s.codes))
        uc, xc, ec, pc = _local_element_codes(w, m, tri, s.poro)
        for codes, vals in ((uc, Fu),):
            for c, v in zip(codes.ravel(), vals.ravel()):
                if c in pos:
                    f[pos[c]] += v
        if s.poro:
            from .fem import element_matrices as _em
            em = _em(w.order_u, X, 1.0, 1.0)
            eta_loc = eta_prev_local[si]
            for e in range(len(tri)):
                ev = np.array([eta_loc[pos[c]] for c in ec[e]])
                Re = em['R'][e] @ ev
                for a in range(3):
                    c = pc[e, a]
                    if c in pos:
                        f[pos[c]] += -Re[a] - w.tau * Z[e, a]
        if dirichlet_value is not None and len(L.lift_cols[si]):
            xD = np.array([dirichlet_value(c, t) for c in L.lift_cols[si]])
            f -= L.K_D[si] @ xD
        out.append(f)
    return out


def schur_bb(K: np.ndarray, cats: List[int]) -> np.ndarray:
    """S_bb = K_bb - K_bI K_II^{-1} K_Ib over the interface set (categories 2, 3, 4)."""
    cats = np.asarray(cats)
    I = np.nonzero(cats < 2)[0]
    b = np.nonzero(cats >= 2)[0]
    if len(I) == 0:
        return K[np.ix_(b, b)].copy()
    return K[np.ix_(b, b)] - K[np.ix_(b, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, b)])


def generalized_inverse(K: np.ndarray, cats: List[int]) -> np.ndarray:
    """K^+ = [[K_ss^{-1}, 0], [0, 0]] with s = all DOFs except the fixed ones.

    For a floating subdomain K has the rigid modes as kernel and removing the
    fixed DOFs leaves a nonsingular K_ss, so K K^+ K = K.
    """
    cats = np.asarray(cats)
    s = np.nonzero(cats != 4)[0]
    Kp = np.zeros_like(K)
    Kp[np.ix_(s, s)] = np.linalg.inv(K[np.ix_(s, s)])
    return Kp


def build_local3d(w: Workload) -> LocalSystem:
    """The 3D torn matrices: K_s of every subdomain of the cube (its tetrahedra's element
    matrices of ``oracle.fem3d`` in the local order of ``oracle.indexing.build3d``,
    Dirichlet DOFs removed, K_D the columns of the Dirichlet codes for lifting)."""
    from .fem3d import Mesh3D, element_matrices as em3
    spec = ix.build(w)
    m = Mesh3D(w.ncell, w.order_u)
    lamP, muP = lame(w.mat_p)
    lamE, muE = lame(w.mat_e)
    k1, k2, k3 = kappas(w.mat_p)
    n = w.ncell
    nloc = 4 if w.order_u == 1 else 10
    Ks, KDs, Dcodes, elems = [], [], [], []
    for s in spec.subs:
        cells = [(k * n + j) * n + i for k in range(s.k0, s.k1) for j in range(s.j0, s.j1)
                 for i in range(s.i0, s.i1)]
        tet = np.array(sorted(6 * c + t for c in cells for t in range(6)))
        elems.append(tet)
        em = em3(w.order_u, m.X[tet], muP if s.poro else muE, (w.mat_p.K / w.mat_p.mu_f) if s.poro else 1.0)
        uc = np.empty((len(tet), 3 * nloc), dtype=np.int64)
        for c, kind in enumerate((0, 1, 6)):
            uc[:, c::3] = 8 * m.pu[tet] + kind
        p1 = m.p1[tet]
        trip = []

        def add(rc, cc, M, sc=1.0):
            trip.append((np.broadcast_to(rc[:, :, None], M.shape).ravel(),
                         np.broadcast_to(cc[:, None, :], M.shape).ravel(), (sc * M).ravel()))
        if s.poro:
            xc, ec, pc = 8 * p1 + 3, 8 * p1 + 2, 8 * p1 + 4
            add(uc, uc, em['A'])
            add(uc, xc, np.transpose(em['B'], (0, 2, 1)))
            add(xc, uc, em['B'])
            add(xc, xc, em['R'], -k3)
            add(xc, ec, em['R'], k1)
            add(ec, xc, em['R'], k1)
            add(ec, ec, em['R'], k2)
            add(ec, pc, em['R'], -1.0)
            add(pc, ec, em['R'], -1.0)
            add(pc, pc, em['Af'], -w.tau)
        else:
            xc = 8 * p1 + 5
            add(uc, uc, em['A'])
            add(uc, xc, np.transpose(em['B'], (0, 2, 1)))
            add(xc, uc, em['B'])
            add(xc, xc, em['R'], -1.0 / lamE)
        rc = np.concatenate([t[0] for t in trip])
        cc = np.concatenate([t[1] for t in trip])
        vv = np.concatenate([t[2] for t in trip])
        pos = {c: i for i, c in enumerate(s.codes)}
        allc = np.unique(np.concatenate([rc, cc]))
        dcodes = np.array([c for c in allc if c not in pos], dtype=np.int64)
        dpos = {c: i for i, c in enumerate(dcodes)}
        ns = len(s.codes)
        K = np.zeros((ns, ns))
        KD = np.zeros((ns, len(dcodes)))
        for r_, c_, v_ in zip(rc, cc, vv):
            if r_ not in pos:
                continue
            if c_ in pos:
                K[pos[r_], pos[c_]] += v_
            else:
                KD[pos[r_], dpos[c_]] += v_
        Ks.append(K)
        KDs.append(KD)
        Dcodes.append(dcodes)
    return LocalSystem(spec, Ks, Dcodes, KDs, elems)
