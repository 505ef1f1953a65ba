"""Monolithic FP64 solve of the fully discrete coupled problem.

Oracle module (test infrastructure only).

Per time step n = 1..N this solves eq. (linalg-system) of Section 2.5 for
(u_P, xi_P, eta, p, u_E, xi_E, lambda):

    A_P u_P + B_P^T xi_P + H_P^T lam                  = F_P^n
    B_P u_P - k3 R_P xi_P + k1 R_P eta                 = 0
              k1 R_P xi_P + k2 R_P eta - R_P p         = 0
                          - R_P eta    - tau A_f p     = -R_P eta^{n-1} - tau Z^n
    A_E u_E + B_E^T xi_E - H_E^T lam                  = F_E^n
    B_E u_E - (1/lambda_E) R_E xi_E                    = 0
    H_P u_P - H_E u_E                                  = 0

with the blocks of that section assembled from the element matrices in
``oracle.fem``.  Multipliers are nodal on the interface nodes that are not
Dirichlet nodes, so H_P, H_E are Boolean.  Dirichlet values are lifted to the
right-hand side.  The matrix is the same at every step (tau and the
coefficients are constant), so it is factorised once with SuperLU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from workloads import Workload, XSPLIT, YSPLIT, CORE, RAW, raw_arrays
from .mesh import Mesh
from .fem import element_matrices, load_vectors, interpolate_l2_error, mass, edge_mass
from .problem import lame, kappas, make_loads


def _coo_add(rows, cols, vals, R, C, V):
    rows.append(R.ravel())
    cols.append(C.ravel())
    vals.append(V.ravel())


@dataclass
class Blocks:
    names: List[str]
    offsets: Dict[str, int]
    sizes: Dict[str, int]
    # lattice node id and component of every DOF in each block
    node: Dict[str, np.ndarray]
    comp: Dict[str, np.ndarray]


class MonolithicSystem:
    """Assembled system of eq. (linalg-system) for one workload.

    lumped_storage: the fluid-content term of row 4 (-R_P eta^n and -R_P eta^{n-1}) with
    the mass matrix lumped to its row sums: the implicit counterpart of the decoupled
    scheme in ``oracle.decoupled`` (row 3 keeps the consistent mass)."""

    def __init__(self, w: Workload, lumped_storage: bool = False):
        t0 = time.perf_counter()
        self.w = w
        self.lumped_storage = lumped_storage
        self.mesh = m = Mesh(w.ncell, w.order_u, w.layout)
        self.loads = make_loads(w)
        lamP, muP = lame(w.mat_p)
        lamE, muE = lame(w.mat_e)
        self.lamP, self.muP, self.lamE, self.muE = lamP, muP, lamE, muE
        self.k1, self.k2, self.k3 = kappas(w.mat_p)
        P = m.tri_poro
        Ev = ~P
        self.triP = np.nonzero(P)[0]
        self.triE = np.nonzero(Ev)[0]
        # closure node sets
        uP_nodes = np.unique(m.pu[P])
        uE_nodes = np.unique(m.pu[Ev])
        sP_nodes = np.unique(m.p1[P])
        sE_nodes = np.unique(m.p1[Ev])
        gam_u = np.intersect1d(uP_nodes, uE_nodes)
        dirU = m.on_side_pu(np.arange(m.nu_lat), w.dirichlet_u)
        dirP = m.on_side_p1(np.arange(m.n1), w.dirichlet_p)
        lam_nodes = gam_u[~dirU[gam_u]]
        # block DOF lists (all DOFs, Dirichlet included)
        def vec(nodes):
            return np.repeat(nodes, 2), np.tile([0, 1], len(nodes))
        node, comp = {}, {}
        node['uP'], comp['uP'] = vec(uP_nodes)
        node['xiP'], comp['xiP'] = sP_nodes, np.zeros(len(sP_nodes), int)
        node['eta'], comp['eta'] = sP_nodes, np.zeros(len(sP_nodes), int)
        node['p'], comp['p'] = sP_nodes, np.zeros(len(sP_nodes), int)
        node['uE'], comp['uE'] = vec(uE_nodes)
        node['xiE'], comp['xiE'] = sE_nodes, np.zeros(len(sE_nodes), int)
        node['lam'], comp['lam'] = vec(lam_nodes)
        names = ['uP', 'xiP', 'eta', 'p', 'uE', 'xiE', 'lam']
        offs, sizes, o = {}, {}, 0
        for nm in names:
            offs[nm] = o
            sizes[nm] = len(node[nm])
            o += sizes[nm]
        self.blocks = Blocks(names, offs, sizes, node, comp)
        self.ndof = o
        # lattice -> position maps
        def pos_map(nodes, nlat):
            mp = -np.ones(nlat, dtype=np.int64)
            mp[nodes] = np.arange(len(nodes))
            return mp
        self.mapuP = pos_map(uP_nodes, m.nu_lat)
        self.mapuE = pos_map(uE_nodes, m.nu_lat)
        self.mapsP = pos_map(sP_nodes, m.n1)
        self.mapsE = pos_map(sE_nodes, m.n1)
        # Dirichlet mask over the full DOF vector
        dmask = np.zeros(self.ndof, dtype=bool)
        dmask[offs['uP']:offs['uP'] + sizes['uP']] = dirU[node['uP']]
        dmask[offs['uE']:offs['uE'] + sizes['uE']] = dirU[node['uE']]
        dmask[offs['p']:offs['p'] + sizes['p']] = dirP[node['p']]
        self.dmask = dmask
        self.free = np.nonzero(~dmask)[0]
        self.dir = np.nonzero(dmask)[0]
        self._assemble()
        self._boundary_edges()
        self.t_assemble = time.perf_counter() - t0

    # ------------------------------------------------------------------
    def _boundary_edges(self):
        """Edges of the mesh on the four sides of the square (side 0: x = 0, 1: x = 1,
        2: y = 0, 3: y = 1): triangle, side, the P1 end nodes and the displacement
        nodes (ends, then the midpoint for P2)."""
        m = self.mesh
        n = m.n
        tri, side, p1n, pun = [], [], [], []
        for k, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
            via, vib = m.tri_vi[:, a], m.tri_vi[:, b]
            vja, vjb = m.tri_vj[:, a], m.tri_vj[:, b]
            for sd, hit in enumerate(((via == 0) & (vib == 0), (via == n) & (vib == n),
                                      (vja == 0) & (vjb == 0), (vja == n) & (vjb == n))):
                for e in np.nonzero(hit)[0]:
                    tri.append(e)
                    side.append(sd)
                    p1n.append((m.p1[e, a], m.p1[e, b]))
                    if m.order_u == 1:
                        pun.append((m.pu[e, a], m.pu[e, b]))
                    else:
                        pun.append((m.pu[e, a], m.pu[e, b], m.pu[e, 3 + k]))
        self.bedge_tri = np.array(tri, dtype=np.int64)
        self.bedge_side = np.array(side, dtype=np.int64)
        self.bedge_p1 = np.array(p1n, dtype=np.int64).reshape(-1, 2)
        self.bedge_pu = np.array(pun, dtype=np.int64).reshape(-1, 2 if m.order_u == 1 else 3)

    def _raw_loads(self, t: float):
        """Load vectors of a RAW load at time t (caller data on the lattices, taken as
        the nodal interpolants in the finite element spaces):
          F_u = (f_h, theta_i) + <t_h, theta_i> on the sides without u Dirichlet data,
          Z   = (z_h, phi_i) + <z_w,h, phi_i> on the poroelastic edges of the sides without
                p Dirichlet data,
        the boundary terms of eqs. (vf1), (vf3), (vf4).  Returns (f over the u blocks, Z
        over the p nodes)."""
        w, m, b = self.w, self.mesh, self.blocks
        o = b.offsets
        raw = raw_arrays(w, t)
        f = np.zeros(self.ndof)
        for tri, ud, key in ((self.triP, self._udP, 'f_p'), (self.triE, self._udE, 'f_e')):
            M = mass(w.order_u, m.X[tri])
            nodes = m.pu[tri]
            blk = o['uP'] if key == 'f_p' else o['uE']
            for c in range(2):
                Fc = np.einsum('eij,ej->ei', M, raw[key][c][nodes])
                np.add.at(f, blk + ud[:, c::2].ravel(), Fc.ravel())
        Z = np.zeros(b.sizes['p'])
        R = mass(1, m.X[self.triP])
        np.add.at(Z, self._sidxP.ravel(), np.einsum('eij,ej->ei', R, raw['z'][m.p1[self.triP]]).ravel())
        h = m.h
        Mu = edge_mass(w.order_u, h)
        M1 = edge_mass(1, h)
        for e, sd, pn, un in zip(self.bedge_tri, self.bedge_side, self.bedge_p1, self.bedge_pu):
            poro = bool(m.tri_poro[e])
            along_u = (un // m.mu) if sd < 2 else (un % m.mu)
            along_1 = (pn // (m.n + 1)) if sd < 2 else (pn % (m.n + 1))
            if not (w.dirichlet_u >> sd) & 1:
                mp = self.mapuP if poro else self.mapuE
                blk = o['uP'] if poro else o['uE']
                for c in range(2):
                    np.add.at(f, blk + 2 * mp[un] + c, Mu @ raw['t_side'][0 if poro else 1, sd, c, along_u])
            if poro and not (w.dirichlet_p >> sd) & 1:
                np.add.at(Z, self.mapsP[pn], M1 @ raw['zw_side'][sd, along_1])
        return f, Z

    # ------------------------------------------------------------------
    def _assemble(self):
        w, m, b = self.w, self.mesh, self.blocks
        rows, cols, vals = [], [], []
        o = b.offsets
        nloc = 3 if w.order_u == 1 else 6
        # poroelastic region ------------------------------------------------
        XP = m.X[self.triP]
        emP = element_matrices(w.order_u, XP, self.muP, w.mat_p.K / w.mat_p.mu_f)
        uidx = self.mapuP[m.pu[self.triP]]                      # (E, nloc)
        ud = np.empty((len(self.triP), 2 * nloc), dtype=np.int64)
        ud[:, 0::2] = 2 * uidx
        ud[:, 1::2] = 2 * uidx + 1
        sidx = self.mapsP[m.p1[self.triP]]                       # (E, 3)
        def blk(rb, ri, cb, ci, M, scale=1.0):
            R = o[rb] + ri[:, :, None] + 0 * ci[:, None, :]
            C = o[cb] + ci[:, None, :] + 0 * ri[:, :, None]
            _coo_add(rows, cols, vals, R, C, scale * M)
        k1, k2, k3, tau = self.k1, self.k2, self.k3, w.tau
        blk('uP', ud, 'uP', ud, emP['A'])
        blk('uP', ud, 'xiP', sidx, np.transpose(emP['B'], (0, 2, 1)))
        blk('xiP', sidx, 'uP', ud, emP['B'])
        blk('xiP', sidx, 'xiP', sidx, emP['R'], -k3)
        blk('xiP', sidx, 'eta', sidx, emP['R'], k1)
        blk('eta', sidx, 'xiP', sidx, emP['R'], k1)
        blk('eta', sidx, 'eta', sidx, emP['R'], k2)
        blk('eta', sidx, 'p', sidx, emP['R'], -1.0)
        if self.lumped_storage:
            lumpR = np.zeros_like(emP['R'])
            idx = np.arange(emP['R'].shape[1])
            lumpR[:, idx, idx] = emP['R'].sum(axis=2)
            blk('p', sidx, 'eta', sidx, lumpR, -1.0)
        else:
            blk('p', sidx, 'eta', sidx, emP['R'], -1.0)
        blk('p', sidx, 'p', sidx, emP['Af'], -tau)
        # elastic region ----------------------------------------------------
        XE = m.X[self.triE]
        emE = element_matrices(w.order_u, XE, self.muE, 1.0)
        uidx = self.mapuE[m.pu[self.triE]]
        udE = np.empty((len(self.triE), 2 * nloc), dtype=np.int64)
        udE[:, 0::2] = 2 * uidx
        udE[:, 1::2] = 2 * uidx + 1
        sidxE = self.mapsE[m.p1[self.triE]]
        blk('uE', udE, 'uE', udE, emE['A'])
        blk('uE', udE, 'xiE', sidxE, np.transpose(emE['B'], (0, 2, 1)))
        blk('xiE', sidxE, 'uE', udE, emE['B'])
        blk('xiE', sidxE, 'xiE', sidxE, emE['R'], -1.0 / self.lamE)
        # interface gluing (Boolean H) --------------------------------------
        nl = b.sizes['lam']
        lam_rows = o['lam'] + np.arange(nl)
        pcol = o['uP'] + 2 * self.mapuP[b.node['lam']] + b.comp['lam']
        ecol = o['uE'] + 2 * self.mapuE[b.node['lam']] + b.comp['lam']
        one = np.ones(nl)
        for R, C, V in ((lam_rows, pcol, one), (pcol, lam_rows, one),
                        (lam_rows, ecol, -one), (ecol, lam_rows, -one)):
            _coo_add(rows, cols, vals, R, C, V)
        K = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(self.ndof, self.ndof)).tocsr()
        K.sum_duplicates()
        self.K = K
        self.Kff = K[self.free][:, self.free].tocsc()
        self.KfD = K[self.free][:, self.dir].tocsr()
        # pieces for the right-hand side
        self._udP, self._sidxP, self._udE = ud, sidx, udE
        self.RP = K[o['eta']:o['eta'] + b.sizes['eta'], o['p']:o['p'] + b.sizes['p']] * -1.0
        # R_P as (p rows) x (eta cols) is the same matrix (symmetric); the storage term of
        # row 4 (R_P, or its lumped form)
        self.R4 = self.RP
        if self.lumped_storage:
            self.R4 = (K[o['p']:o['p'] + b.sizes['p'], o['eta']:o['eta'] + b.sizes['eta']] * -1.0).T.tocsr()

    # ------------------------------------------------------------------
    def rhs(self, t: float, eta_prev: np.ndarray) -> np.ndarray:
        """Full right-hand side of eq. (linalg-system) at time t (all DOFs)."""
        w, m, b, L = self.w, self.mesh, self.blocks, self.loads
        o = b.offsets
        if w.load.kind == RAW:
            f, Z = self._raw_loads(t)
            f[o['p']:o['p'] + b.sizes['p']] = -(self.R4.T @ eta_prev) - w.tau * Z
            return f
        f = np.zeros(self.ndof)
        FuP, ZP = load_vectors(w.order_u, m.X[self.triP], L.fPx, L.fPy, L.z, t)
        np.add.at(f, o['uP'] + self._udP.ravel(), FuP.ravel())
        FuE, _ = load_vectors(w.order_u, m.X[self.triE], L.fEx, L.fEy, L.z, t)
        np.add.at(f, o['uE'] + self._udE.ravel(), FuE.ravel())
        Z = np.zeros(b.sizes['p'])
        np.add.at(Z, self._sidxP.ravel(), ZP.ravel())
        # row 4: -R_P eta^{n-1} - tau Z^n   (R_P symmetric, rows = p test nodes)
        f[o['p']:o['p'] + b.sizes['p']] = -(self.R4.T @ eta_prev) - w.tau * Z
        return f

    def dirichlet_values(self, t: float) -> np.ndarray:
        """Nodal Dirichlet values at time t for every Dirichlet DOF."""
        b, m, L = self.blocks, self.mesh, self.loads
        vals = np.zeros(self.ndof)
        if self.w.load.kind == RAW:
            raw = raw_arrays(self.w, t)
            for nm in ('uP', 'uE'):
                o, n = b.offsets[nm], b.sizes[nm]
                vals[o:o + n] = raw['g_u'][b.comp[nm], b.node[nm]]
            o, n = b.offsets['p'], b.sizes['p']
            vals[o:o + n] = raw['g_p'][b.node['p']]
            return vals[self.dir]
        for nm, fx, fy in (('uP', L.u0x_P if L.uPx is None else L.uPx,
                            L.u0y_P if L.uPy is None else L.uPy),
                           ('uE', L.u0x_E if L.uEx is None else L.uEx,
                            L.u0y_E if L.uEy is None else L.uEy)):
            o, n = b.offsets[nm], b.sizes[nm]
            xy = m.pu_xy(b.node[nm])
            c = b.comp[nm]
            vx = fx(xy[:, 0], xy[:, 1], t)
            vy = fy(xy[:, 0], xy[:, 1], t)
            vals[o:o + n] = np.where(c == 0, vx, vy)
        o, n = b.offsets['p'], b.sizes['p']
        xy = m.p1_xy(b.node['p'])
        pf = L.p0 if L.p is None else L.p
        vals[o:o + n] = pf(xy[:, 0], xy[:, 1], t)
        return vals[self.dir]

    def initial_eta(self, mode: str = "interp") -> np.ndarray:
        """Discrete initial fluid content eta_h^0 (the "projection" of Problem 3).

        mode "interp": nodal interpolant of eta_0 = c0 p0 + alpha div u0 (the
        sign of eq. (mreform)).  mode "steady": eta-component of the discrete
        stationary problem at t = 0 (row 4 replaced by -tau A_f p = -tau Z),
        which is the discretely consistent start for a stationary solution.
        """
        b, m, L = self.blocks, self.mesh, self.loads
        if self.w.load.kind == RAW:
            return raw_arrays(self.w, 0.0)['eta0'][b.node['eta']].copy()
        if mode == "interp":
            xy = m.p1_xy(b.node['eta'])
            return L.eta0(xy[:, 0], xy[:, 1], 0.0)
        if mode != "steady":
            raise ValueError(mode)
        o = b.offsets
        K = self.K.tolil(copy=True)
        pr = slice(o['p'], o['p'] + b.sizes['p'])
        er = slice(o['eta'], o['eta'] + b.sizes['eta'])
        K[pr, er] = 0.0
        K = K.tocsr()
        f = self.rhs(0.0, np.zeros(b.sizes['eta']))
        xD = self.dirichlet_values(0.0)
        Kff = K[self.free][:, self.free].tocsc()
        KfD = K[self.free][:, self.dir]
        x = np.zeros(self.ndof)
        x[self.free] = spla.spsolve(Kff, f[self.free] - KfD @ xD)
        return x[er].copy()

    # ------------------------------------------------------------------
    def factor(self):
        t0 = time.perf_counter()
        self.lu = spla.splu(self.Kff)
        self.t_factor = time.perf_counter() - t0
        return self.lu

    def _residual_ext(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        """b - K_ff x accumulated in x87 extended precision (numpy longdouble)."""
        K = self.Kff_csr
        prod = self._Kdata_ext * x.astype(np.longdouble)[K.indices]
        nz = np.diff(K.indptr) > 0
        y = np.zeros(K.shape[0], dtype=np.longdouble)
        y[nz] = np.add.reduceat(prod, K.indptr[:-1][nz])
        return (b.astype(np.longdouble) - y).astype(np.float64)

    def solve_step(self, t: float, eta_prev: np.ndarray, refine: int = 2) -> np.ndarray:
        """One backward-Euler step; returns the full DOF vector (Dirichlet included).

        The fields differ by up to ~12 orders of magnitude (xi ~ lambda div u
        against u), so one FP64 LU solve leaves relative errors up to ~1e-7 in
        the small fields.  Classical iterative refinement with the residual
        accumulated in extended precision removes them.
        """
        f = self.rhs(t, eta_prev)
        xD = self.dirichlet_values(t)
        rhs = f[self.free] - self.KfD @ xD
        xf = self.lu.solve(rhs)
        if refine:
            if not hasattr(self, 'Kff_csr'):
                self.Kff_csr = self.Kff.tocsr()
                self._Kdata_ext = self.Kff_csr.data.astype(np.longdouble)
            for _ in range(refine):
                xf = xf + self.lu.solve(self._residual_ext(rhs, xf))
        x = np.zeros(self.ndof)
        x[self.free] = xf
        x[self.dir] = xD
        return x

    def split(self, x: np.ndarray) -> Dict[str, np.ndarray]:
        b = self.blocks
        return {nm: x[b.offsets[nm]:b.offsets[nm] + b.sizes[nm]] for nm in b.names}

    # ------------------------------------------------------------------
    def to_lattice(self, x: np.ndarray) -> Dict[str, np.ndarray]:
        """Fields on the global lattices (NaN where a field is not defined).

        ux_P, uy_P, ux_E, uy_E on the displacement lattice; xiP, eta, p, xiE on
        the P1 lattice.
        """
        m, b = self.mesh, self.blocks
        s = self.split(x)
        out = {}
        for nm in ('uP', 'uE'):
            for c, cn in ((0, 'ux'), (1, 'uy')):
                a = np.full(m.nu_lat, np.nan)
                sel = b.comp[nm] == c
                a[b.node[nm][sel]] = s[nm][sel]
                out[f"{cn}_{nm[1]}"] = a
        for nm in ('xiP', 'eta', 'p', 'xiE'):
            a = np.full(m.n1, np.nan)
            a[b.node[nm]] = s[nm]
            out[nm] = a
        return out

    def errors(self, x: np.ndarray, t: float):
        """L2 errors of u over the whole domain and of p over the poro region."""
        m, b, L = self.mesh, self.blocks, self.loads
        s = self.split(x)
        eu2 = 0.0
        for nm, tri, mp, fx, fy in (('uP', self.triP, self.mapuP, L.uPx, L.uPy),
                                    ('uE', self.triE, self.mapuE, L.uEx, L.uEy)):
            idx = mp[m.pu[tri]]
            X = m.X[tri]
            for c, fe in ((0, fx), (1, fy)):
                eu2 += interpolate_l2_error(self.w.order_u, X, s[nm][2 * idx + c], fe, t)
        idx = self.mapsP[m.p1[self.triP]]
        ep2 = interpolate_l2_error(1, m.X[self.triP], s['p'][idx], L.p, t)
        return float(np.sqrt(eu2)), float(np.sqrt(ep2))


@dataclass
class Trajectory:
    system: MonolithicSystem
    states: List[np.ndarray]
    times: List[float]
    t_step: float = 0.0


def solve_steps(w: Workload, nsteps: Optional[int] = None, keep: bool = True,
                eta0: Optional[np.ndarray] = None, init: str = "interp",
                lumped_storage: bool = False) -> Trajectory:
    """Run ``nsteps`` backward-Euler steps of eq. (linalg-system) from t=0."""
    S = MonolithicSystem(w, lumped_storage=lumped_storage)
    S.factor()
    n = w.nsteps if nsteps is None else nsteps
    eta = S.initial_eta(init) if eta0 is None else eta0
    b = S.blocks
    states, times = [], []
    t0 = time.perf_counter()
    for k in range(1, n + 1):
        t = k * w.tau
        x = S.solve_step(t, eta)
        eta = x[b.offsets['eta']:b.offsets['eta'] + b.sizes['eta']].copy()
        if keep or k == n:
            states.append(x)
            times.append(t)
    tr = Trajectory(S, states, times)
    tr.t_step = (time.perf_counter() - t0) / max(n, 1)
    return tr


def linf_l2_errors(tr: Trajectory):
    """max over the kept steps of the L2 errors of u and p (the L-inf(L2) norm of Section 4)."""
    eu = ep = 0.0
    for x, t in zip(tr.states, tr.times):
        a, c = tr.system.errors(x, t)
        eu = max(eu, a)
        ep = max(ep, c)
    return eu, ep
