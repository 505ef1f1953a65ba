"""Monolithic FP64 solve of the fully discrete coupled problem on the unit cube (d = 3).

Oracle module (test infrastructure only).

The same block system as ``oracle.monolithic`` (eq. (linalg-system) of Section 2.5, with
the displacement in three components), assembled from the tetrahedral element matrices
of ``oracle.fem3d`` on the Kuhn mesh, poroelastic for x < 1/2 and elastic for x > 1/2,
multipliers nodal on the interface nodes without Dirichlet data.  Loads are nodal data
(load kind RAW): the body forces, the source, the Dirichlet values and eta^0 on the
lattices, entering as their finite element interpolants, F_u = (f_h, theta) and
Z = (z_h, phi) (no boundary flux or traction data in 3D).  The matrix is factorised once
with SuperLU; each step is refined twice with residuals in extended precision.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from workloads import Workload, RAW, raw_arrays
from .fem3d import Mesh3D, element_matrices
from .monolithic import Blocks
from .problem import lame, kappas


class MonolithicSystem3D:
    def __init__(self, w: Workload):
        if w.dim != 3 or w.load.kind != RAW:
            raise ValueError("the 3D oracle takes 3D workloads with nodal (RAW) loads")
        self.w = w
        self.mesh = m = Mesh3D(w.ncell, w.order_u)
        lamP, muP = lame(w.mat_p)
        lamE, muE = lame(w.mat_e)
        self.lamP, self.muP, self.lamE, self.muE = lamP, muP, lamE, muE
        self.k1, self.k2, self.k3 = kappas(w.mat_p)
        P = m.tet_poro
        self.tetP = np.nonzero(P)[0]
        self.tetE = np.nonzero(~P)[0]
        uP_nodes = np.unique(m.pu[P])
        uE_nodes = np.unique(m.pu[~P])
        sP_nodes = np.unique(m.p1[P])
        sE_nodes = np.unique(m.p1[~P])
        gam = np.intersect1d(uP_nodes, uE_nodes)
        dirU = m.on_faces_pu(np.arange(m.nu_lat), w.dirichlet_u)
        dirP = m.on_faces_p1(np.arange(m.n1_lat), w.dirichlet_p)
        lam_nodes = gam[~dirU[gam]]

        def vec(nodes):
            return np.repeat(nodes, 3), np.tile([0, 1, 2], len(nodes))
        node, comp = {}, {}
        node['uP'], comp['uP'] = vec(uP_nodes)
        for nm, nd in (('xiP', sP_nodes), ('eta', sP_nodes), ('p', sP_nodes), ('xiE', sE_nodes)):
            node[nm], comp[nm] = nd, np.zeros(len(nd), int)
        node['uE'], comp['uE'] = vec(uE_nodes)
        node['lam'], comp['lam'] = vec(lam_nodes)
        names = ['uP', 'xiP', 'eta', 'p', 'uE', 'xiE', 'lam']
        offs, sizes, o = {}, {}, 0
        for nm in names:
            offs[nm] = o
            sizes[nm] = len(node[nm])
            o += sizes[nm]
        self.blocks = Blocks(names, offs, sizes, node, comp)
        self.ndof = o

        def pos_map(nodes, nlat):
            mp = -np.ones(nlat, dtype=np.int64)
            mp[nodes] = np.arange(len(nodes))
            return mp
        self.mapuP = pos_map(uP_nodes, m.nu_lat)
        self.mapuE = pos_map(uE_nodes, m.nu_lat)
        self.mapsP = pos_map(sP_nodes, m.n1_lat)
        self.mapsE = pos_map(sE_nodes, m.n1_lat)
        dmask = np.zeros(self.ndof, dtype=bool)
        dmask[offs['uP']:offs['uP'] + sizes['uP']] = dirU[node['uP']]
        dmask[offs['uE']:offs['uE'] + sizes['uE']] = dirU[node['uE']]
        dmask[offs['p']:offs['p'] + sizes['p']] = dirP[node['p']]
        self.dmask = dmask
        self.free = np.nonzero(~dmask)[0]
        self.dir = np.nonzero(dmask)[0]
        self._assemble()

    def _assemble(self):
        w, m, b = self.w, self.mesh, self.blocks
        o = b.offsets
        rows, cols, vals = [], [], []

        def blk(rb, ri, cb, ci, M, scale=1.0):
            R = o[rb] + np.broadcast_to(ri[:, :, None], M.shape)
            C = o[cb] + np.broadcast_to(ci[:, None, :], M.shape)
            rows.append(R.ravel())
            cols.append(C.ravel())
            vals.append((scale * M).ravel())

        def udofs(mp, tets):
            idx = mp[m.pu[tets]]
            ud = np.empty((len(tets), 3 * idx.shape[1]), dtype=np.int64)
            for c in range(3):
                ud[:, c::3] = 3 * idx + c
            return ud
        emP = element_matrices(w.order_u, m.X[self.tetP], self.muP, w.mat_p.K / w.mat_p.mu_f)
        ud = udofs(self.mapuP, self.tetP)
        sidx = self.mapsP[m.p1[self.tetP]]
        k1, k2, k3, tau = self.k1, self.k2, self.k3, w.tau
        blk('uP', ud, 'uP', ud, emP['A'])
        blk('uP', ud, 'xiP', sidx, np.transpose(emP['B'], (0, 2, 1)))
        blk('xiP', sidx, 'uP', ud, emP['B'])
        blk('xiP', sidx, 'xiP', sidx, emP['R'], -k3)
        blk('xiP', sidx, 'eta', sidx, emP['R'], k1)
        blk('eta', sidx, 'xiP', sidx, emP['R'], k1)
        blk('eta', sidx, 'eta', sidx, emP['R'], k2)
        blk('eta', sidx, 'p', sidx, emP['R'], -1.0)
        blk('p', sidx, 'eta', sidx, emP['R'], -1.0)
        blk('p', sidx, 'p', sidx, emP['Af'], -tau)
        emE = element_matrices(w.order_u, m.X[self.tetE], self.muE, 1.0)
        udE = udofs(self.mapuE, self.tetE)
        sidxE = self.mapsE[m.p1[self.tetE]]
        blk('uE', udE, 'uE', udE, emE['A'])
        blk('uE', udE, 'xiE', sidxE, np.transpose(emE['B'], (0, 2, 1)))
        blk('xiE', sidxE, 'uE', udE, emE['B'])
        blk('xiE', sidxE, 'xiE', sidxE, emE['R'], -1.0 / self.lamE)
        nl = b.sizes['lam']
        lr = o['lam'] + np.arange(nl)
        pc = o['uP'] + 3 * self.mapuP[b.node['lam']] + b.comp['lam']
        ec = o['uE'] + 3 * self.mapuE[b.node['lam']] + b.comp['lam']
        one = np.ones(nl)
        for R, C, V in ((lr, pc, one), (pc, lr, one), (lr, ec, -one), (ec, lr, -one)):
            rows.append(R)
            cols.append(C)
            vals.append(V)
        K = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(self.ndof, self.ndof)).tocsr()
        K.sum_duplicates()
        self.K = K
        self.Kff = K[self.free][:, self.free].tocsc()
        self.KfD = K[self.free][:, self.dir].tocsr()
        self._ud, self._udE, self._sidx = ud, udE, sidx
        self._MP, self._ME, self._RP = emP['M'], emE['M'], emP['R']
        self.RP = K[o['eta']:o['eta'] + b.sizes['eta'], o['p']:o['p'] + b.sizes['p']] * -1.0

    # ------------------------------------------------------------------
    def rhs(self, t: float, eta_prev: np.ndarray) -> np.ndarray:
        """Right-hand side of eq. (linalg-system) at time t: F_u = (f_h, theta) per region,
        row 4 = -R_P eta^{n-1} - tau Z^n with Z = (z_h, phi)."""
        w, m, b = self.w, self.mesh, self.blocks
        o = b.offsets
        raw = raw_arrays(w, t)
        f = np.zeros(self.ndof)
        for tets, ud, M, key, blk in ((self.tetP, self._ud, self._MP, 'f_p', 'uP'),
                                      (self.tetE, self._udE, self._ME, 'f_e', 'uE')):
            nodes = m.pu[tets]
            for c in range(3):
                Fc = np.einsum('eij,ej->ei', M, raw[key][c][nodes])
                np.add.at(f, o[blk] + ud[:, c::3].ravel(), Fc.ravel())
        Z = np.zeros(b.sizes['p'])
        np.add.at(Z, self._sidx.ravel(), np.einsum('eij,ej->ei', self._RP, raw['z'][m.p1[self.tetP]]).ravel())
        f[o['p']:o['p'] + b.sizes['p']] = -(self.RP.T @ eta_prev) - w.tau * Z
        return f

    def dirichlet_values(self, t: float) -> np.ndarray:
        b = self.blocks
        raw = raw_arrays(self.w, t)
        vals = np.zeros(self.ndof)
        for nm in ('uP', 'uE'):
            o, n = b.offsets[nm], b.sizes[nm]
            vals[o:o + n] = raw['g_u'][b.comp[nm], b.node[nm]]
        o, n = b.offsets['p'], b.sizes['p']
        vals[o:o + n] = raw['g_p'][b.node['p']]
        return vals[self.dir]

    def initial_eta(self) -> np.ndarray:
        return raw_arrays(self.w, 0.0)['eta0'][self.blocks.node['eta']].copy()

    def factor(self):
        self.lu = spla.splu(self.Kff)
        K = self.Kff.tocsr()
        self._Kc = K
        self._Kext = K.data.astype(np.longdouble)

    def _residual_ext(self, rhs, x):
        K = self._Kc
        prod = self._Kext * x.astype(np.longdouble)[K.indices]
        nz = np.diff(K.indptr) > 0
        y = np.zeros(K.shape[0], dtype=np.longdouble)
        y[nz] = np.add.reduceat(prod, K.indptr[:-1][nz])
        return (rhs.astype(np.longdouble) - y).astype(np.float64)

    def solve_step(self, t: float, eta_prev: np.ndarray, refine: int = 2) -> np.ndarray:
        f = self.rhs(t, eta_prev)
        xD = self.dirichlet_values(t)
        rhs = f[self.free] - self.KfD @ xD
        xf = self.lu.solve(rhs)
        for _ in range(refine):
            xf = xf + self.lu.solve(self._residual_ext(rhs, xf))
        x = np.zeros(self.ndof)
        x[self.free] = xf
        x[self.dir] = xD
        return x

    def split(self, x):
        b = self.blocks
        return {nm: x[b.offsets[nm]:b.offsets[nm] + b.sizes[nm]] for nm in b.names}

    def to_lattice(self, x) -> Dict[str, np.ndarray]:
        """ux_P, uy_P, uz_P, ux_E, uy_E, uz_E on the displacement lattice; xiP, eta, p, xiE
        on the P1 lattice (NaN where a field is not defined)."""
        m, b = self.mesh, self.blocks
        s = self.split(x)
        out = {}
        for nm in ('uP', 'uE'):
            for c, cn in ((0, 'ux'), (1, 'uy'), (2, 'uz')):
                a = np.full(m.nu_lat, np.nan)
                sel = b.comp[nm] == c
                a[b.node[nm][sel]] = s[nm][sel]
                out[f"{cn}_{nm[1]}"] = a
        for nm in ('xiP', 'eta', 'p', 'xiE'):
            a = np.full(m.n1_lat, np.nan)
            a[b.node[nm]] = s[nm]
            out[nm] = a
        return out


@dataclass
class Trajectory3D:
    system: MonolithicSystem3D
    states: List[np.ndarray]
    times: List[float]


def solve_steps(w: Workload, nsteps: Optional[int] = None) -> Trajectory3D:
    S = MonolithicSystem3D(w)
    S.factor()
    n = w.nsteps if nsteps is None else nsteps
    eta = S.initial_eta()
    b = S.blocks
    states, times = [], []
    for k in range(1, n + 1):
        t = k * w.tau
        x = S.solve_step(t, eta)
        eta = x[b.offsets['eta']:b.offsets['eta'] + b.sizes['eta']].copy()
        states.append(x)
        times.append(t)
    return Trajectory3D(S, states, times)


def patch_data(w: Workload, G=None, u0=(0.01, -0.02, 0.015), p0=0.3, q=(0.0, 0.4, -0.25)):
    """Nodal data of a stationary solution that the P2-P1 spaces contain exactly (the same
    materials in both regions): u_P = G x + u0, p = p0 + q_y y + q_z z (no flux through
    x = 1/2), eta = c0 p + alpha div u_P, and in the elastic region u_E = u_P + w with
    w = (c p (x - 1/2), 0, 0), c = -alpha / (lambda + 2 mu), which keeps u continuous and
    balances the traction (2 mu eps(u) - xi I) n on x = 1/2.  Body forces from the
    momentum equations: f_P = alpha grad p, f_E = -(lambda + mu) c grad p; no source.
    Returns the arrays of a RAW load (the same at every t; P1 displacements need q = 0)."""
    if G is None:
        G = np.array([[0.02, -0.01, 0.03], [0.015, -0.025, 0.01], [-0.02, 0.005, 0.01]])
    lam, mu = lame(w.mat_p)
    alpha, c0 = w.mat_p.alpha, w.mat_p.c0
    cc = -alpha / (lam + 2 * mu)
    r = 1 if w.order_u == 1 else 2
    n = w.ncell
    mu_l, n1 = r * n + 1, n + 1
    I = np.arange(mu_l ** 3)
    xu = np.stack([I % mu_l, (I // mu_l) % mu_l, I // mu_l ** 2], axis=1) / float(r * n)
    J = np.arange(n1 ** 3)
    x1 = np.stack([J % n1, (J // n1) % n1, J // n1 ** 2], axis=1) / float(n)

    def pres(x):
        return p0 + q[1] * x[:, 1] + q[2] * x[:, 2]
    uP = xu @ np.asarray(G).T + np.asarray(u0)
    uE = uP.copy()
    uE[:, 0] += cc * pres(xu) * (xu[:, 0] - 0.5)
    g_u = np.where((xu[:, 0] <= 0.5)[:, None], uP, uE).T.copy()
    gp = np.array([0.0, q[1], q[2]])
    f_p = np.tile((alpha * gp)[:, None], (1, mu_l ** 3))
    f_e = np.tile((-(lam + mu) * cc * gp)[:, None], (1, mu_l ** 3))
    divu = np.trace(G)
    return {"f_p": f_p, "f_e": f_e, "z": np.zeros(n1 ** 3), "t_side": np.zeros(0), "zw_side": np.zeros(0),
            "g_u": g_u, "g_p": pres(x1), "eta0": c0 * pres(x1) + alpha * divu}


def patch_exact(w: Workload, data_kw=None):
    """The exact fields of patch_data on the lattices (for comparisons): the same names as
    MonolithicSystem3D.to_lattice, defined everywhere."""
    kw = data_kw or {}
    G = kw.get("G")
    if G is None:
        G = np.array([[0.02, -0.01, 0.03], [0.015, -0.025, 0.01], [-0.02, 0.005, 0.01]])
    u0 = np.asarray(kw.get("u0", (0.01, -0.02, 0.015)))
    p0 = kw.get("p0", 0.3)
    q = kw.get("q", (0.0, 0.4, -0.25))
    lam, mu = lame(w.mat_p)
    alpha, c0 = w.mat_p.alpha, w.mat_p.c0
    cc = -alpha / (lam + 2 * mu)
    r = 1 if w.order_u == 1 else 2
    n = w.ncell
    mu_l, n1 = r * n + 1, n + 1
    I = np.arange(mu_l ** 3)
    xu = np.stack([I % mu_l, (I // mu_l) % mu_l, I // mu_l ** 2], axis=1) / float(r * n)
    J = np.arange(n1 ** 3)
    x1 = np.stack([J % n1, (J // n1) % n1, J // n1 ** 2], axis=1) / float(n)
    pu = p0 + q[1] * xu[:, 1] + q[2] * xu[:, 2]
    p1 = p0 + q[1] * x1[:, 1] + q[2] * x1[:, 2]
    uP = xu @ G.T + u0
    uE = uP.copy()
    uE[:, 0] += cc * pu * (xu[:, 0] - 0.5)
    divu = np.trace(G)
    divuE1 = divu + cc * p1            # div u_E at the P1 nodes
    out = {}
    for c, cn in enumerate(("ux", "uy", "uz")):
        out[f"{cn}_P"] = uP[:, c]
        out[f"{cn}_E"] = uE[:, c]
    out["p"] = p1
    out["eta"] = c0 * p1 + alpha * divu
    out["xiP"] = alpha * p1 - lam * divu
    out["xiE"] = -lam * divuE1
    return out
