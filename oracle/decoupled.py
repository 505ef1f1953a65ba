"""Decoupled mass balance: the explicit time discretisation of the fluid equations that the
Remark after eq. (linalg-system) (Section 2.5) proposes against the poroelastic/elastic
load imbalance.

Oracle module (test infrastructure only).

The coupled step of eq. (linalg-system) solves for (u_P, xi_P, eta, p, u_E, xi_E,
lambda) at once.  Here a step n takes the fluid content explicitly and then solves the
momentum balance alone, so that a poroelastic subdomain carries only (u_P, xi_P) like an
elastic one carries (u_E, xi_E):

  (1) mass balance (row 4 of eq. (linalg-system)) with the mass matrix lumped (row sums
      m_i of R_P) and the pressure taken from the previous step:
          m_i (eta^n_i - eta^{n-1}_i) = tau (Z^n - A_f p^{n-1})_i
      at every poroelastic node i without pressure Dirichlet data; at a pressure
      Dirichlet node the relation of row 3 with the previous xi,
          eta^n_i = (p_D(t_n)_i - k1 xi^{n-1}_i) / k2;
  (2) momentum balance: rows 1, 2, 5, 6, 7 of eq. (linalg-system) for (u_P, xi_P, u_E,
      xi_E, lambda) with eta^n known (the term k1 R_P eta^n of row 2 moves to the
      right-hand side);
  (3) pressure: xi, eta and p lie in the same P1 space, so row 3 is the nodal identity
      p^n = k1 xi^n + k2 eta^n; p^n = p_D(t_n) at the pressure Dirichlet nodes.

Step (1) is explicit Euler on the semi-discrete system whose storage term uses the lumped
mass, so the scheme converges at first order in tau to the backward-Euler scheme of that
system (``MonolithicSystem(lumped_storage=True)``); it shares the coupled scheme's discrete
stationary states.  Two stability limits follow from the explicit steps: tau below the
explicit diffusion limit of the consolidation operator (~ h^2 / (4 c_v), c_v = (K / mu_f) /
(c0 + alpha^2 / (lambda + 2 mu))), and, at the pressure Dirichlet nodes, a per-step
amplification of about -k1^2 / (k2 k3) = -alpha^2 / (c0 lambda) (xi responds to eta through
row 2), so alpha^2 < c0 lambda: met by the nearly incompressible cases (c0 lambda ~ 1.7e5),
not by alpha = c0 = 1 at nu = 0.3.  Parity of the GPU path is against this module; this
module is pinned against the coupled oracle (stationary and patch solutions, the momentum
step with the coupled eta, first-order convergence in tau) and against closed forms.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List

import numpy as np
import scipy.sparse.linalg as spla

from workloads import Workload
from .monolithic import MonolithicSystem


@dataclass
class DecoupledState:
    """Fluid state carried between steps, on the poroelastic P1 nodes (the 'eta' / 'p'
    block order of the monolithic system)."""
    eta: np.ndarray
    p: np.ndarray
    xi: np.ndarray


class DecoupledSystem:
    """The decoupled step on the assembled blocks of the monolithic system."""

    def __init__(self, w: Workload):
        self.S = S = MonolithicSystem(w)
        self.w = w
        b = S.blocks
        o, n = b.offsets, b.sizes
        self.ieta = np.arange(o['eta'], o['eta'] + n['eta'])
        self.ip = np.arange(o['p'], o['p'] + n['p'])
        self.ixi = np.arange(o['xiP'], o['xiP'] + n['xiP'])
        known = np.zeros(S.ndof, dtype=bool)
        known[S.dir] = True
        known[self.ieta] = True
        known[self.ip] = True
        self.mf = np.nonzero(~known)[0]    # momentum unknowns
        self.kn = np.nonzero(known)[0]
        K = S.K.tocsr()
        self.Kmm = K[self.mf][:, self.mf].tocsc()
        self.Kmk = K[self.mf][:, self.kn].tocsr()
        self.lu = spla.splu(self.Kmm)
        self.Kmm_csr = self.Kmm.tocsr()
        self._ext = self.Kmm_csr.data.astype(np.longdouble)
        # lumped mass (row sums of R_P) and the fluid stiffness A_f (the p-p block is -tau A_f)
        self.mL = np.asarray(S.RP.sum(axis=1)).ravel()
        self.Af = (K[self.ip][:, self.ip] * (-1.0 / w.tau)).tocsr()
        # pressure Dirichlet nodes within the p block
        self.pdir = S.dmask[self.ip]
        self.k1, self.k2 = S.k1, S.k2

    # ------------------------------------------------------------------
    def initial_state(self) -> DecoupledState:
        """eta^0 as the coupled oracle takes it (nodal interpolant, R14), p^0 the nodal
        interpolant of the initial pressure (the Dirichlet values where they apply), xi^0
        from row 3: xi = (p - k2 eta) / k1."""
        S, b, m, L = self.S, self.S.blocks, self.S.mesh, self.S.loads
        eta = S.initial_eta("interp")
        xy = m.p1_xy(b.node['p'])
        p = L.p0(xy[:, 0], xy[:, 1], 0.0) if L.p0 is not None else np.zeros(len(xy))
        p = np.asarray(p, dtype=np.float64).copy()
        xi = (p - self.k2 * eta) / self.k1
        return DecoupledState(eta=eta, p=p, xi=xi)

    def pressure_dirichlet(self, t: float) -> np.ndarray:
        """p_D(t) on the p block (zero where the pressure is free)."""
        S = self.S
        full = np.zeros(S.ndof)
        full[S.dir] = S.dirichlet_values(t)
        return full[self.ip]

    def mass_balance(self, t: float, st: DecoupledState) -> np.ndarray:
        """Step (1): eta^n from eta^{n-1}, p^{n-1}, xi^{n-1}."""
        S, w = self.S, self.w
        f = S.rhs(t, st.eta)
        # row 4 of the coupled right-hand side is -R_P eta^{n-1} - tau Z^n
        tauZ = -f[self.ip] - S.RP.T @ st.eta
        eta = st.eta + (tauZ - w.tau * (self.Af @ st.p)) / self.mL
        pD = self.pressure_dirichlet(t)
        eta[self.pdir] = (pD[self.pdir] - self.k1 * st.xi[self.pdir]) / self.k2
        return eta

    def momentum(self, t: float, eta: np.ndarray, refine: int = 2) -> np.ndarray:
        """Step (2): the full DOF vector with the momentum unknowns solved for the given
        eta (eta and p blocks hold eta and zero; p does not enter rows 1, 2, 5, 6, 7)."""
        S = self.S
        x = np.zeros(S.ndof)
        x[S.dir] = S.dirichlet_values(t)
        x[self.ieta] = eta
        x[self.ip] = 0.0
        f = S.rhs(t, np.zeros_like(eta))  # rows 1, 2, 5, 6, 7 do not depend on eta^{n-1}
        rhs = f[self.mf] - self.Kmk @ x[self.kn]
        xm = self.lu.solve(rhs)
        for _ in range(refine):
            Kc = self.Kmm_csr
            prod = self._ext * xm.astype(np.longdouble)[Kc.indices]
            nz = np.diff(Kc.indptr) > 0
            y = np.zeros(Kc.shape[0], dtype=np.longdouble)
            y[nz] = np.add.reduceat(prod, Kc.indptr[:-1][nz])
            r = (rhs.astype(np.longdouble) - y).astype(np.float64)
            xm = xm + self.lu.solve(r)
        x[self.mf] = xm
        return x

    def step(self, t: float, st: DecoupledState):
        """One decoupled step at time t; returns (full DOF vector, new state)."""
        eta = self.mass_balance(t, st)
        x = self.momentum(t, eta)
        xi = x[self.ixi].copy()
        p = self.k1 * xi + self.k2 * eta
        pD = self.pressure_dirichlet(t)
        p[self.pdir] = pD[self.pdir]
        x[self.ip] = p
        return x, DecoupledState(eta=eta.copy(), p=p.copy(), xi=xi)


@dataclass
class DecoupledTrajectory:
    system: DecoupledSystem
    states: List[np.ndarray]
    times: List[float]


def solve_steps(w: Workload, nsteps: int = None, state: DecoupledState = None) -> DecoupledTrajectory:
    """Run the decoupled scheme for nsteps from t = 0 (or from a given state)."""
    D = DecoupledSystem(w)
    st = D.initial_state() if state is None else state
    n = w.nsteps if nsteps is None else nsteps
    xs, ts = [], []
    for k in range(1, n + 1):
        t = k * w.tau
        x, st = D.step(t, st)
        xs.append(x)
        ts.append(t)
    return DecoupledTrajectory(D, xs, ts)


def fields(D: DecoupledSystem, x: np.ndarray) -> Dict[str, np.ndarray]:
    """The fields of a full DOF vector on the global lattices (as the coupled oracle)."""
    return D.S.to_lattice(x)
