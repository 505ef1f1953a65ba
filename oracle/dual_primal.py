"""Dual-primal gluing of the torn system (FETI-DP style), the SPD-safe variant of the
interface solve.

Oracle module (test infrastructure only).

Tearing a pressure-side field makes the FETI operator indefinite: the torn saddle-point
matrices carry negative-type unknowns (xi, p) whose multipliers turn into negative
eigenvalues of F = sum_s B_s K_s^+ B_s^T.  The Introduction points to BDDC / FETI-DP
preconditioners for three-field Biot; the dual-primal form used here keeps those fields
assembled instead of torn:

* primal unknowns (one global copy): every shared xi_P, p and xi_E DOF, and every shared
  DOF at a corner of the subdomain grid (these also pin the rigid-body modes, so no
  subdomain floats and no coarse projection is needed);
* dual unknowns (torn, glued by multipliers): the other shared DOFs, i.e. u and eta on
  the cut edges.

With K~ the partially assembled matrix (each subdomain's non-primal DOFs torn, the
primal DOFs summed over their owners) and B the signed Boolean rows of the dual DOFs,
the interface problem is F lambda = d with

    F = B K~^{-1} B^T,     d = B K~^{-1} f~,     u = K~^{-1} (f~ - B^T lambda).

The unknowns of positive type (u, eta) and negative type (xi, p) make K~ quasi-definite,
and B touches positive-type unknowns only, so F is a principal block of the inverse of
the positive Schur complement and is symmetric positive definite.

This module writes these definitions out with sparse direct solves (no blocking or
reordering): the partially assembled matrix, F, d, the dual-primal solution and the
primal coarse matrix S_PiPi = K~_PiPi - K~_Pir K~_rr^{-1} K~_rPi.  Its pins: the
solution equals the monolithic one, F is SPD while the dual gluing's F is not, and the
coarse matrix is quasi-definite in the global primal order.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import Workload
from .local import LocalSystem, build_local


class DualPrimal:
    """The partially assembled system of a workload with coupling == "primal"."""

    def __init__(self, w: Workload, L: LocalSystem = None):
        if w.coupling != "primal":
            raise ValueError("dual-primal gluing needs coupling='primal'")
        self.w = w
        self.L = L = build_local(w) if L is None else L
        spec = L.spec
        self.spec = spec
        self.npi = len(spec.primal)
        pidx = {int(c): k for k, c in enumerate(spec.primal)}
        # position of every local DOF in the unknowns of K~: the non-primal local DOFs of
        # all subdomains (subdomain-major, local order), then the primal DOFs
        loc = []
        off = 0
        for s in spec.subs:
            cats = np.asarray(s.cats)
            idx = np.full(len(s.codes), -1, dtype=np.int64)
            r = np.nonzero(cats != 3)[0]
            idx[r] = off + np.arange(len(r))
            off += len(r)
            loc.append(idx)
        self.nr = off
        for s, idx in zip(spec.subs, loc):
            for i, (c, cat) in enumerate(zip(s.codes, s.cats)):
                if cat == 3:
                    idx[i] = self.nr + pidx[int(c)]
        self.loc = loc
        self.n = self.nr + self.npi
        rows, cols, vals = [], [], []
        for idx, K in zip(loc, L.K):
            ii, jj = np.nonzero(K)
            rows.append(idx[ii])
            cols.append(idx[jj])
            vals.append(K[ii, jj])
        self.Kt = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(self.n, self.n))
        nl = spec.n_lambda
        br, bc, bv = [], [], []
        for j, r in enumerate(spec.rows):
            for s, li, sg in r:
                br.append(j)
                bc.append(loc[s][li])
                bv.append(float(sg))
        self.B = sp.csr_matrix((bv, (br, bc)), shape=(nl, self.n))
        self._lu = None

    # ------------------------------------------------------------------
    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.Kt)
        return self._lu

    def assemble(self, f_local: List[np.ndarray]) -> np.ndarray:
        """f~: the local right-hand sides with the primal rows summed over their owners."""
        ft = np.zeros(self.n)
        for idx, f in zip(self.loc, f_local):
            np.add.at(ft, idx, f)
        return ft

    def operator(self) -> np.ndarray:
        """F = B K~^{-1} B^T (dense, N_lambda x N_lambda)."""
        X = self.lu().solve(self.B.T.toarray())
        return self.B @ X

    def apply(self, lam: np.ndarray) -> np.ndarray:
        """F lambda."""
        return self.B @ self.lu().solve(self.B.T @ lam)

    def rhs(self, ft: np.ndarray) -> np.ndarray:
        """d = B K~^{-1} f~."""
        return self.B @ self.lu().solve(ft)

    def solve(self, f_local: List[np.ndarray]) -> Tuple[np.ndarray, List[np.ndarray]]:
        """lambda from F lambda = d (dense solve), then u = K~^{-1} (f~ - B^T lambda); the
        torn solution per subdomain (primal DOFs copied to every owner)."""
        ft = self.assemble(f_local)
        lam = np.linalg.solve(self.operator(), self.rhs(ft))
        u = self.lu().solve(ft - self.B.T @ lam)
        return lam, [u[idx] for idx in self.loc]

    def coarse_matrix(self) -> np.ndarray:
        """S_PiPi = K~_PiPi - K~_Pir K~_rr^{-1} K~_rPi (dense, global primal order)."""
        K = self.Kt.tocsr()
        r = np.arange(self.nr)
        pi = np.arange(self.nr, self.n)
        Krr = K[r][:, r].tocsc()
        Krp = K[r][:, pi].toarray()
        X = spla.splu(Krr).solve(Krp)
        return K[pi][:, pi].toarray() - Krp.T @ X

    def primal_kinds(self) -> np.ndarray:
        """DOF kind of every primal unknown (global primal order)."""
        return np.asarray(self.spec.primal) % 8
