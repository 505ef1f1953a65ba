"""Marshalling of a synthetic workload description into the C ABI structs."""
from __future__ import annotations

from typing import Dict, List

import numpy as np

from . import _binding as B

_LAYOUT = {"xsplit": B.XSPLIT, "ysplit": B.YSPLIT, "core": B.CORE}
_LOAD = {"manufactured": B.LOAD_MANUFACTURED, "periodic": B.LOAD_PERIODIC,
         "point_source": B.LOAD_POINT_SOURCE, "patch": B.LOAD_PATCH, "raw": B.LOAD_RAW}


def mesh_args(w) -> Dict:
    return dict(ncell=w.ncell, order_u=w.order_u, layout=_LAYOUT[w.layout], nsub_x=w.nsub_x,
                nsub_y=w.nsub_y, dirichlet_u=w.dirichlet_u, dirichlet_p=w.dirichlet_p,
                cut_x=getattr(w, "cut_x", None), cut_y=getattr(w, "cut_y", None),
                scheme=B.SCHEME_DECOUPLED if getattr(w, "scheme", "coupled") == "decoupled" else B.SCHEME_COUPLED,
                coupling=B.COUPLING_PRIMAL if getattr(w, "coupling", "dual") == "primal" else B.COUPLING_DUAL,
                dim=getattr(w, "dim", 2), nsub_z=getattr(w, "nsub_z", 1))


def material(m) -> B.Material:
    return B.Material(m.E, m.nu, m.alpha, m.c0, m.K, m.mu_f, m.lame_mode)


def load(w, t: float) -> B.Load:
    from workloads import PATCH_UX, PATCH_UY, PATCH_P
    L = B.Load()
    L.kind = _LOAD[w.load.kind]
    L.t = t
    prm: List[float] = [0.0] * 16
    if w.load.kind == "patch":
        nq = 6 if w.order_u == 2 else 3
        ux = list(PATCH_UX[:nq]) + [0.0] * (6 - nq)
        uy = list(PATCH_UY[:nq]) + [0.0] * (6 - nq)
        pp = [PATCH_P[0], PATCH_P[1] if w.order_u == 2 else 0.0]
        prm[:14] = ux + uy + pp
    elif w.load.kind == "periodic":
        prm[:3] = [w.load.amp, w.load.omega, w.load.phase]
    elif w.load.kind == "point_source":
        prm[:3] = [w.load.cx, w.load.cy, w.load.sigma]
    for i, v in enumerate(prm):
        L.params[i] = v
    if w.load.kind == "raw":
        import torch
        from workloads import raw_arrays
        arrs = raw_arrays(w, t)
        # (empty arrays: data the dimension has no place for, passed as NULL)
        L.attach_raw({k: torch.tensor(v.ravel(), dtype=torch.float64, device="cuda")
                      for k, v in arrs.items() if np.asarray(v).size > 0})
    return L


def opts(tol: float = 1e-10, max_it: int = 1000, start: int = B.START_PREVIOUS,
         check_every: int = 8, ir_max: int = 1, ir_cold: int = 4, tol_corr: float = 1e-3,
         ir_tol: float = 1e-9, tol_inner: float = 0.0, tol_upd: float = 3e-3,
         corr_start: int = B.CORR_PREVIOUS) -> B.SolveOpts:
    """Solve options.  Every step ends with FP64 iterative refinement on the torn
    system: up to ir_max corrections (ir_cold when the step starts without previous
    multipliers), stopping once a correction changes no field by more than ir_tol
    relative.  The pressure p = k1 xi + k2 eta is a small difference of large terms
    at nu -> 1/2, so an interface residual of tol alone does not bound its error.
    tol_inner: first-solve tolerance with FP32 factors (0 = tol).  tol_upd: update test of
    the refinement corrections (0 = off); corr_start: the first correction of a step
    starts from the previous step's total correction when that start has the smaller
    projected residual (CORR_PREVIOUS) or from zero (CORR_ZERO).  With both, the
    64-subdomain FP64 case needs ~38 instead of ~103 iterations per step and stays
    within 4e-10 of the oracle in every field over 16 steps."""
    return B.SolveOpts(tol, tol_corr, ir_tol, max_it, start, check_every, ir_max, ir_cold, tol_inner, tol_upd,
                       corr_start)


def opts_mixed(**kw) -> B.SolveOpts:
    """Defaults of the FP32-factor path: a looser first solve (its operators carry
    FP32 rounding) and more FP64 corrections, each to its residual tolerance (the
    corrections of this path are limited by the FP32 operators, and neither the update
    test nor the warm correction start shortened them)."""
    base = dict(tol_inner=1e-6, tol_corr=1e-4, ir_max=3, ir_cold=5, ir_tol=1e-9, tol_upd=0.0,
                corr_start=B.CORR_ZERO)
    base.update(kw)
    return opts(**base)


def setup(w, stream=None, precision=B.FP64, precond=B.PRECOND_DIRICHLET) -> B.Feti:
    """Create a context and run setup_mesh, assemble, factor_subdomains, init_state."""
    f = B.Feti(stream)
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.factor_subdomains(precision, precond)
    f.init_state(load(w, 0.0))
    return f
