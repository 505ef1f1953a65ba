"""Parity on paths that the other GPU tests do not reach.

* lambda itself against the oracle's multiplier on the two-subdomain case, where the
  nodal multipliers are unique (one row per interface node and component, +1 on the
  poroelastic copy as in the matrix of eq. (linalg-system));
* coarse spaces larger than the persistent kernel's in-block coarse solve (n_c = 588:
  16 x 16 subdomains around a poroelastic core), which take the dense (G^T G)^{-1} and
  the graph-captured iteration chain, in FP64 and with FP32 factors;
* the lumped preconditioner of Section 3.2 (Algorithm 2): the same solution as the
  Dirichlet preconditioner (both reach the monolithic solution, Theorem 3.1), with
  the iteration counts of both printed;
* the checkpoint state: ten steps equal five steps, get_state, set_state on a fresh
  context and five more steps, bit for bit;
* feti_solve between two steps leaves the trajectory unchanged, bit for bit;
* the field export against the oracle's lattice fields.
"""
import numpy as np
import pytest

import workloads as W
from feti_helpers import require_gpu, oracle_reference, torn_reference, per_kind_rel_error, sub_poro_flags

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts, opts_mixed  # noqa: E402

FP64_TOL = 1e-8
MIXED_TOL = 1e-6


def _run_and_compare(w, nsteps, f, o, tol, lats=None, label=""):
    import torch
    if lats is None:
        lats = oracle_reference(w, nsteps)[1]
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    its = []
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        assert st["status"] == 0, st
        f.get_solution(u)
        err = per_kind_rel_error(codes, u.cpu().numpy(), torn_reference(codes, idx["sub_offset"], poro, lats[n - 1]))
        print(f"  {label} step {n}: iters {st['iters']} (first {st['iters_first']}) err {max(err.values()):.1e}",
              flush=True)
        assert max(err.values()) < tol, (label, n, err)
        its.append(st["iters"])
    return its


def test_multipliers_match_the_oracle_lambda_on_two_subdomains():
    import torch
    require_gpu()
    w = W.plain_fp64_small()
    nsteps = 4
    tr_sys, lats = oracle_reference(w, nsteps)
    from oracle.monolithic import solve_steps
    tr = solve_steps(w, nsteps=nsteps)
    S = tr.system
    bl = S.blocks
    lam_ref = {}
    f = setup(w)
    idx = f.export_indexing()
    nl = f.get_sizes()["n_lambda"]
    assert nl == bl.sizes["lam"]
    rows = [(int(idx["code"][idx["sub_offset"][s] + l]), g)
            for s, l, g in zip(idx["brow_sub"][0::2], idx["brow_local"][0::2], idx["brow_sign"][0::2])]
    poro = sub_poro_flags(w)
    lam = torch.empty(nl, dtype=torch.float64, device="cuda")
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), opts(tol=w.tol, max_it=2000))
        assert st["status"] == 0, st
        f.get_solution(lam=lam)
        x = S.split(tr.states[n - 1])["lam"]
        for k, (node, comp) in enumerate(zip(bl.node["lam"], bl.comp["lam"])):
            lam_ref[8 * int(node) + int(comp)] = x[k]
        got = lam.cpu().numpy()
        # row j glues the DOF with this code; its first entry is the poroelastic copy with +1
        ref = np.array([lam_ref[c] for c, _ in rows])
        assert all(poro[s] for s in idx["brow_sub"][0::2]) and all(g == 1 for _, g in rows)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  step {n}: |lambda - lambda_oracle| / |lambda| = {err:.2e}", flush=True)
        assert err < FP64_TOL, (n, err)
    f.close()


_CORE16 = W.pulsed_core(ncell=64, nsub=16, nsteps=3)
_CORE16_ORACLE = {}


@pytest.mark.parametrize("precision", [B.FP64, B.FP32_IR], ids=["fp64", "fp32_ir"])
def test_large_coarse_space_matches_oracle(precision):
    require_gpu()
    w = _CORE16
    if "lats" not in _CORE16_ORACLE:
        _CORE16_ORACLE["lats"] = oracle_reference(w, w.nsteps)[1]
    f = setup(w, precision=precision)
    sz = f.get_sizes()
    print(f"[coarse] {w.name}: n_c {sz['n_c']} N_lambda {sz['n_lambda']}", flush=True)
    assert sz["n_c"] > 192
    if precision == B.FP64:
        o, tol = opts(tol=w.tol, max_it=4000), FP64_TOL
    else:
        o, tol = opts_mixed(tol=w.tol, max_it=4000), MIXED_TOL
    _run_and_compare(w, w.nsteps, f, o, tol, _CORE16_ORACLE["lats"], label=f"prec {precision}")
    f.close()


def test_lumped_preconditioner_reaches_the_same_solution():
    import torch
    require_gpu()
    w = W.nearly_incompressible_scaled(32, 4, nsteps=3)
    lats = oracle_reference(w, w.nsteps)[1]
    sols, its = {}, {}
    for name, pc in (("dirichlet", B.PRECOND_DIRICHLET), ("lumped", B.PRECOND_LUMPED)):
        f = setup(w, precond=pc)
        its[name] = _run_and_compare(w, w.nsteps, f, opts(tol=w.tol, max_it=4000), FP64_TOL, lats, label=name)
        u = torch.empty(f.get_sizes()["sum_ns"], dtype=torch.float64, device="cuda")
        f.get_solution(u)
        sols[name] = u.cpu().numpy()
        f.close()
    d = np.abs(sols["lumped"] - sols["dirichlet"]).max() / np.abs(sols["dirichlet"]).max()
    print(f"  iterations per step: {its}; |u_lumped - u_dirichlet| / |u| = {d:.1e}", flush=True)
    assert d < FP64_TOL


def _traj(w, n, f, o):
    import torch
    for k in range(1, n + 1):
        st = f.step(load(w, k * w.tau), o)
        assert st["status"] == 0, st
    u = torch.empty(f.get_sizes()["sum_ns"], dtype=torch.float64, device="cuda")
    lam = torch.empty(f.get_sizes()["n_lambda"], dtype=torch.float64, device="cuda")
    f.get_solution(u, lam)
    return u.cpu().numpy(), lam.cpu().numpy()


def test_checkpoint_resume_is_bitwise():
    import torch
    require_gpu()
    w = W.nearly_incompressible_scaled(32, 4, nsteps=10)
    o = opts(tol=w.tol, max_it=3000)
    a = setup(w)
    ua, la = _traj(w, 10, a, o)
    a.close()
    b = setup(w)
    for k in range(1, 6):
        b.step(load(w, k * w.tau), o)
    state = torch.empty(b.state_size(), dtype=torch.float64, device="cuda")
    meta = b.get_state(state)
    b.close()
    assert meta == [5, 1, 1, 1], meta
    c = setup(w)
    c.set_state(state, meta)
    for k in range(6, 11):
        c.step(load(w, k * w.tau), o)
    u = torch.empty(c.get_sizes()["sum_ns"], dtype=torch.float64, device="cuda")
    lam = torch.empty(c.get_sizes()["n_lambda"], dtype=torch.float64, device="cuda")
    c.get_solution(u, lam)
    assert np.array_equal(u.cpu().numpy(), ua) and np.array_equal(lam.cpu().numpy(), la)
    with pytest.raises(B.FetiError):
        c.set_state(state, [5, 0, 1, 1])
    c.close()


def test_solve_between_steps_leaves_the_trajectory_unchanged():
    import torch
    require_gpu()
    w = W.nearly_incompressible_scaled(16, 4, nsteps=3)
    o = opts(tol=w.tol, max_it=3000)
    a = setup(w)
    ua, la = _traj(w, 3, a, o)
    a.close()
    b = setup(w)
    b.step(load(w, w.tau), o)
    n = b.get_sizes()["sum_ns"]
    fv = torch.empty(n, dtype=torch.float64, device="cuda")
    b.get_rhs(fv)
    fv2 = (fv * 0.5 + 1.0).contiguous()
    lam = torch.zeros(b.get_sizes()["n_lambda"], dtype=torch.float64, device="cuda")
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    b.solve(fv2, lam, u, o)
    f_after = torch.empty_like(fv)
    b.get_rhs(f_after)
    assert bool((f_after == fv).all())
    for k in (2, 3):
        b.step(load(w, k * w.tau), o)
    ub = torch.empty(n, dtype=torch.float64, device="cuda")
    lb = torch.empty_like(lam)
    b.get_solution(ub, lb)
    assert np.array_equal(ub.cpu().numpy(), ua) and np.array_equal(lb.cpu().numpy(), la)
    b.close()


def test_field_export_matches_oracle_lattice():
    import torch
    require_gpu()
    w = W.nearly_incompressible_scaled(16, 4, nsteps=2)
    lats = oracle_reference(w, 2)[1]
    f = setup(w)
    for k in (1, 2):
        f.step(load(w, k * w.tau), opts(tol=w.tol, max_it=3000))
    sz = f.get_sizes()
    names = {B.FIELD_UX: ("ux_P", "ux_E"), B.FIELD_UY: ("uy_P", "uy_E"), B.FIELD_ETA: ("eta",),
             B.FIELD_XI_P: ("xiP",), B.FIELD_P: ("p",), B.FIELD_XI_E: ("xiE",)}
    for fld, keys in names.items():
        n = sz["n_u"] if fld <= B.FIELD_UY else sz["n_p1"]
        out = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
        f.get_field(fld, out)
        got = out.cpu().numpy()
        ref = np.full(n, np.nan)
        for kk in keys:  # u: either region's value (they agree on the interface)
            v = lats[-1][kk]
            ref = np.where(np.isnan(ref), v, ref)
        has = got != 0.0
        scale = np.nanmax(np.abs(ref))
        err = np.abs(got[has] - ref[has]).max() / scale
        print(f"  field {fld}: {has.sum()} nodes with unknowns, err {err:.1e}", flush=True)
        assert has.sum() > 0 and np.all(np.isfinite(ref[has])) and err < FP64_TOL
    with pytest.raises(B.FetiError):
        f.get_field(9, out)
    f.close()
