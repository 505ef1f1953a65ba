"""Parity of the HIP path with the FP64 oracle, stage by stage and end to end.

Every call goes through the C ABI (libfeti.so).  Floating-point tolerances:
assembled matrices and the local eliminations are compared in the symmetric
diagonal scaling D K D (D = |diag K|^{-1/2}) in which all fields are O(1);
solutions are compared field kind by field kind, relative to the field's
largest magnitude, at the 1e-8 bound required of the FP64 path.
"""
import numpy as np
import pytest

import workloads as W
from oracle import indexing as ix, local as lo
from feti_helpers import (require_gpu, oracle_reference, torn_reference, per_kind_rel_error,
                          sub_poro_flags, cached_oracle_lattices)

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts, mesh_args, material  # noqa: E402

FP64_TOL = 1e-8


def _ctx(w, factor=True, precond=B.PRECOND_DIRICHLET):
    require_gpu()
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    if factor:
        f.factor_subdomains(B.FP64, precond)
    return f


def _export(f, sub, which, n):
    import torch
    out = torch.empty(n * n, dtype=torch.float64, device="cuda")
    f.export_local(sub, which, out)
    return out.cpu().numpy().reshape(n, n)


STAGE_CASES = [
    W.plain_fp64_small().replace(ncell=8),
    W.nearly_incompressible_scaled(8, 4),
    W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3),
    W.pulsed_core(ncell=8, nsub=4, nsteps=1),
]


@pytest.mark.parametrize("w", STAGE_CASES, ids=lambda w: w.name)
def test_assembly_matches_oracle(w):
    print(f"[assembly] {w.name}", flush=True)
    L = lo.build_local(w)
    f = _ctx(w, factor=False)
    for s, Kref in enumerate(L.K):
        n = Kref.shape[0]
        K = _export(f, s, B.EXPORT_K, n)
        d = 1.0 / np.sqrt(np.abs(np.diag(Kref)))
        err = np.abs(d[:, None] * (K - Kref) * d[None, :]).max()
        assert err < 1e-12, (s, err)
    f.close()


@pytest.mark.parametrize("w", STAGE_CASES, ids=lambda w: w.name)
def test_schur_and_generalized_inverse_match_oracle(w):
    print(f"[factor] {w.name}", flush=True)
    L = lo.build_local(w)
    f = _ctx(w)
    for s, (sub, Kref) in enumerate(zip(L.spec.subs, L.K)):
        n = Kref.shape[0]
        d = 1.0 / np.sqrt(np.abs(np.diag(Kref)))
        cats = np.array(sub.cats)
        b = np.nonzero(cats >= 2)[0]
        Sref = lo.schur_bb(Kref, sub.cats)
        S = _export(f, s, B.EXPORT_SBB, len(b))
        db = d[b]
        e1 = np.abs(db[:, None] * (S - Sref) * db[None, :]).max()
        assert e1 < 1e-9, (s, e1)
        Pref = lo.generalized_inverse(Kref, sub.cats)
        Kp = _export(f, s, B.EXPORT_KPLUS, n)
        # in the scaled variables the inverse is (D K D)^{-1} = D^{-1} K^{-1} D^{-1}
        e2 = np.abs((Kp - Pref) / d[:, None] / d[None, :]).max() / np.abs(Pref / d[:, None] / d[None, :]).max()
        assert e2 < 1e-9, (s, e2)
    f.close()


def _dense_operators(w):
    L = lo.build_local(w)
    spec = L.spec
    nl = spec.n_lambda
    Bs = [np.zeros((nl, len(s.codes))) for s in spec.subs]
    for j, r in enumerate(spec.rows):
        for s, loc, sg in r:
            Bs[s][j, loc] = sg
    F = sum(Bm @ lo.generalized_inverse(K, s.cats) @ Bm.T for Bm, K, s in zip(Bs, L.K, spec.subs))
    Bfull = np.hstack(Bs)
    D = np.linalg.inv(Bfull @ Bfull.T)
    M = np.zeros((nl, nl))
    for Bm, K, s in zip(Bs, L.K, spec.subs):
        b = np.nonzero(np.array(s.cats) >= 2)[0]
        M += D @ Bm[:, b] @ lo.schur_bb(K, s.cats) @ Bm[:, b].T @ D
    return F, M


@pytest.mark.parametrize("w", STAGE_CASES, ids=lambda w: w.name)
def test_interface_operators_match_dense_definitions(w):
    import torch
    print(f"[operators] {w.name}", flush=True)
    F, M = _dense_operators(w)
    f = _ctx(w)
    nl = F.shape[0]
    x = np.random.default_rng(7).standard_normal(nl)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    f.apply_F(xd, y)
    ref = F @ x
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()
    f.apply_precond(xd, y)
    ref = M @ x
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()
    f.close()


STEP_CASES = [
    (W.plain_fp64_small(), 10),
    (W.nearly_incompressible_scaled(16, 4), 3),
    (W.nearly_incompressible_scaled(32, 8), 2),
    (W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3, nsteps=2), 2),
    (W.patch_case(order_u=1, ncell=12, nsub_x=4, nsub_y=2, nsteps=2), 2),
    (W.pulsed_core(ncell=16, nsub=4, nsteps=3), 3),
    (W.learned_start_case(3, nsteps=3, ncell=16).replace(nsub_x=4, nsub_y=4), 3),
]


@pytest.mark.parametrize("w,nsteps", STEP_CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_time_steps_match_monolithic_oracle(w, nsteps):
    import torch
    print(f"[steps] {w.name} x{nsteps}", flush=True)
    sysm, lats = oracle_reference(w, nsteps)
    f = setup(w)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts(tol=w.tol, max_it=2000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        assert st["status"] == 0 and st["iters"] < 2000, st
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        print(f"  step {n}: iters {st['iters']} err {err}", flush=True)
        assert max(err.values()) < FP64_TOL, (n, err)
    f.close()


def test_patch_solution_is_exact_for_any_decomposition():
    import torch
    for order, (nx, ny) in ((2, (4, 3)), (1, (2, 4))):
        w = W.patch_case(order_u=order, ncell=12, nsub_x=nx, nsub_y=ny)
        print(f"[patch] {w.name}", flush=True)
        from oracle.problem import make_loads
        ld = make_loads(w)
        f = setup(w)
        idx = f.export_indexing()
        codes = idx["code"].astype(np.int64)
        f.step(load(w, w.tau), opts())
        u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
        f.get_solution(u)
        u = u.cpu().numpy()
        poro = np.repeat(sub_poro_flags(w), np.diff(idx["sub_offset"]))
        r = 1 if order == 1 else 2
        for k, fn in ((0, (ld.uPx, ld.uEx)), (1, (ld.uPy, ld.uEy)), (4, (ld.p, ld.p))):
            sel = codes % 8 == k
            node = codes[sel] // 8
            mu = (r * w.ncell + 1) if k < 2 else (w.ncell + 1)
            hh = 1.0 / (mu - 1)
            x, y = (node % mu) * hh, (node // mu) * hh
            ex = np.where(poro[sel], fn[0](x, y, 0.0), fn[1](x, y, 0.0))
            assert np.abs(u[sel] - ex).max() < 1e-9, (order, k)
        f.close()


def test_start_vectors_and_zero_iterations_for_exact_start():
    import torch
    w = W.nearly_incompressible_scaled(16, 4)
    f = setup(w)
    sz = f.get_sizes()
    st1 = f.step(load(w, w.tau), opts(start=B.START_ZERO))
    lam = torch.empty(sz["n_lambda"], dtype=torch.float64, device="cuda")
    f.get_solution(None, lam)
    # re-solving the same right-hand side from its own solution needs no iteration
    fv = torch.empty(sz["sum_ns"], dtype=torch.float64, device="cuda")
    f.get_rhs(fv)
    u2 = torch.empty_like(fv)
    lam2 = lam.clone()
    st2 = f.solve(fv, lam2, u2, opts(start=B.START_GIVEN))
    assert st1["iters"] > 5
    assert st2["iters_first"] <= 1, st2
    assert torch.allclose(lam2, lam, rtol=0, atol=1e-9 * lam.abs().max().item())
    f.close()


def test_not_converged_is_reported_with_iterate():
    w = W.nearly_incompressible_scaled(16, 4)
    f = setup(w)
    st = f.step(load(w, w.tau), opts(max_it=2, check_every=1, ir_cold=0, ir_max=0), allow=(B.ENOTCONV,))
    assert st["rc"] == B.ENOTCONV and st["iters"] == 2
    f.close()


@pytest.mark.parametrize("start", [B.START_PREVIOUS, B.START_EXTRAPOLATE], ids=["previous", "extrapolated"])
def test_full_size_workload_matches_oracle(start):
    """The 64-subdomain h = 1/128 workload, as bench.py runs it (first solves from the
    previous step's multipliers, or from their extrapolation), against the oracle at
    every step of the bench's horizon (5 warm-up and 20 timed steps)."""
    import time
    import torch
    w = W.nearly_incompressible_large()
    nsteps = 25
    t0 = time.time()
    print("[full] oracle ...", flush=True)
    lats = cached_oracle_lattices(w, nsteps)
    print(f"[full] oracle done in {time.time() - t0:.1f} s", flush=True)
    f = setup(w)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts(tol=w.tol, max_it=3000, start=start)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        print(f"[full] step {n}: iters {st['iters']} res {st['res']:.2e} err {err}", flush=True)
        assert st["status"] == 0
        assert max(err.values()) < FP64_TOL, (n, err)
    f.close()


_UPD_CASE = W.nearly_incompressible_scaled(64, 8, nsteps=8)
_UPD_ORACLE = {}


@pytest.mark.parametrize("mode", ["auto", "graph"])
def test_update_test_and_warm_corrections_match_oracle(mode):
    """Refinement corrections that stop on the size of their updates and start from the
    previous step's correction, on the persistent launch and on the graph-captured
    kernel chain: every step within the FP64 bar of the oracle.  The iteration counts
    of both variants depend on where the iteration on the indefinite F turns erratic,
    which moves with rounding; the update test must not cost more than a quarter over
    corrections run to their residual tolerance from zero (its gain is measured on the
    full-size case by bench.py)."""
    import torch
    w = _UPD_CASE
    print(f"[upd] {w.name} x{w.nsteps} mode {mode}", flush=True)
    if "lats" not in _UPD_ORACLE:
        _UPD_ORACLE["lats"] = oracle_reference(w, w.nsteps)[1]
    lats = _UPD_ORACLE["lats"]
    iters = {}
    for name, o in (("plain", opts(tol=w.tol, max_it=3000, tol_upd=0.0, corr_start=B.CORR_ZERO)),
                    ("upd", opts(tol=w.tol, max_it=3000))):
        assert name == "plain" or (o.tol_upd > 0 and o.corr_start == B.CORR_PREVIOUS)
        f = setup(w)
        if mode == "graph":
            f.set_pcg_mode(B.PCG_GRAPH)
        idx = f.export_indexing()
        codes = idx["code"].astype(np.int64)
        poro = sub_poro_flags(w)
        u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
        its = []
        for n in range(1, w.nsteps + 1):
            st = f.step(load(w, n * w.tau), o)
            assert st["status"] == 0, st
            f.get_solution(u)
            err = per_kind_rel_error(codes, u.cpu().numpy(), torn_reference(codes, idx["sub_offset"], poro,
                                                                             lats[n - 1]))
            its.append(st["iters"])
            print(f"  {name} step {n}: iters {st['iters']} (first {st['iters_first']}) err "
                  f"{max(err.values()):.1e}", flush=True)
            assert max(err.values()) < FP64_TOL, (name, n, err)
        f.close()
        iters[name] = sum(its[1:])
    print(f"  iterations (steps 2..): {iters}", flush=True)
    assert iters["upd"] <= 1.25 * iters["plain"], iters


def test_pcg_mode_is_validated():
    require_gpu()
    f = B.Feti()
    with pytest.raises(B.FetiError):
        f.set_pcg_mode(7)
    f.set_pcg_mode(B.PCG_GRAPH)
    f.set_pcg_mode(B.PCG_AUTO)
    f.close()


def test_correction_start_is_validated():
    w = W.nearly_incompressible_scaled(8, 2)
    require_gpu()
    f = setup(w)
    with pytest.raises(B.FetiError):
        f.step(load(w, w.tau), opts(corr_start=2))
    st = f.step(load(w, w.tau), opts(corr_start=B.CORR_ZERO))
    assert st["status"] == 0, st
    f.close()


def _rhs_after_step(f, L, n):
    import torch
    st = f.step(L, opts())
    assert st["status"] == 0, st
    fv = torch.empty(n, dtype=torch.float64, device="cuda")
    f.get_rhs(fv)
    return fv


def test_cached_load_parts_give_the_same_right_hand_side():
    """Loads that do not depend on time: the element load parts of the first step are
    kept and later steps with the same load start from them.  The right-hand side must
    be bit for bit the one of the full quadrature, and another load must not reuse them."""
    require_gpu()
    # manufactured loads: second step from the same state takes the cached parts
    w = W.nearly_incompressible_scaled(16, 4)
    L = load(w, w.tau)
    a = setup(w)
    n = a.get_sizes()["sum_ns"]
    fa = _rhs_after_step(a, L, n)
    b = setup(w)
    _rhs_after_step(b, L, n)
    b.init_state(load(w, 0.0))
    fb = _rhs_after_step(b, L, n)
    assert bool((fa == fb).all()), float((fa - fb).abs().max())
    a.close()
    b.close()
    # patch loads with other parameters: no reuse of the first load's parts
    wp = W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3)
    L1 = load(wp, wp.tau)
    L2 = load(wp, wp.tau)
    L2.params[0] += 0.25
    L2.params[7] -= 0.5
    c = setup(wp)
    n = c.get_sizes()["sum_ns"]
    _rhs_after_step(c, L1, n)
    c.init_state(L2)
    fc = _rhs_after_step(c, L2, n)
    d = setup(wp)
    d.init_state(L2)
    fd = _rhs_after_step(d, L2, n)
    assert bool((fc == fd).all()), float((fc - fd).abs().max())
    c.close()
    d.close()
