"""Batched time steps: independent problems of uneven size in one cooperative launch
per solve.  A seeded subset of 16 of the 256 draws steps as one batch; every
problem must match its own single-problem run (same discretisation, same
tolerances; the iterates differ only in reduction order) and, for the whole subset,
the FP64 oracle at the 1e-8 bar of the FP64 path.
"""
import numpy as np
import pytest

import workloads as W
from feti_helpers import require_gpu, oracle_reference, torn_reference, per_kind_rel_error, sub_poro_flags

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts, mesh_args, material  # noqa: E402

FP64_TOL = 1e-8


def _subset(k=16, seed=3):
    draws = W.batched_draws()
    idx = np.sort(np.random.default_rng(seed).choice(len(draws), size=k, replace=False))
    return [draws[i] for i in idx]


_STREAM = []


def _stream():
    # a batch needs its contexts on one stream, and not the null stream (a context
    # given the null stream makes a stream of its own)
    import torch
    if not _STREAM:
        _STREAM.append(torch.cuda.Stream())
    return _STREAM[0]


def _ctx(w, keep=True):
    f = B.Feti(_stream())
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.set_keep_assembled(keep)
    f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
    f.init_state(load(w, 0.0))
    return f


def test_batch_matches_single_runs_and_oracle():
    """Every problem of the batch against its own single-problem run and against the
    oracle, at every step."""
    import torch
    require_gpu()
    ws = _subset()
    nsteps = 3
    print("[batch] " + " ".join(w.name for w in ws), flush=True)
    ctxs = [_ctx(w, keep=False) for w in ws]
    singles = [setup(w) for w in ws]
    lats = [oracle_reference(w, nsteps)[1] for w in ws]
    idxs = [f.export_indexing() for f in ctxs]
    batch = B.Batch(ctxs)
    o = opts(tol=1e-10, max_it=3000)
    worst_s = worst_o = 0.0
    for n in range(1, nsteps + 1):
        st, rc = batch.step([load(w, n * w.tau) for w in ws], o)
        _stream().synchronize()
        print(f"  step {n}: iterations per problem {[s['iters'] for s in st]} grid {batch.info()}", flush=True)
        assert rc == 0 and all(s["status"] == 0 for s in st)
        for k, (w, f, g, idx) in enumerate(zip(ws, ctxs, singles, idxs)):
            codes = idx["code"].astype(np.int64)
            u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            f.get_solution(u)
            ub = u.cpu().numpy()
            g.step(load(w, n * w.tau), o)
            g.get_solution(u)
            us = u.cpu().numpy()
            ref = torn_reference(codes, idx["sub_offset"], sub_poro_flags(w), lats[k][n - 1])
            e_single = max(per_kind_rel_error(codes, ub, us).values())
            e_oracle = max(per_kind_rel_error(codes, ub, ref).values())
            worst_s, worst_o = max(worst_s, e_single), max(worst_o, e_oracle)
            assert e_single < FP64_TOL, (w.name, n, e_single)
            assert e_oracle < FP64_TOL, (w.name, n, e_oracle)
        print(f"  step {n}: worst so far vs single {worst_s:.1e}, vs oracle {worst_o:.1e}", flush=True)
    batch.close()
    for f in ctxs + singles:
        f.close()


def test_in_place_factors_refuse_export_and_refactor():
    require_gpu()
    import torch
    w = W.plain_fp64_small()
    f = _ctx(w, keep=False)
    n = f.get_sizes()["max_ns"]
    out = torch.empty(n * n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.FetiError):
        f.export_local(0, B.EXPORT_K, out)
    with pytest.raises(B.FetiError):
        f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
    f.close()


def test_warm_step_of_a_draw_with_a_large_coarse_load_converges():
    """Draw 246 of the batch set converges at its warm steps.  Its interface load is
    dominated by the coarse (rigid-mode) part, so the projected start residual must take
    G^T r from r itself: formed as G^T d - G^T F lambda it cancels down to the rounding of
    G^T d, and the first solve of step 2 then cannot reach its tolerance."""
    import torch
    require_gpu()
    w = W.batched_draws()[246]
    nsteps = 3
    print(f"[draw 246] {w.name}", flush=True)
    f = setup(w)
    o = opts(tol=1e-10, max_it=3000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        print(f"  step {n}: first {st['iters_first']} corrections {st['iters_corr'][:st['ir_steps']]}", flush=True)
        assert st["status"] == 0 and st["iters_first"] < 3000, st
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    f.get_solution(u)
    _, lats = oracle_reference(w, nsteps)
    ref = torn_reference(codes, idx["sub_offset"], sub_poro_flags(w), lats[-1])
    err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
    print(f"  vs oracle {max(err.values()):.1e}", flush=True)
    assert max(err.values()) < FP64_TOL, err
    f.close()


def test_graph_captured_batch_steps_match_host_launched_steps():
    """The batch step replayed as a captured graph gives the same bits as the same step
    launched kernel by kernel from the host, at every step (several replays, with the
    host-launched batch's own work and synchronisations between them)."""
    import torch
    require_gpu()
    ws = _subset(k=8, seed=5)
    nsteps = 6
    print("[graph batch] " + " ".join(w.name for w in ws), flush=True)
    ga = [_ctx(w, keep=False) for w in ws]
    ea = [_ctx(w, keep=False) for w in ws]
    bg, be = B.Batch(ga), B.Batch(ea)
    for b in (bg, be):
        b.set_grid(256)
    bg.set_capture(True)
    be.set_capture(False)
    o = opts(tol=1e-10, max_it=3000)
    for n in range(1, nsteps + 1):
        stg, rcg = bg.step([load(w, n * w.tau) for w in ws], o)
        ste, rce = be.step([load(w, n * w.tau) for w in ws], o)
        _stream().synchronize()
        assert rcg == 0 and rce == 0
        assert [s["iters"] for s in stg] == [s["iters"] for s in ste], n
        assert bg.info()["graph"] == (n > 1) and not be.info()["graph"], n
        for f, g in zip(ga, ea):
            nu = f.get_sizes()["sum_ns"]
            nl = f.get_sizes()["n_lambda"]
            u1 = torch.empty(nu, dtype=torch.float64, device="cuda")
            u2 = torch.empty_like(u1)
            l1 = torch.empty(nl, dtype=torch.float64, device="cuda")
            l2 = torch.empty_like(l1)
            f.get_solution(u1, l1)
            g.get_solution(u2, l2)
            assert torch.equal(u1, u2) and torch.equal(l1, l2), n
        print(f"  step {n}: identical, iterations {[s['iters'] for s in stg]}", flush=True)
    bg.close()
    be.close()
    for f in ga + ea:
        f.close()
