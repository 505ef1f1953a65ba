"""GPU parity of the dual-primal coupling (primal xi / p and corner DOFs, multipliers on
the other u / eta DOFs): the interface operator against the oracle's F = B K~^{-1} B^T
(and the allocation-free entry point against it bit for bit), the preconditioner
against its dense definition, time steps against the monolithic oracle (bar 1e-8 per
field kind, as for the dual coupling), one value per primal DOF, and the 64-subdomain
h = 1/128 workload over the bench's horizon.
"""
import numpy as np
import pytest

import workloads as W
from oracle import local as lo
from feti_helpers import (require_gpu, cached_oracle_lattices, torn_reference, per_kind_rel_error,
                          sub_poro_flags)

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts, mesh_args, material  # noqa: E402

FP64_TOL = 1e-8


def _dp(w):
    return w.replace(coupling="primal")


def _ctx(w):
    require_gpu()
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
    return f


OP_CASES = [
    _dp(W.plain_fp64_small().replace(ncell=8)),
    _dp(W.nearly_incompressible_scaled(8, 4)),
    _dp(W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3)),
    _dp(W.pulsed_core(ncell=8, nsub=4, nsteps=1)),
]


@pytest.mark.parametrize("w", OP_CASES, ids=lambda w: w.name + "_primal")
def test_dual_primal_operators_match_the_oracle(w):
    import torch
    from oracle.dual_primal import DualPrimal
    print(f"[dp operators] {w.name}", flush=True)
    D = DualPrimal(w)
    F = D.operator()
    spec = D.spec
    nl = spec.n_lambda
    # Dirichlet preconditioner: D_B (sum_s B_s S_bb,s B_s^T) D_B with B zero on the primal DOFs
    Bs = []
    for si, s in enumerate(spec.subs):
        Bm = np.zeros((nl, len(s.codes)))
        for j, row in enumerate(spec.rows):
            for sub, loc, sg in row:
                if sub == si:
                    Bm[j, loc] += sg
        Bs.append(Bm)
    Dw = np.linalg.inv(np.hstack(Bs) @ np.hstack(Bs).T)
    M = np.zeros((nl, nl))
    for Bm, K, s in zip(Bs, D.L.K, spec.subs):
        b = np.nonzero(np.array(s.cats) >= 2)[0]
        M += Dw @ Bm[:, b] @ lo.schur_bb(K, s.cats) @ Bm[:, b].T @ Dw
    f = _ctx(w)
    sz = f.get_sizes()
    assert sz["n_lambda"] == nl and sz["n_primal"] == D.npi and sz["n_c"] == 0
    x = np.random.default_rng(11).standard_normal(nl)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    f.apply_F(xd, y)
    ref = F @ x
    got = y.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    y2 = torch.empty_like(xd)
    f.apply_F_noalloc(xd, y2)
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), got)
    f.apply_precond(xd, y)
    ref = M @ x
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()
    f.close()


STEP_CASES = [
    (_dp(W.plain_fp64_small()), 4),
    (_dp(W.nearly_incompressible_scaled(16, 4)), 3),
    (_dp(W.nearly_incompressible_scaled(32, 8)), 2),
    (_dp(W.nearly_incompressible_scaled(24, 4).replace(layout=W.YSPLIT, name="ysplit_p2_h24_4x4")), 3),
    (_dp(W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3, nsteps=2)), 2),
    (_dp(W.patch_case(order_u=1, ncell=12, nsub_x=4, nsub_y=2, nsteps=2)), 2),
    (_dp(W.pulsed_core(ncell=16, nsub=4, nsteps=3)), 3),
    (_dp(W.nearly_incompressible_scaled(24, 4).replace(cut_x=(0, 5, 12, 20, 24), name="xsplit_h24_cuts")), 2),
]


def _primal_copies_agree(codes, sub_offset, u, primal_codes):
    """Every owner of a primal DOF holds the same value (one global unknown)."""
    sel = np.isin(codes, primal_codes)
    vals = {}
    for c, v in zip(codes[sel], u[sel]):
        if c in vals:
            assert v == vals[c], c
        vals[c] = v
    return len(vals)


@pytest.mark.parametrize("w,nsteps", STEP_CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_dual_primal_time_steps_match_monolithic_oracle(w, nsteps):
    import torch
    print(f"[dp steps] {w.name} x{nsteps}", flush=True)
    lats = cached_oracle_lattices(w, nsteps)
    f = setup(w)
    idx = f.export_indexing()
    pr = f.export_primal()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts(tol=w.tol, max_it=2000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        assert st["status"] == 0 and st["iters"] < 2000, st
        f.get_solution(u)
        un = u.cpu().numpy()
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, un, ref)
        print(f"  step {n}: iters {st['iters']} err {err}", flush=True)
        assert max(err.values()) < FP64_TOL, (n, err)
        assert _primal_copies_agree(codes, idx["sub_offset"], un, pr["code"]) == len(pr["code"])
    rho = f.torn_residual()
    print(f"  torn residual {rho:.2e}", flush=True)
    assert rho < 1e-9
    f.close()


def test_dual_primal_full_size_workload_matches_oracle():
    """The 64-subdomain h = 1/128 workload under the dual-primal coupling, as bench.py runs
    it, against the oracle at every step of the bench's horizon (5 warm-up and 20 timed
    steps)."""
    import time
    import torch
    w = _dp(W.nearly_incompressible_large())
    nsteps = 25
    t0 = time.time()
    print("[dp full] oracle ...", flush=True)
    lats = cached_oracle_lattices(w, nsteps)
    print(f"[dp full] oracle done in {time.time() - t0:.1f} s", flush=True)
    f = setup(w)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts(tol=w.tol, max_it=3000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        print(f"[dp full] step {n}: iters {st['iters']} res {st['res']:.2e} err {err}", flush=True)
        assert st["status"] == 0
        assert max(err.values()) < FP64_TOL, (n, err)
    f.close()


def test_dual_primal_is_rejected_where_unsupported():
    require_gpu()
    w = _dp(W.nearly_incompressible_scaled(8, 4))
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    with pytest.raises(B.FetiError) as e:
        f.factor_subdomains(B.FP32_IR, B.PRECOND_DIRICHLET)
    assert e.value.code == B.EINVAL
    f.close()


@pytest.mark.parametrize("coupling", ["dual", "primal"])
def test_refactorisation_reproduces_the_steps_bit_for_bit(coupling):
    """A second feti_factor_subdomains on the same context (the dense coarse inverses of
    G^T G, S_PiPi and W^T F W rebuilt in place) gives the same steps bit for bit as one
    factorisation."""
    require_gpu()
    import torch
    w = W.nearly_incompressible_scaled(16, 4).replace(coupling=coupling)
    o = opts(tol=w.tol, max_it=2000)
    out = []
    for nfact in (1, 2):
        f = B.Feti()
        f.setup_mesh(**mesh_args(w))
        f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
        for _ in range(nfact):
            f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
        f.init_state(load(w, 0.0))
        sz = f.get_sizes()
        for n in range(1, 4):
            st = f.step(load(w, n * w.tau), o)
            assert st["status"] == 0
        u = torch.empty(sz["sum_ns"], dtype=torch.float64, device="cuda")
        lam = torch.empty(sz["n_lambda"], dtype=torch.float64, device="cuda")
        f.get_solution(u=u, lam=lam)
        out.append((u.cpu().numpy(), lam.cpu().numpy()))
        f.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
