"""GPU parity in 3D (Kuhn tetrahedra of the unit cube, P2 or P1 displacement, P1 scalars,
the dual-primal coupling): the stationary polynomial solution reproduced, and time steps
with seeded nodal data against the 3D monolithic oracle at the FP64 bar (1e-8 per field
kind) for several decompositions, with one value per primal DOF and the uz field export.
"""
import numpy as np
import pytest

import workloads as W
from feti_helpers import require_gpu, torn_reference, per_kind_rel_error

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts  # noqa: E402

FP64_TOL = 1e-8


def _poro(w):
    from oracle import indexing as ix
    return [s.poro for s in ix.build(w).subs]


def _run(w, nsteps, lats, tol=FP64_TOL):
    import torch
    f = setup(w)
    idx = f.export_indexing()
    pr = f.export_primal()
    codes = idx["code"].astype(np.int64)
    poro = _poro(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts(tol=w.tol, max_it=3000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        assert st["status"] == 0, st
        f.get_solution(u)
        un = u.cpu().numpy()
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, un, ref)
        print(f"  step {n}: iters {st['iters']} err {err}", flush=True)
        assert max(err.values()) < tol, (n, err)
        sel = np.isin(codes, pr["code"])
        first = {}
        for c, v in zip(codes[sel], un[sel]):
            assert first.setdefault(c, v) == v
    return f


@pytest.mark.parametrize("order", [2, 1])
def test_3d_patch_solution_is_reproduced(order):
    from oracle.monolithic3d import patch_data, patch_exact
    require_gpu()
    w = W.cube_case(ncell=4, order_u=order, nsteps=2).replace(dirichlet_p=0x3F)
    kw = {} if order == 2 else {"q": (0.0, 0.0, 0.0)}
    w.load.raw_fixed = patch_data(w, **kw)
    ex = patch_exact(w, kw)
    lats = [ex, ex]
    print(f"[3d patch] P{order}", flush=True)
    f = _run(w, 2, lats, tol=1e-10)
    f.close()


OP_CASES = [W.cube_case(ncell=4), W.cube_case(ncell=4, order_u=1, nsub=(2, 1, 3))]


@pytest.mark.parametrize("w", OP_CASES, ids=lambda w: w.name)
def test_3d_stages_match_the_oracle(w):
    """The assembled local matrices, their interface Schur complements, F = B K~^{-1} B^T
    and the Dirichlet preconditioner against the oracle's plain definitions."""
    import torch
    from oracle import local as lo
    from oracle.dual_primal import DualPrimal
    from paper_2509_06673_amd.workload import mesh_args, material
    require_gpu()
    print(f"[3d stages] {w.name}", flush=True)
    L = lo.build_local3d(w)
    D = DualPrimal(w, L)
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
    spec = D.spec
    for si, (s, K) in enumerate(zip(spec.subs, L.K)):
        n = len(s.codes)
        out = torch.empty(n * n, dtype=torch.float64, device="cuda")
        f.export_local(si, B.EXPORT_K, out)
        Kg = out.cpu().numpy().reshape(n, n)
        assert np.abs(Kg - K).max() <= 1e-12 * np.abs(K).max(), ("K", si)
        nb = int(sum(1 for c in s.cats if c >= 2))
        out = torch.empty(nb * nb, dtype=torch.float64, device="cuda")
        f.export_local(si, B.EXPORT_SBB, out)
        S = lo.schur_bb(K, s.cats)
        assert np.abs(out.cpu().numpy().reshape(nb, nb) - S).max() <= 1e-9 * np.abs(S).max(), ("S_bb", si)
    nl = spec.n_lambda
    F = D.operator()
    x = np.random.default_rng(3).standard_normal(nl)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    f.apply_F(xd, y)
    ref = F @ x
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"  F rel err {err:.2e}", flush=True)
    assert err <= 1e-9
    f.close()


CASES = [
    (W.cube_case(ncell=4, nsteps=3), 3),
    (W.cube_case(ncell=4, order_u=1, nsub=(2, 1, 3), nsteps=3), 3),
    (W.cube_case(ncell=8, nsub=(4, 2, 2), nsteps=2), 2),
    (W.cube_case(ncell=6, nsub=(2, 3, 2), nsteps=2, nu=0.49), 2),
]


@pytest.mark.parametrize("w,nsteps", CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_3d_time_steps_match_the_monolithic_oracle(w, nsteps):
    import torch
    from oracle.monolithic3d import solve_steps
    require_gpu()
    print(f"[3d steps] {w.name} x{nsteps}", flush=True)
    tr = solve_steps(w, nsteps)
    lats = [tr.system.to_lattice(x) for x in tr.states]
    f = _run(w, nsteps, lats)
    rho = f.torn_residual()
    print(f"  torn residual {rho:.2e}", flush=True)
    assert rho < 1e-9
    sz = f.get_sizes()
    out = torch.empty(sz["n_u"], dtype=torch.float64, device="cuda")
    f.get_field(B.FIELD_UZ, out)
    ref = np.where(np.isnan(lats[-1]["uz_P"]), lats[-1]["uz_E"], lats[-1]["uz_P"])
    got = out.cpu().numpy()
    codes = f.export_indexing()["code"].astype(np.int64)
    nodes = np.unique(codes[codes % 8 == 6] // 8)      # the uz unknowns (Dirichlet nodes are not)
    assert np.abs(got[nodes] - ref[nodes]).max() < FP64_TOL * np.nanmax(np.abs(ref))
    f.close()
