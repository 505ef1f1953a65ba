"""FP32 factors on the matrix cores with FP64 refinement, against the FP64 oracle.

The local eliminations run in FP32 (pivot blocks and W = P^{-1} C accumulated in
FP64); K_s^+, S_bb and the interface blocks are stored in FP32.  The torn
residual, the interface vectors, dot products and the coarse problem stay in
FP64, and refinement corrections win the accuracy back.  The bar for the
solution is 1e-6 relative per field kind after refinement; the FP32 factors
themselves are checked against the FP64 definitions at the level FP32 rounding
of a pivot-free elimination allows (in the symmetric diagonal scaling).
"""
import numpy as np
import pytest

import workloads as W
from oracle import local as lo
from feti_helpers import require_gpu, oracle_reference, torn_reference, per_kind_rel_error, sub_poro_flags

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts_mixed, mesh_args, material  # noqa: E402

MIXED_TOL = 1e-6


def _export(f, sub, which, n):
    import torch
    out = torch.empty(n * n, dtype=torch.float64, device="cuda")
    f.export_local(sub, which, out)
    return out.cpu().numpy().reshape(n, n)


@pytest.mark.parametrize("w", [W.plain_fp64_small().replace(ncell=8), W.nearly_incompressible_scaled(8, 4)],
                         ids=lambda w: w.name)
def test_fp32_factors_close_to_fp64_definitions(w):
    print(f"[fp32 factor] {w.name}", flush=True)
    require_gpu()
    L = lo.build_local(w)
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.factor_subdomains(B.FP32_IR, B.PRECOND_DIRICHLET)
    for s, (sub, Kref) in enumerate(zip(L.spec.subs, L.K)):
        n = Kref.shape[0]
        cats = np.array(sub.cats)
        b = np.nonzero(cats >= 2)[0]
        keep = np.nonzero(cats != 4)[0]
        Sref = lo.schur_bb(Kref, sub.cats)
        S = _export(f, s, B.EXPORT_SBB, len(b))
        d = 1.0 / np.sqrt(np.abs(np.diag(Kref)))
        db = d[b]
        e1 = np.abs(db[:, None] * (S - Sref) * db[None, :]).max() / np.abs(db[:, None] * Sref * db[None, :]).max()
        Kp = _export(f, s, B.EXPORT_KPLUS, n)
        # the refinement converges when K^+ K is close to the identity on the swept DOFs
        E = np.eye(len(keep)) - Kp[np.ix_(keep, keep)] @ Kref[np.ix_(keep, keep)]
        rad = np.abs(np.linalg.eigvals(E)).max()
        print(f"  sub {s}: S_bb scaled rel err {e1:.1e}, spectral radius of I - K32^+ K {rad:.1e}", flush=True)
        assert e1 < 1e-4, (s, e1)
        assert rad < 1e-3, (s, rad)
    f.close()


MIXED_CASES = [
    (W.plain_fp64_small(), 4),
    (W.nearly_incompressible_scaled(16, 4), 3),
    (W.nearly_incompressible_scaled(32, 8), 2),
    (W.pulsed_core(ncell=16, nsub=4, nsteps=3), 3),
    (W.patch_case(order_u=2, ncell=12, nsub_x=4, nsub_y=3, nsteps=2), 2),
]


@pytest.mark.parametrize("w,nsteps", MIXED_CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_mixed_time_steps_match_oracle(w, nsteps):
    import torch
    print(f"[mixed steps] {w.name} x{nsteps}", flush=True)
    sysm, lats = oracle_reference(w, nsteps)
    f = setup(w, precision=B.FP32_IR)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts_mixed(tol=w.tol, max_it=2000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        assert st["status"] == 0, st
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        print(f"  step {n}: iters {st['iters']} first {st['iters_first']} corrections {st['ir_steps']} "
              f"last correction {st['rho']:.1e} err {err}", flush=True)
        assert max(err.values()) < MIXED_TOL, (n, err)
    f.close()


def test_mixed_full_size_workload_matches_oracle():
    """The 64-subdomain h = 1/128 workload with FP32 factors, as bench.py runs it."""
    import torch
    w = W.nearly_incompressible_large()
    nsteps = 3
    print("[mixed full] oracle ...", flush=True)
    sysm, lats = oracle_reference(w, nsteps)
    f = setup(w, precision=B.FP32_IR)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    poro = sub_poro_flags(w)
    u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
    o = opts_mixed(tol=w.tol, max_it=3000)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], poro, lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        print(f"[mixed full] step {n}: iters {st['iters']} first {st['iters_first']} corrections "
              f"{st['ir_steps']} last correction {st['rho']:.1e} err {err}", flush=True)
        assert st["status"] == 0
        assert max(err.values()) < MIXED_TOL, (n, err)
    f.close()
