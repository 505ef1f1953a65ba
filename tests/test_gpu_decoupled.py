"""GPU parity of the decoupled mass balance (the explicit fluid step of the Remark after eq.
(linalg-system)): every torn unknown (u, xi_P, xi_E) and the fluid fields eta^n, p^n against
the decoupled oracle at every step, at the FP64 bar; the checkpoint state continues a
decoupled trajectory bit for bit."""
import numpy as np
import pytest

import workloads as W
from feti_helpers import require_gpu, torn_reference, per_kind_rel_error, sub_poro_flags

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import setup, load, opts  # noqa: E402

FP64_TOL = 1e-8


def _oracle(w, nsteps):
    from oracle.decoupled import solve_steps
    tr = solve_steps(w, nsteps=nsteps)
    return [tr.system.S.to_lattice(x) for x in tr.states]


def _field(f, kind, n):
    import torch
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    f.get_field(kind, out)
    return out.cpu().numpy()


def _rel_on(got, ref):
    sel = ~np.isnan(ref)
    s = np.abs(ref[sel]).max()
    return np.abs(got[sel] - ref[sel]).max() / (s if s > 0 else 1.0)


@pytest.mark.parametrize("w,tol_corr", [
    (W.nearly_incompressible_scaled(32, 4, nsteps=4).replace(scheme="decoupled"), 1e-3),
    (W.nearly_incompressible_scaled(32, 4, nsteps=4).replace(scheme="decoupled"), 1e-2),
    (W.nearly_incompressible_scaled(24, 4, nsteps=3).replace(scheme="decoupled", layout=W.YSPLIT,
                                                              name="ysplit_p2_h24_4x4"), 1e-3),
    (W.nearly_incompressible_scaled(32, 4, nsteps=4).replace(scheme="decoupled", coupling="primal"), 1e-3),
    (W.nearly_incompressible_scaled(24, 4, nsteps=3).replace(scheme="decoupled", layout=W.YSPLIT, coupling="primal",
                                                              name="ysplit_p2_h24_4x4"), 1e-3),
], ids=["xsplit_corr1e-3", "xsplit_corr1e-2", "ysplit_corr1e-3", "xsplit_dual_primal", "ysplit_dual_primal"])
def test_decoupled_steps_match_the_oracle(w, tol_corr):
    import torch
    require_gpu()
    nsteps = w.nsteps
    print(f"[decoupled] {w.name}, {nsteps} steps", flush=True)
    lats = _oracle(w, nsteps)
    f = setup(w)
    idx = f.export_indexing()
    codes = idx["code"].astype(np.int64)
    assert not np.isin(codes % 8, (2, 4)).any()  # no eta / p unknowns in the subdomains
    n1 = f.get_sizes()["n_p1"]
    o = opts(tol=1e-10, max_it=3000, tol_corr=tol_corr)
    for n in range(1, nsteps + 1):
        st = f.step(load(w, n * w.tau), o)
        u = torch.empty(len(codes), dtype=torch.float64, device="cuda")
        f.get_solution(u)
        ref = torn_reference(codes, idx["sub_offset"], sub_poro_flags(w), lats[n - 1])
        err = per_kind_rel_error(codes, u.cpu().numpy(), ref)
        e_eta = _rel_on(_field(f, B.FIELD_ETA, n1), lats[n - 1]["eta"])
        e_p = _rel_on(_field(f, B.FIELD_P, n1), lats[n - 1]["p"])
        print(f"  step {n}: iters {st['iters']}, torn {max(err.values()):.1e}, eta {e_eta:.1e}, p {e_p:.1e}",
              flush=True)
        assert st["status"] == 0
        assert max(err.values()) < FP64_TOL, err
        assert e_eta < FP64_TOL and e_p < FP64_TOL, (e_eta, e_p)
    f.close()


def test_decoupled_checkpoint_continues_bit_for_bit():
    import torch
    require_gpu()
    w = W.nearly_incompressible_scaled(16, 4, nsteps=4).replace(scheme="decoupled")
    o = opts(tol=1e-10, max_it=3000)
    a = setup(w)
    for n in range(1, 5):
        a.step(load(w, n * w.tau), o)
    b = setup(w)
    for n in range(1, 3):
        b.step(load(w, n * w.tau), o)
    nst = b.state_size()
    state = torch.empty(nst, dtype=torch.float64, device="cuda")
    meta = b.get_state(state)
    c = setup(w)
    c.set_state(state, meta)
    for n in range(3, 5):
        c.step(load(w, n * w.tau), o)
    n1 = a.get_sizes()["n_p1"]
    for kind in (B.FIELD_UX, B.FIELD_XI_P, B.FIELD_ETA, B.FIELD_P):
        nn = n1 if kind != B.FIELD_UX else a.get_sizes()["n_u"]
        assert np.array_equal(_field(a, kind, nn), _field(c, kind, nn)), kind
    for f in (a, b, c):
        f.close()
