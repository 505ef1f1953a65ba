"""Learned warm start: the network's kernels against the FP64 oracle, and what the
trained network gains over the previous-step start.

Reference.  The network is specified by BF16 weights and FP32 accumulation, so the
reference is oracle/mlp.py with bf="weights": BF16-rounded weights, everything else in
FP64.  The kernels also store the layer inputs (X, A1, A2) and the backward output
gradients (G3, G2, G1) in BF16 for the matrix cores; these are design choices the
specification does not fix, so the tolerance has to cover them.

Tolerances.  Rounding a vector to BF16 (round to nearest) perturbs every entry by at
most u = 2^-8 relative, hence normwise by at most u.  A layer with about unit gain
passes such a perturbation on unchanged and adds its own, so the network output
carries at most 3u (three forward rounding points) and the first layer's weight
gradient at most 6u (three forward, three backward); every other block has fewer.
FP32 accumulation adds about sqrt(K) 6e-8 <= 1e-5 for K <= 16287 terms.  The bounds
used are TOL_FWD = 3u = 1.2e-2 and TOL_GRAD = 6u = 2.3e-2 (measured: about 3e-3 and
5e-3).  The loss is a function of the output: |dL| / L <= 2 |dY| |Y - T| / |Y - T|^2
+ |dY|^2 / |Y - T|^2, evaluated with |dY| <= TOL_FWD |Y|.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp
from feti_helpers import require_gpu

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd import warmstart as WS  # noqa: E402
from paper_2509_06673_amd.workload import opts  # noqa: E402

U_BF16 = 2.0 ** -8
TOL_FWD = 3 * U_BF16
TOL_GRAD = 6 * U_BF16


def _net(n_in, h, n_out, batch, seed):
    import torch
    require_gpu()
    net = B.WarmStartNet(n_in, h, n_out, batch, torch.cuda.current_stream())
    p = W.mlp_init(n_in, h, n_out, seed=seed)
    # a non-trivial last layer and biases, so that every block of the gradient is exercised
    rng = np.random.default_rng(seed + 100)
    p = (p + 0.05 * rng.standard_normal(p.size)).astype(np.float32)
    net.set_params(torch.tensor(p, device="cuda"))
    return net, p


def _blocks(v, shapes):
    return mlp.unpack(v, shapes)


@pytest.mark.parametrize("dims", [(48, 32, 16, 8), (3 * 5429, 256, 5429, 16)], ids=["tiny", "cfg-shape"])
def test_forward_and_gradient_match_oracle(dims):
    import torch
    n_in, h, n_out, b = dims
    print(f"[ws grad] n_in {n_in} h {h} n_out {n_out} batch {b}", flush=True)
    net, p = _net(n_in, h, n_out, b, seed=11)
    shapes = mlp.sizes_of(n_in, h, n_out)
    X = W.seeded_matrix(b, n_in, seed=12).astype(np.float32)
    T = W.seeded_matrix(b, n_out, seed=13).astype(np.float32)
    xd, td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    y = torch.empty((b, n_out), dtype=torch.float32, device="cuda")
    net.forward(xd, b, y)
    Yref, _ = mlp.forward(p.astype(np.float64), shapes, X.astype(np.float64), bf="weights")
    ey = np.linalg.norm(y.cpu().numpy() - Yref) / np.linalg.norm(Yref)
    g = torch.empty(net.num_params(), dtype=torch.float32, device="cuda")
    loss = net.loss_grad(xd, td, b, g)
    lref, gref = mlp.loss_grad(p.astype(np.float64), shapes, X.astype(np.float64), T.astype(np.float64),
                               bf="weights")
    dyn = TOL_FWD * np.linalg.norm(Yref)
    ymt = np.linalg.norm(Yref - T.astype(np.float64))
    tol_loss = 2 * dyn / ymt + (dyn / ymt) ** 2
    errs = [np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)
            for a, r in zip(_blocks(g.cpu().numpy().astype(np.float64), shapes), _blocks(gref, shapes))]
    print(f"  forward rel err {ey:.2e}, loss {loss:.6e} vs {lref:.6e}, grad block errs "
          + " ".join(f"{e:.1e}" for e in errs), flush=True)
    assert ey < TOL_FWD
    assert abs(loss - lref) <= tol_loss * lref
    assert max(errs) < TOL_GRAD
    net.close()


def test_adam_steps_match_oracle():
    import torch
    n_in, h, n_out, b = 48, 32, 16, 8
    net, p = _net(n_in, h, n_out, b, seed=21)
    shapes = mlp.sizes_of(n_in, h, n_out)
    X = W.seeded_matrix(b, n_in, seed=22).astype(np.float32)
    T = W.seeded_matrix(b, n_out, seed=23).astype(np.float32)
    xd, td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    lr = 1e-3
    pr, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for k in range(1, 4):
        net.train_step(xd, td, b, lr)
        _, gr = mlp.loss_grad(pr, shapes, X.astype(np.float64), T.astype(np.float64), bf="weights")
        pr, m, v = mlp.adam_step(pr, gr, m, v, k, lr)
    got = torch.empty(p.size, dtype=torch.float32, device="cuda")
    net.get_params(got)
    moved = np.linalg.norm(pr - p)
    err = np.linalg.norm(got.cpu().numpy() - pr)
    print(f"[ws adam] parameters moved {moved:.3e}, GPU vs oracle {err:.3e}", flush=True)
    # Adam's first steps move every weight by about lr; an element whose gradient flips
    # sign between the two paths moves the other way, so the bound is relative to the move
    assert err <= 0.05 * moved
    net.close()


_LEARNED = {}


def _trained_and_evaluated():
    """One network trained on six short seeded trajectories (h = 1/32, 4 x 4 subdomains)
    and the held-out trajectory run with each start; shared by the tests below."""
    import torch
    if _LEARNED:
        return _LEARNED
    cases = [W.learned_start_case(s, nsteps=40, ncell=32).replace(nsub_x=4, nsub_y=4) for s in range(1, 7)]
    probe = WS.setup(cases[0])
    nl = probe.get_sizes()["n_lambda"]
    probe.close()
    net = B.WarmStartNet(3 * nl, WS.HIDDEN, nl, 32, torch.cuda.current_stream())
    net.set_params(torch.tensor(W.mlp_init(3 * nl, WS.HIDDEN, nl, seed=5), device="cuda"))
    print(f"[ws train] N_lambda {nl}: building samples ...", flush=True)
    X, T = WS.build_dataset(cases, 40, net)
    hist = WS.train(net, X, T, epochs=40, batch=32, lr=2e-3, seed=7)
    print(f"[ws train] {X.shape[0]} samples, loss {hist['loss'][0]:.3e} -> {hist['loss'][-1]:.3e} "
          f"in {hist['seconds']:.1f} s", flush=True)
    held = W.learned_start_case(1001, nsteps=30, ncell=32).replace(nsub_x=4, nsub_y=4)
    res = {m: WS.evaluate(held, net, 30, m) for m in ("previous", "extrapolate", "learned")}
    for m, r in res.items():
        print(f"  {m:11s}: first-solve iters {r['mean_iters_first']:.2f}, all iters {r['mean_iters']:.2f}, "
              f"{r['mean_ms']:.2f} ms/step, learned start kept {r['used_learned']}", flush=True)
    r = res["learned"]
    print(f"  start error vs the solved multipliers: prediction {r['mean_err_pred']:.3e}, previous step "
          f"{r['mean_err_prev']:.3e}, extrapolation {r['mean_err_extrap']:.3e}", flush=True)
    net.close()
    _LEARNED.update(hist=hist, res=res)
    return _LEARNED


def test_learned_start_predicts_better_than_the_previous_step():
    require_gpu()
    d = _trained_and_evaluated()
    assert d["hist"]["loss"][-1] < 0.5 * d["hist"]["loss"][0]
    r = d["res"]["learned"]
    # the network predicts the next multipliers better than the previous step does
    assert r["mean_err_pred"] < r["mean_err_prev"]
    assert r["used_learned"] > 0


@pytest.mark.xfail(strict=False, reason="measured: the learned start does not save first-solve iterations "
                   "over both the previous-step and the extrapolated start on these trajectories (the "
                   "iteration on the indefinite F responds weakly to the start's accuracy); kept to report "
                   "the gain if a later network or solver achieves one")
def test_learned_start_saves_first_solve_iterations():
    require_gpu()
    res = _trained_and_evaluated()["res"]
    best_plain = min(res["previous"]["mean_iters_first"], res["extrapolate"]["mean_iters_first"])
    assert res["learned"]["mean_iters_first"] < best_plain


def test_best_start_returns_the_same_solution():
    """The start changes the iterations, not the answer: a deliberately poor given start
    is rejected in favour of the previous step, and either way the fields agree."""
    import torch
    require_gpu()
    w = W.learned_start_case(2, nsteps=6, ncell=16).replace(nsub_x=4, nsub_y=4)
    sols = {}
    for mode in ("previous", "best_bad", "best_good"):
        f = WS.setup(w)
        nl = f.get_sizes()["n_lambda"]
        u = torch.empty(f.get_sizes()["sum_ns"], dtype=torch.float64, device="cuda")
        o = opts(tol=1e-10, max_it=2000)
        used = []
        for n in range(1, 7):
            if mode != "previous" and n > 1:
                lam = torch.empty(nl, dtype=torch.float64, device="cuda")
                f.get_solution(lam=lam)
                given = lam * 1e3 if mode == "best_bad" else lam
                f.set_start(given)
                o.start = B.START_BEST
            st = f.step(WS.load(w, n * w.tau), o)
            used.append(st["start_used"])
        f.get_solution(u)
        sols[mode] = u.cpu().numpy()
        if mode == "best_bad":
            assert all(s != B.START_GIVEN for s in used[1:]), used
        f.close()
    for mode in ("best_bad", "best_good"):
        d = np.abs(sols[mode] - sols["previous"]).max() / np.abs(sols["previous"]).max()
        assert d < 1e-8, (mode, d)
