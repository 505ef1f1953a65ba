"""Learned warm start of the interface iteration (include/feti_ws.h), host driver.

Training data come from the plain solver's own trajectories: after each step the
multipliers lambda^n are kept, and a sample pairs the features
[lambda^n, lambda^{n-1}, load^{n+1} at the multiplier rows] with the target
lambda^{n+1} - 2 lambda^n + lambda^{n-1} (the network predicts the correction to
linear extrapolation).  Feature rows, targets, scaling, training and prediction
all run in the library's kernels; this module only orders the calls and moves
rows between device buffers.
"""
from __future__ import annotations

import time
from typing import Dict, List

import numpy as np

from . import _binding as B
from .workload import setup, load, opts as make_opts

HIDDEN = 256


def trajectory_samples(w, net: B.WarmStartNet, X, T, row0: int, nsteps: int, opts) -> int:
    """Run w for nsteps with the previous-step start; write samples from row0 on.
    Returns the number of samples written."""
    import torch
    f = setup(w)
    nl = f.get_sizes()["n_lambda"]
    lams: List = []
    for n in range(1, nsteps + 1):
        f.step(load(w, n * w.tau), opts)
        lam = torch.empty(nl, dtype=torch.float64, device="cuda")
        f.get_solution(lam=lam)
        lams.append(lam)
    ld = torch.empty(nl, dtype=torch.float64, device="cuda")
    row = row0
    # sample for step n + 1 from lambda^n, lambda^{n-1} (1-based steps n >= 2)
    for n in range(2, nsteps):
        f.interface_load(load(w, (n + 1) * w.tau), ld)
        net.make_features(nl, lams[n - 1], lams[n - 2], ld, X[row])
        net.make_target(nl, lams[n], lams[n - 1], lams[n - 2], T[row])
        row += 1
    torch.cuda.synchronize()
    f.close()
    return row - row0


def build_dataset(cases, nsteps: int, net: B.WarmStartNet):
    """Samples of every case (a list of workloads) into device matrices X, T."""
    import torch
    per = nsteps - 2
    X = torch.empty((len(cases) * per, net.n_in), dtype=torch.float32, device="cuda")
    T = torch.empty((len(cases) * per, net.n_out), dtype=torch.float32, device="cuda")
    o = make_opts(tol=1e-10, max_it=3000)
    row = 0
    for w in cases:
        row += trajectory_samples(w, net, X, T, row, nsteps, o)
    return X[:row], T[:row]


def train(net: B.WarmStartNet, X, T, epochs: int = 30, batch: int = 64, lr: float = 1e-3,
          seed: int = 0) -> Dict:
    """Fit the scaling, then Adam over shuffled mini-batches (seeded order) with a
    cosine learning-rate decay.  Returns the loss history per epoch."""
    import torch
    ns = X.shape[0]
    net.fit_scaling(X, T, ns)
    rng = np.random.default_rng(seed)
    nb = max(1, ns // batch)
    total = epochs * nb
    hist = []
    t0 = time.perf_counter()
    k = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(ns)).to("cuda")
        losses = []
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            lr_k = lr * 0.5 * (1.0 + np.cos(np.pi * k / total))
            last = b == nb - 1
            loss = net.train_step(xb, tb, len(idx), float(lr_k), want_loss=last)
            if last:
                losses.append(loss)
            k += 1
        hist.append(float(np.mean(losses)))
    torch.cuda.synchronize()
    return {"loss": hist, "seconds": time.perf_counter() - t0, "steps": total}


def evaluate(w, net, nsteps: int, mode: str, opts=None, precision: int = B.FP64) -> Dict:
    """Held-out trajectory with one start: 'previous', 'extrapolate' or 'learned' (the
    prediction, kept only when its projected residual beats the previous-step start).
    precision: FP64 factors, or FP32 factors with FP64 refinement (FP32_IR, with the
    refinement defaults of workload.opts_mixed unless opts is given).  Time per step
    covers the prediction and the step (stream events)."""
    import torch
    from .workload import opts_mixed
    f = setup(w, precision=precision)
    nl = f.get_sizes()["n_lambda"]
    if opts is not None:
        o = opts
    else:
        o = (opts_mixed if precision == B.FP32_IR else make_opts)(tol=1e-10, max_it=3000)
    lam_hist: List = []
    pred = torch.empty(nl, dtype=torch.float64, device="cuda")
    ld = torch.empty(nl, dtype=torch.float64, device="cuda")
    rec = {"iters": [], "iters_first": [], "ms": [], "used_learned": 0, "err_pred": [], "err_prev": [],
           "err_extrap": []}
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for n in range(1, nsteps + 1):
        t = n * w.tau
        ev0.record(stream)
        if mode == "learned" and len(lam_hist) >= 2:
            f.interface_load(load(w, t), ld)
            net.predict(lam_hist[-1], lam_hist[-2], ld, pred)
            f.set_start(pred)
            o.start = B.START_BEST
        elif mode == "extrapolate":
            o.start = B.START_EXTRAPOLATE
        else:
            o.start = B.START_PREVIOUS
        st = f.step(load(w, t), o)
        ev1.record(stream)
        torch.cuda.synchronize()
        lam = torch.empty(nl, dtype=torch.float64, device="cuda")
        f.get_solution(lam=lam)
        if mode == "learned" and len(lam_hist) >= 2:
            # distance of each start to the multipliers the step solved for
            nrm = float(torch.linalg.norm(lam))
            rec["err_pred"].append(float(torch.linalg.norm(pred - lam)) / nrm)
            rec["err_prev"].append(float(torch.linalg.norm(lam_hist[-1] - lam)) / nrm)
            rec["err_extrap"].append(float(torch.linalg.norm(2 * lam_hist[-1] - lam_hist[-2] - lam)) / nrm)
        lam_hist = (lam_hist + [lam])[-2:]
        if n >= 3:  # every mode has two previous steps from here on
            rec["iters"].append(st["iters"])
            rec["iters_first"].append(st["iters_first"])
            rec["ms"].append(ev0.elapsed_time(ev1))
            rec["used_learned"] += int(st["start_used"] == B.START_GIVEN)
    f.close()
    rec["mean_iters"] = float(np.mean(rec["iters"]))
    rec["mean_iters_first"] = float(np.mean(rec["iters_first"]))
    rec["mean_ms"] = float(np.mean(rec["ms"]))
    for k in ("err_pred", "err_prev", "err_extrap"):
        rec["mean_" + k] = float(np.mean(rec[k])) if rec[k] else float("nan")
    return rec
