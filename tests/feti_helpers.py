"""Shared helpers of the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np

KIND_NAMES = {0: "ux", 1: "uy", 2: "eta", 3: "xiP", 4: "p", 5: "xiE", 6: "uz"}


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need an MI355X: torch.cuda.is_available() is False")
    return torch


def oracle_reference(w, nsteps, init="interp"):
    """Monolithic oracle trajectory; returns (system, list of lattice dicts)."""
    from oracle.monolithic import solve_steps
    tr = solve_steps(w, nsteps=nsteps, init=init)
    return tr.system, [tr.system.to_lattice(x) for x in tr.states]


_ORACLE_CACHE = {}


def cached_oracle_lattices(w, nsteps):
    """oracle_reference's lattices, kept for the test process: the monolithic solution does
    not depend on how the subdomains are glued, so the key leaves the coupling out, and a
    longer cached trajectory serves a shorter request."""
    key = repr(sorted(w.replace(coupling="dual").to_dict().items()))
    have = _ORACLE_CACHE.get(key)
    if have is None or len(have) < nsteps:
        have = oracle_reference(w, nsteps)[1]
        _ORACLE_CACHE[key] = have
    return have[:nsteps]


def torn_reference(codes, sub_offset, sub_poro, lat):
    """Oracle values at every torn local DOF (codes in torn order)."""
    out = np.empty(len(codes))
    kinds = codes % 8
    nodes = codes // 8
    sub_of = np.repeat(np.arange(len(sub_offset) - 1), np.diff(sub_offset))
    poro = np.asarray(sub_poro)[sub_of]
    for k in range(7):
        sel = kinds == k
        if not sel.any():
            continue
        if k < 2 or k == 6:
            a = lat[KIND_NAMES[k] + "_P"]
            b = lat[KIND_NAMES[k] + "_E"]
            out[sel] = np.where(poro[sel], a[nodes[sel]], b[nodes[sel]])
        else:
            out[sel] = lat[KIND_NAMES[k]][nodes[sel]]
    return out


def per_kind_rel_error(codes, got, ref):
    """max |got - ref| / max |ref| for each DOF kind present."""
    kinds = codes % 8
    res = {}
    for k in range(7):
        sel = kinds == k
        if not sel.any():
            continue
        scale = np.abs(ref[sel]).max()
        err = np.abs(got[sel] - ref[sel]).max()
        res[KIND_NAMES[k]] = err / scale if scale > 0 else err
    return res


def sub_poro_flags(w):
    from oracle import indexing as ix
    return [s.poro for s in ix.build(w).subs]
