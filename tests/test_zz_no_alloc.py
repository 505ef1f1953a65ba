"""The interface operator through the entry point that allocates nothing.

feti_apply_F_noalloc keeps its interface-space products in a static per-GPU device
array instead of the context's buffers.  Two calls in a row, the second on a smaller
problem (so the array holds the first call's larger contents when the second starts),
must each give exactly what feti_apply_F gives for the same context and input: the
same kernels run in the same order, so the comparison is bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from feti_helpers import require_gpu

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2509_06673_amd._binding")
from paper_2509_06673_amd.workload import mesh_args, material  # noqa: E402


def _factored(w):
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    f.assemble(material(w.mat_p), material(w.mat_e), w.tau)
    f.factor_subdomains(B.FP64, B.PRECOND_DIRICHLET)
    return f


def test_apply_F_without_allocation_matches_apply_F():
    torch = require_gpu()
    cases = [W.nearly_incompressible_scaled(32, 8), W.plain_fp64_small()]
    ctxs = [_factored(w) for w in cases]
    sizes = [c.get_sizes() for c in ctxs]
    assert sizes[1]["n_lambda"] < sizes[0]["n_lambda"]
    xs = [torch.tensor(np.random.default_rng(11 + k).standard_normal(s["n_lambda"]), device="cuda")
          for k, s in enumerate(sizes)]
    got = [torch.full_like(x, float("nan")) for x in xs]
    # two calls in a row, the second on the smaller problem
    for c, x, y in zip(ctxs, xs, got):
        print(f"[no-alloc] n_lambda {x.numel()}", flush=True)
        c.apply_F_noalloc(x, y)
    torch.cuda.synchronize()
    for c, x, y in zip(ctxs, xs, got):
        ref = torch.empty_like(x)
        c.apply_F(x, ref)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (x.numel(), (y - ref).abs().max().item())
    for c in ctxs:
        c.close()
