"""Host-side checks of bench.py: the one-GPU contract and the algorithmic byte count its
roofline divides by, recomputed from the oracle's own numbering of the 64-subdomain
workload (interface sizes, multiplier rows, floating subdomains)."""
import os
import subprocess
import sys

import numpy as np

import workloads as W
from oracle import indexing as ix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_pcg_bytes_per_iteration_from_the_oracle_numbering():
    w = W.nearly_incompressible_large()
    spec = ix.build(w)
    # interface DOFs: the categories after the two interior ones of the local order
    nb = [int((np.asarray(s.cats) >= 2).sum()) for s in spec.subs]
    n_lambda = len(spec.rows)
    nc = 3 * sum(1 for s in spec.subs if s.floating)  # three rigid modes per floating subdomain (2D)
    assert (max(nb), n_lambda, nc) == (448, 10677, 108)
    b = bench.pcg_bytes_per_iteration(nb, n_lambda, nc, 8)
    # the interface blocks of F and of the preconditioner once each, the coarse inverse
    # twice, twelve multiplier passes: 2 x 8 x sum n_b^2 + 2 x 8 x 108^2 + 12 x 8 x 10677
    assert b == 16 * sum(n * n for n in nb) + 16 * 108 * 108 + 96 * 10677
    assert b == 117670464  # about 118 MB per iteration
