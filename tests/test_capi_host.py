"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every function include/feti.h and
  include/feti_ws.h declare, and the binding covers each;
* the numbering built by the library's host code equals, bit for bit, the
  independent statement in oracle/indexing.py (local DOF codes and order,
  interface sizes, the two entries and signs of every jump row);
* out-of-order calls and invalid descriptions return the documented codes.
"""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import indexing as ix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

P = pytest.importorskip("paper_2509_06673_amd")
from paper_2509_06673_amd import _binding as B  # noqa: E402
from paper_2509_06673_amd.workload import mesh_args  # noqa: E402


def _declared_functions(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(feti_[a-z_A-Z0-9]+)\s*\(", src)))


@pytest.mark.parametrize("header,least", [("feti.h", 15), ("feti_ws.h", 12)])
def test_library_exports_every_declared_symbol(header, least):
    lib = B.load_library()
    names = _declared_functions(header)
    assert len(names) >= least
    for n in names:
        assert hasattr(lib, n), n
        assert n in B._SIGS or n.endswith("last_error"), f"{n} has no binding"


def _compare(w):
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    got = f.export_indexing()
    spec = ix.build(w)
    codes = np.concatenate([np.array(s.codes, dtype=np.int64) for s in spec.subs])
    assert np.array_equal(got["code"].astype(np.int64), codes)
    offs = np.concatenate([[0], np.cumsum([len(s.codes) for s in spec.subs])])
    assert np.array_equal(got["sub_offset"], offs)
    nb = np.array([sum(1 for c in s.cats if c >= 2) for s in spec.subs])
    assert np.array_equal(got["sub_nb"], nb)
    rows = spec.rows.reshape(-1, 3)
    assert np.array_equal(got["brow_sub"], rows[:, 0])
    assert np.array_equal(got["brow_local"], rows[:, 1])
    assert np.array_equal(got["brow_sign"].astype(np.int64), rows[:, 2])
    # interface DOFs are the trailing ones of each subdomain
    for s, n_b in zip(spec.subs, nb):
        assert all(c >= 2 for c in s.cats[len(s.cats) - n_b:])
    sz = f.get_sizes()
    assert sz["n_lambda"] == spec.n_lambda
    assert sz["n_float"] == sum(s.floating for s in spec.subs)
    if w.coupling == "primal":
        pr = f.export_primal()
        assert np.array_equal(pr["code"].astype(np.int64), spec.primal)
        assert np.array_equal(pr["sub_npi"], [sum(1 for c in s.cats if c == 3) for s in spec.subs])
        assert sz["n_primal"] == len(spec.primal)
    else:
        assert sz["n_primal"] == 0
    f.close()


@pytest.mark.parametrize("w", [
    W.plain_fp64_small(),
    W.nearly_incompressible_scaled(16, 4),
    W.nearly_incompressible_scaled(24, 4).replace(nsub_y=3),
    W.patch_case(order_u=1, ncell=8, nsub_x=4, nsub_y=3),
    W.paper_table_case(2, 8, 0.3, nsteps=1),
    W.pulsed_core(ncell=16, nsub=4, nsteps=1),
    W.learned_start_case(1, nsteps=1),
], ids=lambda w: w.name)
def test_indexing_bit_exact_against_oracle(w):
    _compare(w)


@pytest.mark.parametrize("w", [
    W.nearly_incompressible_scaled(16, 4).replace(scheme="decoupled"),
    W.pulsed_core(ncell=16, nsub=4, nsteps=1).replace(scheme="decoupled"),
    W.patch_case(order_u=1, ncell=8, nsub_x=4, nsub_y=3).replace(scheme="decoupled"),
], ids=lambda w: w.name + "_decoupled")
def test_decoupled_indexing_bit_exact_against_oracle(w):
    """The decoupled scheme leaves eta and p out of the subdomain unknowns: the numbering
    (and with it every jump row) against the oracle's statement of the same rule."""
    _compare(w)


@pytest.mark.parametrize("w", [
    W.plain_fp64_small().replace(coupling="primal"),
    W.nearly_incompressible_scaled(16, 4).replace(coupling="primal"),
    W.nearly_incompressible_scaled(24, 4).replace(nsub_y=3, coupling="primal"),
    W.patch_case(order_u=1, ncell=8, nsub_x=4, nsub_y=3).replace(coupling="primal"),
    W.pulsed_core(ncell=16, nsub=4, nsteps=1).replace(coupling="primal"),
    W.nearly_incompressible_scaled(24, 4).replace(coupling="primal", cut_x=(0, 5, 12, 20, 24), layout=W.XSPLIT),
    W.nearly_incompressible_scaled(16, 4).replace(coupling="primal", scheme="decoupled", name="xsplit_h16_decoupled"),
], ids=lambda w: w.name + "_primal")
def test_dual_primal_indexing_bit_exact_against_oracle(w):
    """Dual-primal coupling: local orders (primal DOFs trailing), the jump rows of the dual
    DOFs and the global primal order against the oracle's statement of the same rule."""
    _compare(w)


@pytest.mark.parametrize("w", [
    W.cube_case(ncell=4),
    W.cube_case(ncell=4, order_u=1, nsub=(2, 1, 3)),
    W.cube_case(ncell=8, nsub=(4, 2, 2)),
    W.cube_nearly_incompressible(),
], ids=lambda w: w.name)
def test_3d_indexing_bit_exact_against_oracle(w):
    """d = 3: local orders, jump rows (up to four owners on the grid edges) and the primal
    order (up to eight owners at the grid corners) against the oracle's statement."""
    _compare(w)


@pytest.mark.parametrize("w", [
    W.nearly_incompressible_scaled(16, 4).replace(coupling="primal", dirichlet_u=0),
    W.nearly_incompressible_scaled(12, 4).replace(coupling="primal", order_u=1, nsub_y=3, dirichlet_u=0),
    W.nearly_incompressible_scaled(24, 4).replace(coupling="primal", cut_x=(0, 5, 12, 20, 24), dirichlet_u=0),
    W.cube_case(ncell=4).replace(dirichlet_u=0),
    W.cube_case(ncell=8, nsub=(4, 2, 2)).replace(dirichlet_u=0),
    W.cube_case(ncell=6, nsub=(2, 3, 2)).replace(dirichlet_u=0),
], ids=lambda w: w.name + ("_primal" if w.dim == 2 else ""))
def test_deflation_vectors_integrate_the_normal_jump(w):
    """q_c^T B u is the integral over face c of the jump of u . n (sign of the pair's rows),
    for displacements that are a different quadratic polynomial in every subdomain (linear
    for P1), reproduced exactly by the nodal values: checked against the analytic face
    integrals.  Without displacement Dirichlet data every face node is a dual unknown but
    the primal grid corners; those carry no multiplier (their jump vanishes in the
    dual-primal coupling), so their share of the integral is taken off (2D: h/6 at each end
    of an edge for P2, h/2 for P1; 3D P2: the corners are triangle vertices, whose P2 basis
    functions integrate to zero over the face)."""
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    dfl = f.export_deflation()
    spec = ix.build(w)
    d3 = w.dim == 3
    n, r = w.ncell, (2 if w.order_u == 2 else 1)
    mu = r * n + 1
    rng = np.random.default_rng(5)
    quad = w.order_u == 2
    coef = rng.standard_normal((len(spec.subs), 3, 10))

    def u_of(s, c, x):
        a = coef[s, c]
        v = a[0] + a[1] * x[0] + a[2] * x[1] + a[3] * x[2]
        if quad:
            v = v + a[4] * x[0] ** 2 + a[5] * x[1] ** 2 + a[6] * x[2] ** 2 + a[7] * x[0] * x[1] + \
                a[8] * x[0] * x[2] + a[9] * x[1] * x[2]
        return v
    comp_of = {0: 0, 1: 1, 6: 2}
    rows = spec.rows
    jump = np.zeros(spec.n_lambda)
    for j, (row, code) in enumerate(zip(rows, spec.row_code)):
        node, kind = int(code) // 8, int(code) % 8
        if kind not in comp_of:
            continue
        x = np.array([node % mu, (node // mu) % mu if d3 else node // mu, node // (mu * mu) if d3 else 0]) / float(r * n)
        jump[j] = sum(sg * u_of(s, comp_of[kind], x) for s, _, sg in row)
    cols, wts, nd = dfl["col"], dfl["w"], dfl["n_defl"]
    assert nd > 0 and cols.max() == nd - 1
    unit = (1.0 / n) if not d3 else 0.5 / n ** 2
    got = np.zeros(nd)
    for slot in range(2):
        sel = cols[:, slot] >= 0
        np.add.at(got, cols[sel, slot], wts[sel, slot] * jump[sel] * unit)
    g, gw = np.polynomial.legendre.leggauss(4)
    seen = set()
    nsx, nsy = w.nsub_x, w.nsub_y

    def grid(sid):
        return (sid % nsx, (sid // nsx) % nsy, sid // (nsx * nsy)) if d3 else (sid % nsx, sid // nsx, 0)

    def own_pair(j):
        # a row of the face pair itself: the two subdomains differ along the row's component axis only
        (a, _, _), (b, _, _) = rows[j]
        axis = comp_of[int(spec.row_code[j]) % 8]
        diff = [q for q in range(3) if grid(a)[q] != grid(b)[q]]
        return diff == [axis]
    for c in range(nd):
        js = np.nonzero((cols == c).any(axis=1))[0]
        direct = [j for j in js if own_pair(j)]
        (s1, _, g1), (s2, _, g2) = rows[direct[0]]
        seen.add((min(s1, s2), max(s1, s2)))
        axis = comp_of[int(spec.row_code[direct[0]]) % 8]
        A, Bs = spec.subs[s1], spec.subs[s2]
        lo = [max(A.i0, Bs.i0), max(A.j0, Bs.j0), max(A.k0, Bs.k0)]
        hi = [min(A.i1, Bs.i1), min(A.j1, Bs.j1), min(A.k1, Bs.k1)]
        inpl = [q for q in range(3 if d3 else 2) if q != axis]
        grids = [((hi[q] - lo[q]) / n * 0.5 * (g + 1) + lo[q] / n, (hi[q] - lo[q]) / n * 0.5 * gw) for q in inpl]
        pts = np.meshgrid(*[gq for gq, _ in grids], indexing="ij")
        wq = np.ones_like(pts[0])
        for k, (_, gwk) in enumerate(grids):
            shape = [1] * len(grids)
            shape[k] = -1
            wq = wq * gwk.reshape(shape)
        x = [None, None, None]
        x[axis] = np.full(pts[0].shape, lo[axis] / n)
        for k, q in enumerate(inpl):
            x[q] = pts[k]
        if not d3:
            x[2] = np.zeros(pts[0].shape)
        exp = np.sum(wq * (g1 * u_of(s1, axis, x) + g2 * u_of(s2, axis, x)))
        if not d3:
            t = inpl[0]
            for end in (lo[t], hi[t]):
                xe = [0.0, 0.0, 0.0]
                xe[axis] = lo[axis] / n
                xe[t] = end / n
                exp -= (1.0 / (6 * n) if quad else 0.5 / n) * (g1 * u_of(s1, axis, xe) + g2 * u_of(s2, axis, xe))
        assert abs(got[c] - exp) <= 1e-12 * max(1.0, abs(exp)), (c, got[c], exp)
    assert len(seen) == nd
    f.close()


def test_3d_takes_the_dual_primal_coupling_only():
    f = B.Feti()
    with pytest.raises(B.FetiError) as e:
        f.setup_mesh(**mesh_args(W.cube_case(ncell=4).replace(coupling="dual")))
    assert e.value.code == B.EINVAL
    f.close()


def test_decoupled_subdomains_balance():
    """With eta and p out, a poroelastic subdomain carries (u, xi_P) like an elastic one
    (u, xi_E): the same size for the same cells (the point of the decoupling)."""
    w = W.nearly_incompressible_scaled(32, 4).replace(scheme="decoupled")
    f = B.Feti()
    f.setup_mesh(**mesh_args(w))
    ix_ = f.export_indexing()
    ns = np.diff(ix_["sub_offset"])
    spec = ix.build(w)
    poro = np.array([s.poro for s in spec.subs])
    # mirror pairs across x = 1/2 (columns a and 3 - a of a 4 x 4 grid) have the same size
    for b in range(4):
        for a in range(2):
            assert ns[b * 4 + a] == ns[b * 4 + 3 - a] and poro[b * 4 + a] and not poro[b * 4 + 3 - a]
    f.close()


def test_unknown_scheme_is_rejected():
    f = B.Feti()
    with pytest.raises(B.FetiError) as e:
        f.setup_mesh(ncell=8, order_u=2, layout=0, nsub_x=2, nsub_y=1, scheme=7)
    assert e.value.code == B.EINVAL
    f.close()


def test_uneven_cuts_bit_exact():
    # ncell not divisible by the grid: cuts at floor(a n / nsub)
    w = W.nearly_incompressible_scaled(20, 4).replace(nsub_y=3, ncell=20)
    _compare(w)


def test_caller_cuts_bit_exact():
    # cuts given by the caller (uneven, x = 1/2 kept as a cut for the x-split layout)
    w = W.nearly_incompressible_scaled(24, 4).replace(nsub_x=4, nsub_y=3, cut_x=(0, 3, 12, 20, 24),
                                                      cut_y=(0, 10, 13, 24))
    _compare(w)
    w = W.pulsed_core(ncell=16, nsub=4, nsteps=1).replace(cut_x=(0, 4, 9, 12, 16), cut_y=(0, 4, 5, 12, 16))
    _compare(w)


def test_invalid_cuts_are_rejected():
    for cx in ((0, 4, 4, 8), (1, 2, 5, 8), (0, 2, 5, 7), (0, 3, 5, 8)):
        f = B.Feti()
        with pytest.raises(B.FetiError) as e:
            # the last tuple straddles x = 1/2 in the x-split layout
            f.setup_mesh(ncell=8, order_u=2, layout=0, nsub_x=3, nsub_y=1, cut_x=cx)
        assert e.value.code == B.EINVAL
        f.close()


def test_full_size_counts():
    f = B.Feti()
    f.setup_mesh(**mesh_args(W.nearly_incompressible_large()))
    sz = f.get_sizes()
    assert sz["n_lambda"] == 10677 and sz["max_ns"] == 3045 and sz["max_nb"] == 448
    assert sz["n_float"] == 36 and sz["n_c"] == 108


def test_call_order_and_invalid_input():
    f = B.Feti()
    with pytest.raises(B.FetiError) as e:
        f.assemble(B.Material(1, 0.3, 1, 1, 1, 1, 0), B.Material(1, 0.3, 1, 1, 1, 1, 0), 0.1)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.FetiError) as e:
        f.setup_mesh(ncell=8, order_u=3, layout=0, nsub_x=2, nsub_y=1)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.FetiError) as e:
        # a subdomain straddling x = 1/2
        f.setup_mesh(ncell=8, order_u=2, layout=0, nsub_x=3, nsub_y=1)
    assert e.value.code == B.EINVAL
    f.setup_mesh(ncell=8, order_u=2, layout=0, nsub_x=2, nsub_y=2)
    with pytest.raises(B.FetiError) as e:
        f.setup_mesh(ncell=8, order_u=2, layout=0, nsub_x=2, nsub_y=2)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.FetiError) as e:
        f.factor_subdomains()
    assert e.value.code == B.ESTATE
    # nu >= 1/2 is rejected before any device work
    with pytest.raises(B.FetiError) as e:
        f.assemble(B.Material(1, 0.5, 1, 1, 1, 1, 0), B.Material(1, 0.3, 1, 1, 1, 1, 0), 0.1)
    assert e.value.code == B.EINVAL


def test_binding_structs_match_the_c_layout(tmp_path):
    """Every struct of the ctypes binding has the size and field offsets that a C
    compiler gives the header's typedef (compiled here with gcc)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_2509_06673_amd import _binding as Bd
    pairs = {"feti_mesh_desc": Bd.MeshDesc, "feti_material": Bd.Material, "feti_load": Bd.Load,
             "feti_solve_opts": Bd.SolveOpts, "feti_stats": Bd.Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "feti.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
