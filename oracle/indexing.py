"""Independent statement of the subdomain numbering and the jump maps B_s.

Oracle module (test infrastructure only).  The HIP path's host code builds
the same objects from its own implementation; the tests compare the two
bit for bit.

The paper tears the domain into the two physics regions and glues the
displacement on the interface with a Lagrange multiplier (Section 3.1,
eq. (linalg-system-reformulated)); the multiplier space is represented here
by nodal multipliers, so each multiplier row of the jump operator has one +1
and one -1.  For more than two subdomains every C0 field is glued at every
shared node: u everywhere, eta / xi_P / p between poroelastic subdomains and
xi_E between elastic ones.  A node shared by m subdomains carries m-1
multipliers, chaining the subdomains in increasing id order.

Numbering
---------
* Subdomain s = b*nsub_x + a covers cells [cx[a], cx[a+1]) x [cy[b], cy[b+1])
  with cx[a] = floor(a * ncell / nsub_x) (same for y), or the workload's own cuts
  (Workload.cut_x / cut_y) when it gives them.  Every subdomain lies in
  one physics region.
* DOF kinds: 0 ux, 1 uy, 2 eta, 3 xi_P, 4 p, 5 xi_E.  A DOF is identified by
  code = 8 * lattice_node + kind (displacement lattice for kinds 0, 1, the P1
  lattice otherwise).  Dirichlet DOFs are not unknowns.
* A local DOF is an interface DOF (set b) when another subdomain has the same
  code; otherwise interior (set I).  Categories: 0 interior U (u, eta),
  1 interior P (xi, p), 2 interface U, 3 interface P, 4 fixed.
* A subdomain whose closure holds no Dirichlet displacement node is floating.
  Its fixed DOFs are ux, uy at the lower-left closure corner and ux at the
  upper-right corner; they are interface DOFs kept out of the local
  elimination.
* Local order: sort by (category, field order, node, component) with field
  order u 0, eta 1, xi 2, p 3 and component 0/1 for ux/uy.
* Dual-primal gluing (Workload.coupling == "primal"): a shared code is primal when
  its kind is xi_P, p or xi_E, or when its node sits at a corner of the subdomain
  grid (on a vertical and a horizontal cut line, the outer sides counted); the
  other shared codes (u and eta on the cut edges) are dual.  Categories then read
  2 dual interface DOF, 3 primal interface DOF, and no subdomain floats: the
  primal corners hold every subdomain that has no Dirichlet node.
* Multiplier rows: for each shared code (each dual code under dual-primal
  gluing), with S the sorted subdomains having it, one row per consecutive pair (S[k], S[k+1]) with sign +1 on S[k] and -1
  on S[k+1], except that a poroelastic/elastic pair puts +1 on the poroelastic
  side (the sign of H_P in eq. (linalg-system)).  Rows are sorted by
  (kind, node, k).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from workloads import Workload, XSPLIT, YSPLIT, CORE

KIND_FIELD_ORDER = {0: 0, 1: 0, 2: 1, 3: 2, 4: 3, 5: 2, 6: 0}
U_KINDS = (0, 1, 2, 6)
KIND_COMP = {0: 0, 1: 1, 6: 2}      # displacement component of a u kind (uz: kind 6, 3D)


def _region_poro(layout, xc, yc):
    if layout == XSPLIT:
        return xc < 0.5
    if layout == YSPLIT:
        return yc < 0.5
    if layout == CORE:
        return (xc > 0.25) & (xc < 0.75) & (yc > 0.25) & (yc < 0.75)
    raise ValueError(layout)


def _sides(i, j, nmax, mask):
    out = False
    if mask & 1 and i == 0:
        out = True
    if mask & 2 and i == nmax:
        out = True
    if mask & 4 and j == 0:
        out = True
    if mask & 8 and j == nmax:
        out = True
    return out


@dataclass
class Sub:
    sid: int
    poro: bool
    i0: int
    i1: int
    j0: int
    j1: int
    codes: List[int]        # local order
    cats: List[int]
    floating: bool
    k0: int = 0             # 3D: cell range in z
    k1: int = 0


@dataclass
class IndexSpec:
    subs: List[Sub]
    rows: np.ndarray        # (N_lambda, 2, 3): (sub, local index, sign) for the two entries
    row_code: np.ndarray    # (N_lambda,) code of the glued DOF
    mult: np.ndarray        # (N_lambda,) number of subdomains sharing the DOF
    primal: np.ndarray = None  # dual-primal gluing: the primal codes, in their global order

    @property
    def n_lambda(self):
        return len(self.rows)


def build(w: Workload) -> IndexSpec:
    if w.dim == 3:
        return build3d(w)
    n = w.ncell
    k = w.order_u
    ratio = 1 if k == 1 else 2
    nu = ratio * n              # max displacement lattice index
    mu = nu + 1
    cx, cy = w.cuts()
    subs = []
    owners = {}   # code -> list of subdomain ids
    local_sets = []
    for b in range(w.nsub_y):
        for a in range(w.nsub_x):
            sid = b * w.nsub_x + a
            i0, i1, j0, j1 = cx[a], cx[a + 1], cy[b], cy[b + 1]
            xs = (np.arange(i0, i1) + 0.5) / n
            ys = (np.arange(j0, j1) + 0.5) / n
            XC, YC = np.meshgrid(xs, ys)
            reg = _region_poro(w.layout, XC, YC)
            if not (reg.all() or (~reg).all()):
                raise ValueError(f"subdomain {sid} straddles the interface")
            poro = bool(reg.all())
            codes = []
            has_dir = False
            for J in range(ratio * j0, ratio * j1 + 1):
                for I in range(ratio * i0, ratio * i1 + 1):
                    if _sides(I, J, nu, w.dirichlet_u):
                        has_dir = True
                        continue
                    node = J * mu + I
                    codes += [8 * node + 0, 8 * node + 1]
            for j in range(j0, j1 + 1):
                for i in range(i0, i1 + 1):
                    node = j * (n + 1) + i
                    if poro:
                        if w.scheme == "decoupled":
                            # eta and p are not unknowns of the subdomain problems
                            codes.append(8 * node + 3)
                        else:
                            codes += [8 * node + 2, 8 * node + 3]
                            if not _sides(i, j, n, w.dirichlet_p):
                                codes.append(8 * node + 4)
                    else:
                        codes.append(8 * node + 5)
            for c in codes:
                owners.setdefault(c, []).append(sid)
            local_sets.append((sid, poro, i0, i1, j0, j1, codes, not has_dir))
    dp = w.coupling == "primal"
    if w.coupling not in ("dual", "primal"):
        raise ValueError(w.coupling)
    cxs, cys = set(cx), set(cy)

    def is_primal(c):
        node, kind = c // 8, c % 8
        if kind not in U_KINDS:
            return True
        if kind == 2:      # eta: P1 lattice
            i, j = node % (n + 1), node // (n + 1)
            return i in cxs and j in cys
        I, J = node % mu, node // mu
        return I % ratio == 0 and J % ratio == 0 and I // ratio in cxs and J // ratio in cys

    for sid, poro, i0, i1, j0, j1, codes, floating in local_sets:
        fixed = set()
        if dp:
            floating = False
        if floating:
            A = (ratio * j0) * mu + ratio * i0
            C = (ratio * j1) * mu + ratio * i1
            fixed = {8 * A + 0, 8 * A + 1, 8 * C + 0}
        keyed = []
        for c in codes:
            node, kind = c // 8, c % 8
            shared = len(owners[c]) > 1
            if c in fixed:
                cat = 4
            elif dp:
                cat = (3 if is_primal(c) else 2) if shared else (0 if kind in U_KINDS else 1)
            elif kind in U_KINDS:
                cat = 2 if shared else 0
            else:
                cat = 3 if shared else 1
            comp = 1 if kind == 1 else 0
            keyed.append(((cat, KIND_FIELD_ORDER[kind], node, comp), c, cat))
        keyed.sort()
        subs.append(Sub(sid, poro, i0, i1, j0, j1, [c for _, c, _ in keyed],
                        [ct for _, _, ct in keyed], floating))
    pos = [dict((c, i) for i, c in enumerate(s.codes)) for s in subs]
    rows = []
    for c in sorted(owners, key=lambda c: (c % 8, c // 8)):
        S = sorted(owners[c])
        if len(S) < 2 or (dp and is_primal(c)):
            continue
        for kk in range(len(S) - 1):
            s1, s2 = S[kk], S[kk + 1]
            sg1, sg2 = 1, -1
            if subs[s1].poro != subs[s2].poro and not subs[s1].poro:
                sg1, sg2 = -1, 1
            rows.append(((c % 8, c // 8, kk), c, len(S),
                         ((s1, pos[s1][c], sg1), (s2, pos[s2][c], sg2))))
    rows.sort(key=lambda r: r[0])
    R = np.array([r[3] for r in rows], dtype=np.int64).reshape(-1, 2, 3)
    primal = None
    if dp:
        # global primal order: (field order, node, kind), so the U-type corners (u, eta)
        # come before the P-type fields (xi, p)
        pc = [c for c in owners if len(owners[c]) > 1 and is_primal(c)]
        primal = np.array(sorted(pc, key=lambda c: (KIND_FIELD_ORDER[c % 8], c // 8, c % 8)), dtype=np.int64)
    return IndexSpec(subs, R, np.array([r[1] for r in rows], dtype=np.int64),
                     np.array([r[2] for r in rows], dtype=np.int64), primal)


def build3d(w: Workload) -> IndexSpec:
    """The numbering on the unit cube (d = 3): subdomain s = (c nsub_y + b) nsub_x + a
    covers the cells [cx[a], cx[a+1]) x [cy[b], cy[b+1]) x [cz[c], cz[c+1]) at the even cuts;
    lattices x fastest, then y, then z; displacement kinds ux 0, uy 1, uz 6 (components
    0, 1, 2), the scalar kinds as in 2D; outer faces (bit 0: x = 0, 1: x = 1, 2: y = 0,
    3: y = 1, 4: z = 0, 5: z = 1).  Only the dual-primal gluing: the shared xi / p DOFs
    and the shared DOFs at the corners of the subdomain grid are primal, the other shared
    DOFs (u and eta on the grid's faces and edges, two or four owners) dual, with the
    rows, signs, local order and primal order of the 2D rules."""
    if w.coupling != "primal" or w.layout != XSPLIT or w.scheme != "coupled":
        raise ValueError("3D takes the x-split layout, the coupled scheme and the dual-primal gluing")
    n = w.ncell
    ratio = 1 if w.order_u == 1 else 2
    mu = ratio * n + 1
    n1 = n + 1
    cuts = [[(a * n) // ns for a in range(ns + 1)] for ns in (w.nsub_x, w.nsub_y, w.nsub_z)]
    cx, cy, cz = cuts
    if n % 2 or n // 2 not in cx:
        raise ValueError("a subdomain straddles the interface x = 1/2")

    def face(I, J, K, m, mask):
        return any((mask >> bit) & 1 and hit for bit, hit in
                   enumerate((I == 0, I == m - 1, J == 0, J == m - 1, K == 0, K == m - 1)))
    owners, local_sets = {}, []
    for c in range(w.nsub_z):
        for b in range(w.nsub_y):
            for a in range(w.nsub_x):
                sid = (c * w.nsub_y + b) * w.nsub_x + a
                i0, i1, j0, j1, k0, k1 = cx[a], cx[a + 1], cy[b], cy[b + 1], cz[c], cz[c + 1]
                poro = (i0 + i1) < n            # the cell block lies in x < 1/2
                codes, has_dir = [], False
                for K in range(ratio * k0, ratio * k1 + 1):
                    for J in range(ratio * j0, ratio * j1 + 1):
                        for I in range(ratio * i0, ratio * i1 + 1):
                            if face(I, J, K, mu, w.dirichlet_u):
                                has_dir = True
                                continue
                            node = (K * mu + J) * mu + I
                            codes += [8 * node + 0, 8 * node + 1, 8 * node + 6]
                for k in range(k0, k1 + 1):
                    for j in range(j0, j1 + 1):
                        for i in range(i0, i1 + 1):
                            node = (k * n1 + j) * n1 + i
                            if poro:
                                codes += [8 * node + 2, 8 * node + 3]
                                if not face(i, j, k, n1, w.dirichlet_p):
                                    codes.append(8 * node + 4)
                            else:
                                codes.append(8 * node + 5)
                for cd in codes:
                    owners.setdefault(cd, []).append(sid)
                local_sets.append((sid, poro, i0, i1, j0, j1, k0, k1, codes, has_dir))
    sx, sy, sz = set(cx), set(cy), set(cz)

    def is_primal(cd):
        node, kind = cd // 8, cd % 8
        if kind not in U_KINDS:
            return True
        if kind == 2:
            i, j, k = node % n1, (node // n1) % n1, node // (n1 * n1)
            return i in sx and j in sy and k in sz
        I, J, K = node % mu, (node // mu) % mu, node // (mu * mu)
        return (I % ratio == 0 and J % ratio == 0 and K % ratio == 0 and I // ratio in sx
                and J // ratio in sy and K // ratio in sz)
    subs = []
    for sid, poro, i0, i1, j0, j1, k0, k1, codes, has_dir in local_sets:
        keyed = []
        for cd in codes:
            node, kind = cd // 8, cd % 8
            shared = len(owners[cd]) > 1
            cat = (3 if is_primal(cd) else 2) if shared else (0 if kind in U_KINDS else 1)
            keyed.append(((cat, KIND_FIELD_ORDER[kind], node, KIND_COMP.get(kind, 0)), cd, cat))
        keyed.sort()
        subs.append(Sub(sid, poro, i0, i1, j0, j1, [cd for _, cd, _ in keyed], [ct for _, _, ct in keyed],
                        False, k0, k1))
    pos = [dict((cd, i) for i, cd in enumerate(s.codes)) for s in subs]
    rows = []
    for cd in sorted(owners, key=lambda q: (q % 8, q // 8)):
        S = sorted(owners[cd])
        if len(S) < 2 or is_primal(cd):
            continue
        for kk in range(len(S) - 1):
            s1, s2 = S[kk], S[kk + 1]
            sg1, sg2 = 1, -1
            if subs[s1].poro != subs[s2].poro and not subs[s1].poro:
                sg1, sg2 = -1, 1
            rows.append(((cd % 8, cd // 8, kk), cd, len(S), ((s1, pos[s1][cd], sg1), (s2, pos[s2][cd], sg2))))
    rows.sort(key=lambda r: r[0])
    R = np.array([r[3] for r in rows], dtype=np.int64).reshape(-1, 2, 3)
    pc = [cd for cd in owners if len(owners[cd]) > 1 and is_primal(cd)]
    primal = np.array(sorted(pc, key=lambda q: (KIND_FIELD_ORDER[q % 8], q // 8, q % 8)), dtype=np.int64)
    return IndexSpec(subs, R, np.array([r[1] for r in rows], dtype=np.int64),
                     np.array([r[2] for r in rows], dtype=np.int64), primal)


def closed_form_n_lambda(w: Workload) -> int:
    """Number of multipliers counted directly from the lattice geometry.

    Each glued code shared by m subdomains gives m - 1 rows.  Counted here
    from node multiplicities on the cut lines (no subdomain lists needed).
    """
    n, r = w.ncell, (1 if w.order_u == 1 else 2)
    cx, cy = w.cuts()
    cutx = set(cx[1:-1])
    cuty = set(cy[1:-1])

    def reg_of_cell(i, j):
        return bool(_region_poro(w.layout, (i + 0.5) / n, (j + 0.5) / n))

    def sub_of_cell(i, j):
        a = max(q for q in range(w.nsub_x) if cx[q] <= i)
        b = max(q for q in range(w.nsub_y) if cy[q] <= j)
        return b * w.nsub_x + a

    dp = w.coupling == "primal"
    allx, ally = set(cx), set(cy)
    total = 0
    for J in range(r * n + 1):
        for I in range(r * n + 1):
            on_x = (I % r == 0) and (I // r) in cutx
            on_y = (J % r == 0) and (J // r) in cuty
            if not (on_x or on_y):
                continue
            if dp and I % r == 0 and J % r == 0 and I // r in allx and J // r in ally:
                continue           # a grid corner: primal, no multiplier
            # cells whose closure holds lattice node (I, J)
            ilo = (I - 1) // r if I > 0 else 0
            ihi = min(I // r, n - 1)
            jlo = (J - 1) // r if J > 0 else 0
            jhi = min(J // r, n - 1)
            cells = {(ci, cj) for ci in range(max(ilo, 0), ihi + 1)
                     for cj in range(max(jlo, 0), jhi + 1)
                     if ci * r <= I <= (ci + 1) * r and cj * r <= J <= (cj + 1) * r}
            subs = {sub_of_cell(ci, cj) for ci, cj in cells}
            if len(subs) < 2:
                continue
            if not _sides(I, J, r * n, w.dirichlet_u):
                total += 2 * (len(subs) - 1)
            if dp:
                # on a cut edge: eta is dual, xi and p primal
                if I % r == 0 and J % r == 0:
                    psubs = {sub_of_cell(ci, cj) for ci, cj in cells if reg_of_cell(ci, cj)}
                    total += max(len(psubs) - 1, 0)
                continue
            if I % r == 0 and J % r == 0:
                i, j = I // r, J // r
                psubs = {sub_of_cell(ci, cj) for ci, cj in cells if reg_of_cell(ci, cj)}
                esubs = subs - psubs
                if len(psubs) >= 2:
                    total += 2 * (len(psubs) - 1)          # eta, xi_P
                    if not _sides(i, j, n, w.dirichlet_p):
                        total += len(psubs) - 1            # p
                if len(esubs) >= 2:
                    total += len(esubs) - 1                # xi_E
    return total


def rigid_modes(w: Workload, sub: Sub) -> np.ndarray:
    """Rigid-body modes (n_s, 3) of a subdomain: translations and the rotation
    about the subdomain centre, on the displacement DOFs, zero elsewhere."""
    r = 1 if w.order_u == 1 else 2
    mu = r * w.ncell + 1
    s = 1.0 / (r * w.ncell)
    xc = 0.5 * (sub.i0 + sub.i1) / w.ncell
    yc = 0.5 * (sub.j0 + sub.j1) / w.ncell
    R = np.zeros((len(sub.codes), 3))
    for i, c in enumerate(sub.codes):
        node, kind = c // 8, c % 8
        if kind > 1:
            continue
        x = (node % mu) * s
        y = (node // mu) * s
        R[i, kind] = 1.0
        R[i, 2] = -(y - yc) if kind == 0 else (x - xc)
    return R
