"""Synthetic workload definitions shared by the oracle, the tests and the bench.

This module holds data only: mesh sizes, subdomain grids, material parameters,
time-step settings, load descriptors and the seeded draws that produce them.
It contains none of the discretisation or solver arithmetic, so the oracle and
the HIP path can both take their inputs from here without sharing any of the
method's code.

The workloads are shaped like the paper's tests (Section 4): the unit square,
a poroelastic region glued to an elastic one along a straight interface, a
structured right-triangle mesh, P_k-P1-P1-P1 / P_k-P1 mixed elements and
backward Euler in time.
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass, field, asdict
from typing import Dict, List, Optional, Tuple

import numpy as np

# layouts of the poroelastic region inside the unit square
XSPLIT = "xsplit"   # poroelastic for x < 1/2, elastic for x > 1/2
YSPLIT = "ysplit"   # poroelastic for y < 1/2 (the paper's Test 1 and 2 layout)
CORE = "core"       # poroelastic core [1/4, 3/4]^2 inside an elastic frame

# load kinds
MANUFACTURED = "manufactured"   # closed-form smooth solution (Section 4.1)
PERIODIC = "periodic"           # time-periodic body force and source
POINT_SOURCE = "point_source"   # Gaussian-regularised pulsed source
PATCH = "patch"                 # polynomial solution contained in the FE spaces
RAW = "raw"                     # caller data: nodal loads, boundary data and initial data

# coefficients of the patch-test displacement (1, x, y, x^2, xy, y^2) and pressure (1, y);
# the quadratic terms and the y-term of p are dropped for P1 displacements
PATCH_UX = (0.1, 0.2, -0.3, 0.4, -0.5, 0.6)
PATCH_UY = (-0.2, 0.3, 0.1, -0.3, 0.2, 0.5)
PATCH_P = (0.7, 0.4)


@dataclass
class Material:
    """Parameters of Table 2 for one region."""
    E: float = 1.0
    nu: float = 0.3
    alpha: float = 1.0
    c0: float = 1.0
    K: float = 1.0
    mu_f: float = 1.0
    # 0: textbook mu = E / (2 (1 + nu)); 1: the literal mu = E / (1 + nu) of Table 3
    lame_mode: int = 0


@dataclass
class Load:
    kind: str = MANUFACTURED
    # PERIODIC: amplitude, angular frequency, phase
    amp: float = 1.0
    omega: float = 2.0 * math.pi
    phase: float = 0.0
    # POINT_SOURCE: centre and Gaussian width
    cx: float = 0.5
    cy: float = 0.5
    sigma: float = 1.0 / 32.0
    # RAW: seed of the nodal data drawn by raw_arrays (or fixed arrays given by the caller)
    raw_seed: int = 0
    raw_fixed: Optional[dict] = None


@dataclass
class Workload:
    name: str
    ncell: int                 # cells per side; h = 1 / ncell
    order_u: int               # k of P_k for the displacement (1 or 2)
    layout: str
    nsub_x: int
    nsub_y: int
    mat_p: Material
    mat_e: Material
    tau: float
    nsteps: int
    load: Load
    tol: float = 1e-10
    # bitmask of outer sides (bit 0: x=0, 1: x=1, 2: y=0, 3: y=1) with u Dirichlet
    dirichlet_u: int = 0xF
    # bitmask of outer sides with p Dirichlet (only where the poro region touches them)
    dirichlet_p: int = 0xF
    # subdomain cuts in cells (nsub + 1 increasing values from 0 to ncell); None = the even
    # cuts floor(a ncell / nsub)
    cut_x: Optional[Tuple[int, ...]] = None
    cut_y: Optional[Tuple[int, ...]] = None
    # time discretisation: "coupled" (eq. (linalg-system) at once) or "decoupled" (explicit
    # fluid step, then the momentum balance alone)
    scheme: str = "coupled"
    # gluing of the shared DOFs: "dual" (every shared DOF torn and glued by multipliers) or
    # "primal" (the shared xi / p DOFs and the shared DOFs at subdomain corners are global
    # primal unknowns; multipliers glue only the remaining u and eta DOFs)
    coupling: str = "dual"
    # spatial dimension (2: triangles on the unit square; 3: Kuhn tetrahedra on the unit
    # cube, with an nsub_x x nsub_y x nsub_z subdomain grid at the even cuts)
    dim: int = 2
    nsub_z: int = 1

    def cuts(self) -> Tuple[List[int], List[int]]:
        cx = list(self.cut_x) if self.cut_x is not None else [(a * self.ncell) // self.nsub_x
                                                               for a in range(self.nsub_x + 1)]
        cy = list(self.cut_y) if self.cut_y is not None else [(b * self.ncell) // self.nsub_y
                                                               for b in range(self.nsub_y + 1)]
        return cx, cy

    @property
    def h(self) -> float:
        return 1.0 / self.ncell

    def to_dict(self) -> dict:
        return asdict(self)

    def replace(self, **kw) -> "Workload":
        w = copy.deepcopy(self)
        for k, v in kw.items():
            setattr(w, k, v)
        return w


def _mat(**kw) -> Material:
    return Material(**kw)


# ---------------------------------------------------------------------------
# The five workload families
# ---------------------------------------------------------------------------

def plain_fp64_small() -> Workload:
    """Two subdomains (one per physics), P1 elements, h = 1/16, 10 steps."""
    m = _mat(E=1.0, nu=0.3, alpha=1.0, c0=1.0, K=1.0, mu_f=1.0)
    return Workload(name="xsplit_p1_h16_2sub", ncell=16, order_u=1, layout=XSPLIT,
                    nsub_x=2, nsub_y=1, mat_p=m, mat_e=copy.deepcopy(m), tau=0.01,
                    nsteps=10, load=Load(kind=MANUFACTURED))


def nearly_incompressible_large() -> Workload:
    """64 subdomains (8x8), P2 elements, h = 1/128, nu = 0.49999, 50 steps."""
    m = _mat(E=1e4, nu=0.49999, alpha=1.0, c0=1e-3, K=1e-6, mu_f=1.0)
    return Workload(name="xsplit_p2_h128_8x8", ncell=128, order_u=2, layout=XSPLIT,
                    nsub_x=8, nsub_y=8, mat_p=m, mat_e=copy.deepcopy(m), tau=1e-3,
                    nsteps=50, load=Load(kind=MANUFACTURED))


def nearly_incompressible_scaled(ncell: int, nsub: int, nsteps: int = 3) -> Workload:
    """The same physics as the large case at a smaller mesh, for parity tests."""
    w = nearly_incompressible_large()
    return w.replace(name=f"xsplit_p2_h{ncell}_{nsub}x{nsub}", ncell=ncell,
                     nsub_x=nsub, nsub_y=nsub, nsteps=nsteps)


def learned_start_case(seed: int, nsteps: int = 200, ncell: int = 64) -> Workload:
    """Periodic load of random amplitude, frequency and phase (seeded)."""
    rng = np.random.default_rng(seed)
    amp = float(10.0 ** rng.uniform(-1.0, 1.0))
    omega = float(rng.uniform(2.0 * math.pi, 20.0 * math.pi))
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    m = _mat(E=1e4, nu=0.49999, alpha=1.0, c0=1e-3, K=1e-6, mu_f=1.0)
    return Workload(name=f"xsplit_p2_h{ncell}_8x8_periodic_s{seed}", ncell=ncell, order_u=2,
                    layout=XSPLIT, nsub_x=8, nsub_y=8, mat_p=m, mat_e=copy.deepcopy(m),
                    tau=1e-3, nsteps=nsteps,
                    load=Load(kind=PERIODIC, amp=amp, omega=omega, phase=phase))


def pulsed_core(ncell: int = 256, nsub: int = 32, nsteps: int = 200) -> Workload:
    """Poroelastic core in an elastic frame, pulsed Gaussian source at the centre."""
    m = _mat(E=1e4, nu=0.49999, alpha=1.0, c0=1e-3, K=1e-6, mu_f=1.0)
    return Workload(name=f"core_p2_h{ncell}_{nsub}x{nsub}", ncell=ncell, order_u=2,
                    layout=CORE, nsub_x=nsub, nsub_y=nsub, mat_p=m,
                    mat_e=copy.deepcopy(m), tau=2.0 * math.pi / 200.0, nsteps=nsteps,
                    load=Load(kind=POINT_SOURCE, cx=0.5, cy=0.5, sigma=1.0 / 32.0),
                    dirichlet_p=0)


def paper_table_case(order_u: int, ncell: int, nu: float, nsteps: int = 100,
                     lame_mode: int = 0) -> Workload:
    """Test cases 1 and 2 of Section 4 (Table 3 parameters), y-split layout."""
    m = _mat(E=1e4, nu=nu, alpha=1.0, c0=0.1, K=1.0, mu_f=1.0, lame_mode=lame_mode)
    return Workload(name=f"ysplit_p{order_u}_h{ncell}_nu{nu}", ncell=ncell, order_u=order_u,
                    layout=YSPLIT, nsub_x=1, nsub_y=2, mat_p=m, mat_e=copy.deepcopy(m),
                    tau=1e-4, nsteps=nsteps, load=Load(kind=MANUFACTURED))


def patch_case(order_u: int = 2, ncell: int = 8, nsub_x: int = 4, nsub_y: int = 2,
               nsteps: int = 2, nu: float = 0.3) -> Workload:
    """Polynomial solution reproduced exactly by the discretisation, x-split layout."""
    m = _mat(E=10.0, nu=nu, alpha=1.0, c0=0.5, K=0.2, mu_f=1.0)
    return Workload(name=f"patch_p{order_u}_h{ncell}_{nsub_x}x{nsub_y}", ncell=ncell,
                    order_u=order_u, layout=XSPLIT, nsub_x=nsub_x, nsub_y=nsub_y, mat_p=m,
                    mat_e=copy.deepcopy(m), tau=0.05, nsteps=nsteps, load=Load(kind=PATCH))


def raw_case(ncell: int = 8, nsub_x: int = 4, nsub_y: int = 2, order_u: int = 2, nsteps: int = 3,
             seed: int = 5, layout: str = XSPLIT) -> Workload:
    """Caller-data load (RAW): seeded nodal body forces, source, traction, flux,
    Dirichlet and initial data; u Dirichlet on x = 0 and y = 0 only (traction on x = 1
    and y = 1), p Dirichlet on x = 0 only (flux on the poroelastic parts of y = 0 and
    y = 1)."""
    m = _mat(E=10.0, nu=0.3, alpha=1.0, c0=0.5, K=0.2, mu_f=1.0)
    return Workload(name=f"raw_p{order_u}_h{ncell}_{nsub_x}x{nsub_y}_s{seed}", ncell=ncell, order_u=order_u,
                    layout=layout, nsub_x=nsub_x, nsub_y=nsub_y, mat_p=m, mat_e=copy.deepcopy(m), tau=0.05,
                    nsteps=nsteps, load=Load(kind=RAW, raw_seed=seed), dirichlet_u=0b0101, dirichlet_p=0b0001)


RAW_FIELDS = ("f_p", "f_e", "z", "t_side", "zw_side", "g_u", "g_p", "eta0")


def raw_shapes(w: Workload) -> Dict[str, Tuple[int, ...]]:
    """Array shapes of the RAW data: displacement lattice of mu = k ncell + 1 points per
    side, P1 lattice of n1 = ncell + 1; lattices row-major with x fastest; the side
    arrays are indexed by side (x = 0, x = 1, y = 0, y = 1) and by the lattice index
    along the side (y index on x = const, x index on y = const).  In 3D the lattices are
    cubes (x fastest, then y, then z), the displacement data has three components and
    there are no side data."""
    mu = w.order_u * w.ncell + 1
    n1 = w.ncell + 1
    if w.dim == 3:
        return {"f_p": (3, mu ** 3), "f_e": (3, mu ** 3), "z": (n1 ** 3,), "t_side": (0,), "zw_side": (0,),
                "g_u": (3, mu ** 3), "g_p": (n1 ** 3,), "eta0": (n1 ** 3,)}
    return {"f_p": (2, mu * mu), "f_e": (2, mu * mu), "z": (n1 * n1,), "t_side": (2, 4, 2, mu),
            "zw_side": (4, n1), "g_u": (2, mu * mu), "g_p": (n1 * n1,), "eta0": (n1 * n1,)}


def raw_arrays(w: Workload, t: float) -> Dict[str, np.ndarray]:
    """Nodal data of a RAW load at time t.  With raw_fixed the given arrays (the same at
    every t); otherwise standard-normal arrays drawn from raw_seed, each multiplied by
    its own smooth factor of t (so that every step sees new data)."""
    if w.load.raw_fixed is not None:
        return {k: np.asarray(v, dtype=np.float64) for k, v in w.load.raw_fixed.items()}
    shapes = raw_shapes(w)
    rng = np.random.default_rng(w.load.raw_seed)
    out = {}
    for i, name in enumerate(RAW_FIELDS):
        base = rng.standard_normal(shapes[name])
        fac = 1.0 if name == "eta0" else 1.0 + 0.5 * math.sin(3.0 * t + 0.7 * i)
        out[name] = fac * base
    return out


def cube_case(ncell: int = 4, nsub: Tuple[int, int, int] = (2, 2, 2), order_u: int = 2, nsteps: int = 3,
              seed: int = 7, nu: float = 0.3) -> Workload:
    """3D: the unit cube in Kuhn tetrahedra, poroelastic for x < 1/2, elastic for x > 1/2,
    seeded nodal data (RAW); u Dirichlet on every face, p Dirichlet on the poroelastic
    parts of x = 0, y = 0 and z = 0 (no flux through the others)."""
    m = _mat(E=10.0, nu=nu, alpha=1.0, c0=0.5, K=0.2, mu_f=1.0)
    return Workload(name=f"cube_p{order_u}_h{ncell}_{nsub[0]}x{nsub[1]}x{nsub[2]}_s{seed}", ncell=ncell,
                    order_u=order_u, layout=XSPLIT, nsub_x=nsub[0], nsub_y=nsub[1], mat_p=m,
                    mat_e=copy.deepcopy(m), tau=0.05, nsteps=nsteps, load=Load(kind=RAW, raw_seed=seed),
                    dirichlet_u=0x3F, dirichlet_p=0b010101, coupling="primal", dim=3, nsub_z=nsub[2])


def cube_nearly_incompressible(ncell: int = 16, nsub: int = 4, nsteps: int = 25, seed: int = 11) -> Workload:
    """3D counterpart of the nearly incompressible workload: P2 tetrahedra, h = 1/ncell,
    nsub^3 subdomains, nu = 0.49999, c0 = 1e-3, K = 1e-6, tau = 1e-3, seeded nodal data."""
    m = _mat(E=1e4, nu=0.49999, alpha=1.0, c0=1e-3, K=1e-6, mu_f=1.0)
    return Workload(name=f"cube_p2_h{ncell}_{nsub}x{nsub}x{nsub}", ncell=ncell, order_u=2, layout=XSPLIT,
                    nsub_x=nsub, nsub_y=nsub, mat_p=m, mat_e=copy.deepcopy(m), tau=1e-3, nsteps=nsteps,
                    load=Load(kind=RAW, raw_seed=seed), dirichlet_u=0x3F, dirichlet_p=0b010101,
                    coupling="primal", dim=3, nsub_z=nsub)


BATCH_SEED = 20250906


def batched_draws(nprob: int = 256, seed: int = BATCH_SEED, nsteps: int = 20,
                  max_cells_per_sub: int = 16) -> List[Workload]:
    """Seeded draws of many independent coupled problems of uneven size.

    h ~ U{1/32, 1/48, 1/64, 1/96}; the subdomain grid is drawn uniformly among the
    admissible ones (nsub_x even so the x = 1/2 interface is a cut, at most
    ``max_cells_per_sub`` cells per subdomain side); nu ~ U[0.2, 0.4999],
    E ~ logU[1e2, 1e5], K ~ logU[1e-8, 1], c0 ~ logU[1e-4, 1].
    """
    children = np.random.SeedSequence(seed).spawn(nprob)
    out = []
    for i, child in enumerate(children):
        rng = np.random.default_rng(child)
        ncell = int(rng.choice([32, 48, 64, 96]))
        # an even nsub_x puts a cut exactly on x = 1/2
        grids = [(nx, ny) for nx in (2, 4, 6) for ny in range(2, 7)
                 if math.ceil(ncell / nx) <= max_cells_per_sub
                 and math.ceil(ncell / ny) <= max_cells_per_sub]
        nx, ny = grids[int(rng.integers(len(grids)))]
        nu = float(rng.uniform(0.2, 0.4999))
        E = float(10.0 ** rng.uniform(2.0, 5.0))
        K = float(10.0 ** rng.uniform(-8.0, 0.0))
        c0 = float(10.0 ** rng.uniform(-4.0, 0.0))
        m = _mat(E=E, nu=nu, alpha=1.0, c0=c0, K=K, mu_f=1.0)
        out.append(Workload(name=f"batch{i:03d}_h{ncell}_{nx}x{ny}", ncell=ncell, order_u=2,
                            layout=XSPLIT, nsub_x=nx, nsub_y=ny, mat_p=m,
                            mat_e=copy.deepcopy(m), tau=1e-3, nsteps=nsteps,
                            load=Load(kind=MANUFACTURED)))
    return out


def seeded_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Reproducible standard-normal FP64 vector (test inputs)."""
    return scale * np.random.default_rng(seed).standard_normal(n)


def seeded_matrix(m: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return scale * np.random.default_rng(seed).standard_normal((m, n))


def mlp_init(n_in: int, n_hidden: int, n_out: int, seed: int = 0):
    """Seeded initial weights of the warm-start network (flat FP32, the layout of
    oracle/mlp.py): uniform in +-sqrt(6 / (fan_in + fan_out)) for the weights, zero
    biases; the last layer is scaled by 0.1 so that the untrained network predicts a
    small correction."""
    rng = np.random.default_rng(seed)
    parts = []
    for (fo, fi), scale in (((n_hidden, n_in), 1.0), ((n_hidden, n_hidden), 1.0), ((n_out, n_hidden), 0.1)):
        lim = scale * math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)
