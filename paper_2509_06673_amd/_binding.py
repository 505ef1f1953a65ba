"""ctypes binding of libfeti.so (the C ABI declared in include/feti.h).

Argument marshalling only: every numerical step runs in the HIP library.
Device buffers are passed as torch tensors on the GPU (their data_ptr()), and
the context is bound to a torch stream.  The library must be built first
(``python -m paper_2509_06673_amd.build``); importing this module without it
raises an error rather than falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Dict, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfeti.so")

# status codes
OK, EINVAL, ESTATE, ENOMEM, EHIP, ESINGULAR, ENOTCONV, EBREAKDOWN, ENAN = 0, -1, -2, -3, -4, -5, -6, -7, -8
XSPLIT, YSPLIT, CORE = 0, 1, 2
LOAD_MANUFACTURED, LOAD_PERIODIC, LOAD_POINT_SOURCE, LOAD_PATCH, LOAD_RAW = 0, 1, 2, 3, 4
FP64, FP32_IR = 0, 1
PRECOND_DIRICHLET, PRECOND_LUMPED, PRECOND_NONE = 0, 1, 2
START_PREVIOUS, START_ZERO, START_EXTRAPOLATE, START_GIVEN, START_BEST = 0, 1, 2, 3, 4
CORR_ZERO, CORR_PREVIOUS = 0, 1
PCG_AUTO, PCG_GRAPH = 0, 1
EXPORT_K, EXPORT_SBB, EXPORT_KPLUS = 0, 1, 2
KERNEL_LOCAL_SOLVE, KERNEL_IFACE_GEMV, KERNEL_PRECOND_GEMV, KERNEL_ELIMINATION = 0, 1, 2, 3
FIELD_UX, FIELD_UY, FIELD_ETA, FIELD_XI_P, FIELD_P, FIELD_XI_E, FIELD_UZ = 0, 1, 2, 3, 4, 5, 6

STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ESTATE: "ESTATE", ENOMEM: "ENOMEM", EHIP: "EHIP",
                ESINGULAR: "ESINGULAR", ENOTCONV: "ENOTCONV", EBREAKDOWN: "EBREAKDOWN",
                ENAN: "ENAN"}


SCHEME_COUPLED, SCHEME_DECOUPLED = 0, 1
COUPLING_DUAL, COUPLING_PRIMAL = 0, 1


class MeshDesc(C.Structure):
    _fields_ = [("ncell", C.c_int32), ("order_u", C.c_int32), ("layout", C.c_int32),
                ("nsub_x", C.c_int32), ("nsub_y", C.c_int32), ("dirichlet_u", C.c_uint32),
                ("dirichlet_p", C.c_uint32), ("cut_x", C.POINTER(C.c_int32)), ("cut_y", C.POINTER(C.c_int32)),
                ("scheme", C.c_int32), ("coupling", C.c_int32), ("dim", C.c_int32), ("nsub_z", C.c_int32)]


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("alpha", C.c_double), ("c0", C.c_double),
                ("K", C.c_double), ("mu_f", C.c_double), ("lame_mode", C.c_int32)]


class Load(C.Structure):
    _fields_ = [("kind", C.c_int32), ("t", C.c_double), ("params", C.c_double * 16),
                ("f_p", C.c_void_p), ("f_e", C.c_void_p), ("z", C.c_void_p), ("t_side", C.c_void_p),
                ("zw_side", C.c_void_p), ("g_u", C.c_void_p), ("g_p", C.c_void_p), ("eta0", C.c_void_p)]

    RAW_FIELDS = ("f_p", "f_e", "z", "t_side", "zw_side", "g_u", "g_p", "eta0")

    def attach_raw(self, arrays):
        """RAW data: device tensors (float64, contiguous) by field name; the tensors are
        kept alive with this struct."""
        self._raw_keep = dict(arrays)
        for name in self.RAW_FIELDS:
            t = arrays.get(name)
            setattr(self, name, None if t is None else t.data_ptr())


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_corr", C.c_double), ("ir_tol", C.c_double),
                ("max_it", C.c_int32), ("start", C.c_int32), ("check_every", C.c_int32),
                ("ir_max", C.c_int32), ("ir_cold", C.c_int32), ("tol_inner", C.c_double),
                ("tol_upd", C.c_double), ("corr_start", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("iters_first", C.c_int32), ("ir_steps", C.c_int32),
                ("status", C.c_int32),
                ("start_used", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("rho", C.c_double), ("t_ms", C.c_double * 8), ("iters_corr", C.c_int32 * 4),
                ("corr_warm", C.c_int32)]

    def as_dict(self) -> Dict:
        return {"iters": self.iters, "iters_first": self.iters_first, "ir_steps": self.ir_steps,
                "status": self.status,
                "start_used": self.start_used, "res0": self.res0, "res": self.res,
                "rho": self.rho, "t_ms": list(self.t_ms), "iters_corr": list(self.iters_corr),
                "corr_warm": self.corr_warm}


class FetiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib: Optional[C.CDLL] = None

# Live handles, released in dependency order (batches, networks, contexts) by an exit hook
# that runs before the interpreter and the HIP runtime are torn down, so that no handle is
# left to a finaliser that might run after the runtime is gone.
_LIVE = {"batch": weakref.WeakSet(), "net": weakref.WeakSet(), "ctx": weakref.WeakSet()}


def _release_all():
    for kind in ("batch", "net", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(_release_all)

_SIGS = {
    "feti_create": [C.POINTER(C.c_void_p), C.c_void_p],
    "feti_destroy": [C.c_void_p],
    "feti_setup_mesh": [C.c_void_p, C.POINTER(MeshDesc)],
    "feti_get_sizes": [C.c_void_p, C.POINTER(C.c_int64)],
    "feti_export_indexing": [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int8)],
    "feti_export_primal": [C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_export_deflation": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_assemble": [C.c_void_p, C.POINTER(Material), C.POINTER(Material), C.c_double],
    "feti_factor_subdomains": [C.c_void_p, C.c_int32, C.c_int32],
    "feti_init_state": [C.c_void_p, C.POINTER(Load)],
    "feti_step": [C.c_void_p, C.POINTER(Load), C.POINTER(SolveOpts), C.POINTER(Stats)],
    "feti_solve": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                   C.POINTER(Stats)],
    "feti_get_solution": [C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_set_start": [C.c_void_p, C.c_void_p],
    "feti_state_size": [C.c_void_p, C.POINTER(C.c_int64)],
    "feti_get_state": [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)],
    "feti_set_state": [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)],
    "feti_get_field": [C.c_void_p, C.c_int32, C.c_void_p],
    "feti_export_local": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
    "feti_apply_F": [C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_apply_F_noalloc": [C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_apply_precond": [C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_get_rhs": [C.c_void_p, C.c_void_p],
    "feti_torn_residual": [C.c_void_p, C.POINTER(C.c_double)],
    "feti_time_kernel": [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                         C.POINTER(C.c_double)],
    "feti_interface_load": [C.c_void_p, C.POINTER(Load), C.c_void_p],
    "feti_set_keep_assembled": [C.c_void_p, C.c_int32],
    "feti_set_pcg_mode": [C.c_void_p, C.c_int32],
    "feti_batch_create": [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32],
    "feti_batch_destroy": [C.c_void_p],
    "feti_batch_step": [C.c_void_p, C.POINTER(Load), C.POINTER(SolveOpts), C.POINTER(Stats)],
    "feti_batch_set_grid": [C.c_void_p, C.c_int32],
    "feti_batch_set_capture": [C.c_void_p, C.c_int32],
    "feti_batch_info": [C.c_void_p, C.POINTER(C.c_int32)],
    # learned warm start (include/feti_ws.h)
    "feti_ws_create": [C.POINTER(C.c_void_p), C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32],
    "feti_ws_destroy": [C.c_void_p],
    "feti_ws_sizes": [C.c_void_p, C.POINTER(C.c_int64)],
    "feti_ws_set_params": [C.c_void_p, C.c_void_p],
    "feti_ws_get_params": [C.c_void_p, C.c_void_p],
    "feti_ws_set_scaling": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_ws_fit_scaling": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64],
    "feti_ws_forward": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "feti_ws_loss_grad": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p],
    "feti_ws_train_step": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.POINTER(C.c_double)],
    "feti_ws_make_features": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_ws_make_target": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "feti_ws_predict": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
}


def _torch_device_first():
    """Initialise torch's HIP state before the library makes its first HIP call: a
    torch initialised after that has been seen to find no device.  Nothing happens
    without torch or without a GPU."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load_library(path: str = LIB_PATH) -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2509_06673_amd.build`")
    _torch_device_first()
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.feti_last_error.argtypes = [C.c_void_p]
    lib.feti_last_error.restype = C.c_char_p
    lib.feti_ws_last_error.argtypes = [C.c_void_p]
    lib.feti_ws_last_error.restype = C.c_char_p
    lib.feti_batch_last_error.argtypes = [C.c_void_p]
    lib.feti_batch_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _ptr(t) -> int:
    """Device (or host) address of a torch tensor, or 0 for None."""
    if t is None:
        return 0
    return t.data_ptr()


class Feti:
    """One solver context bound to a torch stream on the current GPU."""

    def __init__(self, stream=None):
        self.lib = load_library()
        self.ctx = C.c_void_p()
        sp = None
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._check(self.lib.feti_create(C.byref(self.ctx), sp), "feti_create")
        _LIVE["ctx"].add(self)

    # -- errors -------------------------------------------------------------
    def last_error(self) -> str:
        return self.lib.feti_last_error(self.ctx).decode()

    def _check(self, rc: int, what: str, allow=()):
        if rc != OK and rc not in allow:
            raise FetiError(rc, f"{what}: {self.last_error() if self.ctx else ''}")
        return rc

    def close(self):
        if self.ctx:
            self.lib.feti_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ----------------------------------------------------------------
    def setup_mesh(self, ncell, order_u, layout, nsub_x, nsub_y, dirichlet_u=0xF, dirichlet_p=0xF,
                   cut_x=None, cut_y=None, scheme=0, coupling=0, dim=2, nsub_z=1):
        cx = (C.c_int32 * len(cut_x))(*cut_x) if cut_x is not None else None
        cy = (C.c_int32 * len(cut_y))(*cut_y) if cut_y is not None else None
        d = MeshDesc(ncell, order_u, layout, nsub_x, nsub_y, dirichlet_u, dirichlet_p,
                     C.cast(cx, C.POINTER(C.c_int32)) if cx is not None else None,
                     C.cast(cy, C.POINTER(C.c_int32)) if cy is not None else None, scheme, coupling, dim, nsub_z)
        return self._check(self.lib.feti_setup_mesh(self.ctx, C.byref(d)), "feti_setup_mesh")

    def get_sizes(self) -> Dict[str, int]:
        a = (C.c_int64 * 11)()
        self._check(self.lib.feti_get_sizes(self.ctx, a), "feti_get_sizes")
        keys = ["n_sub", "sum_ns", "n_lambda", "n_c", "max_ns", "max_nb", "sum_nb", "n_p1",
                "n_u", "n_float", "n_primal"]
        return dict(zip(keys, list(a)))

    def export_indexing(self):
        import numpy as np
        sz = self.get_sizes()
        code = np.zeros(sz["sum_ns"], np.int32)
        off = np.zeros(sz["n_sub"] + 1, np.int32)
        nb = np.zeros(sz["n_sub"], np.int32)
        bs = np.zeros(2 * sz["n_lambda"], np.int32)
        bl = np.zeros(2 * sz["n_lambda"], np.int32)
        sg = np.zeros(2 * sz["n_lambda"], np.int8)
        P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
        self._check(self.lib.feti_export_indexing(self.ctx, P(code, C.c_int32), P(off, C.c_int32),
                                                  P(nb, C.c_int32), P(bs, C.c_int32),
                                                  P(bl, C.c_int32), P(sg, C.c_int8)),
                    "feti_export_indexing")
        return dict(code=code, sub_offset=off, sub_nb=nb, brow_sub=bs, brow_local=bl, brow_sign=sg)


    def export_deflation(self):
        """Dual-primal coupling: per multiplier row two (deflation column, weight) slots (column
        -1: unused), and the number of columns."""
        import numpy as np
        nl = self.get_sizes()["n_lambda"]
        col = np.zeros(max(2 * nl, 1), np.int32)
        w = np.zeros(max(2 * nl, 1), np.float64)
        nd = C.c_int32(0)
        self._check(self.lib.feti_export_deflation(self.ctx, col.ctypes.data_as(C.c_void_p),
                                                   w.ctypes.data_as(C.c_void_p), C.byref(nd)),
                    "feti_export_deflation")
        return {"col": col[:2 * nl].reshape(nl, 2), "w": w[:2 * nl].reshape(nl, 2), "n_defl": int(nd.value)}

    def export_primal(self):
        """Dual-primal coupling: the primal codes in global order and the number of primal
        (trailing interface) DOFs of every subdomain."""
        import numpy as np
        sz = self.get_sizes()
        code = np.zeros(max(sz["n_primal"], 1), np.int32)
        npi = np.zeros(sz["n_sub"], np.int32)
        self._check(self.lib.feti_export_primal(self.ctx, code.ctypes.data_as(C.c_void_p),
                                                npi.ctypes.data_as(C.c_void_p)), "feti_export_primal")
        return {"code": code[:sz["n_primal"]], "sub_npi": npi}
    def assemble(self, mat_p: Material, mat_e: Material, tau: float):
        return self._check(self.lib.feti_assemble(self.ctx, C.byref(mat_p), C.byref(mat_e), tau),
                           "feti_assemble")

    def factor_subdomains(self, precision=FP64, precond=PRECOND_DIRICHLET):
        return self._check(self.lib.feti_factor_subdomains(self.ctx, precision, precond),
                           "feti_factor_subdomains")

    # -- stepping ---------------------------------------------------------------
    def init_state(self, load: Load):
        return self._check(self.lib.feti_init_state(self.ctx, C.byref(load)), "feti_init_state")

    def step(self, load: Load, opts: SolveOpts, allow=()) -> Dict:
        st = Stats()
        rc = self.lib.feti_step(self.ctx, C.byref(load), C.byref(opts), C.byref(st))
        self._check(rc, "feti_step", allow)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def solve(self, f, lam, u, opts: SolveOpts, allow=()) -> Dict:
        st = Stats()
        rc = self.lib.feti_solve(self.ctx, _ptr(f), _ptr(lam), _ptr(u), C.byref(opts), C.byref(st))
        self._check(rc, "feti_solve", allow)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def get_solution(self, u=None, lam=None):
        return self._check(self.lib.feti_get_solution(self.ctx, _ptr(u), _ptr(lam)),
                           "feti_get_solution")

    def set_start(self, lam):
        return self._check(self.lib.feti_set_start(self.ctx, _ptr(lam)), "feti_set_start")

    def state_size(self) -> int:
        n = C.c_int64()
        self._check(self.lib.feti_state_size(self.ctx, C.byref(n)), "feti_state_size")
        return n.value

    def get_state(self, state):
        """Copies the checkpoint state into the device buffer state; returns the 4 flags."""
        meta = (C.c_int64 * 4)()
        self._check(self.lib.feti_get_state(self.ctx, _ptr(state), meta), "feti_get_state")
        return list(meta)

    def set_state(self, state, meta):
        m = (C.c_int64 * 4)(*[int(v) for v in meta])
        return self._check(self.lib.feti_set_state(self.ctx, _ptr(state), m), "feti_set_state")

    def get_field(self, field: int, out):
        return self._check(self.lib.feti_get_field(self.ctx, int(field), _ptr(out)), "feti_get_field")

    def set_pcg_mode(self, mode: int):
        return self._check(self.lib.feti_set_pcg_mode(self.ctx, int(mode)), "feti_set_pcg_mode")

    def set_keep_assembled(self, keep: bool):
        return self._check(self.lib.feti_set_keep_assembled(self.ctx, 1 if keep else 0),
                           "feti_set_keep_assembled")

    def interface_load(self, load: Load, out):
        return self._check(self.lib.feti_interface_load(self.ctx, C.byref(load), _ptr(out)),
                           "feti_interface_load")

    # -- inspection ---------------------------------------------------------------
    def export_local(self, sub: int, which: int, out):
        return self._check(self.lib.feti_export_local(self.ctx, sub, which, _ptr(out)),
                           "feti_export_local")

    def apply_F(self, x, y):
        return self._check(self.lib.feti_apply_F(self.ctx, _ptr(x), _ptr(y)), "feti_apply_F")


    def apply_F_noalloc(self, x, y):
        """y = F x through the entry point that allocates nothing (stream-ordered, no
        synchronisation)."""
        return self._check(self.lib.feti_apply_F_noalloc(self.ctx, _ptr(x), _ptr(y)), "feti_apply_F_noalloc")
    def apply_precond(self, x, y):
        return self._check(self.lib.feti_apply_precond(self.ctx, _ptr(x), _ptr(y)),
                           "feti_apply_precond")

    def get_rhs(self, f):
        return self._check(self.lib.feti_get_rhs(self.ctx, _ptr(f)), "feti_get_rhs")

    # -- measurement --------------------------------------------------------------
    def torn_residual(self) -> float:
        rho = C.c_double()
        self._check(self.lib.feti_torn_residual(self.ctx, C.byref(rho)), "feti_torn_residual")
        return rho.value

    def time_kernel(self, which: int, reps: int = 20):
        ms, work = C.c_double(), C.c_double()
        self._check(self.lib.feti_time_kernel(self.ctx, which, reps, C.byref(ms), C.byref(work)),
                    "feti_time_kernel")
        return ms.value, work.value


class WarmStartNet:
    """The learned warm-start network of include/feti_ws.h on a torch stream."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, max_batch: int, stream=None):
        self.lib = load_library()
        self.h = C.c_void_p()
        sp = None
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        rc = self.lib.feti_ws_create(C.byref(self.h), sp, n_in, n_hidden, n_out, max_batch)
        if rc != OK:
            raise FetiError(rc, "feti_ws_create")
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        _LIVE["net"].add(self)

    def _check(self, rc: int, what: str):
        if rc != OK:
            msg = self.lib.feti_ws_last_error(self.h).decode() if self.h else ""
            raise FetiError(rc, f"{what}: {msg}")
        return rc

    def close(self):
        if self.h:
            self.lib.feti_ws_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self) -> int:
        s = (C.c_int64 * 5)()
        self._check(self.lib.feti_ws_sizes(self.h, s), "feti_ws_sizes")
        return int(s[0])

    def set_params(self, p):
        return self._check(self.lib.feti_ws_set_params(self.h, _ptr(p)), "feti_ws_set_params")

    def get_params(self, p):
        return self._check(self.lib.feti_ws_get_params(self.h, _ptr(p)), "feti_ws_get_params")

    def set_scaling(self, mean, inv_std, out_scale):
        return self._check(self.lib.feti_ws_set_scaling(self.h, _ptr(mean), _ptr(inv_std), _ptr(out_scale)),
                           "feti_ws_set_scaling")

    def fit_scaling(self, x, t, nsamples: int):
        return self._check(self.lib.feti_ws_fit_scaling(self.h, _ptr(x), _ptr(t), nsamples),
                           "feti_ws_fit_scaling")

    def forward(self, x, batch: int, y):
        return self._check(self.lib.feti_ws_forward(self.h, _ptr(x), batch, _ptr(y)), "feti_ws_forward")

    def loss_grad(self, x, t, batch: int, grad) -> float:
        loss = C.c_double()
        self._check(self.lib.feti_ws_loss_grad(self.h, _ptr(x), _ptr(t), batch, C.byref(loss), _ptr(grad)),
                    "feti_ws_loss_grad")
        return loss.value

    def train_step(self, x, t, batch: int, lr: float, want_loss: bool = False):
        loss = C.c_double()
        self._check(self.lib.feti_ws_train_step(self.h, _ptr(x), _ptr(t), batch, lr,
                                                C.byref(loss) if want_loss else None), "feti_ws_train_step")
        return loss.value if want_loss else None

    def make_features(self, n: int, lam_n, lam_nm1, load, x_row):
        return self._check(self.lib.feti_ws_make_features(self.h, n, _ptr(lam_n), _ptr(lam_nm1), _ptr(load),
                                                          _ptr(x_row)), "feti_ws_make_features")

    def make_target(self, n: int, lam_np1, lam_n, lam_nm1, t_row):
        return self._check(self.lib.feti_ws_make_target(self.h, n, _ptr(lam_np1), _ptr(lam_n), _ptr(lam_nm1),
                                                        _ptr(t_row)), "feti_ws_make_target")

    def predict(self, lam_n, lam_nm1, load, lam_out):
        return self._check(self.lib.feti_ws_predict(self.h, _ptr(lam_n), _ptr(lam_nm1), _ptr(load),
                                                    _ptr(lam_out)), "feti_ws_predict")


class Batch:
    """Independent factored contexts stepped together (feti_batch_* of include/feti.h);
    the contexts must outlive the batch."""

    def __init__(self, ctxs):
        self.lib = load_library()
        self.ctxs = list(ctxs)
        arr = (C.c_void_p * len(self.ctxs))(*[c.ctx.value for c in self.ctxs])
        self.h = C.c_void_p()
        rc = self.lib.feti_batch_create(C.byref(self.h), arr, len(self.ctxs))
        if rc != OK:
            raise FetiError(rc, self.ctxs[0].last_error())
        _LIVE["batch"].add(self)

    def _check(self, rc: int, what: str, allow=()):
        if rc != OK and rc not in allow:
            msg = self.lib.feti_batch_last_error(self.h).decode() if self.h else ""
            raise FetiError(rc, f"{what}: {msg}")
        return rc

    def close(self):
        if self.h:
            self.lib.feti_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, loads, opts: SolveOpts, allow=()):
        n = len(self.ctxs)
        la = (Load * n)(*loads)
        st = (Stats * n)()
        rc = self.lib.feti_batch_step(self.h, la, C.byref(opts), st)
        self._check(rc, "feti_batch_step", allow)
        return [s.as_dict() for s in st], rc

    def set_grid(self, grid: int):
        return self._check(self.lib.feti_batch_set_grid(self.h, grid), "feti_batch_set_grid")

    def set_capture(self, on: bool):
        return self._check(self.lib.feti_batch_set_capture(self.h, 1 if on else 0), "feti_batch_set_capture")

    def info(self):
        buf = (C.c_int32 * 12)()
        self._check(self.lib.feti_batch_info(self.h, buf), "feti_batch_info")
        return {"grid": buf[0], "tuned": bool(buf[1]), "candidates": [buf[3 + k] for k in range(buf[2])],
                "graph": bool(buf[11])}
