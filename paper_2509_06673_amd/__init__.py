"""MI355X FETI solver for the coupled poroelasticity / elasticity model.

The numerical work runs in the HIP library ``libfeti.so`` (built from
``csrc/`` by ``python -m paper_2509_06673_amd.build``); this package only
marshals arguments to its C ABI (``include/feti.h``).
"""
from ._binding import (Feti, FetiError, Load, Material, MeshDesc, SolveOpts, Stats,  # noqa: F401
                       load_library, LIB_PATH)
from . import _binding as capi  # noqa: F401
