"""MI355X-native solver for steady anisotropic heat conduction in voxelised
heterogeneous media by the D3Q7 multiple-relaxation-time lattice Boltzmann
method (Fang, Gou, Zhang, Chen, Tao), behind the C ABI of include/mrtlbm.h.

The HIP library (``libmrtlbm.so``, built for gfx950 by ``build.py``) does all
of the work; this package only marshals arguments.  Importing it does not
load the library; the first call does, and raises if it is missing.
"""

from ._lib import (  # noqa: F401
    ADIABATIC,
    F32,
    F64,
    PERIODIC,
    TOL_KEFF,
    TOL_MAXDT,
    MrtlbmError,
    declared_symbols,
    load,
)


def __getattr__(name):
    if name in ("Medium", "batch_solve"):
        from . import solver

        return getattr(solver, name)
    raise AttributeError(name)
