"""MI355X (gfx950) Lennard-Jones MD hot path: cell-list binning, a Verlet pair
list with skin, the truncated LJ force/energy loop and velocity-Verlet
integration, as HIP kernels behind the C ABI of include/md.h.

Importing the package loads libmd355.so and raises ImportError if it has not
been built: there is no CPU fallback.
"""

from . import _abi
from ._abi import MdError

_abi.lib()  # fail loudly when the HIP library is missing

from .engine import Engine, Grid, PairList, Workspace, make_params, stream_handle  # noqa: E402
from .autograd import Field, LJEnergy, TrajectoryMeanPE  # noqa: E402

__all__ = ["Engine", "Grid", "PairList", "Workspace", "make_params", "stream_handle", "MdError", "Field",
           "LJEnergy", "TrajectoryMeanPE"]
