"""MI355X-native differential walk on spheres.

Hot path: hand-written HIP kernels for gfx950 behind the C ABI of
``include/dwos.h`` (``libdwos.so`` in this directory).  ``capi`` is the ctypes
binding with the C names, ``Solver`` an object wrapper over one context, and
``DWoSFunction`` a ``torch.autograd.Function`` whose backward is the
differential walk kernel.  ``cv.Network`` is the learned control variate of
the nested walks (matrix-core kernels of the same library).
"""
from .capi import DwosError, lib  # noqa: F401  (loads libdwos.so or raises)
from .solver import Solver, make_problem  # noqa: F401
from .autograd import DWoSFunction, ShapeModel  # noqa: F401
from .cv import Network  # noqa: F401
from .opt import LargeSteps  # noqa: F401
from .shapeopt import VertexShapeOptimizer, ImplicitShapeOptimizer  # noqa: F401

__all__ = ["Solver", "make_problem", "DWoSFunction", "ShapeModel", "Network", "LargeSteps", "VertexShapeOptimizer",
           "ImplicitShapeOptimizer", "DwosError", "lib"]
