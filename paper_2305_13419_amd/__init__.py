"""Two-fluid (Maxwell + London) FDTD for AMD MI355X.

The time step (Algorithm 1 of arXiv 2305.13419) runs in the HIP kernels of
``libtfl.so``; ``Simulation`` is a thin front end over its C ABI
(``include/tfl.h``).  Importing the package requires the built library.
"""
from . import _lib  # noqa: F401
from .autograd import AdjointProblem, TwoFluidObjective  # noqa: F401
from .sim import Simulation  # noqa: F401

__all__ = ["Simulation", "AdjointProblem", "TwoFluidObjective"]
