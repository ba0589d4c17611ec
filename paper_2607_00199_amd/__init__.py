"""MI355X library for the ALE nodal DG Galerkin-Boltzmann hot path.

The computation lives in the HIP library ``libgb.so`` (C ABI in
``include/gb.h``); this package is its ctypes binding plus small helpers that
marshal synthetic workloads into it.  Importing the package does not touch the
GPU; the first call that needs the library loads it and fails loudly if it is
missing.
"""
from . import _lib  # noqa: F401
from ._lib import *  # noqa: F401,F403
