"""Lattice Boltzmann schemes with relative velocities on AMD MI355X (gfx950).

The compute path is the HIP library liblbmrv.so (C ABI in include/lbmrv.h);
``lbmrv`` is its ctypes binding and ``workloads`` the seeded synthetic inputs.
"""
from . import lbmrv, workloads  # noqa: F401
from .lbmrv import Lbmrv, lattice_tables  # noqa: F401
