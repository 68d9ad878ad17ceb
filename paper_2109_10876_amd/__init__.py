"""MI355X (gfx950) short-range Lennard-Jones molecular dynamics.

The hot path of arXiv 2109.10876 -- LJ pair forces over cell-list-built
Verlet lists on a structure-of-arrays layout inside a velocity-Verlet step --
as hand-written HIP kernels behind the C ABI in ``include/md.h`` (libmd.so).
This package is the thin Python side: ctypes marshalling (``_abi``), a
device-resident system driver (``system.MDSystem``) and a
``torch.autograd.Function`` over the forces and their adjoint (``autograd``).
"""
from . import _abi  # noqa: F401

__all__ = ["MDSystem", "load"]


def load():
    """Load libmd.so; raises if it has not been built."""
    return _abi.load()


def __getattr__(name):
    if name == "MDSystem":
        from .system import MDSystem
        return MDSystem
    raise AttributeError(name)
