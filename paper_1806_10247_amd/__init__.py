"""casclb: cascaded (central-moment) lattice Boltzmann with symmetrized (Strang)
operator-split force and source steps, as hand-written HIP kernels for AMD
Instinct MI355X (gfx950) behind a C ABI (``include/casclb.h``).

``capi`` is the ctypes binding of that ABI (same function names); ``solver``
is a small convenience wrapper around one context.
"""
from . import capi  # noqa: F401
from .capi import LbError  # noqa: F401

__all__ = ["capi", "LbError"]
