"""MI355X-native hot path of the generalized lattice Boltzmann model for gas
flow through tight porous media with Klinkenberg's effect (Chen et al.,
arXiv:1411.7051).

The fused D2Q9 sweep and its read-outs are HIP kernels for gfx950 behind the
C ABI of ``include/lbk.h`` (``liblbk.so``, built by ``build.py``);
``Lattice`` and ``Batch`` (ensembles stepped together) are thin ctypes
bindings over it; ``units`` maps physical conditions (Eqs. 9-11) to lattice
inputs.  ``inputs`` draws the seeded
synthetic media.
"""
from . import inputs  # noqa: F401

__all__ = ["Lattice", "Batch", "ApparentPermeability", "inputs", "units", "make_desc",
           "workspace_bytes"]


def __getattr__(name):
    if name in ("Lattice", "ApparentPermeability", "make_desc", "workspace_bytes"):
        from . import lattice
        return getattr(lattice, name)
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name == "units":
        import importlib
        return importlib.import_module(".units", __name__)
    raise AttributeError(name)
