"""MI355X-native hot path of the generalized lattice Boltzmann model for gas
flow through tight porous media with Klinkenberg's effect (Chen et al.,
arXiv:1411.7051).

The fused D2Q9 sweep and its read-outs are HIP kernels for gfx950 behind the
C ABI of ``include/lbk.h`` (``liblbk.so``, built by ``build.py``);
``Lattice``, ``Batch`` (ensembles stepped together) and ``Lattice3`` (the
same model on a D3Q19 lattice) are thin ctypes bindings over it; ``units``
maps physical conditions (Eqs. 9-11) to lattice inputs.  ``inputs`` draws the
seeded synthetic media.
"""
from . import inputs  # noqa: F401

__all__ = ["Lattice", "Batch", "Lattice3", "ApparentPermeability", "inputs", "units",
           "make_desc", "workspace_bytes"]


def __getattr__(name):
    if name in ("Lattice", "ApparentPermeability", "make_desc", "workspace_bytes"):
        from . import lattice
        return getattr(lattice, name)
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name == "Lattice3":
        from .lattice3 import Lattice3
        return Lattice3
    if name == "units":
        import importlib
        return importlib.import_module(".units", __name__)
    raise AttributeError(name)
