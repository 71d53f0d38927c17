"""MI355X (gfx950) implementation of the per-pixel chain statistics (Appendix A) and the
regional reconstruction filter with its adjoint, from "Regional Adaptive Metropolis Light
Transport" (Otsu et al.).

The compute lives in ``libramlt.so`` (HIP kernels behind the C ABI of ``include/ramlt.h``);
this package only marshals arguments. Importing it does not need a GPU; calling an op
needs the built library and a gfx950 device.
"""

from . import _abi  # noqa: F401
from ._abi import RamltError, RamltFrame  # noqa: F401

__all__ = ["RamltError", "RamltFrame", "ops"]


def __getattr__(name):
    # ``ops`` pulls in torch; load it on first use so the C ABI binding stays light
    if name == "ops":
        import importlib

        return importlib.import_module(__name__ + ".ops")
    raise AttributeError(name)
