"""MI355X (gfx950) hot path of GS-LIVO's Gaussian-map optimisation
(arXiv 2501.08672): projection, tile binning with a device radix sort,
front-to-back alpha compositing and the photometric backward pass to the
Gaussians and each camera's SE(3) pose, behind the C ABI of include/gslivo.h.

The compute runs in libgslivo.so (hand-written HIP); this package only
marshals arguments.  Importing it does not load the library; the first call
does, and fails if the library has not been built.
"""
from ._abi import GslError, SPLAT_BYTES, EXPORTS  # noqa: F401
from . import _abi  # noqa: F401


def __getattr__(name):
    if name in ("ops", "autograd"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
