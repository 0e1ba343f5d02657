"""BOAC candidate evaluation on AMD MI355X (gfx950).

Evaluates candidate head models for Bayesian-optimisation attenuation correction in SPECT brain
imaging: Legendre outline -> partial-volume attenuation map -> attenuated Radon projector -> MLEM ->
Poisson negative log-likelihood, with an exact reverse-mode gradient, all in hand-written HIP kernels
behind the C ABI in include/boac.h. This package is the Python binding (ctypes over torch device
tensors); importing it does not load the library until a Context is created.
"""
from ._lib import BoacError, header_functions, load  # noqa: F401


def __getattr__(name):
    # lazy: importing the package does not import torch or load libboac.so
    if name in ("Context", "Geometry", "SliceBatch", "BoacObjective", "objective"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
