"""MI355X-native coupled enthalpy / flow lattice Boltzmann step for
solid-liquid phase change (Li & He, arXiv 1703.02652).

The compute lives in liblbpc.so (hand-written HIP for gfx950, C ABI in
include/lbpc.h); this package marshals arguments and uses PyTorch for device
memory and streams only.
"""
from ._lib import EXPORTS, LIB_PATH, LbpcConfig, LbpcError, lib
from .cavity import Cavity

__all__ = ["Cavity", "LbpcError", "LbpcConfig", "LbpcLoss", "lib", "LIB_PATH", "EXPORTS"]


def __getattr__(name):
    if name == "LbpcLoss":
        from .cavity import _loss_function
        fn = _loss_function()
        globals()["LbpcLoss"] = fn
        return fn
    raise AttributeError(name)
