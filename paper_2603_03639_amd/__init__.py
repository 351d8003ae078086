"""MI355X-native hot path of ensemble-robust GRAPE on qubit-chain MPS.

The compute lives in the HIP library ``_lib/libtnrg.so`` (C ABI in
``include/tnrg.h``); ``tnrg`` is its ctypes binding and ``autograd`` the
torch.autograd.Function whose backward pass is the adjoint kernel.
"""
from . import tnrg  # noqa: F401  (raises ImportError when the library is missing)
from .tnrg import (Model, MPSBatch, GrapeCall, TnrgError, grape_fidelity_grad,  # noqa: F401
                   fidelity, mps_evolve, mps_overlap)
from .autograd import EnsembleFidelity, ensemble_fidelity  # noqa: F401
from . import serve  # noqa: F401
from . import optimize  # noqa: F401

__all__ = ["tnrg", "Model", "MPSBatch", "GrapeCall", "TnrgError", "grape_fidelity_grad",
           "fidelity", "mps_evolve", "mps_overlap", "EnsembleFidelity", "ensemble_fidelity",
           "serve", "optimize"]
