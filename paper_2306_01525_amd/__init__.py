"""MI355X (gfx950) Meshless Lattice Boltzmann Method: HIP kernels behind a
C-ABI (include/mlbm.h), with a thin PyTorch-side binding.

Importing this package does not touch the GPU; the HIP library is loaded on
first use and its absence raises ImportError.
"""
from ._lib import (MLBM_DEVERR_INDEX, MLBM_DEVERR_NONFINITE,  # noqa: F401
                   MLBM_DEVERR_SINGULAR, MLBM_DEVERR_SPEED, MLBM_FP32_DEV, MLBM_FP64,
                   MLBM_STENCIL_OWN, MLBM_STENCIL_PAPER, MLBMError)


def __getattr__(name):
    if name in ("Plan", "Params"):
        from . import mlbm
        return getattr(mlbm, name)
    if name in ("MLBMRollout", "rollout_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
