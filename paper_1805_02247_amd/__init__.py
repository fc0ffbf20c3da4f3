"""Differentiable particle-mesh forward model and hand-written adjoint on MI355X (gfx950).

The compute path is libpmr.so (HIP); this package only binds it (see ``api``), drives the
reconstruction over it (see ``recon``) and prepares inputs on the host (see ``cosmo``).
"""
from ._lib import (PMR_FP32, PMR_MIXED, PMR_LOSS_DENSITY_L2,  # noqa: F401
                   PMR_LOSS_LOGNORMAL, PMR_HALO_SINGLE, PMR_HALO_TWO, PMR_FFT_YPASS,
                   PMR_FFT_XPASS, PMR_FFT_XPASS_MULTI, PMR_E_STATE, PMR_E_NONFINITE,
                   PmrError)
from .api import (Config, GradientGraph, LossParams, PMContext, PMForward,  # noqa: F401
                  cic_paint, cic_sort, fft_c2r, fft_get_slab, fft_get_tile, fft_r2c,
                  fft_set_slab, fft_set_tile, paint_get_rows, paint_set_rows,
                  workspace_bytes)
from . import recon  # noqa: F401,E402
