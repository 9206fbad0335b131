"""Overlapping-domain-decomposition ptychography (OD2P / OD2Pm / OD2BP) on MI355X.

The hot path lives in libodp.so (HIP kernels for gfx950 behind the C ABI of
include/odp.h); this package is its thin binding.  Importing it does not load
the library; the first call does, and fails loudly if it was not built.
"""
from ._lib import (ODP_BALANCE_ETA, ODP_BALANCE_R, ODP_DFT_SPLIT_BF16, ODP_FFT_F32, ODP_HYBRID_MFMA,  # noqa: F401
                   ODP_STOP_NONE,
                   ODP_STOP_RE, ODP_STOP_RF, EXPORTS, OdpError, lib)
from .api import Geometry, Graph, Plan, State, blind_initial_probe_static, prox_stagm  # noqa: F401
from .autograd import AmplitudeLoss, amplitude_loss  # noqa: F401

__version__ = "0.1.0"
