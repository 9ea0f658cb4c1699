"""MI355X-native VEGAS+ iteration (arXiv:2408.09229 method) behind a C ABI.

The library ``libvegas_hip.so`` (HIP, gfx950) runs every step of the
iteration; this package is its ctypes binding.  Importing it without the
built library raises ImportError: there is no CPU fallback.
"""
from ._binding import (ACC_FP64, ACC_KAHAN, ACC_ORDERED, EXPORTED, LIB_PATH, PREC_FP32,  # noqa: F401
                       PREC_FP64, UserIntegrand, Vegas, VegasBatch, VegasError, batch_workspace_size, make_config,
                       vegas_batch_info, vegas_config, vegas_estimate, vegas_info, vegas_integrand,
                       workspace_size)
from . import _binding as abi  # noqa: F401
