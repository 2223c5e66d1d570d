"""MI355X-native contrast-maximization loss (arXiv 2412.06359, Secs. 3.1-3.3).

The loss and its gradient run in HIP kernels for gfx950 behind the C ABI of
include/cmloss.h (libcmloss.so); this package is the thin Python binding.
"""

from .binding import (CM_FLOW_EXACT, CM_FLOW_FIRST_ORDER, CM_MODE_ATOMIC, CM_MODE_DETERMINISTIC,
                      CM_PATH_AUTO, CM_PATH_DIRECT, LAMBDA_GEO, BatchFullLoss, FullLoss,
                      full_loss, geo_backward, geo_forward, geo_state_bytes, rsat, Tuning,
                      get_tuning, set_tuning,
                      CM_PATH_TILED, PHASES, Batch, BatchCMLoss, CMError, CMLoss, WindowDesc,
                      backward, cm_loss,
                      diagnostics, forward, forward_noalloc, handle, load, profile_enable,
                      profile_read, set_path, get_path, state_bytes, NOALLOC_MAX_STATE_BYTES)

__all__ = ["CM_MODE_ATOMIC", "CM_MODE_DETERMINISTIC", "CMError", "CMLoss", "WindowDesc",
           "backward", "cm_loss", "diagnostics", "forward", "handle", "load", "profile_enable",
           "profile_read", "state_bytes", "PHASES", "CM_PATH_AUTO", "CM_PATH_DIRECT",
           "CM_PATH_TILED", "set_path", "get_path", "Batch", "BatchCMLoss", "CM_FLOW_FIRST_ORDER",
           "CM_FLOW_EXACT", "LAMBDA_GEO", "BatchFullLoss", "FullLoss", "full_loss", "geo_backward",
           "geo_forward", "geo_state_bytes", "rsat", "Tuning", "get_tuning", "set_tuning",
           "forward_noalloc", "NOALLOC_MAX_STATE_BYTES"]
