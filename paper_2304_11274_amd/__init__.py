"""MI355X-native TPFA flux residual / Jacobian / adjoint (arXiv 2304.11274, Sec. 3).

The numerical work runs in libtpfa.so (hand-written HIP for gfx950); this
package only marshals torch tensors into its C ABI (include/tpfa.h).
"""
from ._lib import LIB_PATH, TpfaError, load  # noqa: F401
from .api import (Ensemble, TPFAAnisoResidual, TPFAResidual, TPFATransResidual,  # noqa: F401
                  empty_pitched, empty_sliced, ensemble_run_noalloc, fit_tile_shape,
                  hydrostatic, jacobian, jacobian_be, jvp, offset_pressure, pitch_for,
                  resolve_launch, residual, residual10, residual_and_vjp, residual_be,
                  residual_vjp, sliced_shape, stream_probe, tile_shapes, to_pitched, unslice)

__all__ = ["Ensemble", "TPFAAnisoResidual", "TPFAResidual", "TPFATransResidual", "hydrostatic",
           "jacobian", "jacobian_be", "jvp", "offset_pressure", "residual", "residual10",
           "residual_be", "residual_vjp", "residual_and_vjp", "tile_shapes", "empty_pitched",
           "to_pitched", "pitch_for", "resolve_launch", "stream_probe", "sliced_shape",
           "empty_sliced", "unslice", "ensemble_run_noalloc", "fit_tile_shape", "load",
           "TpfaError", "LIB_PATH"]
