"""MI355X-native TPFA flux residual / Jacobian / adjoint (arXiv 2304.11274, Sec. 3).

The numerical work runs in libtpfa.so (hand-written HIP for gfx950); this
package only marshals torch tensors into its C ABI (include/tpfa.h).
"""
from ._lib import LIB_PATH, TpfaError, load  # noqa: F401
from .api import (Ensemble, TPFAAnisoResidual, TPFAResidual, TPFATransResidual,  # noqa: F401
                  hydrostatic, jacobian, jacobian_be, jvp, offset_pressure, residual,
                  residual10, residual_be, residual_vjp, tile_shapes)

__all__ = ["Ensemble", "TPFAAnisoResidual", "TPFAResidual", "TPFATransResidual", "hydrostatic",
           "jacobian", "jacobian_be", "jvp", "offset_pressure", "residual", "residual10",
           "residual_be", "residual_vjp", "tile_shapes", "load", "TpfaError", "LIB_PATH"]
