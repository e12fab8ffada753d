// FP32 single-grid march kernels with non-temporal stores: every mode kind x rock form (ratios,
// given transmissibilities, per-direction permeability) x tile shape, and the
// VJP with the residual (ratio form).
#include "tpfa_tile.h"

namespace tpfa {

hipError_t launch_march_f32(int kind, int form, int tile, const Args &a, hipStream_t st) {
  switch (form) {
    case 0: return launch_kind<float, 0>(kind, tile, a, st);
    case MODE_TRANS: return launch_kind<float, MODE_TRANS | 0>(kind, tile, a, st);
    case MODE_K3: return launch_kind<float, MODE_K3 | 0>(kind, tile, a, st);
    case MODE_WITH_R:
      return kind == MODE_VJP ? launch_t<float, MODE_VJP | MODE_WITH_R>(tile, a, st)
                              : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

const void *march_kernel_f32(int kind, int form, int tile) {
  switch (form) {
    case 0: return kernel_kind<float, 0>(kind, tile);
    case MODE_TRANS: return kernel_kind<float, MODE_TRANS>(kind, tile);
    case MODE_K3: return kernel_kind<float, MODE_K3>(kind, tile);
    case MODE_WITH_R:
      return kind == MODE_VJP ? kernel_t<float, MODE_VJP | MODE_WITH_R>(tile) : nullptr;
    default: return nullptr;
  }
}

}  // namespace tpfa
