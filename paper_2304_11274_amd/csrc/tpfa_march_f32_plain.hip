// FP32 single-grid march kernels with ordinary stores (rows off
// 128-byte lines): every mode kind x rock form (ratios,
// given transmissibilities, per-direction permeability) x tile shape, and the
// VJP with the residual (ratio form).
#include "tpfa_tile.h"

namespace tpfa {

hipError_t launch_march_f32_plain(int kind, int form, int tile, const Args &a, hipStream_t st) {
  switch (form) {
    case 0: return launch_kind<float, MODE_PLAIN>(kind, tile, a, st);
    case MODE_TRANS: return launch_kind<float, MODE_TRANS | MODE_PLAIN>(kind, tile, a, st);
    case MODE_K3: return launch_kind<float, MODE_K3 | MODE_PLAIN>(kind, tile, a, st);
    case MODE_WITH_R:
      return kind == MODE_VJP ? launch_t<float, MODE_VJP | MODE_WITH_R | MODE_PLAIN>(tile, a, st)
                              : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tpfa
