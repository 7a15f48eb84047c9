// Fused-kernel instantiations: 64 lanes per cell, 7..9 species per lane.
#include "engine_wave.hpp"

namespace camp {

hipError_t wave_run_64_c(const WaveParams& p, int npl, int stage) {
  switch (npl) {
    case 7: return run_wave<7, 64>(p, stage);
    case 8: return run_wave<8, 64>(p, stage);
    case 9: return run_wave<9, 64>(p, stage);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace camp
