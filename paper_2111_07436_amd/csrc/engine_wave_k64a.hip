// Fused-kernel instantiations: 64 lanes per cell, 1..3 species per lane.
#include "engine_wave.hpp"

namespace camp {

hipError_t wave_run_64_a(const WaveParams& p, int npl, int stage) {
  switch (npl) {
    case 1: return run_wave<1, 64>(p, stage);
    case 2: return run_wave<2, 64>(p, stage);
    case 3: return run_wave<3, 64>(p, stage);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace camp
