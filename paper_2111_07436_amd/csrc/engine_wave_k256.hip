// Fused-kernel instantiations: 256 lanes per cell, 1..3 species per lane.
#include "engine_wave.hpp"

namespace camp {

hipError_t wave_run_256(const WaveParams& p, int npl, int stage) {
  switch (npl) {
    case 1: return run_wave<1, 256>(p, stage);
    case 2: return run_wave<2, 256>(p, stage);
    case 3: return run_wave<3, 256>(p, stage);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace camp
