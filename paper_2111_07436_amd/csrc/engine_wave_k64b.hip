// Fused-kernel instantiations: 64 lanes per cell, 4..6 species per lane.
#include "engine_wave.hpp"

namespace camp {

hipError_t wave_run_64_b(const WaveParams& p, int npl, int stage) {
  switch (npl) {
    case 4: return run_wave<4, 64>(p, stage);
    case 5: return run_wave<5, 64>(p, stage);
    case 6: return run_wave<6, 64>(p, stage);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace camp
