// Fused-kernel instantiations: 128 lanes per cell, 1..5 species per lane.
#include "engine_wave.hpp"

namespace camp {

hipError_t wave_run_128(const WaveParams& p, int npl, int stage) {
  switch (npl) {
    case 1: return run_wave<1, 128>(p, stage);
    case 2: return run_wave<2, 128>(p, stage);
    case 3: return run_wave<3, 128>(p, stage);
    case 4: return run_wave<4, 128>(p, stage);
    case 5: return run_wave<5, 128>(p, stage);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace camp
