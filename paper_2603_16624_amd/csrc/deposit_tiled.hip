// Tiled, LDS-binned moment deposit over cell-sorted particles.
#include "internal.h"

namespace ecsim {

bool tiled_supported(const Grid&) { return false; }

hipError_t launch_deposit_tiled(const Grid&, bool, const SpeciesArgs*, int, const void*, void*, void*, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace ecsim
