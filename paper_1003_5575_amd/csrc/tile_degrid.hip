// Tile kernel instantiations for mode kDegrid.
#include "tile_dispatch.h"

namespace rts {
template hipError_t launch_tile_mode<kDegrid>(const Plan &, const TileArgs &, hipStream_t, bool);
}  // namespace rts
