// Tile kernel instantiations for mode kGrid.
#include "tile_dispatch.h"

namespace rts {
template hipError_t launch_tile_mode<kGrid>(const Plan &, const TileArgs &, hipStream_t, bool);
}  // namespace rts
