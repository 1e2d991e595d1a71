// Tile kernel instantiations for mode kFused.
#include "tile_dispatch.h"

namespace rts {
template hipError_t launch_tile_mode<kFused>(const Plan &, const TileArgs &, hipStream_t, bool);
}  // namespace rts
