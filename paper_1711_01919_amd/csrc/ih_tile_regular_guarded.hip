// Tile-pass kernels of one group of variants (see ih_tile_fns.h).
#include "ih_tile.h"

namespace ih {

TileFns tile_fns_regular_guarded(const TileVariant& v)
{
    return pick_v<false, true>(v);
}

}  // namespace ih
