// Tile-pass kernels of one group of variants (see ih_tile_fns.h).
#include "ih_tile.h"

namespace ih {

TileFns tile_fns_table(const TileVariant& v)
{
    return v.guard ? pick_table<true>(v) : pick_table<false>(v);
}

}  // namespace ih
