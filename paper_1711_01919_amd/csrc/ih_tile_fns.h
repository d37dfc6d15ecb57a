// Compiled tile-pass kernels by variant: each ih_tile_*.hip source holds
// one group of them.
#pragma once

#include "ih_internal.h"

namespace ih {

// Single-frame and batched entry of one compiled variant.
struct TileFns {
    const void* single;
    const void* batch;
};

TileFns tile_fns_regular(const TileVariant& v);            // regular stores, unguarded
TileFns tile_fns_regular_guarded(const TileVariant& v);    // regular stores, ragged parts
TileFns tile_fns_nontemporal(const TileVariant& v);        // non-temporal stores, unguarded
TileFns tile_fns_nontemporal_guarded(const TileVariant& v);
TileFns tile_fns_table(const TileVariant& v);              // bins from a table (either guard)

inline TileFns tile_fns(const TileVariant& v)
{
    if (v.table) return tile_fns_table(v);
    if (v.nt) return v.guard ? tile_fns_nontemporal_guarded(v) : tile_fns_nontemporal(v);
    return v.guard ? tile_fns_regular_guarded(v) : tile_fns_regular(v);
}

}  // namespace ih
