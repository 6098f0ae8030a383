// Host-only parameter logic (params.cpp): validation of a parameter set and
// the tile-edge rules shared by the plan's launch geometry.  Not part of the
// ABI.
#pragma once

#include <string>

#include "pppm.h"

namespace pppm {

// PPPM_OK, or the error of the first rule the parameters break, with the
// reason in `why`.
pppm_status validate_params(const pppm_params* p, std::string& why);

// A tile edge B along an axis of K points is usable when the axis is a single
// tile, or every tile (the last, possibly thinner one included) is at least
// P - 1 points thick, so that a stencil only ever reaches into the next tile.
bool tile_edge_ok(int K, int B, int P);

// A usable edge for an axis of K points near the preferred edge b (see
// params.cpp); K itself (a single tile) when no split works.
int split_tile_edge(int K, int b, int P);

}  // namespace pppm
