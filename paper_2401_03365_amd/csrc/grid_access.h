// grid_access.h -- host access to a built grid's internals for the library's
// own translation units (the public handle stays opaque).
#pragma once

#include "mls_internal.h"

namespace mls {
// The host record of a grid built by mls_build_grid.
const GridHost &grid_host(const mls_grid *grid);
}  // namespace mls
