// scan_cmp.hip -- the exhaustive CMP scan kernels: one per (window, tile shape);
// the tile itself is in tile.h.

#include "tile.h"

namespace semb {

hipError_t launch_scan_cmp(const ScanArgs &a, int shape, hipStream_t stream)
{
    return launch_scan_kind<SEMB_KIND_CMP>(a, shape, stream);
}

}  // namespace semb
