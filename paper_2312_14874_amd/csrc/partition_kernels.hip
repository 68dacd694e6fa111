// Instantiation of the two-way partition kernel (the compaction kernel with
// the rejected elements written to the end of the output) for gfx950.
#include "compact.hpp"
#include "scan_table.hpp"

namespace mi355scan {

// 256 threads x 64 elements per tile, [vec]
const CompactKernels kPartition = {
    256, 64,
    {(const void *)&compact_tiles<256, 64, false, 3, true>, (const void *)&compact_tiles<256, 64, true, 3, true>},
    nullptr,
};

}  // namespace mi355scan
