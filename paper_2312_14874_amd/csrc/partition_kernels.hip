// Instantiation of the two-way partition kernel (the compaction kernel with
// the rejected elements written to the end of the output) for gfx950.
#include "compact.hpp"
#include "scan_table.hpp"

namespace mi355scan {

// 1024 threads x 64 elements per tile, each chunk's two runs written on
// their own (longer runs measured no faster here), [predicate kind][vec]
#define MI355SCAN_PARTITION(PK) \
  { (const void *)&compact_tiles<1024, 64, false, 4, true, PK, 1>, \
    (const void *)&compact_tiles<1024, 64, true, 4, true, PK, 1> }
const CompactKernels kPartition = {
    1024, 64,
    {MI355SCAN_PARTITION(kPkUnsigned), MI355SCAN_PARTITION(kPkSigned), MI355SCAN_PARTITION(kPkFloat)},
    nullptr,
};

}  // namespace mi355scan
