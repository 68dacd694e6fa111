// Instantiation of the 64-bit integer scan kernel for gfx950.
#include "scan64.hpp"
#include "scan_table.hpp"

namespace mi355scan {

// 512 threads x 64 elements per tile (two per 16-byte group), one resident
// workgroup per CU, the tile's aggregate published before its in-register
// scan; [0 = integer, 1 = float64][reverse]
const void *kScan64[2][2] = {
    {(const void *)&scan64_tiles<OpsAddU64, 512, 64, 2, false, true>,
     (const void *)&scan64_tiles<OpsAddU64, 512, 64, 2, true, true>},
    {(const void *)&scan64_tiles<OpsAddF64, 512, 64, 2, false, true>,
     (const void *)&scan64_tiles<OpsAddF64, 512, 64, 2, true, true>},
};
const int kScan64Block = 512, kScan64Items = 64;

}  // namespace mi355scan
