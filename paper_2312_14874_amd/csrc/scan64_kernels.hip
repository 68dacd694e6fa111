// Instantiation of the 64-bit integer scan kernel for gfx950.
#include "scan64.hpp"
#include "scan_table.hpp"

namespace mi355scan {

// 32768-element tiles (two elements per 16-byte group), one resident
// workgroup per CU, the tile's aggregate published before its in-register
// scan: integers as 512 threads x 64 elements, float64 as 1024 x 32 (its
// scan takes fewer registers; measured faster); [0 = integer, 1 = float64]
// [reverse]
const void *kScan64[2][2] = {
    {(const void *)&scan64_tiles<OpsAddU64, 512, 64, 2, false, true>,
     (const void *)&scan64_tiles<OpsAddU64, 512, 64, 2, true, true>},
    {(const void *)&scan64_tiles<OpsAddF64, 1024, 32, 4, false, true>,
     (const void *)&scan64_tiles<OpsAddF64, 1024, 32, 4, true, true>},
};
const int kScan64Block[2] = {512, 1024}, kScan64Items[2] = {64, 32};

}  // namespace mi355scan
