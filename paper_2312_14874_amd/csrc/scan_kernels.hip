// Instantiations of the scan kernel templates for gfx950 and the table the
// host dispatcher and the autotuner choose from.
#include "scan_device.hpp"
#include "scan_table.hpp"

namespace mi355scan {

#define MI355SCAN_FNS(KER, B, I, NT)                                                        \
  {{{(const void *)&KER<OpsU32, B, I, false, (NT != 0), false>,                             \
     (const void *)&KER<OpsU32, B, I, false, (NT != 0), true>},                             \
    {(const void *)&KER<OpsU32, B, I, true, (NT != 0), false>,                              \
     (const void *)&KER<OpsU32, B, I, true, (NT != 0), true>}},                             \
   {{(const void *)&KER<OpsF32, B, I, false, (NT != 0), false>,                             \
     (const void *)&KER<OpsF32, B, I, false, (NT != 0), true>},                             \
    {(const void *)&KER<OpsF32, B, I, true, (NT != 0), false>,                              \
     (const void *)&KER<OpsF32, B, I, true, (NT != 0), true>}}}

#define MI355SCAN_TILES(B, I, NT) {B, I, NT, MI355SCAN_FNS(scan_tiles, B, I, NT)}

const KernelShape kShapes[] = {
    MI355SCAN_TILES(256, 16, 1),     // 0
    MI355SCAN_TILES(256, 32, 1),     // 1
    MI355SCAN_TILES(256, 64, 1),     // 2
    MI355SCAN_TILES(256, 96, 1),     // 3
    MI355SCAN_TILES(256, 128, 1),    // 4
    MI355SCAN_TILES(512, 64, 1),     // 5
};
const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// {shape, mode}: see TileMode.
const Config kConfigs[] = {
    {0, 2}, {1, 2}, {2, 2}, {3, 2}, {4, 2}, {5, 2},   // 0-5   tile = workgroup index
    {4, 1}, {2, 1},                                   // 6-7   resident grid, tiles from the counter
    {2, 4}, {4, 4}, {5, 4},                           // 8-10  resident grid, static round robin
    {0, 0},                                           // 11    one tile per workgroup from the counter
};
const int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

const void *kTileSegmentMap = (const void *)&tile_segment_map;

}  // namespace mi355scan
