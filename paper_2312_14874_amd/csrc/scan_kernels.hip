// Instantiations of the scan kernel template for gfx950 and the table the
// host dispatcher and the autotuner choose from.
#include "scan_device.hpp"
#include "scan_table.hpp"

namespace mi355scan {

#define MI355SCAN_SHAPE(B, I, NT)                                               \
  {B, I, NT,                                                                    \
   {{(const void *)&scan_tiles<OpsU32, B, I, false, (NT != 0)>,                 \
     (const void *)&scan_tiles<OpsU32, B, I, true, (NT != 0)>},                 \
    {(const void *)&scan_tiles<OpsF32, B, I, false, (NT != 0)>,                 \
     (const void *)&scan_tiles<OpsF32, B, I, true, (NT != 0)>}}}

const KernelShape kShapes[] = {
    MI355SCAN_SHAPE(256, 16, 0),  MI355SCAN_SHAPE(256, 32, 0),  MI355SCAN_SHAPE(512, 16, 0),
    MI355SCAN_SHAPE(512, 32, 0),  MI355SCAN_SHAPE(1024, 16, 0), MI355SCAN_SHAPE(256, 16, 1),
    MI355SCAN_SHAPE(256, 32, 1),  MI355SCAN_SHAPE(512, 16, 1),  MI355SCAN_SHAPE(512, 32, 1),
    MI355SCAN_SHAPE(1024, 16, 1),
};
const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Configurations 0..9: one tile per workgroup; 10..19: persistent grid.
const Config kConfigs[] = {
    {0, 0}, {1, 0}, {2, 0}, {3, 0}, {4, 0}, {5, 0}, {6, 0}, {7, 0}, {8, 0}, {9, 0},
    {0, 1}, {1, 1}, {2, 1}, {3, 1}, {4, 1}, {5, 1}, {6, 1}, {7, 1}, {8, 1}, {9, 1},
};
const int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

const void *kTileSegmentMap = (const void *)&tile_segment_map;

}  // namespace mi355scan
