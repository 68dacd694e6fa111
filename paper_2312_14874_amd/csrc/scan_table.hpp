// Table of compiled kernel shapes and launchable configurations (host side).
#pragma once
#include <stdint.h>

namespace mi355scan {

struct KernelShape {
  int block;         // threads per workgroup
  int items;         // elements per thread (multiple of 4)
  int nontemporal;   // non-temporal load/store hints
  const void *fn[2][2];   // [0 = 32-bit integer, 1 = float32][segmented]
};

struct Config {
  int shape;         // index into kShapes
  int persistent;    // grid = resident workgroups, tiles taken in a loop
};

extern const KernelShape kShapes[];
extern const int kNumShapes;
extern const Config kConfigs[];
extern const int kNumConfigs;
extern const void *kTileSegmentMap;   // the tile -> first segment kernel

}  // namespace mi355scan
