// Table of compiled kernel shapes and launchable configurations (host side).
#pragma once
#include <stdint.h>

namespace mi355scan {

struct KernelShape {
  int block;         // threads per workgroup
  int items;         // elements per thread (multiple of 4); the tile is block * items
  int nontemporal;   // non-temporal load/store hints
  // [kind: 0 = 32-bit integer sum, 1 = float32 sum, 2 = integer max / min
  //  (keyed), 3 = integer xor][segmented][reverse]
  const void *fn[4][2][2];
  // the streaming-ceiling kernel of this shape (stream_ceiling.hpp): the same
  // tiles and accesses without the scan; null for the unaligned shape
  const void *copy;
};

enum TileMode {
  kModeCounter = 0,      // one tile per workgroup, tile numbers from the counter
  kModePersistent = 1,   // resident grid looping over tiles from the counter
  kModeOrdered = 2,      // tile number = workgroup index
  kModeStatic = 4,       // resident grid (cooperative launch), static round robin
};

struct Config {
  int shape;         // index into kShapes
  int mode;          // TileMode
  int per_cu;        // resident-grid modes: workgroups per CU (0 = as many as fit)
  int cu_pct;        // resident-grid modes: percent of the CUs the grid covers
};

extern const KernelShape kShapes[];
extern const int kNumShapes;
extern const KernelShape kUnalignedShape;   // dword accesses, for buffers not 16-byte aligned
extern const Config kConfigs[];
extern const int kNumConfigs;
extern const void *kTileSegmentMap;   // the tile -> first segment kernel

// Two-pass kernels (Section 2.1 algorithms, for comparison with the single
// pass), one tile shape; indices [0 = 32-bit integer, 1 = float32][vec].
struct TwoPassKernels {
  int block, items;
  const void *totals[2][2][2];      // [op][vec][nontemporal]: tile totals (pass 1, Accumulate)
  const void *local_scan[2][2][2];  // [op][vec][nontemporal]: local scans + totals (pass 1, Prefix Sum)
  const void *offset_scan[2][2];    // [op][vec]: scans with offset (pass 2, Accumulate + Prefix Sum)
  const void *increment[2][2];      // [op][vec]: offset adds (pass 2, Prefix Sum + Increment)
  const void *scan_totals[2];       // [op]: exclusive scan of the tile totals (one workgroup)
  int totals_block;                 // threads of the scan_totals workgroup
};
extern const TwoPassKernels kTwoPass;

// Stream compaction fused with the exclusive scan, one tile shape.
struct CompactKernels {
  int block, items;
  const void *tiles[3][2];   // [predicate kind kPk*][vec]
  const void *set_count;     // writes the count when there is nothing to scan
};
extern const CompactKernels kCompact;
extern const CompactKernels kPartition;   // two-way partition (set_count unused)

// 64-bit scans (flat, 16-byte aligned buffers): [0 = integer sum, 1 = float64
// sum][reverse].
extern const void *kScan64[2][2];
extern const int kScan64Block[2], kScan64Items[2];   // [0 = integer, 1 = float64]

}  // namespace mi355scan
