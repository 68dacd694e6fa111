// Instantiations of the scan kernel templates for gfx950 and the table the
// host dispatcher and the autotuner choose from.
#include "scan_device.hpp"
#include "scan_table.hpp"
#include "two_pass.hpp"
#include "compact.hpp"
#include "stream_ceiling.hpp"

namespace mi355scan {

// fn[kind][seg][rev], kind: 0 = 32-bit integer sum, 1 = float32 sum, 2 = max /
// min (keyed unsigned max), 3 = xor; the integer operators share the integer
// sum's register targets.
// W[op][seg]: waves per SIMD the register allocation targets (per shape,
// the most at which the flat variants do not spill).  Workgroups of 768 and
// 1024 threads need 3 and 4 waves per SIMD to fit at all; some of their
// reverse and segmented variants spill a few registers on rare paths.
#define MI355SCAN_FNS(B, I, NT, VEC, WUF, WFF, WUS, WFS, E)                                   \
  {{{(const void *)&scan_tiles<OpsU32, B, I, false, (NT != 0), false, VEC, WUF, E>,            \
     (const void *)&scan_tiles<OpsU32, B, I, false, (NT != 0), true, VEC, WUF, E>},            \
    {(const void *)&scan_tiles<OpsU32, B, I, true, (NT != 0), false, VEC, WUS, E>,             \
     (const void *)&scan_tiles<OpsU32, B, I, true, (NT != 0), true, VEC, WUS>}},               \
   {{(const void *)&scan_tiles<OpsF32, B, I, false, (NT != 0), false, VEC, WFF, E>,            \
     (const void *)&scan_tiles<OpsF32, B, I, false, (NT != 0), true, VEC, WFF, E>},            \
    {(const void *)&scan_tiles<OpsF32, B, I, true, (NT != 0), false, VEC, WFS>,                \
     (const void *)&scan_tiles<OpsF32, B, I, true, (NT != 0), true, VEC, WFS>}},               \
   {{(const void *)&scan_tiles<OpsMaxU32, B, I, false, (NT != 0), false, VEC, WUF, E>,         \
     (const void *)&scan_tiles<OpsMaxU32, B, I, false, (NT != 0), true, VEC, WUF, E>},         \
    {(const void *)&scan_tiles<OpsMaxU32, B, I, true, (NT != 0), false, VEC, WUS>,             \
     (const void *)&scan_tiles<OpsMaxU32, B, I, true, (NT != 0), true, VEC, WUS>}},            \
   {{(const void *)&scan_tiles<OpsXorU32, B, I, false, (NT != 0), false, VEC, WUF, E>,         \
     (const void *)&scan_tiles<OpsXorU32, B, I, false, (NT != 0), true, VEC, WUF, E>},         \
    {(const void *)&scan_tiles<OpsXorU32, B, I, true, (NT != 0), false, VEC, WUS, E>,          \
     (const void *)&scan_tiles<OpsXorU32, B, I, true, (NT != 0), true, VEC, WUS>}}}

// {block, items, nontemporal, waves per SIMD: u32 flat, f32 flat, u32 segmented, f32 segmented}
#define MI355SCAN_TILES(B, I, NT, WUF, WFF, WUS, WFS, E) \
  {B, I, NT, MI355SCAN_FNS(B, I, NT, true, WUF, WFF, WUS, WFS, E), \
   (const void *)&stream_tiles<B, I, (NT != 0), WUF>}

const KernelShape kShapes[] = {
    MI355SCAN_TILES(256, 16, 1, 7, 6, 5, 5, false),      // 0
    MI355SCAN_TILES(256, 32, 1, 6, 5, 5, 3, false),      // 1
    MI355SCAN_TILES(256, 64, 1, 3, 3, 3, 3, false),      // 2
    MI355SCAN_TILES(256, 96, 1, 3, 2, 2, 2, false),      // 3
    MI355SCAN_TILES(256, 128, 1, 2, 2, 2, 2, false),     // 4
    MI355SCAN_TILES(512, 64, 1, 4, 2, 2, 2, false),      // 5
    MI355SCAN_TILES(512, 128, 1, 2, 2, 2, 2, false),     // 6
    MI355SCAN_TILES(1024, 64, 1, 4, 4, 4, 4, false),     // 7
    MI355SCAN_TILES(768, 128, 1, 3, 3, 3, 3, false),     // 8
    // the tile aggregate is published before the in-register scan (EARLY):
    // flat scans, and forward integer-sum and xor segmented scans in tiles
    // without a segment start; other segmented entries as the shapes above
    MI355SCAN_TILES(512, 128, 1, 2, 2, 2, 2, true),      // 9
    MI355SCAN_TILES(256, 128, 1, 2, 2, 2, 2, true),      // 10
    MI355SCAN_TILES(256, 64, 1, 3, 3, 3, 3, true),       // 11
    MI355SCAN_TILES(1024, 64, 1, 4, 4, 4, 4, true),      // 12
};
const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Inputs or outputs that are not 16-byte aligned: dword accesses.
const KernelShape kUnalignedShape = {256, 32, 1, MI355SCAN_FNS(256, 32, 1, false, 4, 4, 3, 3, false), nullptr};

// {shape, mode, workgroups per CU, percent of CUs}: see TileMode and Config.
const Config kConfigs[] = {
    {0, 2, 0, 100}, {1, 2, 0, 100}, {2, 2, 0, 100},   // 0-5   tile = workgroup index
    {3, 2, 0, 100}, {4, 2, 0, 100}, {5, 2, 0, 100},
    {4, 1, 0, 100}, {2, 1, 0, 100},                   // 6-7   resident grid, tiles from the counter
    {2, 4, 0, 100}, {4, 4, 0, 100}, {5, 4, 0, 100},   // 8-10  resident grid, static round robin
    {0, 0, 0, 100},                                   // 11    one tile per workgroup from the counter
    {4, 1, 1, 100}, {4, 1, 2, 100}, {2, 1, 2, 100},   // 12-19 resident grids of fewer workgroups
    {2, 1, 3, 100}, {5, 1, 1, 100}, {3, 1, 2, 100},
    {4, 4, 2, 100}, {2, 4, 3, 100},
    {6, 1, 1, 100}, {7, 1, 1, 100}, {8, 1, 1, 100},   // 20-22 one big workgroup per CU
    {2, 1, 1, 100}, {3, 1, 1, 100},                   // 23-24
    {6, 4, 1, 100}, {8, 4, 1, 100},                   // 25-26 static round robin, one per CU
    {8, 1, 1, 75}, {8, 1, 1, 88}, {6, 1, 1, 75},      // 27-29 one per CU on part of the CUs
    {9, 1, 1, 100}, {10, 1, 1, 100}, {11, 1, 1, 100},   // 30-32 early publication, one per CU
    {10, 1, 2, 100}, {11, 1, 2, 100},                    // 33-34 early publication, two per CU
    {12, 1, 1, 100},                                     // 35    early publication, sixteen waves per CU
};
const int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

// For each tile boundary p in [0, T]: the first segment index s with
// offsets[s] >= p*TILE + shift (shift 1 for reverse scans, where a segment's
// first logical element is its last physical one).  Plain binary search over
// the S+1 offsets; never reads outside offsets[0..S].
__global__ void tile_segment_map(const int64_t *offsets, int64_t num_segments, int64_t tile,
                                 int64_t tiles, int32_t shift, uint32_t *map) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > tiles) return;
  const int64_t x = p * tile + shift;
  int64_t lo = 0, hi = num_segments + 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (offsets[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  map[p] = (uint32_t)lo;
}

const void *kTileSegmentMap = (const void *)&tile_segment_map;

// two-pass kernels: 256 threads x 64 elements (16384-element tiles); the
// trailing template arguments are the kernel's flags, VEC last
#define MI355SCAN_TP(KERNEL, OP, ...) (const void *)&KERNEL<OP, 256, 64, __VA_ARGS__>
const TwoPassKernels kTwoPass = {
    256, 64,
    {{{MI355SCAN_TP(tile_totals, OpsU32, false, false), MI355SCAN_TP(tile_totals, OpsU32, true, false)},
      {MI355SCAN_TP(tile_totals, OpsU32, false, true), MI355SCAN_TP(tile_totals, OpsU32, true, true)}},
     {{MI355SCAN_TP(tile_totals, OpsF32, false, false), MI355SCAN_TP(tile_totals, OpsF32, true, false)},
      {MI355SCAN_TP(tile_totals, OpsF32, false, true), MI355SCAN_TP(tile_totals, OpsF32, true, true)}}},
    {{{MI355SCAN_TP(scan_tile_offset, OpsU32, true, false, false),
       MI355SCAN_TP(scan_tile_offset, OpsU32, true, true, false)},
      {MI355SCAN_TP(scan_tile_offset, OpsU32, true, false, true),
       MI355SCAN_TP(scan_tile_offset, OpsU32, true, true, true)}},
     {{MI355SCAN_TP(scan_tile_offset, OpsF32, true, false, false),
       MI355SCAN_TP(scan_tile_offset, OpsF32, true, true, false)},
      {MI355SCAN_TP(scan_tile_offset, OpsF32, true, false, true),
       MI355SCAN_TP(scan_tile_offset, OpsF32, true, true, true)}}},
    {{MI355SCAN_TP(scan_tile_offset, OpsU32, false, true, false),
      MI355SCAN_TP(scan_tile_offset, OpsU32, false, true, true)},
     {MI355SCAN_TP(scan_tile_offset, OpsF32, false, true, false),
      MI355SCAN_TP(scan_tile_offset, OpsF32, false, true, true)}},
    {{MI355SCAN_TP(increment_tiles, OpsU32, true, false), MI355SCAN_TP(increment_tiles, OpsU32, true, true)},
     {MI355SCAN_TP(increment_tiles, OpsF32, true, false), MI355SCAN_TP(increment_tiles, OpsF32, true, true)}},
    {(const void *)&scan_totals<OpsU32>, (const void *)&scan_totals<OpsF32>},
    kTotalsBlock,
};

// stream compaction: 1024 threads x 64 elements per tile (one workgroup of
// sixteen waves per CU), kept elements written in runs of four chunks,
// [predicate kind][vec]
__global__ void set_count(int64_t *p, int64_t v) { *p = v; }
#define MI355SCAN_COMPACT(PK) \
  { (const void *)&compact_tiles<1024, 64, false, 4, false, PK, 4>, \
    (const void *)&compact_tiles<1024, 64, true, 4, false, PK, 4> }
const CompactKernels kCompact = {
    1024, 64,
    {MI355SCAN_COMPACT(kPkUnsigned), MI355SCAN_COMPACT(kPkSigned), MI355SCAN_COMPACT(kPkFloat)},
    (const void *)&set_count,
};

}  // namespace mi355scan
