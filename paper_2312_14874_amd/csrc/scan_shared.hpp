// Types shared by the kernels and the host launcher: the tile status word
// encoding, the workspace header and the kernel argument block.
#pragma once
#include <stdint.h>

namespace mi355scan {

// ----------------------------------------------------------------- status words
// A tile's status is one 64-bit word holding a 2-state flag and its value, so a
// single relaxed agent-scope atomic load or store moves both together; no
// fences are needed (nothing else is published through it).
constexpr uint32_t kEmpty = 0;   // nothing published yet
constexpr uint32_t kAgg = 1;     // value = this tile's own aggregate
constexpr uint32_t kPrefix = 2;  // value = inclusive prefix through this tile

// Workspace header (device memory, zeroed once at allocation).  Two status
// arrays alternate between launches: a launch uses array `parity` and cleans
// array 1-parity, which the previous launch left dirty on [0, dirty[1-parity]).
// The workgroup that performs the launch's last counter increment flips the
// parity; by then every workgroup of the launch has read it.  So no memset or
// reset kernel is needed between launches, also inside graphs.
struct alignas(64) WsHeader {
  uint32_t parity;
  uint32_t error;        // error word of the no-allocation scratch workspace
  uint64_t dirty[2];     // words of status array q that may be non-zero
  uint64_t counter[2];   // tile counters, one per status array
  uint64_t reserved[2];
};
static_assert(sizeof(WsHeader) == 64, "header layout");

struct KernelArgs {
  const void *in;
  void *out;
  int64_t n;
  int64_t tiles;              // number of tiles T
  uint64_t total_acquires;    // counter increments of this launch
  WsHeader *hdr;              // null when tiles == 1
  uint64_t *status;           // 2 * capacity words
  int64_t capacity;           // words per status array
  const int64_t *offsets;     // segmented: S+1 CSR offsets
  const uint32_t *tile_seg;   // segmented: first segment per tile boundary (T+1), or null if T == 1
  int64_t num_segments;
  uint32_t spin_limit;
  uint32_t *err;              // set to 1 when a wait exceeds spin_limit (host-visible word)
  uint32_t exclusive;
  uint32_t reverse;
  uint32_t one_tile;          // every workgroup takes exactly one tile
  uint32_t ordered;           // tile = blockIdx.x (no counter; relies on in-order dispatch)
  uint32_t stride;            // static round robin: workgroup b takes tiles b, b+stride, ... (co-resident grid)
  uint64_t *pubcnt;           // ordered mode: publish counters [2][kPubSlots], kPubStride words apart
  uint32_t key;               // keyed operators (max / min): values are scanned as x ^ key
};

// Arguments of the two-pass kernels (one partition of tiles per launch).
struct TwoPassArgs {
  KernelArgs k;      // in, out, n, tiles (of the whole array), exclusive
  void *sums;        // carry type [tiles]: pass-1 totals, then their exclusive prefixes
  void *run;         // carry type: sum of the partitions before this one
  int64_t tile0;     // first tile of this partition
  int64_t ntiles;    // tiles in this partition
};

// Stream compaction: predicates (the selection is computed on the fly from
// each element) and kernel arguments.
constexpr int kPredNonzero = 0;   // keep x whose 32 bits are not all zero
constexpr int kPredGreater = 1;   // keep x > threshold (typed compare)
// The compare a compaction kernel is built for: the predicate and the dtype
// reduce to one of these (kPredNonzero is an unsigned x > 0).
constexpr int kPkUnsigned = 0;
constexpr int kPkSigned = 1;
constexpr int kPkFloat = 2;

struct CompactArgs {
  KernelArgs k;       // in, out, n, tiles, workspace, counter mode fields
  int64_t *count;     // device: number of kept elements, written by the last tile
  uint32_t thr;       // threshold bits of the kernel's compare (kPk*): x > thr
};

// Ordered launches count published tiles in kPubSlots counters per parity
// (spread over separate cache lines so their atomics do not serialise on one
// address); the last tile waits for the count before handing over.
constexpr int kPubSlots = 64;
constexpr int kPubStride = 16;   // 128 bytes
constexpr int kPubWords = 2 * kPubSlots * kPubStride;

}  // namespace mi355scan
