// Device side of the single-pass scan for gfx950 (CDNA4, wave64).
//
// Structure of one launch (one tile per workgroup iteration):
//   1. acquire a tile index from a device counter (dynamic, so every tile a
//      workgroup waits on belongs to a workgroup that is already running);
//   2. load the tile once from HBM into registers with 128-bit loads;
//   3. scan in registers: 4 elements serially per lane, then a 64-lane
//      Hillis-Steele scan over the lane totals with DPP row shifts and row
//      broadcasts (the wave-wide counterpart of the in-register horizontal
//      scan of Section 3.1), chunks chained through lane 63;
//   4. combine the wave totals through LDS into the tile aggregate;
//   5. publish the aggregate in the tile's status word, look back over the
//      predecessors' words to obtain the carry, publish the inclusive prefix
//      (the partition sums of Section 2.1, exchanged only between neighbours
//      as Section 2.2.1 suggests instead of a central barrier);
//   6. add the carry and store the tile once.
// Each element is therefore read once and written once: the two-words-per-
// element traffic that the cache-friendly partitioning of Section 2.2 reaches
// on a CPU, with the tile in registers playing the cache-resident partition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "scan_shared.hpp"

namespace mi355scan {

// --------------------------------------------------------------- element ops
// Integers: everything in uint32_t, wrapping modulo 2^32 (int32 uses the same
// bits).
struct OpsU32 {
  using lane_t = uint32_t;    // per-lane arithmetic (up to 256-element chunks)
  using carry_t = uint32_t;   // chunk, wave, tile and inter-tile arithmetic
  static constexpr bool kExact = true;
  // the operator works on keyed values x ^ key (see OpsMaxU32)
  static constexpr bool kKeyed = false;
  // segmented scans: chunks per plain/segmented branch group, and whether a
  // wave without a segment start takes a separate select-free carry add
  // (both chosen by measurement; the float64 carries of OpsF32 need more
  // registers, so it branches in smaller groups and keeps one carry add)
  static constexpr int kSegGroup = 4;
  static constexpr bool kSplitCarry = true;
  // combine_waves folds the wave totals from one lane each (true) or reads
  // each from LDS into registers of its own (false); measured per type: the
  // float64 totals spill the 768 x 128 kernel in the second form
  static constexpr bool kCombineByLane = false;
  // the operator has an inverse (lsub, csub): a segmented scan then runs the
  // plain scan and takes away, from each element at or after a segment start,
  // the plain prefix before that start (exact in wrapping arithmetic)
  static constexpr bool kInverse = true;
  __device__ static lane_t lzero() { return 0u; }
  __device__ static carry_t czero() { return 0u; }
  __device__ static lane_t ladd(lane_t a, lane_t b) { return a + b; }
  __device__ static carry_t cadd(carry_t a, carry_t b) { return a + b; }
  __device__ static lane_t lsub(lane_t a, lane_t b) { return a - b; }
  __device__ static carry_t csub(carry_t a, carry_t b) { return a - b; }
  __device__ static carry_t widen(lane_t x) { return x; }
  __device__ static lane_t narrow(carry_t x) { return x; }
  __device__ static uint32_t lbits(lane_t x) { return x; }
  __device__ static lane_t lfrom(uint32_t b) { return b; }
  __device__ static uint64_t pack(carry_t v, uint32_t f) { return ((uint64_t)f << 32) | v; }
  __device__ static uint32_t flag_of(uint64_t w) { return (uint32_t)(w >> 32); }
  __device__ static carry_t value_of(uint64_t w) { return (uint32_t)w; }
  __device__ static carry_t canon(carry_t x) { return x; }
};

// float32: lanes add in float32 within a 256-element chunk; chunk totals and
// everything above (wave, tile, inter-tile carry) add in float64, so the only
// float32 roundings an output sees are those inside its own chunk plus two
// final ones.  The status word stores the float64 carry with its two lowest
// mantissa bits replaced by the flag; every carry is kept in that truncated
// ("canonical") form, so the inter-tile chain P_k = canon(P_{k-1} + A_k) has
// one value whichever predecessor a tile's look-back stops at.
struct OpsF32 {
  using lane_t = float;
  using carry_t = double;
  static constexpr bool kExact = false;
  static constexpr bool kKeyed = false;
  static constexpr int kSegGroup = 2;
  static constexpr bool kSplitCarry = false;
  static constexpr bool kCombineByLane = true;
  static constexpr bool kInverse = false;   // rounding: restarts, not differences
  __device__ static lane_t lzero() { return 0.0f; }
  __device__ static carry_t czero() { return 0.0; }
  __device__ static lane_t ladd(lane_t a, lane_t b) { return a + b; }
  __device__ static carry_t cadd(carry_t a, carry_t b) { return a + b; }
  __device__ static carry_t widen(lane_t x) { return (double)x; }
  __device__ static lane_t narrow(carry_t x) { return (float)x; }
  __device__ static uint32_t lbits(lane_t x) { return __builtin_bit_cast(uint32_t, x); }
  __device__ static lane_t lfrom(uint32_t b) { return __builtin_bit_cast(float, b); }
  __device__ static uint64_t pack(carry_t v, uint32_t f) {
    return (__builtin_bit_cast(uint64_t, v) & ~3ull) | f;
  }
  __device__ static uint32_t flag_of(uint64_t w) { return (uint32_t)(w & 3u); }
  __device__ static carry_t value_of(uint64_t w) { return __builtin_bit_cast(double, w & ~3ull); }
  __device__ static carry_t canon(carry_t x) { return value_of(pack(x, 0)); }
};

// Other associative operators of the Introduction's definition, on 32-bit
// integers (everything else as OpsU32: the identity of each is 0 in the form
// the kernel computes on, so lanes shifted in by DPP, the exclusive first
// element and a tile's empty carry need nothing new).
//   max / min: one unsigned max over keyed values k(x) = x ^ key, an order
//   isomorphism (or anti-isomorphism) onto uint32 that sends the operator's
//   identity to 0: key 0 = unsigned max, 0x80000000 = signed max (INT_MIN ->
//   0), 0xFFFFFFFF = unsigned min (complement), 0x7FFFFFFF = signed min.
//   The key is applied to a chunk before its scan and removed after the carry.
struct OpsMaxU32 : OpsU32 {
  static constexpr bool kKeyed = true;
  static constexpr bool kInverse = false;
  __device__ static lane_t ladd(lane_t a, lane_t b) { return a > b ? a : b; }
  __device__ static carry_t cadd(carry_t a, carry_t b) { return a > b ? a : b; }
};
//   xor: bitwise exclusive or (identity 0).
struct OpsXorU32 : OpsU32 {
  __device__ static lane_t ladd(lane_t a, lane_t b) { return a ^ b; }
  __device__ static carry_t cadd(carry_t a, carry_t b) { return a ^ b; }
  __device__ static lane_t lsub(lane_t a, lane_t b) { return a ^ b; }
  __device__ static carry_t csub(carry_t a, carry_t b) { return a ^ b; }
};

// ------------------------------------------------------------ memory helpers
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Raise the launch's error flag (a wait gave up).  The flag may be a word of
// pinned host memory that the host polls without synchronising, hence the
// system scope; it is written only on that rare path.
__device__ __forceinline__ void raise_error(uint32_t *err) {
  if (err) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------- wave (DPP) ops
// DPP controls (GFX9 encoding): row_shr:k = 0x110+k, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.  update_dpp(old=0, ...) returns 0
// (the identity) in lanes without a source, so the add below is a no-op there.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

template <class Op, int CTRL, int ROW_MASK>
__device__ __forceinline__ typename Op::lane_t scan_step(typename Op::lane_t x) {
  return Op::ladd(Op::lfrom(dpp<CTRL, ROW_MASK>(Op::lbits(x))), x);
}

// Inclusive scan over the 64 lanes: 4 shift-and-add steps inside each row of
// 16 lanes, then two row broadcasts (the 64-lane form of the log2(w)-step
// in-register scan of Section 3.1).
template <class Op>
__device__ __forceinline__ typename Op::lane_t wave_scan(typename Op::lane_t x) {
  x = scan_step<Op, 0x111, 0xf>(x);
  x = scan_step<Op, 0x112, 0xf>(x);
  x = scan_step<Op, 0x114, 0xf>(x);
  x = scan_step<Op, 0x118, 0xf>(x);
  x = scan_step<Op, 0x142, 0xa>(x);
  x = scan_step<Op, 0x143, 0xc>(x);
  return x;
}

template <class Op, int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_step(typename Op::lane_t &v, uint32_t &f) {
  typename Op::lane_t vk = Op::lfrom(dpp<CTRL, ROW_MASK>(Op::lbits(v)));
  uint32_t fk = dpp<CTRL, ROW_MASK>(f);
  v = f ? v : Op::ladd(vk, v);
  f = f | fk;
}

// Segmented inclusive scan over the lanes of (value, has-segment-start) pairs
// with the operator (a,fa).(b,fb) = (fb ? b : a+b, fa|fb).
template <class Op>
__device__ __forceinline__ void wave_scan_seg(typename Op::lane_t &v, uint32_t &f) {
  seg_step<Op, 0x111, 0xf>(v, f);
  seg_step<Op, 0x112, 0xf>(v, f);
  seg_step<Op, 0x114, 0xf>(v, f);
  seg_step<Op, 0x118, 0xf>(v, f);
  seg_step<Op, 0x142, 0xa>(v, f);
  seg_step<Op, 0x143, 0xc>(v, f);
}

// Value of the next lane down (lane 0 gets the identity).
__device__ __forceinline__ uint32_t lane_up1(uint32_t x) { return dpp<0x138, 0xf>(x); }

__device__ __forceinline__ uint32_t readlane32(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  uint32_t lo = readlane32((uint32_t)x, l);
  uint32_t hi = readlane32((uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// A wave-uniform copy of lane l's value (32- or 64-bit).
template <class T>
__device__ __forceinline__ T readlane_of(T x, int l) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, readlane64(__builtin_bit_cast(uint64_t, x), l));
  else return __builtin_bit_cast(T, readlane32(__builtin_bit_cast(uint32_t, x), l));
}

// The thread index as a value the compiler cannot see through: per-lane
// addresses built from it at a use site stay there instead of being hoisted
// out of the tile loop, where they would hold registers (or spill) for the
// whole kernel although only rare paths and the look-back need them.
__device__ __forceinline__ uint32_t opaque_tid() {
  uint32_t x = threadIdx.x;
  asm volatile("" : "+v"(x));
  return x;
}

// ------------------------------------------------------------------ look-back
// Run by one whole wave.  Lane l, slot k inspects predecessor base-(64k+l)
// (distance d = 64k+l from tile t = base+1).  dP = nearest PREFIX, dE =
// nearest EMPTY.  The window is usable when every word nearer than the PREFIX
// is an AGG; then the carry is the PREFIX value folded left with the AGG
// values of distances dP-1 .. 0.  Integers may also consume a window of AGGs
// and continue further back (addition is exact); float64 carries wait until
// the PREFIX is in the window so that the fold order is always the canonical
// left-to-right chain.

// Issue the loads of one window.  Every lane loads (an index below 0 reads
// tile 0's word, which lb_examine replaces by an empty PREFIX), so no
// instruction consumes the loaded words before they are examined and their
// round trip can overlap other work.  Tile indices are below 2^30 (checked by
// the host), so they and the byte offsets into the status array fit in 32
// bits.
template <class Op, int K>
__device__ __forceinline__ void lb_window(const uint64_t *st, int32_t base, uint64_t (&w)[K]) {
  const int lane = (int)(opaque_tid() & 63u);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int32_t idx = base - (64 * k + lane);
    w[k] = ld_agent(st + (uint32_t)(idx >= 0 ? idx : 0));
  }
}

// What one examined window decided.
enum LbStep { kLbDone = 0, kLbWait = 1, kLbMove = 2 };

// The look-back's state between polls: the window base (the tile of lane 0's
// word), the sum of the aggregates passed so far, the carry once found, and
// what the last examined window decided.  Passed and returned by value, so
// that it stays in registers (through references the compiler kept the base
// and the running sum in private memory, a round trip per poll).
template <class Op>
struct LbState {
  int32_t base;
  typename Op::carry_t acc;
  typename Op::carry_t out;
  int r;
};

// Examine window w of base s.base: kLbDone with the carry in out, kLbWait
// (a needed word is still EMPTY, or a float window holds no PREFIX yet), or
// kLbMove (integers: a full window of aggregates was added to acc and base
// moved back past it).
template <class Op, int KW>
__device__ __forceinline__ LbState<Op> lb_examine(uint64_t (&w)[KW], LbState<Op> s) {
  using carry_t = typename Op::carry_t;
  const int lane = (int)(opaque_tid() & 63u);
  constexpr int kNone = 1 << 30;
  // predecessors before tile 0: an empty prefix
#pragma unroll
  for (int k = 0; k < KW; ++k)
    if (s.base - (64 * k + lane) < 0) w[k] = Op::pack(Op::czero(), kPrefix);
  int dP = kNone, dE = kNone;
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const uint32_t f = Op::flag_of(w[k]);
    const uint64_t bP = ballot(f == kPrefix);
    const uint64_t bE = ballot(f == kEmpty);
    if (dP == kNone && bP) dP = 64 * k + __builtin_ctzll(bP);
    if (dE == kNone && bE) dE = 64 * k + __builtin_ctzll(bE);
  }
  s.r = kLbWait;
  if (dE < dP) return s;
  if (dP == kNone) {
    if constexpr (Op::kExact) {
      // a full window of aggregates: add them all and move further back
      carry_t part = Op::czero();
#pragma unroll
      for (int k = 0; k < KW; ++k) part = Op::cadd(part, Op::value_of(w[k]));
      part = Op::narrow(readlane32(Op::lbits(wave_scan<Op>(part)), 63));
      s.acc = Op::cadd(s.acc, part);
      s.base -= 64 * KW;
      s.r = kLbMove;
    }
    return s;
  }
  if constexpr (Op::kExact) {
    carry_t part = Op::czero();
#pragma unroll
    for (int k = 0; k < KW; ++k)
      if (64 * k + lane <= dP) part = Op::cadd(part, Op::value_of(w[k]));
    part = Op::narrow(readlane32(Op::lbits(wave_scan<Op>(part)), 63));
    s.out = Op::cadd(s.acc, part);
  } else {
    // left fold from the PREFIX at distance dP down to distance 0; the
    // window index k is kept static so no private array is indexed
    // dynamically
    carry_t c = Op::czero();
#pragma unroll
    for (int k = 0; k < KW; ++k)
      if (k == (dP >> 6)) c = Op::value_of(readlane64(w[k], dP & 63));
#pragma unroll
    for (int k = KW - 1; k >= 0; --k) {
      int l = dP - 1 - 64 * k;
      if (l > 63) l = 63;
      for (; l >= 0; --l) c = Op::canon(Op::cadd(c, Op::value_of(readlane64(w[k], l))));
    }
    s.out = c;
  }
  s.r = kLbDone;
  return s;
}

// Exclusive carry into tile t (t >= 1), starting from an already issued
// window w1 of base t-1 (64*K1 tiles); later polls read 64*K tiles each.
template <class Op, int K1, int K>
__device__ typename Op::carry_t look_back(const uint64_t *st, int64_t t, uint32_t spin_limit,
                                          uint32_t *err, uint64_t (&w1)[K1]) {
  LbState<Op> s{(int32_t)t - 1, Op::czero(), Op::czero(), kLbWait};
  s = lb_examine<Op, K1>(w1, s);
  uint32_t spins = 0;
  while (s.r != kLbDone) {
    if (s.r == kLbWait) {
      if (++spins > spin_limit) {
        if ((opaque_tid() & 63u) == 0) raise_error(err);
        return s.acc;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    uint64_t w[K];
    lb_window<Op, K>(st, s.base, w);
    s = lb_examine<Op, K>(w, s);
  }
  return s.out;
}

// Tile addressing.  Logical element e of a tile is physical pb+e going
// forward and pb+TILE-1-e in reverse (a reverse tile is the same aligned block
// read back to front).  Wave w owns logical [w*WSPAN, (w+1)*WSPAN); in chunk c
// lane l holds the 4-group of logical c*256+4l .. c*256+4l+3.  wave_base is
// the lowest physical element of the wave's span (uniform per wave, kept in
// scalar registers).
template <bool REV, int TILE, int WSPAN>
__device__ __forceinline__ int64_t wave_base(int64_t pb, int wave) {
  return REV ? pb + TILE - (int64_t)WSPAN * (wave + 1) : pb + (int64_t)WSPAN * wave;
}
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Hands the workspace to the next launch: clean the rest of the other status
// array and flip the parity.  Called once per launch, by a workgroup that
// knows every workgroup of the launch has already read the parity.
// Run by nthreads threads: the whole workgroup or one wave (nthreads == 64).
__device__ __forceinline__ void hand_over(const KernelArgs &a, uint32_t p, uint64_t clear_hi, int nthreads) {
  uint64_t *other = a.status + (1 - p) * a.capacity;
  const uint32_t me = opaque_tid() % (uint32_t)nthreads;
  const int tid = (int)me;
  for (uint64_t i = (uint64_t)a.tiles + me; i < clear_hi; i += nthreads) st_agent(other + i, 0ull);
  if (tid == 0) {
    st_agent(&a.hdr->counter[1 - p], 0ull);
    st_agent(&a.hdr->dirty[1 - p], 0ull);
    st_agent(&a.hdr->dirty[p], (uint64_t)a.tiles);
    st_agent32(&a.hdr->parity, 1u - p);
  }
}

// Compile-time shape of a tile: BLOCK threads, ITEMS elements each; wave w
// owns the logical span [w*WSPAN, (w+1)*WSPAN) as CH chunks of 256.
template <int BLOCK, int ITEMS>
struct Shape {
  static_assert(BLOCK % 64 == 0 && ITEMS % 4 == 0, "shape");
  static constexpr int WAVES = BLOCK / 64;
  static constexpr int CH = ITEMS / 4;
  static constexpr int WSPAN = 64 * ITEMS;
  static constexpr int TILE = BLOCK * ITEMS;
};

// ---------------------------------------------------------------- tile steps
// Read-only views of the segment map and the offsets through the constant
// address space: a load from it with a wave-uniform address is a scalar
// (SMEM) load, counted apart from the vector loads, so it returns while the
// tile's data is still in flight.  Both arrays are read-only for the whole
// launch (the map is written by the launch before).
typedef const __attribute__((address_space(4))) uint32_t k_u32;
typedef const __attribute__((address_space(4))) int64_t k_i64;

// Segment starts of tile t as an LDS bitmap (TILE bits, logical order).  Whole
// workgroup (contains barriers).  Returns the waves whose span (WSPAN
// logical elements each) holds a start, bit w for wave w; the bitmap is
// written only when that is not zero.  A tile with at most kScalarHeads
// candidate starts (the common case: segments longer than a tile) reads them
// with scalar loads and one lane sets the bits; a tile with more falls back
// to vector loads spread over the workgroup.
// A tile's candidate segment starts, read ahead with scalar loads: the range
// [s_lo, s_hi) of segments from the tile map and, when there are at most
// kScalarHeads of them (segments longer than a tile, the common case), their
// offsets.  The map entries of a resident workgroup's next tile are loaded
// as soon as the tile is taken and the offsets after its loads are issued,
// so mark_heads does not wait for either at the start of the tile.
constexpr int kScalarHeads = 8;
struct HeadsPre {
  uint32_t s_lo, s_hi;          // segments s_lo .. s_hi-1 may start in the tile
  int32_t e[kScalarHeads];      // logical positions of those starts in the tile (-1: none)
};

template <bool REV>
__device__ __forceinline__ void heads_map(const KernelArgs &a, int64_t t, HeadsPre &h) {
  // tiles < 2^29, so the uniform tile index fits one scalar register
  const int pt = __builtin_amdgcn_readfirstlane((int)(REV ? (a.tiles - 1 - t) : t));
  if (a.tile_seg) {
    h.s_lo = ((k_u32 *)a.tile_seg)[pt];
    h.s_hi = ((k_u32 *)a.tile_seg)[pt + 1];
  } else {
    h.s_lo = 0u;
    h.s_hi = (uint32_t)a.num_segments + 1u;
  }
}

template <int TILE, bool REV>
__device__ __forceinline__ void heads_offsets(const KernelArgs &a, int64_t t, HeadsPre &h) {
  const int64_t cnt = (int64_t)h.s_hi - (int64_t)h.s_lo;
  if (a.tile_seg && cnt > 0 && cnt <= kScalarHeads) {
    const int pt = __builtin_amdgcn_readfirstlane((int)(REV ? (a.tiles - 1 - t) : t));
    const int64_t pb = (int64_t)pt * TILE;
    const int64_t rem = a.n - pb;
    const int valid = rem < TILE ? (int)rem : TILE;
    // indices clamped into [s_lo, s_hi - 1] so every load stays inside offsets[0..S]
#pragma unroll
    for (int k = 0; k < kScalarHeads; ++k) {
      const int64_t s = (int64_t)h.s_lo + (k < cnt ? k : cnt - 1);
      const int64_t ph = ((k_i64 *)a.offsets)[s] - (REV ? 1 : 0);   // physical first element (last for reverse)
      const bool in = k < cnt && (REV ? (s >= 1) : (s < a.num_segments)) && ph >= pb && ph < pb + valid;
      h.e[k] = in ? (REV ? (TILE - 1 - (int)(ph - pb)) : (int)(ph - pb)) : -1;
    }
  }
}

template <int BLOCK, int TILE, int WSPAN, bool REV>
__device__ uint32_t mark_heads(const KernelArgs &a, int64_t t, const HeadsPre &h, uint32_t *heads,
                               uint32_t *flag) {
  const int tid = threadIdx.x;
  const int64_t s_lo = h.s_lo, s_hi = h.s_hi;
  if (s_hi <= s_lo) return 0u;
  const int64_t cnt = s_hi - s_lo;
  if (a.tile_seg && cnt <= kScalarHeads) {
    uint32_t waves = 0u;
#pragma unroll
    for (int k = 0; k < kScalarHeads; ++k)
      if (h.e[k] >= 0) waves |= 1u << (h.e[k] / WSPAN);
    if (!waves) return 0u;
    for (int i = tid; i < TILE / 32; i += BLOCK) heads[i] = 0u;
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < kScalarHeads; ++k)
        if (h.e[k] >= 0) atomicOr(&heads[h.e[k] >> 5], 1u << (h.e[k] & 31));
    }
    __syncthreads();
    return waves;
  }
  const int pt = __builtin_amdgcn_readfirstlane((int)(REV ? (a.tiles - 1 - t) : t));
  const int64_t pb = (int64_t)pt * TILE;
  const int64_t rem = a.n - pb;
  const int valid = rem < TILE ? (int)rem : TILE;
  const int shift = REV ? 1 : 0;
  for (int i = tid; i < TILE / 32; i += BLOCK) heads[i] = 0u;
  if (tid == 0) *flag = 0u;
  __syncthreads();
  for (int64_t s = s_lo + tid; s < s_hi; s += BLOCK) {
    const bool real = REV ? (s >= 1) : (s < a.num_segments);
    const int64_t ph = a.offsets[s] - shift;   // physical first element (last for reverse)
    if (real && ph >= pb && ph < pb + valid) {
      const int e = REV ? (TILE - 1 - (int)(ph - pb)) : (int)(ph - pb);
      atomicOr(&heads[e >> 5], 1u << (e & 31));
      atomicOr(flag, 1u << (e / WSPAN));
    }
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*flag);
}

// Buffer resource over one wave's span of WSPAN elements starting at p, of
// which the first `valid` bytes exist (clamped to [0, 4*WSPAN]).  Buffer
// instructions check every dword against that count (the lane offset plus
// the immediate; the scalar offset is always 0 here): loads beyond it return
// 0, the identity of both operators, and stores beyond it are dropped, so
// ragged tiles need no separate path.  The resource lives in scalar
// registers.
template <int WSPAN>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void *p, int64_t valid) {
  const int nr = valid <= 0 ? 0 : (valid >= 4 * WSPAN ? 4 * WSPAN : (int)valid);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, nr, 0x00020000);
}

// Byte offset of lane l's 4-group of chunk c in its wave's span: forward
// 1024c + 16l; reverse (chunks from the top of the span down, lanes from the
// top of the chunk down) 4*WSPAN - 16 - 16l - 1024c.  The per-chunk constant
// becomes the instruction's immediate offset.
template <bool REV, int WSPAN>
__device__ __forceinline__ uint32_t lane_off(int lane) {
  return REV ? 4u * WSPAN - 16u - 16u * (uint32_t)lane : 16u * (uint32_t)lane;
}
template <bool REV>
__device__ __forceinline__ uint32_t chunk_off(uint32_t lo, int c) {
  return REV ? lo - 1024u * (uint32_t)c : lo + 1024u * (uint32_t)c;
}

constexpr int kNtAux = 2;   // cache policy: non-temporal

// Issue the loads of tile t into R; all are issued before any is used.
// Elements beyond n read as the identity.  VEC: 128-bit accesses (the buffer
// is 16-byte aligned); otherwise four dword accesses per 4-group, same layout.
// One wave's view of one tile in a buffer: the resource over the wave's span
// and the lane's byte offset.  Chunk c of the tile is R[c].
template <class SH, bool NT, bool REV, bool VEC>
struct WaveSpan {
  static constexpr int aux = NT ? kNtAux : 0;
  __amdgpu_buffer_rsrc_t rs;
  uint32_t lo;
  __device__ __forceinline__ WaveSpan(const void *buf, const KernelArgs &a, int64_t t, int wave, int lane) {
    const int64_t ptile = REV ? (a.tiles - 1 - t) : t;
    const int64_t wb = wave_base<REV, SH::TILE, SH::WSPAN>(ptile * (int64_t)SH::TILE, wave);
    rs = span_rsrc<SH::WSPAN>(static_cast<const uint32_t *>(buf) + wb, (a.n - wb) * 4);
    // recomputed per tile, so neither it nor the chunk offsets are hoisted
    // out of the tile loop
    lo = lane_off<REV, SH::WSPAN>((int)(opaque_tid() & 63u));
    (void)lane;
  }
  __device__ __forceinline__ void load(int c, u32x4 &r) const {
    if constexpr (VEC) {
      r = __builtin_amdgcn_raw_buffer_load_b128(rs, chunk_off<REV>(lo, c), 0, aux);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, chunk_off<REV>(lo, c) + 4u * k, 0, aux);
    }
  }
  __device__ __forceinline__ void store(int c, const u32x4 &r) const {
    if constexpr (VEC) {
      __builtin_amdgcn_raw_buffer_store_b128(r, rs, chunk_off<REV>(lo, c), 0, aux);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) __builtin_amdgcn_raw_buffer_store_b32(r[k], rs, chunk_off<REV>(lo, c) + 4u * k, 0, aux);
    }
  }
};

template <class SH, bool NT, bool REV, bool VEC>
__device__ __forceinline__ void load_tile(const KernelArgs &a, int64_t t, int wave, int lane,
                                          u32x4 (&R)[SH::CH]) {
  const WaveSpan<SH, NT, REV, VEC> in(a.in, a, t, wave, lane);
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) in.load(c, R[c]);
}

// One chunk of scan_wave without a segment start, in two steps.
// chunk_lane: in-lane inclusive partials of the lane's 4-group (keyed first).
template <class Op, bool REV>
__device__ __forceinline__ void chunk_lane(u32x4 &r, uint32_t key) {
  constexpr int p0 = REV ? 3 : 0, p1 = REV ? 2 : 1, p2 = REV ? 1 : 2, p3 = REV ? 0 : 3;
  constexpr int ph[4] = {p0, p1, p2, p3};
  if constexpr (Op::kKeyed) r ^= key;
#pragma unroll
  for (int k = 1; k < 4; ++k) r[ph[k]] = Op::lbits(Op::ladd(Op::lfrom(r[ph[k - 1]]), Op::lfrom(r[ph[k]])));
}

// chunk_wave: the wave scan of the lane totals, then the chunk's prefix
// within the wave (uniform, wsum; none for the first chunk) joins the lane's
// offset; inclusive: off + p_k, exclusive: off + p_{k-1}, chosen by selects
// so every chunk stays in its own registers.  wsum grows by the chunk total.
template <class Op, bool REV>
__device__ __forceinline__ void chunk_wave(u32x4 &r, typename Op::carry_t &wsum, bool ex, bool first) {
  using lane_t = typename Op::lane_t;
  constexpr int p0 = REV ? 3 : 0, p1 = REV ? 2 : 1, p2 = REV ? 1 : 2, p3 = REV ? 0 : 3;
  const lane_t x = wave_scan<Op>(Op::lfrom(r[p3]));
  const lane_t lex = Op::lfrom(lane_up1(Op::lbits(x)));   // lane-exclusive value in the chunk
  const lane_t ct = Op::lfrom(readlane32(Op::lbits(x), 63));
  const lane_t off = first ? lex : Op::ladd(Op::narrow(wsum), lex);
  r[p3] = Op::lbits(Op::ladd(off, Op::lfrom(ex ? r[p2] : r[p3])));
  r[p2] = Op::lbits(Op::ladd(off, Op::lfrom(ex ? r[p1] : r[p2])));
  r[p1] = Op::lbits(Op::ladd(off, Op::lfrom(ex ? r[p0] : r[p1])));
  r[p0] = ex ? Op::lbits(off) : Op::lbits(Op::ladd(off, Op::lfrom(r[p0])));
  wsum = Op::cadd(wsum, Op::widen(ct));
  // finish the chunk in its own registers now: without this the compiler
  // defers the lane-offset add to the final carry add (one three-operand add
  // per element), keeping one offset register per chunk alive through the
  // look-back
  asm volatile("" : "+v"(r));
}

template <class Op, bool REV>
__device__ __forceinline__ void plain_chunk(u32x4 &r, typename Op::carry_t &wsum, bool ex, bool first,
                                            uint32_t key) {
  chunk_lane<Op, REV>(r, key);
  chunk_wave<Op, REV>(r, wsum, ex, first);
}

// Total over the 64 lanes of a carry-type value (float64 for OpsF32: both
// halves move through the same DPP row shifts and broadcasts as wave_scan),
// in a fixed order; wave-uniform.
template <class Op>
__device__ __forceinline__ typename Op::carry_t wave_total(typename Op::carry_t x) {
  if constexpr (sizeof(typename Op::carry_t) == 4) {
    return Op::widen(Op::lfrom(readlane32(Op::lbits(wave_scan<Op>(Op::narrow(x))), 63)));
  } else {
    auto step = [](typename Op::carry_t v, auto ctrl_tag, auto mask_tag) {
      constexpr int CTRL = decltype(ctrl_tag)::value, MASK = decltype(mask_tag)::value;
      const uint64_t b = __builtin_bit_cast(uint64_t, v);
      const uint64_t s = ((uint64_t)dpp<CTRL, MASK>((uint32_t)(b >> 32)) << 32) | dpp<CTRL, MASK>((uint32_t)b);
      return Op::cadd(__builtin_bit_cast(typename Op::carry_t, s), v);
    };
    x = step(x, std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xf>{});
    x = step(x, std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xf>{});
    x = step(x, std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xf>{});
    x = step(x, std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xf>{});
    x = step(x, std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xa>{});
    x = step(x, std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xc>{});
    return readlane_of(x, 63);
  }
}

// In-register scan of this wave's span (the 64-lane form of the horizontal
// in-register scan of Section 3.1, chained over the chunks).  Logical element
// k of a lane's 4-group sits in slot ph(k) of R[c]: slot k going forward,
// slot 3-k in reverse tiles, so the values never move between slots and the
// group is stored back as it was loaded.  On return the slot of logical
// element k of chunk c holds its wave-local value (inclusive or exclusive,
// restarted at segment starts), fh (segmented, wave-uniform) is the logical
// position within the wave of its first segment start (WSPAN if none): the
// carry into the wave applies to the elements before it and to no others;
// and (wsum, wflag) is the wave's total (since its last segment start) and
// whether it contains a start.  whead: the wave's span holds a segment start
// (the bitmap in heads is read only then).  Segmented, the chunks go in
// groups of Op::kSegGroup: a group without a start takes the plain scan (one
// uniform branch per group, and the group's chunks still interleave), so
// segment starts cost only in the groups that hold them.
template <class Op, class SH, bool SEG, bool REV>
__device__ __forceinline__ void scan_wave(uint32_t exclusive, uint32_t key, int wave, int lane, bool whead,
                                          const uint32_t *heads, u32x4 (&R)[SH::CH], int &fh_out,
                                          typename Op::carry_t &wsum_out, uint32_t &wflag_out) {
  using lane_t = typename Op::lane_t;
  using carry_t = typename Op::carry_t;
  constexpr int p0 = REV ? 3 : 0, p1 = REV ? 2 : 1, p2 = REV ? 1 : 2, p3 = REV ? 0 : 3;
  constexpr int ph[4] = {p0, p1, p2, p3};
  constexpr int G = SEG ? (Op::kSegGroup < SH::CH ? Op::kSegGroup : SH::CH) : SH::CH;
  static_assert(SH::CH % G == 0, "chunk groups must tile the wave span");
  const bool ex = exclusive != 0u;
  carry_t wsum = Op::czero();
  uint32_t wflag = 0u;
  int fh = SH::WSPAN;

  // Chunk that may hold segment starts (hb: this lane's, bit k = logical k).
  auto seg_chunk = [&](const int c, const uint32_t hb) {
    if constexpr (Op::kKeyed) R[c] ^= key;
    // in-lane inclusive partials, restarting at segment starts
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const lane_t sum = Op::ladd(Op::lfrom(R[c][ph[k - 1]]), Op::lfrom(R[c][ph[k]]));
      R[c][ph[k]] = ((hb >> k) & 1u) ? R[c][ph[k]] : Op::lbits(sum);
    }
    lane_t x = Op::lfrom(R[c][p3]);
    uint32_t f = hb != 0u;
    wave_scan_seg<Op>(x, f);
    const uint32_t cf = readlane32(f, 63);   // the chunk holds a start
    const lane_t lex = Op::lfrom(lane_up1(Op::lbits(x)));
    const lane_t ct = Op::lfrom(readlane32(Op::lbits(x), 63));
    const uint32_t lexf = lane_up1(f);   // a segment starts in an earlier lane of the chunk
    // m marks the elements before the chunk's first start: the chunk's
    // prefix within the wave applies to them
    uint32_t m = 0u;
    if (ex) {
      // out_k = head_k ? 0 : value before k in its segment
#pragma unroll
      for (int k = 3; k >= 0; --k) {
        const uint32_t h = (hb >> k) & 1u;
        const uint32_t before = hb & ((1u << k) - 1u);   // starts strictly before k in the lane
        const lane_t prev = k ? Op::lfrom(R[c][ph[k ? k - 1 : 0]]) : Op::lzero();
        const lane_t v = h ? Op::lzero() : (before ? prev : (k ? Op::ladd(lex, prev) : lex));
        R[c][ph[k]] = Op::lbits(v);
        m |= (!h && !before && !lexf) ? (1u << k) : 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t seen = hb & ((2u << k) - 1u);      // starts at or before k
        if (!seen) R[c][ph[k]] = Op::lbits(Op::ladd(lex, Op::lfrom(R[c][ph[k]])));
        m |= (!seen && !lexf) ? (1u << k) : 0u;
      }
    }
    if (c > 0) {
      const lane_t cp = Op::narrow(wsum);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((m >> k) & 1u) R[c][ph[k]] = Op::lbits(Op::ladd(cp, Op::lfrom(R[c][ph[k]])));
    }
    wsum = cf ? Op::widen(ct) : Op::cadd(wsum, Op::widen(ct));
    wflag |= cf;
    asm volatile("" : "+v"(R[c]));
  };

  // the lane's bitmap word in chunk 0 and its bit offset there (the same in
  // every chunk: a chunk is 8 words); the chunk's word index is a constant
  // offset, so no per-chunk address stays live
  const uint32_t *hw = heads + ((wave * SH::WSPAN + lane * 4) >> 5);
  const int hs = (lane * 4) & 31;
#pragma unroll
  for (int g = 0; g < SH::CH; g += G) {
    uint32_t hb[G];
    uint64_t any = 0ull;
#pragma unroll
    for (int j = 0; j < G; ++j) hb[j] = 0u;
    if constexpr (SEG) {
      if (whead) {
        uint32_t o = 0u;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          hb[j] = (hw[(g + j) * 8] >> hs) & 0xfu;
          o |= hb[j];
        }
        any = ballot(o != 0u);
      }
    }
    if (!SEG || any == 0ull) {
#pragma unroll
      for (int j = 0; j < G; ++j) plain_chunk<Op, REV>(R[g + j], wsum, ex, g + j == 0, key);
    } else {
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint64_t hm = ballot(hb[j] != 0u);   // lanes of the chunk with a start
        if (fh == SH::WSPAN && hm != 0ull) {
          const int l = __builtin_ctzll(hm);
          fh = (g + j) * 256 + l * 4 + __builtin_ctz(__builtin_amdgcn_readlane(hb[j], l));
        }
        seg_chunk(g + j, hb[j]);
      }
    }
  }
  fh_out = fh;
  wsum_out = wsum;
  wflag_out = wflag;
}


// Segment starts by subtraction (operators with an inverse).  For a wave
// whose span holds a segment start, after the plain scan_wave (R: the plain
// wave-local prefixes, inclusive or exclusive; wsum: the wave's total) and
// the plain carry add (R += win everywhere): an element at or after a start h
// takes away S_h, the carried plain prefix of the elements before h
// (exclusive: the value at h; inclusive: the value just before h, which for
// h = 0 is the carry into the wave), which leaves the scan of its segment;
// elements before the first start keep the carry.  Per chunk: without a
// start in the chunk every element takes away the latest S; otherwise the
// wave walks the chunk's starts in logical order (lanes up, then elements in
// the lane) with uniform reads, and each start's S replaces the latest one
// from its position on; the latest S passes to the next chunk (SegRun,
// wave-uniform).  It runs chunk by chunk as
// the tile is stored, so that only the chunk being stored passes through the
// branch: a branch over every register of the tile (the segmented carry add
// beside the plain one, or this correction as one pass) makes the
// segmented kernel spill.
template <class Op>
struct SegRun {
  typename Op::lane_t run;         // S of the wave's latest start so far (none: the identity)
  typename Op::lane_t prev_last;   // the value before the next chunk's first element
};
template <class Op, class SH, bool REV>
__device__ __forceinline__ void seg_subtract_chunk(int c, bool ex, int wave, int lane, const uint32_t *heads,
                                                   u32x4 &r, SegRun<Op> &sr) {
  using lane_t = typename Op::lane_t;
  constexpr int p0 = REV ? 3 : 0, p1 = REV ? 2 : 1, p2 = REV ? 1 : 2, p3 = REV ? 0 : 3;
  constexpr int ph[4] = {p0, p1, p2, p3};
  const uint32_t *hw = heads + ((wave * SH::WSPAN + lane * 4) >> 5);
  const uint32_t hb = (hw[c * 8] >> ((lane * 4) & 31)) & 0xfu;   // bit k: a start at logical element k
  uint64_t hm = ballot(hb != 0u);                                  // lanes of the chunk with a start
  const uint32_t last = readlane32(r[p3], 63);
  if (hm == 0ull) {
    // no start in the chunk: every element takes away the latest S
#pragma unroll
    for (int k = 0; k < 4; ++k) r[ph[k]] = Op::lbits(Op::lsub(Op::lfrom(r[ph[k]]), sr.run));
  } else {
    // the starts in logical order (lanes up, then elements within the lane);
    // each one's S replaces the latest S from its position on
    uint32_t sub[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) sub[k] = Op::lbits(sr.run);
    lane_t cur = sr.run;
    while (hm) {
      const int l = __builtin_ctzll(hm);
      hm &= hm - 1ull;
      const uint32_t bits = __builtin_amdgcn_readlane(hb, l);
      const bool gt = lane > l, ge = lane >= l;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((bits >> k) & 1u) {
          // exclusive: the value at the start; inclusive: the value before it
          uint32_t sv;
          if (ex) sv = readlane32(r[ph[k]], l);
          else if (k > 0) sv = readlane32(r[ph[k > 0 ? k - 1 : 0]], l);
          else sv = l > 0 ? readlane32(r[p3], l - 1) : Op::lbits(sr.prev_last);
          cur = Op::lfrom(sv);
#pragma unroll
          for (int j = 0; j < 4; ++j) sub[j] = (j >= k ? ge : gt) ? sv : sub[j];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) r[ph[k]] = Op::lbits(Op::lsub(Op::lfrom(r[ph[k]]), Op::lfrom(sub[k])));
    sr.run = cur;
  }
  sr.prev_last = Op::lfrom(last);
}

// The plain wave-local prefix before the wave's last segment start (the
// start's exclusive value): the wave's total minus it is the total since that
// start, which the wave contributes to the tile aggregate.  Reads R only.
template <class Op, class SH, bool REV>
__device__ __forceinline__ typename Op::lane_t seg_last_prefix(bool ex, int wave, int lane, const uint32_t *heads,
                                                               const u32x4 (&R)[SH::CH]) {
  constexpr int p0 = REV ? 3 : 0, p1 = REV ? 2 : 1, p2 = REV ? 1 : 2, p3 = REV ? 0 : 3;
  constexpr int ph[4] = {p0, p1, p2, p3};
  const uint32_t *hw = heads + ((wave * SH::WSPAN + lane * 4) >> 5);
  const int hs = (lane * 4) & 31;
  // the last start's logical position (uniform; the wave holds one)
  int last = -1;
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) {
    const uint32_t hb = (hw[c * 8] >> hs) & 0xfu;
    const uint64_t hm = ballot(hb != 0u);
    if (hm != 0ull) {
      const int l = 63 - __builtin_clzll(hm);
      last = c * 256 + l * 4 + (31 - __builtin_clz(__builtin_amdgcn_readlane(hb, l)));
    }
  }
  // exclusive: the value at the start; inclusive: the value before it
  const int at = ex ? last : last - 1;
  if (at < 0) return Op::lzero();
  const int tc = at >> 8, tl = (at & 255) >> 2, tk = at & 3;
  uint32_t val = 0u;
#pragma unroll
  for (int c = 0; c < SH::CH; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (c == tc && k == tk) val = readlane32(R[c][ph[k]], tl);
  return Op::lfrom(val);
}

// Wave totals through LDS: this wave's exclusive prefix (wpre, wpref) and
// the tile aggregate (agg, aggf), all folded left to right.  Contains one
// barrier.  With Op::kCombineByLane lane w reads wave w's total and the fold
// runs on wave-uniform copies, so the waves' totals do not each take
// registers of their own; otherwise every total is read from LDS.
template <class Op, int WAVES>
__device__ __forceinline__ void combine_waves(int wave, int lane, typename Op::carry_t wsum, uint32_t wflag,
                                              typename Op::carry_t *s_wtot, uint32_t *s_wflag,
                                              typename Op::carry_t &wpre, uint32_t &wpref,
                                              typename Op::carry_t &agg, uint32_t &aggf) {
  static_assert(WAVES <= 64, "one lane per wave");
  if (lane == 0) {
    s_wtot[wave] = wsum;
    s_wflag[wave] = wflag;
  }
  __syncthreads();
  const int l = lane < WAVES ? lane : 0;
  const typename Op::carry_t tl = Op::kCombineByLane ? s_wtot[l] : Op::czero();
  const uint32_t fl = Op::kCombineByLane ? s_wflag[l] : 0u;
  wpre = Op::czero();
  agg = Op::czero();
  wpref = 0u;
  aggf = 0u;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    if (w == wave) {
      wpre = agg;
      wpref = aggf;
    }
    const typename Op::carry_t tw = Op::kCombineByLane ? readlane_of(tl, w) : s_wtot[w];
    const uint32_t fw = Op::kCombineByLane ? readlane32(fl, w) : s_wflag[w];
    agg = fw ? tw : Op::cadd(agg, tw);
    aggf |= fw;
  }
}

// Wave 0: the tile's first status word.  Tile 0 and tiles that contain a
// segment start know their inclusive prefix at once; the others publish
// their aggregate.
template <class Op>
__device__ __forceinline__ void publish_first(uint64_t *st, int64_t t, typename Op::carry_t agg, uint32_t aggf) {
  if ((threadIdx.x & 63) != 0) return;
  if (t == 0 || aggf) {
    const typename Op::carry_t pv =
        (t == 0 && !aggf) ? Op::canon(Op::cadd(Op::czero(), Op::canon(agg))) : Op::canon(agg);
    st_agent(st + t, Op::pack(pv, kPrefix));
  } else {
    st_agent(st + t, Op::pack(agg, kAgg));
  }
}

// Add the carry into the wave's values: R = win + R where the carry applies
// (every element unless segmented; segmented, the logical positions before
// fh, the wave's first segment start; logical element k of a lane's group
// sits in slot 3-k of reverse tiles).
template <class Op, class SH, bool SEG, bool REV>
__device__ __forceinline__ void apply_carry(typename Op::carry_t win, u32x4 (&R)[SH::CH], int lane, int fh,
                                            uint32_t key = 0u) {
  using lane_t = typename Op::lane_t;
  const lane_t w32 = Op::narrow(win);
  // element k of chunk c takes the carry when c*256 + k < fh - 4*lane (one
  // compare against a constant per element, no per-chunk register)
  const int d = fh - lane * 4;
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int slot = REV ? 3 - k : k;
      const lane_t l = Op::lfrom(R[c][slot]);
      if constexpr (SEG) R[c][slot] = Op::lbits(c * 256 + k < d ? Op::ladd(w32, l) : l);
      else R[c][slot] = Op::lbits(Op::ladd(w32, l));
    }
    if constexpr (Op::kKeyed) R[c] ^= key;   // back from the keyed form
  }
}

// End of a workgroup in a static round-robin launch: count it; the last
// workgroup (all others have finished, so all have read the parity) hands
// the workspace over.  The counter of the launch's parity serves as the
// count; the hand-over clears the other parity's counter for the next launch.
__device__ __forceinline__ void static_done(const KernelArgs &a, uint32_t parity, int tid, int nthreads,
                                            uint32_t *flag, uint64_t *clear_hi) {
  __syncthreads();
  if (tid == 0) {
    const uint64_t d = __hip_atomic_fetch_add(&a.hdr->counter[parity], 1ull, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    *flag = d == (uint64_t)gridDim.x - 1;
    if (*flag) *clear_hi = ld_agent(&a.hdr->dirty[1 - parity]);
  }
  __syncthreads();
  if (*flag) hand_over(a, parity, *clear_hi, nthreads);
}

// ------------------------------------------------------------------- kernels
// Counter modes: take the next tile from the device counter.  Run by one
// whole wave; the result is uniform (>= tiles when none is left).  The
// launch's last increment hands the workspace over: every workgroup has read
// the parity before its first increment.
// The increment itself (lane 0; the other lanes get 0), so that its round
// trip can overlap other work before acquire_finish reads the result.
__device__ __forceinline__ uint64_t acquire_issue(const KernelArgs &a, uint32_t parity, int lane) {
  return lane == 0 ? __hip_atomic_fetch_add(&a.hdr->counter[parity], 1ull, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                   : 0ull;
}
// Clean the tile's word of the other parity, hand over after the launch's
// last increment; returns the tile number, wave-uniform.
__device__ __forceinline__ int64_t acquire_finish(const KernelArgs &a, uint32_t parity, int lane, uint64_t tk) {
  uint64_t clear_hi = 0;
  uint32_t last = 0;
  if (lane == 0) {
    last = tk == a.total_acquires - 1;
    if (tk < (uint64_t)a.tiles) st_agent(a.status + (1 - parity) * a.capacity + tk, 0ull);
    if (last) clear_hi = ld_agent(&a.hdr->dirty[1 - parity]);
  }
  tk = readlane64(tk, 0);
  if (readlane32(last, 0)) hand_over(a, parity, readlane64(clear_hi, 0), 64);
  return (int64_t)tk;
}
__device__ __forceinline__ int64_t acquire_tile(const KernelArgs &a, uint32_t parity, int lane) {
  return acquire_finish(a, parity, lane, acquire_issue(a, parity, lane));
}

// One tile per workgroup iteration.  Tile numbers come from the device counter
// (dynamic: any workgroup that waits depends only on workgroups that are
// already running), from blockIdx.x with `ordered` (no counter; this relies
// on the dispatcher starting workgroups in index order, so a workgroup's
// predecessors have all been started before it), or round robin over a
// co-resident grid with `stride`.  A resident workgroup takes its next tile
// only when it is ready to load it (after its look-back): tiles then start
// close to index order, which keeps the look-back waits short (taking the
// next tile earlier, during the look-back, measured slower).  The next tile's
// loads are issued between the current tile's stores, into the registers
// each store frees.  Shared-memory values alternate between two slots per
// iteration, so consecutive tiles need no barrier between them.
// MINW: waves per SIMD the register allocation must allow (the number of
// workgroups of 4 waves resident per CU).
// EARLY (flat scans): the tile's aggregate is formed and published before
// the in-register scan, from the lane sums of the in-lane partials, and the
// first look-back poll (64*K1 tiles) is issued right behind it, so that its
// round trip overlaps the scan and successors see the aggregate sooner.
template <class Op, int BLOCK, int ITEMS, bool SEG, bool NT, bool REV, bool VEC, int MINW, bool EARLY = false>
__global__ void __launch_bounds__(BLOCK, MINW) scan_tiles(KernelArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  constexpr int K = 4;   // look-back window = 64*K tiles per poll
  constexpr int K1 = 1;  // EARLY: first poll, issued before the scan
  constexpr bool kEarly = EARLY && !SEG;
  // segmented, operators with an inverse: a tile without a segment start
  // publishes its aggregate before the scan, as kEarly does (forward scans:
  // the reverse variant's registers do not fit it)
  constexpr bool kSegEarly = EARLY && SEG && Op::kInverse && !REV;
  using carry_t = typename Op::carry_t;

  __shared__ carry_t s_wtot[2][SH::WAVES];
  __shared__ uint32_t s_wflag[2][SH::WAVES];
  __shared__ carry_t s_carry[2];
  __shared__ int64_t s_tile[2];
  __shared__ uint64_t s_clear_hi;
  __shared__ uint32_t s_parity, s_flag;
  // segment starts of the tile, one bit per element; two, alternating by
  // tile: a wave may still read the last tile's bits while it stores (the
  // subtraction of segmented scans) when another wave marks the next tile's
  __shared__ uint32_t s_heads[2][SEG ? SH::TILE / 32 : 1];
  __shared__ carry_t s_etot[kSegEarly ? SH::WAVES : 1];   // wave totals of kSegEarly

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const bool multi = a.tiles > 1;
  const bool counter = multi && !a.ordered && !a.stride;
  const bool resident = counter && !a.one_tile;
  uint32_t parity = 0;

  // ------------------------------------------------ first tile
  int64_t t = 0;
  if (multi) {
    if (wave == 0) {
      parity = readlane32(lane == 0 ? ld_agent32(&a.hdr->parity) : 0u, 0);
      if (a.ordered) {
        t = blockIdx.x;
        if (lane == 0) {
          st_agent(a.status + (1 - parity) * a.capacity + t, 0ull);
          s_clear_hi = (t == a.tiles - 1) ? ld_agent(&a.hdr->dirty[1 - parity]) : 0ull;
        }
      } else if (a.stride) {
        t = blockIdx.x;
      } else {
        t = acquire_tile(a, parity, lane);
      }
      if (lane == 0) {
        s_parity = parity;
        s_tile[0] = t;
      }
    }
    __syncthreads();
    parity = s_parity;
    t = s_tile[0];
  }

  u32x4 R[SH::CH];
  if (t < a.tiles) load_tile<SH, NT, REV, VEC>(a, t, wave, lane, R);
  HeadsPre heads_pre;   // segmented: the current tile's segment starts, read ahead
  if constexpr (SEG) {
    if (t < a.tiles) {
      heads_map<REV>(a, t, heads_pre);
      heads_offsets<SH::TILE, REV>(a, t, heads_pre);
    }
  }

  for (int it = 0;; ++it) {
    const int slot = it & 1;
    if (t >= a.tiles) break;
    if (a.stride && tid == 0) st_agent(a.status + (1 - parity) * a.capacity + t, 0ull);

    uint32_t head_waves = 0u;   // bit w: wave w's span holds a segment start
    if constexpr (SEG) head_waves = mark_heads<BLOCK, SH::TILE, SH::WSPAN, REV>(a, t, heads_pre, s_heads[slot], &s_flag);

    // the tile's loads are in flight: scan in registers, combine the waves
    int fh;
    carry_t wsum, wpre, agg;
    uint32_t wflag, wpref, aggf;
    bool first_is_head = false;
    if constexpr (SEG) first_is_head = (head_waves & 1u) && (s_heads[slot][0] & 1u);
    const bool need_carry = t > 0 && !first_is_head;
    if constexpr (kEarly) {
      // lane partials of every chunk as it arrives, and the lane total
      constexpr int p3 = REV ? 0 : 3;
      carry_t lt = Op::czero();
#pragma unroll
      for (int c = 0; c < SH::CH; ++c) {
        chunk_lane<Op, REV>(R[c], a.key);
        lt = Op::cadd(lt, Op::widen(Op::lfrom(R[c][p3])));
      }
      combine_waves<Op, SH::WAVES>(wave, lane, wave_total<Op>(lt), 0u, s_wtot[slot], s_wflag[slot], wpre, wpref,
                                   agg, aggf);
      // publish the aggregate and issue the first poll
      uint64_t w1[K1];
      if (multi && wave == 0) {
        uint64_t *st = a.status + parity * a.capacity;
        publish_first<Op>(st, t, agg, aggf);
        if (a.ordered && lane == 0 && t != a.tiles - 1)
          (void)__hip_atomic_fetch_add(a.pubcnt + (parity * kPubSlots + (t % kPubSlots)) * kPubStride, 1ull,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (need_carry) lb_window<Op, K1>(st, (int32_t)t - 1, w1);
      }
      // the rest of the scan while the poll is in flight
      const bool ex = a.exclusive != 0u;
      wsum = Op::czero();
#pragma unroll
      for (int c = 0; c < SH::CH; ++c) chunk_wave<Op, REV>(R[c], wsum, ex, c == 0);
      fh = SH::WSPAN;
      if (multi && wave == 0) {
        uint64_t *st = a.status + parity * a.capacity;
        carry_t carry = Op::czero();
        if (need_carry) {
          carry = look_back<Op, K1, K>(st, t, a.spin_limit, a.err, w1);
          if (lane == 0) st_agent(st + t, Op::pack(Op::canon(Op::cadd(carry, Op::canon(agg))), kPrefix));
        }
        if (lane == 0) s_carry[slot] = carry;
      }
    } else {
      // kSegEarly, a tile without a segment start: the lanes' sums of the
      // loaded values (R is only read), the wave totals and the aggregate,
      // published with the first poll issued before the scan
      bool seg_early = false;
      uint64_t w1s[K1];
      if constexpr (kSegEarly) {
        seg_early = head_waves == 0u && need_carry && multi;
        if (seg_early) {
          typename Op::lane_t ls = Op::lzero();
#pragma unroll
          for (int c = 0; c < SH::CH; ++c)
            ls = Op::ladd(ls, Op::ladd(Op::ladd(Op::lfrom(R[c][0]), Op::lfrom(R[c][1])),
                                       Op::ladd(Op::lfrom(R[c][2]), Op::lfrom(R[c][3]))));
          const carry_t wt = wave_total<Op>(Op::widen(ls));
          if (lane == 0) s_etot[wave] = wt;
          __syncthreads();
          carry_t ea = Op::czero();
#pragma unroll
          for (int w = 0; w < SH::WAVES; ++w) ea = Op::cadd(ea, s_etot[w]);
          if (wave == 0) {
            uint64_t *st = a.status + parity * a.capacity;
            publish_first<Op>(st, t, ea, 0u);
            lb_window<Op, K1>(st, (int32_t)t - 1, w1s);
          }
        }
      }
      if constexpr (SEG && Op::kInverse) {
        // the flat scan's code for every wave; a wave that holds a segment
        // start contributes its total since the last one (the elements are
        // corrected after the carry, by seg_subtract)
        scan_wave<Op, SH, false, REV>(a.exclusive, a.key, wave, lane, false, s_heads[slot], R, fh, wsum, wflag);
        if ((head_waves >> wave) & 1u) {
          wsum = Op::csub(wsum, Op::widen(seg_last_prefix<Op, SH, REV>(a.exclusive != 0u, wave, lane, s_heads[slot], R)));
          wflag = 1u;
        }
      } else {
        scan_wave<Op, SH, SEG, REV>(a.exclusive, a.key, wave, lane, (head_waves >> wave) & 1u, s_heads[slot], R, fh,
                                    wsum, wflag);
      }
      combine_waves<Op, SH::WAVES>(wave, lane, wsum, wflag, s_wtot[slot], s_wflag[slot], wpre, wpref, agg, aggf);

      // publish, look back, publish the prefix
      if (multi && wave == 0) {
        uint64_t *st = a.status + parity * a.capacity;
        if (!seg_early) publish_first<Op>(st, t, agg, aggf);
        if (a.ordered && lane == 0 && t != a.tiles - 1)
          (void)__hip_atomic_fetch_add(a.pubcnt + (parity * kPubSlots + (t % kPubSlots)) * kPubStride, 1ull,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        carry_t carry = Op::czero();
        if (need_carry) {
          if (seg_early) {
            carry = look_back<Op, K1, K>(st, t, a.spin_limit, a.err, w1s);
          } else {
            uint64_t w[K];
            lb_window<Op, K>(st, (int32_t)t - 1, w);
            carry = look_back<Op, K, K>(st, t, a.spin_limit, a.err, w);
          }
          if (!aggf && lane == 0)
            st_agent(st + t, Op::pack(Op::canon(Op::cadd(carry, Op::canon(agg))), kPrefix));
        }
        if (lane == 0) s_carry[slot] = carry;
      }
    }
    __syncthreads();
    const carry_t carry = need_carry ? s_carry[slot] : Op::czero();
    const carry_t win = wpref ? wpre : Op::cadd(carry, wpre);
    // a wave without a segment start may add the carry everywhere (no selects)
    // segmented by subtraction: the plain carry add here, the correction of a
    // wave that holds a start chunk by chunk as the tile is stored
    const bool fix = SEG && Op::kInverse && ((head_waves >> wave) & 1u);
    SegRun<Op> sr{Op::lzero(), Op::narrow(win)};
    auto store_chunk = [&](const WaveSpan<SH, NT, REV, VEC> &out, const int c) {
      if constexpr (SEG && Op::kInverse) {
        if (fix) seg_subtract_chunk<Op, SH, REV>(c, a.exclusive != 0u, wave, lane, s_heads[slot], R[c], sr);
      }
      out.store(c, R[c]);
    };
    if constexpr (SEG && Op::kInverse) {
      apply_carry<Op, SH, false, REV>(win, R, lane, fh, a.key);
    } else if (SEG && (!Op::kSplitCarry || fh < SH::WSPAN)) {
      apply_carry<Op, SH, SEG, REV>(win, R, lane, fh, a.key);
    } else {
      apply_carry<Op, SH, false, REV>(win, R, lane, fh, a.key);
    }

    // Store the tile and load the next one into the same registers: the
    // first half of the stores goes out while the next tile is taken from the
    // counter; then each further store frees a chunk that the next tile's
    // load fills at once, so reads and writes share the CU's memory
    // pipeline instead of alternating.
    constexpr int KH = SH::CH / 2;
    const WaveSpan<SH, NT, REV, VEC> out(a.out, a, t, wave, lane);
#pragma unroll
    for (int c = 0; c < KH; ++c) store_chunk(out, c);
    int64_t next = a.stride ? t + a.stride : a.tiles;
    if (resident) {
      if (wave == 0) {
        const int64_t tk = acquire_tile(a, parity, lane);
        if (lane == 0) s_tile[slot ^ 1] = tk;
      }
      __syncthreads();
      next = s_tile[slot ^ 1];
    }
    if (next < a.tiles) {
      const WaveSpan<SH, NT, REV, VEC> in(a.in, a, next, wave, lane);
      if constexpr (SEG) heads_map<REV>(a, next, heads_pre);
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) {
        store_chunk(out, c);
        in.load(c - KH, R[c - KH]);
      }
#pragma unroll
      for (int c = SH::CH - KH; c < SH::CH; ++c) in.load(c, R[c]);
      if constexpr (SEG) heads_offsets<SH::TILE, REV>(a, next, heads_pre);
    } else {
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) store_chunk(out, c);
    }

    if (multi && a.ordered) {
      if (t == a.tiles - 1) {
        // wait until every other tile has published (so every workgroup of
        // the launch has read the parity), then hand the workspace over
        if (wave == 0) {
          const uint32_t l = opaque_tid() & 63u;
          const uint64_t *cnt = a.pubcnt + (parity * kPubSlots + l) * kPubStride;
          for (uint32_t spins = 0;; ++spins) {
            uint32_t c = (uint32_t)ld_agent(cnt);
            c = readlane32(wave_scan<OpsU32>(c), 63);
            if ((int64_t)c >= a.tiles - 1) break;
            if (spins > a.spin_limit) {
              if (lane == 0) raise_error(a.err);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          // every increment of this launch has landed: leave both parities'
          // counters at zero, so the next ordered launch on either parity
          // starts from zero whatever ran in between (other modes never
          // touch them)
          st_agent(a.pubcnt + (parity * kPubSlots + l) * kPubStride, 0ull);
          st_agent(a.pubcnt + ((1 - parity) * kPubSlots + l) * kPubStride, 0ull);
        }
        __syncthreads();
        hand_over(a, parity, s_clear_hi, BLOCK);
      }
      break;
    }
    t = next;
  }
  if (multi && a.stride) static_done(a, parity, tid, BLOCK, &s_flag, &s_clear_hi);
}

}  // namespace mi355scan
