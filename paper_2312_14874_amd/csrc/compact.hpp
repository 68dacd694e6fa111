// Stream compaction fused with the exclusive scan: the Introduction's main
// use of prefix sums -- the exclusive scan of a 0/1 selection gives every
// kept element its index in the output (the partitioning / parallel
// filtering use).  One pass: each tile is loaded once, its selection is
// counted and scanned in registers, the tile's carry (number of elements
// kept before it) comes from the same decoupled look-back as the scan, and
// the kept elements are written to their final places.  HBM traffic: 4 bytes
// read per element plus 4 written per kept element.
//
// With PART the kernel is a two-way partition: in addition, an element that
// is not kept goes to out[n-1-r], r being the number of rejected elements
// before it (its index minus the number kept before it), so the rejected
// elements fill the end of the output in reverse order and every element is
// written once (8 bytes of traffic per element).
#pragma once
#include "scan_device.hpp"

namespace mi355scan {

__device__ __forceinline__ bool keep_element(uint32_t x, const CompactArgs &a) {
  if (a.pred == kPredNonzero) return x != 0u;
  if (a.dtype == 0) return (int32_t)x > (int32_t)a.thr;
  if (a.dtype == 1) return x > a.thr;
  return __builtin_bit_cast(float, x) > __builtin_bit_cast(float, a.thr);   // NaN never kept
}

// One tile per iteration of a resident grid (tiles from the device counter,
// the workspace protocol of scan_tiles).  Per chunk each lane keeps a 4-bit
// selection mask (8 chunks per register); the tile total needs only the
// lanes' counts, and a chunk's positions are scanned when it is written.
// The values stay in R until they are written: per chunk, the wave packs its
// kept elements into its own LDS row (every element is written somewhere, so
// no per-element branch) and writes them out as one contiguous run, one
// 128-bit store per lane, instead of one scattered store per element; as in
// scan_tiles, the registers a packed chunk frees take the next tile's chunk at
// once.  The output offsets are wave-uniform and kept in scalar registers:
// a buffer resource the compiler must treat as per-lane would turn every
// store into a loop over its distinct values.
// Counts of kept elements: 32-bit integer sums whose wave totals are folded
// from one lane each (no register per wave's total).
struct OpsCount : OpsU32 {
  static constexpr bool kCombineByLane = true;
};

template <int BLOCK, int ITEMS, bool VEC, int MINW, bool PART = false>
__global__ void __launch_bounds__(BLOCK, MINW) compact_tiles(CompactArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using Op = OpsCount;
  constexpr int K = 4;
  // store cache policy: non-temporal for compaction; the partition's two
  // output streams write faster through the default policy (measured)
  constexpr int SAUX = PART ? 0 : kNtAux;
  constexpr int MW = (SH::CH + 7) / 8;   // mask words
  __shared__ uint32_t s_wtot[SH::WAVES];
  __shared__ uint32_t s_wflag[SH::WAVES];
  __shared__ uint32_t s_carry;
  __shared__ int64_t s_tile;
  __shared__ uint32_t s_parity;
  __shared__ __attribute__((aligned(16))) uint32_t s_stage[SH::WAVES][768];   // see pack
  const KernelArgs &ka = a.k;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const bool multi = ka.tiles > 1;
  uint32_t parity = 0;
  int64_t t = 0;
  if (multi) {
    if (wave == 0) {
      parity = readlane32(lane == 0 ? ld_agent32(&ka.hdr->parity) : 0u, 0);
      t = acquire_tile(ka, parity, lane);
      if (lane == 0) {
        s_parity = parity;
        s_tile = t;
      }
    }
    __syncthreads();
    parity = s_parity;
    t = s_tile;
  }
  u32x4 R[SH::CH];
  if (t < ka.tiles) {
    const WaveSpan<SH, true, false, VEC> in(ka.in, ka, t, wave, lane);
#pragma unroll
    for (int c = 0; c < SH::CH; ++c) in.load(c, R[c]);
  }
  while (t < ka.tiles) {
    // elements of this lane's group in chunk c exist while c*256 + k < rem
    const int64_t wb = wave_base<false, SH::TILE, SH::WSPAN>(t * (int64_t)SH::TILE, wave);
    const int64_t rem64 = ka.n - wb - 4 * lane;
    const int rem = rem64 > SH::WSPAN ? SH::WSPAN : (int)rem64;
    // first pass: the selection masks and the number kept by the lane; the
    // positions are recomputed per chunk when the chunk is written, so no
    // per-chunk offsets are held through the look-back
    uint32_t mask[MW];
    uint32_t lane_kept = 0u;
#pragma unroll
    for (int w = 0; w < MW; ++w) mask[w] = 0u;
#pragma unroll
    for (int c = 0; c < SH::CH; ++c) {
      uint32_t m = 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) m |= (c * 256 + k < rem && keep_element(R[c][k], a)) ? (1u << k) : 0u;
      mask[c / 8] |= m << (4 * (c % 8));
      lane_kept += (uint32_t)__builtin_popcount(m);
      // finish the chunk's bits now: left to itself the compiler keeps every
      // element's bit in a register of its own until the end of the pass
      asm volatile("" : "+v"(mask[c / 8]), "+v"(lane_kept));
    }
    const uint32_t wsum = readlane32(wave_scan<Op>(lane_kept), 63);
    uint32_t wpre, agg, wpref, aggf;
    combine_waves<Op, SH::WAVES>(wave, lane, wsum, 0u, s_wtot, s_wflag, wpre, wpref, agg, aggf);
    if (multi && wave == 0) {
      uint64_t *st = ka.status + parity * ka.capacity;
      publish_first<Op>(st, t, agg, 0u);
      uint32_t carry = 0u;
      if (t > 0) {
        uint64_t w[K];
        lb_window<Op, K>(st, (int32_t)t - 1, w);
        carry = look_back<Op, K, K>(st, t, ka.spin_limit, ka.err, w);
        if (lane == 0) st_agent(st + t, Op::pack(carry + agg, kPrefix));
      }
      if (lane == 0) s_carry = carry;
    }
    __syncthreads();
    // carry and base are wave-uniform; saying so keeps the output buffer
    // resources in scalar registers (a resource the compiler must treat as
    // per-lane turns every store into a loop over its distinct values)
    const uint32_t carry = (uint32_t)__builtin_amdgcn_readfirstlane((int)(t > 0 ? s_carry : 0u));
    if (t == ka.tiles - 1 && tid == 0) *a.count = (int64_t)(carry + agg);
    // kept elements go to out[carry + wpre + (kept in the wave's earlier
    // chunks) + (kept in earlier lanes of the chunk) + (kept before k in the group)]
    const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)(carry + wpre));
    // the kept elements' range out[base, n), clamped to [0, 2^31) bytes: a
    // start beyond n (only after a look-back that gave up) writes nothing
    const int64_t kbytes = (ka.n - (int64_t)base) * 4;
    const bool kok = kbytes > 0;
    uint32_t *stage = s_stage[wave];
    uint32_t cb = 0u;   // kept in the wave's chunks so far (uniform)
    // partition: the wave's rejected elements go to out[rlo, rlo + rej) in
    // reverse order, rlo = n - (rejected before the wave) - (rejected in it);
    // a range outside [0, n) (only after a look-back that gave up) writes nothing
    const int64_t wvalid64 = ka.n - wb;
    const uint32_t wvalid = wvalid64 <= 0 ? 0u : (wvalid64 >= SH::WSPAN ? (uint32_t)SH::WSPAN : (uint32_t)wvalid64);
    uint32_t rej = 0u, rc = 0u;   // rejected in the wave; in its chunks so far
    int64_t rlo = 0;
    bool rok_all = false;
    if constexpr (PART) {
      rej = wvalid - wsum;
      rlo = ka.n - (wb - (int64_t)base) - (int64_t)rej;
      rok_all = rlo >= 0 && rlo + (int64_t)rej <= ka.n;
    }
    // chunk c: scan the lanes' counts, pack the kept elements into the
    // wave's LDS row (wave-private: no barrier; R[c] is free afterwards),
    // write them as one contiguous run
    // Row of the wave's LDS staging area for chunk c: the kept elements in
    // order at [0, kept); with PART the rejected ones at [256, 256 + nrej)
    // in output order (the chunk's last rejected element first, since the
    // rejected elements fill the output from the end); every other element
    // (a rejected one without PART, or one past n) in the lane's spare words
    // at [512, 768).  So every element is written, without a branch.
    auto pack = [&](const int c) -> uint32_t {
      uint32_t m = (mask[c / 8] >> (4 * (c % 8))) & 0xfu;
      // chunk c is packed after chunk c-1 is counted (cb): the chunks' scans
      // are not all hoisted ahead of the stores, which would hold a scan
      // result per chunk in registers
      asm volatile("" : "+v"(m) : "s"(cb));
      const uint32_t x = wave_scan<Op>((uint32_t)__builtin_popcount(m));
      const uint32_t off = lane_up1(x);
      const uint32_t kc = readlane32(x, 63);
      const int64_t v64 = (int64_t)wvalid - 256 * c;
      const uint32_t valid = v64 <= 0 ? 0u : (v64 >= 256 ? 256u : (uint32_t)v64);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t before = (uint32_t)__builtin_popcount(m & ((1u << k) - 1u));
        const bool kept = (m >> k) & 1u;
        uint32_t pos = kept ? off + before : 512u + 4u * (uint32_t)lane + (uint32_t)k;
        if constexpr (PART) {
          // rank among the chunk's rejected elements: (4 lane + k) - (kept before it)
          const uint32_t q = 4u * (uint32_t)lane + (uint32_t)k - off - before;
          if (!kept && c * 256 + k < rem) pos = 256u + (valid - kc) - 1u - q;
        }
        stage[pos] = R[c][k];
      }
      return kc;
    };
    // one 128-bit store per lane: lane l writes row words 4l .. 4l+3 to the
    // run's words 4l .. 4l+3 through a resource that ends at the run's last
    // element (the hardware checks every dword, so a lane past the end
    // writes nothing and the lane at the end only its words inside)
    const u32x4 *srow = reinterpret_cast<const u32x4 *>(stage);
    auto flush = [&](const int c, const uint32_t kept) {
      const int64_t kend = (int64_t)cb + kept;
      const int64_t klim = kbytes < (int64_t)0x7fffffff ? kbytes : (int64_t)0x7fffffff;
      const int krec = kok ? (int)(4 * kend < klim ? 4 * kend : klim) : 0;
      const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
          static_cast<uint32_t *>(ka.out) + (kok ? base : 0u), (short)0, krec, 0x00020000);
      __builtin_amdgcn_raw_buffer_store_b128(srow[lane], rk, 4u * (cb + 4u * (uint32_t)lane), 0, SAUX);
      cb += kept;
      if constexpr (PART) {
        // this chunk's rejected run is out[rlo + rej - rc - nrej, rlo + rej - rc)
        const int64_t v64 = (int64_t)wvalid - 256 * c;
        const uint32_t valid = v64 <= 0 ? 0u : (v64 >= 256 ? 256u : (uint32_t)v64);
        const uint32_t nrej = valid - kept;
        const int64_t r0 = rlo + (int64_t)rej - (int64_t)rc - (int64_t)nrej;
        const bool rok = rok_all && nrej > 0u;
        const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
            static_cast<uint32_t *>(ka.out) + (rok ? r0 : 0), (short)0, rok ? (int)(4u * nrej) : 0, 0x00020000);
        __builtin_amdgcn_raw_buffer_store_b128(srow[64 + lane], rq, 16u * (uint32_t)lane, 0, SAUX);
        rc += nrej;
      }
    };
    // the first half goes out while the next tile is taken from the counter,
    // then each chunk's registers take the next tile's chunk once it is packed
    constexpr int KH = SH::CH / 2;
#pragma unroll
    for (int c = 0; c < KH; ++c) flush(c, pack(c));
    int64_t next = ka.tiles;
    if (multi) {
      if (wave == 0) {
        const int64_t tk = acquire_tile(ka, parity, lane);
        if (lane == 0) s_tile = tk;
      }
      __syncthreads();
      next = s_tile;
    }
    if (next < ka.tiles) {
      const WaveSpan<SH, true, false, VEC> in(ka.in, ka, next, wave, lane);
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) {
        const uint32_t kept = pack(c);
        in.load(c - KH, R[c - KH]);
        flush(c, kept);
      }
#pragma unroll
      for (int c = SH::CH - KH; c < SH::CH; ++c) in.load(c, R[c]);
    } else {
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) flush(c, pack(c));
    }
    t = next;
  }
}

}  // namespace mi355scan
