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
// kept elements into its own LDS row and writes them out as one contiguous
// run (dword stores of consecutive lanes) instead of one scattered store per
// element; as in scan_tiles, the registers a packed chunk frees take the next
// tile's chunk at once.
template <int BLOCK, int ITEMS, bool VEC, int MINW, bool PART = false>
__global__ void __launch_bounds__(BLOCK, MINW) compact_tiles(CompactArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using Op = OpsU32;
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
  __shared__ uint32_t s_stage[SH::WAVES][256];
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
    const uint32_t carry = t > 0 ? s_carry : 0u;
    if (t == ka.tiles - 1 && tid == 0) *a.count = (int64_t)(carry + agg);
    // kept elements go to out[carry + wpre + (kept in the wave's earlier
    // chunks) + (kept in earlier lanes of the chunk) + (kept before k in the group)]
    const uint32_t base = carry + wpre;
    // the kept elements' range out[base, n), clamped to [0, 2^31) bytes: a
    // start beyond n (only after a look-back that gave up) writes nothing
    const int64_t kbytes = (ka.n - (int64_t)base) * 4;
    const bool kok = kbytes > 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        static_cast<uint32_t *>(ka.out) + (kok ? base : 0u), (short)0,
        kok ? (int)(kbytes > 0x7fffffff ? 0x7fffffff : kbytes) : 0, 0x00020000);
    uint32_t *stage = s_stage[wave];
    uint32_t cb = 0u;   // kept in the wave's chunks so far (uniform)
    // partition: the wave's rejected elements go to out[rlo, rlo + rej) in
    // reverse order, rlo = n - (rejected before the wave) - (rejected in it);
    // a range outside [0, n) (only after a look-back that gave up) writes nothing
    const int64_t wvalid64 = ka.n - wb;
    const uint32_t wvalid = wvalid64 <= 0 ? 0u : (wvalid64 >= SH::WSPAN ? (uint32_t)SH::WSPAN : (uint32_t)wvalid64);
    __amdgpu_buffer_rsrc_t rr = rs;
    uint32_t rej = 0u, rc = 0u;   // rejected in the wave; in its chunks so far
    if constexpr (PART) {
      rej = wvalid - wsum;
      const int64_t rlo = ka.n - (wb - (int64_t)base) - (int64_t)rej;
      const bool ok = rlo >= 0 && rlo + (int64_t)rej <= ka.n;
      rr = __builtin_amdgcn_make_buffer_rsrc(static_cast<uint32_t *>(ka.out) + (ok ? rlo : 0), (short)0,
                                             ok ? (int)(4u * rej) : 0, 0x00020000);
    }
    // chunk c: scan the lanes' counts, pack the kept elements into the
    // wave's LDS row (wave-private: no barrier; R[c] is free afterwards),
    // write them as one contiguous run
    auto pack = [&](const int c) -> uint32_t {
      const uint32_t m = (mask[c / 8] >> (4 * (c % 8))) & 0xfu;
      const uint32_t x = wave_scan<Op>((uint32_t)__builtin_popcount(m));
      const uint32_t off = lane_up1(x);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((m >> k) & 1u) stage[off + (uint32_t)__builtin_popcount(m & ((1u << k) - 1u))] = R[c][k];
      const uint32_t kc = readlane32(x, 63);
      if constexpr (PART) {
        // rejected elements after the kept ones in the row: a valid element
        // that is not kept has (4 lane + k) - (kept before it) rejected
        // elements before it in the chunk
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (c * 256 + k < rem && !((m >> k) & 1u))
            stage[kc + 4u * (uint32_t)lane + (uint32_t)k - off - (uint32_t)__builtin_popcount(m & ((1u << k) - 1u))] =
                R[c][k];
      }
      return kc;
    };
    auto flush = [&](const int c, const uint32_t kept) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t idx = 64u * j + lane;
        if (idx < kept) __builtin_amdgcn_raw_buffer_store_b32(stage[idx], rs, 4u * (cb + idx), 0, SAUX);
      }
      cb += kept;
      if constexpr (PART) {
        // row entries [kept, valid) are the chunk's rejected elements in
        // order; the i-th of the wave goes to out[rlo + rej - 1 - i]
        const int64_t v64 = (int64_t)wvalid - 256 * c;
        const uint32_t valid = v64 <= 0 ? 0u : (v64 >= 256 ? 256u : (uint32_t)v64);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t idx = 64u * j + lane;
          if (idx >= kept && idx < valid)
            __builtin_amdgcn_raw_buffer_store_b32(stage[idx], rr, 4u * (rej - 1u - (rc + idx - kept)), 0, SAUX);
        }
        rc += valid - kept;
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
