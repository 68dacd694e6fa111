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

// The predicate as one compare of the element's bits with the threshold's,
// fixed per kernel: kPkUnsigned (uint32 x > t; "not all bits zero" is x > 0),
// kPkSigned (int32), kPkFloat (float32; a NaN is never kept).  A predicate
// read from the arguments per element would branch on it for every element.
template <int PK>
__device__ __forceinline__ bool keep_kind(uint32_t x, uint32_t thr) {
  if constexpr (PK == kPkSigned) return (int32_t)x > (int32_t)thr;
  else if constexpr (PK == kPkFloat) return __builtin_bit_cast(float, x) > __builtin_bit_cast(float, thr);
  else return x > thr;
}

// A value the predicate never keeps: elements past n read as it.
template <int PK>
constexpr uint32_t never_kept() {
  return PK == kPkSigned ? 0x80000000u : (PK == kPkFloat ? 0x7FC00000u : 0u);   // INT32_MIN, NaN, 0
}

// One tile per iteration of a resident grid (tiles from the device counter,
// the workspace protocol of scan_tiles).  Two passes over the tile's values,
// which stay in registers until they are written:
//  - count: each lane counts its kept elements per chunk, three chunks to a
//    word (10 bits each: a chunk keeps at most 256), so one wave scan of a
//    word gives every lane its offset in three chunks and the chunks' totals;
//  - pack and write: per chunk, the wave packs its kept elements into its
//    own LDS row (every element is written somewhere, so no per-element
//    branch) and writes them as one contiguous run, one 128-bit store per
//    lane, instead of one scattered store per element.  A place in the row
//    does not depend on the carry, so the first group of chunks is packed
//    while wave 0's first look-back poll is in flight; the writes follow the
//    look-back.
// The predicate is evaluated once in each pass, one compare per element.
// Elements past n exist only in the wave that holds n; they are replaced
// there, once, by a value that is never kept, so no element needs a bound
// check.  As in scan_tiles, the registers a packed chunk frees take the next
// tile's chunk at once.  The output offsets are wave-uniform and kept in
// scalar registers: a buffer resource the compiler must treat as per-lane
// would turn every store into a loop over its distinct values.
// Counts of kept elements: 32-bit integer sums whose wave totals are folded
// from one lane each (no register per wave's total).
struct OpsCount : OpsU32 {
  static constexpr bool kCombineByLane = true;
};

template <int BLOCK, int ITEMS, bool VEC, int MINW, bool PART, int PK, int FL>
__global__ void __launch_bounds__(BLOCK, MINW) compact_tiles(CompactArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using Op = OpsCount;
  constexpr int K = 4;
  // store cache policy: non-temporal for compaction; the partition's two
  // output streams write faster through the default policy (measured)
  constexpr int SAUX = PART ? 0 : kNtAux;
  constexpr int NW = (SH::CH + 2) / 3;   // count words, three chunks each
  constexpr int KR = FL * 256;           // a group of FL chunks is written as one run
  static_assert((SH::CH / 2) % FL == 0, "groups tile each half of the wave span");
  __shared__ uint32_t s_wtot[SH::WAVES];
  __shared__ uint32_t s_wflag[SH::WAVES];
  __shared__ uint32_t s_carry;
  __shared__ int64_t s_tile;
  __shared__ uint32_t s_parity;
  __shared__ __attribute__((aligned(16))) uint32_t s_stage[SH::WAVES][KR + (PART ? KR : 256)];   // see pack
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
    const int64_t wb = wave_base<false, SH::TILE, SH::WSPAN>(t * (int64_t)SH::TILE, wave);
    const int64_t wvalid64 = ka.n - wb;
    const uint32_t wvalid = wvalid64 <= 0 ? 0u : (wvalid64 >= SH::WSPAN ? (uint32_t)SH::WSPAN : (uint32_t)wvalid64);
    if (PK != kPkUnsigned && wvalid < (uint32_t)SH::WSPAN) {
      // (an unsigned compare never keeps the zeros the loads return past n)
#pragma unroll
      for (int c = 0; c < SH::CH; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if ((uint32_t)(c * 256 + 4 * lane + k) >= wvalid) R[c][k] = never_kept<PK>();
    }
    // count pass: xe[w] holds, per chunk of the word, the kept elements of
    // the chunk in earlier lanes; tot[w] the chunk totals (uniform)
    uint32_t xe[NW], tot[NW];
    uint32_t wsum = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t cw = 0u;
#pragma unroll
      for (int c = 3 * w; c < 3 * w + 3 && c < SH::CH; ++c) {
        uint32_t kc = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) kc += keep_kind<PK>(R[c][k], a.thr) ? 1u : 0u;
        cw |= kc << (10 * (c - 3 * w));
      }
      const uint32_t x = wave_scan<Op>(cw);
      xe[w] = x - cw;
      tot[w] = readlane32(x, 63);
      wsum += (tot[w] & 1023u) + ((tot[w] >> 10) & 1023u) + (tot[w] >> 20);
    }
    uint32_t wpre, agg, wpref, aggf;
    combine_waves<Op, SH::WAVES>(wave, lane, wsum, 0u, s_wtot, s_wflag, wpre, wpref, agg, aggf);
    uint32_t *stage = s_stage[wave];
    // The chunks go in groups of FL, each group written as one run.  Row of
    // the wave's LDS staging area for a group: its kept elements in order at
    // [0, kept).  With PART, a rejected element at group index e goes to
    // KR - 1 + (valid - kept) - e + (kept before it), valid and kept being
    // the group's: the valid ones fill [KR, KR + valid - kept) in output
    // order (the group's last rejected element first, since the rejected
    // elements fill the output from the end); for one past n, (kept before
    // it) is the group's whole count, so it lands in [valid, KR), which no
    // kept element uses.  Without PART a rejected element goes to the lane's
    // spare word KR + 64k + lane.  So every element is written, without a
    // branch.
    auto field = [&](const uint32_t (&w)[NW], const int c) -> uint32_t {
      return (w[c / 3] >> (10u * (uint32_t)(c % 3))) & 1023u;
    };
    // pack chunk c of a group: cg kept in the group's earlier chunks
    // (uniform), rb = KR - 1 + (valid - kept) - 256 (c - first chunk)
    auto pack = [&](const int c, const uint32_t cg, const uint32_t rb) {
      uint32_t p = cg + field(xe, c);   // this lane's first kept position
      // chunk c is packed after the previous one is counted (cg): the
      // chunks' positions are not all hoisted ahead of the stores; and the
      // values are compared again here rather than the count pass's results
      // (a lane mask per element) being kept through the look-back
      asm volatile("" : "+v"(p), "+v"(R[c]) : "s"(cg));
      const uint32_t rbase = rb - 4u * (uint32_t)lane;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool kept = keep_kind<PK>(R[c][k], a.thr);
        const uint32_t other = PART ? rbase - (uint32_t)k + p : (uint32_t)KR + 64u * (uint32_t)k + (uint32_t)lane;
        stage[kept ? p : other] = R[c][k];
        p += kept ? 1u : 0u;
      }
    };
    // a group's kept elements and its elements that exist (uniform)
    auto group_kept = [&](const int g0) -> uint32_t {
      uint32_t kg = 0u;
#pragma unroll
      for (int j = 0; j < FL; ++j) kg += field(tot, g0 + j);
      return kg;
    };
    auto group_valid = [&](const int g0) -> uint32_t {
      const int64_t v64 = (int64_t)wvalid - 256 * g0;
      return v64 <= 0 ? 0u : (v64 >= KR ? (uint32_t)KR : (uint32_t)v64);
    };
    // group g0 .. g0+FL-1 into the wave's row; given the next tile's span
    // (not nullptr), each chunk's registers take the next tile's chunk
    // c - KH once it is packed
    constexpr int KH = SH::CH / 2;
    using Span = WaveSpan<SH, true, false, VEC>;
    auto pack_group = [&](const int g0, const auto in) {
      const uint32_t kg = group_kept(g0), valid = group_valid(g0);
      uint32_t cg = 0u;
#pragma unroll
      for (int j = 0; j < FL; ++j) {
        pack(g0 + j, cg, (uint32_t)(KR - 1) + (valid - kg) - 256u * (uint32_t)j);
        cg += field(tot, g0 + j);
        if constexpr (std::is_pointer_v<decltype(in)>) in->load(g0 + j - KH, R[g0 + j - KH]);
      }
    };
    // publish and issue the first poll; pack the first group (LDS only, its
    // places do not depend on the carry) while the poll is in flight; then
    // look back
    uint64_t w1[1];
    if (multi && wave == 0) {
      uint64_t *st = ka.status + parity * ka.capacity;
      publish_first<Op>(st, t, agg, 0u);
      if (t > 0) lb_window<Op, 1>(st, (int32_t)t - 1, w1);
    }
    pack_group(0, nullptr);
    if (multi && wave == 0) {
      uint64_t *st = ka.status + parity * ka.capacity;
      uint32_t carry = 0u;
      if (t > 0) {
        carry = look_back<Op, 1, K>(st, t, ka.spin_limit, ka.err, w1);
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
    uint32_t cb = 0u;   // kept in the wave's chunks so far (uniform)
    // partition: the wave's rejected elements go to out[rlo, rlo + rej) in
    // reverse order, rlo = n - (rejected before the wave) - (rejected in it);
    // a range outside [0, n) (only after a look-back that gave up) writes nothing
    uint32_t rej = 0u, rc = 0u;   // rejected in the wave; in its chunks so far
    int64_t rlo = 0;
    bool rok_all = false;
    if constexpr (PART) {
      rej = wvalid - wsum;
      rlo = ka.n - (wb - (int64_t)base) - (int64_t)rej;
      rok_all = rlo >= 0 && rlo + (int64_t)rej <= ka.n;
    }
    // FL 128-bit stores per lane and run: lane l writes row words 4l .. 4l+3
    // (+256 i) to the run's words 4l .. 4l+3 (+256 i) through a resource that
    // ends at the run's last element (the hardware checks every dword, so a
    // lane past the end writes nothing and the lane at the end only its
    // words inside)
    const u32x4 *srow = reinterpret_cast<const u32x4 *>(stage);
    auto flush = [&](const uint32_t kept, const uint32_t valid) {
      const int64_t kend = (int64_t)cb + kept;
      const int64_t klim = kbytes < (int64_t)0x7fffffff ? kbytes : (int64_t)0x7fffffff;
      const int krec = kok ? (int)(4 * kend < klim ? 4 * kend : klim) : 0;
      const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
          static_cast<uint32_t *>(ka.out) + (kok ? base : 0u), (short)0, krec, 0x00020000);
#pragma unroll
      for (int i = 0; i < FL; ++i)
        __builtin_amdgcn_raw_buffer_store_b128(srow[64 * i + lane], rk, 4u * (cb + 256u * i + 4u * (uint32_t)lane),
                                               0, SAUX);
      cb += kept;
      if constexpr (PART) {
        // this group's rejected run is out[rlo + rej - rc - nrej, rlo + rej - rc)
        const uint32_t nrej = valid - kept;
        const int64_t r0 = rlo + (int64_t)rej - (int64_t)rc - (int64_t)nrej;
        const bool rok = rok_all && nrej > 0u;
        const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
            static_cast<uint32_t *>(ka.out) + (rok ? r0 : 0), (short)0, rok ? (int)(4u * nrej) : 0, 0x00020000);
#pragma unroll
        for (int i = 0; i < FL; ++i)
          __builtin_amdgcn_raw_buffer_store_b128(srow[KR / 4 + 64 * i + lane], rq, 1024u * i + 16u * (uint32_t)lane,
                                                 0, SAUX);
        rc += nrej;
      }
    };
    auto group = [&](const int g0, const auto in) {
      pack_group(g0, in);
      flush(group_kept(g0), group_valid(g0));
    };
    // the first group, packed before the carry was known, goes out first;
    // the rest of the first half while the next tile is taken from the
    // counter, then the second half's registers take the next tile's chunks
    flush(group_kept(0), group_valid(0));
#pragma unroll
    for (int g0 = FL; g0 < KH; g0 += FL) group(g0, nullptr);
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
      const Span in(ka.in, ka, next, wave, lane);
#pragma unroll
      for (int g0 = KH; g0 < SH::CH; g0 += FL) group(g0, &in);
#pragma unroll
      for (int c = SH::CH - KH; c < SH::CH; ++c) in.load(c, R[c]);
    } else {
#pragma unroll
      for (int g0 = KH; g0 < SH::CH; g0 += FL) group(g0, nullptr);
    }
    t = next;
  }
}

}  // namespace mi355scan
