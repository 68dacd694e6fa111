// Single-pass scans of 64-bit elements: integers (wrapping modulo 2^64;
// int64 and uint64 are the same bits) and float64 sums.  The same decoupled
// look-back as the 32-bit kernel, with a tile's status held in two 64-bit
// words.  Each word carries the 2-bit flag and one 32-bit half of the value
// and is moved by a single relaxed atomic access; a reader takes the pair
// only when both halves carry the same flag (flags only move forward, EMPTY
// -> AGG -> PREFIX, so a pair with different flags is a publication in
// progress and reads as EMPTY), so no fences are needed.  A lane holds two
// elements per 16-byte load; a chunk is 128 elements.  Flat scans, inclusive
// or exclusive, forward or reverse: a reverse scan walks the same physical
// tiles, wave spans, chunks, lanes and element pairs from the top down, so
// every step above works on the logical (reversed) order unchanged.
#pragma once
#include "scan_device.hpp"

namespace mi355scan {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const uint32_t lo = dpp<CTRL, ROW_MASK>((uint32_t)x);
  const uint32_t hi = dpp<CTRL, ROW_MASK>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive wave scan of 64-bit integers: the 32-bit wave_scan's six steps
// (row_shr 1, 2, 4, 8, row_bcast 15, 31), each x += (x of the lane the DPP
// control names) done as a low-half add with carry out and a high-half add
// with carry in that take their DPP operand directly.  Lanes without a source
// lane, or in rows the row mask leaves out, are not written and keep x
// (= x + 0); both adds of a step use the same control, so the carry is only
// read in lanes that wrote it.  A DPP read needs two wait states after a VALU
// write of its source register: the s_nops supply them inside the block and
// on both sides of it (the compiler does not see the DPP reads here).
#define MI355SCAN_DPP_ADD64(CTRL, TAIL)                        \
  "v_add_co_u32_dpp %0, vcc, %0, %0 " CTRL "\n\t"             \
  "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " CTRL "\n\t" TAIL
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  asm("s_nop 1\n\t"
      MI355SCAN_DPP_ADD64("row_shr:1 row_mask:0xf bank_mask:0xf", "s_nop 0\n\t")
      MI355SCAN_DPP_ADD64("row_shr:2 row_mask:0xf bank_mask:0xf", "s_nop 0\n\t")
      MI355SCAN_DPP_ADD64("row_shr:4 row_mask:0xf bank_mask:0xf", "s_nop 0\n\t")
      MI355SCAN_DPP_ADD64("row_shr:8 row_mask:0xf bank_mask:0xf", "s_nop 0\n\t")
      MI355SCAN_DPP_ADD64("row_bcast:15 row_mask:0xa bank_mask:0xf", "s_nop 0\n\t")
      MI355SCAN_DPP_ADD64("row_bcast:31 row_mask:0xc bank_mask:0xf", "s_nop 1")
      : "+v"(lo), "+v"(hi)
      :
      : "vcc");
  return ((uint64_t)hi << 32) | lo;
}
#undef MI355SCAN_DPP_ADD64

__device__ __forceinline__ double f64_of(uint64_t b) { return __builtin_bit_cast(double, b); }
__device__ __forceinline__ uint64_t bits_of(double x) { return __builtin_bit_cast(uint64_t, x); }

// The two element operations, on the 64-bit patterns: add and the inclusive
// scan over the 64 lanes (identity: the all-zero pattern, 0 and +0.0).
struct OpsAddU64 {
  static __device__ __forceinline__ uint64_t add(uint64_t a, uint64_t b) { return a + b; }
  static __device__ __forceinline__ uint64_t wave_scan(uint64_t x) { return wave_scan_u64(x); }
};
struct OpsAddF64 {
  static __device__ __forceinline__ uint64_t add(uint64_t a, uint64_t b) { return bits_of(f64_of(a) + f64_of(b)); }
  template <int CTRL, int ROW_MASK>
  static __device__ __forceinline__ uint64_t step(uint64_t x) { return add(dpp64<CTRL, ROW_MASK>(x), x); }
  // the 32-bit wave_scan's steps; lanes without a source add +0.0
  static __device__ __forceinline__ uint64_t wave_scan(uint64_t x) {
    x = step<0x111, 0xf>(x);
    x = step<0x112, 0xf>(x);
    x = step<0x114, 0xf>(x);
    x = step<0x118, 0xf>(x);
    x = step<0x142, 0xa>(x);
    x = step<0x143, 0xc>(x);
    return x;
  }
};

__device__ __forceinline__ uint64_t lane_up1_64(uint64_t x) { return dpp64<0x138, 0xf>(x); }

// Status pair of tile t: words 2t (low half) and 2t+1 (high half).
__device__ __forceinline__ void publish64(uint64_t *st, int64_t t, uint64_t v, uint32_t flag) {
  st_agent(st + 2 * t, ((uint64_t)flag << 32) | (uint32_t)v);
  st_agent(st + 2 * t + 1, ((uint64_t)flag << 32) | (uint32_t)(v >> 32));
}

// Take the next tile (one wave, uniform result): as acquire_tile, with two
// status words per tile to clear in the other array and 2*tiles words used.
__device__ __forceinline__ void hand_over64(const KernelArgs &a, uint32_t p, uint64_t clear_hi, int nthreads) {
  uint64_t *other = a.status + (1 - p) * a.capacity;
  const uint32_t me = opaque_tid() % (uint32_t)nthreads;
  for (uint64_t i = 2 * (uint64_t)a.tiles + me; i < clear_hi; i += nthreads) st_agent(other + i, 0ull);
  if (me == 0) {
    st_agent(&a.hdr->counter[1 - p], 0ull);
    st_agent(&a.hdr->dirty[1 - p], 0ull);
    st_agent(&a.hdr->dirty[p], 2 * (uint64_t)a.tiles);
    st_agent32(&a.hdr->parity, 1u - p);
  }
}

__device__ __forceinline__ int64_t acquire_tile64(const KernelArgs &a, uint32_t parity, int lane) {
  uint64_t tk = 0, clear_hi = 0;
  uint32_t last = 0;
  if (lane == 0) {
    tk = __hip_atomic_fetch_add(&a.hdr->counter[parity], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = tk == a.total_acquires - 1;
    if (tk < (uint64_t)a.tiles) {
      st_agent(a.status + (1 - parity) * a.capacity + 2 * tk, 0ull);
      st_agent(a.status + (1 - parity) * a.capacity + 2 * tk + 1, 0ull);
    }
    if (last) clear_hi = ld_agent(&a.hdr->dirty[1 - parity]);
  }
  tk = readlane64(tk, 0);
  if (readlane32(last, 0)) hand_over64(a, parity, readlane64(clear_hi, 0), 64);
  return (int64_t)tk;
}

// The status pair of window lane `lane` (tile base - lane), or an empty
// PREFIX before tile 0.
__device__ __forceinline__ void lb_pair64(const uint64_t *st, int64_t base, int lane, uint64_t &lo, uint64_t &hi) {
  const int64_t idx = base - lane;
  lo = ((uint64_t)kPrefix << 32);
  hi = ((uint64_t)kPrefix << 32);
  if (idx >= 0) {
    lo = ld_agent(st + 2 * idx);
    hi = ld_agent(st + 2 * idx + 1);
  }
}

// Carry into tile t (one wave): sum of the aggregates back to the nearest
// PREFIX, read 64 tiles per poll (lane l: tile t-1-l of the window).  With
// PRE the first poll's pair (lo0, hi0) was loaded by the caller, so its round
// trip overlaps the caller's work.
template <class Op, bool PRE = false>
__device__ uint64_t look_back64(const uint64_t *st, int64_t t, uint32_t spin_limit, uint32_t *err,
                                uint64_t lo0 = 0, uint64_t hi0 = 0) {
  const int lane = (int)(opaque_tid() & 63u);
  uint64_t acc = 0;
  int64_t base = t - 1;
  bool pre = PRE;
  for (uint32_t spins = 0;;) {
    uint64_t lo, hi;
    if (pre) {
      lo = lo0;
      hi = hi0;
      pre = false;
    } else {
      lb_pair64(st, base, lane, lo, hi);
    }
    const uint32_t flo = (uint32_t)(lo >> 32), fhi = (uint32_t)(hi >> 32);
    const uint32_t f = flo == fhi ? flo : kEmpty;
    const uint64_t v = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    const uint64_t bP = ballot(f == kPrefix), bE = ballot(f == kEmpty);
    const int dP = bP ? __builtin_ctzll(bP) : 64, dE = bE ? __builtin_ctzll(bE) : 64;
    if (dE < dP) {
      if (++spins > spin_limit) {
        if (lane == 0) raise_error(err);
        return acc;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    // lanes 0..min(dP, 63) hold aggregates (and the PREFIX at dP)
    const uint64_t part = readlane64(Op::wave_scan(lane <= dP ? v : 0ull), 63);
    acc = Op::add(acc, part);
    if (dP < 64) return acc;
    base -= 64;
  }
}

// One wave's span in an 8-byte-element buffer, starting at element wb: 16-byte
// loads and stores, lane l of chunk c at byte 1024c + 16l (REV: lane 63-l of
// chunk CH-1-c); the buffer resource's record count returns 0 beyond n and
// drops stores there.
template <int WSPAN, bool REV>
struct WaveSpan64 {
  static constexpr int CH = WSPAN / 128;
  __amdgpu_buffer_rsrc_t rs;
  uint32_t lo;
  __device__ __forceinline__ WaveSpan64(const void *buf, int64_t n, int64_t wb) {
    const int64_t valid = (n - wb) * 8;
    const int nr = valid <= 0 ? 0 : (valid >= 8 * WSPAN ? 8 * WSPAN : (int)valid);
    rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint64_t *>(static_cast<const uint64_t *>(buf)) + wb,
                                           (short)0, nr, 0x00020000);
    const uint32_t l = opaque_tid() & 63u;
    lo = 16u * (REV ? 63u - l : l);
  }
  static __device__ __forceinline__ uint32_t chunk(int c) { return 1024u * (uint32_t)(REV ? CH - 1 - c : c); }
  __device__ __forceinline__ void load(int c, u32x4 &r) const {
    r = __builtin_amdgcn_raw_buffer_load_b128(rs, lo + chunk(c), 0, kNtAux);
  }
  __device__ __forceinline__ void store(int c, const u32x4 &r) const {
    __builtin_amdgcn_raw_buffer_store_b128(r, rs, lo + chunk(c), 0, kNtAux);
  }
};

__device__ __forceinline__ uint64_t u64_of(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// A wave-uniform 64-bit value in scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return u64_of((uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x),
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)));
}

// Resident grid, tiles from the device counter; ITEMS elements per thread
// (2 per chunk and lane), the wave's span WSPAN = 64 * ITEMS elements.
// EARLY: the tile's aggregate is summed from the lanes' element pairs and
// published before the in-register scan, and wave 0 issues the first
// look-back poll then, so that its round trip overlaps the scan.
template <class Op, int BLOCK, int ITEMS, int MINW, bool REV, bool EARLY = false>
__global__ void __launch_bounds__(BLOCK, MINW) scan64_tiles(KernelArgs a) {
  static_assert(ITEMS % 2 == 0, "two elements per 16-byte group");
  constexpr int WAVES = BLOCK / 64;
  constexpr int CH = ITEMS / 2;
  constexpr int WSPAN = 64 * ITEMS;
  constexpr int64_t TILE = (int64_t)BLOCK * ITEMS;
  using Span = WaveSpan64<WSPAN, REV>;
  // element k (0 = first in logical order) of a lane's 16-byte pair: dwords
  // 2k, 2k+1 forward, 2(1-k), 2(1-k)+1 reverse
  constexpr int E0 = REV ? 2 : 0, E1 = REV ? 0 : 2;
  __shared__ uint64_t s_wtot[WAVES];
  __shared__ uint64_t s_carry;
  __shared__ int64_t s_tile;
  __shared__ uint32_t s_parity;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  // first element of logical tile t's span for this wave (REV: physical tile
  // tiles-1-t, wave spans from the top)
  const auto span_base = [&](int64_t t) -> int64_t {
    const int64_t pt = REV ? a.tiles - 1 - t : t;
    return pt * TILE + (int64_t)(REV ? WAVES - 1 - wave : wave) * WSPAN;
  };
  const bool multi = a.tiles > 1;
  const bool ex = a.exclusive != 0u;
  uint32_t parity = 0;
  int64_t t = 0;
  if (multi) {
    if (wave == 0) {
      parity = readlane32(lane == 0 ? ld_agent32(&a.hdr->parity) : 0u, 0);
      t = acquire_tile64(a, parity, lane);
      if (lane == 0) {
        s_parity = parity;
        s_tile = t;
      }
    }
    __syncthreads();
    parity = s_parity;
    t = (int64_t)uniform64((uint64_t)s_tile);
  }
  u32x4 R[CH];
  if (t < a.tiles) {
    const Span in(a.in, a.n, span_base(t));
#pragma unroll
    for (int c = 0; c < CH; ++c) in.load(c, R[c]);
  }
  while (t < a.tiles) {
    uint64_t wpre = 0, agg = 0;
    uint64_t wlo = 0, whi = 0;   // EARLY: wave 0's first look-back poll
    if constexpr (EARLY) {
      // lane totals of the loaded pairs, the wave totals, the tile aggregate
      uint64_t lt = 0;
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const uint64_t p = Op::add(u64_of(R[c][E0], R[c][E0 + 1]), u64_of(R[c][E1], R[c][E1 + 1]));
        lt = c > 0 ? Op::add(lt, p) : p;
      }
      const uint64_t wt = readlane64(Op::wave_scan(lt), 63);
      if (lane == 0) s_wtot[wave] = wt;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        if (w == wave) wpre = agg;
        agg = w > 0 ? Op::add(agg, s_wtot[w]) : s_wtot[w];
      }
      // the wave's prefix and the aggregate now, in scalar registers (not
      // the fold's partial sums kept until the carry is added)
      wpre = uniform64(wpre);
      agg = uniform64(agg);
      if (multi && wave == 0) {
        uint64_t *st = a.status + parity * a.capacity;
        if (lane == 0) publish64(st, t, agg, t == 0 ? kPrefix : kAgg);
        if (t > 0) lb_pair64(st, t - 1, lane, wlo, whi);
      }
    }
    // in-register scan: per chunk the lane's two elements, then the lanes
    uint64_t wsum = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      // the pair sums are computed again, not kept from the aggregate's loop
      if constexpr (EARLY) asm volatile("" : "+v"(R[c]));
      const uint64_t x0 = u64_of(R[c][E0], R[c][E0 + 1]);
      const uint64_t x1 = Op::add(u64_of(R[c][E1], R[c][E1 + 1]), x0);
      const uint64_t x = Op::wave_scan(x1);
      const uint64_t up = lane_up1_64(x);
      const uint64_t off = c > 0 ? Op::add(up, wsum) : up;
      const uint64_t o0 = ex ? off : Op::add(off, x0);
      const uint64_t o1 = ex ? Op::add(off, x0) : Op::add(off, x1);
      R[c][E0] = (uint32_t)o0;
      R[c][E0 + 1] = (uint32_t)(o0 >> 32);
      R[c][E1] = (uint32_t)o1;
      R[c][E1 + 1] = (uint32_t)(o1 >> 32);
      wsum = c > 0 ? Op::add(wsum, readlane64(x, 63)) : readlane64(x, 63);
      asm volatile("" : "+v"(R[c]));
    }
    if constexpr (EARLY) {
      if (multi && wave == 0) {
        uint64_t *st = a.status + parity * a.capacity;
        uint64_t carry = 0;
        if (t > 0) {
          carry = look_back64<Op, true>(st, t, a.spin_limit, a.err, wlo, whi);
          if (lane == 0) publish64(st, t, Op::add(carry, agg), kPrefix);
        }
        if (lane == 0) s_carry = carry;
      }
    } else {
      // wave totals: this wave's prefix and the tile's aggregate, left to right
      if (lane == 0) s_wtot[wave] = wsum;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        if (w == wave) wpre = agg;
        agg = w > 0 ? Op::add(agg, s_wtot[w]) : s_wtot[w];
      }
    }
    if (!EARLY && multi && wave == 0) {
      uint64_t *st = a.status + parity * a.capacity;
      uint64_t carry = 0;
      if (t == 0) {
        if (lane == 0) publish64(st, t, agg, kPrefix);
      } else {
        if (lane == 0) publish64(st, t, agg, kAgg);
        carry = look_back64<Op>(st, t, a.spin_limit, a.err);
        if (lane == 0) publish64(st, t, Op::add(carry, agg), kPrefix);
      }
      if (lane == 0) s_carry = carry;
    }
    __syncthreads();
    const uint64_t win = t > 0 ? Op::add(s_carry, wpre) : wpre;
    const Span out(a.out, a.n, span_base(t));
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const uint64_t o0 = Op::add(u64_of(R[c][0], R[c][1]), win), o1 = Op::add(u64_of(R[c][2], R[c][3]), win);
      R[c][0] = (uint32_t)o0;
      R[c][1] = (uint32_t)(o0 >> 32);
      R[c][2] = (uint32_t)o1;
      R[c][3] = (uint32_t)(o1 >> 32);
    }
    // store, taking the next tile after the first half, and load it into the
    // registers each further store frees (as scan_tiles does)
    constexpr int KH = CH / 2;
#pragma unroll
    for (int c = 0; c < KH; ++c) out.store(c, R[c]);
    int64_t next = a.tiles;
    if (multi) {
      if (wave == 0) {
        const int64_t tk = acquire_tile64(a, parity, lane);
        if (lane == 0) s_tile = tk;
      }
      __syncthreads();
      next = (int64_t)uniform64((uint64_t)s_tile);
    }
    if (next < a.tiles) {
      const Span in(a.in, a.n, span_base(next));
#pragma unroll
      for (int c = KH; c < CH; ++c) {
        out.store(c, R[c]);
        in.load(c - KH, R[c - KH]);
      }
#pragma unroll
      for (int c = CH - KH; c < CH; ++c) in.load(c, R[c]);
    } else {
#pragma unroll
      for (int c = KH; c < CH; ++c) out.store(c, R[c]);
    }
    t = next;
  }
}

}  // namespace mi355scan
