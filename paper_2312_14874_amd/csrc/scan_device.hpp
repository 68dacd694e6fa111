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

#include "scan_shared.hpp"

namespace mi355scan {

// --------------------------------------------------------------- element ops
// Integers: everything in uint32_t, wrapping modulo 2^32 (int32 uses the same
// bits).
struct OpsU32 {
  using lane_t = uint32_t;    // per-lane arithmetic (up to 256-element chunks)
  using carry_t = uint32_t;   // chunk, wave, tile and inter-tile arithmetic
  static constexpr bool kExact = true;
  __device__ static lane_t lzero() { return 0u; }
  __device__ static carry_t czero() { return 0u; }
  __device__ static lane_t ladd(lane_t a, lane_t b) { return a + b; }
  __device__ static carry_t cadd(carry_t a, carry_t b) { return a + b; }
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

// ------------------------------------------------------------ memory helpers
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u32x4 load4(const uint32_t *p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  else return *reinterpret_cast<const u32x4 *>(p);
}
template <bool NT>
__device__ __forceinline__ void store4(uint32_t *p, u32x4 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
  else *reinterpret_cast<u32x4 *>(p) = v;
}

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

// ------------------------------------------------------------------ look-back
// Run by one whole wave.  Lane l, slot k inspects predecessor t-1-(64k+l)
// (distance d = 64k+l).  dP = nearest PREFIX, dE = nearest EMPTY.  The window
// is usable when every word nearer than the PREFIX is an AGG; then the carry is
// the PREFIX value folded left with the AGG values of distances dP-1 .. 0.
// Integers may also consume a window of AGGs and continue further back
// (addition is exact); float64 carries wait until the PREFIX is in the window
// so that the fold order is always the canonical left-to-right chain.
// Returns the exclusive carry into tile t (t >= 1).
template <class Op, int K>
__device__ typename Op::carry_t look_back(const uint64_t *st, int64_t t, uint32_t spin_limit,
                                          WsHeader *hdr) {
  using carry_t = typename Op::carry_t;
  const int lane = threadIdx.x & 63;
  carry_t acc = Op::czero();
  int64_t base = t - 1;
  uint32_t spins = 0;
  constexpr int kNone = 1 << 30;
  for (;;) {
    uint64_t w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t idx = base - (int64_t)(64 * k + lane);
      w[k] = idx >= 0 ? ld_agent(st + idx) : Op::pack(Op::czero(), kPrefix);
    }
    int dP = kNone, dE = kNone;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t f = Op::flag_of(w[k]);
      const uint64_t bP = ballot(f == kPrefix);
      const uint64_t bE = ballot(f == kEmpty);
      if (dP == kNone && bP) dP = 64 * k + __builtin_ctzll(bP);
      if (dE == kNone && bE) dE = 64 * k + __builtin_ctzll(bE);
    }
    bool wait = dE < dP;
    if (!wait && dP == kNone) {
      if constexpr (Op::kExact) {
        // a full window of aggregates: add them all and move further back
        carry_t part = Op::czero();
#pragma unroll
        for (int k = 0; k < K; ++k) part = Op::cadd(part, Op::value_of(w[k]));
        part = Op::narrow(readlane32(Op::lbits(wave_scan<Op>(part)), 63));
        acc = Op::cadd(acc, part);
        base -= 64 * K;
        continue;
      } else {
        wait = true;
      }
    }
    if (wait) {
      if (++spins > spin_limit) {
        if (lane == 0) st_agent32(&hdr->error, 1u);
        return acc;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    if constexpr (Op::kExact) {
      carry_t part = Op::czero();
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (64 * k + lane <= dP) part = Op::cadd(part, Op::value_of(w[k]));
      part = Op::narrow(readlane32(Op::lbits(wave_scan<Op>(part)), 63));
      return Op::cadd(acc, part);
    } else {
      auto slot = [&](int d) -> uint64_t {
        const int k = d >> 6;
        uint64_t sel = w[0];
#pragma unroll
        for (int kk = 1; kk < K; ++kk) sel = (k == kk) ? w[kk] : sel;
        return readlane64(sel, d & 63);
      };
      carry_t c = Op::value_of(slot(dP));
      for (int d = dP - 1; d >= 0; --d) c = Op::canon(Op::cadd(c, Op::value_of(slot(d))));
      return c;
    }
  }
}

// Physical index of the lowest element of the 4-element group that lane
// `lane` of wave `wave` holds in chunk c.  Logical element e of a tile is
// physical pb+e going forward and pb+TILE-1-e in reverse, so a reverse tile is
// the same aligned block read back to front.
template <int TILE, int WSPAN>
__device__ __forceinline__ int64_t quad_base(uint32_t reverse, int64_t pb, int wave, int c, int lane) {
  const int e0 = wave * WSPAN + c * 256 + lane * 4;
  return reverse ? (pb + TILE - 4 - e0) : (pb + e0);
}

// ------------------------------------------------------------------- kernel
template <class Op, int BLOCK, int ITEMS, bool SEG, bool NT>
__global__ void __launch_bounds__(BLOCK) scan_tiles(KernelArgs a) {
  static_assert(BLOCK % 64 == 0 && ITEMS % 4 == 0, "shape");
  constexpr int WAVES = BLOCK / 64;
  constexpr int CH = ITEMS / 4;            // 256-element chunks per wave
  constexpr int WSPAN = 64 * ITEMS;        // contiguous elements per wave
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int K = 2;                     // look-back window = 64*K tiles
  using lane_t = typename Op::lane_t;
  using carry_t = typename Op::carry_t;

  __shared__ carry_t s_wtot[WAVES];
  __shared__ uint32_t s_wflag[WAVES];
  __shared__ carry_t s_carry;
  __shared__ uint64_t s_tile;
  __shared__ uint64_t s_clear_hi;
  __shared__ uint32_t s_parity, s_last, s_has_heads;
  __shared__ uint32_t s_heads[SEG ? TILE / 32 : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const bool multi = a.tiles > 1;
  const uint32_t *in = static_cast<const uint32_t *>(a.in);
  uint32_t *out = static_cast<uint32_t *>(a.out);
  uint32_t parity = 0;

  for (int iter = 0;; ++iter) {
    // ------------------------------------------------ 1. acquire a tile
    int64_t t;
    if (!multi) {
      if (iter > 0) break;
      t = 0;
    } else {
      if (tid == 0) {
        if (iter == 0) parity = ld_agent32(&a.hdr->parity);
        const uint64_t tk = __hip_atomic_fetch_add(&a.hdr->counter[parity], 1ull,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t last = tk == a.total_acquires - 1;
        if (tk < (uint64_t)a.tiles) st_agent(a.status + (1 - parity) * a.capacity + tk, 0ull);
        s_clear_hi = last ? ld_agent(&a.hdr->dirty[1 - parity]) : 0ull;
        s_tile = tk;
        s_parity = parity;
        s_last = last;
      }
      __syncthreads();
      t = (int64_t)s_tile;
      const uint32_t p = s_parity;
      if (s_last) {
        // last increment of this launch: finish cleaning the other array and
        // hand the workspace to the next launch
        uint64_t *other = a.status + (1 - p) * a.capacity;
        for (uint64_t i = (uint64_t)a.tiles + tid; i < s_clear_hi; i += BLOCK) st_agent(other + i, 0ull);
        if (tid == 0) {
          st_agent(&a.hdr->counter[1 - p], 0ull);
          st_agent(&a.hdr->dirty[1 - p], 0ull);
          st_agent(&a.hdr->dirty[p], (uint64_t)a.tiles);
          st_agent32(&a.hdr->parity, 1u - p);
        }
      }
      if (t >= a.tiles) break;
      parity = p;
    }

    const int64_t ptile = a.reverse ? (a.tiles - 1 - t) : t;   // physical tile
    const int64_t pb = ptile * (int64_t)TILE;
    const int64_t rem = a.n - pb;
    const int valid = rem < TILE ? (int)rem : TILE;
    const bool full = valid == TILE;

    // ------------------------------------------------ segment starts (LDS bitmap)
    bool any_head = false;
    if constexpr (SEG) {
      int64_t s_lo, s_hi;
      if (a.tile_seg) {
        s_lo = a.tile_seg[ptile];
        s_hi = a.tile_seg[ptile + 1];
      } else {
        s_lo = 0;
        s_hi = a.num_segments + 1;
      }
      if (s_hi > s_lo) {
        for (int i = tid; i < TILE / 32; i += BLOCK) s_heads[i] = 0u;
        if (tid == 0) s_has_heads = 0u;
        __syncthreads();
        const int shift = a.reverse ? 1 : 0;
        for (int64_t s = s_lo + tid; s < s_hi; s += BLOCK) {
          const bool real = a.reverse ? (s >= 1) : (s < a.num_segments);
          const int64_t ph = a.offsets[s] - shift;   // physical first element (last for reverse)
          if (real && ph >= pb && ph < pb + valid) {
            const int e = a.reverse ? (TILE - 1 - (int)(ph - pb)) : (int)(ph - pb);
            atomicOr(&s_heads[e >> 5], 1u << (e & 31));
            s_has_heads = 1u;
          }
        }
        __syncthreads();
        any_head = s_has_heads != 0u;
      }
    }

    // ------------------------------------------------ 2. load the tile once
    // raw[c] holds 4 consecutive physical elements; all loads of the tile are
    // issued before any is consumed (the branch is outside the chunk loop so
    // the compiler waits once, not once per chunk).
    u32x4 raw[CH];
    if (full && a.vec_in) {
#pragma unroll
      for (int c = 0; c < CH; ++c) raw[c] = load4<NT>(in + quad_base<TILE, WSPAN>(a.reverse, pb, wave, c, lane));
    } else {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int64_t q = quad_base<TILE, WSPAN>(a.reverse, pb, wave, c, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) raw[c][j] = (q + j < a.n) ? in[q + j] : 0u;
      }
    }
    lane_t v[CH][4];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
#pragma unroll
      for (int k = 0; k < 4; ++k) v[c][k] = Op::lfrom(a.reverse ? raw[c][3 - k] : raw[c][k]);
    }

    // ------------------------------------------------ 3. lane and wave scans
    uint32_t hb[CH];          // segment starts among this lane's 4 elements (bit k)
    lane_t lex[CH];           // lane-exclusive value within the chunk
    uint32_t lexf[CH];        // a segment starts in an earlier lane of the chunk
    lane_t ctot[CH];          // chunk total (lane 63 of the scan)
    uint32_t cflag[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      hb[c] = 0u;
      if constexpr (SEG) {
        if (any_head) {
          const int e0 = wave * WSPAN + c * 256 + lane * 4;
          hb[c] = (s_heads[e0 >> 5] >> (e0 & 31)) & 0xfu;
        }
      }
      // in-lane inclusive partials, restarting at segment starts
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        if constexpr (SEG) v[c][k] = ((hb[c] >> k) & 1u) ? v[c][k] : Op::ladd(v[c][k - 1], v[c][k]);
        else v[c][k] = Op::ladd(v[c][k - 1], v[c][k]);
      }
      lane_t x = v[c][3];
      uint32_t f = hb[c] != 0u;
      if constexpr (SEG) {
        wave_scan_seg<Op>(x, f);
        lexf[c] = lane_up1(f);
        cflag[c] = readlane32(f, 63);
      } else {
        x = wave_scan<Op>(x);
        lexf[c] = 0u;
        cflag[c] = 0u;
      }
      lex[c] = Op::lfrom(lane_up1(Op::lbits(x)));
      ctot[c] = Op::lfrom(readlane32(Op::lbits(x), 63));
    }

    // chunk chain within the wave (uniform values)
    carry_t cpre[CH];
    uint32_t cpref[CH];
    carry_t wsum = Op::czero();
    uint32_t wflag = 0u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      cpre[c] = wsum;
      cpref[c] = wflag;
      wsum = cflag[c] ? Op::widen(ctot[c]) : Op::cadd(wsum, Op::widen(ctot[c]));
      wflag |= cflag[c];
    }

    // ------------------------------------------------ 4. block combine
    if (lane == 0) {
      s_wtot[wave] = wsum;
      s_wflag[wave] = wflag;
    }
    __syncthreads();
    carry_t wpre = Op::czero(), agg = Op::czero();
    uint32_t wpref = 0u, aggf = 0u;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      if (w == wave) {
        wpre = agg;
        wpref = aggf;
      }
      const carry_t tw = s_wtot[w];
      const uint32_t fw = s_wflag[w];
      agg = fw ? tw : Op::cadd(agg, tw);
      aggf |= fw;
    }

    // ------------------------------------------------ 5. publish and look back
    bool first_is_head = false;
    if constexpr (SEG) first_is_head = any_head && (s_heads[0] & 1u);
    const bool need_carry = t > 0 && !first_is_head;
    if (multi && wave == 0) {
      uint64_t *st = a.status + parity * a.capacity;
      if (t == 0 || aggf) {
        // tile 0 and tiles containing a segment start know their prefix now
        const carry_t pv = (t == 0 && !aggf) ? Op::canon(Op::cadd(Op::czero(), Op::canon(agg)))
                                             : Op::canon(agg);
        if (lane == 0) st_agent(st + t, Op::pack(pv, kPrefix));
      } else if (lane == 0) {
        st_agent(st + t, Op::pack(agg, kAgg));
      }
      carry_t carry = Op::czero();
      if (need_carry) {
        carry = look_back<Op, K>(st, t, a.spin_limit, a.hdr);
        if (!aggf && lane == 0)
          st_agent(st + t, Op::pack(Op::canon(Op::cadd(carry, Op::canon(agg))), kPrefix));
      }
      if (lane == 0) s_carry = carry;
    }
    __syncthreads();
    const carry_t carry = need_carry ? s_carry : Op::czero();

    // ------------------------------------------------ 6. add the carry and store once
    const carry_t win = wpref ? wpre : Op::cadd(carry, wpre);   // carry into this wave
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const carry_t cin = cpref[c] ? cpre[c] : Op::cadd(win, cpre[c]);
      const lane_t L = Op::narrow(lexf[c] ? Op::widen(lex[c]) : Op::cadd(cin, Op::widen(lex[c])));
      lane_t o[4];
      if constexpr (SEG) {
        uint32_t seen = 0u;   // a segment starts at or before element k in this lane
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t h = (hb[c] >> k) & 1u;
          if (a.exclusive) {
            o[k] = h ? Op::lzero() : (seen ? v[c][k - (k > 0)] : (k == 0 ? L : Op::ladd(L, v[c][k - (k > 0)])));
          } else {
            seen |= h;
            o[k] = seen ? v[c][k] : Op::ladd(L, v[c][k]);
          }
          if (a.exclusive) seen |= h;
        }
      } else {
        if (a.exclusive) {
          o[0] = L;
          o[1] = Op::ladd(L, v[c][0]);
          o[2] = Op::ladd(L, v[c][1]);
          o[3] = Op::ladd(L, v[c][2]);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) o[k] = Op::ladd(L, v[c][k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) raw[c][k] = Op::lbits(a.reverse ? o[3 - k] : o[k]);
    }
    if (full && a.vec_out) {
#pragma unroll
      for (int c = 0; c < CH; ++c) store4<NT>(out + quad_base<TILE, WSPAN>(a.reverse, pb, wave, c, lane), raw[c]);
    } else {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int64_t q = quad_base<TILE, WSPAN>(a.reverse, pb, wave, c, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (q + j < a.n) out[q + j] = raw[c][j];
      }
    }

    if (a.one_tile || !multi) break;
    __syncthreads();   // LDS is reused by the next tile
  }
}

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

}  // namespace mi355scan
