// Two-pass scans: the multithreaded algorithms of Section 2.1 (Figures
// "Prefix Sum + Increment" and "Accumulate + Prefix Sum") moved to device
// scale, with the cache-friendly partitioning of Section 2.2 as an option.
// A workgroup plays the paper's thread and a tile its partition:
//
//   Prefix Sum + Increment   pass 1: each tile is scanned locally and written,
//                                    its total goes to sums[t];
//                            middle: exclusive scan of sums;
//                            pass 2: each tile adds sums[t] to its results.
//                            HBM traffic: 16 bytes per element.
//   Accumulate + Prefix Sum  pass 1: each tile only adds up its elements
//                                    into sums[t] (no writes);
//                            middle: exclusive scan of sums;
//                            pass 2: each tile is scanned with sums[t] as
//                                    its offset and written.
//                            HBM traffic: 12 bytes per element.
//
// With partitions, the three steps run partition by partition and a running
// total carries the sum of the finished partitions into the next one (the
// paper's offset from the sums array): pass 2 then re-reads data pass 1 has
// just read, which the last-level cache may still hold.
//
// These kernels exist to measure the paper's traffic argument against the
// single-pass kernel (8 bytes per element); they reuse its in-register tile
// scan but need no look-back, so every workgroup takes one tile.
#pragma once
#include "scan_device.hpp"

namespace mi355scan {

// Sum of a 64-bit or 32-bit carry over the lanes of a wave (butterfly).
template <class Op>
__device__ __forceinline__ typename Op::carry_t wave_sum(typename Op::carry_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = Op::cadd(v, __shfl_xor(v, m, 64));
  return v;
}

// Pass 1 of Accumulate + Prefix Sum: sums[t] = total of tile t (carry
// arithmetic: uint32 wrapping, or float64 for float32 elements).  NT: the
// loads bypass the caches (an unpartitioned pass 1 cannot hand its data to
// pass 2 through them anyway).
template <class Op, int BLOCK, int ITEMS, bool NT, bool VEC>
__global__ void __launch_bounds__(BLOCK) tile_totals(TwoPassArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using carry_t = typename Op::carry_t;
  __shared__ carry_t s_w[SH::WAVES];
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int64_t t = a.tile0 + blockIdx.x;
  u32x4 R[SH::CH];
  const WaveSpan<SH, NT, false, VEC> in(a.k.in, a.k, t, wave, lane);
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) in.load(c, R[c]);
  carry_t s = Op::czero();
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) {
    // four elements in lane arithmetic, then one carry add per group
    typename Op::lane_t g = Op::ladd(Op::ladd(Op::lfrom(R[c][0]), Op::lfrom(R[c][1])),
                                     Op::ladd(Op::lfrom(R[c][2]), Op::lfrom(R[c][3])));
    s = Op::cadd(s, Op::widen(g));
  }
  s = wave_sum<Op>(s);
  if (lane == 0) s_w[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    carry_t tot = Op::czero();
#pragma unroll
    for (int w = 0; w < SH::WAVES; ++w) tot = Op::cadd(tot, s_w[w]);
    static_cast<carry_t *>(a.sums)[t] = tot;
  }
}

// Middle step: sums[tile0 .. tile0+ntiles) <- run + exclusive prefix sums of
// themselves, and run <- run + their total.  One workgroup of kTotalsBlock
// threads; thread i takes a contiguous run of entries.  The partition that
// starts at tile 0 takes run = 0 (nothing is read from it).
constexpr int kTotalsBlock = 1024;

template <class Op>
__global__ void __launch_bounds__(kTotalsBlock) scan_totals(TwoPassArgs a) {
  using carry_t = typename Op::carry_t;
  constexpr int W = kTotalsBlock / 64;
  __shared__ carry_t s_w[W];
  __shared__ carry_t s_base;
  carry_t *s = static_cast<carry_t *>(a.sums) + a.tile0;
  carry_t *run = static_cast<carry_t *>(a.run);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = a.ntiles;
  const int64_t per = (m + kTotalsBlock - 1) / kTotalsBlock;
  const int64_t lo = per * tid < m ? per * tid : m;
  const int64_t hi = lo + per < m ? lo + per : m;
  carry_t mine = Op::czero();
  for (int64_t i = lo; i < hi; ++i) mine = Op::cadd(mine, s[i]);
  // inclusive scan of the threads' totals: within the wave, then across waves
  carry_t incl = mine;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const carry_t up = __shfl_up(incl, d, 64);
    if (lane >= d) incl = Op::cadd(up, incl);
  }
  if (lane == 63) s_w[wave] = incl;
  if (tid == 0) s_base = a.tile0 == 0 ? Op::czero() : *run;
  __syncthreads();
  // exclusive prefix of this thread's run: base, the waves below, the lanes below
  carry_t ex = s_base;
  for (int w = 0; w < wave; ++w) ex = Op::cadd(ex, s_w[w]);
  const carry_t below = __shfl_up(incl, 1, 64);
  if (lane) ex = Op::cadd(ex, below);
  for (int64_t i = lo; i < hi; ++i) {
    const carry_t v = s[i];
    s[i] = ex;
    ex = Op::cadd(ex, v);
  }
  if (tid == kTotalsBlock - 1) *run = ex;   // the last thread's running value is the grand total
}

// Scan of one tile with an offset: pass 2 of Accumulate + Prefix Sum (LOCAL
// false: offset = sums[t]) or pass 1 of Prefix Sum + Increment (LOCAL true:
// offset 0, and the tile's total goes to sums[t]).
template <class Op, int BLOCK, int ITEMS, bool LOCAL, bool NT, bool VEC>
__global__ void __launch_bounds__(BLOCK) scan_tile_offset(TwoPassArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using carry_t = typename Op::carry_t;
  __shared__ carry_t s_wtot[SH::WAVES];
  __shared__ uint32_t s_wflag[SH::WAVES];
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int64_t t = a.tile0 + blockIdx.x;
  u32x4 R[SH::CH];
  {
    const WaveSpan<SH, NT, false, VEC> in(a.k.in, a.k, t, wave, lane);
#pragma unroll
    for (int c = 0; c < SH::CH; ++c) in.load(c, R[c]);
  }
  int fh;
  carry_t wsum, wpre, agg;
  uint32_t wflag, wpref, aggf;
  scan_wave<Op, SH, false, false>(a.k.exclusive, 0u, wave, lane, false, nullptr, R, fh, wsum, wflag);
  combine_waves<Op, SH::WAVES>(wave, lane, wsum, wflag, s_wtot, s_wflag, wpre, wpref, agg, aggf);
  carry_t off = Op::czero();
  if constexpr (LOCAL) {
    if (threadIdx.x == 0) static_cast<carry_t *>(a.sums)[t] = agg;
  } else {
    off = static_cast<const carry_t *>(a.sums)[t];
  }
  apply_carry<Op, SH, false, false>(Op::cadd(off, wpre), R, lane, fh);
  const WaveSpan<SH, NT, false, VEC> out(a.k.out, a.k, t, wave, lane);
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) out.store(c, R[c]);
}

// Pass 2 of Prefix Sum + Increment: out[tile t] += sums[t] (the offset is
// narrowed once to the element type, as the single-pass kernel does).
template <class Op, int BLOCK, int ITEMS, bool NT, bool VEC>
__global__ void __launch_bounds__(BLOCK) increment_tiles(TwoPassArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  using carry_t = typename Op::carry_t;
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int64_t t = a.tile0 + blockIdx.x;
  const typename Op::lane_t off = Op::narrow(static_cast<const carry_t *>(a.sums)[t]);
  const WaveSpan<SH, NT, false, VEC> io(a.k.out, a.k, t, wave, lane);
  u32x4 R[SH::CH];
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) io.load(c, R[c]);
#pragma unroll
  for (int c = 0; c < SH::CH; ++c) {
#pragma unroll
    for (int k = 0; k < 4; ++k) R[c][k] = Op::lbits(Op::ladd(off, Op::lfrom(R[c][k])));
    io.store(c, R[c]);
  }
}

}  // namespace mi355scan
