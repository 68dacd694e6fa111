// Streaming ceiling of the scan's memory access pattern (a measurement
// kernel, not a scan).  It moves exactly the scan's two words per element --
// the traffic floor that the cache-friendly partitioning of Section 2.2 aims
// for -- with the scan kernel's tiles, wave spans, 128-bit buffer accesses,
// cache policy, resident grid, tile counter and store/load hand-off, but
// without the in-register scan and the look-back: each element is loaded,
// incremented (out_i = in_i + 1 modulo 2^32, so the result can be checked)
// and stored.  The time of this kernel at a tile shape is the floor that the
// scan kernel of the same shape could reach if its scan and inter-tile carry
// cost nothing; the scan's fraction of it separates the cost of the method
// from the cost of the memory system.
#pragma once

#include "scan_device.hpp"

namespace mi355scan {

template <int BLOCK, int ITEMS, bool NT, int MINW>
__global__ void __launch_bounds__(BLOCK, MINW) stream_tiles(KernelArgs a) {
  using SH = Shape<BLOCK, ITEMS>;
  constexpr bool kVec = true;   // 16-byte aligned buffers only (checked by the host)
  __shared__ int64_t s_tile[2];
  __shared__ uint32_t s_parity;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const bool multi = a.tiles > 1;
  const bool resident = multi && !a.one_tile;
  uint32_t parity = 0;

  int64_t t = 0;
  if (multi) {
    if (wave == 0) {
      parity = readlane32(lane == 0 ? ld_agent32(&a.hdr->parity) : 0u, 0);
      t = acquire_tile(a, parity, lane);
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
  if (t < a.tiles) load_tile<SH, NT, false, kVec>(a, t, wave, lane, R);

  for (int it = 0;; ++it) {
    const int slot = it & 1;
    if (t >= a.tiles) break;
#pragma unroll
    for (int c = 0; c < SH::CH; ++c) R[c] += 1u;

    // the scan kernel's hand-off: half of the stores, the next tile from the
    // counter, then each further store followed by a load into the chunk it
    // freed
    constexpr int KH = SH::CH / 2;
    const WaveSpan<SH, NT, false, kVec> out(a.out, a, t, wave, lane);
#pragma unroll
    for (int c = 0; c < KH; ++c) out.store(c, R[c]);
    int64_t next = a.tiles;
    if (resident) {
      if (wave == 0) {
        const int64_t tk = acquire_tile(a, parity, lane);
        if (lane == 0) s_tile[slot ^ 1] = tk;
      }
      __syncthreads();
      next = s_tile[slot ^ 1];
    }
    if (next < a.tiles) {
      const WaveSpan<SH, NT, false, kVec> in(a.in, a, next, wave, lane);
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) {
        out.store(c, R[c]);
        in.load(c - KH, R[c - KH]);
      }
#pragma unroll
      for (int c = SH::CH - KH; c < SH::CH; ++c) in.load(c, R[c]);
    } else {
#pragma unroll
      for (int c = KH; c < SH::CH; ++c) out.store(c, R[c]);
    }
    t = next;
  }
}

}  // namespace mi355scan
