// Ring-pipelined 3x3 convolution body (operands in LDS, inline-assembly DMA), shared by the
// per-layer ring kernel and the persistent forward kernel.
//
// The tiles a workgroup computes come from a tile source:
//   GridTiles   - every gridDim.x-th tile of the layer's tile list (per-layer launches), in an
//                 XCD-aware order, with the next tile's first chunk prefetched during the last
//                 group of the current one and the weight ring running on across tiles;
//   RunTiles    - consecutive tiles of one slot (one work item of the persistent kernel): the ring
//                 starts and drains inside the call and runs on across the item's tiles.
//
// G taps of weights per ring slot and NBUF slots: the weights of group k + NBUF - 1 are requested
// while group k computes, which hides NBUF - 1 groups of DMA latency.  The next chunk's halo (or the
// next tile's first chunk) is requested at the first group of a chunk.
//
// DMA accounting (per wave, in issue order): every group issues BPW weight copies, and a chunk's
// first group APW halo copies after them.  At the end of group k the weights of group k + 1 must have
// landed; they were requested NBUF - 2 groups earlier, and at least (NBUF - 2) BPW weight copies (plus
// APW halo copies if a halo was requested since) were issued after them, so s_waitcnt vmcnt of that
// count suffices.  A halo requested at a chunk's first group is covered by the wait at the chunk's
// last group (NG - 1 > NBUF - 2 groups later).
// SCHED: 0 scheduling barriers between pipeline steps, 1 none (compiler interleaves),
// 2 scheduling barriers and raised wave priority around the MFMA steps, 3 scheduling barriers and a wave
// priority that falls as the wave gets through the group (3 at its first steps .. 0 at its last): of the
// two waves sharing a SIMD the one behind is issued first, so they reach the barrier together instead of
// one of them finishing its group alone at a lower MFMA rate
#pragma once
#include "conv_common.h"

namespace {

struct GridTiles {
  const Tile *tiles;
  int n, first, stride;
  __device__ GridTiles(const Tile *t, int n_tiles) : tiles(t), n(n_tiles) {
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so the workgroups of
    // one XCD get consecutive tiles (their halos overlap and then hit in that XCD's L2); gridDim.x
    // is a multiple of 8
    stride = gridDim.x;
    first = (blockIdx.x & 7) * (stride >> 3) + (blockIdx.x >> 3);
  }
  __device__ bool valid(int i) const { return i < n; }
  __device__ Tile get(int i) const { return ldc(tiles + i); }
  __device__ int next(int i) const { return i + stride; }
};

// tiles t0 .. t0 + n - 1 of one slot (tile t: rows t * rows .. of the slot)
struct RunTiles {
  int slot, t0, n, rows, slot_rows;
  int first = 0;
  __device__ bool valid(int i) const { return i < n; }
  __device__ Tile get(int i) const {
    const int r0 = (t0 + i) * rows;
    return Tile{slot, r0, slot_rows - r0 < rows ? slot_rows - r0 : rows, 0};
  }
  __device__ int next(int i) const { return i + 1; }
};

// ALIGNED: tiles of CONV_ALIGNED_TILE rows that start on subcarrier boundaries, so a halo is the tile's
// subcarriers plus one on each side (at most 504 + 2 x 56 rows) and the LDS saved goes to a third weight slot
template <int MB, int NW, int G, int NBUF, int ALIGNED = 0>
struct RingShape {
  static constexpr int TILE = 16 * MB * NW;
  static constexpr int HMAX = ALIGNED ? (CONV_ALIGNED_TILE + 2 * 56 + 15) / 16 * 16 : halo_rows_max(TILE);
  static constexpr int NINS = HMAX / 16;
  static constexpr int APW = (NINS + NW - 1) / NW;
  static constexpr int AROWS = APW * NW * 16;
  static constexpr int ZROW = AROWS;
  static constexpr int ABYTES = (AROWS + 1) * ROWB;    // one halo buffer (+ the zero row)
  static constexpr int BROWS = G * 8 * 16;             // 64-byte weight rows per group
  static constexpr int BBYTES = BROWS * ROWB;          // one ring slot
  static constexpr int LDS_BYTES = 2 * ABYTES + NBUF * BBYTES;
};

// lds: RingShape::LDS_BYTES bytes, 16-byte aligned (two halo buffers, then the NBUF weight slots).
// STAG: workgroups start at staggered times (0 .. 34 us, by their index within the XCD), so that the tile
// epilogues of the grid (residual reads and output stores, all CUs at once otherwise) spread over the MFMA
// phases of other CUs instead of arriving at HBM together.
template <typename T, int EPI, int MB, int NW, int G, int NBUF, int SCHED, typename Src, int STAG = 0, int ALIGNED = 0>
__device__ __forceinline__ void conv_ring_body(const ConvArgs<T> &a, const Src &src, lds_u8 *lds, float *lnp) {
  if constexpr (STAG) {
    const uint64_t t0 = wall_clock64();
    const uint64_t wait = (uint64_t)((blockIdx.x >> 3) & 15) * 225;   // device wall clock: 100 MHz
    while (wall_clock64() - t0 < wait) __builtin_amdgcn_s_sleep(8);
  }
  using Sh = RingShape<MB, NW, G, NBUF, ALIGNED>;
  static_assert(!ALIGNED || CONV_ALIGNED_TILE <= Sh::TILE, "aligned tile");
  constexpr int APW = Sh::APW;
  constexpr int ZROW = Sh::ZROW;
  constexpr int KC = 64 / (int)sizeof(T);
  constexpr int NG = 9 / G;                        // weight groups per chunk
  constexpr int BINS = Sh::BROWS / 16;             // weight DMA instructions per group
  constexpr int BPW = BINS / NW;
  static_assert(9 % G == 0 && BINS % NW == 0, "shape");
  static_assert(NBUF >= 2 && NG - 1 > NBUF - 2, "ring depth");
  constexpr int NB_ = (NBUF - 2) * BPW;
  static_assert(NB_ + APW < 16, "vmcnt immediate below");
  constexpr int WAIT_B = (0xF << 8) | (7 << 4) | NB_;            // weights of the next group landed
  constexpr int WAIT_BA = (0xF << 8) | (7 << 4) | (NB_ + APW);   // the same with a halo issued since
  auto lds_a = [&](int b) { return lds + b * Sh::ABYTES; };   // halo buffer b
  lds_u8 *lds_b0 = lds + 2 * Sh::ABYTES;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  if (tid < 4) {
    v16 z = {{0, 0, 0, 0}};
    st16(lds_a(0) + ZROW * ROWB + tid * 16, z);
    st16(lds_a(1) + ZROW * ROWB + tid * 16, z);
  }
  const int nch = (a.c0 + a.c1) / KC;
  const i32x4_t wrs = rsrc_words(a.w, 0x7FFFFFFF);
  // weights of group k (chunk k / NG, taps G * (k % NG) ..) into ring slot b
  auto stage_b = [&](int k, int b) {
    const int c = k / NG, grp = k - NG * c;
    const uint32_t base = (uint32_t)((c * 9 + G * grp) * 8 * 16) * ROWB;
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 16 + (lane >> 2);
      const int piece = (lane & 3) ^ swz(row);
      dma16(wrs, lds_addr(lds_b0 + b * Sh::BBYTES + ins * 16 * ROWB), base + row * ROWB + piece * 16);
    }
  };
  struct Geo {
    int64_t row_base;
    int rel0, halo, S, rps, U;
  };
  auto geo_of = [&](const Tile &tl) {
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    Geo q;
    q.U = g.U;
    q.S = g.S;
    q.rps = 14 * g.U;
    const int s_first = tl.row0 / q.rps;
    const int s_last = (tl.row0 + tl.nrows - 1) / q.rps;
    q.halo = (s_last - s_first + 3) * q.rps;
    q.rel0 = (s_first - 1) * q.rps;
    q.row_base = g.row_base;
    return q;
  };
  auto stage_a = [&](const Geo &q, int c, int b) {
    const T *srcp;
    int cs, coff;
    if (c * KC < a.c0) { srcp = a.src0; cs = a.c0; coff = c * KC; }
    else { srcp = a.src1; cs = a.c1; coff = c * KC - a.c0; }
    const i32x4_t rs = rsrc_words(srcp + q.row_base * cs + coff, q.S * q.rps * cs * (int)sizeof(T));
#pragma unroll
    for (int j = 0; j < APW; ++j) {
      const int ins = wave + NW * j;
      const int h = ins * 16 + (lane >> 2);
      const int piece = (lane & 3) ^ swz(h);
      // rows past the halo read out of range (zeros); the instruction count per wave stays fixed
      const uint32_t voff = h < q.halo ? (uint32_t)((q.rel0 + h) * cs * (int)sizeof(T) + piece * 16) : 0x80000000u;
      dma16(rs, lds_addr(lds_a(b) + ins * 16 * ROWB), voff);
    }
  };

  int ka = 0, kb = 0, gsa = 1 << 20;   // halo buffer, weight-slot counter, groups since a halo request
  int tile = src.first;
  if (src.valid(tile)) {
    const int ngrp0 = NG * nch;
#pragma unroll 1
    for (int j = 0; j < NBUF - 1; ++j) stage_b(j % ngrp0, j);
    stage_a(geo_of(src.get(tile)), 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    dma_barrier();
  }
  for (; src.valid(tile); tile = src.next(tile)) {
    const Tile tl = src.get(tile);
    const Geo q = geo_of(tl);
    int hc[MB], tt[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int r = wave * 16 * MB + mb * 16 + lr;
      const int R = tl.row0 + r;
      const int s = R / q.rps;
      tt[mb] = r < tl.nrows ? (R - s * q.rps) / q.U : -1;
      hc[mb] = R - q.rel0;
    }
    f32x4_t acc[MB][8];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const int ngrp = NG * nch;
    const int next_tile = src.next(tile);
    const bool has_next = src.valid(next_tile);
#pragma unroll 1
    for (int k = 0; k < ngrp; ++k) {
      const int c = k / NG, grp = k - NG * c;
      // weights NBUF - 1 groups ahead (wrapping into the next tile's groups: also after the last tile,
      // which keeps the per-group copy counts the waits below rely on), then the next halo
      stage_b((k + NBUF - 1) % ngrp, (kb + NBUF - 1) % NBUF);
      ++gsa;
      if (grp == 0) {
        if (c + 1 < nch) { stage_a(q, c + 1, (ka + 1) & 1); gsa = 0; }
        else if (has_next) { stage_a(geo_of(src.get(next_tile)), 0, (ka + 1) & 1); gsa = 0; }
      }
      const lds_u8 *la = lds_a(ka & 1);
      const lds_u8 *lbr = lds_b0 + (kb % NBUF) * Sh::BBYTES;
      // the G taps x 8 n-blocks of the group as one software pipeline: weight
      // fragments two steps ahead, the next tap's activation fragments half a tap ahead
      auto load_a = [&](int tg, v16 *af) {
        const int tap = G * grp + tg;
        const int di = tap / 3 - 1, dj = tap % 3 - 1;
        const int off = di * q.rps + dj * q.U;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const bool ok = tt[mb] >= 0 && (dj >= 0 || tt[mb] > 0) && (dj <= 0 || tt[mb] < 13);
          const int row = ok ? hc[mb] + off : ZROW;
          af[mb] = ld16(la + row * ROWB + ((lk ^ swz(row)) << 4));
        }
      };
      auto load_bf = [&](int i) {
        const int brow = i * 16 + lr;   // step i = tg * 8 + nb
        return ld16(lbr + brow * ROWB + ((lk ^ swz(brow)) << 4));
      };
      v16 afc[MB], afn[MB];
      load_a(0, afc);
      v16 b0 = load_bf(0), b1 = load_bf(1);
      if constexpr (SCHED == 2) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < 8 * G; ++i) {
        const int nb = i & 7;
        if constexpr (SCHED == 3) {
          constexpr int Q = (8 * G + 3) / 4;   // steps per priority level
          if (i == 0) __builtin_amdgcn_s_setprio(3);
          else if (i == Q) __builtin_amdgcn_s_setprio(2);
          else if (i == 2 * Q) __builtin_amdgcn_s_setprio(1);
          else if (i == 3 * Q) __builtin_amdgcn_s_setprio(0);
        }
        const v16 b2 = i + 2 < 8 * G ? load_bf(i + 2) : b1;
        if (nb == 4 && i / 8 + 1 < G) load_a(i / 8 + 1, afn);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mma<T>::run(afc[mb], b0, acc[mb][nb]);
        if (nb == 7 && i / 8 + 1 < G) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) afc[mb] = afn[mb];
        }
        b0 = b1;
        b1 = b2;
        if constexpr (SCHED != 1) __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (SCHED == 2 || SCHED == 3) __builtin_amdgcn_s_setprio(0);
      if (gsa <= NBUF - 2) __builtin_amdgcn_s_waitcnt(WAIT_BA);
      else __builtin_amdgcn_s_waitcnt(WAIT_B);
      dma_barrier();
      kb += 1;
      if (grp == NG - 1) ka += 1;
    }
    conv_epilogue<T, MB, EPI>(a, tl, ldc_geo(a.geo + tl.slot), acc, wave, lr, lk, lnp);
  }
  __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS outlives the call
}

}  // namespace
