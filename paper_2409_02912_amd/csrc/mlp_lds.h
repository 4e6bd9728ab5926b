// BF16 message-passing and readout bodies with every operand in LDS, shared by the per-layer
// MLP kernels and the persistent forward kernel.
#pragma once
#include "conv_common.h"

namespace {

constexpr int MLP_ROWS = 128;          // rows per tile, 4 waves x 2 m-blocks
constexpr int MLP_MB = 2;

// BF16 message passing with every operand in LDS.  The two 128x128 weight
// matrices are copied to LDS once per workgroup; 128-row activation tiles are
// DMA'd global -> LDS one tile ahead (double buffer), rows stored as sixteen
// 16-byte pieces XOR-swizzled by the row index so that the sixteen rows of an
// MFMA fragment hit distinct banks.  Each wave owns 32 rows: GEMM 1 reads its
// rows' fragments, writes the hidden activations back over them, and GEMM 2
// reads them again, so the tile needs no barrier between the two GEMMs.  The
// cross-UE sum is taken in registers: a lane holds four consecutive rows of one
// column, which for U = 1, 2, 4 are whole REs (tiles start on RE boundaries);
// U = 3 goes through LDS.  NW waves share a 128-row tile (8 waves: 16 rows each,
// two waves per SIMD to cover LDS latency).
namespace mp2 {
constexpr int AROWB = NRX_D * 2;         // bytes per activation row (bf16)
constexpr int TILEB = MLP_ROWS * AROWB;  // 32 KB
constexpr int WB = NRX_D * NRX_D * 2;    // 32 KB per weight matrix
constexpr int W2B = 4 * 16 * 64;         // readout second layer, prepped [chunk][16][32] bf16
__device__ __forceinline__ int apos(int row, int piece) { return row * AROWB + ((piece ^ (row & 15)) << 4); }
__device__ __forceinline__ int wpos(int c, int nb, int j, int lk) {
  const int row = (c * 8 + nb) * 16 + j;   // 64-byte rows of the prepped [chunk][nb][16][32] operand
  return row * 64 + ((lk ^ swz(row)) << 4);
}
}  // namespace mp2
constexpr int MP_LDS_BYTES = 2 * mp2::WB + 2 * mp2::TILEB;
constexpr int RO_LDS_BYTES = mp2::WB + mp2::W2B + 2 * mp2::TILEB;

// Tile sources of the MLP bodies: the layer's tile list strided over the grid, or the
// MLP_ROWS-row sub-tiles (whole REs) of one larger tile.
struct MlpGridTiles {
  const Tile *tiles;
  int n, first;
  __device__ MlpGridTiles(const Tile *t, int n_tiles) : tiles(t), n(n_tiles), first(blockIdx.x) {}
  __device__ bool valid(int i) const { return i < n; }
  __device__ Tile get(int i) const { return ldc(tiles + i); }
  __device__ int next(int i) const { return i + (int)gridDim.x; }
};
struct SubTiles {
  Tile t;
  int rows;          // rows per sub-tile (a multiple of the slot's UE count, at most MLP_ROWS)
  int first = 0;
  __device__ bool valid(int i) const { return i * rows < t.nrows; }
  __device__ Tile get(int i) const {
    const int r0 = i * rows;
    return Tile{t.slot, t.row0 + r0, t.nrows - r0 < rows ? t.nrows - r0 : rows, 0};
  }
  __device__ int next(int i) const { return i + 1; }
};

// lds: MP_LDS_BYTES bytes (both weight matrices, then two tile buffers).
template <int NW, typename Src>
__device__ __forceinline__ void mp_lds_body(const MlpArgs<bf16_t> &a, const Src &src, lds_u8 *lds) {
  using namespace mp2;
  constexpr int MBW = MLP_ROWS / 16 / NW;   // m-blocks per wave
  lds_u8 *lw1 = lds, *lw2 = lds + WB;
  auto lt = [&](int b) { return lds + 2 * WB + b * TILEB; };
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int ch0 = 8 * lr;
  float vmax = 0.f;
  // biases of this lane's channels, read once: a global load inside the tile loop would make the
  // compiler wait for every outstanding vector-memory operation, the next tile's copy included
  float bias1[8], bias2[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) { bias1[nb] = a.b1[ch0 + nb]; bias2[nb] = a.b2[ch0 + nb]; }

  // weights: 2 x 32 KB, 16 DMA instructions of 1 KB per wave (64-byte rows, swizzled pieces)
  {
    const i32x4_t r1 = rsrc_words(a.w1, WB), r2 = rsrc_words(a.w2, WB);
#pragma unroll
    for (int j = 0; j < WB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 16 + (lane >> 2);
      const uint32_t src = row * 64 + (((lane & 3) ^ swz(row)) << 4);
      dma16(r1, lds_addr(&lw1[ins * 1024]), src);
      dma16(r2, lds_addr(&lw2[ins * 1024]), src);
    }
  }
  // activation tile into buffer b: 32 instructions of 1 KB, 8 per wave; rows past the tile read zero
  auto stage = [&](const Tile &tl, int b) {
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const i32x4_t rs = rsrc_words(a.h + (g.row_base + tl.row0) * NRX_D, tl.nrows * AROWB);
#pragma unroll
    for (int j = 0; j < TILEB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 4 + (lane >> 4);
      const int piece = (lane & 15) ^ (row & 15);
      dma16(rs, lds_addr(lt(b) + ins * 1024), (uint32_t)(row * AROWB + piece * 16));
    }
  };
  int tile = src.first, b = 0;
  if (src.valid(tile)) stage(src.get(tile), 0);
  for (; src.valid(tile); tile = src.next(tile), b ^= 1) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's DMA (weights, this tile) has landed
    dma_barrier();                   // everyone's has; the other buffer's last readers are done
    if (src.valid(src.next(tile))) stage(src.get(src.next(tile)), b ^ 1);
    const Tile tl = src.get(tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const int U = ldc(&a.geo[tl.slot].U);
    lds_u8 *t = lt(b);
    const int rbase = wave * 16 * MBW;
    f32x4_t acc[MBW][8];
    auto gemm = [&](const lds_u8 *w) {
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        v16 af[MBW];
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) af[mb] = ld16(t + apos(rbase + mb * 16 + lr, 4 * c + lk));
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          const v16 bf = ld16(w + wpos(c, nb, lr, lk));
#pragma unroll
          for (int mb = 0; mb < MBW; ++mb) acc[mb][nb] = mfma_bf16(af[mb], bf, acc[mb][nb]);
        }
      }
    };
    gemm(lw1);
    // hidden = ReLU(acc + b1), bf16, over this wave's own rows (LDS operations of a wave stay in order)
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rbase + mb * 16 + 4 * lk + i;
        float v[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          const float x = acc[mb][nb][i] + bias1[nb];
          v[nb] = x > 0.f ? x : 0.f;
        }
        v16 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) q.w[k] = pack_bf2(v[2 * k], v[2 * k + 1]);
        st16(t + apos(r, lr), q);
      }
    gemm(lw2);
    auto emit = [&](int r, const float *v) {
      if (r < tl.nrows) {
        const int64_t grow = g.row_base + tl.row0 + r;
        if (a.out) pack8<bf16_t>::store(a.out + grow * NRX_D + ch0, v);
        if (a.out8) *reinterpret_cast<uint2 *>(a.out8 + grow * NRX_D + ch0) = fp8x8(v, a.out8_inv);
#pragma unroll
        for (int k = 0; k < 8; ++k) vmax = fmaxf(vmax, fabsf(v[k]));
      }
    };
    if (U != 3) {
      // lane rows 4 lk .. 4 lk + 3 of a 16-row block: whole REs for U = 1, 2, 4
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        float m[4][8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) m[i][nb] = acc[mb][nb][i] + bias2[nb];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v[8];
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) {
            float tot = 0.f;
#pragma unroll
            for (int o = 0; o < 4; ++o)
              if (o != i && (o / U) == (i / U)) tot += m[o][nb];
            v[nb] = U == 1 ? 0.f : tot;
          }
          emit(rbase + mb * 16 + 4 * lk + i, v);
        }
      }
    } else {
      // U = 3: messages (bf16) over this wave's rows, then sums across lanes and waves
      dma_barrier();   // every wave has finished GEMM 2 on the tile
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v[8];
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) v[nb] = acc[mb][nb][i] + bias2[nb];
          v16 q;
#pragma unroll
          for (int k = 0; k < 4; ++k) q.w[k] = pack_bf2(v[2 * k], v[2 * k + 1]);
          st16(t + apos(rbase + mb * 16 + 4 * lk + i, lr), q);
        }
      __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS stores are done
      dma_barrier();
      for (int e = tid; e < tl.nrows * 16; e += 64 * NW) {
        const int r = e >> 4, p = e & 15, re0 = r - r % 3;
        float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int o = 0; o < 3; ++o) {
          if (re0 + o == r) continue;
          float x[8];
          pack8<bf16_t>::load((const bf16_t *)(t + apos(re0 + o, p)), x);
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] += x[k];
        }
        const int64_t grow = g.row_base + tl.row0 + r;
        if (a.out) pack8<bf16_t>::store(a.out + grow * NRX_D + 8 * p, v);
        if (a.out8) *reinterpret_cast<uint2 *>(a.out8 + grow * NRX_D + 8 * p) = fp8x8(v, a.out8_inv);
#pragma unroll
        for (int k = 0; k < 8; ++k) vmax = fmaxf(vmax, fabsf(v[k]));
      }
    }
  }
  if (a.amax) atomicMax(a.amax, __float_as_uint(vmax));
}

// BF16 readout with its operands in LDS, organised like mp_lds_kernel: the
// 128x128 first layer and the 128x16 second layer (outputs j >= m_max zero) are
// copied to LDS once, 128-row tiles are DMA'd one ahead, and the hidden layer is
// written back over the wave's own rows.
// lds: RO_LDS_BYTES bytes (first- and second-layer weights, then two tile buffers).
template <int NW, typename Src>
__device__ __forceinline__ void readout_lds_body(const MlpArgs<bf16_t> &a, const Src &src, lds_u8 *lds) {
  using namespace mp2;
  constexpr int MBW = MLP_ROWS / 16 / NW;   // m-blocks per wave
  lds_u8 *lw1 = lds, *lw2 = lds + WB;
  auto lt = [&](int b) { return lds + WB + W2B + b * TILEB; };
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int ch0 = 8 * lr;
  const int M = a.m_max;
  const int NO = a.n_out ? a.n_out : M;
  const float b2 = lr < NO ? a.b2[lr] : 0.f;
  // first-layer biases of this lane's channels, read once (a global load inside the tile loop
  // would make the compiler wait for every outstanding vector-memory operation, the next
  // tile's copy included)
  float bias1[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) bias1[nb] = a.b1[ch0 + nb];
  {
    const i32x4_t r1 = rsrc_words(a.w1, WB), r2 = rsrc_words(a.w2, W2B);
#pragma unroll
    for (int j = 0; j < WB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 16 + (lane >> 2);
      dma16(r1, lds_addr(&lw1[ins * 1024]), row * 64 + (((lane & 3) ^ swz(row)) << 4));
    }
    if (wave < 4) {   // 64 rows of 64 bytes: one instruction per wave of the first four
      const int row = wave * 16 + (lane >> 2);
      dma16(r2, lds_addr(&lw2[wave * 1024]), row * 64 + (((lane & 3) ^ swz(row)) << 4));
    }
  }
  auto stage = [&](const Tile &tl, int b) {
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const i32x4_t rs = rsrc_words(a.h + (g.row_base + tl.row0) * NRX_D, tl.nrows * AROWB);
#pragma unroll
    for (int j = 0; j < TILEB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 4 + (lane >> 4);
      const int piece = (lane & 15) ^ (row & 15);
      dma16(rs, lds_addr(lt(b) + ins * 1024), (uint32_t)(row * AROWB + piece * 16));
    }
  };
  int tile = src.first, b = 0;
  if (src.valid(tile)) stage(src.get(tile), 0);
  for (; src.valid(tile); tile = src.next(tile), b ^= 1) {
    __builtin_amdgcn_s_waitcnt(0);
    dma_barrier();
    if (src.valid(src.next(tile))) stage(src.get(src.next(tile)), b ^ 1);
    const Tile tl = src.get(tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const int U = ldc(&a.geo[tl.slot].U);
    const int64_t llr_off = ldc(&a.geo[tl.slot].llr_off);
    lds_u8 *t = lt(b);
    const int rbase = wave * 16 * MBW;
    f32x4_t acc[MBW][8];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v16 af[MBW];
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) af[mb] = ld16(t + apos(rbase + mb * 16 + lr, 4 * c + lk));
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const v16 bf = ld16(lw1 + wpos(c, nb, lr, lk));
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) acc[mb][nb] = mfma_bf16(af[mb], bf, acc[mb][nb]);
      }
    }
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          const float x = acc[mb][nb][i] + bias1[nb];
          v[nb] = x > 0.f ? x : 0.f;
        }
        v16 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) q.w[k] = pack_bf2(v[2 * k], v[2 * k + 1]);
        st16(t + apos(rbase + mb * 16 + 4 * lk + i, lr), q);
      }
    // second layer: one 16-column block
    f32x4_t o[MBW];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) o[mb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int row = c * 16 + lr;
      const v16 bf = ld16(lw2 + row * 64 + ((lk ^ swz(row)) << 4));
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb)
        o[mb] = mfma_bf16(ld16(t + apos(rbase + mb * 16 + lr, 4 * c + lk)), bf, o[mb]);
    }
    bool bad = false;   // a stored value that is not finite (per-slot health word)
    if (a.chest) {
      // ReadoutChEst: row R = (s * 14 + t) * U + u is entry R of the slot's h layout
      const int Bs = ldc(&a.geo[tl.slot].B);
      const int64_t h_off = ldc(&a.geo[tl.slot].h_off);
      if (lr < 2 * Bs) {
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = rbase + mb * 16 + 4 * lk + i;
            const float v = o[mb][i] + b2;
            if (r < tl.nrows) {
              a.llr[(h_off + (int64_t)(tl.row0 + r) * Bs) * 2 + lr] = v;
              bad |= !__builtin_isfinite(v);
            }
          }
      }
    } else if (lr < M) {
      const int S = g.S;
      // bits per symbol of the slot's UEs by scalar loads (a per-lane load would wait as above)
      const int mu0 = ldc(&a.geo[tl.slot].m[0]), mu1 = ldc(&a.geo[tl.slot].m[1]);
      const int mu2 = ldc(&a.geo[tl.slot].m[2]), mu3 = ldc(&a.geo[tl.slot].m[3]);
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rbase + mb * 16 + 4 * lk + i;
          if (r < tl.nrows) {
            const int R = tl.row0 + r;
            const int s = R / (14 * U);
            const int rem = R - s * 14 * U;
            const int tt = rem / U, u = rem - tt * U;
            const int mu = u == 0 ? mu0 : (u == 1 ? mu1 : (u == 2 ? mu2 : mu3));
            if (!a.only_m || mu == a.only_m) {
              const float v = lr < mu ? o[mb][i] + b2 : 0.f;
              a.llr[llr_off + (((int64_t)u * 14 + tt) * S + s) * M + lr] = v;
              bad |= !__builtin_isfinite(v);
            }
          }
        }
    }
    if (a.slot_flags && __ballot(bad) != 0ull && lane == 0) atomicOr(&a.slot_flags[tl.slot], a.chest ? 2u : 1u);
    if (a.slot_done) {
      dma_barrier();   // every wave of the tile has issued its stores
      if (tid == 0) {
        const int per_slot = (g.S * 14 * U + MLP_ROWS - 1) / MLP_ROWS;
        if (atomicAdd(&a.slot_done[tl.slot], 1u) + 1u == (unsigned)per_slot) a.stamps[tl.slot] = wall_clock64();
      }
    }
  }
}

}  // namespace
