// Per-RE MLPs on MFMA: cross-UE message passing and the LLR readout.
//
// Message passing (Sec. II-A, CGNNit): every UE's state goes through an MLP,
// m_u = W2 ReLU(W1 h_u + b1) + b2, and UE u receives the sum of the messages of
// all *other* UEs at the same RE.  Rows are ordered (slot, s, t, u), so the U
// rows of one RE are adjacent; a tile holds whole REs, both 128x128 GEMMs run on
// MFMA (hidden activations pass through LDS to change from the output to the
// operand layout), and the cross-UE sum is read back from LDS.
//
// ReadoutLLRs (Sec. II-A): l = W2 ReLU(W1 h + b1) + b2 with d -> d -> m_max; both
// layers run on MFMA (the second as one 16-column block, outputs j >= m_max
// having zero weights), the hidden layer passing through LDS.  Outputs
// j >= m_u are written as 0 (masking, Sec. III) in the [u][t][s][j] layout, lane
// j of a row writing output j.
#include <type_traits>

#include "common.h"
#include "internal.h"
#include "conv_common.h"

namespace {

constexpr int MLP_ROWS = 128;          // rows per tile, 4 waves x 2 m-blocks
constexpr int MLP_MB = 2;

// A fragment of row `row` (natural channel order, global) for K chunk c.
template <typename T>
__device__ __forceinline__ v16 afrag_global(const T *row, int c, int lk) {
  constexpr int KC = 64 / (int)sizeof(T);
  return ld16(row + c * KC + lk * (KC / 4));
}

// acc[mb][nb] += A(rows) x W for a 128-deep K; A comes from `afn(mb, c)`.
template <typename T, typename AF>
__device__ __forceinline__ void gemm128(f32x4_t (&acc)[MLP_MB][8], const T *w, int lr, int lk, AF afn) {
  constexpr int KC = 64 / (int)sizeof(T);
  constexpr int NCH = NRX_D / KC;
#pragma unroll
  for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const T *wl = w + lr * KC + lk * (KC / 4);
#pragma unroll 2
  for (int c = 0; c < NCH; ++c) {
    v16 bf[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) bf[nb] = ld16(wl + (size_t)(c * 8 + nb) * 16 * KC);
#pragma unroll
    for (int mb = 0; mb < MLP_MB; ++mb) {
      v16 af = afn(mb, c);
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = mma<T>::run(af, bf[nb], acc[mb][nb]);
    }
  }
}

// LDS staging of a 128-row x 128-channel tile in operand layout: natural
// channel order, row pitch of 128 elements + 16 bytes.
template <typename T>
struct OpTile {
  static constexpr int KC = 64 / (int)sizeof(T);
  static constexpr int PITCHB = NRX_D * (int)sizeof(T) + 16;
  __device__ static __forceinline__ void put8(unsigned char *lds, int row, int ch0, const float *v) {
    T *r = reinterpret_cast<T *>(lds + row * PITCHB);
    pack8<T>::store(r + ch0, v);
  }
  __device__ static __forceinline__ v16 frag(const unsigned char *lds, int row, int c, int lk) {
    return ld16(lds + row * PITCHB + c * 64 + lk * 16);
  }
};

template <typename T>
__global__ __launch_bounds__(256) void mp_kernel(MlpArgs<T> a) {
  // one region reused: hidden activations (operand layout), then fp32 messages
  constexpr int MSG_PITCH = NRX_D + 4;   // floats
  constexpr int BYTES = MLP_ROWS * MSG_PITCH * 4;
  __shared__ __align__(16) unsigned char lds[BYTES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int ch0 = 8 * lr;
  float vmax = 0.f;   // max |aggregate| written by this thread (FP8 calibration)

  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const Tile tl = a.tiles[tile];
    const SlotGeo g = a.geo[tl.slot];
    const int64_t gbase = g.row_base + tl.row0;
    f32x4_t acc[MLP_MB][8];
    // GEMM 1 from global rows
    gemm128<T>(acc, a.w1, lr, lk, [&](int mb, int c) {
      int r = wave * 16 * MLP_MB + mb * 16 + lr;
      r = r < tl.nrows ? r : 0;
      return afrag_global<T>(a.h + (gbase + r) * NRX_D, c, lk);
    });
    __syncthreads();   // previous tile's readers of the LDS region are done
#pragma unroll
    for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 16 * MLP_MB + mb * 16 + 4 * lk + i;
        float v[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          float x = acc[mb][nb][i] + a.b1[ch0 + nb];
          v[nb] = x > 0.f ? x : 0.f;
        }
        if (sizeof(T) == 2) {   // the bf16 path feeds bf16-rounded hidden values to GEMM 2
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) v[nb] = bf2f(f2bf(v[nb]));
        }
        OpTile<T>::put8(lds, r, ch0, v);
        if (a.save_m1 && r < tl.nrows) pack8<T>::store(a.save_m1 + (gbase + r) * NRX_D + ch0, v);
      }
    __syncthreads();
    gemm128<T>(acc, a.w2, lr, lk, [&](int mb, int c) {
      int r = wave * 16 * MLP_MB + mb * 16 + lr;
      return OpTile<T>::frag(lds, r, c, lk);
    });
    __syncthreads();   // all hidden-activation reads done before the region is reused
    float *msg = reinterpret_cast<float *>(lds);
#pragma unroll
    for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 16 * MLP_MB + mb * 16 + 4 * lk + i;
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) msg[r * MSG_PITCH + ch0 + nb] = acc[mb][nb][i] + a.b2[ch0 + nb];
      }
    __syncthreads();
    // aggregation: agg_u = sum over the other UEs of the same RE
    const int U = g.U;
    for (int e = tid; e < tl.nrows * 16; e += 256) {
      const int r = e >> 4, c8 = (e & 15) * 8;
      const int u = r % U, re0 = r - u;
      float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int o = 0; o < U; ++o) {
        if (o == u) continue;
        const float *m = msg + (re0 + o) * MSG_PITCH + c8;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] += m[k];
      }
      if (a.out) pack8<T>::store(a.out + (gbase + r) * NRX_D + c8, v);
      if (a.out8) *reinterpret_cast<uint2 *>(a.out8 + (gbase + r) * NRX_D + c8) = fp8x8(v, a.out8_inv);
#pragma unroll
      for (int k = 0; k < 8; ++k) vmax = fmaxf(vmax, fabsf(v[k]));
    }
  }
  if (a.amax) atomicMax(a.amax, __float_as_uint(vmax));
}

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
__device__ __forceinline__ int apos(int row, int piece) { return row * AROWB + ((piece ^ (row & 15)) << 4); }
__device__ __forceinline__ int wpos(int c, int nb, int j, int lk) {
  const int row = (c * 8 + nb) * 16 + j;   // 64-byte rows of the prepped [chunk][nb][16][32] operand
  return row * 64 + ((lk ^ swz(row)) << 4);
}
}  // namespace mp2

template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void mp_lds_kernel(MlpArgs<bf16_t> a) {
  using namespace mp2;
  constexpr int MBW = MLP_ROWS / 16 / NW;   // m-blocks per wave
  __shared__ __align__(16) unsigned char lw1[WB];
  __shared__ __align__(16) unsigned char lw2[WB];
  __shared__ __align__(16) unsigned char lt[2][TILEB];
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
  auto stage = [&](int tile, int b) {
    const Tile tl = ldc(a.tiles + tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const i32x4_t rs = rsrc_words(a.h + (g.row_base + tl.row0) * NRX_D, tl.nrows * AROWB);
#pragma unroll
    for (int j = 0; j < TILEB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 4 + (lane >> 4);
      const int piece = (lane & 15) ^ (row & 15);
      dma16(rs, lds_addr(&lt[b][ins * 1024]), (uint32_t)(row * AROWB + piece * 16));
    }
  };
  int tile = blockIdx.x, b = 0;
  if (tile < a.n_tiles) stage(tile, 0);
  for (; tile < a.n_tiles; tile += gridDim.x, b ^= 1) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's DMA (weights, this tile) has landed
    dma_barrier();                   // everyone's has; the other buffer's last readers are done
    if (tile + (int)gridDim.x < a.n_tiles) stage(tile + gridDim.x, b ^ 1);
    const Tile tl = ldc(a.tiles + tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const int U = ldc(&a.geo[tl.slot].U);
    unsigned char *t = lt[b];
    const int rbase = wave * 16 * MBW;
    f32x4_t acc[MBW][8];
    auto gemm = [&](const unsigned char *w) {
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
          pack8<bf16_t>::load(reinterpret_cast<const bf16_t *>(t + apos(re0 + o, p)), x);
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
template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void readout_lds_kernel(MlpArgs<bf16_t> a) {
  using namespace mp2;
  constexpr int MBW = MLP_ROWS / 16 / NW;   // m-blocks per wave
  constexpr int W2B = 4 * 16 * 64;       // prepped [chunk][16][32] bf16
  __shared__ __align__(16) unsigned char lw1[WB];
  __shared__ __align__(16) unsigned char lw2[W2B];
  __shared__ __align__(16) unsigned char lt[2][TILEB];
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
  auto stage = [&](int tile, int b) {
    const Tile tl = ldc(a.tiles + tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const i32x4_t rs = rsrc_words(a.h + (g.row_base + tl.row0) * NRX_D, tl.nrows * AROWB);
#pragma unroll
    for (int j = 0; j < TILEB / 1024 / NW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 4 + (lane >> 4);
      const int piece = (lane & 15) ^ (row & 15);
      dma16(rs, lds_addr(&lt[b][ins * 1024]), (uint32_t)(row * AROWB + piece * 16));
    }
  };
  int tile = blockIdx.x, b = 0;
  if (tile < a.n_tiles) stage(tile, 0);
  for (; tile < a.n_tiles; tile += gridDim.x, b ^= 1) {
    __builtin_amdgcn_s_waitcnt(0);
    dma_barrier();
    if (tile + (int)gridDim.x < a.n_tiles) stage(tile + gridDim.x, b ^ 1);
    const Tile tl = ldc(a.tiles + tile);
    const SlotGeo g = ldc_geo(a.geo + tl.slot);
    const int U = ldc(&a.geo[tl.slot].U);
    const int64_t llr_off = ldc(&a.geo[tl.slot].llr_off);
    unsigned char *t = lt[b];
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

template <typename T>
__global__ __launch_bounds__(256) void readout_kernel(MlpArgs<T> a) {
  constexpr int KC = 64 / (int)sizeof(T);
  constexpr int NCH = NRX_D / KC;
  __shared__ __align__(16) unsigned char lds[MLP_ROWS * OpTile<T>::PITCHB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int ch0 = 8 * lr;
  const int M = a.m_max;
  const int NO = a.n_out ? a.n_out : M;
  const float b2 = lr < NO ? a.b2[lr] : 0.f;

  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const Tile tl = a.tiles[tile];
    const SlotGeo g = a.geo[tl.slot];
    const int64_t gbase = g.row_base + tl.row0;
    f32x4_t acc[MLP_MB][8];
    gemm128<T>(acc, a.w1, lr, lk, [&](int mb, int c) {
      int r = wave * 16 * MLP_MB + mb * 16 + lr;
      r = r < tl.nrows ? r : 0;
      return afrag_global<T>(a.h + (gbase + r) * NRX_D, c, lk);
    });
    // hidden layer -> LDS (operand layout) for the second GEMM
#pragma unroll
    for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 16 * MLP_MB + mb * 16 + 4 * lk + i;
        float q[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          float x = acc[mb][nb][i] + a.b1[ch0 + nb];
          q[nb] = x > 0.f ? x : 0.f;
        }
        if (sizeof(T) == 2) {
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) q[nb] = bf2f(f2bf(q[nb]));
        }
        OpTile<T>::put8(lds, r, ch0, q);
        // Var-IO: every readout keeps the hidden layer of its own modulation's rows only
        const bool mine = !a.only_m || a.geo[tl.slot].m[(tl.row0 + r) % g.U] == a.only_m;
        if (a.save_m1 && r < tl.nrows && mine) pack8<T>::store(a.save_m1 + (gbase + r) * NRX_D + ch0, q);
      }
    __syncthreads();
    // second layer: one 16-column MFMA block (outputs j < m_max, rest zero weights)
    f32x4_t o[MLP_MB];
#pragma unroll
    for (int mb = 0; mb < MLP_MB; ++mb) o[mb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const v16 bf = ld16(a.w2 + (c * 16 + lr) * KC + lk * (KC / 4));
#pragma unroll
      for (int mb = 0; mb < MLP_MB; ++mb)
        o[mb] = mma<T>::run(OpTile<T>::frag(lds, wave * 16 * MLP_MB + mb * 16 + lr, c, lk), bf, o[mb]);
    }
    const int U = g.U, S = g.S;
    bool bad = false;   // a stored value that is not finite (per-slot health word)
    if (a.chest) {
      // ReadoutChEst: row R = (s * 14 + t) * U + u is entry R of the slot's h layout
      if (lr < 2 * g.B) {
#pragma unroll
        for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = wave * 16 * MLP_MB + mb * 16 + 4 * lk + i;
            const float v = o[mb][i] + b2;
            if (r < tl.nrows) {
              a.llr[(g.h_off + (int64_t)(tl.row0 + r) * g.B) * 2 + lr] = v;
              bad |= !__builtin_isfinite(v);
            }
          }
      }
    } else if (lr < M) {
#pragma unroll
      for (int mb = 0; mb < MLP_MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = wave * 16 * MLP_MB + mb * 16 + 4 * lk + i;
          if (r < tl.nrows) {
            const int R = tl.row0 + r;
            const int s = R / (14 * U);
            const int rem = R - s * 14 * U;
            const int t = rem / U, u = rem - t * U;
            const int mu = a.geo[tl.slot].m[u];
            if (!a.only_m || mu == a.only_m) {
              const float v = lr < mu ? o[mb][i] + b2 : 0.f;
              a.llr[g.llr_off + (((int64_t)u * 14 + t) * S + s) * M + lr] = v;
              bad |= !__builtin_isfinite(v);
            }
          }
        }
    }
    if (a.slot_flags && __ballot(bad) != 0ull && lane == 0) atomicOr(&a.slot_flags[tl.slot], a.chest ? 2u : 1u);
    __syncthreads();   // LDS reads done before the next tile overwrites it
    if (a.slot_done && tid == 0) {
      // the workgroup that finishes a slot's last readout tile stamps the time (its LLR
      // stores are issued; no fence: a device-scope release would write back the L2 per tile)
      const int per_slot = (S * 14 * U + MLP_ROWS - 1) / MLP_ROWS;
      if (atomicAdd(&a.slot_done[tl.slot], 1u) + 1u == (unsigned)per_slot) a.stamps[tl.slot] = wall_clock64();
    }
  }
}

__global__ void stamp_start_kernel(unsigned int *slot_done, unsigned long long *stamps, unsigned int *flags, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    slot_done[i] = 0u;
    if (flags) flags[i] = 0u;
  }
  if (threadIdx.x == 0) stamps[n] = wall_clock64();
}

__global__ void copy_words_kernel(const unsigned int *src, unsigned int *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void stamp_latency_kernel(const unsigned long long *stamps, int n, double ticks_per_us, float *lat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) lat[i] = (float)((double)(long long)(stamps[i] - stamps[n]) / ticks_per_us);
}

}  // namespace

void launch_stamp_start(unsigned int *slot_done, unsigned long long *stamps, unsigned int *flags, int n,
                        hipStream_t st) {
  hipLaunchKernelGGL(stamp_start_kernel, dim3(1), dim3(256), 0, st, slot_done, stamps, flags, n);
}
void launch_copy_words(const unsigned int *src, unsigned int *dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(copy_words_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
}
void launch_stamp_latency(const unsigned long long *stamps, int n, double ticks_per_us, float *lat, hipStream_t st) {
  hipLaunchKernelGGL(stamp_latency_kernel, dim3((n + 255) / 256), dim3(256), 0, st, stamps, n, ticks_per_us, lat);
}

template <typename T>
void launch_mp(const MlpArgs<T> &a, int grid, hipStream_t st) {
  if constexpr (std::is_same<T, bf16_t>::value) {
    // inference: LDS-staged kernel (the training forward keeps the hidden activations: generic kernel)
    if (!a.save_m1) {
      hipLaunchKernelGGL(mp_lds_kernel<8>, dim3(grid), dim3(512), 0, st, a);
      return;
    }
  }
  hipLaunchKernelGGL(mp_kernel<T>, dim3(grid), dim3(256), 0, st, a);
}
template <typename T>
void launch_readout(const MlpArgs<T> &a, int grid, hipStream_t st) {
  if constexpr (std::is_same<T, bf16_t>::value) {
    if (!a.save_m1) {
      hipLaunchKernelGGL(readout_lds_kernel<8>, dim3(grid), dim3(512), 0, st, a);
      return;
    }
  }
  hipLaunchKernelGGL(readout_kernel<T>, dim3(grid), dim3(256), 0, st, a);
}
template void launch_mp<float>(const MlpArgs<float> &, int, hipStream_t);
template void launch_mp<bf16_t>(const MlpArgs<bf16_t> &, int, hipStream_t);
template void launch_readout<float>(const MlpArgs<float> &, int, hipStream_t);
template void launch_readout<bf16_t>(const MlpArgs<bf16_t> &, int, hipStream_t);
