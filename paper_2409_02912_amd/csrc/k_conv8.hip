// 3x3 resource-grid convolution with FP8 (E4M3) operands on the gfx950 scaled
// MFMA (16x16x128, FP32 accumulation): the CNN updates of the CGNN (Sec. II-A)
// at reduced precision, with a per-layer activation scale and per-output-channel
// weight scales.
//
// Layout and pipeline follow the BF16 kernel with both operands in LDS (the
// global -> LDS copies are issued as inline assembly, see dma16):
//   workgroup = NW waves, one tile of 16*MB*NW rows of one slot
//   wave      = 16*MB rows x 128 output channels (MB x 8 MFMA blocks)
//   K loop    = input-channel chunks of 64 (one 64-byte LDS row per activation
//               row, DMA'd global -> LDS, double buffered); the nine taps of a
//               chunk are consumed in five pairs, one k = 128 MFMA step being
//               (tap 2p, 64 channels) followed by (tap 2p+1, 64 channels); the
//               fifth pair holds tap 8 and zero weights
//   weights   = per tap pair 8 x 16 rows of 128 bytes (16 KB), DMA'd into a
//               two-slot ring one pair ahead; rows XOR-swizzled in 16-byte pieces
//   epilogue  = acc * weight scale, then the shared BF16 epilogue, which also
//               writes the E4M3 copy of the output consumed by the next conv
//
// The activation scale of each input is folded into the weights when they are
// quantised (prep_fp8_kernel): W'[n][k] = W[n][k] * s_in(k), s_w[n] = max|W'[n]|/448,
// W8 = W' / s_w[n], so that sum_k W x = s_w[n] * sum_k W8 x8 with x = s_in x8.
#include "common.h"
#include "internal.h"
#include "conv_common.h"

namespace {

constexpr int NPAIR = 5;          // tap pairs per chunk
constexpr int BROWB = 128;        // bytes per weight row (2 taps x 64 channels)
constexpr int BSLOT = 8 * 16 * BROWB;

__device__ __forceinline__ int bswz(int row) { return row & 7; }

// STAG: staggered start; PRIO: wave priority falling through each tap pair (3 at its first n-blocks .. 0 at its
// last), so that the two waves sharing a SIMD stay level
template <int EPI, int MB, int NW, int STAG, int PRIO = 0>
__global__ __launch_bounds__(64 * NW, 1) void conv3x3_fp8_kernel(ConvArgs<bf16_t> a) {
  constexpr int TILE = 16 * MB * NW;
  constexpr int HMAX = halo_rows_max(TILE);
  constexpr int NINS = HMAX / 16;
  constexpr int APW = (NINS + NW - 1) / NW;       // halo DMA instructions per wave (fixed)
  constexpr int AROWS = APW * NW * 16;
  constexpr int ZROW = AROWS;                      // all-zero row
  constexpr int KC = 64;                           // channels per chunk
  constexpr int BPW = BSLOT / 1024 / NW;           // weight DMA instructions per wave per pair
  static_assert(BSLOT / 1024 % NW == 0, "weight DMA split");
  static_assert(APW < 16, "vmcnt immediate below");
  __shared__ __align__(16) unsigned char lds_a[2][(AROWS + 1) * ROWB];
  __shared__ __align__(16) unsigned char lds_b[2][BSLOT];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar LDS addresses)
  const int lr = lane & 15, lk = lane >> 4;
  if (tid < 4) {
    v16 z = {{0, 0, 0, 0}};
    st16(&lds_a[0][ZROW * ROWB + tid * 16], z);
    st16(&lds_a[1][ZROW * ROWB + tid * 16], z);
  }
  const int nch = (a.c0 + a.c1) / KC;   // even (checked by the host)
  float lnp[1];
  if constexpr (STAG) {   // staggered start (see conv_ring_body): tile epilogues spread over time
    const uint64_t t0 = wall_clock64();
    const uint64_t wait = (uint64_t)((blockIdx.x >> 3) & 15) * 225;
    while (wall_clock64() - t0 < wait) __builtin_amdgcn_s_sleep(8);
  }

  const int G = gridDim.x;
  const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);

  const i32x4_t wrs = rsrc_words(a.w8, 0x7FFFFFFF);
  // weights of step k (chunk k / 5, pair k % 5) into ring slot b
  auto stage_b = [&](int k, int b) {
    const uint32_t base = (uint32_t)k * BSLOT;
    const int ln = lane_here();
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 8 + (ln >> 3);
      const int piece = (ln & 7) ^ bswz(row);
      dma16(wrs, lds_addr(&lds_b[b][ins * 1024]), base + row * BROWB + piece * 16);
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
    const uint8_t *src;
    int cs, coff;
    if (c * KC < a.c0) { src = a.src8_0; cs = a.c0; coff = c * KC; }
    else { src = a.src8_1; cs = a.c1; coff = c * KC - a.c0; }
    const i32x4_t rs = rsrc_words(src + q.row_base * cs + coff, q.S * q.rps * cs);
    const int ln = lane_here();
#pragma unroll
    for (int j = 0; j < APW; ++j) {
      const int ins = wave + NW * j;
      const int h = ins * 16 + (ln >> 2);
      const int piece = (ln & 3) ^ swz(h);
      // rows past the halo read out of range (zeros); the instruction count per wave stays fixed
      const uint32_t voff = h < q.halo ? (uint32_t)((q.rel0 + h) * cs + piece * 16) : 0x80000000u;
      dma16(rs, lds_addr(&lds_a[b][ins * 16 * ROWB]), voff);
    }
  };
  constexpr int WAIT_ALL = 0;
  constexpr int WAIT_KEEP_A = (0xF << 8) | (7 << 4) | APW;   // vmcnt <= APW, no wait on lgkm/exp

  int ka = 0, kb = 0;   // running halo-buffer and weight-slot counters
  int tile = lb;
  if (tile < a.n_tiles) {
    const Tile t0 = ldc(a.tiles + tile);
    stage_b(0, 0);
    stage_a(geo_of(t0), 0, 0);
    __builtin_amdgcn_s_waitcnt(WAIT_ALL);
    dma_barrier();
  }
  for (; tile < a.n_tiles; tile += G) {
    const Tile tl = ldc(a.tiles + tile);
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

    const int ngrp = NPAIR * nch;
    const int next_tile = tile + G;
#pragma unroll 1
    for (int k = 0; k < ngrp; ++k) {
      const int c = k / NPAIR, p = k - NPAIR * c;
      bool a_issued = false;
      if (k + 1 < ngrp) {
        stage_b(k + 1, (kb + 1) & 1);
        if (p == 0 && c + 1 < nch) { stage_a(q, c + 1, (ka + 1) & 1); a_issued = true; }
      } else if (next_tile < a.n_tiles) {
        // prefetch the next tile's first chunk and weight pair
        const Tile tn = ldc(a.tiles + next_tile);
        stage_b(0, (kb + 1) & 1);
        stage_a(geo_of(tn), 0, (ka + 1) & 1);
      }
      // local-address-space pointers: the fragment loads then stay where the scheduling barriers put them
      const lds_u8 *la = (const lds_u8 *)&lds_a[ka & 1][0];
      const lds_u8 *lbr = (const lds_u8 *)&lds_b[kb & 1][0];
      // taps 2p and 2p+1 (tap 9 does not exist: its weights are zero, its rows the zero row)
      const int t1 = 2 * p, t2 = 2 * p + 1;
      const int dj1 = t1 % 3 - 1, dj2 = t2 % 3 - 1;
      const int off1 = (t1 / 3 - 1) * q.rps + dj1 * q.U, off2 = (t2 / 3 - 1) * q.rps + dj2 * q.U;
      i32x8_t af[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int t = tt[mb];
        const bool ok1 = t >= 0 && (dj1 >= 0 || t > 0) && (dj1 <= 0 || t < 13);
        const bool ok2 = t2 < 9 && t >= 0 && (dj2 >= 0 || t > 0) && (dj2 <= 0 || t < 13);
        const int row1 = ok1 ? hc[mb] + off1 : ZROW;
        const int row2 = ok2 ? hc[mb] + off2 : ZROW;
        const v16 x1 = ld16(la + row1 * ROWB + ((lk ^ swz(row1)) << 4));
        const v16 x2 = ld16(la + row2 * ROWB + ((lk ^ swz(row2)) << 4));
        af[mb] = i32x8_t{(int)x1.w[0], (int)x1.w[1], (int)x1.w[2], (int)x1.w[3],
                         (int)x2.w[0], (int)x2.w[1], (int)x2.w[2], (int)x2.w[3]};
      }
      auto load_bf = [&](int nb) {
        const int brow = nb * 16 + lr;
        const v16 y1 = ld16(lbr + brow * BROWB + ((lk ^ bswz(brow)) << 4));
        const v16 y2 = ld16(lbr + brow * BROWB + (((4 + lk) ^ bswz(brow)) << 4));
        return i32x8_t{(int)y1.w[0], (int)y1.w[1], (int)y1.w[2], (int)y1.w[3],
                       (int)y2.w[0], (int)y2.w[1], (int)y2.w[2], (int)y2.w[3]};
      };
      // weight fragments two n-blocks ahead of the MFMAs that use them
      i32x8_t b0 = load_bf(0), b1 = load_bf(1);
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        if constexpr (PRIO) {
          if (nb == 0) __builtin_amdgcn_s_setprio(3);
          else if (nb == 2) __builtin_amdgcn_s_setprio(2);
          else if (nb == 4) __builtin_amdgcn_s_setprio(1);
          else if (nb == 6) __builtin_amdgcn_s_setprio(0);
        }
        const i32x8_t b2 = nb < 6 ? load_bf(nb + 2) : b1;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma_fp8(af[mb], b0, acc[mb][nb]);
        // pins the step's MFMAs here: each accumulator is updated once per pair, so without this the
        // compiler sinks every MFMA of the pair past its end-of-pair wait and barrier, after all its loads
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) asm volatile("" : "+v"(acc[mb][nb]));
        b0 = b1;
        b1 = b2;
        __builtin_amdgcn_sched_barrier(0);
      }
      // the next weight pair must have landed; a halo load issued after it may stay in flight
      if (a_issued) __builtin_amdgcn_s_waitcnt(WAIT_KEEP_A);
      else __builtin_amdgcn_s_waitcnt(WAIT_ALL);
      dma_barrier();
      kb += 1;
      if (p == NPAIR - 1) ka += 1;
    }
    // dequantise: output channel of (nb, lane) is 8 * lr + nb
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
      const float sw = a.wscale[8 * lr + nb];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mb][nb][i] *= sw;
    }
    conv_epilogue<bf16_t, MB, EPI, 1>(a, tl, ldc_geo(a.geo + tl.slot), acc, wave, lr, lk, lnp);
  }
}

// One workgroup per (output channel, layer): per-channel scale of the
// activation-scaled weights, then the E4M3 operand bytes in the kernel's
// [chunk][pair][nb][16][128 B] order (n = 8 * j + nb).
__global__ __launch_bounds__(256) void prep_fp8_kernel(const float *w, const Fp8Job *jobs, uint8_t *w8,
                                                       float *wscale) {
  __shared__ float red[4];
  const Fp8Job J = jobs[blockIdx.y];
  const int n = blockIdx.x, tid = threadIdx.x;
  float m = 0.f;
  for (int e = tid; e < 9 * J.cin_real; e += 256) {
    const int tap = e / J.cin_real, c = e - tap * J.cin_real;
    const float s = c < J.c0 ? J.s0 : J.s1;
    m = fmaxf(m, fabsf(w[J.src + ((int64_t)tap * J.cin_total + c) * NRX_D + n] * s));
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float sw = m > 0.f ? m / 448.f : 1.f;
  const float inv = 1.f / sw;
  if (tid == 0) wscale[J.sdst + n] = sw;
  const int nb = n & 7, j = n >> 3;
  const int nch = J.cin_real / 64;
  for (int e = tid; e < nch * NPAIR * BROWB; e += 256) {
    const int chunk = e / (NPAIR * BROWB), p = (e / BROWB) % NPAIR, b = e % BROWB;
    const int tap = 2 * p + (b >> 6);
    const int c = chunk * 64 + (b & 63);
    float v = 0.f;
    if (tap < 9) {
      const float s = c < J.c0 ? J.s0 : J.s1;
      v = fminf(fmaxf(w[J.src + ((int64_t)tap * J.cin_total + c) * NRX_D + n] * s * inv, -448.f), 448.f);
    }
    const int byte = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xFF;
    w8[J.dst + ((int64_t)((chunk * NPAIR + p) * 8 + nb) * 16 + j) * BROWB + b] = (uint8_t)byte;
  }
}

}  // namespace

const ConvVariant kConv8Variants[NRX_CONV8_VARIANTS] = {
    {8, 2, 2},   // 512-row tiles of 8 waves (4 m-blocks each), 2 waves/SIMD
    {6, 1, 2},   // 384-row tiles of 4 waves (6 m-blocks each)
    {4, 1, 2},   // 256-row tiles of 4 waves (4 m-blocks each)
    {8, 2, 2},   // as 0, workgroups started at staggered times
    {8, 2, 2},   // as 0, wave priority falling through each tap pair
};

void launch_conv8(const ConvArgs<bf16_t> &a, int epi, int variant, int grid, hipStream_t st) {
#define NRX_FP8_CASE(V, M, NWV, STG, PR)                                                               \
  if (variant == V) {                                                                                  \
    if (epi == EPI_LN_RELU)                                                                            \
      hipLaunchKernelGGL((conv3x3_fp8_kernel<EPI_LN_RELU, M, NWV, STG, PR>), dim3(grid), dim3(64 * NWV), 0, st, a); \
    else                                                                                               \
      hipLaunchKernelGGL((conv3x3_fp8_kernel<EPI_RESID, M, NWV, STG, PR>), dim3(grid), dim3(64 * NWV), 0, st, a);   \
    return;                                                                                            \
  }
  NRX_FP8_CASE(0, 4, 8, 0, 0)
  NRX_FP8_CASE(1, 6, 4, 0, 0)
  NRX_FP8_CASE(2, 4, 4, 0, 0)
  NRX_FP8_CASE(3, 4, 8, 1, 0)
  NRX_FP8_CASE(4, 4, 8, 0, 1)
#undef NRX_FP8_CASE
}

void launch_prep_fp8(const float *w, const Fp8Job *jobs, int n_jobs, uint8_t *w8, float *wscale, hipStream_t st) {
  if (n_jobs > 0) hipLaunchKernelGGL(prep_fp8_kernel, dim3(NRX_D, n_jobs), dim3(256), 0, st, w, jobs, w8, wscale);
}
