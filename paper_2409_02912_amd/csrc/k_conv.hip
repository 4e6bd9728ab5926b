// 3x3 resource-grid convolution as an implicit GEMM on MFMA (gfx950).
//
// The CGNN's StateInit and CNN updates (Sec. II-A) are 3x3 convolutions over
// (subcarrier, OFDM symbol) applied to every UE's state.  Activations are
// stored channels-last as rows (slot, s, t, u) x 128 channels, so the 3x3
// neighbourhood of a row is nine fixed row offsets {di*14U + dj*U} and the
// rows of a tile plus one subcarrier of halo on each side are one contiguous
// block of memory.
//
// Work decomposition
//   workgroup = 4 waves, one tile of 64*MB consecutive rows of one slot; the
//               tile shape (MB, waves per SIMD, prefetch) is a compiled variant
//   wave      = 16*MB rows x all 128 output channels (MB x 8 MFMA blocks)
//   K loop    = input-channel chunks of 64 bytes; per chunk the halo block is
//               copied global -> LDS by buffer DMA (double buffered, the next
//               chunk in flight while the current one is consumed) and reused by
//               all nine taps; weights go global -> VGPRs directly (optionally
//               prefetched one tap ahead), since every wave needs all 128 output
//               columns.  LDS rows are XOR-swizzled in 16-byte pieces.
//   t edges   = taps reaching t = -1 or t = 14 read a zero LDS row;
//               s edges = halo rows outside the slot are staged as zeros.
//   epilogue  = bias (+ positional-encoding field) -> store, or LayerNorm over
//               the 128 channels of a row (intra-wave shuffles) -> ReLU, or a
//               residual add; each lane owns 8 consecutive channels of a row so
//               stores are full 16/32-byte vectors.
#include <type_traits>

#include "common.h"
#include "internal.h"
#include "conv_common.h"
#include "conv_ring.h"

#ifndef NRX_LDS_MB
#define NRX_LDS_MB 6
#endif

namespace {

template <typename T, int MB, int EPI, int OCC, bool PREF>
__global__ __launch_bounds__(256, OCC) void conv3x3_kernel(ConvArgs<T> a) {
  constexpr int TILE = 64 * MB;
  constexpr int HMAX = halo_rows_max(TILE);       // rows staged per chunk, multiple of 16
  constexpr int ZROW = HMAX;                       // all-zero row
  constexpr int KC = 64 / (int)sizeof(T);          // channels per chunk
  constexpr int NINS = HMAX / 16;                  // 1 KB DMA instructions per chunk
  __shared__ __align__(16) unsigned char lds[2][(HMAX + 1) * ROWB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lr = lane & 15;   // MFMA row (A) / column (B, D) index
  const int lk = lane >> 4;   // MFMA k-group (A, B) / row-group (D)

  if (tid < 8) {
    v16 z = {{0, 0, 0, 0}};
    st16(&lds[tid >> 2][ZROW * ROWB + (tid & 3) * 16], z);
  }

  const int cin = a.c0 + a.c1;
  const int nch = cin / KC;
  int buf = 0;
  float lnp[EPI == EPI_LN_BWD ? 16 : 1];   // this lane's dgamma / dbeta partial sums (EPI_LN_BWD)
#pragma unroll
  for (int k = 0; k < (EPI == EPI_LN_BWD ? 16 : 1); ++k) lnp[k] = 0.f;

  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so
  // give the workgroups of one XCD consecutive tiles (their halos overlap and
  // then hit in that XCD's L2).  gridDim.x is a multiple of 8.
  const int G = gridDim.x;
  const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  for (int tile = lb; tile < a.n_tiles; tile += G) {
    const Tile tl = a.tiles[tile];
    const SlotGeo g = a.geo[tl.slot];
    const int U = g.U, S = g.S;
    const int rps = 14 * U;                       // rows per subcarrier
    const int s_first = tl.row0 / rps;
    const int s_last = (tl.row0 + tl.nrows - 1) / rps;
    const int halo = (s_last - s_first + 3) * rps;
    const int rel0 = (s_first - 1) * rps;         // slot-relative row of halo row 0

    // per-lane A-row geometry for each m-block
    int hc[MB], tt[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      int r = wave * 16 * MB + mb * 16 + lr;
      int R = tl.row0 + r;
      int s = R / rps;
      int t = (R - s * rps) / U;
      tt[mb] = r < tl.nrows ? t : -1;            // -1 marks rows past the tile
      hc[mb] = R - rel0;
    }

    // Halo staging by buffer -> LDS DMA: rows outside the slot fall outside the
    // buffer range and read as zero (the conv's zero padding in s).
    auto stage = [&](int c, int b) {
      const T *src;
      int cs, coff;
      if (c * KC < a.c0) { src = a.src0; cs = a.c0; coff = c * KC; }
      else { src = a.src1; cs = a.c1; coff = c * KC - a.c0; }
      const T *base = src + g.row_base * cs + coff;
      const int nrec = S * rps * cs * (int)sizeof(T);
      __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, nrec, 0x00020000);
#pragma unroll
      for (int j = 0; j < (NINS + 3) / 4; ++j) {
        const int ins = wave + 4 * j;
        if (ins < NINS && ins * 16 < halo) {
          const int h = ins * 16 + (lane >> 2);
          const int piece = (lane & 3) ^ swz(h);
          const uint32_t voff = (uint32_t)((rel0 + h) * cs * (int)sizeof(T) + piece * 16);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)&lds[b][ins * 16 * ROWB], 16, voff, 0, 0, 0);
        }
      }
    };

    f32x4_t acc[MB][8];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    stage(0, buf ^ 1);
    buf ^= 1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // weight fragment pointer for (chunk, tap, nb): prepped [chunk][tap][nb][16][KC]
    const T *wl = a.w + lr * KC + lk * (KC / 4);
    auto load_b = [&](int c, int tap, v16 *bf) {
      const T *p = wl + (size_t)((c * 9 + tap) * 8) * 16 * KC;
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) bf[nb] = ld16(p + nb * 16 * KC);
    };

    v16 bcur[8], bnxt[8];
    if constexpr (PREF) load_b(0, 0, bcur);
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) stage(c + 1, buf ^ 1);
      const unsigned char *lds_c = &lds[buf][0];
      // rolled: unrolling lets the scheduler hoist weight loads of later taps
      // and exceed the register budget of the 2-waves/SIMD variants
#pragma unroll 1
      for (int tap = 0; tap < 9; ++tap) {
        if constexpr (PREF) {
          if (tap < 8) load_b(c, tap + 1, bnxt);
          else if (c + 1 < nch) load_b(c + 1, 0, bnxt);
        } else {
          load_b(c, tap, bcur);
        }
        const int di = tap / 3 - 1, dj = tap % 3 - 1;
        const int off = di * rps + dj * U;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const bool ok = tt[mb] >= 0 && (dj >= 0 || tt[mb] > 0) && (dj <= 0 || tt[mb] < 13);
          const int row = ok ? hc[mb] + off : ZROW;
          const v16 af = ld16(lds_c + row * ROWB + ((lk ^ swz(row)) << 4));
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = mma<T>::run(af, bcur[nb], acc[mb][nb]);
        }
        if constexpr (PREF) {
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) bcur[nb] = bnxt[nb];
        }
      }
      if (c + 1 < nch) {
        buf ^= 1;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
      }
    }

    conv_epilogue<T, MB, EPI>(a, tl, g, acc, wave, lr, lk, lnp);
  }
  conv_ln_reduce<EPI, 4>(lnp, reinterpret_cast<float *>(&lds[0][0]), a.ln_part, tid, wave, lr, lk);
}


// Variant with both MFMA operands in LDS.  Tiles of 16*MB*NW rows (MB m-blocks
// per wave).  Per 64-byte K chunk the halo block is DMA'd once; the weights of
// each group of three taps (one tap row di) are DMA'd into a two-slot ring one
// group ahead, so the MFMA loop reads only LDS.  Every wave issues a fixed
// number of halo DMA instructions, which lets the wait for the next weight group
// (issued first) leave the halo loads in flight (s_waitcnt vmcnt(APW)).  The
// next tile's first chunk is prefetched during the last group of the current one.
//
// The two halo buffers and the two weight slots are four distinct LDS arrays,
// and the K loop is unrolled over its period (two chunks = six groups) so that
// every access names its array statically: the compiler can then tell that a
// DMA in flight writes a different array than the one being read, and does not
// drain the DMA queue before each LDS read.  Tile metadata is read through the
// constant address space (scalar loads), so it does not wait on the DMA queue
// either.
template <typename T, int EPI, int MB, int NW>
__global__ __launch_bounds__(64 * NW, 1) void conv3x3_lds_kernel(ConvArgs<T> a) {
  constexpr int TILE = 16 * MB * NW;
  constexpr int HMAX = halo_rows_max(TILE);
  constexpr int NINS = HMAX / 16;                  // halo DMA instructions per chunk
  constexpr int APW = (NINS + NW - 1) / NW;       // per wave (fixed)
  constexpr int AROWS = APW * NW * 16;             // rows written per chunk (>= HMAX)
  constexpr int ZROW = AROWS;                      // all-zero row
  constexpr int KC = 64 / (int)sizeof(T);
  constexpr int BROWS = 3 * 8 * 16;                // 64-byte weight rows per 3-tap group
  constexpr int BPW = BROWS / 16 / NW;             // weight DMA instructions per wave per group
  static_assert(APW < 16, "vmcnt immediate below");
  __shared__ __align__(16) unsigned char lds_a0[(AROWS + 1) * ROWB];
  __shared__ __align__(16) unsigned char lds_a1[(AROWS + 1) * ROWB];
  __shared__ __align__(16) unsigned char lds_b0[BROWS * ROWB];
  __shared__ __align__(16) unsigned char lds_b1[BROWS * ROWB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar LDS addresses)
  const int lr = lane & 15, lk = lane >> 4;
  if (tid < 4) {
    v16 z = {{0, 0, 0, 0}};
    st16(&lds_a0[ZROW * ROWB + tid * 16], z);
    st16(&lds_a1[ZROW * ROWB + tid * 16], z);
  }
  const int cin = a.c0 + a.c1;
  const int nch = cin / KC;   // even (checked by the host)
  float lnp[EPI == EPI_LN_BWD ? 16 : 1];
#pragma unroll
  for (int k = 0; k < (EPI == EPI_LN_BWD ? 16 : 1); ++k) lnp[k] = 0.f;

  const int G = gridDim.x;
  const int lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);

  // weight buffer resource (bounds unchecked: offsets are within the layer's block)
  const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc((void *)a.w, 0, 0x7FFFFFFF, 0x00020000);
  auto stage_b = [&](int c, int grp, unsigned char *dst) {
    const uint32_t base = (uint32_t)((c * 9 + 3 * grp) * 8 * 16) * ROWB;
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      const int ins = wave + NW * j;
      const int row = ins * 16 + (lane >> 2);
      const int piece = (lane & 3) ^ swz(row);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, (lds_void *)&dst[ins * 16 * ROWB], 16,
                                                base + row * ROWB + piece * 16, 0, 0, 0);
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
  auto stage_a = [&](const Geo &q, int c, unsigned char *dst) {
    const T *src;
    int cs, coff;
    if (c * KC < a.c0) { src = a.src0; cs = a.c0; coff = c * KC; }
    else { src = a.src1; cs = a.c1; coff = c * KC - a.c0; }
    const __amdgpu_buffer_rsrc_t rs =
        uniform_rsrc(src + q.row_base * cs + coff, q.S * q.rps * cs * (int)sizeof(T));
#pragma unroll
    for (int j = 0; j < APW; ++j) {
      const int ins = wave + NW * j;
      const int h = ins * 16 + (lane >> 2);
      const int piece = (lane & 3) ^ swz(h);
      // rows past the halo read out of range (zeros); the instruction count per wave stays fixed
      const uint32_t voff = h < q.halo ? (uint32_t)((q.rel0 + h) * cs * (int)sizeof(T) + piece * 16) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)&dst[ins * 16 * ROWB], 16, voff, 0, 0, 0);
    }
  };
  constexpr int WAIT_ALL = 0;
  constexpr int WAIT_KEEP_A = (0xF << 8) | (7 << 4) | APW;   // vmcnt <= APW, no wait on lgkm/exp

  int tile = lb;
  if (tile < a.n_tiles) {
    const Tile t0 = ldc(a.tiles + tile);
    stage_b(0, 0, lds_b0);
    stage_a(geo_of(t0), 0, lds_a0);
    __builtin_amdgcn_s_waitcnt(WAIT_ALL);
    __syncthreads();
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

    const int next_tile = tile + G;
    // one group of three taps (tap row di = grp - 1) of chunk c; SI = position in the
    // six-group period, which fixes the arrays read and written
    auto group = [&](auto SI, int c) __attribute__((always_inline)) {
      constexpr int si = decltype(SI)::value;
      constexpr int grp = si % 3;
      unsigned char *la = (si / 3) ? lds_a1 : lds_a0;     // halo of chunk c
      unsigned char *la_next = (si / 3) ? lds_a0 : lds_a1;
      unsigned char *lbr = (si & 1) ? lds_b1 : lds_b0;     // this group's weights
      unsigned char *lb_next = (si & 1) ? lds_b0 : lds_b1;
      const bool last = c + 1 == nch && grp == 2;
      bool a_issued = false;
      if (!last) {
        stage_b(grp == 2 ? c + 1 : c, grp == 2 ? 0 : grp + 1, lb_next);
        if (grp == 0 && c + 1 < nch) { stage_a(q, c + 1, la_next); a_issued = true; }
      } else if (next_tile < a.n_tiles) {
        // prefetch the next tile's first chunk and weight group (period restarts at 0)
        const Tile tn = ldc(a.tiles + next_tile);
        stage_b(0, 0, lb_next);
        stage_a(geo_of(tn), 0, la_next);
      }
      const int di = grp - 1;
#pragma unroll 1
      for (int tj = 0; tj < 3; ++tj) {
        const int dj = tj - 1;
        const int off = di * q.rps + dj * q.U;
        v16 af[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const bool ok = tt[mb] >= 0 && (dj >= 0 || tt[mb] > 0) && (dj <= 0 || tt[mb] < 13);
          const int row = ok ? hc[mb] + off : ZROW;
          af[mb] = ld16(la + row * ROWB + ((lk ^ swz(row)) << 4));
        }
        auto load_bf = [&](int nb) {
          const int brow = (tj * 8 + nb) * 16 + lr;
          return ld16(lbr + brow * ROWB + ((lk ^ swz(brow)) << 4));
        };
        // weight fragments one n-block ahead of the MFMAs that use them; the
        // scheduling barriers keep that order
        v16 bcur = load_bf(0);
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          const v16 bnext = nb < 7 ? load_bf(nb + 1) : bcur;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mma<T>::run(af[mb], bcur, acc[mb][nb]);
          bcur = bnext;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // the next weight group must have landed; a halo load issued after it may stay in flight
      if (a_issued) __builtin_amdgcn_s_waitcnt(WAIT_KEEP_A);
      else __builtin_amdgcn_s_waitcnt(WAIT_ALL);
      dma_barrier();
    };
#pragma unroll 1
    for (int c = 0; c < nch; c += 2) {
      group(std::integral_constant<int, 0>{}, c);
      group(std::integral_constant<int, 1>{}, c);
      group(std::integral_constant<int, 2>{}, c);
      group(std::integral_constant<int, 3>{}, c + 1);
      group(std::integral_constant<int, 4>{}, c + 1);
      group(std::integral_constant<int, 5>{}, c + 1);
    }
    conv_epilogue<T, MB, EPI>(a, tl, ldc_geo(a.geo + tl.slot), acc, wave, lr, lk, lnp);
  }
  conv_ln_reduce<EPI, NW>(lnp, reinterpret_cast<float *>(lds_b0), a.ln_part, tid, wave, lr, lk);
}

// Ring variant: the same operands-in-LDS scheme with the K loop rolled and the global -> LDS
// copies issued as inline assembly (dma16), so buffer slots are chosen at run time without the
// compiler draining the DMA queue before LDS reads (conv_ring.h).  G = 1 with small slots also lets
// two 256-row workgroups share a CU, so one workgroup's epilogue overlaps the other's MFMAs.
template <typename T, int EPI, int MB, int NW, int G, int OCC, int NBUF, int SCHED, int STAG, int ALIGNED>
__global__ __launch_bounds__(64 * NW, OCC) void conv3x3_ring_kernel(ConvArgs<T> a) {
  using Sh = RingShape<MB, NW, G, NBUF, ALIGNED>;
  __shared__ __align__(16) unsigned char lds[Sh::LDS_BYTES];
  float lnp[EPI == EPI_LN_BWD ? 16 : 1];
#pragma unroll
  for (int k = 0; k < (EPI == EPI_LN_BWD ? 16 : 1); ++k) lnp[k] = 0.f;
  conv_ring_body<T, EPI, MB, NW, G, NBUF, SCHED, GridTiles, STAG, ALIGNED>(a, GridTiles(a.tiles, a.n_tiles),
                                                                           (lds_u8 *)lds, lnp);
  const int tid = threadIdx.x, lane = tid & 63;
  conv_ln_reduce<EPI, NW>(lnp, reinterpret_cast<float *>(lds + 2 * Sh::ABYTES), a.ln_part, tid, tid >> 6, lane & 15,
                          lane >> 4);
}

}  // namespace

// Compiled shapes: rows per wave (16*MB), waves per SIMD, B-operand prefetch.
// The autotuner in the host library times them per layer kind.
const ConvVariant kConvVariants[NRX_CONV_VARIANTS] = {
    {4, 1, 1},   // 256-row tiles, 1 wave/SIMD, weights prefetched one tap ahead
    {4, 2, 0},   // 256-row tiles, 2 waves/SIMD, no prefetch
    {2, 2, 1},   // 128-row tiles, 2 waves/SIMD, prefetch
    {2, 2, 0},   // 128-row tiles, 2 waves/SIMD, no prefetch
    {NRX_LDS_MB, 1, 2},   // 384-row tiles, 1 wave/SIMD, weights and halo both through LDS
    {8, 2, 2},            // 512-row tiles of 8 waves (4 m-blocks each), 2 waves/SIMD, operands through LDS
    {4, 2, 3},            // ring kernel: 256-row tiles of 4 waves, 1-tap weight slots, 2 workgroups/CU
    {8, 1, 3},            // ring kernel: 512-row tiles of 8 waves, 3-tap slots, 1 workgroup/CU
    {8, 1, 3},            // ring kernel: 512-row tiles of 8 waves, six 1-tap slots (weights 5 taps ahead)
    {8, 1, 3},            // as 7, scheduling left to the compiler
    {8, 1, 3},            // as 7, raised wave priority over the MFMA steps
    {8, 1, 3},            // as 7, workgroups started at staggered times
    {8, 1, 3},            // as 10, workgroups started at staggered times
    {8, 1, 3, 1},         // as 7 on 504-row tiles of whole subcarriers, three 3-tap weight slots
    {8, 1, 3},            // as 7, wave priority falling through each group (SIMD partners kept level)
};

template <typename T>
void launch_conv(const ConvArgs<T> &a, int epi, int variant, int grid, hipStream_t st) {
  dim3 blk(256);
#define NRX_CONV_CASE(V, MBV, OCCV, PF)                                                        \
  if (variant == V) {                                                                         \
    if (epi == EPI_STORE)                                                                     \
      hipLaunchKernelGGL((conv3x3_kernel<T, MBV, EPI_STORE, OCCV, PF>), dim3(grid), blk, 0, st, a); \
    else if (epi == EPI_LN_RELU)                                                              \
      hipLaunchKernelGGL((conv3x3_kernel<T, MBV, EPI_LN_RELU, OCCV, PF>), dim3(grid), blk, 0, st, a); \
    else if (epi == EPI_RESID)                                                                \
      hipLaunchKernelGGL((conv3x3_kernel<T, MBV, EPI_RESID, OCCV, PF>), dim3(grid), blk, 0, st, a); \
    else if (epi == EPI_LN_RELU_SAVE)                                                         \
      hipLaunchKernelGGL((conv3x3_kernel<T, MBV, EPI_LN_RELU_SAVE, OCCV, PF>), dim3(grid), blk, 0, st, a); \
    else                                                                                      \
      hipLaunchKernelGGL((conv3x3_kernel<T, MBV, EPI_LN_BWD, OCCV, PF>), dim3(grid), blk, 0, st, a); \
    return;                                                                                   \
  }
  NRX_CONV_CASE(0, 4, 1, true)
  NRX_CONV_CASE(1, 4, 2, false)
  NRX_CONV_CASE(2, 2, 2, true)
  NRX_CONV_CASE(3, 2, 2, false)
#undef NRX_CONV_CASE
#define NRX_LDS_CASE(V, M, NWV)                                                                       \
  if (variant == V) {                                                                                \
    dim3 b2(64 * NWV);                                                                               \
    if (epi == EPI_STORE) hipLaunchKernelGGL((conv3x3_lds_kernel<T, EPI_STORE, M, NWV>), dim3(grid), b2, 0, st, a); \
    else if (epi == EPI_LN_RELU)                                                                     \
      hipLaunchKernelGGL((conv3x3_lds_kernel<T, EPI_LN_RELU, M, NWV>), dim3(grid), b2, 0, st, a);    \
    else if (epi == EPI_RESID)                                                                       \
      hipLaunchKernelGGL((conv3x3_lds_kernel<T, EPI_RESID, M, NWV>), dim3(grid), b2, 0, st, a);      \
    else if (epi == EPI_LN_RELU_SAVE)                                                                \
      hipLaunchKernelGGL((conv3x3_lds_kernel<T, EPI_LN_RELU_SAVE, M, NWV>), dim3(grid), b2, 0, st, a); \
    else hipLaunchKernelGGL((conv3x3_lds_kernel<T, EPI_LN_BWD, M, NWV>), dim3(grid), b2, 0, st, a);  \
    return;                                                                                          \
  }
  NRX_LDS_CASE(4, NRX_LDS_MB, 4)
  NRX_LDS_CASE(5, 4, 8)
#undef NRX_LDS_CASE
#define NRX_RING_CASE(V, M, NWV, GV, OCCV, NBV, SCH, STG, ALG)                                            \
  if (variant == V) {                                                                                   \
    dim3 b2(64 * NWV);                                                                                  \
    if (epi == EPI_STORE)                                                                               \
      hipLaunchKernelGGL((conv3x3_ring_kernel<T, EPI_STORE, M, NWV, GV, OCCV, NBV, SCH, STG, ALG>), dim3(grid), b2, 0, st, a); \
    else if (epi == EPI_LN_RELU)                                                                        \
      hipLaunchKernelGGL((conv3x3_ring_kernel<T, EPI_LN_RELU, M, NWV, GV, OCCV, NBV, SCH, STG, ALG>), dim3(grid), b2, 0, st, a); \
    else if (epi == EPI_RESID)                                                                          \
      hipLaunchKernelGGL((conv3x3_ring_kernel<T, EPI_RESID, M, NWV, GV, OCCV, NBV, SCH, STG, ALG>), dim3(grid), b2, 0, st, a); \
    else if (epi == EPI_LN_RELU_SAVE)                                                                   \
      hipLaunchKernelGGL((conv3x3_ring_kernel<T, EPI_LN_RELU_SAVE, M, NWV, GV, OCCV, NBV, SCH, STG, ALG>), dim3(grid), b2, 0, st, a); \
    else                                                                                                \
      hipLaunchKernelGGL((conv3x3_ring_kernel<T, EPI_LN_BWD, M, NWV, GV, OCCV, NBV, SCH, STG, ALG>), dim3(grid), b2, 0, st, a); \
    return;                                                                                             \
  }
  NRX_RING_CASE(6, 4, 4, 1, 2, 2, 0, 0, 0)
  NRX_RING_CASE(7, 4, 8, 3, 1, 2, 0, 0, 0)
  NRX_RING_CASE(8, 4, 8, 1, 1, 6, 0, 0, 0)
  NRX_RING_CASE(9, 4, 8, 3, 1, 2, 1, 0, 0)
  NRX_RING_CASE(10, 4, 8, 3, 1, 2, 2, 0, 0)
  NRX_RING_CASE(11, 4, 8, 3, 1, 2, 0, 1, 0)
  NRX_RING_CASE(12, 4, 8, 3, 1, 2, 2, 1, 0)
  NRX_RING_CASE(13, 4, 8, 3, 1, 3, 0, 0, 1)
  NRX_RING_CASE(14, 4, 8, 3, 1, 2, 3, 0, 0)
#undef NRX_RING_CASE
}

template void launch_conv<float>(const ConvArgs<float> &, int, int, int, hipStream_t);
template void launch_conv<bf16_t>(const ConvArgs<bf16_t> &, int, int, int, hipStream_t);
