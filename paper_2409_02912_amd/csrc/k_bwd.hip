// Backward pass of the CGNN (training, Sec. II-B): weight gradients and the
// backward of message passing and readout.  The data gradients of the 3x3
// convolutions reuse the forward kernel with flipped, transposed weights.
//
// Weight gradient of a 3x3 convolution (split-K over rows, deterministic):
//   dW[tap][c][o] = sum_rows X[neighbour(row, tap)][c] * dY[row][o]
// A workgroup owns one (row partition, tap, 128-channel input slice) and keeps
// the 128x128 block in MFMA accumulators.  Per 32-row step it stages X (shifted
// by the tap, zero outside the grid) and dY transposed into LDS, so that the
// MFMA operands (K = rows) are contiguous 16-byte fragments.  Partition results
// are summed in a fixed order by a separate kernel.
//
// Biases and the folded positional-encoding weights need column sums of dY per
// (symbol t, subcarrier parity relative to the UE's CDM group, edge class):
// the PE bias field has exactly that structure, so its weight gradient is the
// same small table contracted with those sums.
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace {

constexpr int RS = 64;                  // rows per staging step
constexpr int TP = RS + 8;              // LDS pitch (elements) of the transposed tiles

// Staging role of a thread: 4 consecutive rows (4*rg ..) x 8 consecutive channels (8*cg ..).
// Lanes of a wave vary over rg first, so the transposed 4-row LDS stores of one
// channel from 16 lanes form one contiguous 128-byte run.
template <typename T>
struct WgStage {
  float x[4][8], d[4][8];
};
// BF16: the rows as loaded (8 channels = 4 packed words each), half the registers of floats
template <>
struct WgStage<bf16_t> {
  uint32_t x[4][4], d[4][4];
};

// (the FP32 form's staged rows, twice the BF16 bytes, take most of a CU's LDS: one workgroup per CU, so
// it asks for one wave per SIMD; the BF16 form for two)
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 2 ? 2 : 1) void wgrad_kernel(WgradArgs<T> a) {
  __shared__ __align__(16) T xt[2][128 * TP];
  __shared__ __align__(16) T dt[2][128 * TP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;   // 2 x 2 wave grid over the 128 x 128 block
  constexpr int KF = mma<T>::KF;            // K rows per 16-byte fragment
  // one round of workgroups: block -> (partition, job); every block has the same amount of rows
  const int njob = a.n_taps * a.n_slices;
  const int part = blockIdx.x / njob, job = blockIdx.x % njob;
  const int tap = a.tap0 + job / a.n_slices, slice = job % a.n_slices;
  const int di = tap / 3 - 1, dj = tap % 3 - 1;
  const T *src;
  int cs, coff;
  if (slice * 128 < a.c0) { src = a.src0; cs = a.c0; coff = slice * 128; }
  else { src = a.src1; cs = a.c1; coff = slice * 128 - a.c0; }
  const int cwidth = cs - coff < 128 ? cs - coff : 128;
  const int rg = tid & 15, cg = tid >> 4;

  f32x4_t acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int t0 = (int)((int64_t)a.n_tiles * part / a.n_part);
  const int t1 = (int)((int64_t)a.n_tiles * (part + 1) / a.n_part);

  // cursor over the 64-row steps of the partition; tile geometry kept in registers
  struct Cur {
    int ti, k0, nrows, row0, U, S;
    int64_t base;
  };
  auto set_tile = [&](Cur &c, int ti) {
    c.ti = ti;
    c.k0 = 0;
    if (ti < t1) {
      const Tile tl = a.tiles[ti];
      const SlotGeo &g = a.geo[tl.slot];
      c.nrows = tl.nrows;
      c.row0 = tl.row0;
      c.U = g.U;
      c.S = g.S;
      c.base = g.row_base;
    }
  };
  auto next = [&](Cur &c) {
    c.k0 += RS;
    if (c.k0 >= c.nrows) set_tile(c, c.ti + 1);
  };
  auto load = [&](const Cur &c, WgStage<T> &stg) {
    stg = WgStage<T>{};
    if (c.ti >= t1) return;
    const int rps = 14 * c.U;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = c.k0 + 4 * rg + q;
      if (r < c.nrows) {
        const int R = c.row0 + r;
        const int s = R / rps, t = (R - s * rps) / c.U;
        const int64_t grow = c.base + R;
        const int sn = s + di, tn = t + dj;
        const bool xin = sn >= 0 && sn < c.S && tn >= 0 && tn < 14 && 8 * cg < cwidth;
        const T *xs = src + (grow + di * rps + dj * c.U) * cs + coff + 8 * cg;
        if constexpr (sizeof(T) == 2) {
          const v16 dv = ld16(a.dy + grow * NRX_D + 8 * cg);
#pragma unroll
          for (int w = 0; w < 4; ++w) stg.d[q][w] = dv.w[w];
          if (xin) {
            const v16 xv = ld16(xs);
#pragma unroll
            for (int w = 0; w < 4; ++w) stg.x[q][w] = xv.w[w];
          }
        } else {
          pack8<T>::load(a.dy + grow * NRX_D + 8 * cg, stg.d[q]);
          if (xin) pack8<T>::load(xs, stg.x[q]);
        }
      }
    }
  };
  auto store = [&](int b, const WgStage<T> &stg) {
    if constexpr (sizeof(T) == 2) {
      // channel 2w / 2w + 1 of rows (q, q + 1) from the low / high halves of word w: the 4 rows of a channel
      // are contiguous in the transposed tile, one 8-byte store per channel and array
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        uint32_t xl[2], xh[2], dl[2], dh[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          xl[p] = (stg.x[2 * p][w] & 0xFFFFu) | (stg.x[2 * p + 1][w] << 16);
          xh[p] = (stg.x[2 * p][w] >> 16) | (stg.x[2 * p + 1][w] & 0xFFFF0000u);
          dl[p] = (stg.d[2 * p][w] & 0xFFFFu) | (stg.d[2 * p + 1][w] << 16);
          dh[p] = (stg.d[2 * p][w] >> 16) | (stg.d[2 * p + 1][w] & 0xFFFF0000u);
        }
        *reinterpret_cast<uint2 *>(&xt[b][(8 * cg + 2 * w) * TP + 4 * rg]) = make_uint2(xl[0], xl[1]);
        *reinterpret_cast<uint2 *>(&xt[b][(8 * cg + 2 * w + 1) * TP + 4 * rg]) = make_uint2(xh[0], xh[1]);
        *reinterpret_cast<uint2 *>(&dt[b][(8 * cg + 2 * w) * TP + 4 * rg]) = make_uint2(dl[0], dl[1]);
        *reinterpret_cast<uint2 *>(&dt[b][(8 * cg + 2 * w + 1) * TP + 4 * rg]) = make_uint2(dh[0], dh[1]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        T *xp = &xt[b][(8 * cg + e) * TP + 4 * rg];
        T *dp = &dt[b][(8 * cg + e) * TP + 4 * rg];
#pragma unroll
        for (int q = 0; q < 4; ++q) { xp[q] = elem<T>::from_f(stg.x[q][e]); dp[q] = elem<T>::from_f(stg.d[q][e]); }
      }
    }
  };

  // pipeline: LDS buffer b holds step k; registers hold steps k+1 (stg[1-p]) and k+2 (being loaded)
  Cur c0, c1, c2;
  set_tile(c0, t0);
  if (c0.ti < t1) {
    c1 = c0;
    next(c1);
    c2 = c1;
    if (c2.ti < t1) next(c2);
    WgStage<T> s0, s1;
    load(c0, s0);
    store(0, s0);
    load(c1, s1);
    __syncthreads();
    int b = 0;
    while (c0.ti < t1) {
      load(c2, s0);                              // step k+2 in flight
#pragma unroll
      for (int f = 0; f < RS / KF; ++f) {
        v16 bfr[4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
          bfr[n] = ld16(&dt[b][((4 * wn + n) * 16 + lr) * TP + f * KF + lk * (KF / 4)]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const v16 af = ld16(&xt[b][((4 * wm + m) * 16 + lr) * TP + f * KF + lk * (KF / 4)]);
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mma<T>::run(af, bfr[n], acc[m][n]);
        }
      }
      if (c1.ti < t1) store(b ^ 1, s1);          // step k+1 into the other buffer
      __syncthreads();
      b ^= 1;
      c0 = c1;
      c1 = c2;
      if (c2.ti < t1) next(c2);
      s1 = s0;   // rotate register stages: step k+2 becomes k+1
    }
  }
  // partial [part][job][c 128][o 128]; D layout: lane holds c = 4*lk + i, o = lr (per block)
  float *dst = a.partials + ((int64_t)part * njob + job) * 128 * 128;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        dst[((4 * wm + m) * 16 + 4 * lk + i) * 128 + (4 * wn + n) * 16 + lr] = acc[m][n][i];
}

// BF16 weight gradient of a 3x3 convolution, three taps per workgroup.  A workgroup owns one (row
// partition, tap row di, 128-channel input slice) and the three taps dj = -1, 0, 1 of that row: per
// 64-row step it stages dY once (transposed) and the three dj-shifted input windows (transposed, rows
// whose neighbour lies outside the grid zero), so every staged dY row feeds three 128x128 blocks.  Eight
// waves: 4 (32 input channels) x 2 (64 output channels), each holding 3 x 2 x 4 MFMA blocks.  The
// partials go to the same [partition][tap][slice] layout as wgrad_kernel, summed by the same reduce.
constexpr int W3_WAVES = 8;

__global__ __launch_bounds__(64 * W3_WAVES, 1) void wgrad3_kernel(WgradArgs<bf16_t> a) {
  __shared__ __align__(16) bf16_t xt[2][3][128 * TP];
  __shared__ __align__(16) bf16_t dt[2][128 * TP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;   // 32 input channels x 64 output channels per wave
  constexpr int KF = mma<bf16_t>::KF;
  const int njob = 3 * a.n_slices;
  const int part = blockIdx.x / njob, job = blockIdx.x % njob;
  const int dg = job / a.n_slices, slice = job % a.n_slices;
  const int di = dg - 1;
  const bf16_t *src;
  int cs, coff;
  if (slice * 128 < a.c0) { src = a.src0; cs = a.c0; coff = slice * 128; }
  else { src = a.src1; cs = a.c1; coff = slice * 128 - a.c0; }
  const int cwidth = cs - coff < 128 ? cs - coff : 128;

  f32x4_t acc[3][2][4];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[t][m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int t0 = (int)((int64_t)a.n_tiles * part / a.n_part);
  const int t1 = (int)((int64_t)a.n_tiles * (part + 1) / a.n_part);
  struct Cur {
    int ti, k0, nrows, row0, U, S;
    int64_t base;
  };
  auto set_tile = [&](Cur &c, int ti) {
    c.ti = ti;
    c.k0 = 0;
    if (ti < t1) {
      const Tile tl = a.tiles[ti];
      const SlotGeo &g = a.geo[tl.slot];
      c.nrows = tl.nrows;
      c.row0 = tl.row0;
      c.U = g.U;
      c.S = g.S;
      c.base = g.row_base;
    }
  };
  auto next = [&](Cur &c) {
    c.k0 += RS;
    if (c.k0 >= c.nrows) set_tile(c, c.ti + 1);
  };
  // staging pairs of a thread: p = tid + 512 j; which = p / 256 (0..2: input window of tap dj = which - 1,
  // 3: dY); 4 consecutive rows (4 rg ..) x 8 consecutive channels (8 cg ..) of the step
  struct Stage {
    uint32_t v[2][4][4];
  };
  auto load = [&](const Cur &c, Stage &stg) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = tid + 512 * j, which = p >> 8, q = p & 255, rg = q & 15, cg = q >> 4;
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4)
#pragma unroll
        for (int w = 0; w < 4; ++w) stg.v[j][r4][w] = 0u;
      if (c.ti >= t1) continue;
      const int rps = 14 * c.U;
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int r = c.k0 + 4 * rg + r4;
        if (r >= c.nrows) continue;
        const int R = c.row0 + r;
        const int64_t grow = c.base + R;
        if (which == 3) {
          const v16 dv = ld16(a.dy + grow * NRX_D + 8 * cg);
#pragma unroll
          for (int w = 0; w < 4; ++w) stg.v[j][r4][w] = dv.w[w];
        } else {
          const int dj = which - 1;
          const int s = R / rps, t = (R - s * rps) / c.U;
          const int sn = s + di, tn = t + dj;
          if (sn >= 0 && sn < c.S && tn >= 0 && tn < 14 && 8 * cg < cwidth) {
            const v16 xv = ld16(src + (grow + di * rps + dj * c.U) * cs + coff + 8 * cg);
#pragma unroll
            for (int w = 0; w < 4; ++w) stg.v[j][r4][w] = xv.w[w];
          }
        }
      }
    }
  };
  auto store = [&](int b, const Stage &stg) {
    // channel 2w / 2w + 1 of rows (q, q + 1) from the low / high halves of word w: the 4 rows of a channel are
    // contiguous in the transposed tile, one 8-byte store per channel
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = tid + 512 * j, which = p >> 8, q = p & 255, rg = q & 15, cg = q >> 4;
      bf16_t *dst = which == 3 ? dt[b] : xt[b][which];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        uint32_t lo[2], hi[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          lo[h] = (stg.v[j][2 * h][w] & 0xFFFFu) | (stg.v[j][2 * h + 1][w] << 16);
          hi[h] = (stg.v[j][2 * h][w] >> 16) | (stg.v[j][2 * h + 1][w] & 0xFFFF0000u);
        }
        *reinterpret_cast<uint2 *>(&dst[(8 * cg + 2 * w) * TP + 4 * rg]) = make_uint2(lo[0], lo[1]);
        *reinterpret_cast<uint2 *>(&dst[(8 * cg + 2 * w + 1) * TP + 4 * rg]) = make_uint2(hi[0], hi[1]);
      }
    }
  };

  // pipeline: LDS buffer b holds step k; registers hold steps k+1 (s1) and k+2 (being loaded into s0)
  Cur c0, c1, c2;
  set_tile(c0, t0);
  if (c0.ti < t1) {
    c1 = c0;
    next(c1);
    c2 = c1;
    if (c2.ti < t1) next(c2);
    Stage s0, s1;
    load(c0, s0);
    store(0, s0);
    load(c1, s1);
    __syncthreads();
    int b = 0;
    while (c0.ti < t1) {
      load(c2, s0);
#pragma unroll
      for (int f = 0; f < RS / KF; ++f) {
        v16 bfr[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) bfr[n] = ld16(&dt[b][((4 * wn + n) * 16 + lr) * TP + f * KF + lk * (KF / 4)]);
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const v16 af = ld16(&xt[b][t][((2 * wm + m) * 16 + lr) * TP + f * KF + lk * (KF / 4)]);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[t][m][n] = mfma_bf16(af, bfr[n], acc[t][m][n]);
          }
      }
      if (c1.ti < t1) store(b ^ 1, s1);
      __syncthreads();
      b ^= 1;
      c0 = c1;
      c1 = c2;
      if (c2.ti < t1) next(c2);
      s1 = s0;
    }
  }
  // partials [part][tap][slice][c 128][o 128], tap = 3 (di + 1) + (dj + 1)
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    float *dst = a.partials + ((int64_t)part * 9 * a.n_slices + (3 * dg + t) * a.n_slices + slice) * 128 * 128;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[((2 * wm + m) * 16 + 4 * lk + i) * 128 + (4 * wn + n) * 16 + lr] = acc[t][m][n][i];
  }
}

// dw[layout] = sum over partitions, fixed order (added to dw when acc)
__global__ void wgrad_reduce_kernel(const float *partials, int n_part, int n_taps, int tap0, int n_slices,
                                    int cin_real, int cin_total, int conv, int64_t dst_off, float *dw, int acc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int njob = n_taps * n_slices;
  if (e >= (int64_t)njob * 128 * 128) return;
  const int o = e % 128, c = (e / 128) % 128, job = e / (128 * 128);
  const int tap = tap0 + job / n_slices, slice = job % n_slices;
  const int cg = slice * 128 + c;
  if (cg >= cin_real) return;
  double s = 0.0;
  for (int p = 0; p < n_part; ++p) s += partials[((int64_t)p * njob + job) * 128 * 128 + c * 128 + o];
  const int64_t idx = conv ? ((int64_t)tap * cin_total + cg) * 128 + o : (int64_t)cg * 128 + o;
  dw[dst_off + idx] = acc ? dw[dst_off + idx] + (float)s : (float)s;
}

// Column sums of dY per (slot, t, class = parity*3 + edge): partial[slot][t][6][128].
template <typename T>
__global__ __launch_bounds__(256) void colsum_kernel(const T *dy, const SlotGeo *geo, float *partial) {
  __shared__ float red[16][6 * 128];
  const int slot = blockIdx.x, t = blockIdx.y;
  const SlotGeo g = geo[slot];
  const int cg = threadIdx.x & 15, rl = threadIdx.x >> 4;   // 8-channel group, row lane
  float acc[6][8];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[c][k] = 0.f;
  const int n = g.S * g.U;
  for (int q = rl; q < n; q += 16) {
    const int s = q / g.U, u = q - s * g.U;
    const int par = (s - (u >> 1)) & 1;
    const int edge = s == 0 ? 1 : (s == g.S - 1 ? 2 : 0);
    const int cls = par * 3 + edge;
    float v[8];
    pack8<T>::load(dy + (g.row_base + ((int64_t)s * 14 + t) * g.U + u) * NRX_D + 8 * cg, v);
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (c == cls)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[c][k] += v[k];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int k = 0; k < 8; ++k) red[rl][c * 128 + 8 * cg + k] = acc[c][k];
  __syncthreads();
  for (int e = threadIdx.x; e < 6 * 128; e += 256) {
    float sum = 0.f;
    for (int k = 0; k < 16; ++k) sum += red[k][e];
    partial[((int64_t)slot * 14 + t) * 6 * 128 + e] = sum;
  }
}

__device__ __forceinline__ float pe_t_val(int t) {
  // standardised distance (in symbols) to the nearest DMRS symbol; statistics over the 14 symbols
  auto dist = [](int k) {
    int x = k - NRX_DMRS0, y = k - NRX_DMRS1;
    x = x < 0 ? -x : x;
    y = y < 0 ? -y : y;
    return (float)(x < y ? x : y);
  };
  float mean = 0.f, var = 0.f;
#pragma unroll
  for (int k = 0; k < 14; ++k) mean += dist(k);
  mean *= (1.f / 14.f);
#pragma unroll
  for (int k = 0; k < 14; ++k) var += (dist(k) - mean) * (dist(k) - mean);
  return (dist(t) - mean) / sqrtf(var * (1.f / 14.f));
}

// Sum of the per-slot class column sums over slots (fixed order): red[t][768].
__global__ void colsum_reduce_kernel(const float *partial, int n_slots, float *red) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;   // t * 768 + class * 128 + o
  if (e >= 14 * 768) return;
  const int t = e / 768, k = e % 768;
  double s = 0.0;
  for (int sl = 0; sl < n_slots; ++sl) s += partial[((int64_t)sl * 14 + t) * 768 + k];
  red[e] = (float)s;
}

// Bias gradient (sum of all classes; block 9) and, for layers with a folded PE,
// the PE weight gradients of tap blockIdx.x (blocks 0..8).  Thread = output channel.
__global__ void bias_pe_kernel(const float *red, int64_t bias_off, int64_t pe_w_off, int cin_total, int pe_ch,
                               float *dw, int acc) {
  const int o = threadIdx.x, tap = blockIdx.x;
  if (tap == 9) {
    double b = 0.0;
    for (int k = 0; k < 14 * 6; ++k) b += red[k * 128 + o];
    dw[bias_off + o] = acc ? dw[bias_off + o] + (float)b : (float)b;
    return;
  }
  if (pe_w_off < 0) return;
  const int di = tap / 3 - 1, dj = tap % 3 - 1;
  double gt = 0.0, gf = 0.0;
  for (int t = 0; t < 14; ++t) {
    const int tt = t + dj;
    if (tt < 0 || tt >= 14) continue;
    const float pt = pe_t_val(tt);
    for (int par = 0; par < 2; ++par) {
      const float pf = ((par + di) & 1) ? 1.f : -1.f;
      for (int edge = 0; edge < 3; ++edge) {
        if ((edge == 1 && di < 0) || (edge == 2 && di > 0)) continue;
        const double v = red[t * 768 + (par * 3 + edge) * 128 + o];
        gt += v * pt;
        gf += v * pf;
      }
    }
  }
  const int64_t w = pe_w_off + ((int64_t)tap * cin_total + pe_ch) * 128 + o;
  dw[w] = (float)gt;
  dw[w + 128] = (float)gf;
}

// LayerNorm parameter gradients from per-workgroup partials [n][256].
__global__ void ln_reduce_kernel(const float *part, int n, int64_t g_off, int64_t b_off, float *dw) {
  const int c = threadIdx.x;   // 0..255
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += part[(int64_t)k * 256 + c];
  if (c < 128) dw[g_off + c] = (float)s;
  else dw[b_off + c - 128] = (float)s;
}

// --------------------------------------------------------------- MP / readout

template <typename T>
struct OpTileB {
  static constexpr int PITCHB = NRX_D * (int)sizeof(T) + 16;
};

// acc += A x W (128-deep K); A fragments from LDS tile rows, W prepped dense.
template <typename T>
__device__ __forceinline__ void gemm_lds(f32x4_t (&acc)[2][8], const unsigned char *lds, int wave, const T *w,
                                         int lr, int lk) {
  constexpr int KC = 64 / (int)sizeof(T);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 8; ++n) acc[m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const T *wl = w + lr * KC + lk * (KC / 4);
#pragma unroll 2
  for (int c = 0; c < NRX_D / KC; ++c) {
    v16 bf[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) bf[n] = ld16(wl + (size_t)(c * 8 + n) * 16 * KC);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const v16 af = ld16(lds + (wave * 32 + m * 16 + lr) * OpTileB<T>::PITCHB + c * 64 + lk * 16);
#pragma unroll
      for (int n = 0; n < 8; ++n) acc[m][n] = mma<T>::run(af, bf[n], acc[m][n]);
    }
  }
}

// MP backward for one round.  In: dagg (dL/dagg), m1 (saved hidden), h.
// dmsg_v = sum_{u != v} dagg_u; dm1 = (dmsg W2^T) [m1 > 0]; dh += dm1 W1^T.
// Writes dmsg and dm1 (for the weight gradients) and updates dh in place.
template <typename T>
__global__ __launch_bounds__(256) void mp_bwd_kernel(MpBwdArgs<T> a) {
  constexpr int PB = OpTileB<T>::PITCHB;
  constexpr int MSG_PITCH = NRX_D + 4;
  __shared__ __align__(16) unsigned char lds[128 * MSG_PITCH * 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4, ch0 = 8 * lr;
  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const Tile tl = a.tiles[tile];
    const SlotGeo g = a.geo[tl.slot];
    const int64_t gbase = g.row_base + tl.row0;
    const int U = g.U;
    __syncthreads();
    // stage dagg (fp32) to LDS
    float *dg = reinterpret_cast<float *>(lds);
    for (int e = tid; e < tl.nrows * 16; e += 256) {
      const int r = e >> 4, c8 = (e & 15) * 8;
      float v[8];
      pack8<T>::load(a.dagg + (gbase + r) * NRX_D + c8, v);
#pragma unroll
      for (int k = 0; k < 8; ++k) dg[r * MSG_PITCH + c8 + k] = v[k];
    }
    __syncthreads();
    // dmsg for every row (each thread: one row, 8 channels), kept in registers
    float dm[8][8];
    int rows_of[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      rows_of[q] = -1;
      if (e < tl.nrows * 16) {
        const int r = e >> 4, c8 = (e & 15) * 8;
        const int u = r % U, re0 = r - u;
#pragma unroll
        for (int k = 0; k < 8; ++k) dm[q][k] = 0.f;
        for (int o = 0; o < U; ++o) {
          if (o == u) continue;
#pragma unroll
          for (int k = 0; k < 8; ++k) dm[q][k] += dg[(re0 + o) * MSG_PITCH + c8 + k];
        }
        rows_of[q] = e;
      }
    }
    __syncthreads();
    // dmsg -> global (weight gradient input) and LDS (operand layout for dmsg W2^T)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = rows_of[q];
      if (e >= 0) {
        const int r = e >> 4, c8 = (e & 15) * 8;
        pack8<T>::store(a.dmsg + (gbase + r) * NRX_D + c8, dm[q]);
        pack8<T>::store(reinterpret_cast<T *>(lds + r * PB) + c8, dm[q]);
      }
    }
    // zero rows past the tile so the MFMA reads defined values
    for (int e = tid; e < (128 - tl.nrows) * 16; e += 256) {
      const int r = tl.nrows + (e >> 4), c8 = (e & 15) * 8;
      float z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      pack8<T>::store(reinterpret_cast<T *>(lds + r * PB) + c8, z);
    }
    __syncthreads();
    f32x4_t acc[2][8];
    gemm_lds<T>(acc, lds, wave, a.w2t, lr, lk);
    __syncthreads();
    // dm1 = acc [m1 > 0] -> global + LDS
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 32 + m * 16 + 4 * lk + i;
        const bool valid = r < tl.nrows;
        float mv[8], v[8];
        if (valid) pack8<T>::load(a.m1 + (gbase + r) * NRX_D + ch0, mv);
#pragma unroll
        for (int n = 0; n < 8; ++n) v[n] = (valid && mv[n] > 0.f) ? acc[m][n][i] : 0.f;
        if (sizeof(T) == 2) {
#pragma unroll
          for (int n = 0; n < 8; ++n) v[n] = bf2f(f2bf(v[n]));
        }
        if (valid) pack8<T>::store(a.dm1 + (gbase + r) * NRX_D + ch0, v);
        pack8<T>::store(reinterpret_cast<T *>(lds + r * PB) + ch0, v);
      }
    __syncthreads();
    gemm_lds<T>(acc, lds, wave, a.w1t, lr, lk);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 32 + m * 16 + 4 * lk + i;
        if (r < tl.nrows) {
          float hv[8];
          pack8<T>::load(a.dh + (gbase + r) * NRX_D + ch0, hv);
#pragma unroll
          for (int n = 0; n < 8; ++n) hv[n] += acc[m][n][i];
          pack8<T>::store(a.dh + (gbase + r) * NRX_D + ch0, hv);
        }
      }
  }
}

// Readout backward.  dl (llr layout, masked to j < m_u) -> dr = (dl W2^T) [q > 0],
// dh = dr W1^T.  Per-workgroup partials of dW2 = q^T dl and db2 = sum dl.  One call handles the
// 8 output columns j0 .. j0 + 7; ReadoutChEst (up to 16 outputs, the gradient in the h layout)
// takes two calls, the second adding its hidden gradient to dr.
template <typename T>
__global__ __launch_bounds__(256) void readout_bwd_kernel(RoBwdArgs<T> a) {
  constexpr int PB = OpTileB<T>::PITCHB;
  __shared__ __align__(16) unsigned char lds[128 * PB];
  __shared__ float red[4][8 * 128 + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4, ch0 = 8 * lr;
  const int M = a.m_max, J0 = a.j0;
  const int NO = a.n_out ? a.n_out : M;   // columns of w2
  float w2[8][8];
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int j = 0; j < 8; ++j) w2[n][j] = J0 + j < NO ? a.w2[(ch0 + n) * NO + J0 + j] : 0.f;
  float pw[8][8], pb[8];   // this lane's dW2 rows (its 8 channels) and db2
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    pb[n] = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) pw[n][j] = 0.f;
  }
  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const Tile tl = a.tiles[tile];
    const SlotGeo g = a.geo[tl.slot];
    const int64_t gbase = g.row_base + tl.row0;
    const int U = g.U, S = g.S;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 32 + m * 16 + 4 * lk + i;
        const bool valid = r < tl.nrows;
        float dl[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) dl[j] = 0.f;
        float qv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (valid) {
          const int R = tl.row0 + r;
          const int s = R / (14 * U);
          const int rem = R - s * 14 * U;
          const int t = rem / U, u = rem - t * U;
          if (a.chest) {
            // h layout: row R is entry R of the slot, 2B floats
            const float *src = a.dllr + (g.h_off + (int64_t)R * g.B) * 2;
#pragma unroll
            for (int j = 0; j < 8; ++j) dl[j] = J0 + j < 2 * g.B ? src[J0 + j] : 0.f;
          } else {
            const int mu = a.geo[tl.slot].m[u];
            const int mv = (!a.only_m || mu == a.only_m) ? mu : 0;   // Var-IO: other modulations' rows
            const float *src = a.dllr + g.llr_off + (((int64_t)u * 14 + t) * S + s) * M;
#pragma unroll
            for (int j = 0; j < 8; ++j) dl[j] = (J0 + j < M && J0 + j < mv) ? src[J0 + j] : 0.f;
          }
          pack8<T>::load(a.q + (gbase + r) * NRX_D + ch0, qv);
        }
        float dr[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) {
          float x = 0.f;
#pragma unroll
          for (int j = 0; j < 8; ++j) x += dl[j] * w2[n][j];
          dr[n] = qv[n] > 0.f ? x : 0.f;
#pragma unroll
          for (int j = 0; j < 8; ++j) pw[n][j] += qv[n] * dl[j];
        }
        if (lr == 0) {
#pragma unroll
          for (int j = 0; j < 8; ++j) pb[j] += dl[j];
        }
        if (sizeof(T) == 2) {
#pragma unroll
          for (int n = 0; n < 8; ++n) dr[n] = bf2f(f2bf(dr[n]));
        }
        if (valid) {
          if (a.acc_dr) {
            float o[8], v[8];
            pack8<T>::load(a.dr + (gbase + r) * NRX_D + ch0, o);
#pragma unroll
            for (int n = 0; n < 8; ++n) v[n] = o[n] + dr[n];
            pack8<T>::store(a.dr + (gbase + r) * NRX_D + ch0, v);
          } else {
            pack8<T>::store(a.dr + (gbase + r) * NRX_D + ch0, dr);
          }
        }
        pack8<T>::store(reinterpret_cast<T *>(lds + r * PB) + ch0, dr);
      }
    __syncthreads();
    f32x4_t acc[2][8];
    gemm_lds<T>(acc, lds, wave, a.w1t, lr, lk);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 32 + m * 16 + 4 * lk + i;
        if (r < tl.nrows) {
          float v[8];
#pragma unroll
          for (int n = 0; n < 8; ++n) v[n] = acc[m][n][i];
          if (a.accumulate) {
            float o[8];
            pack8<T>::load(a.dh + (gbase + r) * NRX_D + ch0, o);
#pragma unroll
            for (int n = 0; n < 8; ++n) v[n] += o[n];
          }
          pack8<T>::store(a.dh + (gbase + r) * NRX_D + ch0, v);
        }
      }
  }
  // reduce dW2 / db2 over the 4 row groups, then the 4 waves
#pragma unroll
  for (int n = 0; n < 8; ++n) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      pw[n][j] += __shfl_xor(pw[n][j], 16, 64);
      pw[n][j] += __shfl_xor(pw[n][j], 32, 64);
    }
    pb[n] += __shfl_xor(pb[n], 16, 64);
    pb[n] += __shfl_xor(pb[n], 32, 64);
  }
  if (lk == 0) {
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[wave][(ch0 + n) * 8 + j] = pw[n][j];
    if (lr == 0)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[wave][1024 + j] = pb[j];
  }
  __syncthreads();
  for (int e = tid; e < 1032; e += 256)
    a.part[(int64_t)blockIdx.x * 1032 + e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
}

// One thread per 8 channels (16 or 32 bytes) of a row; grid (row blocks, slots).
template <typename T>
__global__ void select_rows_kernel(const T *src, const SlotGeo *geo, int only_m, T *dst) {
  const SlotGeo g = geo[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = idx >> 4;
  if (row >= (int64_t)g.S * 14 * g.U) return;
  const int ch0 = 8 * (int)(idx & 15);
  const int64_t o = (g.row_base + row) * NRX_D + ch0;
  float v[8];
  pack8<T>::load(src + o, v);
  if (g.m[row % g.U] != only_m) {
#pragma unroll
    for (int n = 0; n < 8; ++n) v[n] = 0.f;
  }
  pack8<T>::store(dst + o, v);
}

__global__ void readout_w2_reduce_kernel(const float *part, int n, int m_max, int64_t w2_off, int64_t b2_off,
                                         float *dw, int j0) {
  const int e = threadIdx.x + blockIdx.x * blockDim.x;   // 0..1031
  if (e >= 1032) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += part[(int64_t)k * 1032 + e];
  if (e < 1024) {
    const int c = e / 8, j = j0 + e % 8;
    if (j < m_max) dw[w2_off + c * m_max + j] = (float)s;
  } else if (j0 + e - 1024 < m_max) {
    dw[b2_off + j0 + e - 1024] = (float)s;
  }
}

}  // namespace

template <typename T>
void launch_wgrad(const WgradArgs<T> &a, hipStream_t st) {
  if constexpr (std::is_same<T, bf16_t>::value) {
    if (a.n_taps == 9) {   // 3x3 convolutions: three taps per workgroup
      hipLaunchKernelGGL(wgrad3_kernel, dim3(a.n_part * 3 * a.n_slices), dim3(64 * W3_WAVES), 0, st, a);
      return;
    }
  }
  const int grid = a.n_part * a.n_taps * a.n_slices;
  hipLaunchKernelGGL(wgrad_kernel<T>, dim3(grid), dim3(256), 0, st, a);
}
int wgrad_jobs_per_partition(int n_taps, int n_slices, bool bf16) {
  return (bf16 && n_taps == 9) ? 3 * n_slices : n_taps * n_slices;
}
void launch_wgrad_reduce(const float *partials, int n_part, int n_taps, int tap0, int n_slices, int cin_real,
                         int cin_total, int conv, int64_t dst_off, float *dw, hipStream_t st, bool acc) {
  const int64_t n = (int64_t)n_taps * n_slices * 128 * 128;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partials, n_part,
                     n_taps, tap0, n_slices, cin_real, cin_total, conv, dst_off, dw, acc ? 1 : 0);
}
template <typename T>
void launch_colsum(const T *dy, const SlotGeo *geo, int n_slots, float *partial, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel<T>, dim3(n_slots, 14), dim3(256), 0, st, dy, geo, partial);
}
void launch_bias_pe(const float *partial, int n_slots, int64_t bias_off, int64_t pe_w_off, int cin_total, int pe_ch,
                    float *dw, hipStream_t st, bool acc) {
  // the reduced table lives right after the per-slot partials
  float *red = const_cast<float *>(partial) + (int64_t)n_slots * 14 * 768;
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((14 * 768 + 255) / 256), dim3(256), 0, st, partial, n_slots, red);
  hipLaunchKernelGGL(bias_pe_kernel, dim3(10), dim3(128), 0, st, (const float *)red, bias_off, pe_w_off, cin_total,
                     pe_ch, dw, acc ? 1 : 0);
}
void launch_ln_reduce(const float *part, int n, int64_t g_off, int64_t b_off, float *dw, hipStream_t st) {
  hipLaunchKernelGGL(ln_reduce_kernel, dim3(1), dim3(256), 0, st, part, n, g_off, b_off, dw);
}
template <typename T>
void launch_mp_bwd(const MpBwdArgs<T> &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(mp_bwd_kernel<T>, dim3(grid), dim3(256), 0, st, a);
}
template <typename T>
void launch_select_rows(const T *src, const SlotGeo *geo, int n_slots, int64_t max_rows, int only_m, T *dst,
                        hipStream_t st) {
  const unsigned nb = (unsigned)((max_rows * 16 + 255) / 256);
  hipLaunchKernelGGL(select_rows_kernel<T>, dim3(nb, n_slots), dim3(256), 0, st, src, geo, only_m, dst);
}
template void launch_select_rows<float>(const float *, const SlotGeo *, int, int64_t, int, float *, hipStream_t);
template void launch_select_rows<bf16_t>(const bf16_t *, const SlotGeo *, int, int64_t, int, bf16_t *, hipStream_t);

template <typename T>
void launch_readout_bwd(const RoBwdArgs<T> &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(readout_bwd_kernel<T>, dim3(grid), dim3(256), 0, st, a);
}
void launch_readout_w2_reduce(const float *part, int n, int m_max, int64_t w2_off, int64_t b2_off, float *dw,
                              hipStream_t st, int j0) {
  hipLaunchKernelGGL(readout_w2_reduce_kernel, dim3(5), dim3(256), 0, st, part, n, m_max, w2_off, b2_off, dw, j0);
}

template void launch_wgrad<float>(const WgradArgs<float> &, hipStream_t);
template void launch_wgrad<bf16_t>(const WgradArgs<bf16_t> &, hipStream_t);
template void launch_colsum<float>(const float *, const SlotGeo *, int, float *, hipStream_t);
template void launch_colsum<bf16_t>(const bf16_t *, const SlotGeo *, int, float *, hipStream_t);
template void launch_mp_bwd<float>(const MpBwdArgs<float> &, int, hipStream_t);
template void launch_mp_bwd<bf16_t>(const MpBwdArgs<bf16_t> &, int, hipStream_t);
template void launch_readout_bwd<float>(const RoBwdArgs<float> &, int, hipStream_t);
template void launch_readout_bwd<bf16_t>(const RoBwdArgs<bf16_t> &, int, hipStream_t);
