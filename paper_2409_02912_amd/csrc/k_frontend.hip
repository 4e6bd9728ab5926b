// Receiver front end: DMRS generation, per-UE LS estimates, linear interpolation
// and the NRX input feature rows.
//
// The NRX gets, for every UE stream, an initial LS channel estimate computed from
// the DMRS known to the BS (Sec. II-A).  DMRS: PUSCH type 1, ports 0..3 (CDM
// group u/2 on subcarriers of parity u/2, frequency OCC +-1 for odd ports), on
// symbols 2 and 11, QPSK values from the 3GPP Gold sequence (TS 38.211 5.2.1,
// 6.4.1.1).  LS: the OCC pair (k, k+2) is despread to one estimate at its centre;
// interpolation is linear across pair centres in frequency (flat beyond the
// outermost centres) and linear between the two DMRS symbols in time (flat
// outside).
#include "common.h"
#include "internal.h"

namespace {

// Gold sequence c(0 .. n-1) into a byte array; x1/x2 advance 28 bits per step.
__device__ void gold_bits(uint32_t c_init, int n, uint8_t *out) {
  uint64_t x1 = 1, x2 = c_init & 0x7FFFFFFFu;   // bits i = x(k+i), i < 31
  auto step28 = [&]() {
    uint64_t n1 = ((x1 >> 3) ^ x1) & 0xFFFFFFFull;
    uint64_t n2 = ((x2 >> 3) ^ (x2 >> 2) ^ (x2 >> 1) ^ x2) & 0xFFFFFFFull;
    x1 = ((x1 | (n1 << 31)) >> 28) & 0x7FFFFFFFull;
    x2 = ((x2 | (n2 << 31)) >> 28) & 0x7FFFFFFFull;
  };
  auto step1 = [&]() {
    uint64_t n1 = (x1 ^ (x1 >> 3)) & 1;
    uint64_t n2 = (x2 ^ (x2 >> 1) ^ (x2 >> 2) ^ (x2 >> 3)) & 1;
    x1 = (x1 >> 1) | (n1 << 30);
    x2 = (x2 >> 1) | (n2 << 30);
  };
  for (int k = 0; k < 1600 / 28; ++k) step28();      // 1596
  for (int k = 0; k < 1600 % 28; ++k) step1();       // 1600
  for (int m = 0; m < n; m += 28) {
    uint64_t c = x1 ^ x2;
    for (int i = 0; i < 28 && m + i < n; ++i) out[m + i] = (c >> i) & 1;
    step28();
  }
}

__global__ void dmrs_kernel(const SlotGeo *geo, float2 *dmrs, const unsigned int *slot_mask) {
  __shared__ uint8_t bits[2 * 275 * 12];
  const int slot = blockIdx.x, li = blockIdx.y;
  if (slot_mask && !slot_mask[slot]) return;
  const SlotGeo g = geo[slot];
  const int l = li ? NRX_DMRS1 : NRX_DMRS0;
  if (threadIdx.x == 0) {
    int64_t ci = ((int64_t)131072 * (14 * g.slot_number + l + 1) * (2 * g.n_id + 1) + 2 * g.n_id + g.n_scid) %
                 2147483648LL;
    gold_bits((uint32_t)ci, g.S, bits);
  }
  __syncthreads();
  const float a = 0.70710678118654752f;
  float2 *dst = dmrs + g.dmrs_off + (int64_t)li * (g.S / 2);
  for (int n = threadIdx.x; n < g.S / 2; n += blockDim.x)
    dst[n] = make_float2(a * (1 - 2 * (int)bits[2 * n]), a * (1 - 2 * (int)bits[2 * n + 1]));
}

// pairs layout per slot: [l(2)][u][n][b]
__global__ void ls_pairs_kernel(const SlotGeo *geo, const float2 *y, const float2 *dmrs, float2 *pairs,
                                const int64_t *pair_off, const unsigned int *slot_mask) {
  const int slot = blockIdx.y;
  if (slot_mask && !slot_mask[slot]) return;
  const SlotGeo g = geo[slot];
  const int np = g.S / 4, B = g.B, U = g.U;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * U * np * B) return;
  const int b = idx % B, n = (idx / B) % np, u = (idx / (B * np)) % U, li = idx / (B * np * U);
  const int l = li ? NRX_DMRS1 : NRX_DMRS0;
  const int delta = u >> 1;
  const float2 *r = dmrs + g.dmrs_off + (int64_t)li * (g.S / 2);
  float hr = 0.f, hi = 0.f;
#pragma unroll
  for (int kp = 0; kp < 2; ++kp) {
    const int k = 4 * n + 2 * kp + delta;
    const float w = ((u & 1) && kp == 1) ? -1.f : 1.f;
    const float2 p = r[2 * n + kp];
    const float2 v = y[g.y_off + ((int64_t)k * 14 + l) * B + b];
    // y * conj(w p)
    hr += w * (v.x * p.x + v.y * p.y);
    hi += w * (v.y * p.x - v.x * p.y);
  }
  pairs[pair_off[slot] + idx] = make_float2(0.5f * hr, 0.5f * hi);
}

template <typename T>
__global__ void features_kernel(const SlotGeo *geo, const float2 *y, const float2 *pairs, const int64_t *pair_off,
                                int model_B, int cx, T *X, float2 *h_out, const unsigned int *slot_mask,
                                unsigned int *slot_flags) {
  // one thread per (row, group of 8 input channels): the threads of a row write
  // its cx channels as adjacent 16/32-byte vectors, a wave a contiguous block
  const int slot = blockIdx.y;
  if (slot_mask && !slot_mask[slot]) return;
  const SlotGeo g = geo[slot];
  const int S = g.S, U = g.U, B = g.B;
  const int ngrp = X ? cx / 8 : 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = (int)(e / ngrp), grp = (int)(e - (int64_t)r * ngrp);   // row within the slot, channel group
  if (r >= S * 14 * U) return;   // e grows with the lane: a wave's lane 0 is in range if any lane is
  const int s = r / (14 * U);
  const int rem = r - s * 14 * U;
  const int t = rem / U, u = rem - t * U;
  const int delta = u >> 1, np = S / 4;
  int n0;
  float w;
  const int p0 = 1 + delta, plast = 4 * (np - 1) + 1 + delta;
  if (s <= p0) { n0 = 0; w = 0.f; }
  else if (s >= plast) { n0 = np - 1; w = 0.f; }
  else { n0 = (s - 1 - delta) / 4; w = (float)(s - (4 * n0 + 1 + delta)) * 0.25f; }
  const int n1 = n0 + 1 < np ? n0 + 1 : n0;
  float wt0, wt1;
  if (t <= NRX_DMRS0) { wt0 = 1.f; wt1 = 0.f; }
  else if (t >= NRX_DMRS1) { wt0 = 0.f; wt1 = 1.f; }
  else { wt0 = (float)(NRX_DMRS1 - t) / 9.f; wt1 = (float)(t - NRX_DMRS0) / 9.f; }
  const float2 *P = pairs + pair_off[slot];
  auto hval = [&](int b) {
    float2 hl[2];
#pragma unroll
    for (int li = 0; li < 2; ++li) {
      const float2 a0 = P[(((int64_t)li * U + u) * np + n0) * B + b];
      const float2 a1 = P[(((int64_t)li * U + u) * np + n1) * B + b];
      hl[li] = make_float2((1.f - w) * a0.x + w * a1.x, (1.f - w) * a0.y + w * a1.y);
    }
    return make_float2(wt0 * hl[0].x + wt1 * hl[1].x, wt0 * hl[0].y + wt1 * hl[1].y);
  };
  const float2 *yr = y + g.y_off + ((int64_t)s * 14 + t) * B;
  if (h_out && grp == 0) {
    for (int b = 0; b < B; ++b) h_out[g.h_off + (((int64_t)s * 14 + t) * U + u) * B + b] = hval(b);
  }
  if (slot_flags) {
    // health word of the slot: bit 2 when a received sample is not finite (every sample is a
    // feature of the rows of its RE; the UE-0, group-0 thread of each RE checks its B antennas)
    bool bad = false;
    if (u == 0 && grp == 0)
      for (int b = 0; b < B; ++b) bad |= !__builtin_isfinite(yr[b].x) || !__builtin_isfinite(yr[b].y);
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&slot_flags[slot], 4u);
  }
  if (X) {
    // channel order [Re y | Im y | Re h | Im h], each block model_B wide, zero padded to cx
    float f[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = 8 * grp + k, part = c / model_B, b = c - part * model_B;
      float v = 0.f;
      if (part < 4 && b < B) {
        if (part < 2) { const float2 q = yr[b]; v = part == 0 ? q.x : q.y; }
        else { const float2 q = hval(b); v = part == 2 ? q.x : q.y; }
      }
      f[k] = v;
    }
    pack8<T>::store(X + (g.row_base + r) * cx + 8 * grp, f);
  }
}

// The input features of a block of consecutive rows of one slot in two phases.  Phase 1: one thread per
// (row, antenna) interpolates the LS estimate and reads the received sample, consecutive lanes taking
// consecutive antennas, so that the loads of a row's pairs and samples are contiguous; the values go to
// LDS (and the estimate to h_out).  Phase 2: one thread per (row, 8 channels) assembles its channels from
// LDS and writes them as one 16- or 32-byte vector, a wave a contiguous block of X.
constexpr int FEAT_MAX_B = 16;
template <typename T>
__global__ __launch_bounds__(256) void features_lds_kernel(const SlotGeo *geo, const float2 *y, const float2 *pairs,
                                                           const int64_t *pair_off, int model_B, int cx, T *X,
                                                           float2 *h_out, const unsigned int *slot_mask,
                                                           unsigned int *slot_flags) {
  __shared__ float2 ys[256 / 4][FEAT_MAX_B], hs[256 / 4][FEAT_MAX_B];
  const int slot = blockIdx.y;
  if (slot_mask && !slot_mask[slot]) return;
  const SlotGeo g = geo[slot];
  const int S = g.S, U = g.U, B = g.B;
  const int ngrp = cx / 8, rpb = 256 / ngrp;   // rows per block
  const int rows = S * 14 * U;
  const int r0 = blockIdx.x * rpb;
  if (r0 >= rows) return;
  const int np = S / 4;
  const float2 *P = pairs + pair_off[slot];
  bool bad = false;
  for (int it = threadIdx.x; it < rpb * B; it += 256) {
    const int rl = it / B, b = it - rl * B, r = r0 + rl;
    if (r >= rows) break;   // it grows with rl
    const int s = r / (14 * U);
    const int rem = r - s * 14 * U;
    const int t = rem / U, u = rem - t * U;
    const int delta = u >> 1;
    const int p0 = 1 + delta, plast = 4 * (np - 1) + 1 + delta;
    int n0;
    float w;
    if (s <= p0) { n0 = 0; w = 0.f; }
    else if (s >= plast) { n0 = np - 1; w = 0.f; }
    else { n0 = (s - 1 - delta) / 4; w = (float)(s - (4 * n0 + 1 + delta)) * 0.25f; }
    const int n1 = n0 + 1 < np ? n0 + 1 : n0;
    float wt0, wt1;
    if (t <= NRX_DMRS0) { wt0 = 1.f; wt1 = 0.f; }
    else if (t >= NRX_DMRS1) { wt0 = 0.f; wt1 = 1.f; }
    else { wt0 = (float)(NRX_DMRS1 - t) / 9.f; wt1 = (float)(t - NRX_DMRS0) / 9.f; }
    float2 hl[2];
#pragma unroll
    for (int li = 0; li < 2; ++li) {
      const float2 a0 = P[(((int64_t)li * U + u) * np + n0) * B + b];
      const float2 a1 = P[(((int64_t)li * U + u) * np + n1) * B + b];
      hl[li] = make_float2((1.f - w) * a0.x + w * a1.x, (1.f - w) * a0.y + w * a1.y);
    }
    const float2 h = make_float2(wt0 * hl[0].x + wt1 * hl[1].x, wt0 * hl[0].y + wt1 * hl[1].y);
    const float2 yv = y[g.y_off + ((int64_t)s * 14 + t) * B + b];
    // health word bit 2: a received sample that is not finite (checked once per RE, by its UE-0 row)
    if (u == 0) bad |= !__builtin_isfinite(yv.x) || !__builtin_isfinite(yv.y);
    ys[rl][b] = yv;
    hs[rl][b] = h;
    if (h_out) h_out[g.h_off + (((int64_t)s * 14 + t) * U + u) * B + b] = h;
  }
  if (slot_flags && __ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&slot_flags[slot], 4u);
  __syncthreads();
  const int rl = threadIdx.x / ngrp, grp = threadIdx.x - rl * ngrp, r = r0 + rl;
  if (r >= rows) return;
  // channel order [Re y | Im y | Re h | Im h], each block model_B wide, zero padded to cx
  float f[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = 8 * grp + k, part = c / model_B, b = c - part * model_B;
    float v = 0.f;
    if (part < 4 && b < B) {
      const float2 q = part < 2 ? ys[rl][b] : hs[rl][b];
      v = (part & 1) ? q.y : q.x;
    }
    f[k] = v;
  }
  pack8<T>::store(X + (g.row_base + r) * cx + 8 * grp, f);
}

}  // namespace

void launch_dmrs(const SlotGeo *geo, int n_slots, float2 *dmrs, hipStream_t st, const unsigned int *slot_mask) {
  hipLaunchKernelGGL(dmrs_kernel, dim3(n_slots, 2), dim3(256), 0, st, geo, dmrs, slot_mask);
}

void launch_ls_pairs(const SlotGeo *geo, int n_slots, int max_pairs_total, const float2 *y, const float2 *dmrs,
                     float2 *pairs, const int64_t *pair_off, int, hipStream_t st, const unsigned int *slot_mask) {
  dim3 grid((max_pairs_total + 255) / 256, n_slots);
  hipLaunchKernelGGL(ls_pairs_kernel, grid, dim3(256), 0, st, geo, y, dmrs, pairs, pair_off, slot_mask);
}

template <typename T>
void launch_features(const SlotGeo *geo, const int64_t *, int n_slots, int64_t max_rows, const float2 *y,
                     const float2 *pairs, const int64_t *pair_off, int model_B, int cx, T *X, float2 *h_out,
                     hipStream_t st, const unsigned int *slot_mask, unsigned int *slot_flags) {
  if (X && cx / 8 >= 4 && 256 % (cx / 8) == 0 && model_B <= FEAT_MAX_B) {
    // the input features: blocks of 256 / (cx / 8) rows staged through LDS
    const int rpb = 256 / (cx / 8);
    dim3 grid((unsigned)((max_rows + rpb - 1) / rpb), n_slots);
    hipLaunchKernelGGL(features_lds_kernel<T>, grid, dim3(256), 0, st, geo, y, pairs, pair_off, model_B, cx, X, h_out,
                       slot_mask, slot_flags);
    return;
  }
  const int64_t threads = max_rows * (X ? cx / 8 : 1);   // one per (row, 8-channel group)
  dim3 grid((unsigned)((threads + 255) / 256), n_slots);
  hipLaunchKernelGGL(features_kernel<T>, grid, dim3(256), 0, st, geo, y, pairs, pair_off, model_B, cx, X, h_out,
                     slot_mask, slot_flags);
}
template void launch_features<float>(const SlotGeo *, const int64_t *, int, int64_t, const float2 *, const float2 *,
                                     const int64_t *, int, int, float *, float2 *, hipStream_t,
                                     const unsigned int *, unsigned int *);
template void launch_features<bf16_t>(const SlotGeo *, const int64_t *, int, int64_t, const float2 *,
                                      const float2 *, const int64_t *, int, int, bf16_t *, float2 *, hipStream_t,
                                      const unsigned int *, unsigned int *);
