// Slot generator for the per-RE MU-MIMO OFDM model of Eq. (1):
//   y[s,t] = sum_u H[s,t,u] x[s,t,u] + n[s,t],  n ~ CN(0, N0 I).
// Channel: tapped delay line, tau_l = l * spacing, exponential power-delay
// profile, sum-of-sinusoids Doppler per tap (M = 16 sinusoids, angles
// 2 pi (n + theta)/M), exponential correlation rho^|i-j| across BS antennas via
// its closed-form lower Cholesky factor.  Data: Gray QAM (TS 38.211 5.1) on the
// non-DMRS symbols in frequency-first order; DMRS type 1 on symbols 2 and 11.
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) with
// counter = (batch, slot, stream, element), key = seed; uniforms are
// (2 * (w >> 9) + 1) * 2^-24, Gaussians by Box-Muller.
#include "common.h"
#include "internal.h"

namespace {

constexpr int NSIN = 16;
constexpr float TSYM = 2192.0f / (2048.0f * 30e3f);

struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = {hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ u4 draw(const SimParams &p, int slot, int stream, uint32_t el) {
  return philox({p.batch, (uint32_t)slot, (uint32_t)stream, el}, p.key0, p.key1);
}
__device__ __forceinline__ float unif(uint32_t w) { return (float)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8f; }

__device__ __forceinline__ float2 qam(uint32_t bits, int m) {
  // axis labels: real uses bits 0,2,4,6; imaginary bits 1,3,5,7
  const int K = m / 2;
  float re = 1.f - 2.f * ((bits >> (2 * (K - 1))) & 1), im = 1.f - 2.f * ((bits >> (2 * (K - 1) + 1)) & 1);
  for (int k = K - 2; k >= 0; --k) {
    re = (1.f - 2.f * ((bits >> (2 * k)) & 1)) * ((float)(1 << (K - 1 - k)) - re);
    im = (1.f - 2.f * ((bits >> (2 * k + 1)) & 1)) * ((float)(1 << (K - 1 - k)) - im);
  }
  const float sc = m == 2 ? 0.70710678118654752f
                   : m == 4 ? 0.31622776601683794f : m == 6 ? 0.15430334996209191f : 0.076696498884737041f;
  return make_float2(sc * re, sc * im);
}

__global__ void sim_params_kernel(SimParams p, const SlotGeo *geo, int n_slots, float *fd, float *snr_db, float *n0,
                                  float *n0_ws) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  const float snr = p.snr_lo + (p.snr_hi - p.snr_lo) * unif(draw(p, slot, 4, 0).x) + geo[slot].snr_off;
  const float nv = powf(10.f, -snr / 10.f);
  if (snr_db) snr_db[slot] = snr;
  if (n0) n0[slot] = nv;
  n0_ws[slot] = nv;
  for (int u = 0; u < NRX_MAXU; ++u) fd[slot * NRX_MAXU + u] = p.doppler_max_hz * unif(draw(p, slot, 4, 1 + u).x);
}

// g[slot-offset + ((u*B + b')*L + l)*14 + t]
__global__ void sim_taps_kernel(SimParams p, const SlotGeo *geo, const int64_t *tap_off, const float *fd, float2 *g) {
  const int slot = blockIdx.y;
  const SlotGeo G = geo[slot];
  const int L = p.n_taps, B = G.B;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= G.U * B * L) return;
  const int u = idx / (L * B);
  float un[20];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    u4 w = draw(p, slot, 2, (uint32_t)(idx * 8 + k));
    un[4 * k] = unif(w.x); un[4 * k + 1] = unif(w.y); un[4 * k + 2] = unif(w.z); un[4 * k + 3] = unif(w.w);
  }
  const float theta = un[0];
  const float f = fd[slot * NRX_MAXU + u];
  float2 *dst = g + tap_off[slot] + (int64_t)idx * 14;
  for (int t = 0; t < 14; ++t) {
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int n = 0; n < NSIN; ++n) {
      const float alpha = 6.28318530717958648f * ((float)n + theta) / (float)NSIN;
      const float ph = 6.28318530717958648f * (f * cosf(alpha) * (float)t * TSYM + un[1 + n]);
      float sn, cs;
      sincosf(ph, &sn, &cs);
      re += cs; im += sn;
    }
    dst[t] = make_float2(0.25f * re, 0.25f * im);
  }
}

// spatial mixing and PDP weight: hm[((u*B + b)*L + l)*14 + t]
__global__ void sim_mix_kernel(SimParams p, const SlotGeo *geo, const int64_t *tap_off, const float2 *g, float2 *hm) {
  const int slot = blockIdx.y;
  const SlotGeo G = geo[slot];
  const int L = p.n_taps, B = G.B;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= G.U * B * L * 14) return;
  const int t = idx % 14, l = (idx / 14) % L, b = (idx / (14 * L)) % B, u = idx / (14 * L * B);
  float psum = 0.f;
  for (int k = 0; k < L; ++k) psum += expf(-(float)(k * p.tap_spacing_ns) / p.tap_decay_ns);
  const float amp = sqrtf(expf(-(float)(l * p.tap_spacing_ns) / p.tap_decay_ns) / psum);
  const float rho = p.rho, sq = sqrtf(1.f - rho * rho);
  const float2 *gs = g + tap_off[slot];
  float re = 0.f, im = 0.f;
  for (int bp = 0; bp <= b; ++bp) {
    // lower Cholesky factor of rho^|i-j|: L[b][0] = rho^b, L[b][b'] = rho^(b-b') sqrt(1-rho^2)
    const float c = (bp == 0 ? powf(rho, (float)b) : powf(rho, (float)(b - bp)) * sq);
    if (c == 0.f) continue;
    const float2 v = gs[((int64_t)((u * B + bp) * L + l)) * 14 + t];
    re += c * v.x; im += c * v.y;
  }
  hm[tap_off[slot] + idx] = make_float2(amp * re, amp * im);
}

__global__ void sim_grid_kernel(SimParams p, const SlotGeo *geo, const int64_t *tap_off, const float2 *hm,
                                const float2 *dmrs, const float *n0_ws, float2 *y, float2 *h_true) {
  const int slot = blockIdx.y;
  const SlotGeo G = geo[slot];
  const int S = G.S, U = G.U, B = G.B, L = p.n_taps;
  const int re = blockIdx.x * blockDim.x + threadIdx.x;
  if (re >= S * 14) return;
  const int s = re / 14, t = re - s * 14;
  float2 ph[32];
  for (int l = 0; l < L; ++l) {
    const int64_t idx = ((int64_t)s * l * p.scs_khz * p.tap_spacing_ns) % 1000000;
    float sn, cs;
    sincosf(-6.28318530717958648f * ((float)idx * 1e-6f), &sn, &cs);
    ph[l] = make_float2(cs, sn);
  }
  const bool is_dmrs = (t == NRX_DMRS0 || t == NRX_DMRS1);
  const int tdata = t < NRX_DMRS0 ? t : (t < NRX_DMRS1 ? t - 1 : t - 2);
  float2 x[4];
  for (int u = 0; u < U; ++u) {
    if (is_dmrs) {
      const int delta = u >> 1;
      if (((s - delta) & 1) == 0) {
        const int n = (s - delta) >> 2, kp = ((s - delta) >> 1) & 1;
        const float2 r = dmrs[G.dmrs_off + (t == NRX_DMRS1 ? S / 2 : 0) + 2 * n + kp];
        const float w = ((u & 1) && kp) ? -1.f : 1.f;
        x[u] = make_float2(w * r.x, w * r.y);
      } else {
        x[u] = make_float2(0.f, 0.f);
      }
    } else {
      const uint32_t e = (uint32_t)(tdata * S + s);
      const uint32_t w0 = draw(p, slot, 1, ((uint32_t)u << 16) | e).x;
      x[u] = qam(w0 & ((1u << G.m[u]) - 1u), G.m[u]);
    }
  }
  const float sig = sqrtf(n0_ws[slot] * 0.5f);
  const float2 *hs = hm + tap_off[slot];
  for (int b = 0; b < B; ++b) {
    float yr = 0.f, yi = 0.f;
    for (int u = 0; u < U; ++u) {
      float hr = 0.f, hi = 0.f;
      const float2 *hp = hs + ((int64_t)(u * B + b) * L) * 14 + t;
      for (int l = 0; l < L; ++l) {
        const float2 a = hp[l * 14];
        hr += a.x * ph[l].x - a.y * ph[l].y;
        hi += a.x * ph[l].y + a.y * ph[l].x;
      }
      if (h_true) h_true[G.h_off + (((int64_t)s * 14 + t) * U + u) * B + b] = make_float2(hr, hi);
      yr += hr * x[u].x - hi * x[u].y;
      yi += hr * x[u].y + hi * x[u].x;
    }
    const u4 w = draw(p, slot, 3, (uint32_t)((s * 14 + t) * B + b));
    const float r = sqrtf(-2.f * logf(unif(w.x)));
    float sn, cs;
    sincosf(6.28318530717958648f * unif(w.y), &sn, &cs);
    y[G.y_off + ((int64_t)s * 14 + t) * B + b] = make_float2(yr + sig * r * cs, yi + sig * r * sn);
  }
}

__global__ void sim_bits_kernel(SimParams p, const SlotGeo *geo, int m_max, uint8_t *bits) {
  const int slot = blockIdx.y;
  const SlotGeo G = geo[slot];
  const int nd = G.S * 12;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= G.U * nd) return;
  const int u = idx / nd, e = idx - u * nd;
  const uint32_t w0 = draw(p, slot, 1, ((uint32_t)u << 16) | (uint32_t)e).x;
  uint8_t *dst = bits + G.bits_off + (int64_t)idx * m_max;
  for (int j = 0; j < m_max; ++j) dst[j] = j < G.m[u] ? (uint8_t)((w0 >> j) & 1u) : 0;
}

}  // namespace

void launch_sim(const SimParams &p, const SlotGeo *geo, const int64_t *tap_off, int n_slots, int64_t max_re,
                int max_ubl, int m_max, const float2 *dmrs, float2 *g_raw, float2 *g_mix, float *fd_n0, float2 *y,
                float2 *h_true, uint8_t *bits, float *snr_db, float *n0, int64_t max_bits, hipStream_t st) {
  // fd_n0: per-UE Doppler [n_slots][4] followed by N0 [n_slots]
  float *fd = fd_n0, *n0_ws = fd_n0 + (int64_t)n_slots * NRX_MAXU;
  hipLaunchKernelGGL(sim_params_kernel, dim3((n_slots + 63) / 64), dim3(64), 0, st, p, geo, n_slots, fd, snr_db, n0,
                     n0_ws);
  hipLaunchKernelGGL(sim_taps_kernel, dim3((max_ubl + 63) / 64, n_slots), dim3(64), 0, st, p, geo, tap_off, fd, g_raw);
  hipLaunchKernelGGL(sim_mix_kernel, dim3((max_ubl * 14 + 255) / 256, n_slots), dim3(256), 0, st, p, geo, tap_off,
                     (const float2 *)g_raw, g_mix);
  hipLaunchKernelGGL(sim_grid_kernel, dim3((unsigned)((max_re + 127) / 128), n_slots), dim3(128), 0, st, p, geo,
                     tap_off, (const float2 *)g_mix, dmrs, (const float *)n0_ws, y, h_true);
  if (bits)
    hipLaunchKernelGGL(sim_bits_kernel, dim3((unsigned)((max_bits + 255) / 256), n_slots), dim3(256), 0, st, p, geo,
                       m_max, bits);
}
