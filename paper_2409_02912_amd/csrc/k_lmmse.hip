// Classical judge / fallback: LMMSE equalisation and max-log Gray-QAM demapping.
//
// The paper's baseline receiver is LS channel estimation with interpolation,
// LMMSE equalisation and demapping (Sec. III-B).  Per data RE, with the channel
// estimate taken as exact and unit-energy symbols:
//   G = H^H H + N0 I (U x U), solved by an fp64 Cholesky factorisation,
//   z~ = G^-1 H^H y, d_u = 1 - N0 [G^-1]_uu, z_u = z~_u / d_u,
//   post-equaliser noise variance (1 - d_u) / d_u,
// then max-log LLRs as logits (Eq. (2), positive = bit 1) per QAM axis, since a
// Gray QAM label is the product of two Gray PAM labels (TS 38.211 5.1).
// One thread per RE; the solve is fp64, the demapper fp32.
#include "common.h"
#include "internal.h"

namespace {

struct cd { double re, im; };
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cmulc(cd a, cd b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; } // conj(a) b

// PAM level of axis label bits c[0..K-1] (unnormalised), TS 38.211 5.1 recursion
__device__ __forceinline__ float pam_level(int label, int K) {
  float v = 1.f - 2.f * ((label >> (K - 1)) & 1);
  for (int k = K - 2; k >= 0; --k) v = (1.f - 2.f * ((label >> k) & 1)) * ((float)(1 << (K - 1 - k)) - v);
  return v;
}

__device__ void axis_llr(float z, float inv_var, int K, float scale, float *out /* K values */) {
  float d0[4] = {1e30f, 1e30f, 1e30f, 1e30f}, d1[4] = {1e30f, 1e30f, 1e30f, 1e30f};
  for (int lab = 0; lab < (1 << K); ++lab) {
    float e = z - scale * pam_level(lab, K);
    float d = e * e;
    for (int k = 0; k < K; ++k) {
      if ((lab >> k) & 1) d1[k] = fminf(d1[k], d);
      else d0[k] = fminf(d0[k], d);
    }
  }
  for (int k = 0; k < K; ++k) out[k] = (d0[k] - d1[k]) * inv_var;
}

__global__ void lmmse_kernel(const SlotGeo *geo, int m_max, const float2 *y, const float2 *h, const float *n0dev,
                             float *llr, const unsigned int *slot_mask) {
  const int slot = blockIdx.y;
  if (slot_mask && !slot_mask[slot]) return;
  const SlotGeo g = geo[slot];
  const int S = g.S, U = g.U, B = g.B;
  const int re = blockIdx.x * blockDim.x + threadIdx.x;
  if (re >= S * 14) return;
  const int s = re / 14, t = re - s * 14;
  if (t == NRX_DMRS0 || t == NRX_DMRS1) {
    for (int u = 0; u < U; ++u)
      for (int j = 0; j < m_max; ++j) llr[g.llr_off + (((int64_t)u * 14 + t) * S + s) * m_max + j] = 0.f;
    return;
  }
  const double n0 = n0dev ? (double)n0dev[slot] : (double)g.n0;
  const float2 *yr = y + g.y_off + ((int64_t)s * 14 + t) * B;
  const float2 *hr = h + g.h_off + ((int64_t)s * 14 + t) * U * B;
  cd G[4][4], rhs[4];
  for (int u = 0; u < U; ++u) {
    rhs[u] = {0, 0};
    for (int v = 0; v <= u; ++v) G[u][v] = {0, 0};
  }
  for (int b = 0; b < B; ++b) {
    cd hb[4];
    for (int u = 0; u < U; ++u) { float2 q = hr[u * B + b]; hb[u] = {(double)q.x, (double)q.y}; }
    const float2 yq = yr[b];
    const cd yb = {(double)yq.x, (double)yq.y};
    for (int u = 0; u < U; ++u) {
      cd p = cmulc(hb[u], yb);
      rhs[u].re += p.re; rhs[u].im += p.im;
      for (int v = 0; v <= u; ++v) {   // G[u][v] = sum_b conj(h_u) h_v   (lower triangle)
        cd q = cmulc(hb[u], hb[v]);
        G[u][v].re += q.re; G[u][v].im += q.im;
      }
    }
  }
  // G is Hermitian: G[u][v] (u >= v) stored as conj(h_u) h_v; Cholesky needs A[u][v] = sum conj(h_u) h_v
  for (int u = 0; u < U; ++u) G[u][u].re += n0;
  // Cholesky A = L L^H, L lower with real diagonal (A[u][v] for u >= v)
  cd L[4][4];
  for (int j = 0; j < U; ++j) {
    double dsum = G[j][j].re;
    for (int k = 0; k < j; ++k) dsum -= L[j][k].re * L[j][k].re + L[j][k].im * L[j][k].im;
    const double ljj = sqrt(dsum);
    L[j][j] = {ljj, 0};
    for (int i = j + 1; i < U; ++i) {
      // A[i][j] = conj(G[i][j]) orientation: G[i][j] = sum conj(h_i) h_j; A = H^H H has A[i][j] = sum conj(h_i) h_j
      cd sum = G[i][j];
      for (int k = 0; k < j; ++k) {
        cd p = cmul(L[i][k], {L[j][k].re, -L[j][k].im});
        sum.re -= p.re; sum.im -= p.im;
      }
      L[i][j] = {sum.re / ljj, sum.im / ljj};
    }
  }
  // forward solve L w = rhs, back solve L^H z = w
  cd wv[4], z[4];
  for (int i = 0; i < U; ++i) {
    cd sum = rhs[i];
    for (int k = 0; k < i; ++k) { cd p = cmul(L[i][k], wv[k]); sum.re -= p.re; sum.im -= p.im; }
    wv[i] = {sum.re / L[i][i].re, sum.im / L[i][i].re};
  }
  for (int i = U - 1; i >= 0; --i) {
    cd sum = wv[i];
    for (int k = i + 1; k < U; ++k) { cd p = cmulc(L[k][i], z[k]); sum.re -= p.re; sum.im -= p.im; }
    z[i] = {sum.re / L[i][i].re, sum.im / L[i][i].re};
  }
  // diag of G^-1 = sum_k |(L^-1)[k][u]|^2 ; L^-1 lower triangular
  cd Li[4][4];
  for (int c = 0; c < U; ++c) {
    for (int i = 0; i < U; ++i) {
      if (i < c) { Li[i][c] = {0, 0}; continue; }
      cd sum = {i == c ? 1.0 : 0.0, 0.0};
      for (int k = c; k < i; ++k) { cd p = cmul(L[i][k], Li[k][c]); sum.re -= p.re; sum.im -= p.im; }
      Li[i][c] = {sum.re / L[i][i].re, sum.im / L[i][i].re};
    }
  }
  for (int u = 0; u < U; ++u) {
    double ginv = 0;
    for (int k = u; k < U; ++k) ginv += Li[k][u].re * Li[k][u].re + Li[k][u].im * Li[k][u].im;
    const double d = 1.0 - n0 * ginv;
    const double var = fmax((1.0 - d) / d, 1e-12);
    const float zr = (float)(z[u].re / d), zi = (float)(z[u].im / d);
    const float inv_var = (float)(1.0 / var);
    const int m = g.m[u], K = m / 2;
    const float scale = m == 2 ? 0.70710678118654752f
                        : m == 4 ? 0.31622776601683794f : m == 6 ? 0.15430334996209191f : 0.076696498884737041f;
    float lr[4], li[4];
    axis_llr(zr, inv_var, K, scale, lr);
    axis_llr(zi, inv_var, K, scale, li);
    float *dst = llr + g.llr_off + (((int64_t)u * 14 + t) * S + s) * m_max;
    for (int j = 0; j < m_max; ++j) {
      float v = 0.f;
      if (j < m) v = (j & 1) ? li[j >> 1] : lr[j >> 1];
      // fallback of a flagged slot: what LMMSE cannot produce either is an erasure
      if (slot_mask && !isfinite(v)) v = 0.f;
      dst[j] = v;
    }
  }
}

}  // namespace

void launch_lmmse(const SlotGeo *geo, const int64_t *, int n_slots, int64_t max_re, int m_max, const float2 *y,
                  const float2 *h, const float *n0dev, float *llr, hipStream_t st, const unsigned int *slot_mask) {
  dim3 grid((unsigned)((max_re + 127) / 128), n_slots);
  hipLaunchKernelGGL(lmmse_kernel, grid, dim3(128), 0, st, geo, m_max, y, h, n0dev, llr, slot_mask);
}
