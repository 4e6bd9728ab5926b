// Weight preparation, BCE loss and Adam.
//
// Weight preparation turns the fp32 master weights (natural layout: convolutions
// [3][3][C_in][C_out], dense [C_in][C_out]) into MFMA operand layouts in the
// compute precision, and folds the positional-encoding input channels of a
// convolution into a bias field.  The PE (distance in symbols to the nearest
// DMRS symbol, standardised over the slot; +-1 for REs off/on the UE's DMRS comb)
// depends on (s, t) only through t, the subcarrier parity relative to the UE's
// CDM group and whether s is the first or last subcarrier, so its 3x3
// convolution is a [2][3][14][C_out] table.
//
// BCE (Sec. II-B): softplus(l) - b l over the data REs of every UE's m_u bits,
// averaged; the loss is reduced in fp64, deterministically (fixed partial order).
// Adam: Kingma & Ba, bias-corrected.
#include "common.h"
#include "internal.h"

namespace {

__device__ __forceinline__ float pe_t_value(int t) {
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

template <typename T>
__global__ void prep_kernel(const float *w, const PrepJob *jobs, int n_jobs, int64_t total, T *wprep,
                            float *fields) {
  constexpr int KC = 64 / (int)sizeof(T);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int jb = 0;
  int64_t base = 0;
  while (jb < n_jobs && e >= base + jobs[jb].count) { base += jobs[jb].count; ++jb; }
  const PrepJob J = jobs[jb];
  const int64_t k = e - base;
  if (J.kind == 2) {
    // PE field [par][edge][t][o]
    const int o = k % NRX_D, t = (k / NRX_D) % 14, edge = (k / (NRX_D * 14)) % 3, par = k / (NRX_D * 42);
    float acc = 0.f;
    for (int i = 0; i < 3; ++i) {
      const int di = i - 1;
      if ((edge == 1 && di < 0) || (edge == 2 && di > 0)) continue;
      const float pf = ((par + di) & 1) ? 1.f : -1.f;
      for (int j = 0; j < 3; ++j) {
        const int tt = t + j - 1;
        if (tt < 0 || tt >= 14) continue;
        if (o >= J.d_out) continue;
        const int64_t wt = J.src + ((int64_t)(i * 3 + j) * J.cin_total + J.cin_real) * J.d_out + o;
        acc += w[wt] * pe_t_value(tt) + w[wt + J.d_out] * pf;
      }
    }
    fields[J.dst + k] = acc;
    return;
  }
  if (J.kind == 6) {
    // bias / LayerNorm vector padded with zeros to 128 channels
    fields[J.dst + k] = k < J.cin_real ? w[J.src + k] : 0.f;
    return;
  }
  const int kl = k % KC;   // channel within the K chunk (natural order)
  if (J.kind == 4) {
    // narrow dense [chunk][16][KC]: column j = output j (zero beyond n_out)
    const int j = (k / KC) % 16, chunk = k / (16 * KC);
    const int c = chunk * KC + kl;
    wprep[J.dst + k] = elem<T>::from_f(j < J.n_out && c < J.cin_real ? w[J.src + (int64_t)c * J.n_out + j] : 0.f);
    return;
  }
  const int j = (k / KC) % 16, nb = (k / (16 * KC)) % 8;
  const int n = nperm(nb, j);
  float v = 0.f;
  if (J.kind == 1) {
    const int chunk = k / (128 * KC);
    const int c = chunk * KC + kl;
    if (c < J.cin_real && n < J.d_out) v = w[J.src + (int64_t)c * J.d_out + n];
  } else if (J.kind == 5) {
    // transposed dense: B[k = c][n] = W[n][c]
    const int chunk = k / (128 * KC);
    const int c = chunk * KC + kl;
    v = w[J.src + (int64_t)n * NRX_D + c];
  } else {
    const int tap = (k / (128 * KC)) % 9, chunk = k / (1152 * KC);
    const int c = chunk * KC + kl;
    if (J.kind == 0) {
      // activation channel c -> master input channel (block convs: 128-wide segments of d channels)
      const int cm = J.seg ? (c / NRX_D) * J.seg + (c % NRX_D) : c;
      const bool in = J.seg ? (c % NRX_D) < J.seg : true;
      if (in && cm < J.cin_real && n < J.d_out) v = w[J.src + ((int64_t)tap * J.cin_total + cm) * J.d_out + n];
    } else {
      // transposed, flipped: K = original output channel c, N = original input channel cin_first + n
      v = w[J.src + ((int64_t)(8 - tap) * J.cin_total + J.cin_first + n) * NRX_D + c];
    }
  }
  wprep[J.dst + k] = elem<T>::from_f(v);
}

__global__ void bce_kernel(const SlotGeo *geo, int m_max, const float *llr, const uint8_t *bits, float *dllr,
                           double *partials, unsigned long long *perr, double inv_n) {
  const int slot = blockIdx.y;
  const SlotGeo g = geo[slot];
  const int S = g.S, U = g.U;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // (u, t, s)
  double loss = 0.0;
  unsigned long long nerr = 0;
  if (idx < U * 14 * S) {
    const int u = idx / (14 * S), t = (idx / S) % 14, s = idx % S;
    const float *l = llr + g.llr_off + (int64_t)idx * m_max;
    float *dl = dllr ? dllr + g.llr_off + (int64_t)idx * m_max : nullptr;
    const bool data = t != NRX_DMRS0 && t != NRX_DMRS1;
    const int td = t < NRX_DMRS0 ? t : (t < NRX_DMRS1 ? t - 1 : t - 2);
    const uint8_t *b = bits + g.bits_off + ((int64_t)u * S * 12 + (int64_t)td * S + s) * m_max;
    for (int j = 0; j < m_max; ++j) {
      float gr = 0.f;
      if (data && j < g.m[u]) {
        const double x = l[j];
        const double y = b[j];
        loss += fmax(x, 0.0) + log1p(exp(-fabs(x))) - y * x;
        gr = (float)((1.0 / (1.0 + exp(-x)) - y) * inv_n);
        nerr += ((x > 0.0) != (b[j] != 0));
      }
      if (dl) dl[j] = gr;
    }
  }
  // block reduction (fixed order)
  __shared__ double sl[256];
  __shared__ unsigned long long se[256];
  sl[threadIdx.x] = loss;
  se[threadIdx.x] = nerr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) { sl[threadIdx.x] += sl[threadIdx.x + w]; se[threadIdx.x] += se[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t pi = (int64_t)slot * gridDim.x + blockIdx.x;
    partials[pi] = sl[0];
    perr[pi] = se[0];
  }
}

__global__ void reduce_kernel(const double *partials, const unsigned long long *perr, int64_t n, double *loss,
                              unsigned long long *nerr, double inv_n) {
  __shared__ double sl[256];
  __shared__ unsigned long long se[256];
  double a = 0.0;
  unsigned long long c = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) { a += partials[i]; c += perr[i]; }
  sl[threadIdx.x] = a;
  se[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) { sl[threadIdx.x] += sl[threadIdx.x + w]; se[threadIdx.x] += se[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (loss) *loss = sl[0] * inv_n;
    if (nerr) *nerr = se[0];
  }
}

// Channel-estimate loss of the double readout: one thread per (s, t, u) row of the h layout, its
// B complex entries (2B floats) of the slot.
__global__ void mse_kernel(const SlotGeo *geo, const float *hest, const float *htrue, float *dhest, float gscale,
                           double *partials, unsigned long long *pzero) {
  const int slot = blockIdx.y;
  const SlotGeo g = geo[slot];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  double loss = 0.0;
  if (idx < g.S * 14 * g.U) {
    const int64_t o = (g.h_off + (int64_t)idx * g.B) * 2;
    for (int j = 0; j < 2 * g.B; ++j) {
      const double e = (double)hest[o + j] - (double)htrue[o + j];
      loss += e * e;
      if (dhest) dhest[o + j] = (float)((double)gscale * e);
    }
  }
  __shared__ double sl[256];
  sl[threadIdx.x] = loss;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sl[threadIdx.x] += sl[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t pi = (int64_t)slot * gridDim.x + blockIdx.x;
    partials[pi] = sl[0];
    pzero[pi] = 0ull;
  }
}

__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

template <typename T>
void launch_prep(const float *w, const PrepJob *jobs, int n_jobs, int64_t total, T *wprep, float *fields,
                 hipStream_t st) {
  hipLaunchKernelGGL(prep_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, w, jobs, n_jobs, total,
                     wprep, fields);
}
template void launch_prep<float>(const float *, const PrepJob *, int, int64_t, float *, float *, hipStream_t);
template void launch_prep<bf16_t>(const float *, const PrepJob *, int, int64_t, bf16_t *, float *, hipStream_t);

void launch_bce(const SlotGeo *geo, const int64_t *, int n_slots, int64_t max_ute, int m_max, const float *llr,
                const uint8_t *bits, float *dllr, double *partials, int n_part_per_slot, double *loss,
                unsigned long long *nerr, double inv_n, hipStream_t st) {
  unsigned long long *perr = reinterpret_cast<unsigned long long *>(partials + (int64_t)n_slots * n_part_per_slot);
  hipLaunchKernelGGL(bce_kernel, dim3(n_part_per_slot, n_slots), dim3(256), 0, st, geo, m_max, llr, bits, dllr,
                     partials, perr, inv_n);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, (const double *)partials,
                     (const unsigned long long *)perr, (int64_t)n_slots * n_part_per_slot, loss, nerr, inv_n);
  (void)max_ute;
}

void launch_mse(const SlotGeo *geo, int n_slots, const float *hest, const float *htrue, float *dhest, float gscale,
                double *partials, int n_part, double *loss, double inv_n, hipStream_t st) {
  unsigned long long *pz = reinterpret_cast<unsigned long long *>(partials + (int64_t)n_slots * n_part);
  hipLaunchKernelGGL(mse_kernel, dim3(n_part, n_slots), dim3(256), 0, st, geo, hest, htrue, dhest, gscale, partials,
                     pz);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, (const double *)partials,
                     (const unsigned long long *)pz, (int64_t)n_slots * n_part, loss, nullptr, inv_n);
}

void launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
}
