// Device pieces shared by the convolution kernels: halo sizing, the fused
// epilogue (bias + positional-encoding field, LayerNorm + ReLU, residual add,
// LayerNorm backward) and the LayerNorm-backward partial-sum reduction.
#pragma once
#include "common.h"
#include "internal.h"

namespace {

constexpr int ROWB = 64;   // bytes per LDS row (one 64-byte K chunk of one activation row)

__host__ __device__ constexpr int halo_rows_max(int tile_rows) {
  int best = 0;
  for (int U = 1; U <= 4; ++U) {
    int v = ((tile_rows - 1) / (14 * U) + 4) * 14 * U;
    best = v > best ? v : best;
  }
  return (best + 15) / 16 * 16;
}

typedef __attribute__((address_space(3))) void lds_void;

// Load through the constant address space: with a uniform address this becomes a
// scalar load, which is not ordered behind outstanding vector-memory (DMA) work.
template <typename X>
__device__ __forceinline__ X ldc(const X *p) {
  return *(const __attribute__((address_space(4))) X *)p;
}
typedef int i32x4_t __attribute__((ext_vector_type(4)));

// Buffer descriptor words of a wave-uniform base address and size (raw buffer,
// no stride; reads past nbytes return zero).
__device__ __forceinline__ i32x4_t rsrc_words(const void *base, int nbytes) {
  const uint64_t b = (uint64_t)base;
  i32x4_t r;
  r.x = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  r.y = __builtin_amdgcn_readfirstlane((int)((b >> 32) & 0xFFFF));
  r.z = __builtin_amdgcn_readfirstlane(nbytes);
  r.w = 0x00020000;
  return r;
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const lds_void *)p);
}

// LDS bytes addressed in the local address space: bodies that receive their LDS region as a pointer
// use these, so no generic-to-local pointer conversion is left for the compiler to check at run time.
typedef __attribute__((address_space(3))) unsigned char lds_u8;
__device__ __forceinline__ uint32_t lds_addr(const lds_u8 *p) {
  return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)p);
}
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v16 ld16(const lds_u8 *p) {
  const u32x4_t x = *(const __attribute__((address_space(3))) u32x4_t *)p;
  return v16{{x.x, x.y, x.z, x.w}};
}
__device__ __forceinline__ void st16(lds_u8 *p, v16 v) {
  *(__attribute__((address_space(3))) u32x4_t *)p = u32x4_t{v.w[0], v.w[1], v.w[2], v.w[3]};
}
using ::ld16;   // the generic-pointer forms stay visible beside these
using ::st16;

// Global -> LDS copy of 16 bytes per lane (lane i writes lds + 16 i) through the
// buffer unit.  Written as inline assembly so that the compiler's wait-count pass
// does not tie later LDS reads of other buffers to it; the kernels order it
// explicitly (s_waitcnt vmcnt and a barrier before the data is read).  M0 holds
// the LDS address; these kernels use M0 for nothing else, and the s_nop covers
// the M0-write to LDS-DMA hazard.
__device__ __forceinline__ void dma16(const i32x4_t &rsrc, uint32_t lds, uint32_t voff) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
               :
               : "s"(lds), "v"(voff), "s"(rsrc)
               : "memory");
}

// The lane id, recomputed where it is used: the empty volatile assembly hides the value, so
// offsets derived from it are computed in place instead of being hoisted out of the K loop
// and held (or spilled) in registers across it.
__device__ __forceinline__ int lane_here() {
  int l = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  asm volatile("" : "+v"(l));
  return l;
}

// Workgroup barrier for the DMA-pipelined kernels.  __syncthreads() carries a
// workgroup release fence, which drains every outstanding vector-memory operation,
// including the LDS DMA deliberately left in flight across the barrier.  Here each
// wave first waits for exactly the DMA it needs (s_waitcnt issued by the caller),
// all LDS reads before the barrier have been consumed by MFMAs, and the signal
// fences stop the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void dma_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// the fields of a slot's geometry the convolutions use (S, U, row_base), by scalar loads
__device__ __forceinline__ SlotGeo ldc_geo(const SlotGeo *p) {
  SlotGeo g{};
  g.S = ldc(&p->S);
  g.U = ldc(&p->U);
  g.row_base = ldc(&p->row_base);
  return g;
}
// a tile descriptor as one 16-byte scalar load (three used fields would make a
// 12-byte load, which has no scalar form)
__device__ __forceinline__ Tile ldc(const Tile *p) {
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x4 v = *(const __attribute__((address_space(4))) i32x4 *)p;
  return Tile{v.x, v.y, v.z, v.w};
}

// Buffer resource of a wave-uniform base address and size, built from scalar
// registers (a descriptor the compiler cannot prove uniform is used through a
// per-lane loop).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void *base, int nbytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), 0,
                                           __builtin_amdgcn_readfirstlane(nbytes), 0x00020000);
}

// Epilogue of one tile: bias (+ PE field) -> store | LayerNorm + ReLU | residual
// add | LayerNorm backward.  Lane owns channels 8*lr .. +7 of rows 4*lk + i.
template <typename T, int MB, int EPI, int LB = (MB % 2 == 0 ? 2 : 1)>
__device__ __forceinline__ void conv_epilogue(const ConvArgs<T> &a, const Tile &tl, const SlotGeo &g,
                                              f32x4_t (&acc)[MB][8], int wave, int lr, int lk, float *lnp) {
  const int U = g.U, S = g.S, rps = 14 * U;
  const int ch0 = 8 * lr;          // this lane's 8 consecutive output channels
  if constexpr (EPI == EPI_LN_BWD) {
    // acc = dL/da with a = ReLU(LN(z)); resid holds a, save_z holds z, save_stats (mean, rstd).
    // dz = rstd (dzhat - mean(dzhat) - zhat mean(dzhat zhat)), dzhat = g * dn, dn = da [a > 0]
    float gam[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) gam[nb] = a.ln_g[ch0 + nb];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 16 * MB + mb * 16 + 4 * lk + i;
        const bool valid = r < tl.nrows;
        const int64_t grow = g.row_base + tl.row0 + (valid ? r : 0);
        float av[8], zv[8];
        pack8<T>::load(a.resid + grow * NRX_D + ch0, av);
        pack8<T>::load(a.save_z + grow * NRX_D + ch0, zv);
        const float mean = a.save_stats[2 * grow], rstd = a.save_stats[2 * grow + 1];
        float dn[8], zh[8], dzh[8], s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          dn[nb] = (valid && av[nb] > 0.f) ? acc[mb][nb][i] : 0.f;
          zh[nb] = (zv[nb] - mean) * rstd;
          dzh[nb] = dn[nb] * gam[nb];
          s1 += dzh[nb];
          s2 += dzh[nb] * zh[nb];
          lnp[nb] += dn[nb] * zh[nb];
          lnp[8 + nb] += dn[nb];
        }
        s1 = row_sum16(s1) * (1.0f / NRX_D);
        s2 = row_sum16(s2) * (1.0f / NRX_D);
        float dz[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) dz[nb] = rstd * (dzh[nb] - s1 - zh[nb] * s2);
        if (valid) pack8<T>::store(a.out + grow * NRX_D + ch0, dz);
      }
    }
    return;
  }
  constexpr bool LN = EPI == EPI_LN_RELU || EPI == EPI_LN_RELU_SAVE;
  float bias[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) bias[nb] = a.bias[ch0 + nb];

  // PE field: its row is fixed by (subcarrier class, symbol), found with float
  // reciprocals (quotients below 2^12 with at least 0.5/rps to the next integer, far
  // above the rounding error); rows past the tile use row 0.  Loads go out two
  // m-blocks at a time before any is used.
  if (EPI != EPI_RESID && a.pe) {   // (the residual convolutions carry no PE field)
    const float inv_rps = 1.0f / (float)rps, inv_u = 1.0f / (float)U;
    constexpr int PB = 1;
#pragma unroll
    for (int mb0 = 0; mb0 < MB; mb0 += PB) {
      float pev[PB][4][8];
#pragma unroll
      for (int q = 0; q < PB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = wave * 16 * MB + (mb0 + q) * 16 + 4 * lk + i;
          const int R = tl.row0 + (r < tl.nrows ? r : 0);
          const int s = (int)(((float)R + 0.5f) * inv_rps);
          const int rem = R - s * rps;
          const int t = (int)(((float)rem + 0.5f) * inv_u);
          const int u = rem - t * U;
          const int par = (s - (u >> 1)) & 1;
          const int edge = s == 0 ? 1 : (s == S - 1 ? 2 : 0);
          const float4 *pf = reinterpret_cast<const float4 *>(a.pe + ((size_t)((par * 3 + edge) * 14 + t)) * NRX_D + ch0);
          const float4 x0 = pf[0], x1 = pf[1];
          pev[q][i][0] = x0.x; pev[q][i][1] = x0.y; pev[q][i][2] = x0.z; pev[q][i][3] = x0.w;
          pev[q][i][4] = x1.x; pev[q][i][5] = x1.y; pev[q][i][6] = x1.z; pev[q][i][7] = x1.w;
        }
#pragma unroll
      for (int q = 0; q < PB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) acc[mb0 + q][nb][i] += pev[q][i][nb];
    }
  }

  if constexpr (LN) {
    float lng[8], lnb[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) { lng[nb] = a.ln_g[ch0 + nb]; lnb[nb] = a.ln_b[ch0 + nb]; }
    // statistics of LB m-blocks (4 LB rows) together: every butterfly step of the row
    // sums runs over all of them before the next, so the steps do not wait on each other
#pragma unroll
    for (int mb0 = 0; mb0 < MB; mb0 += LB) {
      float mean[LB * 4], rstd[LB * 4];
#pragma unroll
      for (int q = 0; q < LB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float sm = 0.f;
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) {
            acc[mb0 + q][nb][i] += bias[nb];
            sm += acc[mb0 + q][nb][i];
          }
          mean[4 * q + i] = sm;
        }
      row_sum16_n<LB * 4>(mean);
#pragma unroll
      for (int k = 0; k < LB * 4; ++k) mean[k] *= a.ln_inv;
      // channels at or beyond the state depth carry exact zeros (zero weights and bias):
      // each adds mean^2 to the sum of squared deviations, removed in one step
#pragma unroll
      for (int q = 0; q < LB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float sq = 0.f;
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) {
            const float dv = acc[mb0 + q][nb][i] - mean[4 * q + i];
            sq += dv * dv;
          }
          rstd[4 * q + i] = sq;
        }
      row_sum16_n<LB * 4>(rstd);
#pragma unroll
      for (int k = 0; k < LB * 4; ++k) {
        const float var = fmaxf(rstd[k] - a.ln_pad * mean[k] * mean[k], 0.f) * a.ln_inv;
        rstd[k] = rsqrtf(var + 1e-5f);
      }
      if constexpr (EPI == EPI_LN_RELU_SAVE) {
#pragma unroll
        for (int q = 0; q < LB; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = wave * 16 * MB + (mb0 + q) * 16 + 4 * lk + i;
            if (r < tl.nrows) {
              const int64_t grow = g.row_base + tl.row0 + r;
              float z[8];
#pragma unroll
              for (int nb = 0; nb < 8; ++nb) z[nb] = acc[mb0 + q][nb][i];
              pack8<T>::store(a.save_z + grow * NRX_D + ch0, z);
              if (lr == 0) { a.save_stats[2 * grow] = mean[4 * q + i]; a.save_stats[2 * grow + 1] = rstd[4 * q + i]; }
            }
          }
      }
#pragma unroll
      for (int q = 0; q < LB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) {
            const float n = (acc[mb0 + q][nb][i] - mean[4 * q + i]) * (rstd[4 * q + i] * lng[nb]) + lnb[nb];
            acc[mb0 + q][nb][i] = n > 0.f ? n : 0.f;
          }
    }
  }

  float vmax = 0.f;   // max |output| of this lane (calibration of FP8 scales)
  int om[4] = {0, 0, 0, 0};   // Var-IO StateInit: bits per symbol of the slot's UEs (scalar loads)
  if constexpr (EPI == EPI_STORE) {
    if (a.only_m) {
#pragma unroll
      for (int k = 0; k < 4; ++k) om[k] = ldc(&a.geo[tl.slot].m[k]);
    }
  }
  // residual rows of the lane (EPI_RESID), requested RB m-blocks at a time before any of
  // them is used; rows past the tile read row 0 and are not stored
  constexpr int RB = MB % 2 == 0 ? 2 : 1;
  v16 rraw[EPI == EPI_RESID ? RB : 1][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    if constexpr (EPI == EPI_RESID && sizeof(T) == 2) {
      if (mb % RB == 0) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = wave * 16 * MB + (mb + q) * 16 + 4 * lk + i;
            const int64_t grow = g.row_base + tl.row0 + (r < tl.nrows ? r : 0);
            rraw[q][i] = ld16(a.resid + grow * NRX_D + ch0);
          }
      }
      // keeps the scheduler from hoisting the next batch above this m-block's stores
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // every row is computed (straight-line code across rows); rows past the tile are not stored
      const int r = wave * 16 * MB + mb * 16 + 4 * lk + i;
      const bool valid = r < tl.nrows;
      const int64_t grow = g.row_base + tl.row0 + (valid ? r : 0);
      float v[8];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) v[nb] = LN ? acc[mb][nb][i] : acc[mb][nb][i] + bias[nb];
      if constexpr (EPI == EPI_RESID) {
        if constexpr (sizeof(T) == 2) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            v[2 * k] += __uint_as_float(rraw[mb % RB][i].w[k] << 16);
            v[2 * k + 1] += __uint_as_float(rraw[mb % RB][i].w[k] & 0xFFFF0000u);
          }
        } else {
          float rsd[8];
          pack8<T>::load(a.resid + grow * NRX_D + ch0, rsd);
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) v[nb] += rsd[nb];
        }
      }
      bool keep = valid;
      if constexpr (EPI == EPI_STORE) {
        if (a.only_m) {   // Var-IO StateInit: this launch writes its modulation's UEs only
          const int u = (tl.row0 + r) % U;
          keep = keep && (u == 0 ? om[0] : (u == 1 ? om[1] : (u == 2 ? om[2] : om[3]))) == a.only_m;
        }
      }
      if (keep) {
        if (a.out) pack8<T>::store(a.out + grow * NRX_D + ch0, v);
        if (a.out8) *reinterpret_cast<uint2 *>(a.out8 + grow * NRX_D + ch0) = fp8x8(v, a.out8_inv);
        if (a.amax) {
#pragma unroll
          for (int nb = 0; nb < 8; ++nb) vmax = fmaxf(vmax, fabsf(v[nb]));
        }
      }
    }
  }
  if (a.amax) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, m, 64));
    if (lr == 0 && lk == 0) atomicMax(a.amax, __float_as_uint(vmax));
  }
}

// Final dgamma/dbeta reduction of the LayerNorm-backward epilogue (after the tile loop).
template <int EPI, int NW>
__device__ __forceinline__ void conv_ln_reduce(float *lnp, float *red, float *out, int tid, int wave, int lr, int lk) {
  if constexpr (EPI == EPI_LN_BWD) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      lnp[k] += __shfl_xor(lnp[k], 16, 64);
      lnp[k] += __shfl_xor(lnp[k], 32, 64);
    }
    __syncthreads();
    if (lk == 0) {
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        red[wave * 256 + 8 * lr + nb] = lnp[nb];
        red[wave * 256 + 128 + 8 * lr + nb] = lnp[8 + nb];
      }
    }
    __syncthreads();
    if (tid < 256) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += red[w * 256 + tid];
      out[(int64_t)blockIdx.x * 256 + tid] = v;
    }
  }
}

}  // namespace
