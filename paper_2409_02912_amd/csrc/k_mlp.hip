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
#include "mlp_lds.h"

namespace {


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

template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void mp_lds_kernel(MlpArgs<bf16_t> a) {
  __shared__ __align__(16) unsigned char lds[MP_LDS_BYTES];
  mp_lds_body<NW>(a, MlpGridTiles(a.tiles, a.n_tiles), (lds_u8 *)lds);
}

template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void readout_lds_kernel(MlpArgs<bf16_t> a) {
  __shared__ __align__(16) unsigned char lds[RO_LDS_BYTES];
  readout_lds_body<NW>(a, MlpGridTiles(a.tiles, a.n_tiles), (lds_u8 *)lds);
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
