// Device-side helpers shared by the libnrx kernels (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NRX_T 14                 // OFDM symbols per slot
#define NRX_DMRS0 2              // DMRS symbols (type A, l0 = 2, one additional position)
#define NRX_DMRS1 11
#define NRX_D 128                // state depth supported by the kernels
#define NRX_MAXU 4

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8_t;

typedef uint16_t bf16_t;  // storage type of bfloat16 activations and weights

// float -> bfloat16, round to nearest even (the hardware conversion of gfx950)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Scalar element traits for the two activation storage types.
template <typename T> struct elem;
template <> struct elem<float> {
  __device__ static __forceinline__ float to_f(float x) { return x; }
  __device__ static __forceinline__ float from_f(float x) { return x; }
};
template <> struct elem<bf16_t> {
  __device__ static __forceinline__ float to_f(bf16_t x) { return bf2f(x); }
  __device__ static __forceinline__ bf16_t from_f(float x) { return f2bf(x); }
};

// 16 bytes of operand data
struct __align__(16) v16 { uint32_t w[4]; };

__device__ __forceinline__ v16 ld16(const void *p) { return *reinterpret_cast<const v16 *>(p); }
__device__ __forceinline__ void st16(void *p, v16 v) { *reinterpret_cast<v16 *>(p) = v; }

// MFMA on one 16x16 output block.  D layout (all variants): lane l holds rows
// 4*(l/16)+i, i = 0..3, of column l%16.
//   bf16 16x16x32: lane l holds A[l%16][8*(l/16) .. +7] and B[8*(l/16) .. +7][l%16]
//   fp32 16x16x4 : lane l holds A[l%16][l/16] and B[l/16][l%16]; a 16-byte fragment
//                  (channels 4*(l/16) .. +3 of a 16-channel chunk) feeds four k-steps,
//                  step q taking channel 4*(l/16) + q, so chunks keep natural order
__device__ __forceinline__ f32x4_t mfma_bf16(v16 a, v16 b, f32x4_t c) {
  bf16x8_t av, bv;
  __builtin_memcpy(&av, &a, 16);
  __builtin_memcpy(&bv, &b, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4_t mfma_f32x4(v16 a, v16 b, f32x4_t c) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w[q]), __uint_as_float(b.w[q]), c, 0, 0, 0);
  return c;
}

template <typename T> struct mma;
template <> struct mma<float> {
  // one 16-byte fragment covers K = 16 (four fp32 k-steps)
  static constexpr int KF = 16;
  __device__ static __forceinline__ f32x4_t run(v16 a, v16 b, f32x4_t c) { return mfma_f32x4(a, b, c); }
};
template <> struct mma<bf16_t> {
  static constexpr int KF = 32;
  __device__ static __forceinline__ f32x4_t run(v16 a, v16 b, f32x4_t c) { return mfma_bf16(a, b, c); }
};

// LDS rows of 64 bytes hold four 16-byte pieces; piece p of row h sits in slot
// p ^ swz(h) so that 16 consecutive rows read at the same piece hit distinct banks.
__host__ __device__ __forceinline__ int swz(int h) { return (h >> 1) & 3; }

// Output-channel permutation used by every MFMA GEMM here: n-block nb, column j
// of the MFMA output holds channel 8*j + nb, so a lane owns 8 consecutive
// channels of each of its rows.
__host__ __device__ __forceinline__ int nperm(int nb, int j) { return 8 * j + nb; }

// FP8 (OCP E4M3) MFMA, 16x16x128, unit block scales: lane l holds 32 bytes of
// A row l%16 and of B column l%16 for k-group l/16; A and B use the same
// k order, so any pairing of operand bytes with input channels that both sides
// share gives the dot product.
__device__ __forceinline__ f32x4_t mfma_fp8(const i32x8_t &a, const i32x8_t &b, f32x4_t c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// 8 floats -> 8 E4M3 bytes of x * inv (saturated to the finite range +-448)
__device__ __forceinline__ uint2 fp8x8(const float *x, float inv) {
  float q[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) q[k] = fminf(fmaxf(x[k] * inv, -448.f), 448.f);
  int lo = 0, hi = 0;
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], lo, false);
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], lo, true);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[4], q[5], hi, false);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[6], q[7], hi, true);
  return make_uint2((unsigned)lo, (unsigned)hi);
}

__device__ __forceinline__ float shfl_xor16(float v, int m) { return __shfl_xor(v, m, 64); }

// v plus the value of the lane that the DPP control CTRL selects within each row of 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes that share l/16 (the lanes owning one row's channels), all
// lanes receiving it: a butterfly over the 16-lane DPP row (swap neighbours, swap
// pairs, mirror each half, mirror the row) in four VALU adds, no LDS traffic.
__device__ __forceinline__ float row_sum16(float v) {
  v = dpp_add<0xB1>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141>(v);   // row_half_mirror
  v = dpp_add<0x140>(v);   // row_mirror
  return v;
}

// row_sum16 of N independent values, each butterfly step applied to all of them in turn
template <int N>
__device__ __forceinline__ void row_sum16_n(float (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = dpp_add<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = dpp_add<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = dpp_add<0x141>(v[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = dpp_add<0x140>(v[k]);
}

// 8 consecutive channels <-> 16/32 bytes
template <typename T> struct pack8;
template <> struct pack8<bf16_t> {
  __device__ static __forceinline__ void load(const bf16_t *p, float *o) {
    v16 v = ld16(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(v.w[i] << 16);
      o[2 * i + 1] = __uint_as_float(v.w[i] & 0xFFFF0000u);
    }
  }
  __device__ static __forceinline__ void store(bf16_t *p, const float *x) {
    v16 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v.w[i] = pack_bf2(x[2 * i], x[2 * i + 1]);
    st16(p, v);
  }
};
template <> struct pack8<float> {
  __device__ static __forceinline__ void load(const float *p, float *o) {
    v16 a = ld16(p), b = ld16(p + 4);
#pragma unroll
    for (int i = 0; i < 4; ++i) { o[i] = __uint_as_float(a.w[i]); o[4 + i] = __uint_as_float(b.w[i]); }
  }
  __device__ static __forceinline__ void store(float *p, const float *x) {
    v16 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) { a.w[i] = __float_as_uint(x[i]); b.w[i] = __float_as_uint(x[4 + i]); }
    st16(p, a);
    st16(p + 4, b);
  }
};

// Per-slot geometry used by the row-tiled kernels (device copy of the plan).
struct SlotGeo {
  int32_t S;          // subcarriers
  int32_t U;          // UEs
  int32_t B;          // antennas of the slot
  int32_t m[4];       // bits per symbol of each UE
  int32_t slot_number, n_id, n_scid;
  float n0;
  float snr_off;      // slot_sim: dB added to the drawn SNR
  int64_t row_base;   // first activation row of the slot
  int64_t y_off;      // complex elements
  int64_t h_off;      // complex elements
  int64_t llr_off;    // floats
  int64_t bits_off;   // bytes
  int64_t dmrs_off;   // complex elements into the DMRS table ([2][S/2] per slot)
};

struct __align__(16) Tile {
  int32_t slot;
  int32_t row0;       // first row within the slot
  int32_t nrows;
  int32_t pad;
};
