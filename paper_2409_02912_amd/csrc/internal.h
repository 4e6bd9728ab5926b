// Internal launch interfaces between the libnrx host code and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

enum { EPI_STORE = 0, EPI_LN_RELU = 1, EPI_RESID = 2 };

template <typename T>
struct ConvArgs {
  const T *src0;            // [rows][c0]
  const T *src1;            // [rows][c1] or null (channel concatenation)
  int c0, c1;
  const T *w;               // prepped [chunk][tap][nb][16][KC]
  const float *bias;        // [128]
  const float *pe;          // positional-encoding field [2][3][14][128] or null
  const float *ln_g, *ln_b; // [128] (EPI_LN_RELU)
  const T *resid;           // [rows][128] (EPI_RESID)
  T *out;                   // [rows][128]
  T *save_z;                // pre-LN output (EPI_LN_RELU, training) or null
  float *save_stats;        // [rows][2] mean, rstd (EPI_LN_RELU, training)
  const SlotGeo *geo;
  const Tile *tiles;
  int n_tiles;
};

struct ConvVariant {
  int mb;     // MFMA m-blocks (16 rows) per wave: tile = 64 * mb rows
  int occ;    // waves per SIMD the kernel is built for
  int pref;   // weights prefetched one tap ahead
};
#define NRX_CONV_VARIANTS 4
extern const ConvVariant kConvVariants[NRX_CONV_VARIANTS];

template <typename T>
void launch_conv(const ConvArgs<T> &a, int epi, int variant, int grid, hipStream_t st);

// Weight preparation: fp32 master -> MFMA operand layouts and PE fields.
struct PrepJob {
  int32_t kind;        // 0 conv, 1 dense, 2 PE field, 3 conv transposed+flipped (dgrad), 4 narrow dense
  int32_t cin_real;    // input channels present in the master tensor (conv: without PE)
  int32_t cin_total;   // input channels of the master tensor (incl. PE channels)
  int32_t n_chunks;    // K chunks of the prepped operand
  int32_t cin_first;   // first master input channel used (dgrad slices)
  int32_t n_out;       // output columns of the master tensor (narrow dense: m_max)
  int64_t src;         // element offset into the master weights
  int64_t dst;         // element offset into the prepped (T) or field (fp32) buffer
  int64_t count;       // prepped elements of this job
};

template <typename T>
void launch_prep(const float *w, const PrepJob *jobs, int n_jobs, int64_t total, T *wprep,
                 float *fields, hipStream_t st);

// Front end: DMRS generation, LS pair estimates, interpolation + feature rows.
void launch_dmrs(const SlotGeo *geo, int n_slots, float2 *dmrs, hipStream_t st);
void launch_ls_pairs(const SlotGeo *geo, int n_slots, int max_pairs_total, const float2 *y,
                     const float2 *dmrs, float2 *pairs, const int64_t *pair_off, int max_u_b_pairs,
                     hipStream_t st);
template <typename T>
void launch_features(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re,
                     const float2 *y, const float2 *pairs, const int64_t *pair_off, int model_B,
                     int cx, T *X, float2 *h_out, hipStream_t st);

// Message passing and readout.
template <typename T>
struct MlpArgs {
  const T *h;               // [rows][128]
  const T *w1, *w2;         // prepped dense [chunk][nb][16][KC]; readout w2: [chunk][16][KC]
  const float *b1, *b2;     // [128] / [m_max]
  T *out;                   // MP: aggregated messages [rows][128]
  T *save_m1;               // MP/readout hidden activations (training) or null
  float *llr;               // readout output
  int m_max;
  const SlotGeo *geo;
  const Tile *tiles;
  int n_tiles;
};
template <typename T>
void launch_mp(const MlpArgs<T> &a, int grid, hipStream_t st);
template <typename T>
void launch_readout(const MlpArgs<T> &a, int grid, hipStream_t st);

// LMMSE + max-log judge.
void launch_lmmse(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re, int m_max,
                  const float2 *y, const float2 *h, const float *n0dev, float *llr, hipStream_t st);

// Slot simulator.
struct SimParams {
  int n_taps, tap_spacing_ns, scs_khz;
  float tap_decay_ns, doppler_max_hz, rho, snr_lo, snr_hi;
  uint32_t key0, key1, batch;
};
void launch_sim(const SimParams &p, const SlotGeo *geo, const int64_t *tap_off, int n_slots, int64_t max_re,
                int max_ubl, int m_max, const float2 *dmrs, float2 *g_raw, float2 *g_mix, float *fd_n0, float2 *y,
                float2 *h_true, uint8_t *bits, float *snr_db, float *n0, int64_t max_bits, hipStream_t st);

// Training kernels.
void launch_bce(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re, int m_max,
                const float *llr, const uint8_t *bits, float *dllr, double *partials, int n_part,
                double *loss, unsigned long long *nerr, double inv_n, hipStream_t st);
void launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st);
