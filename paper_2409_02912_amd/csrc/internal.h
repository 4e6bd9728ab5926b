// Internal launch interfaces between the libnrx host code and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

enum { EPI_STORE = 0, EPI_LN_RELU = 1, EPI_RESID = 2, EPI_LN_BWD = 3, EPI_LN_RELU_SAVE = 4 };  // 4: EPI_LN_RELU keeping z and its statistics (training)

template <typename T>
struct ConvArgs {
  const T *src0;            // [rows][c0]
  const T *src1;            // [rows][c1] or null (channel concatenation)
  int c0, c1;
  const T *w;               // prepped [chunk][tap][nb][16][KC]
  const float *bias;        // [128]
  const float *pe;          // positional-encoding field [2][3][14][128] or null
  const float *ln_g, *ln_b; // [128] (EPI_LN_RELU; zero beyond the state depth d)
  float ln_inv;             // 1 / d: LayerNorm statistics over the first d channels (the rest are zero)
  float ln_pad;             // 128 - d, the number of zero channels
  const T *resid;           // [rows][128] (EPI_RESID)
  T *out;                   // [rows][128]
  T *save_z;                // pre-LN output (EPI_LN_RELU, training; input of EPI_LN_BWD) or null
  float *save_stats;        // [rows][2] mean, rstd (EPI_LN_RELU, training; input of EPI_LN_BWD)
  float *ln_part;           // EPI_LN_BWD: per-workgroup [256] partial sums of dL/dgamma, dL/dbeta
  const SlotGeo *geo;
  const Tile *tiles;
  int n_tiles;
  // FP8 operands (conv3x3_fp8 kernels): E4M3 activations [rows][c0] / [rows][c1],
  // prepped weights [chunk][tap pair][nb][16][128 B] and per-output-channel scales
  const uint8_t *src8_0, *src8_1;
  const uint8_t *w8;
  const float *wscale;
  uint8_t *out8;            // E4M3 copy of the output, out * out8_inv, or null (out may then be null)
  float out8_inv;
  unsigned int *amax;       // max |output| over the launch (float bits, atomicMax), or null
  int only_m;               // EPI_STORE (Var-IO StateInit): store only the rows of UEs with this many bits
};

struct ConvVariant {
  int mb;     // tile = 64 * mb rows (MFMA m-blocks per wave for 4-wave workgroups)
  int occ;    // waves per SIMD the kernel is built for
  int pref;   // 1: weights prefetched one tap ahead; 2: weights and halo through LDS (K loop unrolled
              // over two chunks: even chunk counts only); 3: the same, rolled (ring kernel)
  int aligned = 0;   // 1: tiles of CONV_ALIGNED_TILE rows starting on subcarrier boundaries
};
constexpr int CONV_ALIGNED_TILE = 504;   // whole subcarriers for U = 1..4 (14 U rows each)
#define NRX_CONV_VARIANTS 15
extern const ConvVariant kConvVariants[NRX_CONV_VARIANTS];
constexpr int CONV_DEFAULT_VARIANT = 14;   // a new model's variant for every conv class
#define NRX_CONV8_VARIANTS 5
constexpr int NRX_N_MODS = 4;   // modulations by bits per symbol: 2, 4, 6, 8 (index bits / 2 - 1)
constexpr int CONV8_DEFAULT_VARIANT = 0;   // ... and for the E4M3 block convs of FP8 models
extern const ConvVariant kConv8Variants[NRX_CONV8_VARIANTS];   // mb = tile rows / 64

// FP8 convolution (EPI_LN_RELU or EPI_RESID) on E4M3 operands a.src8_*, a.w8, a.wscale.
void launch_conv8(const ConvArgs<bf16_t> &a, int epi, int variant, int grid, hipStream_t st);

// Quantisation of one conv layer's weights to E4M3 with the input activation
// scales folded in (s0 for input channels < c0, s1 above).
struct Fp8Job {
  int64_t src;         // element offset of the master conv tensor [3][3][cin_total][128]
  int32_t cin_real;    // input channels quantised (multiple of 64; PE channels excluded)
  int32_t cin_total;
  int32_t c0;          // channels of the first input
  float s0, s1;        // activation scales of the two inputs
  int64_t dst;         // byte offset of the prepped operand
  int64_t sdst;        // float offset of the 128 weight scales
};
void launch_prep_fp8(const float *w, const Fp8Job *jobs, int n_jobs, uint8_t *w8, float *wscale, hipStream_t st);

template <typename T>
void launch_conv(const ConvArgs<T> &a, int epi, int variant, int grid, hipStream_t st);

// Weight preparation: fp32 master -> MFMA operand layouts and PE fields.
struct PrepJob {
  int32_t kind;        // 0 conv, 1 dense, 2 PE field, 3 conv transposed+flipped (dgrad), 4 narrow dense,
                       // 5 dense transposed, 6 vector zero-padded to 128 (into the field buffer)
  int32_t cin_real;    // input channels present in the master tensor (conv: without PE)
  int32_t cin_total;   // input channels of the master tensor (incl. PE channels)
  int32_t n_chunks;    // K chunks of the prepped operand
  int32_t cin_first;   // first master input channel used (dgrad slices)
  int32_t n_out;       // output columns of the master tensor (narrow dense: m_max)
  int64_t src;         // element offset into the master weights
  int64_t dst;         // element offset into the prepped (T) or field (fp32) buffer
  int64_t count;       // prepped elements of this job
  int32_t d_out;       // output columns of the master conv/dense tensor (the state depth d <= 128)
  int32_t seg;         // master input channels per 128-wide activation segment (0: identity map)
};

template <typename T>
void launch_prep(const float *w, const PrepJob *jobs, int n_jobs, int64_t total, T *wprep,
                 float *fields, hipStream_t st);

// Front end: DMRS generation, LS pair estimates, interpolation + feature rows.
// slot_mask (nullable, device, one word per slot): when given, slots whose word is 0 are skipped.
void launch_dmrs(const SlotGeo *geo, int n_slots, float2 *dmrs, hipStream_t st,
                 const unsigned int *slot_mask = nullptr);
void launch_ls_pairs(const SlotGeo *geo, int n_slots, int max_pairs_total, const float2 *y,
                     const float2 *dmrs, float2 *pairs, const int64_t *pair_off, int max_u_b_pairs,
                     hipStream_t st, const unsigned int *slot_mask = nullptr);
template <typename T>
void launch_features(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re,
                     const float2 *y, const float2 *pairs, const int64_t *pair_off, int model_B,
                     int cx, T *X, float2 *h_out, hipStream_t st, const unsigned int *slot_mask = nullptr,
                     unsigned int *slot_flags = nullptr);   // OR-ed with 4 for a slot whose y is not all finite

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
  uint8_t *out8;                  // MP: E4M3 copy of the aggregated messages (out * out8_inv) or null
  float out8_inv;
  unsigned int *amax;             // MP: max |aggregate| (float bits, atomicMax) or null
  unsigned int *slot_done;        // readout: finished tiles per slot (zeroed by launch_stamp_start)
  unsigned long long *stamps;     // readout: wall-clock time at which each slot's last tile finished
  unsigned int *slot_flags;       // readout: per-slot health word, OR-ed with bit 0 (LLR readout) or bit 1
                                  // (ReadoutChEst) when a value the launch stores for the slot is not finite
  int chest;                      // readout: ReadoutChEst -- llr is a channel estimate in the h layout
                                  // ([s][t][u][b] complex at geo.h_off), outputs j < 2B of the slot
  int n_out;                      // readout: columns of w2 / b2 (0: m_max)
  int only_m;                     // readout (Var-IO): write only the rows of UEs with this many bits (0: all)
};
template <typename T>
void launch_mp(const MlpArgs<T> &a, int grid, hipStream_t st);
// Zeroes the per-slot tile counters and health words (flags, nullable) and records the start time in
// stamps[n_slots].
void launch_stamp_start(unsigned int *slot_done, unsigned long long *stamps, unsigned int *flags, int n_slots,
                        hipStream_t st);
// dst[i] = src[i], i < n (device words)
void launch_copy_words(const unsigned int *src, unsigned int *dst, int n, hipStream_t st);
// latency_us[i] = (stamps[i] - stamps[n]) / rate
void launch_stamp_latency(const unsigned long long *stamps, int n_slots, double ticks_per_us, float *latency_us,
                          hipStream_t st);
template <typename T>
void launch_readout(const MlpArgs<T> &a, int grid, hipStream_t st);

// LMMSE + max-log judge.
// slot_mask (nullable): only slots with a non-zero word are demapped, and their LLRs that are not finite
// are written as 0 (the fallback of a flagged NRX slot).
void launch_lmmse(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re, int m_max,
                  const float2 *y, const float2 *h, const float *n0dev, float *llr, hipStream_t st,
                  const unsigned int *slot_mask = nullptr);

// Persistent forward (BF16 inference): one launch runs every layer of the CGNN over every slot.
// A work item is (stage, slot, run of up to item_tiles consecutive tiles of the slot).  Slots form groups
// of consecutive slots; the items of a group come after those of the groups before it, and inside a
// group they are ordered by stage, then slot, then tile, so every item comes after the items it reads.
// Workgroups claim items in that order from a counter.  A conv item on tiles ta .. tb - 1 waits for the
// previous stage's tiles ta - 1 .. tb of its slot (the 3x3 halo), an MLP item for tiles ta .. tb - 1.
enum { PK_CONV_STORE = 0, PK_CONV_LN = 1, PK_CONV_RESID = 2, PK_MP = 3, PK_READOUT = 4 };
struct PersistStage {
  int32_t kind;                 // PK_*
  int32_t pad;
  ConvArgs<bf16_t> c;           // conv stages (tiles/n_tiles unused)
  MlpArgs<bf16_t> m;            // MLP stages (tiles/n_tiles unused)
};
struct PersistArgs {
  const PersistStage *stages;
  int32_t n_stages;
  int32_t n_groups;
  const SlotGeo *geo;
  const int32_t *tile_base;     // per slot (n + 1 entries): index of its first tile in the batch
  const int32_t *item_base;     // per slot (n + 1 entries): index of its first item in a stage
  const int32_t *tile_rows;     // per slot: rows per tile (whole REs, at most PERSIST_TILE)
  const int32_t *group_slot;    // per group (n_groups + 1 entries): its first slot
  int32_t item_tiles;           // consecutive tiles of one slot per work item
  unsigned int *ctl;            // [0] next item to claim, [1] abort (a wait ran out); zeroed before the launch
  unsigned int *done;           // [stage][tile of the batch]: finished flags (zeroed before the launch)
  unsigned int *slot_done;      // per slot: readout tiles finished (zeroed before the launch)
  unsigned long long *stamps;   // per slot: wall clock when its last readout item finished
  unsigned int *slot_flags;     // per-slot health word; bit 3 when a wait of one of its items ran out
  int32_t spin_limit;           // polls of a dependency flag before the wait gives up
};
constexpr int PERSIST_TILE = 512;       // rows per persistent tile (before rounding down to whole REs)
constexpr int PERSIST_ITEM_TILES = 4;   // most tiles per work item (large batches)

// Item it of the persistent order -> (stage, slot, item of the slot).  IB(i) reads item_base[i], GS(i)
// group_slot[i]; the same code runs in the kernel (scalar loads) and on the host.
struct PersistIdx {
  int stage, slot, item;
};
template <typename IB, typename GS>
__host__ __device__ inline PersistIdx persist_decode(int it, int n_stages, int n_groups, IB ib, GS gs) {
  auto last_at_most = [](int lo, int hi, int x, auto key) {   // largest i in [lo, hi] with key(i) <= x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (key(mid) <= x) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  const int g = last_at_most(0, n_groups - 1, it, [&](int i) { return n_stages * ib(gs(i)); });
  const int gs0 = gs(g), gs1 = gs(g + 1);
  const int i0 = ib(gs0), ig = ib(gs1) - i0;
  const int k = it - n_stages * i0;
  PersistIdx r;
  r.stage = k / ig;
  const int gi = i0 + (k - r.stage * ig);
  r.slot = last_at_most(gs0, gs1 - 1, gi, [&](int i) { return ib(i); });
  r.item = gi - ib(r.slot);
  return r;
}
// Workgroups of the persistent kernel that fit on the device at once (0 if it cannot run).
int persist_max_grid();
void launch_persist(const PersistArgs &a, int grid, hipStream_t st);
// Clears n words (a fill kernel: no memset node in a captured graph).
void launch_zero_words(unsigned int *p, int64_t n, hipStream_t st);

// Slot simulator.
struct SimParams {
  int n_taps, tap_spacing_ns, scs_khz;
  float tap_decay_ns, doppler_max_hz, rho, snr_lo, snr_hi;
  uint32_t key0, key1, batch;
};
void launch_sim(const SimParams &p, const SlotGeo *geo, const int64_t *tap_off, int n_slots, int64_t max_re,
                int max_ubl, int m_max, const float2 *dmrs, float2 *g_raw, float2 *g_mix, float *fd_n0, float2 *y,
                float2 *h_true, uint8_t *bits, float *snr_db, float *n0, int64_t max_bits, hipStream_t st);

// Backward pass.
template <typename T>
struct WgradArgs {
  const T *src0, *src1;     // layer input [rows][c0] / [rows][c1] (channel concatenation)
  int c0, c1;
  const T *dy;              // output gradient [rows][128]
  const SlotGeo *geo;
  const Tile *tiles;        // row tiles of the batch (partitioned among workgroups)
  int n_tiles, n_part;      // n_part: row partitions (multiple of 8)
  int n_taps, tap0;         // taps tap0 .. tap0 + n_taps - 1 (dense layers: 1 tap, the centre)
  int n_slices;             // 128-channel input slices
  float *partials;          // [n_part][n_taps * n_slices][128][128]
};
template <typename T>
void launch_wgrad(const WgradArgs<T> &a, hipStream_t st);
// workgroups launch_wgrad runs per row partition (BF16 3x3 convolutions take three taps per workgroup)
int wgrad_jobs_per_partition(int n_taps, int n_slices, bool bf16);
void launch_wgrad_reduce(const float *partials, int n_part, int n_taps, int tap0, int n_slices, int cin_real,
                         int cin_total, int conv, int64_t dst_off, float *dw, hipStream_t st,
                         bool acc = false);
template <typename T>
void launch_colsum(const T *dy, const SlotGeo *geo, int n_slots, float *partial, hipStream_t st);
void launch_bias_pe(const float *partial, int n_slots, int64_t bias_off, int64_t pe_w_off, int cin_total, int pe_ch,
                    float *dw, hipStream_t st,
                    bool acc = false);
void launch_ln_reduce(const float *part, int n, int64_t g_off, int64_t b_off, float *dw, hipStream_t st);

template <typename T>
struct MpBwdArgs {
  const T *dagg, *m1;       // [rows][128]
  const T *w1t, *w2t;       // transposed prepped dense weights
  T *dmsg, *dm1;            // outputs for the weight gradients
  T *dh;                    // updated in place
  const SlotGeo *geo;
  const Tile *tiles;
  int n_tiles;
};
template <typename T>
void launch_mp_bwd(const MpBwdArgs<T> &a, int grid, hipStream_t st);

// dst = src on the rows of UEs with only_m bits per symbol, 0 on the others ([rows][128]; Var-IO StateInit).
template <typename T>
void launch_select_rows(const T *src, const SlotGeo *geo, int n_slots, int64_t max_rows, int only_m, T *dst,
                        hipStream_t st);

template <typename T>
struct RoBwdArgs {
  const float *dllr;        // llr layout
  const T *q;               // saved hidden (post ReLU) [rows][128]
  const float *w2;          // master readout w2 [128][m_max]
  const T *w1t;             // transposed prepped readout w1
  T *dr;                    // hidden-layer gradient [rows][128] (for dW1)
  T *dh;                    // gradient w.r.t. the state read out [rows][128]
  int accumulate;           // add to dh (a readout before the last CGNN iteration) instead of writing it
  float *part;              // per-workgroup [1032] partials of dW2 (128 x 8) and db2 (8)
  int m_max;                // outputs of the readout (columns of w2)
  int j0;                   // first of the 8 output columns this call handles
  int chest;                // ReadoutChEst: dllr is the gradient of a channel estimate (h layout)
  int acc_dr;               // add this call's hidden gradient to dr (the second column group)
  int n_out;                // columns of w2 (0: m_max)
  int only_m;               // Var-IO: only the rows of UEs with this many bits contribute (0: all)
  const SlotGeo *geo;
  const Tile *tiles;
  int n_tiles;
};
template <typename T>
void launch_readout_bwd(const RoBwdArgs<T> &a, int grid, hipStream_t st);
void launch_readout_w2_reduce(const float *part, int n, int m_max, int64_t w2_off, int64_t b2_off, float *dw,
                              hipStream_t st, int j0 = 0);

// Training kernels.
void launch_bce(const SlotGeo *geo, const int64_t *re_base, int n_slots, int64_t n_re, int m_max,
                const float *llr, const uint8_t *bits, float *dllr, double *partials, int n_part,
                double *loss, unsigned long long *nerr, double inv_n, hipStream_t st);
// Double-readout channel loss: per slot, sum over its h-layout entries of (hest - htrue)^2 (fp64),
// dhest = gscale * (hest - htrue); *loss = total * inv_n.
void launch_mse(const SlotGeo *geo, int n_slots, const float *hest, const float *htrue, float *dhest, float gscale,
                double *partials, int n_part, double *loss, double inv_n, hipStream_t st);
void launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st);
