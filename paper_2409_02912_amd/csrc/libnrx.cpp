// libnrx host side: validation, batch plans, workspace layout and the C ABI.
//
// A "plan" is everything derived from a batch's slot descriptors: per-slot
// geometry, the row tiles of every kernel and the workspace layout.  Plans are
// cached by a hash of the descriptors; their device-side tables are staged in
// pinned host memory and copied into the caller's workspace with an async copy on
// the caller's stream at every call, so a call only enqueues work.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/libnrx.h"
#include "internal.h"

// ------------------------------------------------------------------ errors --

static thread_local std::string g_err;

static nrx_status fail(nrx_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(NRX_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char *nrx_last_error(void) { return g_err.c_str(); }

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ----------------------------------------------------------------- layouts --

namespace {

constexpr int MLP_TILE = 128;
constexpr int PERSIST_GROUP = 1024;        // tiles per slot group of the persistent forward (one item per CU)
// conv tiles of 128, 256, 384 and 512 rows (mb = 2, 4, 6, 8), and of 504 rows: whole subcarriers for
// every UE count (504 = 36, 18, 12, 9 subcarriers of 14, 28, 42, 56 rows)
constexpr int N_TILE_SIZES = 5;
constexpr int ALIGNED_TILES = 4;
inline int tile_size_index(int mb) { return mb / 2 - 1; }
inline int tile_rows_of_index(int i) { return i == ALIGNED_TILES ? CONV_ALIGNED_TILE : 128 * (i + 1); }
inline int variant_tiles(const ConvVariant &v) { return v.aligned ? ALIGNED_TILES : tile_size_index(v.mb); }

struct TensorInfo {
  std::string name;
  int64_t off;
  int ndim;
  int shape[4];
};

struct ConvLayer {
  int64_t w = 0, b = 0;         // master offsets
  int cin_real = 0, cin_total = 0, n_chunks = 0;
  int64_t prep = 0;             // element offset in the prepped buffer
  int64_t field = -1;           // element offset in the field buffer (PE folded) or -1
  int64_t w8 = -1, ws8 = -1;    // FP8 models: byte offset of the E4M3 operand, float offset of its scales
  int64_t bpad = -1;            // d < 128: bias padded to 128 channels (field buffer offset)
};

struct BlockLayer {
  ConvLayer a, b;
  int64_t g = 0, beta = 0;
  int64_t gpad = -1, betapad = -1;   // d < 128: LayerNorm parameters padded with zeros
  int mp_round = -1;            // message-passing round before this block, or -1
  // backward: prepped data-gradient weights (offsets in the backward prepped buffer)
  int64_t bg_b = 0, bg_a_h = 0, bg_a_agg = -1;
};

struct DenseLayer {
  int64_t w1 = 0, b1 = 0, w2 = 0, b2 = 0;
  int64_t b1pad = -1, b2pad = -1;   // d < 128: biases padded with zeros
  int64_t p1 = 0, p2 = -1;      // prepped offsets
  int64_t t1 = -1, t2 = -1;     // backward: prepped transposed weights
};

struct Plan {
  int n = 0;
  std::vector<SlotGeo> geo;
  std::vector<Tile> ct[N_TILE_SIZES], mt, rt;
  std::vector<int64_t> pair_off, tap_off;
  // persistent forward: per slot the first tile and the first item of a stage (n + 1 entries each) and rows
  // per tile (whole REs, at most PERSIST_TILE); slot groups (first slot of each, n_groups + 1 entries) of at
  // least PERSIST_GROUP tiles
  std::vector<int32_t> ptile_base, pitem_base, ptile_rows, pgroup;
  int pitem_tiles = 1;           // consecutive tiles per persistent work item
  // batches that mix modulations: per modulation (index m / 2 - 1) the conv and readout tiles of the slots
  // with a UE of that modulation, which the Var-IO StateInit and readout launches of that modulation walk
  bool mod_lists = false;
  std::vector<Tile> ctm[NRX_N_MODS][N_TILE_SIZES], rtm[NRX_N_MODS];
  int64_t rows = 0, max_rows = 0, max_re = 0, max_pairs = 0, max_ute = 0, max_bits = 0;
  int64_t dmrs_total = 0, pairs_total = 0, n_data_bits = 0;
  int max_ubl = 0;
  // device table blob
  size_t off_geo = 0, off_ct[N_TILE_SIZES] = {}, off_mt = 0, off_rt = 0, off_pair = 0, off_tap = 0;
  size_t off_ptb = 0, off_pib = 0, off_ptr = 0, off_pg = 0, meta_bytes = 0;
  size_t off_ctm[NRX_N_MODS][N_TILE_SIZES] = {}, off_rtm[NRX_N_MODS] = {};
  std::vector<char> blob;        // host image of the device tables
  void *pinned = nullptr;        // pinned copy, allocated on first upload
  void *packed_geo = nullptr;    // lmmse_demap: pinned geometry copy with h offsets into its workspace
  ~Plan() {
    // an asynchronous copy (or a graph replay) may still read the pinned tables
    if (pinned || packed_geo) (void)hipDeviceSynchronize();
    if (pinned) (void)hipHostFree(pinned);
    if (packed_geo) (void)hipHostFree(packed_geo);
  }
};
using PlanRef = std::shared_ptr<Plan>;

// A pinned host buffer; freed after the device has drained (an asynchronous copy may still read it).
struct PinnedBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  ~PinnedBuf() {
    if (ptr) {
      (void)hipDeviceSynchronize();
      (void)hipHostFree(ptr);
    }
  }
};

// Plans are keyed on every descriptor field (compared in full on a hit) and kept for the
// PLAN_CACHE_MAX most recently used batches; a model's graph or saved forward holds its plan alive
// after eviction.
constexpr size_t PLAN_CACHE_MAX = 256;
struct PlanCache {
  std::mutex mu;
  struct Entry { PlanRef plan; uint64_t used; };
  std::map<std::vector<int64_t>, Entry> plans;
  uint64_t tick = 0;
};

PlanCache g_plans;  // shared by model-free calls and models

std::vector<int64_t> plan_key(const nrx_slot_desc *d, int n, int sim_taps) {
  std::vector<int64_t> k;
  k.reserve(2 + (size_t)n * 18);
  k.push_back(n);
  k.push_back(sim_taps);
  for (int i = 0; i < n; ++i) {
    const nrx_slot_desc &s = d[i];
    int32_t n0b, offb;
    memcpy(&n0b, &s.n0, 4);
    memcpy(&offb, &s.snr_offset_db, 4);
    const int64_t f[] = {s.n_prb, s.n_ant, s.n_ue, s.bits_per_sym[0], s.bits_per_sym[1], s.bits_per_sym[2],
                         s.bits_per_sym[3], s.slot_number, s.n_id, s.n_scid, n0b, offb,
                         s.y_offset, s.h_offset, s.llr_offset, s.bits_offset};
    // UEs beyond n_ue do not take part: their bits_per_sym entries are not part of the key
    for (int j = 0; j < 16; ++j) k.push_back((j >= 3 + s.n_ue && j < 7) ? 0 : f[j]);
  }
  return k;
}

int num_cu();   // compute units of the current device (256 when it cannot be queried)

// Validates the descriptors of a batch.  max_ant bounds n_ant, m_max the bits per symbol.
nrx_status validate_slots(const nrx_slot_desc *d, int n, int max_ant, int m_max) {
  if (!d || n <= 0) return fail(NRX_ERR_INVALID, "no slot descriptors");
  for (int i = 0; i < n; ++i) {
    const nrx_slot_desc &s = d[i];
    if (s.n_prb < 1 || s.n_prb > 275) return fail(NRX_ERR_SHAPE, "slot %d: n_prb %d outside 1..275", i, s.n_prb);
    if (s.n_ant < 1 || s.n_ant > max_ant)
      return fail(NRX_ERR_SHAPE, "slot %d: n_ant %d outside 1..%d", i, s.n_ant, max_ant);
    if (s.n_ue < 1 || s.n_ue > 4) return fail(NRX_ERR_SHAPE, "slot %d: n_ue %d outside 1..4", i, s.n_ue);
    for (int u = 0; u < s.n_ue; ++u) {
      int m = s.bits_per_sym[u];
      if (m != 2 && m != 4 && m != 6 && m != 8) return fail(NRX_ERR_SHAPE, "slot %d UE %d: bits_per_sym %d", i, u, m);
      if (m > m_max) return fail(NRX_ERR_SHAPE, "slot %d UE %d: bits_per_sym %d > m_max %d", i, u, m, m_max);
    }
    if (s.n_scid < 0 || s.n_scid > 1 || s.n_id < 0 || s.n_id > 65535 || s.slot_number < 0 || s.slot_number > 1023)
      return fail(NRX_ERR_SHAPE, "slot %d: DMRS scrambling parameters out of range", i);
    if (s.y_offset < 0 || s.h_offset < 0 || s.llr_offset < 0 || s.bits_offset < 0)
      return fail(NRX_ERR_INVALID, "slot %d: negative offset", i);
    if (!(std::fabs(s.snr_offset_db) <= 60.f)) return fail(NRX_ERR_SHAPE, "slot %d: snr_offset_db outside -60..60", i);
    if (s.dmrs_sym_mask != 0 && s.dmrs_sym_mask != ((1u << NRX_DMRS0) | (1u << NRX_DMRS1)))
      return fail(NRX_ERR_UNSUPPORTED, "slot %d: dmrs_sym_mask 0x%x: only DMRS on symbols 2 and 11 is implemented", i,
                  s.dmrs_sym_mask);
  }
  return NRX_OK;
}

// Validates descriptors and builds (or fetches) the plan.  max_ant bounds n_ant.
nrx_status get_plan(const nrx_slot_desc *d, int n, int max_ant, int m_max, int sim_taps, PlanRef *out) {
  if (nrx_status v = validate_slots(d, n, max_ant, m_max)) return v;
  std::vector<int64_t> key = plan_key(d, n, sim_taps);
  PlanRef evicted;   // released after the lock (its destructor synchronises the device)
  std::lock_guard<std::mutex> lk(g_plans.mu);
  auto it = g_plans.plans.find(key);
  if (it != g_plans.plans.end()) {
    it->second.used = ++g_plans.tick;
    *out = it->second.plan;
    return NRX_OK;
  }
  if (g_plans.plans.size() >= PLAN_CACHE_MAX) {
    auto lru = g_plans.plans.begin();
    for (auto e = g_plans.plans.begin(); e != g_plans.plans.end(); ++e)
      if (e->second.used < lru->second.used) lru = e;
    evicted = std::move(lru->second.plan);
    g_plans.plans.erase(lru);
  }
  auto P = std::make_shared<Plan>();
  P->n = n;
  int64_t row = 0, dm = 0, pr = 0, tp = 0;
  for (int i = 0; i < n; ++i) {
    const nrx_slot_desc &s = d[i];
    SlotGeo g{};
    g.S = 12 * s.n_prb;
    g.U = s.n_ue;
    g.B = s.n_ant;
    for (int u = 0; u < 4; ++u) g.m[u] = u < s.n_ue ? s.bits_per_sym[u] : 0;
    g.slot_number = s.slot_number;
    g.n_id = s.n_id;
    g.n_scid = s.n_scid;
    g.n0 = s.n0;
    g.snr_off = s.snr_offset_db;
    g.row_base = row;
    g.y_off = s.y_offset;
    g.h_off = s.h_offset;
    g.llr_off = s.llr_offset;
    g.bits_off = s.bits_offset;
    g.dmrs_off = dm;
    P->geo.push_back(g);
    const int64_t rows = (int64_t)g.S * 14 * g.U;
    for (int k = 0; k < N_TILE_SIZES; ++k) {
      const int tr = tile_rows_of_index(k);
      for (int64_t r = 0; r < rows; r += tr)
        P->ct[k].push_back(Tile{i, (int32_t)r, (int32_t)std::min<int64_t>(tr, rows - r), 0});
    }
    const int mtr = (MLP_TILE / g.U) * g.U;
    for (int64_t r = 0; r < rows; r += mtr)
      P->mt.push_back(Tile{i, (int32_t)r, (int32_t)std::min<int64_t>(mtr, rows - r), 0});
    for (int64_t r = 0; r < rows; r += MLP_TILE)
      P->rt.push_back(Tile{i, (int32_t)r, (int32_t)std::min<int64_t>(MLP_TILE, rows - r), 0});
    P->pair_off.push_back(pr);
    P->tap_off.push_back(tp);
    const int64_t npairs = 2LL * g.U * (g.S / 4) * g.B;
    const int ubl = g.U * g.B * std::max(sim_taps, 1);
    row += rows;
    dm += g.S;
    pr += npairs;
    tp += (int64_t)ubl * 14;
    P->max_rows = std::max(P->max_rows, rows);
    P->max_re = std::max<int64_t>(P->max_re, (int64_t)g.S * 14);
    P->max_pairs = std::max(P->max_pairs, npairs);
    P->max_ute = std::max<int64_t>(P->max_ute, (int64_t)g.U * 14 * g.S);
    P->max_bits = std::max<int64_t>(P->max_bits, (int64_t)g.U * 12 * g.S);
    P->max_ubl = std::max(P->max_ubl, ubl);
    int nb = 0;
    for (int u = 0; u < g.U; ++u) nb += g.m[u];
    P->n_data_bits += (int64_t)nb * 12 * g.S;
  }
  P->pair_off.push_back(pr);
  P->tap_off.push_back(tp);
  {
    int32_t tb = 0, ib = 0, in_group = 0;
    std::vector<int32_t> cnt(n);
    for (int i = 0; i < n; ++i) {
      const int U = P->geo[i].U;
      const int tr = (PERSIST_TILE / U) * U;
      const int64_t rows_i = (int64_t)P->geo[i].S * 14 * U;
      cnt[i] = (int32_t)((rows_i + tr - 1) / tr);
      P->ptile_rows.push_back(tr);
      tb += cnt[i];
    }
    // several tiles per item amortise an item's start (claim, waits, pipeline fill) in large batches; a
    // small batch (one slot in the real-time regime) keeps one tile per item so that it fills the device
    P->pitem_tiles = std::max(1, std::min(PERSIST_ITEM_TILES, tb / (4 * num_cu())));
    tb = 0;
    P->pgroup.push_back(0);
    for (int i = 0; i < n; ++i) {
      P->ptile_base.push_back(tb);
      P->pitem_base.push_back(ib);
      tb += cnt[i];
      ib += (cnt[i] + P->pitem_tiles - 1) / P->pitem_tiles;
      in_group += cnt[i];
      if (in_group >= PERSIST_GROUP && i + 1 < n) { P->pgroup.push_back(i + 1); in_group = 0; }
    }
    P->ptile_base.push_back(tb);
    P->pitem_base.push_back(ib);
    P->pgroup.push_back(n);
  }
  P->rows = row;
  P->dmrs_total = dm;
  P->pairs_total = pr;
  {
    std::vector<int> slot_mods(n, 0);   // bit mi: the slot has a UE of modulation 2 (mi + 1)
    int all = 0;
    for (int i = 0; i < n; ++i) {
      for (int u = 0; u < P->geo[i].U; ++u) slot_mods[i] |= 1 << (P->geo[i].m[u] / 2 - 1);
      all |= slot_mods[i];
    }
    P->mod_lists = __builtin_popcount(all) > 1;
    if (P->mod_lists)
      for (int mi = 0; mi < NRX_N_MODS; ++mi) {
        if (!(all >> mi & 1)) continue;
        for (int k = 0; k < N_TILE_SIZES; ++k)
          for (const Tile &t : P->ct[k])
            if (slot_mods[t.slot] >> mi & 1) P->ctm[mi][k].push_back(t);
        for (const Tile &t : P->rt)
          if (slot_mods[t.slot] >> mi & 1) P->rtm[mi].push_back(t);
      }
  }
  size_t o = 0;
  P->off_geo = o; o = align256(o + sizeof(SlotGeo) * P->geo.size());
  for (int k = 0; k < N_TILE_SIZES; ++k) { P->off_ct[k] = o; o = align256(o + sizeof(Tile) * P->ct[k].size()); }
  P->off_mt = o; o = align256(o + sizeof(Tile) * P->mt.size());
  P->off_rt = o; o = align256(o + sizeof(Tile) * P->rt.size());
  P->off_pair = o; o = align256(o + sizeof(int64_t) * P->pair_off.size());
  P->off_tap = o; o = align256(o + sizeof(int64_t) * P->tap_off.size());
  P->off_ptb = o; o = align256(o + sizeof(int32_t) * P->ptile_base.size());
  P->off_pib = o; o = align256(o + sizeof(int32_t) * P->pitem_base.size());
  P->off_ptr = o; o = align256(o + sizeof(int32_t) * P->ptile_rows.size());
  P->off_pg = o; o = align256(o + sizeof(int32_t) * P->pgroup.size());
  for (int mi = 0; mi < NRX_N_MODS; ++mi) {
    for (int k = 0; k < N_TILE_SIZES; ++k) { P->off_ctm[mi][k] = o; o = align256(o + sizeof(Tile) * P->ctm[mi][k].size()); }
    P->off_rtm[mi] = o; o = align256(o + sizeof(Tile) * P->rtm[mi].size());
  }
  P->meta_bytes = o;
  P->blob.assign(o, 0);
  char *b = P->blob.data();
  memcpy(b + P->off_geo, P->geo.data(), sizeof(SlotGeo) * P->geo.size());
  for (int k = 0; k < N_TILE_SIZES; ++k) memcpy(b + P->off_ct[k], P->ct[k].data(), sizeof(Tile) * P->ct[k].size());
  memcpy(b + P->off_mt, P->mt.data(), sizeof(Tile) * P->mt.size());
  memcpy(b + P->off_rt, P->rt.data(), sizeof(Tile) * P->rt.size());
  memcpy(b + P->off_pair, P->pair_off.data(), sizeof(int64_t) * P->pair_off.size());
  memcpy(b + P->off_tap, P->tap_off.data(), sizeof(int64_t) * P->tap_off.size());
  memcpy(b + P->off_ptb, P->ptile_base.data(), sizeof(int32_t) * P->ptile_base.size());
  memcpy(b + P->off_pib, P->pitem_base.data(), sizeof(int32_t) * P->pitem_base.size());
  memcpy(b + P->off_ptr, P->ptile_rows.data(), sizeof(int32_t) * P->ptile_rows.size());
  memcpy(b + P->off_pg, P->pgroup.data(), sizeof(int32_t) * P->pgroup.size());
  for (int mi = 0; mi < NRX_N_MODS; ++mi) {
    for (int k = 0; k < N_TILE_SIZES; ++k)
      memcpy(b + P->off_ctm[mi][k], P->ctm[mi][k].data(), sizeof(Tile) * P->ctm[mi][k].size());
    memcpy(b + P->off_rtm[mi], P->rtm[mi].data(), sizeof(Tile) * P->rtm[mi].size());
  }
  *out = P;
  g_plans.plans[std::move(key)] = PlanCache::Entry{std::move(P), ++g_plans.tick};
  return NRX_OK;
}

// Enqueues the copy of the plan's device tables into the workspace.
nrx_status plan_upload(Plan *P, char *dst, hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(g_plans.mu);
    if (!P->pinned) {
      if (hipHostMalloc(&P->pinned, P->meta_bytes, hipHostMallocDefault) != hipSuccess)
        return fail(NRX_ERR_HIP, "hipHostMalloc of %zu bytes failed", P->meta_bytes);
      memcpy(P->pinned, P->blob.data(), P->meta_bytes);
    }
  }
  HIPCHK(hipMemcpyAsync(dst, P->pinned, P->meta_bytes, hipMemcpyHostToDevice, st));
  return NRX_OK;
}

struct Dev {
  const SlotGeo *geo;
  const Tile *ct[N_TILE_SIZES], *mt, *rt;
  const Tile *ctm[NRX_N_MODS][N_TILE_SIZES], *rtm[NRX_N_MODS];
  const int64_t *pair_off, *tap_off;
  const int32_t *ptile_base, *pitem_base, *ptile_rows, *pgroup;
};

Dev dev_tables(const Plan *P, char *ws) {
  Dev d;
  d.geo = (const SlotGeo *)(ws + P->off_geo);
  for (int k = 0; k < N_TILE_SIZES; ++k) d.ct[k] = (const Tile *)(ws + P->off_ct[k]);
  d.mt = (const Tile *)(ws + P->off_mt);
  d.rt = (const Tile *)(ws + P->off_rt);
  d.pair_off = (const int64_t *)(ws + P->off_pair);
  d.tap_off = (const int64_t *)(ws + P->off_tap);
  d.ptile_base = (const int32_t *)(ws + P->off_ptb);
  d.pitem_base = (const int32_t *)(ws + P->off_pib);
  d.ptile_rows = (const int32_t *)(ws + P->off_ptr);
  d.pgroup = (const int32_t *)(ws + P->off_pg);
  for (int mi = 0; mi < NRX_N_MODS; ++mi) {
    for (int k = 0; k < N_TILE_SIZES; ++k) d.ctm[mi][k] = (const Tile *)(ws + P->off_ctm[mi][k]);
    d.rtm[mi] = (const Tile *)(ws + P->off_rtm[mi]);
  }
  return d;
}

int g_num_cu = 0;
int num_cu() {
  if (!g_num_cu) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) g_num_cu = p.multiProcessorCount;
    if (g_num_cu <= 0) g_num_cu = 256;
  }
  return g_num_cu;
}

// captured forward launch sequences, keyed by batch plan and buffer addresses
struct GraphKey {
  const void *plan, *w, *y, *h, *llr, *ws;
  bool save;
  uint64_t variants;   // conv kernel variant per layer class, 4 bits each
  uint64_t epoch;      // FP8 activation-scale version (scales are kernel arguments)
  int iters;           // CGNN iterations run
  int64_t llr_stride;  // > 0: a readout after every iteration
  const void *hest;    // ReadoutChEst output or null
  int64_t h_stride;
  bool operator<(const GraphKey &o) const {
    return std::tie(plan, w, y, h, llr, ws, save, variants, epoch, iters, llr_stride, hest, h_stride) <
           std::tie(o.plan, o.w, o.y, o.h, o.llr, o.ws, o.save, o.variants, o.epoch, o.iters, o.llr_stride, o.hest,
                    o.h_stride);
  }
};

constexpr size_t GRAPH_CACHE_MAX = 64;   // captured forward graphs kept per model (least recently used evicted)
struct Graphs {
  hipStream_t cap = nullptr;
  // the plan's pinned tables (and a persistent forward's stage table) feed the graph
  struct Entry { hipGraphExec_t exec; PlanRef plan; uint64_t used; std::shared_ptr<PinnedBuf> ptable; };
  std::map<GraphKey, Entry> execs;
  uint64_t tick = 0;
};

}  // namespace

// ------------------------------------------------------------------- model --

struct nrx_model {
  nrx_model_config cfg;
  std::vector<TensorInfo> tensors;
  int64_t n_w = 0;
  int cx = 0;                           // feature channels of the StateInit input
  // StateInit: one shared (m = 0), or under Var-IO one per modulation m = 2, 4, .. m_max
  struct StateInit { ConvLayer c; int m; };
  std::vector<StateInit> cins;
  std::vector<BlockLayer> blocks;
  std::vector<DenseLayer> mp;
  // ReadoutLLRs: one shared layer (m = 0, m_max outputs, masked to m_u), or under Var-IO (flags bit 2)
  // one per modulation m = 2, 4, .. m_max with m outputs, each applied to the UEs of its modulation
  struct Readout { DenseLayer l; int m; };
  std::vector<Readout> ros;
  bool chest = false;                   // flags bit 1: second readout ReadoutChEst (double readout)
  DenseLayer ro_ch;
  std::vector<PrepJob> jobs;
  int64_t prep_elems = 0, field_elems = 0, prep_total = 0;
  void *pinned_jobs = nullptr;
  std::vector<PrepJob> bjobs;           // backward weight preparation
  int64_t bprep_elems = 0;
  void *pinned_bjobs = nullptr;
  size_t tsize = 4;                     // bytes per activation / operand element
  Graphs *graphs = nullptr;        // captured forward graphs (flags bit 0)
  // FP8 models: E4M3 conv operands with per-layer activation scales
  //   act_scale[i] (i < C): input h_i of block i; [C + i]: conv_a output of block i;
  //   [2C + r]: aggregated messages of round r
  bool fp8 = false;
  bool calibrating = false;             // forward records max |activation| instead of using FP8
  int fp8_layers = 3;                   // FP8 models: bit 0 conv_a / conv_a_mp in E4M3, bit 1 conv_b
  bool calibrated = false;
  std::vector<float> act_scale;
  uint64_t scale_epoch = 0;
  int64_t w8_bytes = 0, n_wscale = 0;
  std::vector<Fp8Job> fp8jobs;
  void *pinned_fp8jobs = nullptr;
  std::vector<void *> retired_pinned;   // job tables replaced while copies may be in flight
  // conv kernel variant per layer class (autotuned; indices into kConvVariants)
  int conv_variant[NRX_K_NCLASS] = {1, 1, 1, 1, 1, 1, 1};
  // per-class event timing (diagnostics)
  bool profile = false;
  struct Ev { int cls; hipEvent_t a, b; };
  std::vector<Ev> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[NRX_K_NCLASS] = {0};
  int64_t prof_n[NRX_K_NCLASS] = {0};
  // CGNN iterations run by the forward (inference-time depth control, Sec. IV-B); 0 = all
  int n_iter = 0;
  // last save_acts forward (for nrx_backward): its workspace, batch, depth and readouts kept
  const void *saved_ws = nullptr;
  PlanRef saved_plan;                   // held: an evicted plan's address is not reused while it is saved
  int64_t save_seq = 0;                 // save_acts forwards run so far (the token of the last one)
  int saved_iters = 0;
  bool saved_multi = false;
  bool saved_chest = false;
  // persistent forward (flags bit 3): stage tables by contents, and the one the last forward used
  struct PTable { std::shared_ptr<PinnedBuf> buf; uint64_t used; };
  std::map<std::string, PTable> ptables;
  uint64_t ptable_tick = 0;
  std::shared_ptr<PinnedBuf> last_ptable;
  std::mutex mu;
};

static void add_tensor(nrx_model *m, const std::string &name, std::vector<int> shape) {
  TensorInfo t;
  t.name = name;
  t.off = m->n_w;
  t.ndim = (int)shape.size();
  int64_t n = 1;
  for (int i = 0; i < 4; ++i) t.shape[i] = i < t.ndim ? shape[i] : 1;
  for (int v : shape) n *= v;
  m->tensors.push_back(t);
  m->n_w += n;
}

static int64_t toff(nrx_model *m, const std::string &name) {
  for (auto &t : m->tensors)
    if (t.name == name) return t.off;
  return -1;
}

extern "C" nrx_status nrx_model_create(const nrx_model_config *cfg, nrx_model **out) {
  if (!cfg || !out) return fail(NRX_ERR_INVALID, "null argument");
  const nrx_model_config &c = *cfg;
  if (c.d < 8 || c.d > NRX_D || c.d % 8) return fail(NRX_ERR_SHAPE, "d = %d: state depth must be a multiple of 8 in 8..128", c.d);
  if (c.n_ant != 4 && c.n_ant != 8 && c.n_ant != 16) return fail(NRX_ERR_SHAPE, "n_ant %d not in {4, 8, 16}", c.n_ant);
  if (c.n_blocks < 1 || c.n_blocks > 16) return fail(NRX_ERR_SHAPE, "n_blocks %d outside 1..16", c.n_blocks);
  if (c.n_rounds < 0 || c.n_rounds > c.n_blocks) return fail(NRX_ERR_SHAPE, "n_rounds %d outside 0..n_blocks", c.n_rounds);
  if (c.m_max != 2 && c.m_max != 4 && c.m_max != 6 && c.m_max != 8) return fail(NRX_ERR_SHAPE, "m_max %d", c.m_max);
  if (c.precision != NRX_FP32 && c.precision != NRX_BF16 && c.precision != NRX_FP8)
    return fail(NRX_ERR_UNSUPPORTED, "precision %d not available", c.precision);
  if (c.precision == NRX_FP8 && c.d != NRX_D) return fail(NRX_ERR_UNSUPPORTED, "FP8 models need d = 128");
  if ((c.flags & 8) && (c.precision != NRX_BF16 || (c.flags & 4)))
    return fail(NRX_ERR_UNSUPPORTED, "the persistent forward (flags bit 3) runs BF16 models with shared input and output layers");
  if (c.flags & ~15) return fail(NRX_ERR_INVALID, "unknown model flags 0x%x", c.flags);
  if ((c.flags & 2) && c.n_ant > 8)
    return fail(NRX_ERR_SHAPE, "ReadoutChEst has 2 n_ant outputs, at most 16: n_ant %d > 8", c.n_ant);
  auto m = std::make_unique<nrx_model>();
  m->chest = (c.flags & 2) != 0;
  m->cfg = c;
  m->tsize = c.precision == NRX_FP32 ? 4 : 2;   // FP8 models keep BF16 for everything but the block convs
  m->fp8 = c.precision == NRX_FP8;
  // convolution variants until nrx_conv_variant / nrx_autotune choose others: the fastest at the headline
  // batch (BF16 ring kernel with SIMD-levelled wave priority; the first E4M3 kernel for FP8 block convs)
  for (int cls = NRX_K_CONV_IN; cls <= NRX_K_CONV_B; ++cls)
    m->conv_variant[cls] = m->fp8 && cls != NRX_K_CONV_IN ? CONV8_DEFAULT_VARIANT : CONV_DEFAULT_VARIANT;
  const int d = c.d, B = c.n_ant;
  m->cx = std::max(32, 4 * B);
  std::vector<int> mpb;
  for (int r = 0; r < c.n_rounds; ++r) mpb.push_back((r * c.n_blocks) / c.n_rounds);
  std::vector<int> io_mods;   // modulation of each StateInit / ReadoutLLRs (0: shared)
  if (c.flags & 4)
    for (int mm = 2; mm <= c.m_max; mm += 2) io_mods.push_back(mm);
  else
    io_mods.push_back(0);
  auto io_prefix = [](const char *layer, int mm) {
    return mm ? std::string(layer) + ".m" + std::to_string(mm) + "." : std::string(layer) + ".";
  };
  for (int mm : io_mods) {
    add_tensor(m.get(), io_prefix("conv_in", mm) + "w", {3, 3, 4 * B + 2, d});
    add_tensor(m.get(), io_prefix("conv_in", mm) + "b", {d});
  }
  for (int i = 0; i < c.n_blocks; ++i) {
    bool ismp = false;
    for (int v : mpb) ismp = ismp || v == i;
    const int cin = ismp ? 2 * d + 2 : d;
    const std::string p = "blk" + std::to_string(i);
    add_tensor(m.get(), p + ".conv_a.w", {3, 3, cin, d});
    add_tensor(m.get(), p + ".conv_a.b", {d});
    add_tensor(m.get(), p + ".ln.g", {d});
    add_tensor(m.get(), p + ".ln.b", {d});
    add_tensor(m.get(), p + ".conv_b.w", {3, 3, d, d});
    add_tensor(m.get(), p + ".conv_b.b", {d});
  }
  for (int r = 0; r < c.n_rounds; ++r) {
    const std::string p = "mp" + std::to_string(r);
    add_tensor(m.get(), p + ".w1", {d, d});
    add_tensor(m.get(), p + ".b1", {d});
    add_tensor(m.get(), p + ".w2", {d, d});
    add_tensor(m.get(), p + ".b2", {d});
  }
  for (int mm : io_mods) {
    const std::string p = io_prefix("readout", mm);
    add_tensor(m.get(), p + "w1", {d, d});
    add_tensor(m.get(), p + "b1", {d});
    add_tensor(m.get(), p + "w2", {d, mm ? mm : c.m_max});
    add_tensor(m.get(), p + "b2", {mm ? mm : c.m_max});
  }
  if (m->chest) {   // appended, so a weight vector without them is a prefix of this one
    add_tensor(m.get(), "readout_ch.w1", {d, d});
    add_tensor(m.get(), "readout_ch.b1", {d});
    add_tensor(m.get(), "readout_ch.w2", {d, 2 * B});
    add_tensor(m.get(), "readout_ch.b2", {2 * B});
  }

  // weight preparation jobs
  const int KC = 64 / (int)m->tsize;
  // seg: master input channels per 128-wide activation segment (block convs: d; StateInit: identity)
  auto conv_job = [&](ConvLayer &L, int64_t w, int64_t b, int cin_real, int cin_total, int cin_pad, bool pe, int seg) {
    L.w = w; L.b = b; L.cin_real = cin_real; L.cin_total = cin_total; L.n_chunks = cin_pad / KC;
    L.prep = m->prep_elems;
    PrepJob j{0, cin_real, cin_total, L.n_chunks, 0, 0, w, L.prep, (int64_t)cin_pad * 9 * 128, d, seg};
    m->jobs.push_back(j);
    m->prep_elems += j.count;
    if (pe) {
      L.field = m->field_elems;
      PrepJob f{2, cin_real, cin_total, 0, 0, 0, w, L.field, 2 * 3 * 14 * 128, d, 0};
      m->jobs.push_back(f);
      m->field_elems += f.count;
    }
  };
  auto dense_job = [&](int64_t w, int64_t &p) {
    p = m->prep_elems;
    PrepJob j{1, d, d, NRX_D / KC, 0, 0, w, p, (int64_t)NRX_D * 128, d, 0};
    m->jobs.push_back(j);
    m->prep_elems += j.count;
  };
  // d < 128: vectors padded with zeros, placed in the field buffer after the PE fields
  std::vector<std::pair<int64_t, int64_t *>> pads;
  auto pad_vec = [&](int64_t src, int64_t *dst) { if (d < NRX_D) pads.push_back({src, dst}); };
  m->cins.resize(io_mods.size());
  for (size_t i = 0; i < io_mods.size(); ++i) {
    m->cins[i].m = io_mods[i];
    conv_job(m->cins[i].c, toff(m.get(), io_prefix("conv_in", io_mods[i]) + "w"),
             toff(m.get(), io_prefix("conv_in", io_mods[i]) + "b"), 4 * B, 4 * B + 2, m->cx, true, 0);
  }
  m->mp.resize(c.n_rounds);
  for (int i = 0; i < c.n_blocks; ++i) {
    const std::string p = "blk" + std::to_string(i);
    BlockLayer L;
    for (int r = 0; r < c.n_rounds; ++r)
      if (mpb[r] == i) L.mp_round = r;
    const bool isb = L.mp_round >= 0;
    conv_job(L.a, toff(m.get(), p + ".conv_a.w"), toff(m.get(), p + ".conv_a.b"), isb ? 2 * d : d,
             isb ? 2 * d + 2 : d, isb ? 2 * NRX_D : NRX_D, isb, d);
    L.g = toff(m.get(), p + ".ln.g");
    L.beta = toff(m.get(), p + ".ln.b");
    conv_job(L.b, toff(m.get(), p + ".conv_b.w"), toff(m.get(), p + ".conv_b.b"), d, d, NRX_D, false, d);
    if (m->fp8) {
      for (ConvLayer *cl : {&L.a, &L.b}) {
        cl->w8 = m->w8_bytes;
        m->w8_bytes += (int64_t)(cl->cin_real / 64) * 5 * 8 * 16 * 128;
        cl->ws8 = m->n_wscale;
        m->n_wscale += NRX_D;
      }
    }
    m->blocks.push_back(L);
  }
  if (m->fp8) m->act_scale.assign(2 * c.n_blocks + c.n_rounds, 1.0f);
  for (int r = 0; r < c.n_rounds; ++r) {
    const std::string p = "mp" + std::to_string(r);
    DenseLayer &L = m->mp[r];
    L.w1 = toff(m.get(), p + ".w1"); L.b1 = toff(m.get(), p + ".b1");
    L.w2 = toff(m.get(), p + ".w2"); L.b2 = toff(m.get(), p + ".b2");
    dense_job(L.w1, L.p1);
    dense_job(L.w2, L.p2);
  }
  for (int mm : io_mods) {
    const std::string p = io_prefix("readout", mm);
    nrx_model::Readout R;
    R.m = mm;
    R.l.w1 = toff(m.get(), p + "w1"); R.l.b1 = toff(m.get(), p + "b1");
    R.l.w2 = toff(m.get(), p + "w2"); R.l.b2 = toff(m.get(), p + "b2");
    dense_job(R.l.w1, R.l.p1);
    R.l.p2 = m->prep_elems;
    PrepJob j{4, d, d, NRX_D / KC, 0, mm ? mm : c.m_max, R.l.w2, R.l.p2, (int64_t)NRX_D * 16, d, 0};
    m->jobs.push_back(j);
    m->prep_elems += j.count;
    m->ros.push_back(R);
  }
  if (m->chest) {
    DenseLayer &L = m->ro_ch;
    L.w1 = toff(m.get(), "readout_ch.w1"); L.b1 = toff(m.get(), "readout_ch.b1");
    L.w2 = toff(m.get(), "readout_ch.w2"); L.b2 = toff(m.get(), "readout_ch.b2");
    dense_job(L.w1, L.p1);
    L.p2 = m->prep_elems;
    PrepJob j{4, d, d, NRX_D / KC, 0, 2 * B, L.w2, L.p2, (int64_t)NRX_D * 16, d, 0};
    m->jobs.push_back(j);
    m->prep_elems += j.count;
  }
  // backward jobs: flipped/transposed conv weights and transposed dense weights
  auto bjob = [&](int kind, int64_t src, int cin_total, int cin_first, int64_t count) {
    const int64_t off = m->bprep_elems;
    m->bjobs.push_back(PrepJob{kind, d, cin_total, d / KC, cin_first, 0, src, off, count, d, 0});
    m->bprep_elems += count;
    return off;
  };
  for (int i = 0; i < c.n_blocks; ++i) {
    BlockLayer &L = m->blocks[i];
    L.bg_b = bjob(3, L.b.w, d, 0, 9LL * 128 * d);
    L.bg_a_h = bjob(3, L.a.w, L.a.cin_total, 0, 9LL * 128 * d);
    if (L.mp_round >= 0) L.bg_a_agg = bjob(3, L.a.w, L.a.cin_total, d, 9LL * 128 * d);
  }
  for (int r = 0; r < c.n_rounds; ++r) {
    m->mp[r].t1 = bjob(5, m->mp[r].w1, d, 0, (int64_t)d * 128);
    m->mp[r].t2 = bjob(5, m->mp[r].w2, d, 0, (int64_t)d * 128);
  }
  for (auto &R : m->ros) R.l.t1 = bjob(5, R.l.w1, d, 0, (int64_t)d * 128);
  if (m->chest) m->ro_ch.t1 = bjob(5, m->ro_ch.w1, d, 0, (int64_t)d * 128);
  if (d < NRX_D) {
    for (auto &ci : m->cins) pad_vec(ci.c.b, &ci.c.bpad);
    for (auto &L : m->blocks) {
      pad_vec(L.a.b, &L.a.bpad);
      pad_vec(L.b.b, &L.b.bpad);
      pad_vec(L.g, &L.gpad);
      pad_vec(L.beta, &L.betapad);
    }
    for (auto &L : m->mp) { pad_vec(L.b1, &L.b1pad); pad_vec(L.b2, &L.b2pad); }
    for (auto &R : m->ros) pad_vec(R.l.b1, &R.l.b1pad);
    if (m->chest) pad_vec(m->ro_ch.b1, &m->ro_ch.b1pad);
    for (auto &pv : pads) {
      *pv.second = m->field_elems;
      m->jobs.push_back(PrepJob{6, d, d, 0, 0, 0, pv.first, m->field_elems, NRX_D, d, 0});
      m->field_elems += NRX_D;
    }
  }
  // field jobs index a separate buffer; the prep kernel walks jobs in order over one index space
  m->prep_total = 0;
  for (auto &j : m->jobs) m->prep_total += j.count;
  *out = m.release();
  return NRX_OK;
}

extern "C" nrx_status nrx_model_destroy(nrx_model *m) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  if (m->graphs) {
    if (!m->graphs->execs.empty()) (void)hipDeviceSynchronize();   // no replay may still run
    for (auto &kv : m->graphs->execs) (void)hipGraphExecDestroy(kv.second.exec);
    if (m->graphs->cap) (void)hipStreamDestroy(m->graphs->cap);
    delete m->graphs;
  }
  if (m->pinned_bjobs) (void)hipHostFree(m->pinned_bjobs);
  for (auto &e : m->pending) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  for (auto e : m->pool) (void)hipEventDestroy(e);
  if (m->pinned_jobs) (void)hipHostFree(m->pinned_jobs);
  if (m->pinned_fp8jobs) (void)hipHostFree(m->pinned_fp8jobs);
  for (void *p : m->retired_pinned) (void)hipHostFree(p);
  delete m;
  return NRX_OK;
}

extern "C" int64_t nrx_weight_count(const nrx_model *m) { return m ? m->n_w : -1; }

extern "C" nrx_status nrx_weight_tensor(const nrx_model *m, int32_t idx, char *name, int32_t name_len, int64_t *offset,
                                        int32_t *ndim, int32_t shape[4]) {
  if (!m || idx < 0 || idx >= (int)m->tensors.size()) return fail(NRX_ERR_INVALID, "tensor index out of range");
  const TensorInfo &t = m->tensors[idx];
  if (name && name_len > 0) snprintf(name, name_len, "%s", t.name.c_str());
  if (offset) *offset = t.off;
  if (ndim) *ndim = t.ndim;
  if (shape)
    for (int i = 0; i < 4; ++i) shape[i] = t.shape[i];
  return NRX_OK;
}

// -------------------------------------------------------- forward workspace --

namespace {

// Blocks completed at the end of each CGNN iteration: iteration r is message-passing round r and
// the state-update blocks up to the next round (Sec. II-A); without message passing the whole
// stack is one iteration.
// Does a UE of the batch use modulation m (bits per symbol)?  (Var-IO runs only those layers.)
bool batch_uses(const Plan *P, int m) {
  for (auto &g : P->geo)
    for (int u = 0; u < g.U; ++u)
      if (g.m[u] == m) return true;
  return false;
}

std::vector<int> iteration_ends(const nrx_model_config &c) {
  std::vector<int> e;
  if (c.n_rounds == 0) e.push_back(c.n_blocks);
  for (int r = 0; r < c.n_rounds; ++r) e.push_back(((r + 1) * c.n_blocks) / c.n_rounds);
  return e;
}

struct FwdLayout {
  size_t meta, jobs, wprep, fields, dmrs, pairs, X, done, stamps, flags;   // the same for save and inference
  size_t pstages = 0, pctl = 0;   // persistent forward (model flags bit 3, inference): stage table, control words
  size_t h8 = 0, a8 = 0, agg8 = 0, w8 = 0, wsc = 0, f8jobs = 0, amax = 0;   // FP8 models
  std::vector<size_t> h;      // h_0 .. h_C (inference: one buffer)
  std::vector<size_t> z, a;   // per block (inference: one a buffer, no z)
  std::vector<size_t> stats;  // per block (training)
  std::vector<size_t> agg, m1;  // per round (inference: one agg)
  std::vector<size_t> q;      // readout hidden after each CGNN iteration (training)
  std::vector<size_t> q_ch;   // the same for ReadoutChEst
  // backward (training layout only)
  size_t bjobs = 0, bprep = 0, zero = 0, dh = 0, dz = 0, dagg = 0, dmsg = 0, dm1 = 0, dr = 0;
  size_t wpart = 0, cpart = 0, lpart = 0, rpart = 0;
  size_t total;
};

// stages of the persistent forward: StateInit, message-passing rounds, two convs per block, readout
int persist_stages(const nrx_model *m) { return 2 + m->cfg.n_rounds + 2 * m->cfg.n_blocks; }

constexpr int WGRAD_PARTS = 512;      // bound on row partitions of the weight-gradient kernel
constexpr int BWD_GRID_MAX = 4096;    // bound on per-workgroup partial buffers

FwdLayout fwd_layout(const nrx_model *m, const Plan *P, bool save) {
  FwdLayout L;
  const size_t ts = m->tsize;
  const size_t act = align256((size_t)P->rows * NRX_D * ts);
  size_t o = 0;
  L.meta = o; o = align256(o + P->meta_bytes);
  L.jobs = o; o = align256(o + sizeof(PrepJob) * m->jobs.size());
  L.wprep = o; o = align256(o + (size_t)m->prep_elems * ts);
  L.fields = o; o = align256(o + (size_t)std::max<int64_t>(m->field_elems, 1) * 4);
  L.dmrs = o; o = align256(o + (size_t)P->dmrs_total * 8);
  L.pairs = o; o = align256(o + (size_t)P->pairs_total * 8);
  L.X = o; o = align256(o + (size_t)P->rows * m->cx * ts);
  L.done = o; o = align256(o + (size_t)P->n * 4);
  L.stamps = o; o = align256(o + (size_t)(P->n + 1) * 8);
  L.flags = o; o = align256(o + (size_t)P->n * 4);
  const int C = m->cfg.n_blocks, R = m->cfg.n_rounds;
  if ((m->cfg.flags & 8) && !save) {
    const int ns = persist_stages(m);
    L.pstages = o; o = align256(o + sizeof(PersistStage) * ns);
    // two control words (claim counter, abort), then one finished flag per (stage, tile)
    L.pctl = o; o = align256(o + 4 * (64 + (size_t)ns * P->ptile_base.back()));
  }
  if (m->fp8) {
    const size_t act8 = align256((size_t)P->rows * NRX_D);
    L.h8 = o; o += act8;
    L.a8 = o; o += act8;
    L.agg8 = o; o += act8;
    L.w8 = o; o = align256(o + (size_t)m->w8_bytes);
    L.wsc = o; o = align256(o + (size_t)m->n_wscale * 4);
    L.f8jobs = o; o = align256(o + sizeof(Fp8Job) * 2 * C);
    L.amax = o; o = align256(o + m->act_scale.size() * 4);
  }
  if (!save) {
    L.h.push_back(o); o += act;
    L.a.push_back(o); o += act;
    L.agg.push_back(o); o += act;
  } else {
    for (int i = 0; i <= C; ++i) { L.h.push_back(o); o += act; }
    for (int i = 0; i < C; ++i) { L.z.push_back(o); o += act; }
    for (int i = 0; i < C; ++i) { L.a.push_back(o); o += act; }
    for (int i = 0; i < C; ++i) { L.stats.push_back(o); o = align256(o + (size_t)P->rows * 8); }
    for (int r = 0; r < R; ++r) { L.agg.push_back(o); o += act; }
    for (int r = 0; r < R; ++r) { L.m1.push_back(o); o += act; }
    for (size_t k = 0; k < iteration_ends(m->cfg).size(); ++k) { L.q.push_back(o); o += act; }
    if (m->chest)
      for (size_t k = 0; k < iteration_ends(m->cfg).size(); ++k) { L.q_ch.push_back(o); o += act; }
    L.bjobs = o; o = align256(o + sizeof(PrepJob) * m->bjobs.size());
    L.bprep = o; o = align256(o + (size_t)m->bprep_elems * ts);
    L.zero = o; o = align256(o + 128 * 4);
    L.dh = o; o += act;
    L.dz = o; o += act;
    L.dagg = o; o += act;
    L.dmsg = o; o += act;
    L.dm1 = o; o += act;
    L.dr = o; o += act;
    // partitions x (taps x slices) 128x128 partial blocks: <= 2 per CU for the one-tap-per-workgroup kernel,
    // <= 3 per CU for the three-tap kernel (one workgroup per CU)
    L.wpart = o; o = align256(o + (size_t)3 * num_cu() * 128 * 128 * 4);
    L.cpart = o; o = align256(o + (size_t)(P->n + 1) * 14 * 768 * 4);   // per-slot partials + reduced table
    L.lpart = o; o = align256(o + (size_t)BWD_GRID_MAX * 256 * 4);
    // dW2 partials: one set per readout for ReadoutLLRs, two (column groups) for ReadoutChEst
    L.rpart = o;
    o = align256(o + (m->ros.size() + (m->chest ? 2 : 0)) * iteration_ends(m->cfg).size() * BWD_GRID_MAX * 1032 * 4);
  }
  L.total = o;
  return L;
}

// Brackets a launch with events when profiling is on.
struct ProfMark {
  nrx_model *m;
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t get(nrx_model *m) {
    if (!m->pool.empty()) { hipEvent_t e = m->pool.back(); m->pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  ProfMark(nrx_model *mm, int c, hipStream_t s) : m(mm), cls(c), st(s) {
    if (!m->profile) return;
    a = get(m); b = get(m);
    (void)hipEventRecord(a, st);
  }
  ~ProfMark() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    m->pending.push_back({cls, a, b});
  }
};

// pinned copy of the preparation job table (allocated on first use: model creation stays host-only)
nrx_status model_pinned(nrx_model *m) {
  std::lock_guard<std::mutex> lk(m->mu);
  if (m->pinned_jobs) return NRX_OK;
  if (hipHostMalloc(&m->pinned_jobs, sizeof(PrepJob) * m->jobs.size(), hipHostMallocDefault) != hipSuccess)
    return fail(NRX_ERR_HIP, "hipHostMalloc failed");
  memcpy(m->pinned_jobs, m->jobs.data(), sizeof(PrepJob) * m->jobs.size());
  return NRX_OK;
}

// Stage kinds of the persistent forward over the first c_run blocks, in the order forward_impl adds them.
std::vector<int> persist_kinds(const nrx_model *m, int c_run) {
  std::vector<int> k{PK_CONV_STORE};
  for (int i = 0; i < c_run; ++i) {
    if (m->blocks[i].mp_round >= 0) k.push_back(PK_MP);
    k.push_back(PK_CONV_LN);
    k.push_back(PK_CONV_RESID);
  }
  k.push_back(PK_READOUT);
  return k;
}

// Persistent stage tables in pinned host memory, keyed by their contents: a table never changes once
// made, so an asynchronous copy (or a graph replay) always reads what its call wrote.
constexpr size_t PERSIST_TABLES_MAX = 32;
constexpr int PERSIST_SPIN_LIMIT = 1 << 21;   // polls of one dependency flag (far above any legal wait)
int g_persist_grid = -1;
int persist_grid() {
  if (g_persist_grid < 0) g_persist_grid = persist_max_grid();
  return g_persist_grid;
}
std::shared_ptr<PinnedBuf> persist_table(nrx_model *m, const std::vector<PersistStage> &pst) {
  const size_t bytes = sizeof(PersistStage) * pst.size();
  std::string key((const char *)pst.data(), bytes);
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = m->ptables.find(key);
  if (it != m->ptables.end()) {
    it->second.used = ++m->ptable_tick;
    m->last_ptable = it->second.buf;
    return it->second.buf;
  }
  if (m->ptables.size() >= PERSIST_TABLES_MAX) {
    auto lru = m->ptables.begin();
    for (auto e = m->ptables.begin(); e != m->ptables.end(); ++e)
      if (e->second.used < lru->second.used) lru = e;
    m->ptables.erase(lru);   // a graph that captured it keeps its own reference
  }
  auto b = std::make_shared<PinnedBuf>();
  if (hipHostMalloc(&b->ptr, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
  b->bytes = bytes;
  memcpy(b->ptr, pst.data(), bytes);
  m->ptables[key] = nrx_model::PTable{b, ++m->ptable_tick};
  m->last_ptable = b;
  return b;
}

template <typename T>
nrx_status forward_impl(nrx_model *m, const Plan *P, const FwdLayout &L, const float *w, const float *y, float *h_ls,
                        float *llr, bool save, char *ws, hipStream_t st, int n_run = 0, int64_t llr_stride = 0,
                        float *hest = nullptr, int64_t h_stride = 0) {
  nrx_status ps = model_pinned(m);
  if (ps != NRX_OK) return ps;
  if (plan_upload(const_cast<Plan *>(P), ws + L.meta, st) != NRX_OK) return NRX_ERR_HIP;
  HIPCHK(hipMemcpyAsync(ws + L.jobs, m->pinned_jobs, sizeof(PrepJob) * m->jobs.size(), hipMemcpyHostToDevice, st));
  const Dev D = dev_tables(P, ws + L.meta);
  T *wprep = (T *)(ws + L.wprep);
  float *fields = (float *)(ws + L.fields);
  float2 *dmrs = (float2 *)(ws + L.dmrs);
  float2 *pairs = (float2 *)(ws + L.pairs);
  T *X = (T *)(ws + L.X);
  unsigned int *slot_flags = (unsigned int *)(ws + L.flags);
  launch_stamp_start((unsigned int *)(ws + L.done), (unsigned long long *)(ws + L.stamps), slot_flags, P->n, st);
  {
    ProfMark pm(m, NRX_K_FRONTEND, st);
    launch_prep<T>(w, (const PrepJob *)(ws + L.jobs), (int)m->jobs.size(), m->prep_total, wprep, fields, st);
    launch_dmrs(D.geo, P->n, dmrs, st);
    launch_ls_pairs(D.geo, P->n, (int)P->max_pairs, (const float2 *)y, dmrs, pairs, D.pair_off, 0, st);
    launch_features<T>(D.geo, nullptr, P->n, P->max_rows, (const float2 *)y, pairs, D.pair_off, m->cfg.n_ant, m->cx,
                       X, (float2 *)h_ls, st, nullptr, slot_flags);
  }
  // FP8 models: E4M3 block-conv operands (or, while calibrating, BF16 convs that record max |activation|)
  const bool f8 = m->fp8 && !m->calibrating && !save;
  // which block convs run in E4M3 (the others in BF16); an E4M3 conv reads E4M3 copies of its inputs, so
  // their producers write those copies (and BF16 where a BF16 conv reads them)
  const bool f8a = f8 && (m->fp8_layers & 1), f8b = f8 && (m->fp8_layers & 2);
  uint8_t *h8 = m->fp8 ? (uint8_t *)(ws + L.h8) : nullptr;
  uint8_t *a8 = m->fp8 ? (uint8_t *)(ws + L.a8) : nullptr;
  uint8_t *agg8 = m->fp8 ? (uint8_t *)(ws + L.agg8) : nullptr;
  unsigned int *amax = m->calibrating ? (unsigned int *)(ws + L.amax) : nullptr;
  const int C = m->cfg.n_blocks;
  auto inv_scale = [&](int idx) { return 1.0f / m->act_scale[idx]; };
  if (f8) {
    if (!m->calibrated) return fail(NRX_ERR_INVALID, "FP8 model has no activation scales (nrx_calibrate)");
    ProfMark pm(m, NRX_K_FRONTEND, st);
    HIPCHK(hipMemcpyAsync(ws + L.f8jobs, m->pinned_fp8jobs, sizeof(Fp8Job) * m->fp8jobs.size(),
                          hipMemcpyHostToDevice, st));
    launch_prep_fp8(w, (const Fp8Job *)(ws + L.f8jobs), (int)m->fp8jobs.size(), (uint8_t *)(ws + L.w8),
                    (float *)(ws + L.wsc), st);
  }
  if (amax) HIPCHK(hipMemsetAsync(amax, 0, m->act_scale.size() * 4, st));

  const int grid_mlp = std::min<int>((int)std::max(P->mt.size(), P->rt.size()), num_cu() * 4);
  // persistent forward (model flags bit 3): the layers below are collected as stages of one launch
  // instead of being launched one by one (plain BF16 inference: one readout, no second readout)
  const bool persist = std::is_same<T, bf16_t>::value && (m->cfg.flags & 8) && !save && !f8 && !amax &&
                       llr_stride == 0 && !hest && L.pctl;
  std::vector<PersistStage> pst;
  auto add_stage = [&](int kind, const void *args) {
    if constexpr (std::is_same<T, bf16_t>::value) {
      PersistStage e{};
      e.kind = kind;
      if (kind <= PK_CONV_RESID) e.c = *(const ConvArgs<bf16_t> *)args;
      else e.m = *(const MlpArgs<bf16_t> *)args;
      pst.push_back(e);
    }
  };
  // launch one conv of layer class cls with its selected variant (E4M3 kernels when fp8op)
  auto conv = [&](ConvArgs<T> ca, int epi, int cls, bool fp8op) {
    if (persist) {
      add_stage(epi == EPI_STORE ? PK_CONV_STORE : (epi == EPI_LN_RELU ? PK_CONV_LN : PK_CONV_RESID), &ca);
      return;
    }
    int v = m->conv_variant[cls];
    if (fp8op) v = std::min(v, NRX_CONV8_VARIANTS - 1);
    else if (m->fp8 && cls != NRX_K_CONV_IN) v = CONV_DEFAULT_VARIANT;   // a block conv kept in BF16
    else if (kConvVariants[v].pref == 2 && ((ca.c0 + ca.c1) / (64 / (int)sizeof(T))) % 2)
      v = 1;   // the LDS-operand kernels walk the input channels two chunks at a time
    const ConvVariant &cv = fp8op ? kConv8Variants[v] : kConvVariants[v];
    const int ti = variant_tiles(cv);
    ca.tiles = D.ct[ti];
    ca.n_tiles = (int)P->ct[ti].size();
    if (ca.only_m && P->mod_lists) {   // Var-IO StateInit: only the slots with a UE of this modulation
      ca.tiles = D.ctm[ca.only_m / 2 - 1][ti];
      ca.n_tiles = (int)P->ctm[ca.only_m / 2 - 1][ti].size();
    }
    int grid = std::min<int>(ca.n_tiles, num_cu() * cv.occ);
    grid = (grid + 7) / 8 * 8;    // the kernel's XCD-aware order needs a multiple of 8
    ProfMark pm(m, cls, st);
    if constexpr (std::is_same<T, bf16_t>::value) {
      if (fp8op) { launch_conv8(ca, epi, v, grid, st); return; }
    }
    launch_conv<T>(ca, epi, v, grid, st);
  };
  auto buf = [&](size_t off) { return (T *)(ws + off); };
  // a bias / LayerNorm vector: the master weights, or its zero-padded copy when d < 128
  auto vec = [&](int64_t master, int64_t pad) { return pad >= 0 ? fields + pad : w + master; };

  ConvArgs<T> a{};
  a.geo = D.geo;
  a.ln_inv = 1.0f / (float)m->cfg.d;
  a.ln_pad = (float)(NRX_D - m->cfg.d);
  // StateInit
  a.src0 = X; a.c0 = m->cx; a.src1 = nullptr; a.c1 = 0;
  a.out = buf(L.h[0]);
  for (auto &ci : m->cins) {   // Var-IO: one launch per modulation the batch uses, each storing its UEs' rows
    if (ci.m && !batch_uses(P, ci.m)) continue;
    ConvArgs<T> a0 = a;
    a0.w = wprep + ci.c.prep;
    a0.bias = vec(ci.c.b, ci.c.bpad);
    a0.pe = fields + ci.c.field;
    a0.only_m = ci.m;
    if (f8a) { a0.out8 = h8; a0.out8_inv = inv_scale(0); }
    if (amax) a0.amax = amax + 0;
    conv(a0, EPI_STORE, NRX_K_CONV_IN, false);
  }
  // CGNN iterations run (depth control) and, with llr_stride > 0, a readout after each of them
  const std::vector<int> ends = iteration_ends(m->cfg);
  if (n_run <= 0 || n_run > (int)ends.size()) n_run = (int)ends.size();
  const int c_run = ends[n_run - 1];
  // ReadoutLLRs to run: the shared one, or (Var-IO) those of the modulations the batch uses
  std::vector<const nrx_model::Readout *> ros_run;
  for (auto &R : m->ros)
    if (!R.m || batch_uses(P, R.m)) ros_run.push_back(&R);
  auto readout = [&](int blocks_done, int k, bool last) {
    MlpArgs<T> ra{};
    for (size_t i = 0; i < ros_run.size(); ++i) {
      const nrx_model::Readout &R = *ros_run[i];
      ra = MlpArgs<T>{};
      ra.h = buf(L.h[save ? blocks_done : 0]);
      ra.w1 = wprep + R.l.p1;
      ra.b1 = vec(R.l.b1, R.l.b1pad);
      ra.b2 = w + R.l.b2;
      ra.w2 = wprep + R.l.p2;
      ra.save_m1 = save ? buf(L.q[k]) : nullptr;
      ra.llr = llr + (int64_t)k * llr_stride;
      ra.m_max = m->cfg.m_max;
      ra.n_out = R.m;
      ra.only_m = R.m;
      ra.geo = D.geo;
      ra.tiles = D.rt;
      ra.n_tiles = (int)P->rt.size();
      // the pass completes at the last launch of the last readout
      const bool fin = last && i + 1 == ros_run.size();
      if (R.m && P->mod_lists && !fin && !persist) {   // Var-IO: only the slots with a UE of this modulation
        ra.tiles = D.rtm[R.m / 2 - 1];
        ra.n_tiles = (int)P->rtm[R.m / 2 - 1].size();
      }
      ra.slot_done = fin ? (unsigned int *)(ws + L.done) : nullptr;
      ra.stamps = fin ? (unsigned long long *)(ws + L.stamps) : nullptr;
      ra.slot_flags = slot_flags;
      if (persist) {   // the persistent kernel counts finished readout tiles itself
        ra.slot_done = nullptr;
        ra.stamps = nullptr;
        add_stage(PK_READOUT, &ra);
        continue;
      }
      ProfMark pm(m, NRX_K_READOUT, st);
      launch_readout<T>(ra, grid_mlp, st);
    }
    if (hest) {   // ReadoutChEst on the same state (double readout)
      MlpArgs<T> ca = ra;
      ca.tiles = D.rt;
      ca.n_tiles = (int)P->rt.size();
      ca.w1 = wprep + m->ro_ch.p1;
      ca.b1 = vec(m->ro_ch.b1, m->ro_ch.b1pad);
      ca.b2 = w + m->ro_ch.b2;
      ca.w2 = wprep + m->ro_ch.p2;
      ca.save_m1 = save ? buf(L.q_ch[k]) : nullptr;
      ca.llr = hest + (int64_t)k * h_stride;
      ca.m_max = 2 * m->cfg.n_ant;
      ca.n_out = 0;
      ca.only_m = 0;
      ca.chest = 1;
      ca.slot_done = nullptr;
      ca.stamps = nullptr;
      ProfMark pm(m, NRX_K_READOUT, st);
      launch_readout<T>(ca, grid_mlp, st);
    }
  };
  for (int i = 0; i < c_run; ++i) {
    const BlockLayer &B = m->blocks[i];
    T *h_in = buf(L.h[save ? i : 0]);
    T *h_out = buf(L.h[save ? i + 1 : 0]);
    T *abuf = buf(L.a[save ? i : 0]);
    T *agg = nullptr;
    if (B.mp_round >= 0) {
      const int r = B.mp_round;
      agg = buf(L.agg[save ? r : 0]);
      MlpArgs<T> ma{};
      ma.h = h_in;
      ma.w1 = wprep + m->mp[r].p1;
      ma.w2 = wprep + m->mp[r].p2;
      ma.b1 = vec(m->mp[r].b1, m->mp[r].b1pad);
      ma.b2 = vec(m->mp[r].b2, m->mp[r].b2pad);
      ma.out = agg;
      if (f8a) { ma.out = nullptr; ma.out8 = agg8; ma.out8_inv = inv_scale(2 * C + r); }
      if (amax) ma.amax = amax + 2 * C + r;
      ma.save_m1 = save ? buf(L.m1[r]) : nullptr;
      ma.geo = D.geo;
      ma.tiles = D.mt;
      ma.n_tiles = (int)P->mt.size();
      if (persist) {
        add_stage(PK_MP, &ma);
      } else {
        ProfMark pm(m, NRX_K_MP, st);
        launch_mp<T>(ma, grid_mlp, st);
      }
    }
    ConvArgs<T> ca = a;
    ca.src0 = h_in; ca.c0 = NRX_D;
    ca.src1 = agg; ca.c1 = agg ? NRX_D : 0;
    ca.w = wprep + B.a.prep;
    ca.bias = vec(B.a.b, B.a.bpad);
    ca.pe = B.a.field >= 0 ? fields + B.a.field : nullptr;
    ca.ln_g = vec(B.g, B.gpad);
    ca.ln_b = vec(B.beta, B.betapad);
    ca.out = abuf;
    ca.save_z = save ? buf(L.z[i]) : nullptr;
    ca.save_stats = save ? (float *)(ws + L.stats[i]) : nullptr;
    if (f8a) {
      ca.src8_0 = h8;
      ca.src8_1 = agg ? agg8 : nullptr;
      ca.w8 = (const uint8_t *)(ws + L.w8) + B.a.w8;
      ca.wscale = (const float *)(ws + L.wsc) + B.a.ws8;
    }
    if (f8b) {   // conv_b reads the E4M3 copy of a only
      ca.out = nullptr;
      ca.out8 = a8;
      ca.out8_inv = inv_scale(C + i);
    }
    if (amax) ca.amax = amax + C + i;
    conv(ca, save ? EPI_LN_RELU_SAVE : EPI_LN_RELU, agg ? NRX_K_CONV_A_MP : NRX_K_CONV_A, f8a);
    ConvArgs<T> cb = a;
    cb.src0 = abuf; cb.c0 = NRX_D; cb.src1 = nullptr; cb.c1 = 0;
    cb.w = wprep + B.b.prep;
    cb.bias = vec(B.b.b, B.b.bpad);
    cb.pe = nullptr;
    cb.resid = h_in;
    cb.out = h_out;
    if (f8b) {
      cb.src8_0 = a8;
      cb.w8 = (const uint8_t *)(ws + L.w8) + B.b.w8;
      cb.wscale = (const float *)(ws + L.wsc) + B.b.ws8;
    }
    if (f8a && i + 1 < C) { cb.out8 = h8; cb.out8_inv = inv_scale(i + 1); }
    if (amax && i + 1 < C) cb.amax = amax + i + 1;
    conv(cb, EPI_RESID, NRX_K_CONV_B, f8b);
    if (llr_stride > 0 && i + 1 < c_run) {
      for (int k = 0; k < n_run - 1; ++k)
        if (ends[k] == i + 1) readout(i + 1, k, false);
    }
  }
  readout(c_run, llr_stride > 0 ? n_run - 1 : 0, true);
  if (persist) {
    const std::vector<int> kinds = persist_kinds(m, c_run);
    bool same = kinds.size() == pst.size();
    for (size_t i = 0; same && i < pst.size(); ++i) same = kinds[i] == pst[i].kind;
    if (!same) return fail(NRX_ERR_INVALID, "persistent stage list out of step with the layer sequence");
    const int grid = persist_grid();
    if (grid <= 0) return fail(NRX_ERR_UNSUPPORTED, "the persistent forward kernel does not fit on this device");
    std::shared_ptr<PinnedBuf> tab = persist_table(m, pst);
    if (!tab) return fail(NRX_ERR_HIP, "hipHostMalloc of the persistent stage table failed");
    HIPCHK(hipMemcpyAsync(ws + L.pstages, tab->ptr, tab->bytes, hipMemcpyHostToDevice, st));
    const int64_t n_tiles = P->ptile_base.back();
    unsigned int *ctl = (unsigned int *)(ws + L.pctl);
    launch_zero_words(ctl, 64 + (int64_t)pst.size() * n_tiles, st);
    PersistArgs pa{};
    pa.stages = (const PersistStage *)(ws + L.pstages);
    pa.n_stages = (int)pst.size();
    pa.n_groups = (int)P->pgroup.size() - 1;
    pa.geo = D.geo;
    pa.tile_base = D.ptile_base;
    pa.item_base = D.pitem_base;
    pa.item_tiles = P->pitem_tiles;
    pa.tile_rows = D.ptile_rows;
    pa.group_slot = D.pgroup;
    pa.ctl = ctl;
    pa.done = ctl + 64;
    pa.slot_done = (unsigned int *)(ws + L.done);
    pa.stamps = (unsigned long long *)(ws + L.stamps);
    pa.slot_flags = slot_flags;
    pa.spin_limit = PERSIST_SPIN_LIMIT;
    launch_persist(pa, grid, st);
  }
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

}  // namespace

namespace {
template <typename F>
nrx_status graph_forward(nrx_model *m, const PlanRef &PR, const GraphKey &key, F run, hipStream_t st);
}  // namespace

extern "C" size_t nrx_workspace_bytes(nrx_model *m, const nrx_slot_desc *slots, int32_t n, int32_t save_acts) {
  if (!m) return 0;
  PlanRef PR;
  if (get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR) != NRX_OK) return 0;
  Plan *P = PR.get();
  return fwd_layout(m, P, save_acts != 0).total;
}

namespace {
nrx_status forward_entry(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n, const float *y,
                         float *h_ls, float *llr, int64_t llr_stride, int32_t save_acts, void *ws, size_t ws_bytes,
                         hipStream_t st, float *hest = nullptr, int64_t h_stride = 0) {
  if (!m || !w || !y || !llr || !ws) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  if (m->fp8 && save_acts) return fail(NRX_ERR_UNSUPPORTED, "FP8 models are inference-only (train in BF16)");
  if (m->cfg.d != NRX_D && save_acts) return fail(NRX_ERR_UNSUPPORTED, "training needs d = 128");
  const FwdLayout L = fwd_layout(m, P, save_acts != 0);
  if (ws_bytes < L.total) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, L.total);
  const int iters = m->n_iter > 0 ? m->n_iter : (int)iteration_ends(m->cfg).size();
  auto run = [&](hipStream_t s2) {
    if (m->cfg.precision == NRX_FP32)
      return forward_impl<float>(m, P, L, w, y, h_ls, llr, save_acts != 0, (char *)ws, s2, iters, llr_stride, hest,
                                 h_stride);
    return forward_impl<bf16_t>(m, P, L, w, y, h_ls, llr, save_acts != 0, (char *)ws, s2, iters, llr_stride, hest,
                                h_stride);
  };
  if ((m->cfg.flags & 1) && !m->profile) {
    // replay the whole launch sequence from a graph captured once per (batch, buffers)
    uint64_t vs = 0;   // the classes' variants, 8 bits each
    static_assert(NRX_K_NCLASS * 8 <= 56 && NRX_CONV_VARIANTS <= 256, "variant key");
    for (int c = 0; c < NRX_K_NCLASS; ++c) vs |= (uint64_t)m->conv_variant[c] << (8 * c);
    vs |= (uint64_t)m->fp8_layers << 56;
    s = graph_forward(m, PR,
                      GraphKey{P, w, y, h_ls, llr, ws, save_acts != 0, vs, m->scale_epoch, iters, llr_stride, hest,
                               h_stride},
                      run, st);
  } else {
    s = run(st);
  }
  if (s == NRX_OK && save_acts) {
    std::lock_guard<std::mutex> lk(m->mu);
    m->saved_ws = ws;
    m->saved_plan = PR;
    ++m->save_seq;
    m->saved_iters = iters;
    m->saved_multi = llr_stride > 0;
    m->saved_chest = hest != nullptr;
  }
  return s;
}
}  // namespace

extern "C" nrx_status nrx_forward(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n, const float *y,
                                  float *h_ls, float *llr, int32_t save_acts, void *ws, size_t ws_bytes,
                                  hipStream_t st) {
  return forward_entry(m, w, slots, n, y, h_ls, llr, 0, save_acts, ws, ws_bytes, st);
}

extern "C" nrx_status nrx_forward_iters(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                        const float *y, float *h_ls, float *llr, int64_t llr_stride, int32_t save_acts,
                                        void *ws, size_t ws_bytes, hipStream_t st) {
  if (llr_stride <= 0) return fail(NRX_ERR_INVALID, "llr_stride must be positive");
  return forward_entry(m, w, slots, n, y, h_ls, llr, llr_stride, save_acts, ws, ws_bytes, st);
}

extern "C" nrx_status nrx_forward_chest(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                        const float *y, float *h_ls, float *llr, int64_t llr_stride, float *h_est,
                                        int64_t h_stride, int32_t save_acts, void *ws, size_t ws_bytes,
                                        hipStream_t st) {
  if (!m || !h_est) return fail(NRX_ERR_INVALID, "null argument");
  if (!m->chest) return fail(NRX_ERR_INVALID, "the model has no ReadoutChEst (config flags bit 1)");
  if (llr_stride < 0 || (llr_stride > 0 && h_stride <= 0))
    return fail(NRX_ERR_INVALID, "llr_stride must be >= 0, and h_stride positive with per-iteration readouts");
  return forward_entry(m, w, slots, n, y, h_ls, llr, llr_stride, save_acts, ws, ws_bytes, st, h_est, h_stride);
}

extern "C" nrx_status nrx_set_iterations(nrx_model *m, int32_t n_iter) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  const int n_max = (int)iteration_ends(m->cfg).size();
  if (n_iter < 0 || n_iter > n_max) return fail(NRX_ERR_INVALID, "n_iter %d outside 0..%d", n_iter, n_max);
  m->n_iter = n_iter;
  return NRX_OK;
}

extern "C" int32_t nrx_num_iterations(const nrx_model *m) {
  return m ? (int32_t)iteration_ends(m->cfg).size() : 0;
}

extern "C" int64_t nrx_persist_schedule(nrx_model *m, const nrx_slot_desc *slots, int32_t n, int32_t *stage,
                                        int32_t *slot, int32_t *tile, int32_t *n_tiles, int64_t cap, int32_t *kinds,
                                        int32_t kinds_cap) {
  if (!m || !stage || !slot || !tile || !n_tiles || !kinds) return (fail(NRX_ERR_INVALID, "null argument"), -1);
  if (!(m->cfg.flags & 8)) return (fail(NRX_ERR_INVALID, "the model has no persistent forward (flags bit 3)"), -1);
  PlanRef PR;
  if (get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR) != NRX_OK) return -1;
  const Plan *P = PR.get();
  const std::vector<int> ends = iteration_ends(m->cfg);
  const int n_run = m->n_iter > 0 ? m->n_iter : (int)ends.size();
  const std::vector<int> k = persist_kinds(m, ends[n_run - 1]);
  const int ns = (int)k.size();
  const int64_t items = (int64_t)ns * P->pitem_base.back();
  if (cap < items || kinds_cap < ns) return (fail(NRX_ERR_SHAPE, "room for %lld items and %d stages needed",
                                                   (long long)items, ns), -1);
  for (int i = 0; i < ns; ++i) kinds[i] = k[i];
  const int ng = (int)P->pgroup.size() - 1;
  for (int64_t it = 0; it < items; ++it) {
    const PersistIdx x = persist_decode((int)it, ns, ng, [&](int i) { return P->pitem_base[i]; },
                                        [&](int i) { return P->pgroup[i]; });
    const int cnt = P->ptile_base[x.slot + 1] - P->ptile_base[x.slot];
    stage[it] = x.stage;
    slot[it] = x.slot;
    tile[it] = x.item * P->pitem_tiles;
    n_tiles[it] = std::min(P->pitem_tiles, cnt - tile[it]);
  }
  return items;
}

namespace {
template <typename F>
nrx_status graph_forward(nrx_model *m, const PlanRef &PR, const GraphKey &key, F run, hipStream_t st) {
  Plan *P = PR.get();
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(m->mu);
    if (!m->graphs) m->graphs = new Graphs();
    auto it = m->graphs->execs.find(key);
    if (it != m->graphs->execs.end()) {
      exec = it->second.exec;
      it->second.used = ++m->graphs->tick;
    }
  }
  if (!exec) {
    // host-side allocations happen before the capture
    nrx_status ps = model_pinned(m);
    if (ps != NRX_OK) return ps;
    if (m->cfg.flags & 8) {
      // the persistent forward's stage table (pinned) is made by an eager pass on the caller's stream
      ps = run(st);
      if (ps != NRX_OK) return ps;
    }
    {
      std::lock_guard<std::mutex> lk(g_plans.mu);
      if (!P->pinned) {
        if (hipHostMalloc(&P->pinned, P->meta_bytes, hipHostMallocDefault) != hipSuccess)
          return fail(NRX_ERR_HIP, "hipHostMalloc failed");
        memcpy(P->pinned, P->blob.data(), P->meta_bytes);
      }
    }
    if (!m->graphs->cap) HIPCHK(hipStreamCreateWithFlags(&m->graphs->cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    {
      std::lock_guard<std::mutex> lk(m->mu);
      m->last_ptable.reset();   // set by a persistent forward to the stage table the graph will copy
    }
    HIPCHK(hipStreamBeginCapture(m->graphs->cap, hipStreamCaptureModeThreadLocal));
    nrx_status s = run(m->graphs->cap);
    hipError_t e = hipStreamEndCapture(m->graphs->cap, &graph);
    if (s != NRX_OK) { if (graph) (void)hipGraphDestroy(graph); return s; }
    if (e != hipSuccess) return fail(NRX_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(NRX_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(m->mu);
    if (m->graphs->execs.size() >= GRAPH_CACHE_MAX) {
      auto lru = m->graphs->execs.begin();
      for (auto e = m->graphs->execs.begin(); e != m->graphs->execs.end(); ++e)
        if (e->second.used < lru->second.used) lru = e;
      (void)hipDeviceSynchronize();   // no replay of the evicted graph may still run
      (void)hipGraphExecDestroy(lru->second.exec);
      m->graphs->execs.erase(lru);
    }
    m->graphs->execs[key] = Graphs::Entry{exec, PR, ++m->graphs->tick, m->last_ptable};
  }
  HIPCHK(hipGraphLaunch(exec, st));
  return NRX_OK;
}
}  // namespace

extern "C" nrx_status nrx_slot_latency(nrx_model *m, const nrx_slot_desc *slots, int32_t n, const void *ws,
                                       float *latency_us, hipStream_t st) {
  if (!m || !ws || !latency_us) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const FwdLayout L = fwd_layout(m, P, false);
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(NRX_ERR_HIP, "wall clock rate unavailable");
  launch_stamp_latency((const unsigned long long *)((const char *)ws + L.stamps), P->n, khz / 1000.0, latency_us, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" nrx_status nrx_slot_flags(nrx_model *m, const nrx_slot_desc *slots, int32_t n, const void *ws,
                                     size_t ws_bytes, uint32_t *flags, hipStream_t st) {
  if (!m || !ws || !flags) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const FwdLayout L = fwd_layout(m, P, false);   // the flags sit at the same offset in the training layout
  if (ws_bytes < L.flags + (size_t)P->n * 4)
    return fail(NRX_ERR_WORKSPACE, "workspace %zu bytes is not a forward workspace of this batch", ws_bytes);
  launch_copy_words((const unsigned int *)((const char *)ws + L.flags), (unsigned int *)flags, P->n, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" int64_t nrx_saved_token(const nrx_model *m) {
  if (!m) return 0;
  std::lock_guard<std::mutex> lk(const_cast<nrx_model *>(m)->mu);
  return m->saved_ws ? m->save_seq : 0;
}

extern "C" nrx_status nrx_check_token(const nrx_model *m, const void *ws, int64_t token) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  std::lock_guard<std::mutex> lk(const_cast<nrx_model *>(m)->mu);
  if (!m->saved_ws || m->save_seq == 0) return fail(NRX_ERR_INVALID, "no save_acts forward has run on this model");
  if (token != m->save_seq || ws != m->saved_ws)
    return fail(NRX_ERR_INVALID, "stale activations: the backward belongs to forward %lld, the workspace holds forward "
                "%lld", (long long)token, (long long)m->save_seq);
  return NRX_OK;
}

extern "C" nrx_status nrx_profile_enable(nrx_model *m, int32_t enable) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  std::lock_guard<std::mutex> lk(m->mu);
  m->profile = enable != 0;
  return NRX_OK;
}

extern "C" nrx_status nrx_profile_read(nrx_model *m, int32_t cls, double *ms_total, int64_t *launches, int32_t reset) {
  if (!m || cls < 0 || cls >= NRX_K_NCLASS) return fail(NRX_ERR_INVALID, "bad model or class");
  std::lock_guard<std::mutex> lk(m->mu);
  for (auto &e : m->pending) {
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    m->prof_ms[e.cls] += ms;
    m->prof_n[e.cls] += 1;
    m->pool.push_back(e.a);
    m->pool.push_back(e.b);
  }
  m->pending.clear();
  if (ms_total) *ms_total = m->prof_ms[cls];
  if (launches) *launches = m->prof_n[cls];
  if (reset)
    for (int i = 0; i < NRX_K_NCLASS; ++i) { m->prof_ms[i] = 0; m->prof_n[i] = 0; }
  return NRX_OK;
}

namespace {
// block convs of FP8 models run the E4M3 kernel family
int n_conv_variants(const nrx_model *m, int cls) {
  return m->fp8 && cls != NRX_K_CONV_IN ? NRX_CONV8_VARIANTS : NRX_CONV_VARIANTS;
}
}  // namespace

extern "C" nrx_status nrx_fp8_layers(nrx_model *m, int32_t mask, int32_t *current) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  if (!m->fp8) return fail(NRX_ERR_INVALID, "not an FP8 model");
  if (mask > 3) return fail(NRX_ERR_INVALID, "fp8 layer mask %d (bits 0, 1)", mask);
  if (mask >= 0) m->fp8_layers = mask;
  if (current) *current = m->fp8_layers;
  return NRX_OK;
}

extern "C" nrx_status nrx_conv_variant(nrx_model *m, int32_t cls, int32_t variant, int32_t *current,
                                       int32_t *n_variants) {
  if (!m || cls < NRX_K_CONV_IN || cls > NRX_K_CONV_B) return fail(NRX_ERR_INVALID, "bad model or class");
  const int nv = n_conv_variants(m, cls);
  if (variant >= nv) return fail(NRX_ERR_INVALID, "variant %d out of range", variant);
  if (variant >= 0) m->conv_variant[cls] = variant;
  if (current) *current = m->conv_variant[cls];
  if (n_variants) *n_variants = nv;
  return NRX_OK;
}

namespace {
const char *kClassName[NRX_K_NCLASS] = {"frontend", "conv_in", "conv_a", "conv_a_mp", "conv_b", "mp", "readout"};

std::string tune_key(const nrx_model *m, const Plan *P, int cls) {
  int maxu = 0;
  for (auto &g : P->geo) maxu = std::max(maxu, g.U);
  char b[256];
  snprintf(b, sizeof b, "gfx950|%s|%s|rows=%lld|slots=%d|maxU=%d|B=%d",
           m->cfg.precision == NRX_FP32 ? "fp32" : (m->cfg.precision == NRX_FP8 ? "fp8" : "bf16"),
           kClassName[cls], (long long)P->rows, P->n, maxu, m->cfg.n_ant);
  return b;
}
}  // namespace

extern "C" nrx_status nrx_autotune(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                   const float *y, float *llr, void *ws, size_t ws_bytes, const char *cache_path,
                                   hipStream_t st) {
  if (!m) return fail(NRX_ERR_INVALID, "null model");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const int classes[4] = {NRX_K_CONV_IN, NRX_K_CONV_A, NRX_K_CONV_A_MP, NRX_K_CONV_B};
  // cached choices
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    int found = 0, pick[NRX_K_NCLASS];
    if (f) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        for (int c : classes) {
          const std::string k = "\"key\": \"" + tune_key(m, P, c) + "\"";
          const char *q = strstr(line, k.c_str());
          const char *vq = strstr(line, "\"variant\": ");
          if (q && vq) {
            int v = atoi(vq + 11);
            if (v >= 0 && v < n_conv_variants(m, c)) { pick[c] = v; found |= 1 << c; }
          }
        }
      }
      fclose(f);
    }
    bool all = true;
    for (int c : classes) all = all && (found >> c & 1);
    if (all) {
      for (int c : classes) m->conv_variant[c] = pick[c];
      return NRX_OK;
    }
  }
  const bool prof_was = m->profile;
  const int flags_was = m->cfg.flags;
  m->cfg.flags &= ~1;   // trials run eagerly (no graph per trial)
  struct Restore {
    nrx_model *m;
    int f;
    ~Restore() { m->cfg.flags = f; }
  } restore{m, flags_was};
  double best[NRX_K_NCLASS];
  int bestv[NRX_K_NCLASS];
  for (int c = 0; c < NRX_K_NCLASS; ++c) { best[c] = 1e30; bestv[c] = m->conv_variant[c]; }
  for (int v = 0; v < NRX_CONV_VARIANTS; ++v) {
    for (int c : classes) m->conv_variant[c] = std::min(v, n_conv_variants(m, c) - 1);
    m->profile = false;
    s = nrx_forward(m, w, slots, n, y, nullptr, llr, 0, ws, ws_bytes, st);   // warm-up
    if (s != NRX_OK) { m->profile = prof_was; return s; }
    m->profile = true;
    for (int c = 0; c < NRX_K_NCLASS; ++c) nrx_profile_read(m, c, nullptr, nullptr, 1);
    for (int r = 0; r < 2; ++r) {
      s = nrx_forward(m, w, slots, n, y, nullptr, llr, 0, ws, ws_bytes, st);
      if (s != NRX_OK) { m->profile = prof_was; return s; }
    }
    for (int c : classes) {
      double ms;
      int64_t cnt;
      s = nrx_profile_read(m, c, &ms, &cnt, 0);
      if (s != NRX_OK) { m->profile = prof_was; return s; }
      if (cnt > 0 && ms / cnt < best[c]) { best[c] = ms / cnt; bestv[c] = std::min(v, n_conv_variants(m, c) - 1); }
    }
    nrx_profile_read(m, 0, nullptr, nullptr, 1);
  }
  m->profile = prof_was;
  for (int c : classes) m->conv_variant[c] = bestv[c];
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      for (int c : classes)
        if (best[c] < 1e30)
          fprintf(f, "{\"key\": \"%s\", \"variant\": %d, \"ms\": %.4f}\n", tune_key(m, P, c).c_str(), bestv[c],
                  best[c]);
      fclose(f);
    }
  }
  return NRX_OK;
}

namespace {

template <typename T>
nrx_status backward_impl(nrx_model *m, const Plan *P, const FwdLayout &L, const float *w, const float *dllr,
                         float *dw, char *ws, hipStream_t st, int n_run, int64_t llr_stride,
                         const float *dhest = nullptr, int64_t h_stride = 0) {
  {
    std::lock_guard<std::mutex> lk(m->mu);
    if (!m->pinned_bjobs) {
      if (hipHostMalloc(&m->pinned_bjobs, sizeof(PrepJob) * m->bjobs.size(), hipHostMallocDefault) != hipSuccess)
        return fail(NRX_ERR_HIP, "hipHostMalloc failed");
      memcpy(m->pinned_bjobs, m->bjobs.data(), sizeof(PrepJob) * m->bjobs.size());
    }
  }
  HIPCHK(hipMemcpyAsync(ws + L.bjobs, m->pinned_bjobs, sizeof(PrepJob) * m->bjobs.size(), hipMemcpyHostToDevice, st));
  const Dev D = dev_tables(P, ws + L.meta);
  T *bp = (T *)(ws + L.bprep);
  launch_prep<T>(w, (const PrepJob *)(ws + L.bjobs), (int)m->bjobs.size(), m->bprep_elems, bp, nullptr, st);
  HIPCHK(hipMemsetAsync(ws + L.zero, 0, 128 * 4, st));
  auto buf = [&](size_t off) { return (T *)(ws + off); };
  const float *zero = (const float *)(ws + L.zero);
  float *wpart = (float *)(ws + L.wpart), *cpart = (float *)(ws + L.cpart);
  float *lpart = (float *)(ws + L.lpart), *rpart = (float *)(ws + L.rpart);
  const int d = NRX_D;
  const int ti256 = tile_size_index(4);
  const int grid_mlp = std::min<int>((int)std::max(P->mt.size(), P->rt.size()), std::min(num_cu() * 4, BWD_GRID_MAX));

  auto wgrad = [&](const T *src0, int c0, const T *src1, int c1, const T *dy, bool conv, int cin_real, int cin_total,
                   int64_t dst, bool acc = false) {
    WgradArgs<T> a{};
    a.src0 = src0; a.c0 = c0; a.src1 = src1; a.c1 = c1;
    a.dy = dy;
    a.geo = D.geo;
    a.tiles = D.ct[ti256];
    a.n_tiles = (int)P->ct[ti256].size();
    a.n_taps = conv ? 9 : 1;
    a.tap0 = conv ? 0 : 4;
    a.n_slices = (c0 + c1 + 127) / 128;
    // one round of workgroups (2 per CU; 1 for the 8-wave three-tap kernel), all with the same number of rows
    const int jobs = wgrad_jobs_per_partition(a.n_taps, a.n_slices, std::is_same<T, bf16_t>::value);
    const int per_cu = jobs == a.n_taps * a.n_slices ? 2 : 1;
    a.n_part = std::max(1, std::min(WGRAD_PARTS, (per_cu * num_cu()) / jobs));
    a.partials = wpart;
    launch_wgrad<T>(a, st);
    launch_wgrad_reduce(wpart, a.n_part, a.n_taps, a.tap0, a.n_slices, cin_real, cin_total, conv ? 1 : 0, dst, dw,
                        st, acc);
  };
  auto bias = [&](const T *dy, int64_t bias_off, int64_t pe_w_off, int cin_total, int pe_ch, bool acc = false) {
    launch_colsum<T>(dy, D.geo, P->n, cpart, st);
    launch_bias_pe(cpart, P->n, bias_off, pe_w_off, cin_total, pe_ch, dw, st, acc);
  };
  auto dgrad = [&](const T *src, const T *wt, int epi, int cls, T *out, const T *resid, const T *z, const float *stats,
                   const float *g) {
    ConvArgs<T> a{};
    a.src0 = src; a.c0 = d; a.src1 = nullptr; a.c1 = 0;
    a.w = wt;
    a.bias = zero;
    a.pe = nullptr;
    a.ln_g = g;
    a.resid = resid;
    a.out = out;
    a.save_z = const_cast<T *>(z);
    a.save_stats = const_cast<float *>(stats);
    a.ln_part = lpart;
    a.geo = D.geo;
    // the LayerNorm-backward epilogue spills in the 8-wave and 2-waves-per-SIMD variants; the one-wave-per-SIMD
    // LDS-operand variant (384-row tiles) holds it in registers
    int v = epi == EPI_LN_BWD ? 4 : m->conv_variant[cls];
    if (kConvVariants[v].pref == 2 && ((a.c0 + a.c1) / (64 / (int)sizeof(T))) % 2) v = 1;
    const ConvVariant &cv = kConvVariants[v];
    const int ti = variant_tiles(cv);
    a.tiles = D.ct[ti];
    a.n_tiles = (int)P->ct[ti].size();
    int grid = std::min<int>(a.n_tiles, std::min(num_cu() * cv.occ, BWD_GRID_MAX));
    grid = (grid + 7) / 8 * 8;
    launch_conv<T>(a, epi, v, grid, st);
    return grid;
  };

  T *dh = buf(L.dh), *dz = buf(L.dz);
  // readouts: the last one starts dh; with llr_stride > 0 (multi-loss) the readout after each
  // earlier CGNN iteration adds its gradient where the reverse pass reaches that iteration's end
  const std::vector<int> ends = iteration_ends(m->cfg);
  const int c_run = ends[n_run - 1];
  const int n_ro = llr_stride > 0 ? n_run : 1;
  int ro_done = 0;
  // dW2 partial sets: per ReadoutLLRs (one, or one per Var-IO modulation), then the two column groups
  // of ReadoutChEst; each holds the partials of every readout
  const int64_t set_floats = (int64_t)ends.size() * BWD_GRID_MAX * 1032;
  auto chest_part = [&](int g) { return rpart + (int64_t)(m->ros.size() + g) * set_floats; };
  // the ReadoutLLRs the forward ran (Var-IO: the batch's modulations); the others get a zero gradient
  std::vector<int> ro_run;
  for (size_t i = 0; i < m->ros.size(); ++i) {
    const int mm = m->ros[i].m;
    if (!mm || batch_uses(P, mm)) {
      ro_run.push_back((int)i);
    } else {
      const DenseLayer &l = m->ros[i].l;
      HIPCHK(hipMemsetAsync(dw + l.w1, 0, (size_t)(l.b2 + mm - l.w1) * sizeof(float), st));
    }
  }
  auto readout_back = [&](int k, int blocks_done) {
    const bool acc = ro_done > 0;
    RoBwdArgs<T> a{};
    for (size_t i = 0; i < ro_run.size(); ++i) {
      const nrx_model::Readout &R = m->ros[ro_run[i]];
      a = RoBwdArgs<T>{};
      a.dllr = dllr + (int64_t)k * llr_stride;
      a.q = buf(L.q[k]);
      a.w2 = w + R.l.w2;
      a.w1t = bp + R.l.t1;
      a.dr = buf(L.dr);
      a.dh = dh;
      a.accumulate = (acc || i > 0) ? 1 : 0;
      a.part = rpart + (int64_t)ro_run[i] * set_floats + (int64_t)ro_done * grid_mlp * 1032;
      a.m_max = m->cfg.m_max;
      a.n_out = R.m;
      a.only_m = R.m;
      a.geo = D.geo;
      a.tiles = D.rt;
      a.n_tiles = (int)P->rt.size();
      launch_readout_bwd<T>(a, grid_mlp, st);
      wgrad(buf(L.h[blocks_done]), d, nullptr, 0, buf(L.dr), false, d, d, R.l.w1, acc);
      bias(buf(L.dr), R.l.b1, -1, 0, 0, acc);
    }
    if (dhest) {
      // ReadoutChEst on the same state: its 2B outputs in groups of 8 columns, adding to dh
      RoBwdArgs<T> c = a;
      c.dllr = dhest + (int64_t)k * h_stride;
      c.q = buf(L.q_ch[k]);
      c.w2 = w + m->ro_ch.w2;
      c.w1t = bp + m->ro_ch.t1;
      c.accumulate = 1;
      c.m_max = 2 * m->cfg.n_ant;
      c.n_out = 0;
      c.only_m = 0;
      c.chest = 1;
      for (int g = 0; 8 * g < c.m_max; ++g) {
        c.j0 = 8 * g;
        c.acc_dr = g > 0;
        c.part = chest_part(g) + (int64_t)ro_done * grid_mlp * 1032;
        launch_readout_bwd<T>(c, grid_mlp, st);
      }
      wgrad(buf(L.h[blocks_done]), d, nullptr, 0, buf(L.dr), false, d, d, m->ro_ch.w1, acc);
      bias(buf(L.dr), m->ro_ch.b1, -1, 0, 0, acc);
    }
    ++ro_done;
  };
  readout_back(n_ro - 1, c_run);
  for (int i = c_run - 1; i >= 0; --i) {
    if (n_ro > 1) {
      for (int k = 0; k < n_ro - 1; ++k)
        if (ends[k] == i + 1) readout_back(k, i + 1);
    }
    const BlockLayer &B = m->blocks[i];
    T *h_in = buf(L.h[i]);
    T *a_i = buf(L.a[i]);
    // conv_b: h_{i+1} = h_i + conv_b(a_i)
    wgrad(a_i, d, nullptr, 0, dh, true, d, d, B.b.w);
    bias(dh, B.b.b, -1, 0, 0);
    const int gl = dgrad(dh, bp + B.bg_b, EPI_LN_BWD, NRX_K_CONV_B, dz, a_i, buf(L.z[i]), (const float *)(ws + L.stats[i]),
                         w + B.g);
    launch_ln_reduce(lpart, gl, B.g, B.beta, dw, st);
    // conv_a on [h_i (, agg_r)] (+ PE)
    if (B.mp_round >= 0) {
      const int r = B.mp_round;
      T *agg = buf(L.agg[r]);
      wgrad(h_in, d, agg, d, dz, true, 2 * d, B.a.cin_total, B.a.w);
      bias(dz, B.a.b, B.a.w, B.a.cin_total, 2 * d);
      dgrad(dz, bp + B.bg_a_h, EPI_RESID, NRX_K_CONV_A_MP, dh, dh, nullptr, nullptr, nullptr);
      dgrad(dz, bp + B.bg_a_agg, EPI_STORE, NRX_K_CONV_A_MP, buf(L.dagg), nullptr, nullptr, nullptr, nullptr);
      MpBwdArgs<T> ma{};
      ma.dagg = buf(L.dagg);
      ma.m1 = buf(L.m1[r]);
      ma.w1t = bp + m->mp[r].t1;
      ma.w2t = bp + m->mp[r].t2;
      ma.dmsg = buf(L.dmsg);
      ma.dm1 = buf(L.dm1);
      ma.dh = dh;
      ma.geo = D.geo;
      ma.tiles = D.mt;
      ma.n_tiles = (int)P->mt.size();
      launch_mp_bwd<T>(ma, grid_mlp, st);
      wgrad(buf(L.m1[r]), d, nullptr, 0, buf(L.dmsg), false, d, d, m->mp[r].w2);
      bias(buf(L.dmsg), m->mp[r].b2, -1, 0, 0);
      wgrad(h_in, d, nullptr, 0, buf(L.dm1), false, d, d, m->mp[r].w1);
      bias(buf(L.dm1), m->mp[r].b1, -1, 0, 0);
    } else {
      wgrad(h_in, d, nullptr, 0, dz, true, d, d, B.a.w);
      bias(dz, B.a.b, -1, 0, 0);
      dgrad(dz, bp + B.bg_a_h, EPI_RESID, NRX_K_CONV_A, dh, dh, nullptr, nullptr, nullptr);
    }
  }
  for (int i : ro_run) {
    const nrx_model::Readout &R = m->ros[i];
    launch_readout_w2_reduce(rpart + (int64_t)i * set_floats, n_ro * grid_mlp, R.m ? R.m : m->cfg.m_max, R.l.w2,
                             R.l.b2, dw, st);
  }
  if (dhest) {
    for (int g = 0; 8 * g < 2 * m->cfg.n_ant; ++g)
      launch_readout_w2_reduce(chest_part(g), n_ro * grid_mlp, 2 * m->cfg.n_ant, m->ro_ch.w2, m->ro_ch.b2, dw, st,
                               8 * g);
  } else if (m->chest) {
    // no channel-estimate loss: ReadoutChEst gets a zero gradient (its tensors close the vector)
    HIPCHK(hipMemsetAsync(dw + m->ro_ch.w1, 0, (size_t)(m->n_w - m->ro_ch.w1) * sizeof(float), st));
  }
  // StateInit (no data gradient needed)
  const int B4 = 4 * m->cfg.n_ant;
  for (auto &ci : m->cins) {
    if (!ci.m) {
      wgrad(buf(L.X), m->cx, nullptr, 0, dh, true, B4, B4 + 2, ci.c.w);
      bias(dh, ci.c.b, ci.c.w, B4 + 2, B4);
    } else if (batch_uses(P, ci.m)) {
      // Var-IO: this modulation's StateInit sees the gradient of its UEs' rows only
      launch_select_rows<T>(dh, D.geo, P->n, P->max_rows, ci.m, dz, st);
      wgrad(buf(L.X), m->cx, nullptr, 0, dz, true, B4, B4 + 2, ci.c.w);
      bias(dz, ci.c.b, ci.c.w, B4 + 2, B4);
    } else {
      HIPCHK(hipMemsetAsync(dw + ci.c.w, 0, (size_t)(ci.c.b + m->cfg.d - ci.c.w) * sizeof(float), st));
    }
  }
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

}  // namespace

namespace {
nrx_status backward_entry(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n, const float *dllr,
                          int64_t llr_stride, float *dw, void *ws, size_t ws_bytes, hipStream_t st,
                          const float *dhest = nullptr, int64_t h_stride = 0) {
  if (!m || !w || !dllr || !dw || !ws) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  int iters;
  {
    std::lock_guard<std::mutex> lk(m->mu);
    if (m->saved_ws != ws || m->saved_plan.get() != P)
      return fail(NRX_ERR_INVALID, "no save_acts forward of this batch on this workspace");
    if (m->saved_multi != (llr_stride > 0))
      return fail(NRX_ERR_INVALID, "the saved forward %s per-iteration readouts",
                  m->saved_multi ? "has" : "has no");
    if (dhest && !m->saved_chest) return fail(NRX_ERR_INVALID, "the saved forward ran no ReadoutChEst");
    iters = m->saved_iters;
  }
  const FwdLayout L = fwd_layout(m, P, true);
  if (ws_bytes < L.total) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, L.total);
  if (m->cfg.precision == NRX_FP32)
    return backward_impl<float>(m, P, L, w, dllr, dw, (char *)ws, st, iters, llr_stride, dhest, h_stride);
  return backward_impl<bf16_t>(m, P, L, w, dllr, dw, (char *)ws, st, iters, llr_stride, dhest, h_stride);
}
}  // namespace

extern "C" nrx_status nrx_backward(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                   const float *dllr, float *dw, void *ws, size_t ws_bytes, hipStream_t st) {
  return backward_entry(m, w, slots, n, dllr, 0, dw, ws, ws_bytes, st);
}

extern "C" nrx_status nrx_backward_iters(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                         const float *dllr, int64_t llr_stride, float *dw, void *ws, size_t ws_bytes,
                                         hipStream_t st) {
  if (llr_stride <= 0) return fail(NRX_ERR_INVALID, "llr_stride must be positive");
  return backward_entry(m, w, slots, n, dllr, llr_stride, dw, ws, ws_bytes, st);
}

extern "C" nrx_status nrx_backward_chest(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                         const float *dllr, int64_t llr_stride, const float *dh_est, int64_t h_stride,
                                         float *dw, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!m || !dh_est) return fail(NRX_ERR_INVALID, "null argument");
  if (!m->chest) return fail(NRX_ERR_INVALID, "the model has no ReadoutChEst (config flags bit 1)");
  if (llr_stride < 0 || (llr_stride > 0 && h_stride <= 0))
    return fail(NRX_ERR_INVALID, "llr_stride must be >= 0, and h_stride positive with per-iteration readouts");
  return backward_entry(m, w, slots, n, dllr, llr_stride, dw, ws, ws_bytes, st, dh_est, h_stride);
}

// --------------------------------------------------------- model-free calls --

namespace {
struct FrontLayout {
  size_t meta, dmrs, pairs, h, total;
};
FrontLayout front_layout(const Plan *P, bool need_h) {
  FrontLayout L;
  size_t o = 0;
  L.meta = o; o = align256(o + P->meta_bytes);
  L.dmrs = o; o = align256(o + (size_t)P->dmrs_total * 8);
  L.pairs = o; o = align256(o + (size_t)P->pairs_total * 8);
  int64_t hel = 0;
  for (auto &g : P->geo) hel += (int64_t)g.S * 14 * g.U * g.B;
  L.h = o; o = align256(o + (need_h ? (size_t)hel * 8 : 0));
  L.total = o;
  return L;
}
// internal LS estimates use a packed h layout: slot offsets are recomputed
}  // namespace

extern "C" size_t lmmse_workspace_bytes(const nrx_slot_desc *slots, int32_t n) {
  PlanRef PR;
  if (get_plan(slots, n, 16, 8, 0, &PR) != NRX_OK) return 0;
  Plan *P = PR.get();
  return front_layout(P, true).total + align256(sizeof(SlotGeo) * (size_t)n);
}

static nrx_status ls_into(const Plan *P, const FrontLayout &L, const float *y, float *h, const SlotGeo *geo_h,
                          char *ws, hipStream_t st, const unsigned int *slot_mask = nullptr) {
  const Dev D = dev_tables(P, ws + L.meta);
  float2 *dmrs = (float2 *)(ws + L.dmrs);
  float2 *pairs = (float2 *)(ws + L.pairs);
  launch_dmrs(D.geo, P->n, dmrs, st, slot_mask);
  launch_ls_pairs(D.geo, P->n, (int)P->max_pairs, (const float2 *)y, dmrs, pairs, D.pair_off, 0, st, slot_mask);
  launch_features<float>(geo_h ? geo_h : D.geo, nullptr, P->n, P->max_rows, (const float2 *)y, pairs, D.pair_off, 16,
                         0, (float *)nullptr, (float2 *)h, st, slot_mask);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" nrx_status nrx_ls_estimate(const nrx_slot_desc *slots, int32_t n, const float *y, float *h, void *ws,
                                      size_t ws_bytes, hipStream_t st) {
  if (!y || !h || !ws) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, 16, 8, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const FrontLayout L = front_layout(P, false);
  if (ws_bytes < L.total) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, L.total);
  if (plan_upload(P, (char *)ws + L.meta, st) != NRX_OK) return NRX_ERR_HIP;
  return ls_into(P, L, y, h, nullptr, (char *)ws, st);
}


namespace {
// LS (when h is null) + LMMSE + max-log over the batch, or with slot_mask only over its flagged slots
nrx_status lmmse_impl(const nrx_slot_desc *slots, int32_t n, int32_t m_max, const float *y, const float *h,
                      const float *n0dev, const unsigned int *slot_mask, float *llr, void *ws, size_t ws_bytes,
                      hipStream_t st) {
  if (!y || !llr || !ws) return fail(NRX_ERR_INVALID, "null argument");
  if (m_max != 2 && m_max != 4 && m_max != 6 && m_max != 8) return fail(NRX_ERR_SHAPE, "m_max %d", m_max);
  PlanRef PR;
  nrx_status s = get_plan(slots, n, 16, m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const FrontLayout L = front_layout(P, h == nullptr);
  const size_t need = L.total + align256(sizeof(SlotGeo) * (size_t)n);
  if (ws_bytes < need) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  char *w = (char *)ws;
  if (plan_upload(P, w + L.meta, st) != NRX_OK) return NRX_ERR_HIP;
  const Dev D = dev_tables(P, w + L.meta);
  const SlotGeo *geo = D.geo;
  const float *hh = h;
  if (!h) {
    // packed internal estimate: a geometry copy with h offsets into the workspace buffer
    void *pg;
    {
      std::lock_guard<std::mutex> lk(g_plans.mu);
      if (!P->packed_geo) {
        if (hipHostMalloc(&pg, sizeof(SlotGeo) * n, hipHostMallocDefault) != hipSuccess)
          return fail(NRX_ERR_HIP, "hipHostMalloc failed");
        SlotGeo *gp = (SlotGeo *)pg;
        int64_t off = 0;
        for (int i = 0; i < n; ++i) {
          gp[i] = P->geo[i];
          gp[i].h_off = off;
          off += (int64_t)gp[i].S * 14 * gp[i].U * gp[i].B;
        }
        P->packed_geo = pg;
      }
      pg = P->packed_geo;
    }
    SlotGeo *gdev = (SlotGeo *)(w + L.total);
    HIPCHK(hipMemcpyAsync(gdev, pg, sizeof(SlotGeo) * n, hipMemcpyHostToDevice, st));
    s = ls_into(P, L, y, (float *)(w + L.h), gdev, w, st, slot_mask);
    if (s != NRX_OK) return s;
    geo = gdev;
    hh = (const float *)(w + L.h);
  }
  launch_lmmse(geo, nullptr, P->n, P->max_re, m_max, (const float2 *)y, (const float2 *)hh, n0dev, llr, st,
               slot_mask);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}
}  // namespace

extern "C" nrx_status lmmse_demap(const nrx_slot_desc *slots, int32_t n, int32_t m_max, const float *y, const float *h,
                                  const float *n0dev, float *llr, void *ws, size_t ws_bytes, hipStream_t st) {
  return lmmse_impl(slots, n, m_max, y, h, n0dev, nullptr, llr, ws, ws_bytes, st);
}

extern "C" nrx_status nrx_fallback_lmmse(const nrx_slot_desc *slots, int32_t n, int32_t m_max, const float *y,
                                         const float *h, const float *n0dev, const uint32_t *flags, float *llr,
                                         void *ws, size_t ws_bytes, hipStream_t st) {
  if (!flags) return fail(NRX_ERR_INVALID, "null flags");
  return lmmse_impl(slots, n, m_max, y, h, n0dev, (const unsigned int *)flags, llr, ws, ws_bytes, st);
}

// ------------------------------------------------ allocation-free judge --
//
// lmmse_demap_noalloc runs the kernels of lmmse_demap with every buffer they need beyond y, h and llr
// (the per-slot tables, the DMRS sequences, the LS pair estimates and the interpolated LS estimate)
// carved out of one file-scope device array, so the call allocates nothing: no hipMalloc, no pinned
// host staging, no plan-cache entry.  Each device holds its own copy of the array; its address is
// taken once per device with hipGetSymbolAddress, and only that address reaches kernels and copies.

static __device__ __align__(256) unsigned char scratch[NRX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the first call per device).
nrx_status scratch_of_current_device(char **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(NRX_ERR_UNSUPPORTED, "device index %d >= %d", dev,
                                                         NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(NRX_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = (char *)g_scratch_ptr[dev];
  return NRX_OK;
}

// Scratch layout of one call: [SlotGeo n][pair offsets n+1][DMRS][LS pairs][interpolated LS estimate].
struct NoAllocLayout {
  size_t geo, pair_off, dmrs, pairs, h, total;
  int64_t max_re, max_pairs, max_rows;
};
NoAllocLayout noalloc_layout(const nrx_slot_desc *d, int n, bool need_h) {
  NoAllocLayout L{};
  int64_t dmrs = 0, pairs = 0, hel = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t S = 12LL * d[i].n_prb, U = d[i].n_ue, B = d[i].n_ant;
    dmrs += S;
    pairs += 2 * U * (S / 4) * B;
    hel += S * 14 * U * B;
    L.max_re = std::max(L.max_re, S * 14);
    L.max_pairs = std::max(L.max_pairs, 2 * U * (S / 4) * B);
    L.max_rows = std::max(L.max_rows, S * 14 * U);
  }
  size_t o = 0;
  L.geo = o; o = align256(o + sizeof(SlotGeo) * (size_t)n);
  L.pair_off = o; o = align256(o + sizeof(int64_t) * (size_t)(n + 1));
  L.dmrs = o; o = align256(o + (size_t)dmrs * 8);
  L.pairs = o; o = align256(o + (size_t)pairs * 8);
  L.h = o; o = align256(o + (need_h ? (size_t)hel * 8 : 0));
  L.total = o;
  return L;
}
}  // namespace

extern "C" size_t lmmse_noalloc_scratch_bytes(const nrx_slot_desc *slots, int32_t n, int32_t internal_ls) {
  if (validate_slots(slots, n, 16, 8) != NRX_OK) return 0;
  return noalloc_layout(slots, n, internal_ls != 0).total;
}

extern "C" nrx_status lmmse_demap_noalloc(const nrx_slot_desc *slots, int32_t n, int32_t m_max, const float *y,
                                          const float *h, const float *n0dev, float *llr, hipStream_t st) {
  if (!y || !llr) return fail(NRX_ERR_INVALID, "null argument");
  if (m_max != 2 && m_max != 4 && m_max != 6 && m_max != 8) return fail(NRX_ERR_SHAPE, "m_max %d", m_max);
  if (nrx_status v = validate_slots(slots, n, 16, m_max)) return v;
  const NoAllocLayout L = noalloc_layout(slots, n, h == nullptr);
  if (L.total > (size_t)NRX_NOALLOC_SCRATCH_BYTES)
    return fail(NRX_ERR_WORKSPACE, "batch needs %zu bytes of scratch, above the fixed %zu-byte array of the "
                "allocation-free call: split the batch or use lmmse_demap", L.total,
                (size_t)NRX_NOALLOC_SCRATCH_BYTES);
  char *w = nullptr;
  if (nrx_status v = scratch_of_current_device(&w)) return v;
  // host image of the tables; the internal estimate is packed slot after slot in the scratch
  const size_t tbytes = L.dmrs;
  thread_local std::vector<char> img;
  if (img.size() < tbytes) img.resize(tbytes);
  std::fill(img.begin(), img.begin() + tbytes, 0);
  SlotGeo *geo = (SlotGeo *)(img.data() + L.geo);
  int64_t *poff = (int64_t *)(img.data() + L.pair_off);
  int64_t dm = 0, pr = 0, ho = 0;
  for (int i = 0; i < n; ++i) {
    const nrx_slot_desc &s = slots[i];
    SlotGeo g{};
    g.S = 12 * s.n_prb;
    g.U = s.n_ue;
    g.B = s.n_ant;
    for (int u = 0; u < 4; ++u) g.m[u] = u < s.n_ue ? s.bits_per_sym[u] : 0;
    g.slot_number = s.slot_number;
    g.n_id = s.n_id;
    g.n_scid = s.n_scid;
    g.n0 = s.n0;
    g.snr_off = s.snr_offset_db;
    g.y_off = s.y_offset;
    g.h_off = h ? s.h_offset : ho;
    g.llr_off = s.llr_offset;
    g.bits_off = s.bits_offset;
    g.dmrs_off = dm;
    geo[i] = g;
    poff[i] = pr;
    dm += g.S;
    pr += 2LL * g.U * (g.S / 4) * g.B;
    ho += (int64_t)g.S * 14 * g.U * g.B;
  }
  poff[n] = pr;
  // pageable source: the copy has read the host image when hipMemcpyAsync returns
  HIPCHK(hipMemcpyAsync(w, img.data(), tbytes, hipMemcpyHostToDevice, st));
  const SlotGeo *dgeo = (const SlotGeo *)(w + L.geo);
  const int64_t *dpoff = (const int64_t *)(w + L.pair_off);
  const float *hh = h;
  if (!h) {
    float2 *dmrs = (float2 *)(w + L.dmrs);
    float2 *pairs = (float2 *)(w + L.pairs);
    launch_dmrs(dgeo, n, dmrs, st);
    launch_ls_pairs(dgeo, n, (int)L.max_pairs, (const float2 *)y, dmrs, pairs, dpoff, 0, st);
    launch_features<float>(dgeo, nullptr, n, L.max_rows, (const float2 *)y, pairs, dpoff, 16, 0, (float *)nullptr,
                           (float2 *)(w + L.h), st);
    HIPCHK(hipGetLastError());
    hh = (const float *)(w + L.h);
  }
  launch_lmmse(dgeo, nullptr, n, L.max_re, m_max, (const float2 *)y, (const float2 *)hh, n0dev, llr, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" size_t nrx_bce_workspace_bytes(const nrx_slot_desc *slots, int32_t n, int32_t m_max) {
  PlanRef PR;
  if (get_plan(slots, n, 16, m_max, 0, &PR) != NRX_OK) return 0;
  Plan *P = PR.get();
  const int64_t nb = (P->max_ute + 255) / 256;
  return align256(P->meta_bytes) + align256((size_t)n * nb * 16);
}

extern "C" nrx_status nrx_bce(const nrx_slot_desc *slots, int32_t n, int32_t m_max, const float *llr,
                              const uint8_t *bits, float *dllr, double *loss, unsigned long long *nerr, void *ws,
                              size_t ws_bytes, hipStream_t st) {
  if (!llr || !bits || !ws) return fail(NRX_ERR_INVALID, "null argument");
  if (m_max != 2 && m_max != 4 && m_max != 6 && m_max != 8) return fail(NRX_ERR_SHAPE, "m_max %d", m_max);
  PlanRef PR;
  nrx_status s = get_plan(slots, n, 16, m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const int64_t nb = (P->max_ute + 255) / 256;
  const size_t need = align256(P->meta_bytes) + align256((size_t)n * nb * 16);
  if (ws_bytes < need) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  if (P->n_data_bits <= 0) return fail(NRX_ERR_SHAPE, "no data bits");
  char *w = (char *)ws;
  if (plan_upload(P, w, st) != NRX_OK) return NRX_ERR_HIP;
  const Dev D = dev_tables(P, w);
  launch_bce(D.geo, nullptr, P->n, P->max_ute, m_max, llr, bits, dllr, (double *)(w + align256(P->meta_bytes)),
             (int)nb, loss, nerr, 1.0 / (double)P->n_data_bits, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" size_t nrx_mse_workspace_bytes(const nrx_slot_desc *slots, int32_t n) {
  PlanRef PR;
  if (get_plan(slots, n, 16, 8, 0, &PR) != NRX_OK) return 0;
  Plan *P = PR.get();
  const int64_t nb = (P->max_ute + 255) / 256;
  return align256(P->meta_bytes) + align256((size_t)n * nb * 16);
}

extern "C" nrx_status nrx_mse(const nrx_slot_desc *slots, int32_t n, const float *h_est, const float *h_true,
                              float gamma, float *dh_est, double *loss, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!h_est || !h_true || !ws) return fail(NRX_ERR_INVALID, "null argument");
  PlanRef PR;
  nrx_status s = get_plan(slots, n, 16, 8, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const int64_t nb = (P->max_ute + 255) / 256;
  const size_t need = align256(P->meta_bytes) + align256((size_t)n * nb * 16);
  if (ws_bytes < need) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, need);
  int64_t n_c = 0;   // complex entries of the batch
  for (auto &g : P->geo) n_c += (int64_t)g.S * 14 * g.U * g.B;
  char *w = (char *)ws;
  if (plan_upload(P, w, st) != NRX_OK) return NRX_ERR_HIP;
  const Dev D = dev_tables(P, w);
  launch_mse(D.geo, P->n, h_est, h_true, dh_est, (float)(2.0 * (double)gamma / (double)n_c),
             (double *)(w + align256(P->meta_bytes)), (int)nb, loss, 1.0 / (double)n_c, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

extern "C" nrx_status nrx_adam(float *w, const float *g, float *mm, float *v, int64_t n, int64_t step, float lr,
                               float beta1, float beta2, float eps, hipStream_t st) {
  if (!w || !g || !mm || !v || n <= 0 || step < 1) return fail(NRX_ERR_INVALID, "bad Adam arguments");
  const float c1 = 1.f - (float)pow((double)beta1, (double)step);
  const float c2 = 1.f - (float)pow((double)beta2, (double)step);
  launch_adam(w, g, mm, v, n, lr, beta1, beta2, eps, c1, c2, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

// ---------------------------------------------------------------- simulator --

namespace {
struct SimLayout {
  size_t meta, dmrs, fd, graw, gmix, total;
};
SimLayout sim_layout(const Plan *P) {
  SimLayout L;
  size_t o = 0;
  L.meta = o; o = align256(o + P->meta_bytes);
  L.dmrs = o; o = align256(o + (size_t)P->dmrs_total * 8);
  L.fd = o; o = align256(o + (size_t)P->n * 5 * 4);
  L.graw = o; o = align256(o + (size_t)P->tap_off.back() * 8);
  L.gmix = o; o = align256(o + (size_t)P->tap_off.back() * 8);
  L.total = o;
  return L;
}
nrx_status sim_check(const nrx_sim_config *c) {
  if (!c) return fail(NRX_ERR_INVALID, "null sim config");
  if (c->n_taps < 1 || c->n_taps > 32) return fail(NRX_ERR_SHAPE, "n_taps %d outside 1..32", c->n_taps);
  if (c->tap_spacing_ns < 0 || c->tap_decay_ns <= 0.f) return fail(NRX_ERR_SHAPE, "bad delay profile");
  if (c->rho < 0.f || c->rho >= 1.f) return fail(NRX_ERR_SHAPE, "rho outside [0, 1)");
  if (c->scs_khz <= 0 || c->doppler_max_hz < 0.f) return fail(NRX_ERR_SHAPE, "bad scs / doppler");
  return NRX_OK;
}
}  // namespace

extern "C" size_t slot_sim_workspace_bytes(const nrx_sim_config *cfg, const nrx_slot_desc *slots, int32_t n) {
  if (sim_check(cfg) != NRX_OK) return 0;
  PlanRef PR;
  if (get_plan(slots, n, 16, 8, cfg->n_taps, &PR) != NRX_OK) return 0;
  Plan *P = PR.get();
  return sim_layout(P).total;
}

extern "C" nrx_status slot_sim(const nrx_sim_config *cfg, uint64_t seed, uint32_t batch_index,
                               const nrx_slot_desc *slots, int32_t n, int32_t m_max, float *y, float *h_true,
                               uint8_t *bits, float *snr_db, float *n0, void *ws, size_t ws_bytes, hipStream_t st) {
  nrx_status s = sim_check(cfg);
  if (s != NRX_OK) return s;
  if (!y || !ws) return fail(NRX_ERR_INVALID, "null argument");
  if (m_max != 2 && m_max != 4 && m_max != 6 && m_max != 8) return fail(NRX_ERR_SHAPE, "m_max %d", m_max);
  PlanRef PR;
  s = get_plan(slots, n, 16, m_max, cfg->n_taps, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const SimLayout L = sim_layout(P);
  if (ws_bytes < L.total) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, L.total);
  char *w = (char *)ws;
  if (plan_upload(P, w + L.meta, st) != NRX_OK) return NRX_ERR_HIP;
  const Dev D = dev_tables(P, w + L.meta);
  float2 *dmrs = (float2 *)(w + L.dmrs);
  launch_dmrs(D.geo, P->n, dmrs, st);
  SimParams sp;
  sp.n_taps = cfg->n_taps;
  sp.tap_spacing_ns = cfg->tap_spacing_ns;
  sp.scs_khz = cfg->scs_khz;
  sp.tap_decay_ns = cfg->tap_decay_ns;
  sp.doppler_max_hz = cfg->doppler_max_hz;
  sp.rho = cfg->rho;
  sp.snr_lo = cfg->snr_db_lo;
  sp.snr_hi = cfg->snr_db_hi;
  sp.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  sp.key1 = (uint32_t)(seed >> 32);
  sp.batch = batch_index;
  launch_sim(sp, D.geo, D.tap_off, P->n, P->max_re, P->max_ubl, m_max, dmrs, (float2 *)(w + L.graw),
             (float2 *)(w + L.gmix), (float *)(w + L.fd), (float2 *)y, (float2 *)h_true, bits, snr_db, n0,
             P->max_bits, st);
  HIPCHK(hipGetLastError());
  return NRX_OK;
}

// ------------------------------------------------------------------- FP8 scales --

namespace {
// quantisation jobs of the block convs from the current activation scales, in a
// fresh pinned table (the previous one may still be the source of a queued copy)
nrx_status build_fp8_jobs(nrx_model *m) {
  const int C = m->cfg.n_blocks;
  std::vector<Fp8Job> jobs;
  for (int i = 0; i < C; ++i) {
    const BlockLayer &B = m->blocks[i];
    const float s_agg = B.mp_round >= 0 ? m->act_scale[2 * C + B.mp_round] : 1.0f;
    jobs.push_back(Fp8Job{B.a.w, B.a.cin_real, B.a.cin_total, NRX_D, m->act_scale[i], s_agg, B.a.w8, B.a.ws8});
    jobs.push_back(Fp8Job{B.b.w, B.b.cin_real, B.b.cin_total, NRX_D, m->act_scale[C + i], 1.0f, B.b.w8, B.b.ws8});
  }
  void *p = nullptr;
  if (hipHostMalloc(&p, sizeof(Fp8Job) * jobs.size(), hipHostMallocDefault) != hipSuccess)
    return fail(NRX_ERR_HIP, "hipHostMalloc failed");
  memcpy(p, jobs.data(), sizeof(Fp8Job) * jobs.size());
  std::lock_guard<std::mutex> lk(m->mu);
  if (m->pinned_fp8jobs) m->retired_pinned.push_back(m->pinned_fp8jobs);
  m->pinned_fp8jobs = p;
  m->fp8jobs = jobs;
  m->calibrated = true;
  m->scale_epoch += 1;
  return NRX_OK;
}
}  // namespace

extern "C" int32_t nrx_act_scale_count(const nrx_model *m) {
  return m && m->fp8 ? (int32_t)m->act_scale.size() : 0;
}

extern "C" nrx_status nrx_act_scales(nrx_model *m, const float *set, float *get, int32_t n) {
  if (!m || !m->fp8) return fail(NRX_ERR_INVALID, "not an FP8 model");
  if (n != (int32_t)m->act_scale.size()) return fail(NRX_ERR_SHAPE, "expected %zu scales, got %d", m->act_scale.size(), n);
  if (set) {
    for (int i = 0; i < n; ++i)
      if (!(set[i] > 0.f) || !std::isfinite(set[i])) return fail(NRX_ERR_INVALID, "scale %d is not a positive number", i);
    std::copy(set, set + n, m->act_scale.begin());
    nrx_status s = build_fp8_jobs(m);
    if (s != NRX_OK) return s;
  }
  if (get) std::copy(m->act_scale.begin(), m->act_scale.end(), get);
  return NRX_OK;
}

extern "C" nrx_status nrx_calibrate(nrx_model *m, const float *w, const nrx_slot_desc *slots, int32_t n,
                                    const float *y, float *llr, void *ws, size_t ws_bytes, float headroom,
                                    hipStream_t st) {
  if (!m || !w || !y || !llr || !ws) return fail(NRX_ERR_INVALID, "null argument");
  if (!m->fp8) return fail(NRX_ERR_INVALID, "not an FP8 model");
  if (!(headroom >= 1.0f)) return fail(NRX_ERR_INVALID, "headroom %g < 1", headroom);
  PlanRef PR;
  nrx_status s = get_plan(slots, n, m->cfg.n_ant, m->cfg.m_max, 0, &PR);
  Plan *P = PR.get();
  if (s != NRX_OK) return s;
  const FwdLayout L = fwd_layout(m, P, false);
  if (ws_bytes < L.total) return fail(NRX_ERR_WORKSPACE, "workspace %zu < required %zu bytes", ws_bytes, L.total);
  m->calibrating = true;
  s = forward_impl<bf16_t>(m, P, L, w, y, nullptr, llr, false, (char *)ws, st);
  m->calibrating = false;
  if (s != NRX_OK) return s;
  std::vector<float> amax(m->act_scale.size());
  HIPCHK(hipMemcpyAsync(amax.data(), (char *)ws + L.amax, amax.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t i = 0; i < amax.size(); ++i)
    m->act_scale[i] = amax[i] > 0.f && std::isfinite(amax[i]) ? amax[i] * headroom / 448.0f : 1.0f;
  return build_fp8_jobs(m);
}
