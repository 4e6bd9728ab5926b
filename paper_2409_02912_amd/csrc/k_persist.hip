// Persistent CGNN forward (BF16 inference): one launch for every layer of every slot of a batch.
//
// The batch is cut into tiles of whole REs (at most PERSIST_TILE rows) per slot, and every layer
// (StateInit conv, message passing, the two convs of each residual block, readout; Sec. II-A) is a
// stage.  A work item is one (stage, slot, tile).  The host lists the items so that each item comes
// after every item it depends on, and workgroups claim items in list order from a global counter:
//   - a conv item of stage s needs tiles t - 1 .. t + 1 of stage s - 1 of its slot (3x3 halo);
//   - a message-passing or readout item needs tile t of stage s - 1 (per-RE work).
// These waits also cover every buffer reuse of the in-place inference layout: an item that
// overwrites rows of a buffer waits, directly or through the chain of stages, for all readers of the
// old contents of those rows (the halo readers of the stage before).
//
// Progress: an item waits only for items earlier in the list.  Items are claimed in list order, and
// only by running workgroups, so the earliest unfinished item is held by a running workgroup whose
// dependencies are all finished: it completes, and by induction every item does, whatever number of
// workgroups the device runs at once.  Each wait is also bounded (spin_limit polls); a wait that runs
// out marks the slot in its health word (bit 3) and the item proceeds.
//
// Memory ordering: an item's producer makes its stores visible at device scope (release fence: L2
// write-back across the XCDs) before setting its flag; a consumer reads the flag at device scope and
// invalidates its caches (acquire fence) before its loads and LDS copies.
#include "common.h"
#include "internal.h"
#include "conv_common.h"
#include "conv_ring.h"
#include "mlp_lds.h"

namespace {

// the conv shape of the persistent kernel: 512-row tiles of 8 waves, 3-tap weight slots, 2 slots, wave priority
// falling through each group (the per-layer variants 7 and 14)
constexpr int PK_MB = 4, PK_NW = 8, PK_G = 3, PK_NBUF = 2, PK_SCHED = 3;
using PkRing = RingShape<PK_MB, PK_NW, PK_G, PK_NBUF>;
static_assert(PkRing::TILE == PERSIST_TILE, "tile");
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int PK_LDS = cmax(PkRing::LDS_BYTES, cmax(MP_LDS_BYTES, RO_LDS_BYTES));

// Waits until *f is set, at most `limit` polls; a wait that runs out sets the abort word, after which
// no wait of the launch blocks (the launch still ends, its results flagged).
__device__ __forceinline__ bool wait_flag(const unsigned int *f, unsigned int *abort, int limit) {
  for (int n = 0; __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u; ++n) {
    if ((n & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (n >= limit) {
      __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__global__ __launch_bounds__(64 * PK_NW, 1) void persist_kernel(PersistArgs p) {
  __shared__ __align__(16) unsigned char lds_raw[PK_LDS];
  lds_u8 *lds = (lds_u8 *)lds_raw;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  float lnp[1] = {0.f};
  // the previous item of this workgroup, whose flags are set when the next one is claimed: the flag stores
  // and the claim form one divergent block per iteration, so no lane takes a path around the barrier below
  int prev_stage = -1, prev_gt = 0, prev_nt = 0, prev_slot = 0, prev_cnt = 0, prev_kind = 0;
  for (;;) {
    if (tid == 0) {
      if (prev_stage >= 0) {
        // every wave's stores of that item completed before the barrier that ended it; one release fence
        // writes the L2 back, so that other XCDs see the rows before the flags
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int nt = ldc(p.tile_base + ldc(p.group_slot + p.n_groups));
        for (int t = 0; t < prev_nt; ++t)
          __hip_atomic_store(p.done + (int64_t)prev_stage * nt + prev_gt + t, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        if (prev_kind == PK_READOUT && p.stamps) {
          if (atomicAdd(&p.slot_done[prev_slot], (unsigned)prev_nt) + (unsigned)prev_nt == (unsigned)prev_cnt)
            p.stamps[prev_slot] = wall_clock64();
        }
      }
      s_item = (int)atomicAdd(p.ctl, 1u);
    }
    __syncthreads();
    // uniform from here on: the item is decoded from the group and item tables by scalar loads
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    const int NS = p.n_stages;
    const int n_tiles = ldc(p.tile_base + ldc(p.group_slot + p.n_groups));
    if (it >= NS * ldc(p.item_base + ldc(p.group_slot + p.n_groups))) break;
    const PersistIdx ix = persist_decode(it, NS, p.n_groups, [&](int i) { return ldc(p.item_base + i); },
                                         [&](int i) { return ldc(p.group_slot + i); });
    const int stage = ix.stage, slot = ix.slot;
    const int base = ldc(p.tile_base + slot), cnt = ldc(p.tile_base + slot + 1) - base;
    const int ta = ix.item * p.item_tiles;
    const int tb = ta + p.item_tiles < cnt ? ta + p.item_tiles : cnt;
    const int kind = ldc(&p.stages[stage].kind);
    const bool conv = kind <= PK_CONV_RESID;
    if (tid == 0 && stage > 0) {
      const unsigned int *prev = p.done + (int64_t)(stage - 1) * n_tiles + base;
      const int lo = conv && ta > 0 ? ta - 1 : ta;
      const int hi = conv && tb < cnt ? tb : tb - 1;
      bool ok = true;
      for (int t = lo; t <= hi; ++t) ok = wait_flag(prev + t, p.ctl + 1, p.spin_limit) && ok;
      if (!ok) atomicOr(&p.slot_flags[slot], 8u);
    }
    // the dependencies' stores are visible before any wave reads (the acquire invalidates stale lines)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    const int rows = ldc(p.tile_rows + slot);
    const int U = ldc(&p.geo[slot].U);
    const int slot_rows = ldc(&p.geo[slot].S) * 14 * U;
    // the stage's arguments stay in memory, read through the constant address space where used
    // (scalar loads that can be repeated instead of held in registers)
    typedef const __attribute__((address_space(4))) PersistStage cstage;
    cstage *S = (cstage *)(p.stages + stage);
    if (kind <= PK_CONV_RESID) {
      const ConvArgs<bf16_t> &c = *(const ConvArgs<bf16_t> *)&S->c;
      const RunTiles run{slot, ta, tb - ta, rows, slot_rows};
      if (kind == PK_CONV_STORE)
        conv_ring_body<bf16_t, EPI_STORE, PK_MB, PK_NW, PK_G, PK_NBUF, PK_SCHED>(c, run, lds, lnp);
      else if (kind == PK_CONV_LN)
        conv_ring_body<bf16_t, EPI_LN_RELU, PK_MB, PK_NW, PK_G, PK_NBUF, PK_SCHED>(c, run, lds, lnp);
      else
        conv_ring_body<bf16_t, EPI_RESID, PK_MB, PK_NW, PK_G, PK_NBUF, PK_SCHED>(c, run, lds, lnp);
    } else {
      const MlpArgs<bf16_t> &m = *(const MlpArgs<bf16_t> *)&S->m;
      const int r0 = ta * rows, r1 = tb * rows < slot_rows ? tb * rows : slot_rows;
      const SubTiles sub{Tile{slot, r0, r1 - r0, 0}, (MLP_ROWS / U) * U};
      if (kind == PK_MP) mp_lds_body<PK_NW>(m, sub, lds);
      else readout_lds_body<PK_NW>(m, sub, lds);
    }
    // every wave's stores have completed (to its XCD's L2) and LDS is free for the next item
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    prev_stage = stage;
    prev_gt = base + ta;
    prev_nt = tb - ta;
    prev_slot = slot;
    prev_cnt = cnt;
    prev_kind = kind;
  }
}

__global__ void zero_words_kernel(unsigned int *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

int persist_max_grid() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel, 64 * PK_NW, 0) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}

void launch_persist(const PersistArgs &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(persist_kernel, dim3(grid), dim3(64 * PK_NW), 0, st, a);
}

void launch_zero_words(unsigned int *p, int64_t n, hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024)), dim3(256),
                     0, st, p, n);
}
