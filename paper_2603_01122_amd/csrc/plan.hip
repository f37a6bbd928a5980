// plan.hip -- batched many-human prediction: one persistent rollout launch per
// cycle for every active human, captured with the normalisation in a hipGraph
// per ring entry (and rollout variant), after one prelude launch that updates
// every human's belief and clears the grids, with per-cycle descriptors
// refreshed by a single host-to-device copy.
//
// Scheduling: the particles of every human are cut into tiles of three sizes
// (P, P/2 and P/4 particles per thread).  Each kind's tiles are dealt evenly
// to 8 queues, one per XCD (workgroups are dispatched round-robin over the
// XCDs, so block b starts on queue b mod 8), and each queue hands out its big
// tiles first, then its halves, then its quarters; a block whose queue is
// empty takes from the next ones.  The host sizes the split per cycle so that,
// after whole rounds of big tiles on every resident block, the rest is spread
// as evenly as the tile sizes allow over the CUs: the blocks finish together
// instead of a few CUs running a last round of big tiles while the rest of the
// chip idles.  Every cycle's results depend only on (human id, cycle, seed),
// never on the slot, the tile sizes or the tile order: histogram updates are
// integer atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "belief.hpp"
#include "smooth.hpp"

namespace capred {

constexpr int kMaxObs = 8;
constexpr int kXcds = 8;
constexpr int kQueueWords = kXcds;   // tile counters per ring entry, one per XCD
constexpr int kTileKinds = 3;    // P, P/2, P/4 particles per thread
constexpr int kZeroBlocks = 2048;  // blocks of the grid clear

struct SlotDev {
  RolloutDesc rd;          // rollout of this cycle (start, ring-entry outputs)
  BeliefModel bm;          // continuous model for the update
  double* log_belief;      // belief state [G][B]
  float* probs;            // ring-entry probabilities or null
  int64_t n_cells;         // H * nx * ny
  int32_t n_obs;           // new transitions this cycle
  int32_t reset;           // write the uniform prior before updating
  float obs[(kMaxObs + 1) * 2];
  int32_t smooth_r;        // 0: probs = count / N; > 0: Gaussian-smoothed probs
  SmoothWeights smooth_w;  // normalised 1-D kernel, smooth_w.w[d + smooth_r]
  int32_t prev_x0, prev_y0;  // start of the previous cycle that wrote this ring entry
  int32_t full_clear;        // 1: the ring entry's content is unknown (clear every cell)
  int32_t kt_begin[kTileKinds];  // per tile kind: tickets of earlier slots (within the kind)
  int32_t kt_first[kTileKinds];  // per tile kind: first particle of this slot's tiles
  int32_t in_union;              // 1: this slot's probabilities join the union grid
};

struct CycleHeader {
  uint32_t seed_lo, seed_hi, cycle;
  int32_t n_active, n_tiles, per_tile;
  int32_t kind_begin[kTileKinds + 1];      // ticket ranges of the three tile kinds
  int32_t tile_begin[CAP_MAX_SLOTS + 1];   // per-human launches: prefix of P-sized tiles
  int32_t step_begin[CAP_MAX_SLOTS + 1];   // prefix of horizons (one work item per step)
  int32_t smooth_begin[CAP_MAX_SLOTS + 1]; // prefix of smoothing tiles
  float* union_out;                        // ring entry's union grid [union_H][ny][nx] or null
  int32_t union_H, union_nx, union_ny;
};

// Union grid of the humans sharing a frame (Sec. IV-B: one occupancy map of
// all humans for the planner): the point-wise maximum of their probabilities,
// accumulated with integer atomic max on the FP32 bit patterns (for values
// >= 0 the IEEE order is the unsigned-integer order), so the result is exact
// and independent of the order of contributions.  Cells start at 0 (cleared
// in the grid-clear kernel) and only nonzero probabilities are sent.
__device__ __forceinline__ void union_max_at(const CycleHeader* H, int t, size_t cell_in_plane,
                                             float v) {
  if (v > 0.f && t <= H->union_H) {
    const size_t plane = (size_t)H->union_nx * H->union_ny;
    __hip_atomic_fetch_max(as_global(reinterpret_cast<uint32_t*>(H->union_out)) +
                               (size_t)(t - 1) * plane + cell_in_plane,
                           __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ const SlotDev* slots_of(const uint8_t* base) {
  return reinterpret_cast<const SlotDev*>(base + sizeof(CycleHeader));
}

// ---------------------------------------------------------------- kernels
// Belief update of slot s (one block).
__device__ __forceinline__ void update_slot(const uint8_t* __restrict__ base, int s,
                                            BeliefShared& sh) {
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  if (s >= H->n_active) return;
  const SlotDev& sd = slots_of(base)[s];
  const int J = sd.bm.G * sd.bm.B;
  if (sd.reset) {
    for (int j = threadIdx.x; j < J; j += blockDim.x) sd.log_belief[j] = -log((double)J);
    __syncthreads();
  }
  belief_update_block(sd.bm, sd.obs, sd.n_obs, sd.log_belief, const_cast<double*>(sd.rd.belief),
                      sh);
}

__global__ void __launch_bounds__(kBeliefThreads)
    plan_update_kernel(const uint8_t* __restrict__ base, int only) {
  __shared__ BeliefShared sh;
  update_slot(base, only >= 0 ? only : (int)blockIdx.x, sh);
}

// Clearing and normalising work only where a ring entry's grids can be
// nonzero.  After step t every particle lies in the reach window of its start
// (clipped to the grid), so a ring entry's counts and probabilities are zero
// outside the window of the cycle that last wrote it; a cycle therefore
// clears, and afterwards normalises, the bounding box of that window and of
// its own window (the latter also makes a replayed rollout start from zero).
// A ring entry whose content is unknown (first use after admission) is done
// in full.  Work items are the steps of all active humans (step_begin prefix).
__device__ __forceinline__ int slot_of_step(const CycleHeader* H, int item) {
  int lo = 0, hi = H->n_active;  // largest s with step_begin[s] <= item
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (H->step_begin[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ Window clear_region(const SlotDev& sd, int t) {
  const RolloutDesc& d = sd.rd;
  if (sd.full_clear) return Window{0, 0, d.nx, d.ny};
  const Window a = step_window_at(d, d.X0, d.Y0, t);
  const Window b = step_window_at(d, sd.prev_x0, sd.prev_y0, t);
  if (a.w == 0 || a.h == 0) return b;
  if (b.w == 0 || b.h == 0) return a;
  const int x0 = min(a.x0, b.x0), y0 = min(a.y0, b.y0);
  const int x1 = max(a.x0 + a.w, b.x0 + b.w), y1 = max(a.y0 + a.h, b.y0 + b.h);
  return Window{x0, y0, x1 - x0, y1 - y0};
}

__device__ __forceinline__ void item_range(const CycleHeader* H, int only, int* i0, int* i1) {
  const int na = H->n_active;
  *i0 = only >= 0 ? (only < na ? H->step_begin[only] : 0) : 0;
  *i1 = only >= 0 ? (only < na ? H->step_begin[only + 1] : 0) : H->step_begin[na];
}

// Clears the counts (and off-grid counters) of every active slot (only < 0) --
// or of slot `only` -- and resets the tile queues for the rollout that follows.
// Block `blk` of `nblk` of the clear (see plan_zero_kernel).
__device__ __forceinline__ void zero_items(const uint8_t* __restrict__ base,
                                           uint32_t* __restrict__ queues, int only, int blk,
                                           int nblk) {
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  if (blk == 0 && threadIdx.x < kQueueWords) queues[threadIdx.x] = 0u;
  const SlotDev* sl = slots_of(base);
  int i0, i1;
  item_range(H, only, &i0, &i1);
  for (int it = i0 + blk; it < i1; it += nblk) {
    const int s = __builtin_amdgcn_readfirstlane(slot_of_step(H, it));
    const SlotDev& sd = sl[s];
    const int t = it - H->step_begin[s] + 1;
    const Window r = clear_region(sd, t);
    global_ptr<uint32_t> p = as_global(sd.rd.counts) + (size_t)(t - 1) * sd.rd.nx * sd.rd.ny +
                             (size_t)r.y0 * sd.rd.nx + r.x0;
    // one wavefront per row of the region, lanes along the row (coalesced)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int y = wave; y < r.h; y += nw)
      for (int x = lane; x < r.w; x += 64) p[(size_t)y * sd.rd.nx + x] = 0u;
    if (threadIdx.x == 0 && sd.rd.offgrid) as_global(sd.rd.offgrid)[t - 1] = 0u;
  }
  // the union grid (the per-human launches clear it with the first human's
  // clear; a replay of the rollout alone, only = -2, leaves it)
  if (H->union_out && (only == -1 || only == 0)) {
    const size_t n = (size_t)H->union_H * H->union_nx * H->union_ny;
    global_ptr<uint32_t> u = as_global(reinterpret_cast<uint32_t*>(H->union_out));
    for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n;
         i += (size_t)nblk * blockDim.x)
      u[i] = 0u;
  }
}

__global__ void __launch_bounds__(256)
    plan_zero_kernel(const uint8_t* __restrict__ base, uint32_t* __restrict__ queues, int only) {
  zero_items(base, queues, only, (int)blockIdx.x, (int)gridDim.x);
}

// The start of a batched cycle in one launch: blocks [0, n_slots) update the
// beliefs (one per slot), the rest clear the grids and reset the tile queues.
// The two are independent, so they run side by side instead of one after the
// other (and one launch gap fewer).
__global__ void __launch_bounds__(kBeliefThreads)
    plan_prelude_kernel(const uint8_t* __restrict__ base, uint32_t* __restrict__ queues,
                        int n_slots) {
  __shared__ BeliefShared sh;
  if ((int)blockIdx.x < n_slots)
    update_slot(base, (int)blockIdx.x, sh);
  else
    zero_items(base, queues, -1, (int)blockIdx.x - n_slots, (int)gridDim.x - n_slots);
}

__global__ void __launch_bounds__(256)
    plan_normalize_kernel(const uint8_t* __restrict__ base, int only) {
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  const SlotDev* sl = slots_of(base);
  int i0, i1;
  item_range(H, only, &i0, &i1);
  const int items = i1 - i0;
  if (items <= 0) return;
  // A (slot, step) item takes `per` blocks when the grid has room, its rows
  // dealt round-robin to their waves: with one block per item each wave
  // walks tens of rows of a late step's window, one dependent load and store
  // after another.
  const int per = max(1, (int)gridDim.x / items);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int u = (int)blockIdx.x; u < items * per; u += (int)gridDim.x) {
    const int it = i0 + u / per, band = u - (u / per) * per;
    const int s = __builtin_amdgcn_readfirstlane(slot_of_step(H, it));
    const SlotDev& sd = sl[s];
    if (!sd.probs || sd.smooth_r > 0) continue;
    const int t = it - H->step_begin[s] + 1;
    const Window r = clear_region(sd, t);
    const size_t origin = (size_t)(t - 1) * sd.rd.nx * sd.rd.ny + (size_t)r.y0 * sd.rd.nx + r.x0;
    global_ptr<const uint32_t> q = as_global(static_cast<const uint32_t*>(sd.rd.counts)) + origin;
    global_ptr<float> p = as_global(sd.probs) + origin;
    const float N = (float)sd.rd.N;
    const bool un = sd.in_union != 0;
    const size_t corner = (size_t)r.y0 * sd.rd.nx + r.x0;
    for (int y = band * nw + wave; y < r.h; y += per * nw)
      for (int x = lane; x < r.w; x += 64) {
        const size_t c = (size_t)y * sd.rd.nx + x;
        const float v = (float)q[c] / N;
        p[c] = v;
        if (un) union_max_at(H, t, corner + c, v);
      }
  }
}

// Smoothing tiles (step, band of kBandRows rows, 256 columns) of every slot
// that asks for Gaussian-smoothed probabilities, as one index space
// (smooth_begin prefix) walked by a persistent grid.
__global__ void __launch_bounds__(kSmoothThreads)
    plan_smooth_kernel(const uint8_t* __restrict__ base, int only) {
  extern __shared__ float tile[];
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  const SlotDev* sl = slots_of(base);
  const int na = H->n_active;
  const int b0 = only >= 0 ? (only < na ? H->smooth_begin[only] : 0) : 0;
  const int b1 = only >= 0 ? (only < na ? H->smooth_begin[only + 1] : 0) : H->smooth_begin[na];
  for (int b = b0 + (int)blockIdx.x; b < b1; b += (int)gridDim.x) {
    int lo = 0, hi = na;  // largest s with smooth_begin[s] <= b
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (H->smooth_begin[mid] <= b) lo = mid;
      else hi = mid;
    }
    const int s = __builtin_amdgcn_readfirstlane(lo);
    const SlotDev& sd = sl[s];
    const int nx = sd.rd.nx, ny = sd.rd.ny;
    const int tx = (nx + kSmoothThreads - 1) / kSmoothThreads;
    const int ty = (ny + kBandRows - 1) / kBandRows;
    const int local = b - H->smooth_begin[s];
    const int t = local / (tx * ty);
    const int rem = local - t * tx * ty;
    const int by = rem / tx, bx = rem - by * tx;
    const size_t plane = (size_t)ny * nx;
    float* un = sd.in_union && t + 1 <= H->union_H
                    ? H->union_out + (size_t)t * H->union_nx * H->union_ny
                    : nullptr;
    smooth_block(sd.rd.counts + (size_t)t * plane, sd.probs + (size_t)t * plane, ny, nx,
                 sd.smooth_r, (float)sd.rd.N, sd.smooth_w.w, by * kBandRows,
                 bx * kSmoothThreads, tile, un);
    __syncthreads();  // the next tile rewrites `tile`
  }
}

// Slot of ticket `local` within tile kind k: the largest s whose kind-k
// tickets start at or before it (slots without such tiles share the next
// slot's start and are skipped by "largest").
__device__ __forceinline__ int slot_of_kind_tile(const SlotDev* sl, int n_active, int k,
                                                 int local) {
  int lo = 0, hi = n_active;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sl[mid].kt_begin[k] <= local) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int KT, int P, bool SHIFT, bool MS>
__global__ void __launch_bounds__(1024)
    plan_rollout_kernel(const uint8_t* __restrict__ base, uint32_t* __restrict__ queues, int cap) {
  __shared__ TileShared sh;
  __shared__ float4 ctl[MS ? CAP_MAX_U : 1];
  __shared__ int s_tile[2];
  extern __shared__ uint32_t win[];
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  const SlotDev* sl = slots_of(base);
  for (int i = threadIdx.x; i < 2 * cap; i += blockDim.x) win[i] = 0u;
  const int home = blockIdx.x % kXcds;
  for (;;) {
    if (threadIdx.x == 0) {
      // queue q holds, of each kind k, the kind's tiles [n_k q / 8, n_k (q + 1) / 8)
      int kind = -1, local = 0;
      for (int i = 0; i < kXcds && kind < 0; ++i) {
        const int q = (home + i) % kXcds;
        int lo[kTileKinds], size = 0;
        for (int k = 0; k < kTileKinds; ++k) {
          const int nk = H->kind_begin[k + 1] - H->kind_begin[k];
          lo[k] = (int)(((int64_t)nk * q) / kXcds);
          size += (int)(((int64_t)nk * (q + 1)) / kXcds) - lo[k];
        }
        if (size == 0) continue;
        int j = (int)atomicAdd(queues + q, 1u);
        if (j >= size) continue;
        for (int k = 0; k < kTileKinds; ++k) {
          const int nk = H->kind_begin[k + 1] - H->kind_begin[k];
          const int cnt = (int)(((int64_t)nk * (q + 1)) / kXcds) - lo[k];
          if (j < cnt) {
            kind = k;
            local = lo[k] + j;
            break;
          }
          j -= cnt;
        }
      }
      s_tile[0] = kind;
      s_tile[1] = local;
    }
    __syncthreads();
    const int kind = __builtin_amdgcn_readfirstlane(s_tile[0]);
    if (kind < 0) break;
    const int local = __builtin_amdgcn_readfirstlane(s_tile[1]);
    const int s = __builtin_amdgcn_readfirstlane(slot_of_kind_tile(sl, H->n_active, kind, local));
    const int per = (int)blockDim.x * (P >> kind);
    const int64_t first = sl[s].kt_first[kind] + (int64_t)(local - sl[s].kt_begin[kind]) * per;
    // rollout_tile starts and ends with a barrier: s_tile is not rewritten
    // before every thread has read it.  The host only makes kinds whose size
    // P >> kind is at least one particle per thread.
    if (kind == 0) {
      rollout_tile<KT, P, SHIFT, MS>(sl[s].rd, first, H->seed_lo, H->seed_hi, sh, win, cap, ctl);
    } else if constexpr (P >= 2) {
      if (kind == 1 || P == 2)
        rollout_tile<KT, P / 2, SHIFT, MS>(sl[s].rd, first, H->seed_lo, H->seed_hi, sh, win, cap,
                                           ctl);
      else
        rollout_tile<KT, (P >= 4 ? P / 4 : 1), SHIFT, MS>(sl[s].rd, first, H->seed_lo,
                                                          H->seed_hi, sh, win, cap, ctl);
    }
  }
}

// One human's tiles, one block per tile (the per-human reference launch).
template <int KT, int P, bool SHIFT, bool MS>
__global__ void __launch_bounds__(1024)
    plan_rollout_one_kernel(const uint8_t* __restrict__ base, int s, int cap) {
  __shared__ TileShared sh;
  __shared__ float4 ctl[MS ? CAP_MAX_U : 1];
  extern __shared__ uint32_t win[];
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(base);
  for (int i = threadIdx.x; i < 2 * cap; i += blockDim.x) win[i] = 0u;
  const int64_t first = (int64_t)blockIdx.x * H->per_tile;
  rollout_tile<KT, P, SHIFT, MS>(slots_of(base)[s].rd, first, H->seed_lo, H->seed_hi, sh, win,
                                 cap, ctl);
}

// ---------------------------------------------------------------- host
struct HostSlot {
  bool active = false;
  SlotDev tmpl;            // static part (rollout/belief model, buffers)
  cap_grid grid;
  uint32_t* counts = nullptr;
  uint32_t* offgrid = nullptr;
  float* probs = nullptr;
  double* belief = nullptr;
  int64_t n_cells = 0;
  float last[2] = {0.f, 0.f};
  int n_staged = 0;
  float staged[kMaxObs * 2];
  bool reset = false;
  int32_t ent_x0[4] = {0, 0, 0, 0}, ent_y0[4] = {0, 0, 0, 0};  // last start per ring entry
  bool ent_full[4] = {true, true, true, true};                 // ring entry content unknown
};

struct Entry {
  uint32_t* queues = nullptr;   // this entry's tile counter (device)
  uint8_t* dev = nullptr;       // header + slots
  uint8_t* host = nullptr;      // pinned mirror
  hipGraphExec_t main[2] = {nullptr, nullptr};  // [shift variant]
  hipEvent_t done = nullptr;
  bool pending = false;
};

typedef void (*RolloutFn)(const uint8_t*, uint32_t*, int);
typedef void (*RolloutOneFn)(const uint8_t*, int, int);

}  // namespace capred

struct cap_plan {
  cap_plan_config cfg;
  std::vector<capred::HostSlot> slots;
  std::vector<capred::Entry> ring;
  uint32_t* queues = nullptr;   // one tile counter per ring entry (device)
  size_t entry_bytes = 0;
  int cap_words = 0;            // LDS window words per buffer
  int grid_blocks[2] = {0, 0};  // persistent blocks per launch, per rollout variant
  int n_cus = 1;                // compute units of the device
  int smooth_blocks = 0;        // persistent blocks of the smoothing stage (0: no stage)
  int per_tile = 0;
  const void* rollout_fn[2] = {nullptr, nullptr};      // [shift variant]
  const void* rollout_one_fn[2] = {nullptr, nullptr};
  int last_variant = 0;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_update = nullptr;
  hipStream_t last_stream = nullptr;
  bool have_last = false;
  int64_t last_run_entry = -1;
  // last staged totals
  int64_t particles = 0, psteps = 0;
  int32_t tiles = 0;
  // union stage: frame, horizon and caller's [ring][H][ny][nx] buffer (null: off)
  cap_grid union_frame{};
  int32_t union_H = 0;
  float* union_dev = nullptr;
};

namespace capred {

template <int KT, int P, bool MS>
static void pick_fns_p(const void** r, const void** one) {
  r[0] = (const void*)plan_rollout_kernel<KT, P, false, MS>;
  r[1] = (const void*)plan_rollout_kernel<KT, P, true, MS>;
  one[0] = (const void*)plan_rollout_one_kernel<KT, P, false, MS>;
  one[1] = (const void*)plan_rollout_one_kernel<KT, P, true, MS>;
}

template <int KT, bool MS>
static void pick_fns(int P, const void** r, const void** one) {
  switch (P) {
    case 1: pick_fns_p<KT, 1, MS>(r, one); break;
    case 2: pick_fns_p<KT, 2, MS>(r, one); break;
    default: pick_fns_p<KT, 4, MS>(r, one); break;
  }
}

// Kernels of a plan: by K (power-of-two K use the point-symmetric specialisations,
// which every slot is checked against), with the multi-speed draw when the
// plan's control set has several speeds.
static void select_kernels(int K, int S, int P, const void** r, const void** one) {
  if (S > 1) {
    switch (K) {
      case 4: pick_fns<4, true>(P, r, one); break;
      case 8: pick_fns<8, true>(P, r, one); break;
      case 16: pick_fns<16, true>(P, r, one); break;
      default: pick_fns<32, true>(P, r, one); break;
    }
    return;
  }
  switch (K) {
    case 4: pick_fns<4, false>(P, r, one); break;
    case 8: pick_fns<8, false>(P, r, one); break;
    case 16: pick_fns<16, false>(P, r, one); break;
    case 32: pick_fns<32, false>(P, r, one); break;
    default: pick_fns<0, false>(P, r, one); break;
  }
}

static size_t header_bytes(int n_active) {
  return sizeof(CycleHeader) + (size_t)n_active * sizeof(SlotDev);
}

static cap_status launch_rollout(cap_plan* p, const Entry& e, int variant, hipStream_t s) {
  const uint8_t* base = e.dev;
  uint32_t* q = e.queues;
  void* args[] = {(void*)&base, (void*)&q, (void*)&p->cap_words};
  CAP_HIP(hipLaunchKernel(p->rollout_fn[variant], dim3(p->grid_blocks[variant]), dim3(p->cfg.block_threads), args,
                          window_lds_bytes(p->cap_words, p->per_tile), s));
  return CAP_OK;
}

static cap_status record_graphs(cap_plan* p, Entry& e) {
  hipStream_t s = p->cap_stream;
  hipGraph_t g = nullptr;
  const int minus1 = -1;
  // persistent rollout -> normalise, once per rollout variant (the clear runs
  // in the prelude launch before it)
  for (int v = 0; v < 2; ++v) {
    CAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    cap_status st = launch_rollout(p, e, v, s);
    hipLaunchKernelGGL(plan_normalize_kernel, dim3(4096), dim3(256), 0, s, (const uint8_t*)e.dev,
                       minus1);
    if (p->smooth_blocks > 0)
      hipLaunchKernelGGL(plan_smooth_kernel, dim3(p->smooth_blocks), dim3(kSmoothThreads),
                         smooth_lds_bytes(p->cfg.max_smooth_radius), s, (const uint8_t*)e.dev,
                         minus1);
    hipError_t err = hipStreamEndCapture(s, &g);
    if (st != CAP_OK) return st;
    if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
    CAP_HIP(hipGraphInstantiate(&e.main[v], g, nullptr, nullptr, 0));
    CAP_HIP(hipGraphDestroy(g));
  }
  return CAP_OK;
}

static void destroy_plan(cap_plan* p) {
  if (!p) return;
  for (auto& e : p->ring) {
    for (int v = 0; v < 2; ++v)
      if (e.main[v]) (void)hipGraphExecDestroy(e.main[v]);
    if (e.done) (void)hipEventDestroy(e.done);
    if (e.dev) (void)hipFree(e.dev);
    if (e.host) (void)hipHostFree(e.host);
  }
  if (p->queues) (void)hipFree(p->queues);
  if (p->ev_update) (void)hipEventDestroy(p->ev_update);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

// Cuts the active slots' particles into the three tile kinds of the persistent
// launch.  Work is counted in units of blockDim particles (a human of N
// particles has ceil(N / blockDim) units; its last unit may be partial); a
// kind-k tile holds P >> k units.  With R resident blocks on C CUs and U units
// in all, whole rounds of big tiles (one per block) take the first
// P R floor(U / (P R)) units.  The remainder Ur is spread over the CUs, one
// tile per CU at a time, largest first: one big tile per CU for as long as Ur
// exceeds 4 C; then, for what is left, quarters (Ur <= C), halves and quarters
// (Ur <= 2 C) or big tiles and halves (Ur <= 4 C), with as many tiles as CUs
// (or fewer).  A tile that ends up alone on its CU runs faster than one of a
// pair, so the last tiles even out the CUs rather than the blocks.  Each
// human's units that do not fill a big tile become its own smaller tiles; big
// tiles of the last humans are then split until the targets are met.
// cnt[s][k] is the number of kind-k tiles of slot s.
static void split_tiles(const int32_t* units, int n, int P, int R, int C,
                        int32_t (*cnt)[kTileKinds]) {
  int64_t U = 0;
  for (int i = 0; i < n; ++i) U += units[i];
  int64_t t_half = 0, t_quarter = 0;   // targets (tiles)
  C = std::max(1, std::min(C, R));
  if (P >= 4) {
    int64_t Ur = U % ((int64_t)P * R);
    while (Ur > 4 * (int64_t)C) Ur -= 4 * (int64_t)C;
    if (Ur == 0) {
    } else if (Ur <= C) {
      t_quarter = Ur;
    } else if (Ur <= 2 * (int64_t)C) {
      t_half = Ur - C;
      t_quarter = 2 * (int64_t)C - Ur;
    } else {
      const int64_t big = (Ur - 2 * (int64_t)C + 1) / 2;
      t_half = (Ur - 4 * big) / 2;
      t_quarter = Ur - 4 * big - 2 * t_half;
    }
  } else if (P == 2) {
    // kind 1 is the one-unit tile
    int64_t Ur = U % (2 * (int64_t)R);
    while (Ur > 2 * (int64_t)C) Ur -= 2 * (int64_t)C;
    if (Ur <= C) t_half = Ur;
    else t_half = 2 * (int64_t)C - Ur;
  }
  int64_t have_half = 0, have_quarter = 0;
  for (int i = 0; i < n; ++i) {
    const int u = units[i];
    cnt[i][0] = u / P;
    const int rem = u - cnt[i][0] * P;
    if (P >= 4) {
      cnt[i][1] = rem / 2;
      cnt[i][2] = rem & 1;
    } else {
      cnt[i][1] = rem;   // P == 2: rem is 0 or 1 one-unit tiles; P == 1: 0
      cnt[i][2] = 0;
    }
    have_half += cnt[i][1];
    have_quarter += cnt[i][2];
  }
  int64_t need_half = t_half - have_half, need_quarter = t_quarter - have_quarter;
  for (int i = n - 1; i >= 0 && (need_half > 0 || need_quarter > 0); --i) {
    while (cnt[i][0] > 0 && (need_half > 0 || need_quarter > 0)) {
      --cnt[i][0];
      if (P == 2) {
        cnt[i][1] += 2;
        need_half -= 2;
      } else if (need_half >= 2) {
        cnt[i][1] += 2;
        need_half -= 2;
      } else if (need_half == 1) {
        cnt[i][1] += 1;
        cnt[i][2] += 2;
        need_half -= 1;
        need_quarter -= 2;
      } else {
        cnt[i][2] += 4;
        need_quarter -= 4;
      }
    }
  }
}

static bool same_frame(const cap_grid& a, const cap_grid& b) {
  return a.x0 == b.x0 && a.y0 == b.y0 && a.cell == b.cell && a.nx == b.nx && a.ny == b.ny;
}

// Fills ring entry e's host mirror from the active slots; returns its size.
static size_t build_entry(cap_plan* p, int e, uint64_t seed, uint32_t cycle) {
  uint8_t* hostp = p->ring[e].host;
  CycleHeader* H = reinterpret_cast<CycleHeader*>(hostp);
  SlotDev* out = reinterpret_cast<SlotDev*>(hostp + sizeof(CycleHeader));
  H->seed_lo = (uint32_t)seed;
  H->seed_hi = (uint32_t)(seed >> 32);
  H->cycle = cycle;
  H->per_tile = p->per_tile;
  int n = 0, tiles = 0, steps_total = 0, sblocks = 0, variant = 0;
  int64_t parts = 0, steps = 0;
  for (auto& hs : p->slots) {
    if (!hs.active) continue;
    SlotDev& sd = out[n];
    std::memcpy(&sd, &hs.tmpl, sizeof(SlotDev));
    const int R = p->cfg.ring;
    const int re = (int)(cycle % (uint32_t)R);
    sd.rd.cycle = cycle;
    sd.rd.counts = hs.counts + (size_t)re * hs.n_cells;
    sd.rd.offgrid = hs.offgrid ? hs.offgrid + (size_t)re * sd.rd.H : nullptr;
    sd.probs = hs.probs ? hs.probs + (size_t)re * hs.n_cells : nullptr;
    sd.rd.belief = hs.belief + (size_t)re * sd.bm.G * sd.bm.B;
    sd.n_cells = hs.n_cells;
    sd.reset = hs.reset ? 1 : 0;
    sd.in_union = p->union_dev && sd.probs && same_frame(hs.grid, p->union_frame) ? 1 : 0;
    variant |= sd.rd.shift ? 1 : 0;
    hs.reset = false;
    sd.n_obs = hs.n_staged;
    sd.obs[0] = hs.last[0];
    sd.obs[1] = hs.last[1];
    for (int i = 0; i < 2 * hs.n_staged; ++i) sd.obs[2 + i] = hs.staged[i];
    if (hs.n_staged > 0) {
      hs.last[0] = hs.staged[2 * hs.n_staged - 2];
      hs.last[1] = hs.staged[2 * hs.n_staged - 1];
    }
    hs.n_staged = 0;
    // the rollout starts from the newest observed position (validated at staging)
    sd.rd.X0 = (int32_t)lattice_coord((double)hs.last[0], hs.grid.x0, hs.grid.cell);
    sd.rd.Y0 = (int32_t)lattice_coord((double)hs.last[1], hs.grid.y0, hs.grid.cell);
    sd.prev_x0 = hs.ent_x0[re];
    sd.prev_y0 = hs.ent_y0[re];
    sd.full_clear = hs.ent_full[re] ? 1 : 0;
    hs.ent_x0[re] = sd.rd.X0;
    hs.ent_y0[re] = sd.rd.Y0;
    hs.ent_full[re] = false;
    H->tile_begin[n] = tiles;
    H->step_begin[n] = steps_total;
    H->smooth_begin[n] = sblocks;
    tiles += (int)((sd.rd.N + p->per_tile - 1) / p->per_tile);
    steps_total += sd.rd.H;
    if (sd.smooth_r > 0 && sd.probs)
      sblocks += sd.rd.H * ((sd.rd.ny + kBandRows - 1) / kBandRows) *
                 ((sd.rd.nx + kSmoothThreads - 1) / kSmoothThreads);
    parts += sd.rd.N;
    steps += (int64_t)sd.rd.N * sd.rd.H;
    ++n;
  }
  H->tile_begin[n] = tiles;
  H->step_begin[n] = steps_total;
  H->smooth_begin[n] = sblocks;
  H->n_active = n;
  if (p->union_dev) {
    const int re = (int)(cycle % (uint32_t)p->cfg.ring);
    const size_t cells = (size_t)p->union_H * p->union_frame.nx * p->union_frame.ny;
    H->union_out = p->union_dev + (size_t)re * cells;
    H->union_H = p->union_H;
    H->union_nx = p->union_frame.nx;
    H->union_ny = p->union_frame.ny;
  } else {
    H->union_out = nullptr;
    H->union_H = H->union_nx = H->union_ny = 0;
  }
  p->last_variant = variant;
  // tile kinds of the persistent launch
  {
    const int nthr = p->cfg.block_threads, P = p->cfg.particles_per_thread;
    std::vector<int32_t> units(n);
    std::vector<int32_t> flat((size_t)n * kTileKinds);
    int32_t(*cnt)[kTileKinds] = reinterpret_cast<int32_t(*)[kTileKinds]>(flat.data());
    for (int i = 0; i < n; ++i) units[i] = (int32_t)((out[i].rd.N + nthr - 1) / nthr);
    split_tiles(units.data(), n, P, std::max(1, p->grid_blocks[variant]), p->n_cus, cnt);
    int32_t kb = 0;
    for (int k = 0; k < kTileKinds; ++k) {
      H->kind_begin[k] = kb;
      int32_t in_kind = 0;
      for (int i = 0; i < n; ++i) {
        out[i].kt_begin[k] = in_kind;
        in_kind += cnt[i][k];
      }
      kb += in_kind;
    }
    H->kind_begin[kTileKinds] = kb;
    for (int i = 0; i < n; ++i) {
      int32_t first = 0;
      for (int k = 0; k < kTileKinds; ++k) {
        out[i].kt_first[k] = first;
        first += cnt[i][k] * nthr * std::max(1, P >> k);
      }
    }
    H->n_tiles = kb;
    p->tiles = kb;
  }
  p->particles = parts;
  p->psteps = steps;
  return header_bytes(n);
}

static cap_status wait_entry(cap_plan* p, int e) {
  Entry& en = p->ring[e];
  if (en.pending) {
    CAP_HIP(hipEventSynchronize(en.done));
    en.pending = false;
  }
  return CAP_OK;
}

static cap_status check_position(const HostSlot& hs, float x, float y, int H, int32_t reach) {
  if (!std::isfinite(x) || !std::isfinite(y)) return fail(CAP_E_INVALID, "position is not finite");
  const double X = lattice_coord((double)x, hs.grid.x0, hs.grid.cell);
  const double Y = lattice_coord((double)y, hs.grid.y0, hs.grid.cell);
  const double r = (double)H * (double)reach;
  if (std::fabs(X) + r > 2.1e9 || std::fabs(Y) + r > 2.1e9)
    return fail(CAP_E_INVALID, "position + H steps leave the int32 lattice of the grid");
  return CAP_OK;
}

}  // namespace capred

using namespace capred;

extern "C" cap_status cap_plan_create(const cap_plan_config* cfg_in, cap_plan** out) {
  if (!cfg_in || !out) return fail(CAP_E_INVALID, "config or out is NULL");
  *out = nullptr;
  cap_plan_config cfg = *cfg_in;
  Controls pc;
  cap_status st = make_controls(cfg.K, cfg.speed, cfg.dt, cfg.n_speeds, cfg.speeds, 0u, &pc);
  if (st != CAP_OK) return st;
  if (pc.S > 1 && cfg.K != 4 && cfg.K != 8 && cfg.K != 16 && cfg.K != 32)
    return fail(CAP_E_UNSUPPORTED, "several speeds need K in {4, 8, 16, 32}");
  if (cfg.n_slots < 1 || cfg.n_slots > CAP_MAX_SLOTS) return fail(CAP_E_INVALID, "n_slots out of range");
  if (cfg.max_obs < 1 || cfg.max_obs > kMaxObs) return fail(CAP_E_INVALID, "max_obs must be in [1, 8]");
  if (cfg.ring == 0) cfg.ring = 2;
  if (cfg.ring < 1 || cfg.ring > 4) return fail(CAP_E_INVALID, "ring must be in [1, 4]");
  if (cfg.block_threads == 0) cfg.block_threads = 1024;
  if (cfg.block_threads != 256 && cfg.block_threads != 512 && cfg.block_threads != 1024)
    return fail(CAP_E_INVALID, "block_threads must be 256, 512 or 1024");
  if (cfg.particles_per_thread == 0) cfg.particles_per_thread = 1;
  if (cfg.particles_per_thread != 1 && cfg.particles_per_thread != 2 &&
      cfg.particles_per_thread != 4)
    return fail(CAP_E_INVALID, "particles_per_thread must be 1, 2 or 4");
  if (cfg.lds_bytes == 0) cfg.lds_bytes = 40 * 1024;
  if (cfg.lds_bytes < 2048 || cfg.lds_bytes > 144 * 1024)
    return fail(CAP_E_INVALID, "lds_bytes must be in [2 KiB, 144 KiB]");
  if (cfg.max_smooth_radius < 0 || cfg.max_smooth_radius > kMaxSmoothRadius)
    return fail(CAP_E_INVALID, "max_smooth_radius must be in [0, 16]");
  cap_plan* p = new cap_plan();
  p->cfg = cfg;
  p->slots.resize(cfg.n_slots);
  p->ring.resize(cfg.ring);
  p->per_tile = cfg.block_threads * cfg.particles_per_thread;
  p->cap_words = cfg.lds_bytes / (2 * (int)sizeof(uint32_t));
  select_kernels(cfg.K, pc.S, cfg.particles_per_thread, p->rollout_fn, p->rollout_one_fn);
  const size_t dyn = window_lds_bytes(p->cap_words, p->per_tile);
  hipError_t e = hipSuccess;
  for (int v = 0; v < 2; ++v) {
    e = hipFuncSetAttribute(p->rollout_fn[v], hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    (void)e;  // not required on gfx950; the occupancy query below validates the size
  }
  // each variant's persistent grid fills the chip at that variant's own
  // occupancy (the shifted variant needs more registers)
  int per_cu[2] = {0, 0};
  for (int v = 0; v < 2 && e == hipSuccess; ++v)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[v], p->rollout_fn[v],
                                                     cfg.block_threads, dyn);
  if (e != hipSuccess || per_cu[0] < 1 || per_cu[1] < 1) {
    destroy_plan(p);
    return e != hipSuccess ? hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor")
                           : fail(CAP_E_INVALID, "LDS window too large for one block per CU");
  }
  const int cus = cap_device_cu_count();
  p->n_cus = std::max(1, cus);
  for (int v = 0; v < 2; ++v)
    p->grid_blocks[v] = cfg.grid_blocks > 0 ? cfg.grid_blocks : std::max(1, cus) * per_cu[v];
  p->cfg.grid_blocks = p->grid_blocks[0];
  if (cfg.max_smooth_radius > 0) {
    const size_t sl = smooth_lds_bytes(cfg.max_smooth_radius);
    (void)hipFuncSetAttribute((const void*)plan_smooth_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sl);
    int pc = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, (const void*)plan_smooth_kernel,
                                                     kSmoothThreads, sl);
    if (e != hipSuccess || pc < 1) {
      destroy_plan(p);
      return e != hipSuccess ? hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor")
                             : fail(CAP_E_INVALID, "smoothing tile does not fit a CU");
    }
    p->smooth_blocks = std::max(1, cus) * pc;
  }
  p->entry_bytes = header_bytes(cfg.n_slots);
  hipError_t he;
#define CAP_TRY(call)                       \
  do {                                      \
    he = (call);                            \
    if (he != hipSuccess) {                 \
      destroy_plan(p);                      \
      return hip_fail(he, #call);           \
    }                                       \
  } while (0)
  CAP_TRY(hipMalloc(&p->queues, (size_t)cfg.ring * kQueueWords * sizeof(uint32_t)));
  CAP_TRY(hipMemset(p->queues, 0, (size_t)cfg.ring * kQueueWords * sizeof(uint32_t)));
  for (int e = 0; e < cfg.ring; ++e) p->ring[e].queues = p->queues + (size_t)e * kQueueWords;
  CAP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  CAP_TRY(hipEventCreateWithFlags(&p->ev_update, hipEventDisableTiming));
  for (auto& en : p->ring) {
    CAP_TRY(hipMalloc(&en.dev, p->entry_bytes));
    CAP_TRY(hipMemset(en.dev, 0, p->entry_bytes));
    CAP_TRY(hipHostMalloc(&en.host, p->entry_bytes, hipHostMallocDefault));
    std::memset(en.host, 0, p->entry_bytes);
    CAP_TRY(hipEventCreateWithFlags(&en.done, hipEventDisableTiming));
  }
  CAP_TRY(hipDeviceSynchronize());
#undef CAP_TRY
  for (auto& en : p->ring) {
    st = record_graphs(p, en);
    if (st != CAP_OK) {
      destroy_plan(p);
      return st;
    }
  }
  *out = p;
  return CAP_OK;
}

extern "C" void cap_plan_destroy(cap_plan* plan) {
  if (!plan) return;
  for (int e = 0; e < (int)plan->ring.size(); ++e) (void)wait_entry(plan, e);
  destroy_plan(plan);
}

extern "C" cap_status cap_plan_set_slot(cap_plan* p, int32_t slot, const cap_slot_desc* d) {
  if (!p || !d) return fail(CAP_E_INVALID, "plan or desc is NULL");
  if (slot < 0 || slot >= p->cfg.n_slots) return fail(CAP_E_INVALID, "slot out of range");
  HostSlot& hs = p->slots[slot];
  if (hs.active) return fail(CAP_E_CAPACITY, "slot is occupied");
  cap_model m{p->cfg.K, p->cfg.speed, p->cfg.dt, d->B, d->beta, d->G, d->goals,
              p->cfg.n_speeds, p->cfg.speeds, d->speed_mask};
  Controls c;
  cap_status st = check_model(&m, &c);
  if (st != CAP_OK) return st;
  if ((st = check_grid(&d->grid)) != CAP_OK) return st;
  if (!d->counts_dev || !d->log_belief_dev || !d->belief_dev)
    return fail(CAP_E_INVALID, "counts, log_belief and belief buffers are required");
  if ((st = check_smoothing(d->smooth_sigma, d->smooth_radius, p->cfg.max_smooth_radius)) !=
      CAP_OK)
    return st;
  if (d->smooth_radius > 0 && !d->probs_dev)
    return fail(CAP_E_INVALID, "smoothing needs probs_dev");
  HostSlot ns;
  std::memset(&ns.tmpl, 0, sizeof(SlotDev));
  st = make_rollout_desc(c, m.dt, m.B, m.beta, m.G, m.goals, d->grid, d->N, d->H, &ns.tmpl.rd);
  if (st != CAP_OK) return st;
  ns.grid = d->grid;
  if ((m.K == 4 || m.K == 8 || m.K == 16 || m.K == 32) && !ns.tmpl.rd.sym)
    return fail(CAP_E_UNSUPPORTED, "the lattice step table of this grid is not point-symmetric");
  if ((st = check_position(ns, d->last_xy[0], d->last_xy[1], d->H,
                           std::max(ns.tmpl.rd.Rx, ns.tmpl.rd.Ry))) != CAP_OK)
    return st;
  ns.tmpl.rd.human = d->human_id;
  ns.tmpl.bm = make_belief_model(c, m.dt, m.B, m.beta, m.G, m.goals);
  ns.tmpl.log_belief = d->log_belief_dev;
  ns.tmpl.smooth_r = d->smooth_radius;
  smooth_weights(d->smooth_sigma, d->smooth_radius, &ns.tmpl.smooth_w);
  ns.counts = d->counts_dev;
  ns.offgrid = d->offgrid_dev;
  ns.probs = d->probs_dev;
  ns.belief = d->belief_dev;
  ns.n_cells = (int64_t)d->H * d->grid.nx * d->grid.ny;
  ns.last[0] = d->last_xy[0];
  ns.last[1] = d->last_xy[1];
  ns.reset = d->reset_belief != 0;
  ns.active = true;
  hs = ns;
  return CAP_OK;
}

extern "C" cap_status cap_plan_clear_slot(cap_plan* p, int32_t slot) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (slot < 0 || slot >= p->cfg.n_slots) return fail(CAP_E_INVALID, "slot out of range");
  p->slots[slot].active = false;
  p->slots[slot].n_staged = 0;
  return CAP_OK;
}

extern "C" cap_status cap_plan_set_speed_mask(cap_plan* p, int32_t slot, uint32_t mask) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (slot < 0 || slot >= p->cfg.n_slots || !p->slots[slot].active)
    return fail(CAP_E_INVALID, "slot is not active");
  return set_speed_mask(&p->slots[slot].tmpl.rd, mask);
}

extern "C" cap_status cap_plan_reset_belief(cap_plan* p, int32_t slot) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (slot < 0 || slot >= p->cfg.n_slots || !p->slots[slot].active)
    return fail(CAP_E_INVALID, "slot is not active");
  p->slots[slot].reset = true;
  return CAP_OK;
}

extern "C" cap_status cap_plan_stage_obs(cap_plan* p, int32_t slot, const float* xy,
                                         int32_t n_new) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (slot < 0 || slot >= p->cfg.n_slots || !p->slots[slot].active)
    return fail(CAP_E_INVALID, "slot is not active");
  HostSlot& hs = p->slots[slot];
  if (n_new < 0 || hs.n_staged + n_new > p->cfg.max_obs)
    return fail(CAP_E_CAPACITY, "more staged observations than max_obs");
  if (n_new > 0 && !xy) return fail(CAP_E_INVALID, "xy is NULL");
  const int32_t reach = std::max(hs.tmpl.rd.Rx, hs.tmpl.rd.Ry);
  for (int i = 0; i < n_new; ++i) {
    cap_status st = check_position(hs, xy[2 * i], xy[2 * i + 1], hs.tmpl.rd.H, reach);
    if (st != CAP_OK) return st;
  }
  for (int i = 0; i < 2 * n_new; ++i) hs.staged[2 * hs.n_staged + i] = xy[i];
  hs.n_staged += n_new;
  return CAP_OK;
}

extern "C" cap_status cap_plan_stage_obs_many(cap_plan* p, int32_t n, const int32_t* slots,
                                              const float* xy) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (n < 0) return fail(CAP_E_INVALID, "n must be >= 0");
  if (n > 0 && (!slots || !xy)) return fail(CAP_E_INVALID, "slots or xy is NULL");
  // validate every entry first, so that a rejected call stages nothing
  std::vector<int32_t> adds((size_t)p->cfg.n_slots, 0);
  for (int i = 0; i < n; ++i) {
    const int32_t slot = slots[i];
    if (slot < 0 || slot >= p->cfg.n_slots || !p->slots[slot].active)
      return fail(CAP_E_INVALID, "slot is not active");
    const HostSlot& hs = p->slots[slot];
    if (hs.n_staged + ++adds[slot] > p->cfg.max_obs)
      return fail(CAP_E_CAPACITY, "more staged observations than max_obs");
    const int32_t reach = std::max(hs.tmpl.rd.Rx, hs.tmpl.rd.Ry);
    cap_status st = check_position(hs, xy[2 * i], xy[2 * i + 1], hs.tmpl.rd.H, reach);
    if (st != CAP_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    HostSlot& hs = p->slots[slots[i]];
    hs.staged[2 * hs.n_staged] = xy[2 * i];
    hs.staged[2 * hs.n_staged + 1] = xy[2 * i + 1];
    ++hs.n_staged;
  }
  return CAP_OK;
}

static cap_status begin_cycle(cap_plan* p, uint64_t seed, uint32_t cycle, hipStream_t s,
                              int* e_out, size_t* bytes) {
  if (cycle >= 0x7FFFFFFFu) return fail(CAP_E_INVALID, "cycle must be < 2^31 - 1");
  const int e = (int)(cycle % (uint32_t)p->cfg.ring);
  cap_status st = wait_entry(p, e);
  if (st != CAP_OK) return st;
  *bytes = build_entry(p, e, seed, cycle);
  CAP_HIP(hipMemcpyAsync(p->ring[e].dev, p->ring[e].host, *bytes, hipMemcpyHostToDevice, s));
  if (p->have_last && p->last_stream != s) CAP_HIP(hipStreamWaitEvent(s, p->ev_update, 0));
  *e_out = e;
  p->last_run_entry = e;
  return CAP_OK;
}

extern "C" cap_status cap_plan_run(cap_plan* p, uint64_t seed, uint32_t cycle, void* stream) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  hipStream_t s = as_stream(stream);
  int e = 0;
  size_t bytes = 0;
  cap_status st = begin_cycle(p, seed, cycle, s, &e, &bytes);
  if (st != CAP_OK) return st;
  Entry& en = p->ring[e];
  // belief update and grid clear in one direct launch (a graph of one node
  // costs more host time), then its event, which the next cycle's stream waits on
  hipLaunchKernelGGL(plan_prelude_kernel, dim3(p->cfg.n_slots + kZeroBlocks), dim3(kBeliefThreads),
                     0, s, (const uint8_t*)en.dev, en.queues, p->cfg.n_slots);
  CAP_HIP(hipGetLastError());
  CAP_HIP(hipEventRecord(p->ev_update, s));
  CAP_HIP(hipGraphLaunch(en.main[p->last_variant], s));
  CAP_HIP(hipEventRecord(en.done, s));
  en.pending = true;
  p->last_stream = s;
  p->have_last = true;
  return CAP_OK;
}

extern "C" cap_status cap_plan_run_plain(cap_plan* p, uint64_t seed, uint32_t cycle,
                                         void* stream) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  hipStream_t s = as_stream(stream);
  int e = 0;
  size_t bytes = 0;
  cap_status st = begin_cycle(p, seed, cycle, s, &e, &bytes);
  if (st != CAP_OK) return st;
  Entry& en = p->ring[e];
  const CycleHeader* H = reinterpret_cast<const CycleHeader*>(en.host);
  const SlotDev* sl = reinterpret_cast<const SlotDev*>(en.host + sizeof(CycleHeader));
  const uint8_t* base = en.dev;
  for (int i = 0; i < H->n_active; ++i) {
    hipLaunchKernelGGL(plan_update_kernel, dim3(1), dim3(kBeliefThreads), 0, s, base, i);
    if (i == H->n_active - 1) CAP_HIP(hipEventRecord(p->ev_update, s));
    const unsigned zb = (unsigned)std::min(sl[i].rd.H, 2048);
    hipLaunchKernelGGL(plan_zero_kernel, dim3(zb), dim3(256), 0, s, base, en.queues, i);
    const int tiles = H->tile_begin[i + 1] - H->tile_begin[i];
    int si = i;
    void* args[] = {(void*)&base, (void*)&si, (void*)&p->cap_words};
    CAP_HIP(hipLaunchKernel(p->rollout_one_fn[sl[i].rd.shift ? 1 : 0], dim3(tiles), dim3(p->cfg.block_threads), args,
                            window_lds_bytes(p->cap_words, p->per_tile), s));
    if (sl[i].probs && sl[i].smooth_r == 0) {
      const unsigned nb = (unsigned)std::min(4 * sl[i].rd.H, 4096);
      hipLaunchKernelGGL(plan_normalize_kernel, dim3(nb), dim3(256), 0, s, base, i);
    }
    if (sl[i].probs && sl[i].smooth_r > 0) {
      const int nb = std::min(H->smooth_begin[i + 1] - H->smooth_begin[i], 4096);
      hipLaunchKernelGGL(plan_smooth_kernel, dim3(nb), dim3(kSmoothThreads),
                         smooth_lds_bytes(sl[i].smooth_r), s, base, i);
    }
  }
  if (H->n_active == 0) CAP_HIP(hipEventRecord(p->ev_update, s));
  CAP_HIP(hipGetLastError());
  CAP_HIP(hipEventRecord(en.done, s));
  en.pending = true;
  p->last_stream = s;
  p->have_last = true;
  return CAP_OK;
}

extern "C" cap_status cap_plan_replay_rollout(cap_plan* p, void* stream, void* ev_start,
                                              void* ev_end) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (p->last_run_entry < 0) return fail(CAP_E_INVALID, "no cycle has run on this plan");
  hipStream_t s = as_stream(stream);
  const Entry& en = p->ring[p->last_run_entry];
  const int replay = -2;  // every slot, union grid untouched
  hipLaunchKernelGGL(plan_zero_kernel, dim3(kZeroBlocks), dim3(256), 0, s, (const uint8_t*)en.dev,
                     en.queues, replay);
  if (ev_start) CAP_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(ev_start), s));
  cap_status st = launch_rollout(p, en, p->last_variant, s);
  if (st != CAP_OK) return st;
  if (ev_end) CAP_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(ev_end), s));
  CAP_HIP(hipGetLastError());
  return CAP_OK;
}

extern "C" cap_status cap_plan_sync(cap_plan* p) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  for (int e = 0; e < (int)p->ring.size(); ++e) {
    cap_status st = wait_entry(p, e);
    if (st != CAP_OK) return st;
  }
  return CAP_OK;
}

extern "C" cap_status cap_plan_stats(const cap_plan* p, int64_t* particles,
                                     int64_t* particle_steps, int32_t* tiles) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  int64_t parts = 0, steps = 0;
  int32_t t = 0;
  for (const auto& hs : p->slots) {
    if (!hs.active) continue;
    parts += hs.tmpl.rd.N;
    steps += (int64_t)hs.tmpl.rd.N * hs.tmpl.rd.H;
    t += (int32_t)((hs.tmpl.rd.N + p->per_tile - 1) / p->per_tile);
  }
  if (particles) *particles = parts;
  if (particle_steps) *particle_steps = steps;
  if (tiles) *tiles = t;
  return CAP_OK;
}

extern "C" cap_status cap_plan_tile_split(const int32_t* units, int32_t n,
                                          int32_t particles_per_thread, int32_t resident_blocks,
                                          int32_t cus, int32_t* counts) {
  if (n < 0 || n > CAP_MAX_SLOTS) return fail(CAP_E_INVALID, "n must be in [0, CAP_MAX_SLOTS]");
  if (particles_per_thread != 1 && particles_per_thread != 2 && particles_per_thread != 4)
    return fail(CAP_E_INVALID, "particles_per_thread must be 1, 2 or 4");
  if (resident_blocks < 1 || cus < 1) return fail(CAP_E_INVALID, "resident_blocks and cus >= 1");
  if (n > 0 && (!units || !counts)) return fail(CAP_E_INVALID, "units or counts is NULL");
  for (int i = 0; i < n; ++i)
    if (units[i] < 0) return fail(CAP_E_INVALID, "units must be >= 0");
  split_tiles(units, n, particles_per_thread, resident_blocks, cus,
              reinterpret_cast<int32_t(*)[kTileKinds]>(counts));
  return CAP_OK;
}

extern "C" cap_status cap_plan_set_union(cap_plan* p, const cap_grid* frame, int32_t H,
                                         float* union_dev) {
  if (!p) return fail(CAP_E_INVALID, "plan is NULL");
  if (!union_dev) {
    p->union_dev = nullptr;
    p->union_H = 0;
    return CAP_OK;
  }
  cap_status st = check_grid(frame);
  if (st != CAP_OK) return st;
  if (H < 1 || H > 4096) return fail(CAP_E_INVALID, "union H must be in [1, 4096]");
  p->union_frame = *frame;
  p->union_H = H;
  p->union_dev = union_dev;
  return CAP_OK;
}

extern "C" cap_status cap_plan_tuning(const cap_plan* p, cap_plan_config* out) {
  if (!p || !out) return fail(CAP_E_INVALID, "plan or out is NULL");
  *out = p->cfg;
  return CAP_OK;
}
