// batch.hip -- an ensemble of fully periodic lattices of uneven size, each with
// its own relaxation time, advanced together: each time step walks a work list
// of (lattice, cell range) items in one launch (phase 0) or one launch per
// lane width (phase 1), and runs of steps replay as one captured HIP graph.
//
// The per-cell update is the same fused BGK collide-and-stream as the single
// lattice path (OpenLB User Guide 1.6, Introduction, collision and streaming
// equations; Core Concepts, BGK listing), in the same in-place AA layout, so
// every lattice of a batch is also an ordinary lattice handle (a view) whose
// populations, moments and totals are read with the single-lattice calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "fluid_path.hpp"
#include "handle.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;
using lbm_detail::fail;

namespace {

struct BatchLat {
  uint64_t pop_off;  // element offset of the lattice's populations in the batch buffer
  int nx, ny, nz;
  int px;      // cells from one stored x-row to the next (member_pitch)
  uint32_t N;  // stored cells, px ny nz (phase 0 also runs over the padding slots)
  PopIndex pix;  // placement of the lattice's populations
  double omega;
  int c;    // phase-1 cells per lane (row_lane_cells); phase 0 always moves 8 bytes a lane
  int tpr;  // lanes per x-row = nx / c
};

// A work item carries its lattice's parameters, so a block needs one scalar
// load (no dependent second load) before it can address memory.
struct BatchItem {
  uint64_t pop_off;
  double omega;
  int px;
  PopIndex pix;
  int nx, ny, nz;
  int c, tpr;
  uint32_t first;  // phase 0: first cell; phase 1: first x-row
  uint32_t count;  // phase 0: cells; phase 1: rows
};

// One launch advances every lattice of the batch through one phase; phase 1
// takes one launch per lane width LC (cells per lane of its items' rows), so
// each width gets the registers, and with them the occupancy, of its own row
// body instead of the widest body's.  Items never span two lattices, so a
// block's lattice is uniform and the barriers of the phase-1 row body are
// reached by the whole block.
template <int Q, typename S, bool SHIFT, int PHASE, int LC>
__global__ void __launch_bounds__(512)
    batch_step_kernel(S* __restrict__ base, const BatchItem* __restrict__ items, int nitems) {
  using T = typename Store<S>::T;
  constexpr int CM = Pack8<S>::C;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  for (int it = (int)blockIdx.x; it < nitems; it += (int)gridDim.x) {
    // 16-bit phase 0 walks the items in descending order, so that it starts
    // on the rows phase 1 wrote last (ensemble FP16 step 321.4 -> 318.7 us;
    // FP32 and phase 1 unchanged).  Phase 1 with one block per item deals
    // runs of XCD_RUN consecutive items to one XCD (the hardware deals blocks
    // to the 8 XCDs in turn: blocks b, b + 8, b + 16, ... share one), so that
    // the lines consecutive items share at their row ends are fetched into
    // one L2 (ensemble step FP32 0.641 -> 0.619 ms, FP16 0.322 -> 0.305 ms;
    // runs of 2 / 16 / 256 items: 0.633 / 0.621 / 0.622 and 0.316 / 0.306 /
    // 0.311 ms).
    constexpr int XCD_RUN = 64;
    int itx = (PHASE == 0 && sizeof(S) == 2) ? nitems - 1 - it : it;
    if (PHASE == 1 && (int)gridDim.x == nitems && it < nitems / (8 * XCD_RUN) * (8 * XCD_RUN))
      itx = XCD_RUN * (8 * (it / (8 * XCD_RUN)) + (it & 7)) + ((it >> 3) % XCD_RUN);
    const BatchItem item = items[itx];
    const BatchItem& L = item;
    StepParams<T> p{};
    p.base = (T)Store<S>::unit;
    p.omega = (T)L.omega;
    p.kguo = (T)(1.0 - 0.5 * L.omega);
    S* pop = base + L.pop_off;
    if (PHASE == 0) {
      // 8 bytes a lane whatever nx is: phase 0 is local to each cell, and a
      // lane that runs past the last cell only touches padding slots (the
      // population runs are padded to a multiple of 64 cells or whole chunks)
      const uint32_t c0 = item.first + (uint32_t)CM * threadIdx.x;
      if (c0 < item.first + item.count) fluid_cells_p0<Q, S, SHIFT, CM>(pop, L.pix, c0, p);
    } else {
      const int rloc = (int)threadIdx.x / L.tpr;
      const int t = (int)threadIdx.x - rloc * L.tpr;
      const bool active = rloc < (int)item.count;
      const int row = (int)item.first + rloc;
      S* tile = (S*)smem_raw + (size_t)rloc * Shifted<Q>::count() * L.px;
      // only 16-bit members have padded rows (member_pitch).  FP32 rows load
      // through the caches (measured: ensemble phase 1 755 -> 721 us; 16-bit
      // storage gains nothing, and the single lattice's 256-cell rows lose)
      fluid_rows_p1<Q, S, SHIFT, LC, sizeof(S) == 2, sizeof(S) != 4>(
          pop, L.nx, L.px, L.ny, L.nz, L.pix, row, active, t, tile, p);
      __syncthreads();  // the next item reuses the LDS tile
    }
  }
}

// Phase 0 over every item, or phase 1 over the items of lane width lc.
template <int Q, typename S, bool SHIFT>
void launch_batch(const void* base, const BatchItem* items, int nitems, int phase, int lc,
                  int grid, int threads, size_t lds0, hipStream_t stream) {
  constexpr int CM = Pack8<S>::C;
  if (phase == 0) {
    // lds0: unused LDS that only caps the resident blocks per CU (0 = none)
    hipLaunchKernelGGL((batch_step_kernel<Q, S, SHIFT, 0, CM>), dim3(grid), dim3(threads), lds0,
                       stream, (S*)base, items, nitems);
    return;
  }
  const size_t lds = (size_t)threads * CM * Shifted<Q>::count() * sizeof(S);
  if (lc == CM)
    hipLaunchKernelGGL((batch_step_kernel<Q, S, SHIFT, 1, CM>), dim3(grid), dim3(threads), lds,
                       stream, (S*)base, items, nitems);
  else if (CM == 4 && lc == 2)
    hipLaunchKernelGGL((batch_step_kernel<Q, S, SHIFT, 1, (CM == 4 ? 2 : 1)>), dim3(grid),
                       dim3(threads), lds, stream, (S*)base, items, nitems);
  else
    hipLaunchKernelGGL((batch_step_kernel<Q, S, SHIFT, 1, 1>), dim3(grid), dim3(threads), lds,
                       stream, (S*)base, items, nitems);
}

using LaunchFn = void (*)(const void*, const BatchItem*, int, int, int, int, int, size_t,
                           hipStream_t);

template <int Q, bool SHIFT>
LaunchFn launch_for_storage(int s) {
  switch (s) {
    case LBM_STORE_F64: return launch_batch<Q, double, SHIFT>;
    case LBM_STORE_F32: return launch_batch<Q, float, SHIFT>;
    case LBM_STORE_F16: return launch_batch<Q, _Float16, SHIFT>;
    default: return launch_batch<Q, bf16s, SHIFT>;
  }
}

LaunchFn launcher(int q, int storage, bool shifted) {
  if (q == 9) return shifted ? launch_for_storage<9, true>(storage) : launch_for_storage<9, false>(storage);
  return shifted ? launch_for_storage<19, true>(storage) : launch_for_storage<19, false>(storage);
}

constexpr int MIN_THREADS = 128;  // smallest block; sizes the phase-0 item table
constexpr int MAX_THREADS = 512;

// Stored row pitch of a member with rows of nx cells in s-byte storage: odd
// rows of 16-bit storage get one padding slot, so that they too move 2 cells
// (4 bytes) a lane in phase 1 instead of 1 (phase 1 FP16 on the ensemble,
// 1-cell rows 4.4 TB/s against 5.9 for 2-cell rows).
int member_pitch(int nx, size_t s) { return (s == 2 && nx % 2 == 1) ? nx + 1 : nx; }

// Phase-1 cells per lane for rows of nx cells in s-byte storage: the widest
// aligned lane (8, then 4 bytes) whose cell count divides nx, else 1; except
// that 16-bit rows take 2 cells (4 bytes) a lane wherever a row fits the
// block, measured faster than 4 on the ensemble (phase 1 FP16 432 -> 408-415
// us), whose row body needs 162 VGPRs against 93.
int row_lane_cells(int nx, size_t s) {
  const int cmax = 8 / (int)s;
  if (cmax == 4 && nx % 2 == 0 && nx / 2 <= MAX_THREADS) return 2;
  if (nx % cmax == 0) return cmax;
  if (cmax == 4 && nx % 2 == 0) return 2;
  return 1;
}
const int THREAD_CHOICES[] = {128, 256, 512};
// 0 = one block per item (the grid covers the whole work list); otherwise
// that many resident blocks per compute unit loop over the items
const int BLOCKS_PER_CU_CHOICES[] = {0, 2, 4, 8, 16};

struct BatchLayout {
  std::vector<size_t> pop_off, aux_off, aux_size;  // bytes, per lattice
  size_t pop_total = 0, items0_off = 0, items1_off = 0, scratch_off = 0, scratch_bytes = 0,
         aux_total = 0;
  size_t max_items0 = 0, max_items1 = 0;
};

lbm_status batch_layout(lbm_descriptor d, int count, const int* dims, lbm_storage s,
                        BatchLayout* L, std::string* why) {
  if (count <= 0 || !dims) {
    *why = "count must be positive and dims non-NULL";
    return LBM_ERR_ARG;
  }
  L->pop_off.resize(count);
  L->aux_off.resize(count);
  L->aux_size.resize(count);
  size_t pop = 0, aux = 0, items0 = 0, items1 = 0, max_cells = 0;
  for (int b = 0; b < count; ++b) {
    size_t pb = 0;
    const int px = dims[3 * b] > 0 ? member_pitch(dims[3 * b], storage_bytes(s)) : dims[3 * b];
    lbm_status st = lbm_required_bytes(d, px, dims[3 * b + 1], dims[3 * b + 2], s, &pb, nullptr);
    if (st) {
      *why = "lattice " + std::to_string(b) + ": " + lbm_last_error(nullptr);
      return st;
    }
    const size_t N = (size_t)dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
    // a member's aux holds no scratch of its own: the members share one
    const size_t ab = aux_layout(N, 0).total;
    L->pop_off[b] = pop;
    L->aux_off[b] = aux;
    L->aux_size[b] = ab;
    pop += pb;  // each part is a multiple of 256 bytes
    aux += ab;
    max_cells = std::max(max_cells, N);
    const int lanes = px / row_lane_cells(px, storage_bytes(s));
    if (lanes > MAX_THREADS) {
      *why = "lattice " + std::to_string(b) + ": an x-row needs " + std::to_string(lanes) +
             " lanes, more than " + std::to_string(MAX_THREADS);
      return LBM_ERR_UNSUPPORTED;
    }
    // at least one lane-cell per thread, over the stored cells
    items0 += ((size_t)px * dims[3 * b + 1] * dims[3 * b + 2] + MIN_THREADS - 1) / MIN_THREADS;
    items1 += (size_t)dims[3 * b + 1] * dims[3 * b + 2];  // at most one row per item
  }
  if (pop / storage_bytes(s) >= 4294967296.0) {
    *why = "the batch's populations exceed 2^32 elements";
    return LBM_ERR_UNSUPPORTED;
  }
  L->pop_total = pop;
  L->items0_off = align256(aux);
  L->items1_off = align256(L->items0_off + sizeof(BatchItem) * items0);
  L->max_items0 = items0;
  L->max_items1 = items1;
  L->scratch_off = align256(L->items1_off + sizeof(BatchItem) * items1);
  L->scratch_bytes = scratch_size(max_cells);
  L->aux_total = align256(L->scratch_off + L->scratch_bytes);
  return LBM_OK;
}

}  // namespace

struct lbm_batch {
  int desc = 0, q = 0, count = 0, storage = 0;
  bool shifted = false;
  unsigned char* pop = nullptr;
  unsigned char* aux = nullptr;
  hipStream_t stream = nullptr;
  int device = 0, num_cu = 0;
  int lds_per_cu = 0;  // bytes of LDS per compute unit (phase-0 occupancy cap; 0 = unknown)
  BatchLayout lay;
  std::vector<lbm_lattice*> views;
  std::vector<BatchLat> lats;
  long long total_cells = 0;
  // launch shape per propagation phase: threads per block and resident
  // blocks per CU (0 = one block per work item)
  int threads[2] = {256, 256}, blocks_per_cu[2] = {8, 8};
  int nitems0 = 0, nitems1 = 0;
  // phase-1 items by lane width: the table holds the items of width lane_c[k]
  // at lane_first[k] .. lane_first[k] + lane_n[k] - 1 (widest first)
  int lane_c[3] = {0, 0, 0}, lane_first[3] = {0, 0, 0}, lane_n[3] = {0, 0, 0};
  int max_tpr = 1;  // widest row in lanes: blocks need at least this many threads
  // the device item tables match nitems0 / nitems1 / lane_*; false after a
  // HIP failure while uploading them (stepping is refused until a rebuild)
  bool tables_ok = false;
  int graph_steps = 0;
  hipGraphExec_t graph = nullptr;
  std::string err;
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}

#define BHIP_TRY(b, call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail((b), LBM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

void drop_batch_graph(lbm_batch* b) {
  if (b->graph) {
    // a replay may still be running on the batch's stream
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
}

// Cut every lattice into phase-0 items (runs of t0 lanes of 8 bytes) and
// phase-1 items (as many whole x-rows as t1 lanes hold).
lbm_status build_items(lbm_batch* b, int t0, int t1) {
  if (t1 < b->max_tpr)
    return bfail(b, LBM_ERR_ARG, "phase-1 threads per block must cover the widest row (" +
                                     std::to_string(b->max_tpr) + " lanes)");
  std::vector<BatchItem> i0, i1;
  i0.reserve(b->lay.max_items0);
  i1.reserve(b->lay.max_items1);
  for (int l = 0; l < b->count; ++l) {
    const BatchLat& L = b->lats[l];
    BatchItem it{L.pop_off, L.omega, L.px, L.pix, L.nx, L.ny, L.nz, L.c, L.tpr, 0, 0};
    const uint32_t chunk = (uint32_t)t0 * (uint32_t)(8 / storage_bytes(b->storage));
    for (uint32_t c = 0; c < L.N; c += chunk) {
      it.first = c;
      it.count = std::min<uint32_t>(chunk, L.N - c);
      i0.push_back(it);
    }
    const uint32_t rows = (uint32_t)L.ny * (uint32_t)L.nz;
    const uint32_t per = (uint32_t)(t1 / L.tpr);
    for (uint32_t r = 0; r < rows; r += per) {
      it.first = r;
      it.count = std::min<uint32_t>(per, rows - r);
      i1.push_back(it);
    }
  }
  // group the phase-1 items by lane width (one launch per width)
  std::stable_sort(i1.begin(), i1.end(),
                   [](const BatchItem& a, const BatchItem& c) { return a.c > c.c; });
  int lane_c[3] = {0, 0, 0}, lane_first[3] = {0, 0, 0}, lane_n[3] = {0, 0, 0};
  int nk = 0;
  for (size_t k = 0; k < i1.size(); ++k) {
    if (k == 0 || i1[k].c != i1[k - 1].c) {
      if (nk == 3) return bfail(b, LBM_ERR_ARG, "more than three lane widths");  // 1, 2 and 4 only
      lane_c[nk] = i1[k].c;
      lane_first[nk] = (int)k;
      ++nk;
    }
    ++lane_n[nk - 1];
  }
  if (i0.size() > b->lay.max_items0 || i1.size() > b->lay.max_items1)
    return bfail(b, LBM_ERR_ARG, "item table overflow");
  // from here on the device tables change: the batch describes them again
  // only once both uploads have completed
  b->tables_ok = false;
  BHIP_TRY(b, hipMemcpyAsync(b->aux + b->lay.items0_off, i0.data(), sizeof(BatchItem) * i0.size(),
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->aux + b->lay.items1_off, i1.data(), sizeof(BatchItem) * i1.size(),
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  for (int k = 0; k < 3; ++k) {
    b->lane_c[k] = lane_c[k];
    b->lane_first[k] = lane_first[k];
    b->lane_n[k] = lane_n[k];
  }
  b->nitems0 = (int)i0.size();
  b->nitems1 = (int)i1.size();
  b->threads[0] = t0;
  b->threads[1] = t1;
  b->tables_ok = true;
  drop_batch_graph(b);
  return LBM_OK;
}

void launch_one(lbm_batch* b, int phase) {
  const LaunchFn fn = launcher(b->q, b->storage, b->shifted);
  const int bpc = b->blocks_per_cu[phase];
  auto grid_for = [&](int n) {
    return bpc == 0 ? std::max(1, n) : std::max(1, std::min(n, bpc * b->num_cu));
  };
  if (phase == 0) {
    // One block per item in 128-thread blocks: at most four resident per CU,
    // as the single lattice's phase 0 (ensemble FP32 phase 0 562 against 580
    // us uncapped; wider blocks and FP16 measured no gain from a cap)
    size_t lds0 = 0;
    if (bpc == 0 && b->threads[0] == 128 && b->lds_per_cu > 0) {
      const size_t cap = (size_t)(b->lds_per_cu / 4) & ~(size_t)1023;
      if (cap <= 65536) lds0 = cap;
    }
    fn(b->pop, (const BatchItem*)(b->aux + b->lay.items0_off), b->nitems0, 0, 0,
       grid_for(b->nitems0), b->threads[0], lds0, b->stream);
    return;
  }
  const BatchItem* items1 = (const BatchItem*)(b->aux + b->lay.items1_off);
  for (int k = 0; k < 3; ++k)
    if (b->lane_n[k] > 0)
      fn(b->pop, items1 + b->lane_first[k], b->lane_n[k], 1, b->lane_c[k], grid_for(b->lane_n[k]),
         b->threads[1], 0, b->stream);
}

lbm_status benter(lbm_batch* b) {
  if (!b) return LBM_ERR_ARG;
  b->err.clear();
  BHIP_TRY(b, hipSetDevice(b->device));
  return LBM_OK;
}

// All views must be initialised and in the same propagation phase.
lbm_status common_phase(lbm_batch* b, int* phase) {
  for (int l = 0; l < b->count; ++l) {
    const lbm_lattice* v = b->views[l];
    if (!v->initialized)
      return bfail(b, LBM_ERR_STATE, "lattice " + std::to_string(l) + " is not initialised");
    if (!v->consistent)
      return bfail(b, LBM_ERR_STATE, "lattice " + std::to_string(l) +
                                         ": a HIP failure interrupted an earlier step; initialise "
                                         "the populations again");
    if (v->phase != b->views[0]->phase)
      return bfail(b, LBM_ERR_STATE, "lattices are in different propagation phases");
  }
  *phase = b->views[0]->phase;
  return LBM_OK;
}

void advance_views(lbm_batch* b, int n) {
  for (lbm_lattice* v : b->views) {
    v->phase ^= (n & 1);
    v->steps += n;
  }
}

// Enqueue n steps of every member from propagation phase `phase` (graph
// replays where set up).  Returns LBM_ERR_HIP on a HIP failure.
lbm_status enqueue_batch_steps(lbm_batch* b, int n, int phase) {
  int left = n;
  if (b->graph_steps > 0 && n >= b->graph_steps) {
    if (phase != 0) {
      launch_one(b, 1);
      phase = 0;
      --left;
    }
    if (!b->graph && left >= b->graph_steps) {
      hipGraph_t g = nullptr;
      BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      for (int s = 0; s < b->graph_steps; ++s) launch_one(b, s & 1);
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      }
      e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->graph = nullptr;
        return bfail(b, LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
    }
    while (b->graph && left >= b->graph_steps) {
      BHIP_TRY(b, hipGraphLaunch(b->graph, b->stream));
      left -= b->graph_steps;
    }
  }
  for (int s = 0; s < left; ++s) {
    launch_one(b, phase);
    phase ^= 1;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_required_bytes(lbm_descriptor d, int count, const int* dims, lbm_storage s,
                                    size_t* pop_bytes, size_t* aux_bytes) {
  BatchLayout L;
  std::string why;
  lbm_status st = batch_layout(d, count, dims, s, &L, &why);
  if (st) return lbm_detail::fail(nullptr, st, why);
  if (pop_bytes) *pop_bytes = L.pop_total;
  if (aux_bytes) *aux_bytes = L.aux_total;
  return LBM_OK;
}

lbm_status lbm_batch_create(lbm_batch** out, lbm_descriptor d, int count, const int* dims,
                            const double* tau, lbm_storage s, unsigned flags, void* dev_pop,
                            size_t pop_bytes, void* dev_aux, size_t aux_bytes, void* hip_stream) {
  if (!out) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  BatchLayout L;
  std::string why;
  lbm_status st = batch_layout(d, count, dims, s, &L, &why);
  if (st) return lbm_detail::fail(nullptr, st, why);
  if (!tau) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "tau is NULL");
  if (!dev_pop || !dev_aux) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "device buffers must not be NULL");
  if (pop_bytes < L.pop_total || aux_bytes < L.aux_total)
    return lbm_detail::fail(nullptr, LBM_ERR_ARG, "buffers smaller than lbm_batch_required_bytes");
  if (((uintptr_t)dev_pop & 255u) || ((uintptr_t)dev_aux & 255u))
    return lbm_detail::fail(nullptr, LBM_ERR_ARG, "device buffers must be 256-byte aligned");
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "out of host memory");
  b->desc = d;
  b->q = qof(d);
  b->count = count;
  b->storage = s;
  b->shifted = (flags & LBM_FLAG_SHIFTED) != 0;
  b->pop = (unsigned char*)dev_pop;
  b->aux = (unsigned char*)dev_aux;
  b->stream = (hipStream_t)hip_stream;
  b->lay = L;
  auto undo = [&](lbm_status code, const std::string& msg) {
    for (lbm_lattice* v : b->views) {
      v->batch = nullptr;
      lbm_lattice_destroy(v);
    }
    delete b;
    return lbm_detail::fail(nullptr, code, msg);
  };
  if (hipGetDevice(&b->device) != hipSuccess) return undo(LBM_ERR_HIP, "hipGetDevice failed");
  if (hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device) !=
      hipSuccess)
    return undo(LBM_ERR_HIP, "hipDeviceGetAttribute failed");
  if (hipDeviceGetAttribute(&b->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                            b->device) != hipSuccess) {
    b->lds_per_cu = 0;        // no occupancy cap
    (void)hipGetLastError();  // and no stale error for the next launch check
  }
  std::vector<uint8_t> mat;
  for (int l = 0; l < count; ++l) {
    const int nx = dims[3 * l], ny = dims[3 * l + 1], nz = dims[3 * l + 2];
    lbm_lattice* v = nullptr;
    const int px = member_pitch(nx, storage_bytes(s));
    size_t pb = 0;
    lbm_required_bytes(d, px, ny, nz, s, &pb, nullptr);
    st = lbm_detail::create_lattice(&v, d, nx, ny, nz, tau[l], s, flags, b->pop + L.pop_off[l], pb,
                                    b->aux + L.aux_off[l], L.aux_size[l], hip_stream, 0,
                                    b->aux + L.scratch_off, L.scratch_bytes, px);
    if (st) return undo(st, "lattice " + std::to_string(l) + ": " + lbm_last_error(nullptr));
    b->views.push_back(v);
    mat.assign((size_t)nx * ny * nz, 1);  // fully fluid, periodic on every axis
    st = lbm_set_geometry(v, mat.data(), d == LBM_D2Q9 ? 3u : 7u);
    if (st) return undo(st, "lattice " + std::to_string(l) + ": " + lbm_last_error(v));
    v->batch = b;
    BatchLat bl;
    bl.pop_off = L.pop_off[l] / storage_bytes(s);
    bl.nx = nx;
    bl.ny = ny;
    bl.nz = nz;
    bl.px = px;
    bl.N = (uint32_t)((size_t)px * ny * nz);
    bl.pix = v->pix;
    bl.omega = v->omega;
    bl.c = row_lane_cells(px, storage_bytes(s));
    bl.tpr = px / bl.c;
    b->max_tpr = std::max(b->max_tpr, bl.tpr);
    b->lats.push_back(bl);
    b->total_cells += (long long)v->N;
  }
  int t0 = 128;
  while (t0 < b->max_tpr) t0 *= 2;
  t0 = std::max(256, t0);
  st = build_items(b, t0, t0);
  if (st) return undo(st, b->err);
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_lattice(lbm_batch* b, int index, lbm_lattice** view) {
  if (!b || !view) return LBM_ERR_ARG;
  if (index < 0 || index >= b->count) return bfail(b, LBM_ERR_ARG, "index out of range");
  *view = b->views[index];
  return LBM_OK;
}

namespace {

lbm_status check_shape(lbm_batch* b, int threads, int blocks_per_cu) {
  bool ok = false;
  for (int t : THREAD_CHOICES) ok |= t == threads;
  if (!ok) return bfail(b, LBM_ERR_ARG, "threads must be 128, 256 or 512");
  if (blocks_per_cu < 0 || blocks_per_cu > 64)
    return bfail(b, LBM_ERR_ARG, "blocks_per_cu in 0..64 (0 = one block per work item)");
  return LBM_OK;
}

// Both phases' shapes at once; the item tables are rebuilt when a thread
// count changes (or an earlier upload failed).  On error the batch keeps its
// previous shapes.
lbm_status apply_shapes(lbm_batch* b, const int (&threads)[2], const int (&bpc)[2]) {
  if (threads[0] != b->threads[0] || threads[1] != b->threads[1] || !b->tables_ok) {
    const lbm_status st = build_items(b, threads[0], threads[1]);
    if (st != LBM_OK) return st;
  }
  b->blocks_per_cu[0] = bpc[0];
  b->blocks_per_cu[1] = bpc[1];
  drop_batch_graph(b);
  return LBM_OK;
}

}  // namespace

lbm_status lbm_batch_set_launch(lbm_batch* b, int threads, int blocks_per_cu) {
  lbm_status st = benter(b);
  if (st) return st;
  if ((st = check_shape(b, threads, blocks_per_cu))) return st;
  return apply_shapes(b, {threads, threads}, {blocks_per_cu, blocks_per_cu});
}

lbm_status lbm_batch_set_phase_launch(lbm_batch* b, int phase, int threads, int blocks_per_cu) {
  lbm_status st = benter(b);
  if (st) return st;
  if (phase != 0 && phase != 1) return bfail(b, LBM_ERR_ARG, "phase must be 0 or 1");
  if ((st = check_shape(b, threads, blocks_per_cu))) return st;
  int t[2] = {b->threads[0], b->threads[1]}, c[2] = {b->blocks_per_cu[0], b->blocks_per_cu[1]};
  t[phase] = threads;
  c[phase] = blocks_per_cu;
  return apply_shapes(b, t, c);
}

lbm_status lbm_batch_get_phase_launch(const lbm_batch* b, int phase, int* threads,
                                      int* blocks_per_cu) {
  if (!b || (phase != 0 && phase != 1)) return LBM_ERR_ARG;
  if (threads) *threads = b->threads[phase];
  if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu[phase];
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int n) {
  lbm_status st = benter(b);
  if (st) return st;
  if (n < 0) return bfail(b, LBM_ERR_ARG, "n must be >= 0");
  if (!b->tables_ok)
    return bfail(b, LBM_ERR_STATE,
                 "a HIP failure interrupted the upload of the work-item tables: set the launch "
                 "shape again");
  int phase = 0;
  st = common_phase(b, &phase);
  if (st) return st;
  st = enqueue_batch_steps(b, n, phase);
  if (st == LBM_OK) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      st = bfail(b, LBM_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  }
  if (st != LBM_OK) {
    // some launches may already be queued: the members' phase and step counts
    // no longer describe the device state
    for (lbm_lattice* v : b->views) v->consistent = false;
    drop_batch_graph(b);
    return st;
  }
  advance_views(b, n);
  return LBM_OK;
}

lbm_status lbm_batch_set_graph_steps(lbm_batch* b, int steps) {
  lbm_status st = benter(b);
  if (st) return st;
  if (steps < 0 || (steps & 1)) return bfail(b, LBM_ERR_ARG, "graph length must be even and >= 0");
  if (steps > 0 && b->stream == nullptr)
    return bfail(b, LBM_ERR_ARG, "graph replay needs a created (non-null) stream");
  drop_batch_graph(b);
  b->graph_steps = steps;
  return LBM_OK;
}

namespace {

// Two untimed steps, then trial_steps timed ones (an even count: the
// propagation phase is unchanged) with an event after every launch; ms[ph]
// receives the mean time of phase ph's launches and *total the mean step.
lbm_status time_trial(lbm_batch* b, int phase, int trial_steps, std::vector<hipEvent_t>& ev,
                      double (&ms)[2], double* total) {
  launch_one(b, phase);
  launch_one(b, phase ^ 1);
  (void)hipEventRecord(ev[0], b->stream);
  for (int s = 0; s < trial_steps; ++s) {
    launch_one(b, phase ^ (s & 1));
    (void)hipEventRecord(ev[s + 1], b->stream);
  }
  if (hipEventSynchronize(ev[trial_steps]) != hipSuccess)
    return bfail(b, LBM_ERR_HIP, "autotune trial failed");
  ms[0] = ms[1] = 0.0;
  for (int s = 0; s < trial_steps; ++s) {
    float m = 0.f;
    (void)hipEventElapsedTime(&m, ev[s], ev[s + 1]);
    ms[phase ^ (s & 1)] += m;
  }
  ms[0] /= trial_steps / 2;
  ms[1] /= trial_steps / 2;
  *total = 0.5 * (ms[0] + ms[1]);
  advance_views(b, trial_steps + 2);
  return LBM_OK;
}

}  // namespace

lbm_status lbm_batch_autotune(lbm_batch* b, int trial_steps, int* threads, int* blocks_per_cu,
                              double* best_ms_per_step) {
  lbm_status st = benter(b);
  if (st) return st;
  if (trial_steps < 2 || trial_steps > 1000 || (trial_steps & 1))
    return bfail(b, LBM_ERR_ARG, "trial_steps must be even, 2..1000");
  int phase = 0;
  st = common_phase(b, &phase);
  if (st) return st;
  std::vector<hipEvent_t> ev(trial_steps + 1, nullptr);  // one per launch boundary
  lbm_status result = LBM_OK;
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      result = bfail(b, LBM_ERR_HIP, "hipEventCreate failed");
      break;
    }
  // every candidate shape for both phases; per phase, the fastest launches
  double best_step = 1e300, best_ph[2] = {1e300, 1e300};
  int step_t = b->threads[1], step_b = b->blocks_per_cu[1];
  int ph_t[2] = {b->threads[0], b->threads[1]};
  int ph_b[2] = {b->blocks_per_cu[0], b->blocks_per_cu[1]};
  for (int t : THREAD_CHOICES) {
    if (result != LBM_OK) break;
    if (t < b->max_tpr) continue;
    if ((result = build_items(b, t, t)) != LBM_OK) break;
    for (int bpc : BLOCKS_PER_CU_CHOICES) {
      b->blocks_per_cu[0] = b->blocks_per_cu[1] = bpc;
      double ms[2], total = 0.0;
      if ((result = time_trial(b, phase, trial_steps, ev, ms, &total)) != LBM_OK) break;
      if (total < best_step) {
        best_step = total;
        step_t = t;
        step_b = bpc;
      }
      for (int ph = 0; ph < 2; ++ph)
        if (ms[ph] < best_ph[ph]) {
          best_ph[ph] = ms[ph];
          ph_t[ph] = t;
          ph_b[ph] = bpc;
        }
    }
  }
  // The phases' fastest shapes combined are kept only if the combination,
  // timed as such, beats the best common shape: each phase runs on the cache
  // state the other leaves behind.
  int use_t[2] = {step_t, step_t}, use_b[2] = {step_b, step_b};
  double best = best_step;
  if (result == LBM_OK && (ph_t[0] != ph_t[1] || ph_b[0] != ph_b[1])) {
    b->blocks_per_cu[0] = ph_b[0];
    b->blocks_per_cu[1] = ph_b[1];
    result = build_items(b, ph_t[0], ph_t[1]);
    double ms[2], total = 0.0;
    if (result == LBM_OK) result = time_trial(b, phase, trial_steps, ev, ms, &total);
    if (result == LBM_OK && total < best_step) {
      best = total;
      use_t[0] = ph_t[0];
      use_t[1] = ph_t[1];
      use_b[0] = ph_b[0];
      use_b[1] = ph_b[1];
    }
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (result != LBM_OK) {
    // trial steps may have been queued without being counted: as after a
    // failed lbm_batch_step, the members' phases no longer describe the device
    for (lbm_lattice* v : b->views) v->consistent = false;
    return result;
  }
  b->blocks_per_cu[0] = use_b[0];
  b->blocks_per_cu[1] = use_b[1];
  st = build_items(b, use_t[0], use_t[1]);
  if (st) return st;
  if (threads) *threads = use_t[1];
  if (blocks_per_cu) *blocks_per_cu = use_b[1];
  if (best_ms_per_step) *best_ms_per_step = best;
  return LBM_OK;
}

lbm_status lbm_batch_get_info(const lbm_batch* b, int* count, long long* total_cells,
                              int* threads, int* blocks_per_cu) {
  if (!b) return LBM_ERR_ARG;
  if (count) *count = b->count;
  if (total_cells) *total_cells = b->total_cells;
  if (threads) *threads = b->threads[1];
  if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu[1];
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_ERR_ARG;
  hipError_t e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  drop_batch_graph(b);
  for (lbm_lattice* v : b->views) {
    v->batch = nullptr;
    lbm_lattice_destroy(v);
  }
  delete b;
  return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
