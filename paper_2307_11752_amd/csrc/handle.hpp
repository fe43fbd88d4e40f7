// handle.hpp -- host-side state of a lattice handle, shared by the C ABI
// implementation (lbm.hip) and the batched ensemble (batch.hip).  Internal:
// not part of the installed interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "lattice.hpp"
#include "lbm.h"

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
constexpr int RED_FIELDS = 8;  // mass, jx, jy, jz, sum|u|^2, max|u|, fluid count, spare

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Device scratch of a lattice: the per-block partial totals of lbm_totals, or
// one chunk of the moments staged for lbm_moments (4 doubles per cell).  A
// lattice's own scratch sits in its aux buffer; the members of a batch share
// one scratch area of the batch's aux buffer.
constexpr size_t SCRATCH_MIN = sizeof(double) * RED_BLOCKS * RED_FIELDS;  // 64 KiB
constexpr size_t SCRATCH_MAX = (size_t)1 << 20;                           // 1 MiB
constexpr size_t MOMENT_BYTES_PER_CELL = 4 * sizeof(double);
inline size_t scratch_size(size_t N) {
  const size_t b = MOMENT_BYTES_PER_CELL * N;
  return align256(b < SCRATCH_MIN ? SCRATCH_MIN : (b > SCRATCH_MAX ? SCRATCH_MAX : b));
}

struct AuxLayout {
  size_t link, mov, cls, result, scratch, total;
};

// Aux buffer of a lattice of N cells with `scratch` bytes of its own scratch
// (0 for a batch member, which uses the batch's).
inline AuxLayout aux_layout(size_t N, size_t scratch) {
  AuxLayout a;
  a.link = 0;
  a.mov = align256(a.link + 4 * N);
  a.cls = align256(a.mov + 4 * N);  // one byte per cell: CELL_FLUID | CELL_MOVING
  a.result = align256(a.cls + N);
  a.scratch = align256(a.result + sizeof(double) * RED_FIELDS);
  a.total = align256(a.scratch + scratch);
  return a;
}

inline int qof(int d) { return d == LBM_D2Q9 ? 9 : 19; }

// Distance in elements between consecutive population arrays: N rounded up to
// 64 elements, so that every array starts on a 256-byte boundary whatever N is.
inline size_t pop_stride(size_t N) { return (N + 63) & ~size_t(63); }

// Chunk size of the blocked placement, in bytes per population run.  Probes
// of the phase-0 access pattern on MI355X (TGV 256^3, FP32): arrays 421-432
// us, chunks of 2048 / 4096 / 8192 / 16384 / 32768 cells 395 / 392 / 387 /
// 404 / 410 us (a streaming copy of the same bytes: 384 us).
constexpr size_t POP_CHUNK_BYTES = 32768;

// The placement of a lattice's populations: blocked when the lattice spans
// more than one chunk and the whole buffer stays below 2^32 bytes (so every
// byte offset fits 32 bits), else one array per population.
inline lbm::PopIndex pop_index(int q, size_t N, size_t s) {
  const size_t B = POP_CHUNK_BYTES / s;
  uint32_t lb = 0;
  while (((size_t)1 << lb) < B) ++lb;
  const size_t chunks = (N + B - 1) / B;
  if (N > B && (size_t)q * chunks * B * s < ((size_t)1 << 32))
    return lbm::PopIndex{lb, (uint32_t)(B - 1), (uint32_t)(q * B), (uint32_t)B};
  return lbm::PopIndex{31u, 0x7fffffffu, 0u, (uint32_t)pop_stride(N)};
}

// Elements the placement spans.
inline size_t pop_elements(int q, const lbm::PopIndex& L, size_t N) {
  if (L.bstride) return (size_t)L.bstride * ((N + L.mask) >> L.lb);
  return (size_t)q * L.pstride;
}

inline size_t storage_bytes(int s) {
  switch (s) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    case LBM_STORE_F16: return 2;
    case LBM_STORE_BF16: return 2;
  }
  return 0;
}


// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct lbm_lattice {
  int desc = 0, q = 0, nx = 0, ny = 0, nz = 0;
  size_t N = 0;
  // Cells from one stored x-row to the next: nx, or nx + 1 for a batch member
  // whose odd rows are padded (the padding slots hold no cell).
  int px = 0;
  lbm::PopIndex pix{};  // placement of the populations (pop_index)
  int storage = 0;
  bool shifted = false;
  double tau = 0.0, omega = 0.0;
  double g[3] = {0, 0, 0}, uw[3] = {0, 0, 0};
  void* pop = nullptr;
  size_t pop_bytes = 0;
  unsigned char* aux = nullptr;
  size_t aux_bytes = 0;
  AuxLayout lay{};
  unsigned char* scratch = nullptr;  // device scratch (see scratch_size)
  size_t scratch_bytes = 0;
  // False after a HIP failure while steps were being enqueued: the device state
  // no longer matches phase / steps, so stepping and reading are refused until
  // the populations are initialised again.
  bool consistent = true;
  hipStream_t stream = nullptr;
  int device = 0;
  bool has_geometry = false, initialized = false, all_fluid = false, has_moving_cells = false;
  unsigned periodic = 0;
  int phase = 0;
  long long steps = 0;
  long long nfluid = 0;
  int bx = 256, nxb = 1;
  int lds_per_cu = 0;  // bytes of LDS per compute unit (occupancy caps)
  // Replay of a captured run of graph_steps steps (0 = direct launches).  The
  // graph bakes in the kernel arguments, so any parameter change drops it.
  int graph_steps = 0;
  hipGraphExec_t graph = nullptr;
  // Non-null for a lattice owned by a batch (lbm_batch_lattice): the batch
  // advances it, and calls that would change what the batch launch assumes
  // are refused.
  const void* batch = nullptr;
  std::string err;
};


namespace lbm_detail {
lbm_status fail(lbm_lattice* h, lbm_status st, const std::string& msg);
void drop_graph(lbm_lattice* h);
// lbm_lattice_create with an explicit scratch area: own_scratch bytes of the
// aux buffer (lbm_lattice_create uses scratch_size(N)), or, with
// own_scratch == 0, the caller's shared scratch of shared_bytes; px > nx
// stores the populations with that row pitch (0 = nx).
lbm_status create_lattice(lbm_lattice** out, lbm_descriptor d, int nx, int ny, int nz,
                          double tau, lbm_storage s, unsigned flags, void* dev_pop,
                          size_t pop_bytes, void* dev_aux, size_t aux_bytes, void* hip_stream,
                          size_t own_scratch, unsigned char* shared, size_t shared_bytes,
                          int px = 0);
}  // namespace lbm_detail

#define HIP_TRY(h, call)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return lbm_detail::fail((h), LBM_ERR_HIP,                                           \
                              std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)
