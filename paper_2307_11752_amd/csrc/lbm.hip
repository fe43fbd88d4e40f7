// lbm.hip -- gfx950 kernels and the C ABI (include/lbm.h) of the fused BGK
// collide-and-stream step with bounce-back walls, moving walls, periodic wrap
// and Guo forcing.
//
// Propagation: in-place AA pattern on one population
// buffer.  The stream equation of the guide (f_i(t+1, x+c_i) = f*_i(t, x),
// Introduction, "Lattice Boltzmann Methods") is realised without a second
// lattice by alternating two kernels:
//
//   phase 0 (natural layout, slot i of x holds f_i(x)):
//     read  f_i = A[i][x];   collide;   write A[opp(i)][x] = f*_i
//   phase 1 (swapped layout, slot opp(i) of x holds f*_i(x) of the last step):
//     read  f_j = A[opp(j)][x - c_j]        (or A[j][x] if x - c_j is a wall)
//     collide
//     write A[i][x + c_i] = f*_i            (or A[opp(i)][x] if x + c_i is a wall)
//
// Each slot is read and written by exactly one cell per launch, so neither
// kernel races and each population crosses HBM once per step in each
// direction.  Halfway bounce-back (the wall lies half way along the link)
// becomes a redirected slot inside the cell itself; a moving wall (material 3)
// subtracts 2 w_i rho (c_i.u_w)/c_s^2 from the reflected population, applied
// where the reflected value is written.  Periodic axes wrap the neighbour
// index; fluid cells never touch a non-periodic edge (geometry check).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"
#include "fluid_path.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

// A stored population held in a full register (16-bit values zero-extended),
// so that a conditional reload overwrites a whole register.
template <typename S>
struct RawReg {
  using type = uint32_t;
  static __device__ __forceinline__ type load(const S* p) {
    if constexpr (sizeof(S) == 2) return *(const uint16_t*)p;
    else return *(const uint32_t*)p;
  }
  static __device__ __forceinline__ type load_nt(const S* p) {
    if constexpr (sizeof(S) == 2) return __builtin_nontemporal_load((const uint16_t*)p);
    else return __builtin_nontemporal_load((const uint32_t*)p);
  }
  static __device__ __forceinline__ typename Store<S>::T cvt(type r) {
    S v;
    if constexpr (sizeof(S) == 2) {
      const uint16_t h = (uint16_t)r;
      __builtin_memcpy(&v, &h, 2);
    } else {
      __builtin_memcpy(&v, &r, 4);
    }
    return Store<S>::cvt(v);
  }
};
template <>
struct RawReg<double> {
  using type = double;
  static __device__ __forceinline__ double load(const double* p) { return *p; }
  static __device__ __forceinline__ double load_nt(const double* p) {
    return __builtin_nontemporal_load(p);
  }
  static __device__ __forceinline__ double cvt(double r) { return r; }
};

// ---------------------------------------------------------------------------
// The fused step kernel.  One thread per cell; a block covers a run of up to
// blockDim.x cells along x of one (y, z) row.
//   MASKED = false: every cell is fluid (fully periodic box); no link words.
// ---------------------------------------------------------------------------
template <int Q, typename S, bool SHIFT, int PHASE, bool MASKED>
__global__ void __launch_bounds__(256)
    step_kernel(S* __restrict__ pop, const uint32_t* __restrict__ link,
                const uint32_t* __restrict__ mov, int nx, int ny, int nz, PopIndex L, int nxb,
                StepParams<typename Store<S>::T> p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  // Masked phase 1 with two blocks per row (rows of 257..512 cells): runs of
  // XCD_ROWS consecutive rows, both halves of each, go to one XCD (the
  // hardware deals blocks to the 8 XCDs in turn, so blocks b, b + 8, b + 16,
  // ... share one), so that the lines the halves share at the middle of a row
  // are fetched into one L2 and each XCD works on one band of rows (channel
  // step FP32 0.2148 -> 0.2047 ms, FP16 0.1258 -> 0.1202 ms; runs of 1 / 4 /
  // 64 / 256 rows: 0.2123 / 0.2055 / 0.2129 / 0.2153 ms in FP32).  Blocks
  // past the last whole run keep the plain order.  With 16-bit storage the
  // rows run in descending order, so that phase 1 starts on the rows phase 0
  // wrote last: that state (about 1.4 times the last-level cache for the
  // 512 x 128 x 128 channel) then partly comes from that cache (FP16 step
  // 0.1292 -> 0.1271 ms; FP32 storage, and the fully fluid row kernels, lose
  // from this order).
  constexpr int XCD_ROWS = 16;
  constexpr bool REV = MASKED && PHASE == 1 && sizeof(S) == 2;
  const int nrows = ny * nz;
  const int b = (int)blockIdx.x;
  int r = b / nxb;
  int xb = b - r * nxb;
  if (MASKED && PHASE == 1 && nxb == 2) {
    constexpr int span = 16 * XCD_ROWS;  // blocks of one run on each of the 8 XCDs
    if (b < (int)gridDim.x / span * span) {
      const int k = (b >> 3) % (2 * XCD_ROWS);
      r = XCD_ROWS * (8 * (b / span) + (b & 7)) + (k >> 1);
      xb = k & 1;
    }
  }
  const int row = REV ? nrows - 1 - r : r;
  const int x = xb * (int)blockDim.x + (int)threadIdx.x;
  if (x >= nx) return;
  const int y = row % ny;
  const int z = row / ny;
  const uint32_t idx = (uint32_t)x + (uint32_t)nx * (uint32_t)(y + ny * z);

  const Nbr nb = make_nbr(x, y, z, nx, ny, nz);
  uint32_t lw = LINK_FLUID, mv = 0;
  T f[Q];
  if (MASKED && PHASE == 1) {
    // The neighbour loads do not wait for the link word (waiting would expose
    // one memory latency per wave); a wall cell's lanes read values nobody
    // uses, and the populations reflected by a wall are then re-read from the
    // cell's own slots.
    // The stored values are kept raw, one full register each, until every
    // load is in flight: a 16-bit value converted inside the wall branch
    // would make each branch wait for its own load.
    using U = typename RawReg<S>::type;
    U raw[Q];
    lw = link[idx];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const uint32_t off = L.at(V::opp[i], nb.at(-V::cx[i], -V::cy[i], -V::cz[i]));
      raw[i] = V::cx[i] == 0 ? RawReg<S>::load_nt(pop + off) : RawReg<S>::load(pop + off);
    }
    if (!(lw & LINK_FLUID)) return;
    if (p.has_moving && (lw & LINK_HAS_MOVING)) mv = mov[idx];
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if ((lw >> (V::opp[i] - 1)) & 1u) raw[i] = RawReg<S>::load(pop + L.at(i, idx));
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = RawReg<S>::cvt(raw[i]);
  } else {
    if (MASKED) {
      lw = link[idx];
      if (!(lw & LINK_FLUID)) return;
      if (p.has_moving && (lw & LINK_HAS_MOVING)) mv = mov[idx];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      uint32_t off;
      if (PHASE == 0)
        off = L.at(i, idx);
      else
        off = L.at(V::opp[i], nb.at(-V::cx[i], -V::cy[i], -V::cz[i]));
      // Streaming data is touched once per launch: x-aligned accesses bypass
      // the caches; x-shifted ones (phase 1, c_x != 0) share lines with the
      // neighbouring wave and stay cached.
      if (PHASE == 0 || V::cx[i] == 0)
        f[i] = load_nt<S>(pop + off);
      else
        f[i] = Store<S>::load(pop + off);
    }
  }

  const T rho = collide<Q, SHIFT, T>(f, p);

#pragma unroll
  for (int i = 0; i < Q; ++i) {
    T v = f[i];
    if (MASKED && i > 0 && ((mv >> (i - 1)) & 1u)) v -= rho * p.mw[i];
    uint32_t off;
    if (PHASE == 0) {
      off = L.at(V::opp[i], idx);
    } else {
      off = L.at(i, nb.at(V::cx[i], V::cy[i], V::cz[i]));
      if (MASKED && i > 0 && ((lw >> (i - 1)) & 1u)) off = L.at(V::opp[i], idx);
    }
    if (PHASE == 0 || V::cx[i] == 0)
      store_nt<S>(pop + off, v);
    else
      Store<S>::store(pop + off, v);
  }
}

// ---------------------------------------------------------------------------
// Fully-fluid fast path.  Every lane moves 8 bytes per population per
// direction (C = 8 / sizeof(S) consecutive cells), all HBM accesses aligned
// and non-temporal.
//
// Phase 0 needs no neighbour: flat cell indexing.
// Phase 1 works on whole x-rows: a row's populations arriving from x -/+ 1
// are loaded aligned into LDS and read back shifted (with the periodic wrap
// inside the row); outgoing x-shifted populations are written shifted into
// LDS and stored aligned.  This removes the misaligned accesses that
// otherwise cost about 12 % of bandwidth in this phase.
// ---------------------------------------------------------------------------
template <int Q, typename S, bool SHIFT, int C>
__global__ void __launch_bounds__(256)
    step_p0_flat_kernel(S* __restrict__ pop, uint32_t N, PopIndex L,
                        StepParams<typename Store<S>::T> p) {
  // FP32 takes the blocks in descending order (TGV 256^3: phase 0 384 -> 378
  // us, phase 1 after it unchanged; 16-bit storage loses from this order)
  const unsigned bid = sizeof(S) == 4 ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const uint32_t c0 = (uint32_t)C * (bid * blockDim.x + threadIdx.x);
  if (c0 >= N) return;
  fluid_cells_p0<Q, S, SHIFT, C>(pop, L, c0, p);
}

template <int Q, typename S, bool SHIFT>
__global__ void __launch_bounds__(256)
    step_p1_rows_kernel(S* __restrict__ pop, int nx, int ny, int nz, PopIndex L, int tpr,
                        int rows_per_block, StepParams<typename Store<S>::T> p) {
  constexpr int C = Pack8<S>::C;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int rloc = (int)threadIdx.x / tpr;
  const int t = (int)threadIdx.x - rloc * tpr;
  const int row = (int)blockIdx.x * rows_per_block + rloc;
  S* tile = (S*)smem_raw + (size_t)rloc * Shifted<Q>::count() * nx;
  fluid_rows_p1<Q, S, SHIFT, C>(pop, nx, nx, ny, nz, L, row, row < ny * nz, t, tile, p);
}

// Phase 1 with each x-row held by 2^lr_log2 = nx / C lanes of one wave (a
// power of two up to 64, so a wave covers 64 / 2^lr_log2 whole rows).  No LDS
// and no barrier: the x-shifted populations move between lanes in registers.
// ONE_ROW (nx = 64 C): the wave's row is uniform, so every row address is
// scalar and the lanes only carry their x offset.
template <int Q, typename S, bool SHIFT, int C, bool ONE_ROW>
__global__ void __launch_bounds__(256)
    step_p1_wave_kernel(S* __restrict__ pop, int nx, int ny, int nz, PopIndex L, int lr_log2,
                        StepParams<typename Store<S>::T> p) {
  const int lane = (int)(threadIdx.x & 63u);
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if constexpr (ONE_ROW) {
    const int row = __builtin_amdgcn_readfirstlane(wave);
    if (row >= ny * nz) return;
    fluid_rows_p1_wave<Q, S, SHIFT, C>(pop, nx, ny, nz, L, row, lane, (lane - 1) & 63,
                                       (lane + 1) & 63, p);
  } else {
    const int lr = 1 << lr_log2;
    const int t = lane & (lr - 1);
    const int first = lane - t;
    const int row = (wave << (6 - lr_log2)) + (lane >> lr_log2);
    if (row >= ny * nz) return;  // whole rows drop out together
    fluid_rows_p1_wave<Q, S, SHIFT, C>(pop, nx, ny, nz, L, row, t, first + ((t - 1) & (lr - 1)),
                                       first + ((t + 1) & (lr - 1)), p);
  }
}

// ---------------------------------------------------------------------------
// Masked phase 0 (lattices with walls), same lane shape as the fluid path.
// Every lane loads its C cells' slots aligned and non-temporal together with
// their class bytes (waiting for the classes first would expose one memory
// latency per wave; the local phase needs only the fluid and moving-link
// bits, so one byte per cell instead of the 4-byte link word), collides the
// fluid cells and writes every slot back: non-fluid cells keep their values,
// so each line is written whole and each slot still has a single writer.
// ---------------------------------------------------------------------------
template <int C>
struct ClassVec {
  // the C cells' class bytes (CELL_FLUID | CELL_MOVING), one load per lane
  static __device__ __forceinline__ void load(const uint8_t* p, uint32_t (&cl)[C]) {
    if constexpr (C == 1) {
      cl[0] = __builtin_nontemporal_load(p);
    } else if constexpr (C == 2) {
      const uint32_t v = __builtin_nontemporal_load((const uint16_t*)p);
      cl[0] = v & 0xffu;
      cl[1] = v >> 8;
    } else {
      const uint32_t v = __builtin_nontemporal_load((const uint32_t*)p);
      cl[0] = v & 0xffu;
      cl[1] = (v >> 8) & 0xffu;
      cl[2] = (v >> 16) & 0xffu;
      cl[3] = v >> 24;
    }
  }
};

template <int Q, typename S, bool SHIFT>
__global__ void __launch_bounds__(256)
    step_p0_masked_kernel(S* __restrict__ pop, const uint8_t* __restrict__ cls,
                          const uint32_t* __restrict__ mov, uint32_t N, PopIndex L,
                          StepParams<typename Store<S>::T> p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  constexpr int C = Pack8<S>::C;
  const uint32_t c0 = (uint32_t)C * (blockIdx.x * blockDim.x + threadIdx.x);
  if (c0 >= N) return;
  // cell classes and populations are requested together: waiting for the
  // classes before issuing the population loads would expose one memory
  // latency per wave
  uint32_t cl[C];
  ClassVec<C>::load(cls + c0, cl);
  const uint32_t lo = L.cell(c0) * (uint32_t)sizeof(S);
  S sv[Q][C];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    Pack8<S>::unpack(__builtin_nontemporal_load(at_byte<raw8>(pop + (size_t)i * L.pstride, lo)), sv[i]);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    if (!(cl[k] & CELL_FLUID)) continue;
    const uint32_t mv = (p.has_moving && (cl[k] & CELL_MOVING)) ? mov[c0 + k] : 0u;
    T f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::cvt(sv[i][k]);
    const T rho = collide<Q, SHIFT, T>(f, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T v = f[i];
      if (i > 0 && ((mv >> (i - 1)) & 1u)) v -= rho * p.mw[i];
      sv[V::opp[i]][k] = Store<S>::pack(v);
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(Pack8<S>::pack(sv[i]), at_byte<raw8>(pop + (size_t)i * L.pstride, lo));
}

// ---------------------------------------------------------------------------
// Decoding of the stored state (used off the per-step path).
// ---------------------------------------------------------------------------
// sidx: the cell's stored position (x + px (y + ny z)); nb: its neighbours' stored positions.
template <int Q, typename S>
__device__ __forceinline__ S load_phase(const S* pop, uint32_t lw, int i, uint32_t sidx,
                                        const Nbr& nb, int phase, const PopIndex& L) {
  using V = Vel<Q>;
  if (phase == 0 || i == 0) return pop[L.at(i, sidx)];
  const int o = V::opp[i];
  if ((lw >> (o - 1)) & 1u) return pop[L.at(i, sidx)];
  return pop[L.at(o, nb.at(-V::cx[i], -V::cy[i], -V::cz[i]))];
}

__device__ __forceinline__ void cell_coords(uint32_t idx, int nx, int ny, int& x, int& y, int& z) {
  x = (int)(idx % (uint32_t)nx);
  const uint32_t r = idx / (uint32_t)nx;
  y = (int)(r % (uint32_t)ny);
  z = (int)(r / (uint32_t)ny);
}

// Stored position of cell idx = x + nx (y + ny z) when x-rows are px cells apart.
__device__ __forceinline__ uint32_t stored_cell(uint32_t idx, int nx, int px) {
  if (px == nx) return idx;
  const uint32_t r = idx / (uint32_t)nx;
  return idx + r * (uint32_t)(px - nx);
}

// f (double, natural layout, unshifted) of every cell; zeros for non-fluid cells.
template <int Q, typename S, bool SHIFT>
__global__ void get_pop_kernel(const S* __restrict__ pop, const uint32_t* __restrict__ link,
                               double* __restrict__ out, int nx, int ny, int nz, int px,
                               uint32_t N, PopIndex L, int phase) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x) {
    const uint32_t lw = link[idx];
    int x, y, z;
    cell_coords(idx, nx, ny, x, y, z);
    const Nbr nb = make_nbr(x, y, z, nx, ny, nz, px);
    const uint32_t sidx = stored_cell(idx, nx, px);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = 0.0;
      if (lw & LINK_FLUID) {
        v = Store<S>::to_f64(load_phase<Q, S>(pop, lw, i, sidx, nb, phase, L));
        if (SHIFT) v += weight<Q, double>(i);
      }
      out[(size_t)i * N + idx] = v;
    }
  }
}

// Populations from double natural layout; phase becomes 0.
template <int Q, typename S, bool SHIFT>
__global__ void set_pop_kernel(S* __restrict__ pop, const double* __restrict__ in, int nx, int px,
                               uint32_t N, PopIndex L) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x) {
    const uint32_t sidx = stored_cell(idx, nx, px);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = in[(size_t)i * N + idx];
      if (SHIFT) v -= weight<Q, double>(i);
      pop[L.at(i, sidx)] = Store<S>::from_f64(v);
    }
  }
}

// Second-order equilibrium of (rho, u), evaluated in double, on fluid cells.
template <int Q, typename S, bool SHIFT>
__global__ void init_eq_kernel(S* __restrict__ pop, const uint32_t* __restrict__ link,
                               const double* __restrict__ rho_in, const double* __restrict__ u_in,
                               int nx, int px, uint32_t N, PopIndex L) {
  using V = Vel<Q>;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x) {
    const bool fluid = (link[idx] & LINK_FLUID) != 0;
    const uint32_t sidx = stored_cell(idx, nx, px);
    const double rho = rho_in ? rho_in[idx] : 1.0;
    double u[3] = {0.0, 0.0, 0.0};
    if (u_in)
      for (int a = 0; a < V::D; ++a) u[a] = u_in[(size_t)a * N + idx];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double w = weight<Q, double>(i);
      const double cu = V::cx[i] * u[0] + V::cy[i] * u[1] + V::cz[i] * u[2];
      double feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      if (SHIFT) feq -= w;
      pop[L.at(i, sidx)] = Store<S>::from_f64(fluid ? feq : 0.0);
    }
  }
}

// rho and shifted u of cells begin .. begin+count-1 (double accumulation),
// zeros off the fluid, written as OutT: rho_out[idx - begin] and
// u_out[a * ustride + idx - begin] for component a.
template <int Q, typename S, bool SHIFT, typename OutT>
__global__ void moments_kernel(const S* __restrict__ pop, const uint32_t* __restrict__ link,
                               OutT* __restrict__ rho_out, OutT* __restrict__ u_out, int nx,
                               int ny, int nz, int px, PopIndex L, int phase, double gx,
                               double gy, double gz, uint32_t begin, uint32_t count,
                               uint32_t ustride) {
  using V = Vel<Q>;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += gridDim.x * blockDim.x) {
    const uint32_t idx = begin + k;
    const uint32_t lw = link[idx];
    double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
    if (lw & LINK_FLUID) {
      int x, y, z;
      cell_coords(idx, nx, ny, x, y, z);
      const Nbr nb = make_nbr(x, y, z, nx, ny, nz, px);
      const uint32_t sidx = stored_cell(idx, nx, px);
      double sf = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double v = Store<S>::to_f64(load_phase<Q, S>(pop, lw, i, sidx, nb, phase, L));
        sf += v;
        j[0] += V::cx[i] * v;
        j[1] += V::cy[i] * v;
        j[2] += V::cz[i] * v;
      }
      rho = SHIFT ? 1.0 + sf : sf;
      u[0] = j[0] / rho + 0.5 * gx;
      u[1] = j[1] / rho + 0.5 * gy;
      u[2] = V::D == 3 ? j[2] / rho + 0.5 * gz : 0.0;
    }
    if (rho_out) rho_out[k] = (OutT)rho;
    if (u_out) {
      u_out[k] = (OutT)u[0];
      u_out[(size_t)ustride + k] = (OutT)u[1];
      u_out[2 * (size_t)ustride + k] = (OutT)u[2];
    }
  }
}

// Per-block partial totals in double: mass, momentum (unshifted sum c f),
// sum |u|^2 and max |u| (shifted u), fluid count.
template <int Q, typename S, bool SHIFT>
__global__ void __launch_bounds__(RED_THREADS)
    totals_partial_kernel(const S* __restrict__ pop, const uint32_t* __restrict__ link,
                          double* __restrict__ partials, int nx, int ny, int nz, int px,
                          uint32_t N, PopIndex L, int phase, double gx, double gy, double gz) {
  using V = Vel<Q>;
  double acc[RED_FIELDS] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x) {
    const uint32_t lw = link[idx];
    if (!(lw & LINK_FLUID)) continue;
    int x, y, z;
    cell_coords(idx, nx, ny, x, y, z);
    const Nbr nb = make_nbr(x, y, z, nx, ny, nz, px);
    const uint32_t sidx = stored_cell(idx, nx, px);
    double sf = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double v = Store<S>::to_f64(load_phase<Q, S>(pop, lw, i, sidx, nb, phase, L));
      sf += v;
      j[0] += V::cx[i] * v;
      j[1] += V::cy[i] * v;
      j[2] += V::cz[i] * v;
    }
    const double rho = SHIFT ? 1.0 + sf : sf;
    const double ux = j[0] / rho + 0.5 * gx, uy = j[1] / rho + 0.5 * gy;
    const double uz = V::D == 3 ? j[2] / rho + 0.5 * gz : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    acc[0] += rho;
    acc[1] += j[0];
    acc[2] += j[1];
    acc[3] += j[2];
    acc[4] += uu;
    acc[5] = fmax(acc[5], sqrt(uu));
    acc[6] += 1.0;
  }
  __shared__ double red[RED_FIELDS][RED_THREADS];
#pragma unroll
  for (int k = 0; k < RED_FIELDS; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < RED_FIELDS; ++k) {
        if (k == 5)
          red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        else
          red[k][threadIdx.x] += red[k][threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < RED_FIELDS) partials[blockIdx.x * RED_FIELDS + threadIdx.x] = red[threadIdx.x][0];
}

// Sum the per-block partials in a fixed order (deterministic).
__global__ void __launch_bounds__(RED_THREADS)
    totals_final_kernel(const double* __restrict__ partials, double* __restrict__ result,
                        int nblocks) {
  __shared__ double red[RED_FIELDS][RED_THREADS];
  double acc[RED_FIELDS] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
#pragma unroll
    for (int k = 0; k < RED_FIELDS; ++k) {
      const double v = partials[b * RED_FIELDS + k];
      acc[k] = (k == 5) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
#pragma unroll
  for (int k = 0; k < RED_FIELDS; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < RED_FIELDS; ++k) {
        if (k == 5)
          red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        else
          red[k][threadIdx.x] += red[k][threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < RED_FIELDS) result[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

namespace lbm_detail {

thread_local std::string g_create_error;

lbm_status fail(lbm_lattice* h, lbm_status st, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return st;
}

void drop_graph(lbm_lattice* h) {
  if (h->graph) {
    // a replay may still be running on the lattice's stream
    (void)hipStreamSynchronize(h->stream);
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
}

}  // namespace lbm_detail

using lbm_detail::drop_graph;
using lbm_detail::fail;
using lbm_detail::g_create_error;

namespace {

bool tau_ok(double tau) { return (std::isinf(tau) && tau > 0) || (std::isfinite(tau) && tau > 0.5); }

template <int Q>
lbm_status build_links(int nx, int ny, int nz, const uint8_t* mat, unsigned periodic,
                       std::vector<uint32_t>* link, std::vector<uint32_t>* mov, long long* nfluid,
                       bool* has_moving, std::string* why) {
  using V = Vel<Q>;
  const size_t N = (size_t)nx * ny * nz;
  for (size_t i = 0; i < N; ++i)
    if (mat[i] > 3) {
      *why = "material " + std::to_string(mat[i]) + " at cell " + std::to_string(i) +
             " is not supported (only 0..3)";
      return LBM_ERR_UNSUPPORTED;
    }
  if (link) {
    link->assign(N, 0u);
    mov->assign(N, 0u);
  }
  long long nf = 0;
  bool hm = false;
  const int dims[3] = {nx, ny, nz};
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t idx = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
        if (mat[idx] != 1) continue;
        ++nf;
        uint32_t w = LINK_FLUID, m = 0;
        for (int i = 1; i < Q; ++i) {
          int c[3] = {x + V::cx[i], y + V::cy[i], z + V::cz[i]};
          for (int a = 0; a < 3; ++a) {
            if (c[a] >= 0 && c[a] < dims[a]) continue;
            if (!((periodic >> a) & 1u)) {
              *why = "fluid cell (" + std::to_string(x) + "," + std::to_string(y) + "," +
                     std::to_string(z) + ") streams out of the box along non-periodic axis " +
                     std::to_string(a);
              return LBM_ERR_GEOMETRY;
            }
            c[a] = (c[a] + dims[a]) % dims[a];
          }
          const uint8_t mn = mat[(size_t)c[0] + (size_t)nx * ((size_t)c[1] + (size_t)ny * c[2])];
          if (mn == 0) {
            *why = "fluid cell (" + std::to_string(x) + "," + std::to_string(y) + "," +
                   std::to_string(z) + ") borders a material-0 cell";
            return LBM_ERR_GEOMETRY;
          }
          if (mn == 2) w |= 1u << (i - 1);
          if (mn == 3) {
            w |= (1u << (i - 1)) | LINK_HAS_MOVING;
            m |= 1u << (i - 1);
            hm = true;
          }
        }
        if (link) {
          (*link)[idx] = w;
          (*mov)[idx] = m;
        }
      }
  *nfluid = nf;
  *has_moving = hm;
  return LBM_OK;
}

lbm_status check_dims(lbm_descriptor d, int nx, int ny, int nz, std::string* why) {
  if (d != LBM_D2Q9 && d != LBM_D3Q19) {
    *why = "unknown descriptor";
    return LBM_ERR_ARG;
  }
  if (nx <= 0 || ny <= 0 || nz <= 0) {
    *why = "lattice sizes must be positive";
    return LBM_ERR_ARG;
  }
  if (d == LBM_D2Q9 && nz != 1) {
    *why = "D2Q9 needs nz == 1";
    return LBM_ERR_ARG;
  }
  const double cells = (double)pop_stride((size_t)nx * ny * nz);
  if (cells * qof(d) >= 4294967296.0) {
    *why = "q*N must stay below 2^32 (32-bit population offsets)";
    return LBM_ERR_UNSUPPORTED;
  }
  return LBM_OK;
}

template <typename T>
StepParams<T> make_params(const lbm_lattice* h) {
  StepParams<T> p{};
  p.omega = (T)h->omega;
  p.kguo = (T)(1.0 - 0.5 * h->omega);
  for (int a = 0; a < 3; ++a) p.g[a] = (T)h->g[a];
  p.has_force = (h->g[0] != 0.0 || h->g[1] != 0.0 || h->g[2] != 0.0) ? 1 : 0;
  const int q = h->q;
  double uwdot = 0.0;
  for (int i = 0; i < 19; ++i) p.mw[i] = T(0);
  for (int i = 0; i < q; ++i) {
    double w, cu;
    if (q == 9) {
      w = Vel<9>::w36[i] / 36.0;
      cu = Vel<9>::cx[i] * h->uw[0] + Vel<9>::cy[i] * h->uw[1];
    } else {
      w = Vel<19>::w36[i] / 36.0;
      cu = Vel<19>::cx[i] * h->uw[0] + Vel<19>::cy[i] * h->uw[1] + Vel<19>::cz[i] * h->uw[2];
    }
    p.mw[i] = (T)(6.0 * w * cu);  // 2 w_i (c_i.u_w) / c_s^2
    uwdot += fabs(cu);
  }
  p.has_moving = (h->has_moving_cells && uwdot != 0.0) ? 1 : 0;
  return p;
}

// Dynamic LDS that caps a launch at `blocks_per_cu` resident blocks per
// compute unit (and at least `need` bytes, the kernel's own tile).  The
// streaming kernels run faster with fewer resident waves than their register
// use allows: each wave keeps 2 q row segments of different arrays in flight,
// and more of them only spread HBM accesses over more DRAM pages.  The counts
// used below were measured on MI355X (160 KiB of LDS per CU).
inline size_t occupancy_lds(const lbm_lattice* h, int blocks_per_cu, size_t need) {
  if (blocks_per_cu <= 0 || h->lds_per_cu <= 0) return need;
  const size_t cap = (size_t)(h->lds_per_cu / blocks_per_cu) & ~(size_t)1023;
  return (cap > need && cap <= 65536) ? cap : need;
}

// log2(nx / c) when an x-row splits into a power of two of at most 64 lanes of
// c cells each (one wave then holds whole rows), else -1.
inline int wave_row_log2(int nx, int c) {
  if (c < 1 || nx % c != 0) return -1;
  const int lr = nx / c;
  if (lr > 64 || (lr & (lr - 1)) != 0) return -1;
  int l = 0;
  while ((1 << l) < lr) ++l;
  return l;
}

// ---------------------------------------------------------------------------
// Typed dispatch
// ---------------------------------------------------------------------------
template <int Q, typename S, bool SHIFT>
struct Ops {
  using T = typename Store<S>::T;

  static void launch_p1_wave(lbm_lattice* h, S* pop, PopIndex L, int lrw, const StepParams<T>& p) {
    if constexpr (sizeof(S) == 2) {
      constexpr int C = Pack8<S>::C;
      const unsigned threads = 128;
      const size_t lds = occupancy_lds(h, 4, 0);
      const size_t rows = (size_t)h->ny * h->nz;
      const size_t waves = (rows + (64 >> lrw) - 1) / (64 >> lrw);
      const unsigned nb = (unsigned)((waves * 64 + threads - 1) / threads);
      if (lrw == 6)
        hipLaunchKernelGGL((step_p1_wave_kernel<Q, S, SHIFT, C, true>), dim3(nb), dim3(threads), lds,
                           h->stream, pop, h->nx, h->ny, h->nz, L, lrw, p);
      else
        hipLaunchKernelGGL((step_p1_wave_kernel<Q, S, SHIFT, C, false>), dim3(nb), dim3(threads),
                           lds, h->stream, pop, h->nx, h->ny, h->nz, L, lrw, p);
    }
  }

  static void step(lbm_lattice* h, int phase) {
    StepParams<T> p = make_params<T>(h);
    p.base = (T)Store<S>::unit;
    S* pop = (S*)h->pop;
    const uint32_t* link = (const uint32_t*)(h->aux + h->lay.link);
    const uint32_t* mov = (const uint32_t*)(h->aux + h->lay.mov);
    const dim3 grid((unsigned)(h->nxb * h->ny * h->nz)), block((unsigned)h->bx);
    const uint32_t N = (uint32_t)h->N;
    const PopIndex L = h->pix;
    constexpr int C = Pack8<S>::C;  // cells per 8-byte lane
    const int tpr = h->nx / C;
    // 16-bit storage: rows of nx = 4 * 2^k <= 256 cells fit one wave (and
    // never straddle two chunks of the blocked placement)
    const bool rows_whole = L.bstride == 0 || (L.mask + 1u) % (uint32_t)h->nx == 0;
    const int lrw = sizeof(S) == 2 && rows_whole ? wave_row_log2(h->nx, C) : -1;
    if (h->all_fluid && phase == 0) {
      // fully fluid fast path (measured launch shapes): phase 0 over flat
      // cell ranges whatever nx is (the last lane may run into the padding of
      // the population runs); 128 threads and four blocks per CU with 8-byte
      // lanes, except 16-bit storage, which runs 2 cells (4 bytes) a lane in
      // 256-thread blocks, six per CU (TGV 256^3 FP16: 188 against 197 us)
      constexpr int C0 = sizeof(S) == 2 ? 2 : C;
      const unsigned threads = sizeof(S) == 2 ? 256 : 128;
      const unsigned nb = (unsigned)(((h->N + C0 - 1) / C0 + threads - 1) / threads);
      hipLaunchKernelGGL((step_p0_flat_kernel<Q, S, SHIFT, C0>), dim3(nb), dim3(threads),
                         occupancy_lds(h, sizeof(S) == 2 ? 6 : 4, 0), h->stream, pop, N, L, p);
    } else if (h->all_fluid && (lrw >= 0 || (h->nx % C == 0 && tpr <= 256))) {
      // phase 1 on whole rows, one wave per row for 16-bit storage (128
      // threads, four blocks per CU), else through the LDS row tile (blocks of
      // whole rows, about 128 threads and four blocks per CU; rows wider than
      // 128 lanes one per block, three blocks per CU)
      if (lrw >= 0) {
        launch_p1_wave(h, pop, L, lrw, p);
      } else {
        const int rpb = tpr >= 128 ? 1 : 128 / tpr;
        const int rows = h->ny * h->nz;
        const unsigned nb = (unsigned)((rows + rpb - 1) / rpb);
        const size_t lds = (size_t)rpb * Shifted<Q>::count() * h->nx * sizeof(S);
        hipLaunchKernelGGL((step_p1_rows_kernel<Q, S, SHIFT>), dim3(nb), dim3(rpb * tpr),
                           occupancy_lds(h, rpb * tpr <= 128 ? 4 : 3, lds), h->stream, pop, h->nx,
                           h->ny, h->nz, L, tpr, rpb, p);
      }
    } else if (!h->all_fluid && h->N % C == 0 && h->N >= 65536 && phase == 0) {
      // (small lattices are latency-bound: the per-cell kernel below, with
      // more and smaller blocks, is faster there).  Six blocks per CU for
      // 4- and 8-byte storage (measured); 16-bit storage gains nothing from a cap.
      const unsigned threads = 128;
      const unsigned nb = (unsigned)((h->N / C + threads - 1) / threads);
      hipLaunchKernelGGL((step_p0_masked_kernel<Q, S, SHIFT>), dim3(nb), dim3(threads),
                         occupancy_lds(h, sizeof(S) >= 4 ? 6 : 0, 0), h->stream, pop,
                         (const uint8_t*)(h->aux + h->lay.cls), mov, N, L, p);
    } else if (h->all_fluid) {  // phase 1, rows the row kernels do not take
      hipLaunchKernelGGL((step_kernel<Q, S, SHIFT, 1, false>), grid, block, 0, h->stream, pop,
                         link, mov, h->nx, h->ny, h->nz, L, h->nxb, p);
    } else {
      if (phase == 0)
        hipLaunchKernelGGL((step_kernel<Q, S, SHIFT, 0, true>), grid, block, 0, h->stream, pop,
                           link, mov, h->nx, h->ny, h->nz, L, h->nxb, p);
      else
        hipLaunchKernelGGL((step_kernel<Q, S, SHIFT, 1, true>), grid, block, 0, h->stream, pop,
                           link, mov, h->nx, h->ny, h->nz, L, h->nxb, p);
    }
  }

  static unsigned blocks(size_t N) {
    size_t b = (N + 255) / 256;
    return (unsigned)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
  }

  static void get_pop(lbm_lattice* h, double* out) {
    hipLaunchKernelGGL((get_pop_kernel<Q, S, SHIFT>), dim3(blocks(h->N)), dim3(256), 0, h->stream,
                       (const S*)h->pop, (const uint32_t*)(h->aux + h->lay.link), out, h->nx,
                       h->ny, h->nz, h->px, (uint32_t)h->N, h->pix, h->phase);
  }
  static void set_pop(lbm_lattice* h, const double* in) {
    hipLaunchKernelGGL((set_pop_kernel<Q, S, SHIFT>), dim3(blocks(h->N)), dim3(256), 0, h->stream,
                       (S*)h->pop, in, h->nx, h->px, (uint32_t)h->N, h->pix);
  }
  static void init_eq(lbm_lattice* h, const double* rho, const double* u) {
    hipLaunchKernelGGL((init_eq_kernel<Q, S, SHIFT>), dim3(blocks(h->N)), dim3(256), 0, h->stream,
                       (S*)h->pop, (const uint32_t*)(h->aux + h->lay.link), rho, u, h->nx,
                       h->px, (uint32_t)h->N, h->pix);
  }
  template <typename OutT>
  static void moments(lbm_lattice* h, OutT* rho, OutT* u, uint32_t begin, uint32_t count,
                      uint32_t ustride) {
    hipLaunchKernelGGL((moments_kernel<Q, S, SHIFT, OutT>), dim3(blocks(count)), dim3(256), 0,
                       h->stream, (const S*)h->pop, (const uint32_t*)(h->aux + h->lay.link), rho,
                       u, h->nx, h->ny, h->nz, h->px, h->pix, h->phase, h->g[0], h->g[1],
                       h->g[2], begin, count, ustride);
  }
  static void moments_f64(lbm_lattice* h, double* rho, double* u, uint32_t begin, uint32_t count,
                          uint32_t ustride) {
    moments<double>(h, rho, u, begin, count, ustride);
  }
  static void moments_f32(lbm_lattice* h, float* rho, float* u, uint32_t begin, uint32_t count,
                          uint32_t ustride) {
    moments<float>(h, rho, u, begin, count, ustride);
  }
  static void totals(lbm_lattice* h, double* partials, double* result) {
    hipLaunchKernelGGL((totals_partial_kernel<Q, S, SHIFT>), dim3(RED_BLOCKS), dim3(RED_THREADS),
                       0, h->stream, (const S*)h->pop, (const uint32_t*)(h->aux + h->lay.link),
                       partials, h->nx, h->ny, h->nz, h->px, (uint32_t)h->N, h->pix, h->phase,
                       h->g[0], h->g[1], h->g[2]);
    hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(RED_THREADS), 0, h->stream, partials,
                       result, RED_BLOCKS);
  }
};

struct OpTable {
  void (*step)(lbm_lattice*, int);
  void (*get_pop)(lbm_lattice*, double*);
  void (*set_pop)(lbm_lattice*, const double*);
  void (*init_eq)(lbm_lattice*, const double*, const double*);
  void (*moments_f64)(lbm_lattice*, double*, double*, uint32_t, uint32_t, uint32_t);
  void (*moments_f32)(lbm_lattice*, float*, float*, uint32_t, uint32_t, uint32_t);
  void (*totals)(lbm_lattice*, double*, double*);
};

template <int Q, typename S, bool SHIFT>
OpTable table() {
  using O = Ops<Q, S, SHIFT>;
  return OpTable{O::step, O::get_pop, O::set_pop, O::init_eq, O::moments_f64, O::moments_f32,
                 O::totals};
}

template <int Q, bool SHIFT>
OpTable table_for_storage(int s) {
  switch (s) {
    case LBM_STORE_F64: return table<Q, double, SHIFT>();
    case LBM_STORE_F32: return table<Q, float, SHIFT>();
    case LBM_STORE_F16: return table<Q, _Float16, SHIFT>();
    default: return table<Q, bf16s, SHIFT>();
  }
}

OpTable ops(const lbm_lattice* h) {
  if (h->q == 9)
    return h->shifted ? table_for_storage<9, true>(h->storage)
                      : table_for_storage<9, false>(h->storage);
  return h->shifted ? table_for_storage<19, true>(h->storage)
                    : table_for_storage<19, false>(h->storage);
}

lbm_status launch_check(lbm_lattice* h) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, LBM_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return LBM_OK;
}

lbm_status enter(lbm_lattice* h) {
  if (!h) return LBM_ERR_ARG;
  h->err.clear();
  HIP_TRY(h, hipSetDevice(h->device));
  return LBM_OK;
}

// The populations can be stepped or decoded: initialised, and not left
// behind by a failed step (see lbm_lattice::consistent).
lbm_status readable(lbm_lattice* h) {
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "lattice not initialised");
  if (!h->consistent)
    return fail(h, LBM_ERR_STATE,
                "a HIP failure interrupted an earlier step: initialise the populations again");
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// Library-owned scratch for lbm_totals_noalloc: the per-block partial totals
// and the final sums live in this file-scope device array instead of the
// lattice's aux scratch.  Each GPU holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is not a device address in host
// code).  Every call on one GPU shares that GPU's copy.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_PARTIALS = (size_t)RED_BLOCKS * RED_FIELDS;
constexpr size_t STATIC_DOUBLES = STATIC_PARTIALS + RED_FIELDS;  // 64 KiB + 64 B
static __device__ __align__(256) double scratch[STATIC_DOUBLES];
// The reduction always runs RED_BLOCKS blocks, whatever the lattice size, so
// this fixed array holds the partials of any lattice.
static_assert(STATIC_PARTIALS == (size_t)RED_BLOCKS * RED_FIELDS, "partials per reduction");

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on h's device (h's device must be current).
lbm_status static_scratch(lbm_lattice* h, double** out) {
  if (h->device < 0 || h->device >= MAX_DEVICES)
    return fail(h, LBM_ERR_UNSUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[h->device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(h, LBM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    g_scratch_ptr[h->device] = (double*)ptr;
  }
  *out = g_scratch_ptr[h->device];
  return LBM_OK;
}

// Reduce the totals of h through `partials` (RED_BLOCKS * RED_FIELDS doubles)
// into `result` (RED_FIELDS doubles), copy them to the host and finish the
// statistics.  sync.
lbm_status reduce_totals(lbm_lattice* h, double* partials, double* result, double* mass,
                         double momentum[3], double stats[3]) {
  ops(h).totals(h, partials, result);
  lbm_status st = launch_check(h);
  if (st) return st;
  double r[RED_FIELDS];
  HIP_TRY(h, hipMemcpyAsync(r, result, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (mass) *mass = r[0];
  if (momentum)
    for (int a = 0; a < 3; ++a) momentum[a] = r[1 + a];
  const double nf = r[6];
  if (stats) {
    stats[0] = nf > 0 ? r[0] / nf : 0.0;
    stats[1] = nf > 0 ? 0.5 * r[4] / nf : 0.0;
    stats[2] = r[5];
  }
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(r[k])) return fail(h, LBM_ERR_NONFINITE, "non-finite value in the totals");
  return LBM_OK;
}

// Enqueue n steps on the lattice's stream (graph replays where set up),
// updating the phase launch by launch.  Returns LBM_ERR_HIP on a HIP failure.
lbm_status enqueue_steps(lbm_lattice* h, int n) {
  const OpTable t = ops(h);
  int left = n;
  if (h->graph_steps > 0 && n >= h->graph_steps) {
    // The captured run starts in phase 0 and has an even length, so it can be
    // replayed whenever the lattice is in phase 0.
    if (h->phase != 0) {
      t.step(h, 1);
      h->phase = 0;
      --left;
    }
    if (!h->graph && left >= h->graph_steps) {
      hipGraph_t g = nullptr;
      HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      for (int s = 0; s < h->graph_steps; ++s) t.step(h, s & 1);
      hipError_t e = hipStreamEndCapture(h->stream, &g);
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(h, LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      }
      e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        h->graph = nullptr;
        return fail(h, LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
    }
    while (h->graph && left >= h->graph_steps) {
      HIP_TRY(h, hipGraphLaunch(h->graph, h->stream));
      left -= h->graph_steps;
    }
  }
  for (int s = 0; s < left; ++s) {
    t.step(h, h->phase);
    h->phase ^= 1;
  }
  return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

lbm_status lbm_required_bytes(lbm_descriptor d, int nx, int ny, int nz, lbm_storage s,
                              size_t* pop_bytes, size_t* aux_bytes) {
  std::string why;
  lbm_status st = check_dims(d, nx, ny, nz, &why);
  if (st) return fail(nullptr, st, why);
  if (storage_bytes(s) == 0) return fail(nullptr, LBM_ERR_ARG, "unknown storage type");
  const size_t N = (size_t)nx * ny * nz;
  if (pop_bytes) {
    const PopIndex L = pop_index(qof(d), N, storage_bytes(s));
    *pop_bytes = align256(pop_elements(qof(d), L, N) * storage_bytes(s));
  }
  if (aux_bytes) *aux_bytes = aux_layout(N, scratch_size(N)).total;
  return LBM_OK;
}

lbm_status lbm_validate_geometry(lbm_descriptor d, int nx, int ny, int nz,
                                 const uint8_t* material, unsigned periodic_mask) {
  std::string why;
  lbm_status st = check_dims(d, nx, ny, nz, &why);
  if (st) return fail(nullptr, st, why);
  if (!material) return fail(nullptr, LBM_ERR_ARG, "material is NULL");
  long long nf;
  bool hm;
  st = d == LBM_D2Q9
           ? build_links<9>(nx, ny, nz, material, periodic_mask, nullptr, nullptr, &nf, &hm, &why)
           : build_links<19>(nx, ny, nz, material, periodic_mask, nullptr, nullptr, &nf, &hm, &why);
  if (st) return fail(nullptr, st, why);
  return LBM_OK;
}

lbm_status lbm_lattice_create(lbm_lattice** out, lbm_descriptor d, int nx, int ny, int nz,
                              double tau, lbm_storage s, unsigned flags, void* dev_pop,
                              size_t pop_bytes, void* dev_aux, size_t aux_bytes,
                              void* hip_stream) {
  const size_t N = (nx > 0 && ny > 0 && nz > 0) ? (size_t)nx * ny * nz : 0;
  return lbm_detail::create_lattice(out, d, nx, ny, nz, tau, s, flags, dev_pop, pop_bytes, dev_aux,
                                    aux_bytes, hip_stream, scratch_size(N), nullptr, 0);
}

}  // extern "C"

lbm_status lbm_detail::create_lattice(lbm_lattice** out, lbm_descriptor d, int nx, int ny, int nz,
                                      double tau, lbm_storage s, unsigned flags, void* dev_pop,
                                      size_t pop_bytes, void* dev_aux, size_t aux_bytes,
                                      void* hip_stream, size_t own_scratch, unsigned char* shared,
                                      size_t shared_bytes, int px) {
  if (!out) return fail(nullptr, LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  const int pitch = px > 0 ? px : nx;
  if (pitch < nx) return fail(nullptr, LBM_ERR_ARG, "row pitch below nx");
  size_t need_pop = 0;
  // the populations are stored as a lattice of pitch x ny x nz cells
  lbm_status st = lbm_required_bytes(d, pitch, ny, nz, s, &need_pop, nullptr);
  if (st) return st;
  const size_t need_aux = aux_layout((size_t)nx * ny * nz, own_scratch).total;
  if (own_scratch == 0 && (!shared || shared_bytes < SCRATCH_MIN))
    return fail(nullptr, LBM_ERR_ARG, "a lattice without its own scratch needs a shared one");
  if (!tau_ok(tau)) return fail(nullptr, LBM_ERR_ARG, "tau must be > 0.5 (or +inf for pure streaming)");
  if (flags & ~LBM_FLAG_SHIFTED) return fail(nullptr, LBM_ERR_ARG, "unknown flags");
  if (!dev_pop || !dev_aux) return fail(nullptr, LBM_ERR_ARG, "device buffers must not be NULL");
  if (pop_bytes < need_pop || aux_bytes < need_aux)
    return fail(nullptr, LBM_ERR_ARG,
                "buffers too small: need pop " + std::to_string(need_pop) + " aux " +
                    std::to_string(need_aux));
  if (((uintptr_t)dev_pop & 255u) || ((uintptr_t)dev_aux & 255u))
    return fail(nullptr, LBM_ERR_ARG, "device buffers must be 256-byte aligned");
  lbm_lattice* h = new (std::nothrow) lbm_lattice();
  if (!h) return fail(nullptr, LBM_ERR_ARG, "out of host memory");
  h->desc = d;
  h->q = qof(d);
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->N = (size_t)nx * ny * nz;
  h->px = pitch;
  h->pix = pop_index(h->q, (size_t)pitch * ny * nz, storage_bytes(s));
  h->storage = s;
  h->shifted = (flags & LBM_FLAG_SHIFTED) != 0;
  h->tau = tau;
  h->omega = std::isinf(tau) ? 0.0 : 1.0 / tau;
  h->pop = dev_pop;
  h->pop_bytes = pop_bytes;
  h->aux = (unsigned char*)dev_aux;
  h->aux_bytes = aux_bytes;
  h->lay = aux_layout(h->N, own_scratch);
  h->scratch = own_scratch ? h->aux + h->lay.scratch : shared;
  h->scratch_bytes = own_scratch ? own_scratch : shared_bytes;
  h->stream = (hipStream_t)hip_stream;
  h->bx = nx >= 256 ? 256 : ((nx + 63) / 64) * 64;
  h->nxb = (nx + h->bx - 1) / h->bx;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&h->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              h->device);
  if (e != hipSuccess) {
    delete h;
    return fail(nullptr, LBM_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
  }
  *out = h;
  return LBM_OK;
}

extern "C" {

lbm_status lbm_set_geometry(lbm_lattice* h, const uint8_t* material, unsigned periodic_mask) {
  lbm_status st = enter(h);
  if (st) return st;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (!material) return fail(h, LBM_ERR_ARG, "material is NULL");
  if (periodic_mask > 7u) return fail(h, LBM_ERR_ARG, "periodic_mask uses bits 0..2 only");
  std::vector<uint32_t> link, mov;
  long long nf = 0;
  bool hm = false;
  std::string why;
  st = h->q == 9 ? build_links<9>(h->nx, h->ny, h->nz, material, periodic_mask, &link, &mov, &nf,
                                  &hm, &why)
                 : build_links<19>(h->nx, h->ny, h->nz, material, periodic_mask, &link, &mov,
                                   &nf, &hm, &why);
  if (st) return fail(h, st, why);
  HIP_TRY(h, hipMemcpyAsync(h->aux + h->lay.link, link.data(), 4 * h->N, hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->aux + h->lay.mov, mov.data(), 4 * h->N, hipMemcpyHostToDevice,
                            h->stream));
  std::vector<uint8_t> cls(h->N);
  for (size_t i = 0; i < h->N; ++i)
    cls[i] = (uint8_t)(((link[i] & LINK_FLUID) ? CELL_FLUID : 0u) |
                       ((link[i] & LINK_HAS_MOVING) ? CELL_MOVING : 0u));
  HIP_TRY(h, hipMemcpyAsync(h->aux + h->lay.cls, cls.data(), h->N, hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  drop_graph(h);
  h->periodic = periodic_mask;
  h->nfluid = nf;
  h->has_moving_cells = hm;
  h->all_fluid = (size_t)nf == h->N;
  h->has_geometry = true;
  h->initialized = false;
  h->phase = 0;
  h->steps = 0;
  return LBM_OK;
}

lbm_status lbm_set_wall_velocity(lbm_lattice* h, const double u_w[3]) {
  if (!h) return LBM_ERR_ARG;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (!u_w) return fail(h, LBM_ERR_ARG, "u_w is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(u_w[a])) return fail(h, LBM_ERR_ARG, "u_w must be finite");
  if (h->q == 9 && u_w[2] != 0.0) return fail(h, LBM_ERR_ARG, "D2Q9 wall velocity needs u_w[2] == 0");
  for (int a = 0; a < 3; ++a) h->uw[a] = u_w[a];
  drop_graph(h);
  return LBM_OK;
}

lbm_status lbm_set_body_force(lbm_lattice* h, const double g[3]) {
  if (!h) return LBM_ERR_ARG;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (!g) return fail(h, LBM_ERR_ARG, "g is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g[a])) return fail(h, LBM_ERR_ARG, "g must be finite");
  if (h->q == 9 && g[2] != 0.0) return fail(h, LBM_ERR_ARG, "D2Q9 body force needs g[2] == 0");
  for (int a = 0; a < 3; ++a) h->g[a] = g[a];
  drop_graph(h);
  return LBM_OK;
}

lbm_status lbm_set_tau(lbm_lattice* h, double tau) {
  if (!h) return LBM_ERR_ARG;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (!tau_ok(tau)) return fail(h, LBM_ERR_ARG, "tau must be > 0.5 (or +inf for pure streaming)");
  h->tau = tau;
  h->omega = std::isinf(tau) ? 0.0 : 1.0 / tau;
  drop_graph(h);
  return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_lattice* h, const double* rho_dev, const double* u_dev) {
  lbm_status st = enter(h);
  if (st) return st;
  if (!h->has_geometry) return fail(h, LBM_ERR_STATE, "set the geometry first");
  ops(h).init_eq(h, rho_dev, u_dev);
  st = launch_check(h);
  if (st) return st;
  h->phase = 0;
  h->steps = 0;
  h->initialized = true;
  h->consistent = true;
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_lattice* h, const double* f_dev) {
  lbm_status st = enter(h);
  if (st) return st;
  if (!f_dev) return fail(h, LBM_ERR_ARG, "f_dev is NULL");
  if (!h->has_geometry) return fail(h, LBM_ERR_STATE, "set the geometry first");
  ops(h).set_pop(h, f_dev);
  st = launch_check(h);
  if (st) return st;
  h->phase = 0;
  h->steps = 0;
  h->initialized = true;
  h->consistent = true;
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_lattice* h, double* f_dev) {
  lbm_status st = enter(h);
  if (st) return st;
  if (!f_dev) return fail(h, LBM_ERR_ARG, "f_dev is NULL");
  st = readable(h);
  if (st) return st;
  ops(h).get_pop(h, f_dev);
  return launch_check(h);
}

lbm_status lbm_step(lbm_lattice* h, int n) {
  lbm_status st = enter(h);
  if (st) return st;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (n < 0) return fail(h, LBM_ERR_ARG, "n must be >= 0");
  if (!h->initialized) return fail(h, LBM_ERR_STATE, "initialise the populations first");
  st = readable(h);
  if (st) return st;
  st = enqueue_steps(h, n);
  if (st == LBM_OK) st = launch_check(h);
  if (st != LBM_OK) {
    // some launches may already be queued: phase and step count no longer
    // describe the device state
    h->consistent = false;
    drop_graph(h);
    return st;
  }
  h->steps += n;
  return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_lattice* h, int steps) {
  lbm_status st = enter(h);
  if (st) return st;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  if (steps < 0 || (steps & 1)) return fail(h, LBM_ERR_ARG, "graph length must be even and >= 0");
  if (steps > 0 && h->stream == nullptr)
    return fail(h, LBM_ERR_ARG, "graph replay needs a created (non-null) stream");
  drop_graph(h);
  h->graph_steps = steps;
  return LBM_OK;
}

lbm_status lbm_moments(lbm_lattice* h, double* rho, double* u) {
  lbm_status st = enter(h);
  if (st) return st;
  st = readable(h);
  if (st) return st;
  if (!rho && !u) return LBM_OK;
  // cells are decoded in chunks into the scratch (rho, then the three u
  // components, each `chunk` doubles) and copied out; the host waits for each
  const OpTable t = ops(h);
  const size_t chunk = h->scratch_bytes / MOMENT_BYTES_PER_CELL;
  double* sr = (double*)h->scratch;
  double* su = sr + chunk;
  for (size_t begin = 0; begin < h->N; begin += chunk) {
    const size_t n = h->N - begin < chunk ? h->N - begin : chunk;
    t.moments_f64(h, rho ? sr : nullptr, u ? su : nullptr, (uint32_t)begin, (uint32_t)n,
                  (uint32_t)chunk);
    st = launch_check(h);
    if (st) return st;
    if (rho)
      HIP_TRY(h, hipMemcpyAsync(rho + begin, sr, n * sizeof(double), hipMemcpyDeviceToHost,
                                h->stream));
    if (u)
      for (int a = 0; a < 3; ++a)
        HIP_TRY(h, hipMemcpyAsync(u + (size_t)a * h->N + begin, su + (size_t)a * chunk,
                                  n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

lbm_status lbm_moments_device(lbm_lattice* h, float* rho_dev, float* u_dev) {
  lbm_status st = enter(h);
  if (st) return st;
  st = readable(h);
  if (st) return st;
  if (!rho_dev && !u_dev) return LBM_OK;
  ops(h).moments_f32(h, rho_dev, u_dev, 0u, (uint32_t)h->N, (uint32_t)h->N);
  return launch_check(h);
}

lbm_status lbm_totals(lbm_lattice* h, double* mass, double momentum[3], double stats[3]) {
  lbm_status st = enter(h);
  if (st) return st;
  st = readable(h);
  if (st) return st;
  return reduce_totals(h, (double*)h->scratch, (double*)(h->aux + h->lay.result), mass, momentum,
                       stats);
}

lbm_status lbm_totals_noalloc(lbm_lattice* h, double* mass, double momentum[3],
                              double stats[3]) {
  lbm_status st = enter(h);
  if (st) return st;
  st = readable(h);
  if (st) return st;
  double* base = nullptr;
  st = static_scratch(h, &base);
  if (st) return st;
  return reduce_totals(h, base, base + STATIC_PARTIALS, mass, momentum, stats);
}

lbm_status lbm_get_info(const lbm_lattice* h, long long* steps, long long* fluid_cells) {
  if (!h) return LBM_ERR_ARG;
  if (steps) *steps = h->steps;
  if (fluid_cells) *fluid_cells = h->nfluid;
  return LBM_OK;
}

lbm_status lbm_lattice_destroy(lbm_lattice* h) {
  if (!h) return LBM_ERR_ARG;
  if (h->batch) return fail(h, LBM_ERR_STATE, "lattice belongs to a batch: use the lbm_batch_* calls");
  hipError_t e = hipSetDevice(h->device);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  drop_graph(h);
  delete h;
  return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

const char* lbm_status_string(lbm_status st) {
  switch (st) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_GEOMETRY: return "geometry rejected";
    case LBM_ERR_UNSUPPORTED: return "unsupported";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_STATE: return "invalid call order";
    case LBM_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_lattice* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
