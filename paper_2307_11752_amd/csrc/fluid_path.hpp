// fluid_path.hpp -- cell-range bodies of the fully-fluid fast path, shared by
// the single-lattice kernels (lbm.hip) and the batched ensemble (batch.hip).
//
// Every lane moves C consecutive cells of one population (C * sizeof(S) bytes,
// at most 8) with one aligned, non-temporal access per direction; PopIndex
// places the populations in the buffer.
//   phase 0 needs no neighbour: flat cell ranges;
//   phase 1 works on whole x-rows: the populations a row receives from x -/+ 1
//   are loaded aligned into LDS and read back shifted (with the periodic wrap
//   inside the row); outgoing x-shifted populations are written shifted into
//   LDS and stored aligned.  This removes the one-element misalignment of the
//   AA pattern's neighbour accesses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

typedef uint32_t raw8 __attribute__((ext_vector_type(2)));

template <int BYTES>
struct RawOf;
template <>
struct RawOf<2> {
  using type = uint16_t;
};
template <>
struct RawOf<4> {
  using type = uint32_t;
};
template <>
struct RawOf<8> {
  using type = raw8;
};

// C consecutive values of storage type S as one machine word.
template <typename S, int C_>
struct Lane {
  static constexpr int C = C_;
  using raw = typename RawOf<C_ * (int)sizeof(S)>::type;
  static __device__ __forceinline__ void unpack(raw r, S (&v)[C]) { __builtin_memcpy(v, &r, sizeof(raw)); }
  static __device__ __forceinline__ raw pack(const S (&v)[C]) {
    raw r;
    __builtin_memcpy(&r, v, sizeof(raw));
    return r;
  }
};

template <typename S>
using Pack8 = Lane<S, 8 / (int)sizeof(S)>;

// A lane's word at a uniform base plus a 32-bit byte offset.  Offsets inside
// one population array always fit (q * N < 2^32 elements), and this form lets
// the hardware add a scalar base to a 32-bit vector offset instead of holding
// one 64-bit address per direction in vector registers.
// (The base passes through readfirstlane so that the compiler keeps it apart
// from the vector offset; it must be the same in every lane.)
template <typename R>
using global_ptr = __attribute__((address_space(1))) R*;

template <typename R, typename S>
__device__ __forceinline__ global_ptr<R> at_byte(const S* base, uint32_t byte_off) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return (global_ptr<R>)((__attribute__((address_space(1))) char*)(((uint64_t)hi << 32) | lo) + byte_off);
}

template <int Q>
struct Shifted {
  // number of velocities with c_x != 0, and the rank of velocity i among them
  static constexpr int count() {
    int n = 0;
    for (int i = 0; i < Q; ++i) n += Vel<Q>::cx[i] != 0;
    return n;
  }
  static constexpr int rank(int i) {
    int n = 0;
    for (int k = 0; k < i; ++k) n += Vel<Q>::cx[k] != 0;
    return n;
  }
};

// Phase 0 of cells c0 .. c0+C-1 (all fluid): read own slots, collide, write
// f*_i into slot opp(i).  L places the populations (C consecutive cells of a
// population are adjacent: c0 % C == 0 and C divides the chunk size).
template <int Q, typename S, bool SHIFT, int C>
__device__ __forceinline__ void fluid_cells_p0(S* __restrict__ pop, const PopIndex& L, uint32_t c0,
                                               const StepParams<typename Store<S>::T>& p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  using W = Lane<S, C>;
  using R = typename W::raw;
  const uint32_t lo = L.cell(c0) * (uint32_t)sizeof(S);
  S sv[Q][C];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    W::unpack(__builtin_nontemporal_load(at_byte<R>(pop + (size_t)i * L.pstride, lo)), sv[i]);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    T f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::cvt(sv[i][k]);
    collide<Q, SHIFT, T>(f, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) sv[V::opp[i]][k] = Store<S>::pack(f[i]);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(W::pack(sv[i]), at_byte<R>(pop + (size_t)i * L.pstride, lo));
}

// Phase 1 of x-row `row` (= y + ny z) of a fully fluid periodic lattice, lane
// t covering cells x = C t .. C t + C - 1.  Stored rows are px >= nx cells
// apart (px % C == 0); with PADDED, the slots x = nx .. px - 1 of each row hold
// no cell: lanes there compute values nobody reads and send nothing along the
// row.  L places the populations; tile: NS * px values of LDS for this row.
// NT_LOADS = false reads through the caches (for rows that share lines with
// their neighbours, as short rows do).  Contains block barriers: every thread
// of the block must call it (inactive lanes with active = false).
template <int Q, typename S, bool SHIFT, int C, bool PADDED = false, bool NT_LOADS = true>
__device__ __forceinline__ void fluid_rows_p1(S* __restrict__ pop, int nx, int px, int ny, int nz,
                                              const PopIndex& L, int row, bool active, int t, S* tile,
                                              const StepParams<typename Store<S>::T>& p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  using W = Lane<S, C>;
  const int y = active ? row % ny : 0;
  const int z = active ? row / ny : 0;
  const int Y[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int Z[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  const int x0 = C * t;

  using R = typename W::raw;
  S sv[Q][C];
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const uint32_t off = L.cell((uint32_t)px * (uint32_t)(Y[1 - V::cy[i]] + ny * Z[1 - V::cz[i]]) + x0);
      const auto src = at_byte<R>(pop + (size_t)V::opp[i] * L.pstride, off * (uint32_t)sizeof(S));
      const R r = NT_LOADS ? __builtin_nontemporal_load(src) : *src;
      if (V::cx[i] == 0)
        W::unpack(r, sv[i]);
      else
        *(typename W::raw*)(tile + Shifted<Q>::rank(i) * px + x0) = r;
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cx[i] == 0) continue;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        int xs = x0 + k - V::cx[i];
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        sv[i][k] = tile[Shifted<Q>::rank(i) * px + xs];
      }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T f[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = Store<S>::cvt(sv[i][k]);
      collide<Q, SHIFT, T>(f, p);
#pragma unroll
      for (int i = 0; i < Q; ++i) sv[i][k] = Store<S>::pack(f[i]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cx[i] == 0) {
        const uint32_t off = L.cell((uint32_t)px * (uint32_t)(Y[1 + V::cy[i]] + ny * Z[1 + V::cz[i]]) + x0);
        __builtin_nontemporal_store(W::pack(sv[i]), at_byte<R>(pop + (size_t)i * L.pstride, off * (uint32_t)sizeof(S)));
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
          if (PADDED && x0 + k >= nx) continue;  // a padding slot sends nothing
          int xd = x0 + k + V::cx[i];
          xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
          tile[Shifted<Q>::rank(i) * px + xd] = sv[i][k];
        }
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cx[i] == 0) continue;
      const uint32_t off = L.cell((uint32_t)px * (uint32_t)(Y[1 + V::cy[i]] + ny * Z[1 + V::cz[i]]) + x0);
      __builtin_nontemporal_store(*(const R*)(tile + Shifted<Q>::rank(i) * px + x0),
                                  at_byte<R>(pop + (size_t)i * L.pstride, off * (uint32_t)sizeof(S)));
    }
  }
}

// One value taken from lane `src` of the wave (ds_bpermute; every lane of the
// wave that reaches this call takes part).
template <typename S>
__device__ __forceinline__ S lane_take(S v, int src) {
  static_assert(sizeof(S) == 2 || sizeof(S) == 4 || sizeof(S) == 8, "element size");
  constexpr int W = sizeof(S) == 8 ? 2 : 1;
  uint32_t w[W] = {};
  __builtin_memcpy(w, &v, sizeof(S));
#pragma unroll
  for (int j = 0; j < W; ++j) w[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)w[j]);
  S r;
  __builtin_memcpy(&r, w, sizeof(S));
  return r;
}

// v[k] <- the row's element k - s (s = +1 or -1) for a lane holding C
// consecutive cells of an x-row: the element that crosses into this lane
// comes from lane `left` (s = +1) or `right` (s = -1), the lanes holding the
// preceding and following cells (periodic within the row).
template <typename S, int C>
__device__ __forceinline__ void shift_along_row(S (&v)[C], int s, int left, int right) {
  if (s > 0) {
    const S edge = lane_take(v[C - 1], left);
#pragma unroll
    for (int k = C - 1; k > 0; --k) v[k] = v[k - 1];
    v[0] = edge;
  } else {
    const S edge = lane_take(v[0], right);
#pragma unroll
    for (int k = 0; k < C - 1; ++k) v[k] = v[k + 1];
    v[C - 1] = edge;
  }
}

// Phase 1 of x-row `row` (= y + ny z) of a fully fluid periodic lattice held
// by nx / C lanes of one wave, lane t covering cells x = C t .. C t + C - 1
// (`left` / `right`: the lanes holding row positions t - 1 and t + 1, wrapped).
// Every access is an aligned, non-temporal row segment; populations with
// c_x != 0 move one cell between lanes in registers after loading and before
// storing, so no LDS tile and no barrier is needed.  A row must not straddle
// two chunks of L (nx divides the chunk size), so that a row's slots are
// addressed from the row start plus x.
template <int Q, typename S, bool SHIFT, int C>
__device__ __forceinline__ void fluid_rows_p1_wave(S* __restrict__ pop, int nx, int ny, int nz,
                                                   const PopIndex& L, int row, int t, int left,
                                                   int right,
                                                   const StepParams<typename Store<S>::T>& p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  using W = Lane<S, C>;
  const int y = row % ny;
  const int z = row / ny;
  const int Y[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int Z[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  using R = typename W::raw;
  const uint32_t x0 = (uint32_t)(C * t);

  // incoming: f_i(x) = A[opp(i)][x - c_i]
  S sv[Q][C];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t r = L.cell((uint32_t)nx * (uint32_t)(Y[1 - V::cy[i]] + ny * Z[1 - V::cz[i]]));
    W::unpack(__builtin_nontemporal_load(at_byte<R>(pop + (size_t)V::opp[i] * L.pstride, (r + x0) * (uint32_t)sizeof(S))), sv[i]);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    if (V::cx[i] != 0) shift_along_row<S, C>(sv[i], V::cx[i], left, right);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    T f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::cvt(sv[i][k]);
    collide<Q, SHIFT, T>(f, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) sv[i][k] = Store<S>::pack(f[i]);
    // one cell at a time: interleaving the C collisions only raises register
    // pressure (and lowers occupancy) in a kernel bound by memory
    __builtin_amdgcn_sched_barrier(0);
  }
  // outgoing: A[i][x + c_i] = f*_i(x)
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (V::cx[i] != 0) shift_along_row<S, C>(sv[i], V::cx[i], left, right);
    const uint32_t r = L.cell((uint32_t)nx * (uint32_t)(Y[1 + V::cy[i]] + ny * Z[1 + V::cz[i]]));
    __builtin_nontemporal_store(W::pack(sv[i]), at_byte<R>(pop + (size_t)i * L.pstride, (r + x0) * (uint32_t)sizeof(S)));
  }
}

}  // namespace lbm
