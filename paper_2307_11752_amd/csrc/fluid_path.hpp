// fluid_path.hpp -- cell-range bodies of the fully-fluid fast path, shared by
// the single-lattice kernels (lbm.hip) and the batched ensemble (batch.hip).
//
// Every lane moves C consecutive cells of one population (C * sizeof(S) bytes,
// at most 8) with one aligned, non-temporal access per direction.
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
// f*_i into slot opp(i).  PS is the population stride (a multiple of 64
// elements) and c0 % C == 0.
template <int Q, typename S, bool SHIFT, int C>
__device__ __forceinline__ void fluid_cells_p0(S* __restrict__ pop, uint32_t PS, uint32_t c0,
                                               const StepParams<typename Store<S>::T>& p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  using L = Lane<S, C>;
  S sv[Q][C];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    L::unpack(__builtin_nontemporal_load((const typename L::raw*)(pop + (uint32_t)i * PS + c0)), sv[i]);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    T f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::cvt(sv[i][k]);
    collide<Q, SHIFT, T>(f, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) sv[V::opp[i]][k] = Store<S>::pack(f[i]);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(L::pack(sv[i]), (typename L::raw*)(pop + (uint32_t)i * PS + c0));
}

// Phase 1 of x-row `row` (= y + ny z) of a fully fluid periodic lattice, lane
// t covering cells x = C t .. C t + C - 1.  PS: population stride; tile:
// NS * nx values of LDS for this row.  Contains block barriers: every thread
// of the block must call it (inactive lanes with active = false).  nx % C == 0.
template <int Q, typename S, bool SHIFT, int C>
__device__ __forceinline__ void fluid_rows_p1(S* __restrict__ pop, int nx, int ny, int nz,
                                              uint32_t PS, int row, bool active, int t, S* tile,
                                              const StepParams<typename Store<S>::T>& p) {
  using T = typename Store<S>::T;
  using V = Vel<Q>;
  using L = Lane<S, C>;
  const int y = active ? row % ny : 0;
  const int z = active ? row / ny : 0;
  const int Y[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int Z[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  const int x0 = C * t;

  S sv[Q][C];
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int o = V::opp[i];
      const uint32_t base = (uint32_t)o * PS + (uint32_t)nx * (uint32_t)(Y[1 - V::cy[i]] + ny * Z[1 - V::cz[i]]);
      const typename L::raw r = __builtin_nontemporal_load((const typename L::raw*)(pop + base + x0));
      if (V::cx[i] == 0)
        L::unpack(r, sv[i]);
      else
        *(typename L::raw*)(tile + Shifted<Q>::rank(i) * nx + x0) = r;
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
        sv[i][k] = tile[Shifted<Q>::rank(i) * nx + xs];
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
        const uint32_t base = (uint32_t)i * PS + (uint32_t)nx * (uint32_t)(Y[1 + V::cy[i]] + ny * Z[1 + V::cz[i]]);
        __builtin_nontemporal_store(L::pack(sv[i]), (typename L::raw*)(pop + base + x0));
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int xd = x0 + k + V::cx[i];
          xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
          tile[Shifted<Q>::rank(i) * nx + xd] = sv[i][k];
        }
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cx[i] == 0) continue;
      const uint32_t base = (uint32_t)i * PS + (uint32_t)nx * (uint32_t)(Y[1 + V::cy[i]] + ny * Z[1 + V::cz[i]]);
      __builtin_nontemporal_store(*(const typename L::raw*)(tile + Shifted<Q>::rank(i) * nx + x0),
                                  (typename L::raw*)(pop + base + x0));
    }
  }
}

}  // namespace lbm
