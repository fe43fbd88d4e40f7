// lattice.hpp -- velocity sets, storage converters and the per-cell BGK + Guo
// update used by the gfx950 kernels in lbm.hip.
//
// Method: OpenLB User Guide, release 1.6 (arXiv:2307.11752).  Velocity sets:
// Core Concepts, "Descriptor" (the D2Q9 listing; D3Q19 is only drawn, so its
// set is the standard one: rest, 6 face and 12 edge neighbours, weights 1/3,
// 1/18, 1/36).  Collision: Introduction, "Lattice Boltzmann Methods" (BGK
// operator) and the BGK listing of "Collision Operators".  Forcing: Simulation
// Models, "Coupling Between Momentum and Energy Equations" (velocity shift
// u + F/2 and the Guo forcing term).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity sets.  Weights are stored as multiples of 1/36 so that both float
// and double get the correctly rounded value of the exact fraction.
// ---------------------------------------------------------------------------
template <int Q>
struct Vel;

template <>
struct Vel<9> {
  static constexpr int D = 2;
  static constexpr int cx[9] = {0, -1, -1, -1, 0, 1, 1, 1, 0};
  static constexpr int cy[9] = {0, 1, 0, -1, -1, -1, 0, 1, 1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
  static constexpr int w36[9] = {16, 1, 4, 1, 4, 1, 4, 1, 4};
};

template <>
struct Vel<19> {
  static constexpr int D = 3;
  static constexpr int cx[19] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
  static constexpr int cy[19] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
  static constexpr int cz[19] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};
  static constexpr int opp[19] = {0, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                                  1, 2,  3,  4,  5,  6,  7,  8,  9};
  static constexpr int w36[19] = {12, 2, 2, 2, 1, 1, 1, 1, 1, 1, 2, 2, 2, 1, 1, 1, 1, 1, 1};
};

template <int Q, typename T>
__host__ __device__ constexpr T weight(int i) {
  return T(Vel<Q>::w36[i]) / T(36);
}

// ---------------------------------------------------------------------------
// Storage converters.  F64 storage computes in double, every other storage
// type in float.
// ---------------------------------------------------------------------------
struct bf16s {
  uint16_t bits;
};

template <typename S>
struct Store;

template <>
struct Store<double> {
  using T = double;
  static constexpr double unit = 1.0;
  static __device__ __forceinline__ T load(const double* p) { return *p; }
  static __device__ __forceinline__ void store(double* p, T v) { *p = v; }
  static __device__ __forceinline__ double to_f64(double v) { return v; }
  static __device__ __forceinline__ double from_f64(double v) { return v; }
  static __device__ __forceinline__ T cvt(double v) { return v; }
  static __device__ __forceinline__ double pack(T v) { return v; }
};

template <>
struct Store<float> {
  using T = float;
  static constexpr float unit = 1.0f;
  static __device__ __forceinline__ T load(const float* p) { return *p; }
  static __device__ __forceinline__ void store(float* p, T v) { *p = v; }
  static __device__ __forceinline__ double to_f64(float v) { return (double)v; }
  static __device__ __forceinline__ float from_f64(double v) { return (float)v; }
  static __device__ __forceinline__ T cvt(float v) { return v; }
  static __device__ __forceinline__ float pack(T v) { return v; }
};

// FP16 storage holds the value times 2^12 (an exact power-of-two scale).  The
// weight-shifted populations of a slow flow, |f - w| down to ~1e-7, then sit
// in binary16's normal range (from 6.1e-5 / 2^12 = 1.5e-8) instead of among
// its subnormals, whose fixed spacing of 6e-8 would otherwise be the rounding
// error; any |value| < 16 still fits.  The step kernels work on the scaled
// values directly: the collision is homogeneous of degree one in (f, base)
// (StepParams::base, the density of the shifted rest state), so they only
// set base = 2^12 and convert without any multiply; the decoding and encoding
// routines (to_f64, from_f64) apply the scale.
constexpr float F16_SCALE = 4096.0f;

template <>
struct Store<_Float16> {
  using T = float;
  static constexpr float unit = F16_SCALE;  // stored value of 1.0
  static __device__ __forceinline__ T load(const _Float16* p) { return (float)*p; }
  static __device__ __forceinline__ void store(_Float16* p, T v) { *p = (_Float16)v; }
  static __device__ __forceinline__ double to_f64(_Float16 v) {
    return (double)(float)v / (double)F16_SCALE;
  }
  static __device__ __forceinline__ _Float16 from_f64(double v) {
    return (_Float16)(v * (double)F16_SCALE);
  }
  static __device__ __forceinline__ T cvt(_Float16 v) { return (float)v; }
  static __device__ __forceinline__ _Float16 pack(T v) { return (_Float16)v; }
};

// bfloat16: the upper half of an IEEE single; float -> bf16 rounds to nearest
// even (gfx950 converts in hardware, v_cvt_pk_bf16_f32, two values at a time).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}

template <>
struct Store<bf16s> {
  using T = float;
  static constexpr float unit = 1.0f;
  static __device__ __forceinline__ T load(const bf16s* p) {
    return __uint_as_float((uint32_t)p->bits << 16);
  }
  static __device__ __forceinline__ void store(bf16s* p, T v) { p->bits = f32_to_bf16_rne(v); }
  static __device__ __forceinline__ double to_f64(bf16s v) {
    return (double)__uint_as_float((uint32_t)v.bits << 16);
  }
  // double -> float -> bf16 (two roundings; only initialisation and
  // set_populations use it).
  static __device__ __forceinline__ bf16s from_f64(double v) {
    bf16s r;
    r.bits = f32_to_bf16_rne((float)v);
    return r;
  }
  static __device__ __forceinline__ T cvt(bf16s v) { return __uint_as_float((uint32_t)v.bits << 16); }
  static __device__ __forceinline__ bf16s pack(T v) {
    bf16s r;
    r.bits = f32_to_bf16_rne(v);
    return r;
  }
};

// Non-temporal (cache-bypassing) single-value access in the compute type.
template <typename S>
__device__ __forceinline__ typename Store<S>::T load_nt(const S* p) {
  return Store<S>::cvt(__builtin_nontemporal_load(p));
}
template <>
__device__ __forceinline__ float load_nt<bf16s>(const bf16s* p) {
  return __uint_as_float((uint32_t)__builtin_nontemporal_load((const uint16_t*)p) << 16);
}
template <typename S>
__device__ __forceinline__ void store_nt(S* p, typename Store<S>::T v) {
  __builtin_nontemporal_store(Store<S>::pack(v), p);
}
template <>
__device__ __forceinline__ void store_nt<bf16s>(bf16s* p, float v) {
  __builtin_nontemporal_store(f32_to_bf16_rne(v), (uint16_t*)p);
}

// ---------------------------------------------------------------------------
// Link words.  One 32-bit word per cell: bit 31 marks a fluid cell, bit k-1
// (k = 1..q-1) marks that the neighbour x + c_k is a bounce-back wall
// (material 2 or 3), bit 30 that at least one of those walls moves; the
// moving links themselves are in a second word per cell (same bit layout).
// ---------------------------------------------------------------------------
constexpr uint32_t LINK_FLUID = 1u << 31;
constexpr uint32_t LINK_HAS_MOVING = 1u << 30;
// Cell classes, one byte per cell (the local phase needs no more than these
// two bits of the link word): fluid, and has a moving-wall link.
constexpr uint32_t CELL_FLUID = 1u;
constexpr uint32_t CELL_MOVING = 2u;

// Placement of the populations in the buffer: population i of cell c sits at
// element i * pstride + (c >> lb) * bstride + (c & mask).
//   blocked: the cells fall into chunks of 2^lb; a chunk holds the q runs of
//            its populations back to back (pstride = 2^lb, bstride = q 2^lb),
//            so the slots a run of cells touches lie close together in HBM;
//   arrays:  one array per population (lb = 31, mask = 2^31 - 1, bstride = 0:
//            the chunk term vanishes for every cell index, pstride = N
//            rounded up to 64).
// Offsets are 32-bit: the whole buffer holds fewer than 2^32 elements, and a
// blocked buffer fewer than 2^32 bytes.
struct PopIndex {
  uint32_t lb, mask, bstride, pstride;
  __host__ __device__ __forceinline__ uint32_t cell(uint32_t c) const {
    return (c >> lb) * bstride + (c & mask);
  }
  __host__ __device__ __forceinline__ uint32_t at(int i, uint32_t c) const {
    return (uint32_t)i * pstride + cell(c);
  }
};

template <typename T>
struct StepParams {
  T base;       // stored value of 1.0 (Store<S>::unit): the rest density of shifted storage
  T omega;      // 1/tau
  T kguo;       // 1 - omega/2
  T g[3];       // body acceleration
  T mw[19];     // 6 w_i (c_i . u_w): moving-wall momentum term per unit density
  int has_force;
  int has_moving;
};

// Velocity i + H (H = (Q - 1) / 2) is the opposite of velocity i for
// 1 <= i <= H, with the same weight.
template <int Q>
constexpr bool pairs_are_opposite() {
  constexpr int H = (Q - 1) / 2;
  for (int i = 1; i <= H; ++i)
    if (Vel<Q>::opp[i] != i + H || Vel<Q>::cx[i + H] != -Vel<Q>::cx[i] ||
        Vel<Q>::cy[i + H] != -Vel<Q>::cy[i] || Vel<Q>::cz[i + H] != -Vel<Q>::cz[i] ||
        Vel<Q>::w36[i + H] != Vel<Q>::w36[i])
      return false;
  return true;
}

// 1 / rho.  float: the hardware reciprocal (within about one ulp, and
// biased: used as is, the bias accumulates in u over many steps) refined by
// one Newton step, r + r (1 - v r), which leaves an error far below half an
// ulp before the final rounding.  double: a division.
__device__ __forceinline__ float reciprocal(float v) {
  const float r = __builtin_amdgcn_rcpf(v);
  return fmaf(r, fmaf(-v, r, 1.0f), r);
}
__device__ __forceinline__ double reciprocal(double v) { return 1.0 / v; }

// One BGK + Guo collision of a cell held in registers (in place).
//   rho = base + sum f  (base = p.base when f stores f_i - w_i, else 0;
//                        p.base = 1 unless the storage holds scaled values)
//   u   = j/rho + g/2                                  (Guo velocity shift)
//   feq_i - base*w_i = w_i (sum f + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
//   f*_i = f_i + omega (feq_i - f_i) + (1 - omega/2) w_i (3 (c_i - u).F + 9 (c_i.u)(c_i.F))
// with F = rho g.  Returns rho.
// Evaluated by opposite pairs (i, i + H): with A = sum f - 1.5 rho u.u, the
// equilibrium is P + M for velocity i and P - M for its opposite, P = w_i (A +
// 4.5 rho (c_i.u)^2) and M = 3 w_i rho c_i.u; the Guo source likewise is
// G_P + G_M and G_P - G_M, G_P = (1 - omega/2) w_i (9 (c_i.u)(c_i.F) - 3 u.F)
// and G_M = 3 (1 - omega/2) w_i c_i.F.  The relaxation keeps the form
// f + omega (feq - f), whose rounding is that of the small non-equilibrium part.
// Compile-time loop: f(integral_constant<int, K>) for K = B .. E-1, so that
// the velocity components are constants inside the body.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// a x + b y + c z for a lattice velocity (a, b, c), components in {-1, 0, 1}.
// Zero components contribute no instruction (a product with 0 cannot be
// folded away by the compiler: it must keep NaN and signed-zero semantics),
// and unit ones only a sign.  Equal in value to the full dot product.
template <int A, int B, int C, typename T>
__device__ __forceinline__ T cdot(T x, T y, T z) {
  if constexpr (A != 0) {
    T r = A > 0 ? x : -x;
    if constexpr (B != 0) r = B > 0 ? r + y : r - y;
    if constexpr (C != 0) r = C > 0 ? r + z : r - z;
    return r;
  } else if constexpr (B != 0) {
    T r = B > 0 ? y : -y;
    if constexpr (C != 0) r = C > 0 ? r + z : r - z;
    return r;
  } else if constexpr (C != 0) {
    return C > 0 ? z : -z;
  } else {
    return T(0);
  }
}

// acc + s v for a compile-time sign s in {-1, 0, 1}; `first` marks an
// accumulator that holds nothing yet (it then becomes s v, not 0 + s v).
template <int Sg, typename T>
__device__ __forceinline__ void accumulate(T& acc, bool& first, T v) {
  if constexpr (Sg != 0) {
    if (first)
      acc = Sg > 0 ? v : -v;
    else
      acc = Sg > 0 ? acc + v : acc - v;
    first = false;
  }
}

// One BGK + Guo collision of a cell held in registers (in place).
//   rho = base + sum f  (base = p.base when f stores f_i - w_i, else 0;
//                        p.base = 1 unless the storage holds scaled values)
//   u   = j/rho + g/2                                  (Guo velocity shift)
//   feq_i - base*w_i = w_i (sum f + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
//   f*_i = f_i + omega (feq_i - f_i) + (1 - omega/2) w_i (3 (c_i - u).F + 9 (c_i.u)(c_i.F))
// with F = rho g.  Returns rho.
// Evaluated by opposite pairs (i, i + H): with A = sum f - 1.5 rho u.u, the
// equilibrium is P + M for velocity i and P - M for its opposite, P = w_i (A +
// 4.5 rho (c_i.u)^2) and M = 3 w_i rho c_i.u; the Guo source likewise is
// G_P + G_M and G_P - G_M, G_P = (1 - omega/2) w_i (9 (c_i.u)(c_i.F) - 3 u.F)
// and G_M = 3 (1 - omega/2) w_i c_i.F.  The relaxation keeps the form
// f + omega (feq - f), whose rounding is that of the small non-equilibrium part.
template <int Q, bool SHIFT, typename T>
__device__ __forceinline__ T collide(T (&f)[Q], const StepParams<T>& p) {
  using V = Vel<Q>;
  constexpr int H = (Q - 1) / 2;
  static_assert(pairs_are_opposite<Q>(), "velocity i + H must be the opposite of velocity i");
  T sf = f[0], jx = T(0), jy = T(0), jz = T(0);
  bool fx = true, fy = true, fz = true;
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const T d = f[k] - f[k + H];
    sf += f[k] + f[k + H];
    accumulate<V::cx[k]>(jx, fx, d);
    accumulate<V::cy[k]>(jy, fy, d);
    accumulate<V::cz[k]>(jz, fz, d);
  });
  const T rho = SHIFT ? p.base + sf : sf;
  const T inv = reciprocal(rho);
  T ux = jx * inv, uy = jy * inv, uz = V::D == 3 ? jz * inv : T(0);
  if (p.has_force) {
    ux += T(0.5) * p.g[0];
    uy += T(0.5) * p.g[1];
    if (V::D == 3) uz += T(0.5) * p.g[2];
  }
  const T uu = V::D == 3 ? ux * ux + uy * uy + uz * uz : ux * ux + uy * uy;
  const T A = sf - T(1.5) * rho * uu;
  const T om = p.omega;
  f[0] = fma(om, weight<Q, T>(0) * A - f[0], f[0]);
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const T w = weight<Q, T>(k);
    const T cu = cdot<V::cx[k], V::cy[k], V::cz[k]>(ux, uy, uz);
    const T rc = rho * cu;
    // w multiplies last: a folded constant such as 3 w would carry its own
    // rounding (1/6 is not a binary fraction), a bias the odd part would add
    // to the momentum of every collision
    const T P = w * fma(T(4.5) * rc, cu, A);
    const T M = w * (T(3) * rc);
    f[k] = fma(om, (P + M) - f[k], f[k]);
    f[k + H] = fma(om, (P - M) - f[k + H], f[k + H]);
  });
  // The Guo source is a block of its own behind a uniform branch, so that
  // unforced lattices skip it instead of computing and discarding it.
  if (p.has_force) {
    const T Fx = rho * p.g[0], Fy = rho * p.g[1], Fz = V::D == 3 ? rho * p.g[2] : T(0);
    const T uF = V::D == 3 ? ux * Fx + uy * Fy + uz * Fz : ux * Fx + uy * Fy;
    const T kg = p.kguo;
    f[0] += kg * weight<Q, T>(0) * (T(-3) * uF);
    static_for<1, H + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const T kw = kg * weight<Q, T>(k);
      const T cu = cdot<V::cx[k], V::cy[k], V::cz[k]>(ux, uy, uz);
      const T cF = cdot<V::cx[k], V::cy[k], V::cz[k]>(Fx, Fy, Fz);
      const T GP = kw * fma(T(9) * cu, cF, T(-3) * uF);
      const T GM = kw * (T(3) * cF);
      f[k] += GP + GM;
      f[k + H] += GP - GM;
    });
  }
  return rho;
}

// ---------------------------------------------------------------------------
// Neighbour addressing.  Coordinates wrap on every axis; on non-periodic axes
// fluid cells never sit on the edge, so the wrap is never taken there.
// ---------------------------------------------------------------------------
struct Nbr {
  int X[3];
  uint32_t R[3][3];  // R[dy+1][dz+1] = nx*(y' + ny*z')
  __device__ __forceinline__ uint32_t at(int dx, int dy, int dz) const {
    return (uint32_t)X[dx + 1] + R[dy + 1][dz + 1];
  }
};

// px: cells from one stored x-row to the next (nx, or more for padded rows).
__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, int nx, int ny, int nz, int px) {
  Nbr n;
  n.X[0] = x == 0 ? nx - 1 : x - 1;
  n.X[1] = x;
  n.X[2] = x == nx - 1 ? 0 : x + 1;
  const int Y[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int Z[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) n.R[a][b] = (uint32_t)px * (uint32_t)(Y[a] + ny * Z[b]);
  return n;
}
__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, int nx, int ny, int nz) {
  return make_nbr(x, y, z, nx, ny, nz, nx);
}

}  // namespace lbm
