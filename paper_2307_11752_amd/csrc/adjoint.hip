// adjoint.hip -- porous D3Q19 channel and its hand-written discrete adjoint:
// the gradient of an outlet-plane objective with respect to a per-cell
// porosity field, by reverse time stepping with checkpointed recomputation.
//
// Model (OpenLB User Guide 1.6, Simulation Models, "Porous Media Model"): the
// porosity d in [0, 1] (0 solid, 1 fluid) scales the velocity of the
// Maxwellian; here the equilibrium and the Guo term of the fused BGK
// collision both use v = d u with the force-shifted u = j/rho + g/2, and
// d = 1 is the plain collision.  Objective: the mean force-shifted x-velocity
// over the fluid cells of one x-plane after `steps` steps from rest.
// Gradients: the guide's adjoint-LBM option of "Derivative Computation"
// (Flow Control and Optimization), derived for this discrete scheme:
//   mu = Stream^T lambda^{t+1}; lambda^t = (dC/df)^T mu; dJ/dd += (dC/dd)^T mu
// at the state f^t (C = collision).  With G_a = sum_i mu_i (omega dfeq_i/dv_a
// + dS_i/dv_a) and E = sum_i mu_i (omega feq_i + S_i) / rho:
//   lambda^t_j = (1 - omega) mu_j + E - d (G.j)/rho^2 + (d/rho) G.c_j
//   dJ/dd     += G.u
// Storage and arithmetic are FP32 (the objective is reduced in FP64); the
// stored value is f_i - w_i, so that the small deviations from rest keep
// their precision (the gradient with respect to f is unchanged by the shift).
// Populations use the natural layout of two ping-pong lattices (a plain
// push step), so that checkpoints and recomputed states are ordinary arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

constexpr int Q = 19;
using V = Vel<Q>;

struct PorousLayout {
  size_t state_bytes = 0;  // one population set, Q * PS floats
  size_t fa = 0, fb = 0, ckpt = 0, seg = 0, la = 0, lb = 0, por = 0, link = 0, red = 0, total = 0;
  int nckpt = 0;
};

PorousLayout porous_layout(size_t N, int steps, int every) {
  PorousLayout L;
  L.state_bytes = align256(sizeof(float) * Q * pop_stride(N));
  L.nckpt = (steps + every - 1) / every;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.fa = take(L.state_bytes);
  L.fb = take(L.state_bytes);
  L.ckpt = take(L.state_bytes * (size_t)std::max(L.nckpt, 1));
  L.seg = take(L.state_bytes * (size_t)every);
  L.la = take(L.state_bytes);
  L.lb = take(L.state_bytes);
  L.por = take(sizeof(float) * N);
  L.link = take(sizeof(uint32_t) * N);
  L.red = take(sizeof(double) * (RED_BLOCKS + 8));
  L.total = off;
  return L;
}

// Collision quantities of one cell from its stored values fs_i = f_i - w_i:
// drho = sum fs (rho = 1 + drho), j, u (force-shifted), v = d u.
struct CellState {
  float drho, rho, j[3], u[3], v[3];
};

__device__ __forceinline__ CellState cell_state(const float (&fs)[Q], float d, const float* g) {
  CellState c;
  float s = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    s += fs[i];
    jx += (float)V::cx[i] * fs[i];
    jy += (float)V::cy[i] * fs[i];
    jz += (float)V::cz[i] * fs[i];
  }
  c.drho = s;
  c.rho = 1.f + s;
  c.j[0] = jx;
  c.j[1] = jy;
  c.j[2] = jz;
  const float inv = 1.f / c.rho;
  for (int a = 0; a < 3; ++a) {
    c.u[a] = c.j[a] * inv + 0.5f * g[a];
    c.v[a] = d * c.u[a];
  }
  return c;
}

// feq_i - w_i (shifted equilibrium) and the Guo term of velocity i.
__device__ __forceinline__ void feq_and_guo(const CellState& c, float omega, const float* g,
                                            int i, float* feqs, float* S) {
  const float w = weight<Q, float>(i);
  const float cv = (float)V::cx[i] * c.v[0] + (float)V::cy[i] * c.v[1] + (float)V::cz[i] * c.v[2];
  const float vv = c.v[0] * c.v[0] + c.v[1] * c.v[1] + c.v[2] * c.v[2];
  *feqs = w * (c.drho + c.rho * (3.f * cv + 4.5f * cv * cv - 1.5f * vv));
  const float F[3] = {c.rho * g[0], c.rho * g[1], c.rho * g[2]};
  const float cF = (float)V::cx[i] * F[0] + (float)V::cy[i] * F[1] + (float)V::cz[i] * F[2];
  const float vF = c.v[0] * F[0] + c.v[1] * F[1] + c.v[2] * F[2];
  *S = (1.f - 0.5f * omega) * w * (3.f * (cF - vF) + 9.f * cv * cF);
}

struct PorousParams {
  float omega;
  float g[3];
};

// Porous BGK + Guo collision of one cell held in registers: f (stored values
// f_i - w_i) and its porosity d in, the post-collision stored values out.
// Evaluated by opposite pairs (i, i + H): the shifted equilibrium is P + M and
// P - M, P = w (drho - 1.5 rho v.v + 4.5 rho (c.v)^2) and M = 3 w rho c.v; the
// Guo term is GP + GM and GP - GM, GP = k w (9 (c.v)(c.F) - 3 v.F) and
// GM = 3 k w c.F.  The weight multiplies last (a folded constant such as 3 w
// would bias the momentum by its own rounding).
__device__ __forceinline__ void porous_collide_cell(const float (&f)[Q], float d,
                                                    const PorousParams& p, float (&out)[Q]) {
  const CellState c = cell_state(f, d, p.g);
  constexpr int H = (Q - 1) / 2;
  static_assert(pairs_are_opposite<Q>(), "velocity i + H must be the opposite of velocity i");
  const float k = 1.f - 0.5f * p.omega;
  const float F[3] = {c.rho * p.g[0], c.rho * p.g[1], c.rho * p.g[2]};
  const float vF = c.v[0] * F[0] + c.v[1] * F[1] + c.v[2] * F[2];
  const float A = c.drho - 1.5f * c.rho * (c.v[0] * c.v[0] + c.v[1] * c.v[1] + c.v[2] * c.v[2]);
  {
    const float w = weight<Q, float>(0);
    out[0] = fmaf(p.omega, w * A - f[0], f[0]) + k * w * (-3.f * vF);
  }
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const float w = weight<Q, float>(i);
    const float cv = (float)V::cx[i] * c.v[0] + (float)V::cy[i] * c.v[1] + (float)V::cz[i] * c.v[2];
    const float cF = (float)V::cx[i] * F[0] + (float)V::cy[i] * F[1] + (float)V::cz[i] * F[2];
    const float rc = c.rho * cv;
    const float P = w * fmaf(4.5f * rc, cv, A);
    const float M = w * (3.f * rc);
    const float GP = k * w * fmaf(9.f * cv, cF, -3.f * vF);
    const float GM = k * w * (3.f * cF);
    out[i] = fmaf(p.omega, (P + M) - f[i], f[i]) + (GP + GM);
    out[i + H] = fmaf(p.omega, (P - M) - f[i + H], f[i + H]) + (GP - GM);
  }
}

// Block order of the per-cell kernels: runs of XCD_RUN consecutive blocks
// (rows of the lattice) go to one XCD (the hardware deals blocks to the 8
// XCDs in turn, so blocks b, b + 8, b + 16, ... share one L2); blocks past the
// last whole run keep the plain order.  Gradient of the 128 x 64 x 64 channel
// 25.8 -> 25.0 ms (forward 7.02 -> 6.96, backward 18.76 -> 18.06 ms; runs of
// 64 blocks: 25.3 ms).
__device__ __forceinline__ uint32_t xcd_run_block() {
  constexpr uint32_t XCD_RUN = 16, span = 8 * XCD_RUN;
  const uint32_t b = blockIdx.x;
  if (b >= gridDim.x / span * span) return b;
  return XCD_RUN * (8 * (b / span) + (b & 7)) + ((b >> 3) % XCD_RUN);
}

// Forward: collide every fluid cell of src with its porosity and push to dst
// (wall links reflect into the cell's own opposite slot).  One cell per thread.
__global__ void __launch_bounds__(256)
    porous_step_kernel(const float* __restrict__ src, float* __restrict__ dst,
                       const float* __restrict__ por, const uint32_t* __restrict__ link, int nx,
                       int ny, int nz, uint32_t N, uint32_t PS, PorousParams p) {
  const uint32_t idx = xcd_run_block() * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const uint32_t lw = link[idx];
  if (!(lw & LINK_FLUID)) return;
  const int x = (int)(idx % (uint32_t)nx);
  const int r = (int)(idx / (uint32_t)nx);
  const Nbr nb = make_nbr(x, r % ny, r / ny, nx, ny, nz);
  float f[Q], out[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = src[(uint32_t)i * PS + idx];
  porous_collide_cell(f, por[idx], p, out);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool wall = i > 0 && ((lw >> (i - 1)) & 1u);
    const uint32_t off = wall ? (uint32_t)V::opp[i] * PS + idx
                              : (uint32_t)i * PS + nb.at(V::cx[i], V::cy[i], V::cz[i]);
    dst[off] = out[i];
  }
}

// Adjoint of one cell's collision: f (stored values at step t), mu (the
// pulled adjoint of step t + 1) and porosity d in; lambda^t of the cell out;
// returns the cell's contribution G.u to dJ/dd.
__device__ __forceinline__ float porous_adjoint_cell(const float (&f)[Q], const float (&mu)[Q],
                                                     float d, const PorousParams& p,
                                                     float (&lam)[Q]) {
  const CellState c = cell_state(f, d, p.g);
  const float k = 1.f - 0.5f * p.omega;
  const float F[3] = {c.rho * p.g[0], c.rho * p.g[1], c.rho * p.g[2]};
  // G_a = sum_i mu_i (omega dfeq_i/dv_a + dS_i/dv_a) and rho E = sum_i mu_i
  // (omega feq_i + S_i) depend on mu only through the moments of m_i = w_i mu_i:
  // M0 = sum m_i, M1 = sum m_i c_i, M2 = sum m_i c_i c_i.  With
  //   dfeq_i/dv_a = w_i rho (3 c_ia + 9 (c_i.v) c_ia - 3 v_a),
  //   dS_i/dv_a   = k w_i (9 c_ia (c_i.F) - 3 F_a),
  //   feq_i       = w_i rho (1 + 3 c_i.v + 4.5 (c_i.v)^2 - 1.5 v.v),
  //   S_i         = k w_i (3 c_i.F - 3 v.F + 9 (c_i.v)(c_i.F)):
  //   G   = omega rho (3 M1 + 9 M2 v - 3 M0 v) + k (9 M2 F - 3 M0 F),
  //   rho E = omega rho (M0 (1 - 1.5 v.v) + 3 M1.v + 4.5 v.M2 v)
  //           + k (3 M1.F - 3 M0 v.F + 9 v.M2 F).
  float m0 = 0.f, m1[3] = {0.f, 0.f, 0.f};
  float mxx = 0.f, myy = 0.f, mzz = 0.f, mxy = 0.f, mxz = 0.f, myz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float m = weight<Q, float>(i) * mu[i];
    const int cx = V::cx[i], cy = V::cy[i], cz = V::cz[i];
    m0 += m;
    if (cx) m1[0] += cx > 0 ? m : -m;
    if (cy) m1[1] += cy > 0 ? m : -m;
    if (cz) m1[2] += cz > 0 ? m : -m;
    if (cx) mxx += m;
    if (cy) myy += m;
    if (cz) mzz += m;
    if (cx && cy) mxy += cx * cy > 0 ? m : -m;
    if (cx && cz) mxz += cx * cz > 0 ? m : -m;
    if (cy && cz) myz += cy * cz > 0 ? m : -m;
  }
  const float* v = c.v;
  const float M2v[3] = {mxx * v[0] + mxy * v[1] + mxz * v[2], mxy * v[0] + myy * v[1] + myz * v[2],
                        mxz * v[0] + myz * v[1] + mzz * v[2]};
  const float M2F[3] = {mxx * F[0] + mxy * F[1] + mxz * F[2], mxy * F[0] + myy * F[1] + myz * F[2],
                        mxz * F[0] + myz * F[1] + mzz * F[2]};
  float G[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    G[a] = p.omega * c.rho * (3.f * m1[a] + 9.f * M2v[a] - 3.f * m0 * v[a]) +
           k * (9.f * M2F[a] - 3.f * m0 * F[a]);
  const float vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const float vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
  const float m1v = m1[0] * v[0] + m1[1] * v[1] + m1[2] * v[2];
  const float m1F = m1[0] * F[0] + m1[1] * F[1] + m1[2] * F[2];
  const float vM2v = v[0] * M2v[0] + v[1] * M2v[1] + v[2] * M2v[2];
  const float vM2F = v[0] * M2F[0] + v[1] * M2F[1] + v[2] * M2F[2];
  const float E = p.omega * (m0 * (1.f - 1.5f * vv) + 3.f * m1v + 4.5f * vM2v) +
                  k * (3.f * m1F - 3.f * m0 * vF + 9.f * vM2F) / c.rho;
  const float Arho = E - d * (G[0] * c.j[0] + G[1] * c.j[1] + G[2] * c.j[2]) / (c.rho * c.rho);
  const float s = d / c.rho;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    lam[i] = (1.f - p.omega) * mu[i] + Arho +
             s * (G[0] * (float)V::cx[i] + G[1] * (float)V::cy[i] + G[2] * (float)V::cz[i]);
  return G[0] * c.u[0] + G[1] * c.u[1] + G[2] * c.u[2];
}

// Adjoint of one step at state f (natural layout): pull mu from lam_next,
// write lam_cur, accumulate the porosity gradient.  One cell per thread.
__global__ void __launch_bounds__(256)
    porous_adjoint_kernel(const float* __restrict__ f_t, const float* __restrict__ lam_next,
                          float* __restrict__ lam_cur, float* __restrict__ grad,
                          const float* __restrict__ por, const uint32_t* __restrict__ link,
                          int nx, int ny, int nz, uint32_t N, uint32_t PS, PorousParams p) {
  const uint32_t idx = xcd_run_block() * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const uint32_t lw = link[idx];
  if (!(lw & LINK_FLUID)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) lam_cur[(uint32_t)i * PS + idx] = 0.f;
    return;
  }
  const int x = (int)(idx % (uint32_t)nx);
  const int r = (int)(idx / (uint32_t)nx);
  const Nbr nb = make_nbr(x, r % ny, r / ny, nx, ny, nz);
  float mu[Q], f[Q], lam[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool wall = i > 0 && ((lw >> (i - 1)) & 1u);
    const uint32_t off = wall ? (uint32_t)V::opp[i] * PS + idx
                              : (uint32_t)i * PS + nb.at(V::cx[i], V::cy[i], V::cz[i]);
    mu[i] = lam_next[off];
    f[i] = f_t[(uint32_t)i * PS + idx];
  }
  grad[idx] += porous_adjoint_cell(f, mu, por[idx], p, lam);
#pragma unroll
  for (int i = 0; i < Q; ++i) lam_cur[(uint32_t)i * PS + idx] = lam[i];
}

// Rest state (rho = 1, u = 0: f_i = w_i), stored shifted: zero everywhere.
__global__ void porous_init_kernel(float* __restrict__ f, uint32_t N, uint32_t PS) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x)
#pragma unroll
    for (int i = 0; i < Q; ++i) f[(uint32_t)i * PS + idx] = 0.f;
}

__global__ void fill_kernel(float* __restrict__ a, size_t n, float v) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    a[k] = v;
}

// Objective (one block): mean of u_x over the fluid cells of plane x = px.
__global__ void __launch_bounds__(256)
    porous_objective_kernel(const float* __restrict__ f, const uint32_t* __restrict__ link,
                            int px, int nx, int ny, int nz, uint32_t PS, float gx,
                            double* __restrict__ out) {
  __shared__ double s_sum[256];
  __shared__ double s_cnt[256];
  double sum = 0.0, cnt = 0.0;
  for (int r = threadIdx.x; r < ny * nz; r += blockDim.x) {
    const uint32_t idx = (uint32_t)px + (uint32_t)nx * (uint32_t)r;
    if (!(link[idx] & LINK_FLUID)) continue;
    double drho = 0.0, jx = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double v = f[(uint32_t)i * PS + idx];
      drho += v;
      jx += V::cx[i] * v;
    }
    sum += jx / (1.0 + drho) + 0.5 * gx;
    cnt += 1.0;
  }
  s_sum[threadIdx.x] = sum;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_cnt[0] > 0 ? s_sum[0] / s_cnt[0] : 0.0;
    out[1] = s_cnt[0];
  }
}

// lambda^T on the objective plane: d(mean u_x)/df_i = (c_ix/rho - j_x/rho^2)/n.
__global__ void porous_lambda_final_kernel(const float* __restrict__ f,
                                           const uint32_t* __restrict__ link,
                                           float* __restrict__ lam, int px, int nx, int ny,
                                           int nz, uint32_t PS, const double* __restrict__ obj) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ny * nz) return;
  const uint32_t idx = (uint32_t)px + (uint32_t)nx * (uint32_t)r;
  if (!(link[idx] & LINK_FLUID)) return;
  const float n = (float)obj[1];
  float drho = 0.f, jx = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float v = f[(uint32_t)i * PS + idx];
    drho += v;
    jx += (float)V::cx[i] * v;
  }
  const float rho = 1.f + drho;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    lam[(uint32_t)i * PS + idx] = ((float)V::cx[i] / rho - jx / (rho * rho)) / n;
}

unsigned grid_for(size_t n, unsigned threads = 256) {
  return (unsigned)std::max<size_t>(1, (n + threads - 1) / threads);
}

}  // namespace

struct lbm_porous {
  int nx = 0, ny = 0, nz = 0;
  size_t N = 0, PS = 0;
  int steps = 0, every = 0, plane_x = 0;
  double tau = 0.0;
  PorousParams p{};
  unsigned char* work = nullptr;
  PorousLayout lay;
  hipStream_t stream = nullptr;
  int device = 0;
  bool have_forward = false;
  int final_buf = 0;  // 0: fa, 1: fb holds f^T
  long long generation = 0;  // forward runs completed
  double J = 0.0;
  std::string err;
};

namespace {

lbm_status pfail(lbm_porous* h, lbm_status st, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    lbm_detail::fail(nullptr, st, msg);
  return st;
}

#define PHIP_TRY(h, call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return pfail((h), LBM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

float* fptr(lbm_porous* h, size_t off) { return (float*)(h->work + off); }
// Checkpoint slot k: the state f^{k * every}.
float* ckpt_ptr(lbm_porous* h, int k) {
  return fptr(h, h->lay.ckpt + h->lay.state_bytes * (size_t)k);
}

// 128-thread blocks for both step kernels (measured: forward 7.9 -> 7.4 ms,
// backward 20.3 -> 19.8 ms per gradient at 128x64x64 against 256 threads; the
// 40 MB states sit in the last-level cache, and occupancy caps only slowed them)
constexpr unsigned POROUS_THREADS = 128;

void launch_step(lbm_porous* h, const float* src, float* dst) {
  const uint32_t* link = (const uint32_t*)(h->work + h->lay.link);
  const float* por = fptr(h, h->lay.por);
  hipLaunchKernelGGL(porous_step_kernel, dim3(grid_for(h->N, POROUS_THREADS)),
                     dim3(POROUS_THREADS), 0, h->stream, src, dst, por, link, h->nx, h->ny,
                     h->nz, (uint32_t)h->N, (uint32_t)h->PS, h->p);
}

void launch_adjoint(lbm_porous* h, const float* f_t, const float* lam_next, float* lam_cur,
                    float* grad) {
  const uint32_t* link = (const uint32_t*)(h->work + h->lay.link);
  const float* por = fptr(h, h->lay.por);
  hipLaunchKernelGGL(porous_adjoint_kernel, dim3(grid_for(h->N, POROUS_THREADS)),
                     dim3(POROUS_THREADS), 0, h->stream, f_t, lam_next, lam_cur, grad, por, link,
                     h->nx, h->ny, h->nz, (uint32_t)h->N, (uint32_t)h->PS, h->p);
}

lbm_status check_args(int nx, int ny, int nz, int steps, int every, std::string* why) {
  if (nx <= 0 || ny <= 0 || nz <= 0) {
    *why = "lattice sizes must be positive";
    return LBM_ERR_ARG;
  }
  if (steps < 1 || every < 1 || every > steps) {
    *why = "need steps >= 1 and 1 <= checkpoint_every <= steps";
    return LBM_ERR_ARG;
  }
  if ((double)Q * pop_stride((size_t)nx * ny * nz) >= 4294967296.0) {
    *why = "q*N must stay below 2^32";
    return LBM_ERR_UNSUPPORTED;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_porous_required_bytes(int nx, int ny, int nz, int steps, int checkpoint_every,
                                     size_t* work_bytes) {
  std::string why;
  lbm_status st = check_args(nx, ny, nz, steps, checkpoint_every, &why);
  if (st) return lbm_detail::fail(nullptr, st, why);
  if (work_bytes) *work_bytes = porous_layout((size_t)nx * ny * nz, steps, checkpoint_every).total;
  return LBM_OK;
}

lbm_status lbm_porous_create(lbm_porous** out, int nx, int ny, int nz, double tau,
                             const uint8_t* material, unsigned periodic_mask, const double g[3],
                             int steps, int checkpoint_every, int plane_x, void* dev_work,
                             size_t work_bytes, void* hip_stream) {
  if (!out) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  lbm_status st = check_args(nx, ny, nz, steps, checkpoint_every, &why);
  if (st) return lbm_detail::fail(nullptr, st, why);
  if (!(std::isfinite(tau) && tau > 0.5)) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "tau must be > 0.5");
  if (!material || !g || !dev_work) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "NULL argument");
  if (plane_x < 0 || plane_x >= nx) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "plane_x out of range");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g[a])) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "g must be finite");
  const size_t N = (size_t)nx * ny * nz;
  const PorousLayout L = porous_layout(N, steps, checkpoint_every);
  if (work_bytes < L.total) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "work buffer too small");
  if ((uintptr_t)dev_work & 255u) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "work buffer must be 256-byte aligned");
  for (size_t i = 0; i < N; ++i)
    if (material[i] == 3) return lbm_detail::fail(nullptr, LBM_ERR_UNSUPPORTED, "moving walls are not supported with porosity");
  // geometry rule and link words: the same check as lbm_set_geometry
  st = lbm_validate_geometry(LBM_D3Q19, nx, ny, nz, material, periodic_mask);
  if (st) return st;
  std::vector<uint32_t> link(N, 0u);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t idx = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
        if (material[idx] != 1) continue;
        uint32_t w = LINK_FLUID;
        for (int i = 1; i < Q; ++i) {
          const int xn = (x + V::cx[i] + nx) % nx, yn = (y + V::cy[i] + ny) % ny,
                    zn = (z + V::cz[i] + nz) % nz;
          if (material[(size_t)xn + (size_t)nx * ((size_t)yn + (size_t)ny * zn)] != 1)
            w |= 1u << (i - 1);
        }
        link[idx] = w;
      }
  lbm_porous* h = new (std::nothrow) lbm_porous();
  if (!h) return lbm_detail::fail(nullptr, LBM_ERR_ARG, "out of host memory");
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->N = N;
  h->PS = pop_stride(N);
  h->steps = steps;
  h->every = checkpoint_every;
  h->plane_x = plane_x;
  h->tau = tau;
  h->p.omega = (float)(1.0 / tau);
  for (int a = 0; a < 3; ++a) h->p.g[a] = (float)g[a];
  h->work = (unsigned char*)dev_work;
  h->lay = L;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipMemcpyAsync(h->work + L.link, link.data(), sizeof(uint32_t) * N, hipMemcpyHostToDevice,
                     h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return lbm_detail::fail(nullptr, LBM_ERR_HIP, "uploading the geometry failed");
  }
  *out = h;
  return LBM_OK;
}

lbm_status lbm_porous_forward(lbm_porous* h, const float* porosity_dev, double* J) {
  if (!h) return LBM_ERR_ARG;
  h->err.clear();
  if (!porosity_dev || !J) return pfail(h, LBM_ERR_ARG, "NULL argument");
  PHIP_TRY(h, hipSetDevice(h->device));
  // the checkpoints of an earlier run are overwritten from here on
  h->have_forward = false;
  PHIP_TRY(h, hipMemcpyAsync(h->work + h->lay.por, porosity_dev, sizeof(float) * h->N,
                             hipMemcpyDeviceToDevice, h->stream));
  // f^t lives in checkpoint slot t / every when every divides t, else in
  // fa / fb by the parity of t: each step writes its result where it is kept,
  // with no copies (f^steps, never a checkpoint, ends in fa / fb)
  float* bufs[2] = {fptr(h, h->lay.fa), fptr(h, h->lay.fb)};
  auto state = [&](int t) {
    return t % h->every == 0 && t < h->steps ? ckpt_ptr(h, t / h->every) : bufs[t & 1];
  };
  hipLaunchKernelGGL(porous_init_kernel, dim3(grid_for(h->N)), dim3(256), 0, h->stream, state(0),
                     (uint32_t)h->N, (uint32_t)h->PS);
  for (int t = 0; t < h->steps; ++t) launch_step(h, state(t), state(t + 1));
  const int cur = h->steps & 1;
  double* red = (double*)(h->work + h->lay.red);
  hipLaunchKernelGGL(porous_objective_kernel, dim3(1), dim3(256), 0, h->stream, bufs[cur],
                     (const uint32_t*)(h->work + h->lay.link), h->plane_x, h->nx, h->ny, h->nz,
                     (uint32_t)h->PS, h->p.g[0], red);
  PHIP_TRY(h, hipGetLastError());
  double r[2];
  PHIP_TRY(h, hipMemcpyAsync(r, red, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  PHIP_TRY(h, hipStreamSynchronize(h->stream));
  h->final_buf = cur;
  h->have_forward = true;
  ++h->generation;
  h->J = r[0];
  *J = r[0];
  if (!std::isfinite(r[0])) return pfail(h, LBM_ERR_NONFINITE, "non-finite objective");
  return LBM_OK;
}

lbm_status lbm_porous_backward(lbm_porous* h, float* grad_dev) {
  if (!h) return LBM_ERR_ARG;
  h->err.clear();
  if (!grad_dev) return pfail(h, LBM_ERR_ARG, "grad_dev is NULL");
  if (!h->have_forward) return pfail(h, LBM_ERR_STATE, "run lbm_porous_forward first");
  PHIP_TRY(h, hipSetDevice(h->device));
  const uint32_t* link = (const uint32_t*)(h->work + h->lay.link);
  const float* fT = fptr(h, h->final_buf ? h->lay.fb : h->lay.fa);
  float* lam[2] = {fptr(h, h->lay.la), fptr(h, h->lay.lb)};
  const size_t nstate = h->lay.state_bytes / sizeof(float);
  hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, h->stream, lam[0], nstate, 0.f);
  hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, h->stream, grad_dev, h->N, 0.f);
  hipLaunchKernelGGL(porous_lambda_final_kernel, dim3(grid_for((size_t)h->ny * h->nz)), dim3(256),
                     0, h->stream, fT, link, lam[0], h->plane_x, h->nx, h->ny, h->nz,
                     (uint32_t)h->PS, (const double*)(h->work + h->lay.red));
  int cur = 0;  // lam[cur] holds lambda^{t+1}
  for (int k = h->lay.nckpt - 1; k >= 0; --k) {
    const int t0 = k * h->every;
    const int t1 = std::min(t0 + h->every, h->steps);
    // the segment's states: f^{t0} in its checkpoint, f^{t0+1} .. f^{t1-1}
    // recomputed into the segment buffer (slot t - t0; slot 0 is not used)
    float* ck = ckpt_ptr(h, k);
    float* seg = fptr(h, h->lay.seg);
    auto state = [&](int t) { return t == t0 ? ck : seg + nstate * (size_t)(t - t0); };
    for (int t = t0 + 1; t < t1; ++t) launch_step(h, state(t - 1), state(t));
    for (int t = t1 - 1; t >= t0; --t) {
      launch_adjoint(h, state(t), lam[cur], lam[cur ^ 1], grad_dev);
      cur ^= 1;
    }
  }
  PHIP_TRY(h, hipGetLastError());
  PHIP_TRY(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

lbm_status lbm_porous_get_final(lbm_porous* h, double* f_dev) {
  if (!h) return LBM_ERR_ARG;
  if (!f_dev) return pfail(h, LBM_ERR_ARG, "f_dev is NULL");
  if (!h->have_forward) return pfail(h, LBM_ERR_STATE, "run lbm_porous_forward first");
  PHIP_TRY(h, hipSetDevice(h->device));
  // natural layout, FP64, dense stride N
  std::vector<float> host(h->lay.state_bytes / sizeof(float));
  PHIP_TRY(h, hipMemcpyAsync(host.data(), h->work + (h->final_buf ? h->lay.fb : h->lay.fa),
                             h->lay.state_bytes, hipMemcpyDeviceToHost, h->stream));
  PHIP_TRY(h, hipStreamSynchronize(h->stream));
  std::vector<double> dense((size_t)Q * h->N);
  std::vector<uint32_t> link(h->N);
  PHIP_TRY(h, hipMemcpyAsync(link.data(), h->work + h->lay.link, sizeof(uint32_t) * h->N,
                             hipMemcpyDeviceToHost, h->stream));
  PHIP_TRY(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < Q; ++i)
    for (size_t idx = 0; idx < h->N; ++idx)
      dense[(size_t)i * h->N + idx] =
          (link[idx] & LINK_FLUID) ? (double)host[(size_t)i * h->PS + idx] + Vel<Q>::w36[i] / 36.0 : 0.0;
  PHIP_TRY(h, hipMemcpyAsync(f_dev, dense.data(), sizeof(double) * dense.size(),
                             hipMemcpyHostToDevice, h->stream));
  PHIP_TRY(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

lbm_status lbm_porous_generation(const lbm_porous* h, long long* generation) {
  if (!h || !generation) return LBM_ERR_ARG;
  *generation = h->generation;
  return LBM_OK;
}

lbm_status lbm_porous_destroy(lbm_porous* h) {
  if (!h) return LBM_ERR_ARG;
  hipError_t e = hipSetDevice(h->device);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  delete h;
  return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

const char* lbm_porous_last_error(const lbm_porous* h) { return h ? h->err.c_str() : ""; }

}  // extern "C"
