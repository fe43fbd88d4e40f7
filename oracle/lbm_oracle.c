/*
 * lbm_oracle.c -- FP64 CPU oracle for the fused BGK collide-and-stream step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header or table
 * with the HIP path: its descriptor tables are written out here on their own.
 *
 * Source: "OpenLB User Guide, release 1.6" (arXiv:2307.11752).  Every routine
 * names the passage it follows.  Where the guide is silent the reading used is
 * stated next to the code (readings R1..R10 in the header comment of each
 * routine).  The implementation is deliberately plain: a two-lattice push
 * (read lattice A, collide, push every post-collision population to its
 * destination in lattice B), all arithmetic in IEEE double, no blocking, no
 * fusion beyond what the guide's collide-then-stream order states.  Build with
 * -O2 -ffp-contract=off and without -ffast-math so every operation is a single
 * correctly rounded double operation in the order written.
 *
 * Layout of every population array: structure of arrays, f[i*N + idx] with
 * idx = x + nx*(y + ny*z) (x fastest), N = nx*ny*nz.  Velocity fields are
 * u[a*N + idx] for a = 0,1,2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Descriptors.
 *
 * D2Q9 is the guide's own listing "Definition of the D2Q9 descriptor" (Core
 * Concepts, section "Descriptor"): velocity table, opposite table, weights
 * {4/9, 1/36, 1/9, ...} and c_s^2 = 1/3, copied entry by entry.
 *
 * D3Q19 is only drawn in the guide (Introduction, figure of discrete velocity
 * sets), never tabulated.  Reading R1: the standard D3Q19 set -- one rest
 * velocity (weight 1/3), the six face neighbours (1/18) and the twelve edge
 * neighbours (1/36), c_s^2 = 1/3.  The ordering follows the convention of the
 * D2Q9 listing: entries 1..9 are one half of the moving velocities and entry
 * i+9 is the opposite of entry i, so opposite(i) = i +/- 9.
 * ------------------------------------------------------------------------- */
enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };

static const int C9[9][3] = {
    {0, 0, 0},
    {-1, 1, 0}, {-1, 0, 0}, {-1, -1, 0}, {0, -1, 0},
    {1, -1, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}};
static const int OPP9[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
static const double W9[9] = {4.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0};

static const int C19[19][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
    {-1, -1, 0}, {-1, 1, 0}, {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
static const int OPP19[19] = {0,  10, 11, 12, 13, 14, 15, 16, 17, 18,
                              1,  2,  3,  4,  5,  6,  7,  8,  9};
static const double W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const double CS2 = 1.0 / 3.0;

typedef struct {
  int q;
  int dim;
  const int (*c)[3];
  const int *opp;
  const double *w;
} desc_t;

static int get_desc(int d, desc_t *out) {
  if (d == ORC_D2Q9) {
    out->q = 9; out->dim = 2; out->c = C9; out->opp = OPP9; out->w = W9;
    return 0;
  }
  if (d == ORC_D3Q19) {
    out->q = 19; out->dim = 3; out->c = C19; out->opp = OPP19; out->w = W19;
    return 0;
  }
  return -1;
}

/* Status codes (negative = error), mirrored in the Python loader. */
#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_GEOMETRY (-2)
#define ORC_ERR_UNSUPPORTED (-3)

/* Material numbers (Geometry chapter, "Setting Material Numbers", figure
 * caption): 0 = no dynamics, 1 = fluid, 2 = no-slip (bounce-back) boundary,
 * 3 = velocity boundary.  Reading R2: material 3 is realised as the guide's
 * BounceBackVelocity dynamics (Initial and Boundary Conditions, "Additional
 * Options"), i.e. a bounce-back wall that moves with the prescribed velocity.
 * 4 (pressure) and 5 (curved) are not part of this path. */
#define MAT_NONE 0
#define MAT_FLUID 1
#define MAT_WALL 2
#define MAT_MOVING 3

int orc_descriptor(int d, int *q, int *dim, int *c_out, double *w_out,
                   int *opp_out, double *cs2_out) {
  desc_t D;
  if (get_desc(d, &D)) return ORC_ERR_ARG;
  if (q) *q = D.q;
  if (dim) *dim = D.dim;
  for (int i = 0; i < D.q; ++i) {
    if (c_out) for (int a = 0; a < 3; ++a) c_out[3 * i + a] = D.c[i][a];
    if (w_out) w_out[i] = D.w[i];
    if (opp_out) opp_out[i] = D.opp[i];
  }
  if (cs2_out) *cs2_out = CS2;
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Second-order equilibrium (Core Concepts, "Dynamics": equilibria::SecondOrder
 * approximating the Maxwell-Boltzmann distribution, Introduction section 1.1).
 * The guide names it but does not print it.  Reading R3: the second-order
 * Hermite expansion
 *   feq_i = w_i rho [1 + (c_i.u)/cs2 + (c_i.u)^2/(2 cs2^2) - (u.u)/(2 cs2)].
 * ------------------------------------------------------------------------- */
void orc_equilibrium(int d, double rho, const double *u, double *feq) {
  desc_t D;
  if (get_desc(d, &D)) return;
  double uu = 0.0;
  for (int a = 0; a < D.dim; ++a) uu += u[a] * u[a];
  for (int i = 0; i < D.q; ++i) {
    double cu = 0.0;
    for (int a = 0; a < D.dim; ++a) cu += D.c[i][a] * u[a];
    feq[i] = D.w[i] * rho *
             (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* ---------------------------------------------------------------------------
 * Guo source term (Simulation Models, "Coupling Between Momentum and Energy
 * Equations", equation for the force-corrected population):
 *   S_i = (1 - omega/2) w_i [ (c_i - u)/cs2 + (c_i.u) c_i / cs2^2 ] . F
 * with omega = 1/tau and u the force-shifted velocity.  Reading R4: the
 * FORCE field holds an acceleration g (the velocity shift adds FORCE/2 to u,
 * and the constant-force example drives Poiseuille flow with an acceleration),
 * so the momentum source F entering S_i is the force density rho*g.
 * ------------------------------------------------------------------------- */
void orc_guo_source(int d, double omega, double rho, const double *u,
                    const double *g, double *S) {
  desc_t D;
  if (get_desc(d, &D)) return;
  double F[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D.dim; ++a) F[a] = rho * g[a];
  for (int i = 0; i < D.q; ++i) {
    double cu = 0.0;
    for (int a = 0; a < D.dim; ++a) cu += D.c[i][a] * u[a];
    double s = 0.0;
    for (int a = 0; a < D.dim; ++a)
      s += ((D.c[i][a] - u[a]) / CS2 + cu * D.c[i][a] / (CS2 * CS2)) * F[a];
    S[i] = (1.0 - omega / 2.0) * D.w[i] * s;
  }
}

/* ---------------------------------------------------------------------------
 * Cell moments (momenta::BulkTuple: rho = sum_i f_i, j = sum_i c_i f_i) and the
 * Guo velocity shift u = j/rho + g/2 (Simulation Models, "Coupling Between
 * Momentum and Energy Equations", velocity-shift equation and listing).
 * Reading R5: this shifted velocity is also the velocity the path reports.
 * ------------------------------------------------------------------------- */
void orc_cell_moments(int d, const double *f, const double *g, double *rho_out,
                      double *u_out) {
  desc_t D;
  if (get_desc(d, &D)) return;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < D.q; ++i) {
    rho += f[i];
    for (int a = 0; a < D.dim; ++a) j[a] += D.c[i][a] * f[i];
  }
  *rho_out = rho;
  for (int a = 0; a < 3; ++a) u_out[a] = 0.0;
  for (int a = 0; a < D.dim; ++a) u_out[a] = j[a] / rho + g[a] / 2.0;
}

/* ---------------------------------------------------------------------------
 * BGK collision of one cell, in place (Introduction section 1.1, collision
 * equation with the BGK operator; Core Concepts, BGK collision listing:
 * f_i <- (1 - omega) f_i + omega feq_i), followed by the Guo source (forcing::Guo
 * combination rule, Core Concepts "Dynamics").  g = 0 gives plain BGK.
 * ------------------------------------------------------------------------- */
void orc_collide(int d, double omega, const double *g, double *f,
                 double *rho_out, double *u_out) {
  desc_t D;
  if (get_desc(d, &D)) return;
  double rho, u[3], feq[19], S[19];
  orc_cell_moments(d, f, g, &rho, u);
  orc_equilibrium(d, rho, u, feq);
  orc_guo_source(d, omega, rho, u, g, S);
  for (int i = 0; i < D.q; ++i) {
    f[i] = (1.0 - omega) * f[i];
    f[i] = f[i] + omega * feq[i];
    f[i] = f[i] + S[i];
  }
  if (rho_out) *rho_out = rho;
  if (u_out) for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

/* ---------------------------------------------------------------------------
 * Geometry check.  Mirrors the guide's geometry statistics check that the
 * material layout is consistent (Input and Output, "Console Output"): a fluid
 * cell must see, along every lattice velocity, either another fluid cell or a
 * bounce-back wall (2 or 3); a neighbour of material 0, or a neighbour outside
 * the box along a non-periodic axis, is an error.  Materials above 3 are not
 * supported on this path.
 * ------------------------------------------------------------------------- */
static int wrap_coord(int v, int n, int periodic, int *ok) {
  if (v >= 0 && v < n) return v;
  if (!periodic) { *ok = 0; return 0; }
  return ((v % n) + n) % n;
}

int orc_check_geometry(int d, int nx, int ny, int nz, const uint8_t *mat,
                       unsigned periodic) {
  desc_t D;
  if (get_desc(d, &D) || nx <= 0 || ny <= 0 || nz <= 0 || !mat) return ORC_ERR_ARG;
  if (d == ORC_D2Q9 && nz != 1) return ORC_ERR_ARG;
  long N = (long)nx * ny * nz;
  for (long idx = 0; idx < N; ++idx)
    if (mat[idx] > MAT_MOVING) return ORC_ERR_UNSUPPORTED;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long idx = x + (long)nx * (y + (long)ny * z);
        if (mat[idx] != MAT_FLUID) continue;
        for (int i = 1; i < D.q; ++i) {
          int ok = 1;
          int xn = wrap_coord(x + D.c[i][0], nx, periodic & 1u, &ok);
          int yn = wrap_coord(y + D.c[i][1], ny, periodic & 2u, &ok);
          int zn = wrap_coord(z + D.c[i][2], nz, periodic & 4u, &ok);
          if (!ok) return ORC_ERR_GEOMETRY;
          if (mat[xn + (long)nx * (yn + (long)ny * zn)] == MAT_NONE)
            return ORC_ERR_GEOMETRY;
        }
      }
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Equilibrium initialisation (Initial and Boundary Conditions, "Define
 * Initial Conditions": define rho and u, then set the populations to the
 * local equilibrium).  rho == NULL means rho = 1, u == NULL means u = 0.
 * Non-fluid cells are set to zero (they carry no populations).
 * ------------------------------------------------------------------------- */
int orc_init_equilibrium(int d, int nx, int ny, int nz, const uint8_t *mat,
                         const double *rho, const double *u, double *f) {
  desc_t D;
  if (get_desc(d, &D) || !f || !mat) return ORC_ERR_ARG;
  long N = (long)nx * ny * nz;
  for (long idx = 0; idx < N; ++idx) {
    double feq[19], uc[3] = {0.0, 0.0, 0.0};
    double r = rho ? rho[idx] : 1.0;
    if (u) for (int a = 0; a < D.dim; ++a) uc[a] = u[a * N + idx];
    if (mat[idx] == MAT_FLUID) {
      orc_equilibrium(d, r, uc, feq);
      for (int i = 0; i < D.q; ++i) f[i * N + idx] = feq[i];
    } else {
      for (int i = 0; i < D.q; ++i) f[i * N + idx] = 0.0;
    }
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * One time step: collide every fluid cell of A, then push each post-collision
 * population along its velocity into B (Introduction section 1.1, streaming
 * equation f_i(t+1, x+c_i) = f*_i(t, x)).
 *
 * Boundaries, for a fluid cell x and destination y = x + c_i (wrapped on
 * periodic axes):
 *   mat(y) == 1: B_i(y) = f*_i(x)                               (streaming)
 *   mat(y) == 2: B_opp(i)(x) = f*_i(x)                          (bounce-back)
 *   mat(y) == 3: B_opp(i)(x) = f*_i(x) - 2 w_i rho(x) (c_i.u_w)/cs2
 * Reading R6: bounce-back is the halfway, link-wise rule (the wall lies half
 * way between x and y); the guide states the BounceBack dynamics only as a
 * "zero velocity" wall.  Reading R7: the moving wall (BounceBackVelocity,
 * "prescribes a nonzero velocity") uses the momentum correction
 * -2 w_i rho (c_i.u_w)/cs2 with rho the density of the fluid cell at time t.
 *
 * Non-fluid cells of B are copied from A unchanged.  omega = 1/tau; omega = 0
 * (with g = 0, u_w = 0) is pure streaming.
 * ------------------------------------------------------------------------- */
int orc_step(int d, int nx, int ny, int nz, const uint8_t *mat,
             unsigned periodic, double omega, const double *g,
             const double *uw, const double *A, double *B, int nthreads) {
  desc_t D;
  if (get_desc(d, &D) || !mat || !A || !B || !g || !uw) return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  const int q = D.q;
#ifdef _OPENMP
  /* the thread count applies to this call only */
  const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
#endif
  /* Non-fluid cells keep their (meaningless) contents. */
  for (long idx = 0; idx < N; ++idx)
    if (mat[idx] != MAT_FLUID)
      for (int i = 0; i < q; ++i) B[i * N + idx] = A[i * N + idx];

  /* Each destination slot of B is written by exactly one fluid cell, so
   * z-planes can be processed independently. */
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        const long idx = x + (long)nx * (y + (long)ny * z);
        if (mat[idx] != MAT_FLUID) continue;
        double f[19], rho, u[3];
        for (int i = 0; i < q; ++i) f[i] = A[i * N + idx];
        orc_collide(d, omega, g, f, &rho, u);
        for (int i = 0; i < q; ++i) {
          int ok = 1;
          const int xn = wrap_coord(x + D.c[i][0], nx, periodic & 1u, &ok);
          const int yn = wrap_coord(y + D.c[i][1], ny, periodic & 2u, &ok);
          const int zn = wrap_coord(z + D.c[i][2], nz, periodic & 4u, &ok);
          const long nb = xn + (long)nx * (yn + (long)ny * zn);
          const int m = ok ? mat[nb] : MAT_NONE;
          if (m == MAT_FLUID) {
            B[i * N + nb] = f[i];
          } else if (m == MAT_WALL) {
            B[D.opp[i] * N + idx] = f[i];
          } else if (m == MAT_MOVING) {
            double cu = 0.0;
            for (int a = 0; a < D.dim; ++a) cu += D.c[i][a] * uw[a];
            B[D.opp[i] * N + idx] = f[i] - 2.0 * D.w[i] * rho * cu / CS2;
          }
          /* m == MAT_NONE next to fluid is rejected by orc_check_geometry. */
        }
      }
    }
  }
  return ORC_OK;
}

/* n steps, ping-ponging between f and work; the result ends in f. */
int orc_run(int d, int nx, int ny, int nz, const uint8_t *mat, unsigned periodic,
            double omega, const double *g, const double *uw, int nsteps,
            double *f, double *work, int nthreads) {
  desc_t D;
  if (get_desc(d, &D) || nsteps < 0) return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  double *a = f, *b = work;
  for (int s = 0; s < nsteps; ++s) {
    int st = orc_step(d, nx, ny, nz, mat, periodic, omega, g, uw, a, b, nthreads);
    if (st) return st;
    double *t = a; a = b; b = t;
  }
  if (a != f) memcpy(f, a, sizeof(double) * (size_t)D.q * (size_t)N);
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Macroscopic fields of every fluid cell (rho and the shifted u of
 * orc_cell_moments); non-fluid cells report rho = 0, u = 0.
 * ------------------------------------------------------------------------- */
int orc_moments(int d, int nx, int ny, int nz, const uint8_t *mat,
                const double *g, const double *f, double *rho, double *u) {
  desc_t D;
  if (get_desc(d, &D) || !mat || !f) return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  for (long idx = 0; idx < N; ++idx) {
    double fc[19], r = 0.0, uc[3] = {0.0, 0.0, 0.0};
    if (mat[idx] == MAT_FLUID) {
      for (int i = 0; i < D.q; ++i) fc[i] = f[i * N + idx];
      orc_cell_moments(d, fc, g, &r, uc);
    }
    if (rho) rho[idx] = r;
    if (u) for (int a = 0; a < 3; ++a) u[a * N + idx] = uc[a];
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Global totals over fluid cells, summed sequentially in cell order:
 * mass M = sum rho, momentum J = sum_i c_i f_i (unshifted, so that in a fully
 * periodic box with body force J(t+1) = J(t) + M g holds exactly in exact
 * arithmetic).  Also the lattice statistics of the guide's "Extract Data From
 * a Simulation" lesson: average density, average energy (half the average of
 * |u|^2 over fluid cells) and maximum |u|, with the shifted velocity.
 * ------------------------------------------------------------------------- */
int orc_totals(int d, int nx, int ny, int nz, const uint8_t *mat,
               const double *g, const double *f, double *mass, double *mom,
               double *stats /* avRho, avEnergy, maxU */) {
  desc_t D;
  if (get_desc(d, &D) || !mat || !f) return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  double M = 0.0, J[3] = {0.0, 0.0, 0.0}, e = 0.0, umax = 0.0;
  long nfluid = 0;
  for (long idx = 0; idx < N; ++idx) {
    if (mat[idx] != MAT_FLUID) continue;
    double fc[19], r, u[3];
    for (int i = 0; i < D.q; ++i) {
      fc[i] = f[i * N + idx];
      for (int a = 0; a < D.dim; ++a) J[a] += D.c[i][a] * fc[i];
    }
    orc_cell_moments(d, fc, g, &r, u);
    M += r;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    e += uu;
    if (sqrt(uu) > umax) umax = sqrt(uu);
    ++nfluid;
  }
  if (mass) *mass = M;
  if (mom) for (int a = 0; a < 3; ++a) mom[a] = J[a];
  if (stats) {
    stats[0] = nfluid ? M / nfluid : 0.0;
    stats[1] = nfluid ? 0.5 * e / nfluid : 0.0;
    stats[2] = umax;
  }
  return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ===========================================================================
 * Porous BGK and its discrete adjoint.
 *
 * Porous media model (Simulation Models, "Porous Media Model"): each cell
 * carries a porosity d in [0, 1] (0 solid, 1 fluid), a factor that scales the
 * velocity of the Maxwellian (the guide's latticePorosity comment).  Reading
 * R15: the equilibrium and the Guo term both use v = d u with the
 * force-shifted u = j/rho + g/2; d = 1 is exactly the plain collision above.
 * Only resting walls (material 2) are allowed with porosity.
 * ========================================================================= */
void orc_porous_collide(int d, double omega, const double *g, double por, double *f,
                        double *rho_out, double *u_out) {
  desc_t D;
  if (get_desc(d, &D)) return;
  double rho, u[3], v[3] = {0.0, 0.0, 0.0}, feq[19], S[19];
  orc_cell_moments(d, f, g, &rho, u);
  for (int a = 0; a < D.dim; ++a) v[a] = por * u[a];
  orc_equilibrium(d, rho, v, feq);
  orc_guo_source(d, omega, rho, v, g, S);
  for (int i = 0; i < D.q; ++i) {
    f[i] = (1.0 - omega) * f[i];
    f[i] = f[i] + omega * feq[i];
    f[i] = f[i] + S[i];
  }
  if (rho_out) *rho_out = rho;
  if (u_out) for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

int orc_porous_step(int d, int nx, int ny, int nz, const uint8_t *mat, unsigned periodic,
                    double omega, const double *g, const double *por, const double *A,
                    double *B, int nthreads) {
  desc_t D;
  if (get_desc(d, &D) || !mat || !A || !B || !g || !por) return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  const int q = D.q;
#ifdef _OPENMP
  /* the thread count applies to this call only */
  const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
#endif
  for (long idx = 0; idx < N; ++idx) {
    if (mat[idx] == MAT_MOVING) return ORC_ERR_UNSUPPORTED;
    if (mat[idx] != MAT_FLUID)
      for (int i = 0; i < q; ++i) B[i * N + idx] = A[i * N + idx];
  }
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long idx = x + (long)nx * (y + (long)ny * z);
        if (mat[idx] != MAT_FLUID) continue;
        double f[19];
        for (int i = 0; i < q; ++i) f[i] = A[i * N + idx];
        orc_porous_collide(d, omega, g, por[idx], f, NULL, NULL);
        for (int i = 0; i < q; ++i) {
          int ok = 1;
          const int xn = wrap_coord(x + D.c[i][0], nx, periodic & 1u, &ok);
          const int yn = wrap_coord(y + D.c[i][1], ny, periodic & 2u, &ok);
          const int zn = wrap_coord(z + D.c[i][2], nz, periodic & 4u, &ok);
          const long nb = xn + (long)nx * (yn + (long)ny * zn);
          if (ok && mat[nb] == MAT_FLUID)
            B[i * N + nb] = f[i];
          else
            B[D.opp[i] * N + idx] = f[i];
        }
      }
  return ORC_OK;
}

/* Objective: mean x-velocity (force-shifted, as reported by the moments) over
 * the fluid cells of the plane x = plane_x. */
double orc_porous_objective(int d, int nx, int ny, int nz, const uint8_t *mat,
                            const double *g, const double *f, int plane_x) {
  desc_t D;
  if (get_desc(d, &D)) return NAN;
  const long N = (long)nx * ny * nz;
  double sum = 0.0;
  long n = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      const long idx = plane_x + (long)nx * (y + (long)ny * z);
      if (mat[idx] != MAT_FLUID) continue;
      double fc[19], rho, u[3];
      for (int i = 0; i < D.q; ++i) fc[i] = f[i * N + idx];
      orc_cell_moments(d, fc, g, &rho, u);
      sum += u[0];
      ++n;
    }
  return n ? sum / n : 0.0;
}

/* Discrete adjoint of the porous step, reverse over all time steps.
 * Forward: f^{t+1} = Stream(Collide(f^t; d)), J = objective(f^T).
 * lambda^T = dJ/df^T; for t = T-1 .. 0:
 *   mu = Stream^T lambda^{t+1}   (pull: mu_i(x) = lambda_i(x + c_i), or
 *                                  lambda_opp(i)(x) across a wall)
 *   lambda^t = (dCollide/df)^T mu,  dJ/dd += (dCollide/dd)^T mu,
 * both at the state f^t.  With v = d u, u = j/rho + g/2:
 *   dfeq_i/dv_a = w_i rho (3 c_ia + 9 (c_i.v) c_ia - 3 v_a)
 *   dS_i/dv_a   = (1 - omega/2) w_i (-3 F_a + 9 c_ia (c_i.F)),  F = rho g
 *   dfeq_i/drho|v = feq_i / rho,  dS_i/drho|v = S_i / rho
 *   dv_a/drho = -d j_a / rho^2,  dv_a/dj_b = d delta_ab / rho,  dv_a/dd = u_a
 * All states f^0 .. f^T are kept (no checkpointing).  J and grad[N] are
 * outputs; grad is zero on non-fluid cells. */
int orc_porous_gradient(int d, int nx, int ny, int nz, const uint8_t *mat, unsigned periodic,
                        double omega, const double *g, const double *por, int nsteps,
                        const double *f0, int plane_x, double *J, double *grad, int nthreads) {
  desc_t D;
  if (get_desc(d, &D) || nsteps < 0 || !f0 || !grad || !J || plane_x < 0 || plane_x >= nx)
    return ORC_ERR_ARG;
  const long N = (long)nx * ny * nz;
  const int q = D.q;
  const size_t state = (size_t)q * (size_t)N;
  double *hist = (double *)malloc(sizeof(double) * state * (size_t)(nsteps + 1));
  double *lam = (double *)calloc(state, sizeof(double));
  double *lam_prev = (double *)calloc(state, sizeof(double));
  if (!hist || !lam || !lam_prev) {
    free(hist); free(lam); free(lam_prev);
    return ORC_ERR_ARG;
  }
  memcpy(hist, f0, sizeof(double) * state);
  for (int t = 0; t < nsteps; ++t) {
    int st = orc_porous_step(d, nx, ny, nz, mat, periodic, omega, g, por, hist + state * t,
                             hist + state * (t + 1), nthreads);
    if (st) {
      free(hist); free(lam); free(lam_prev);
      return st;
    }
  }
  const double *fT = hist + state * (size_t)nsteps;
  *J = orc_porous_objective(d, nx, ny, nz, mat, g, fT, plane_x);

  /* lambda^T: derivative of the plane mean of u_x = j_x/rho + g_x/2 */
  long nplane = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      if (mat[plane_x + (long)nx * (y + (long)ny * z)] == MAT_FLUID) ++nplane;
  for (int z = 0; z < nz && nplane; ++z)
    for (int y = 0; y < ny; ++y) {
      const long idx = plane_x + (long)nx * (y + (long)ny * z);
      if (mat[idx] != MAT_FLUID) continue;
      double rho = 0.0, jx = 0.0;
      for (int i = 0; i < q; ++i) {
        rho += fT[i * N + idx];
        jx += D.c[i][0] * fT[i * N + idx];
      }
      for (int i = 0; i < q; ++i)
        lam[i * N + idx] = (D.c[i][0] / rho - jx / (rho * rho)) / (double)nplane;
    }
  for (long idx = 0; idx < N; ++idx) grad[idx] = 0.0;
  const double k = 1.0 - omega / 2.0;

  for (int t = nsteps - 1; t >= 0; --t) {
    const double *ft = hist + state * (size_t)t;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const long idx = x + (long)nx * (y + (long)ny * z);
          if (mat[idx] != MAT_FLUID) {
            for (int i = 0; i < q; ++i) lam_prev[i * N + idx] = 0.0;
            continue;
          }
          double mu[19], fc[19], feq[19], S[19];
          for (int i = 0; i < q; ++i) {
            int ok = 1;
            const int xn = wrap_coord(x + D.c[i][0], nx, periodic & 1u, &ok);
            const int yn = wrap_coord(y + D.c[i][1], ny, periodic & 2u, &ok);
            const int zn = wrap_coord(z + D.c[i][2], nz, periodic & 4u, &ok);
            const long nb = xn + (long)nx * (yn + (long)ny * zn);
            if (ok && mat[nb] == MAT_FLUID)
              mu[i] = lam[i * N + nb];
            else
              mu[i] = lam[D.opp[i] * N + idx];
            fc[i] = ft[i * N + idx];
          }
          double rho, u[3], v[3] = {0.0, 0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
          orc_cell_moments(d, fc, g, &rho, u);
          for (int i = 0; i < q; ++i)
            for (int a = 0; a < D.dim; ++a) j[a] += D.c[i][a] * fc[i];
          const double dp = por[idx];
          for (int a = 0; a < D.dim; ++a) v[a] = dp * u[a];
          orc_equilibrium(d, rho, v, feq);
          orc_guo_source(d, omega, rho, v, g, S);
          double F[3] = {0.0, 0.0, 0.0};
          for (int a = 0; a < D.dim; ++a) F[a] = rho * g[a];
          double G[3] = {0.0, 0.0, 0.0}, E = 0.0;
          for (int i = 0; i < q; ++i) {
            double cv = 0.0, cF = 0.0;
            for (int a = 0; a < D.dim; ++a) {
              cv += D.c[i][a] * v[a];
              cF += D.c[i][a] * F[a];
            }
            for (int a = 0; a < D.dim; ++a) {
              const double dfeq = D.w[i] * rho * (3.0 * D.c[i][a] + 9.0 * cv * D.c[i][a] - 3.0 * v[a]);
              const double dS = k * D.w[i] * (-3.0 * F[a] + 9.0 * D.c[i][a] * cF);
              G[a] += mu[i] * (omega * dfeq + dS);
            }
            E += mu[i] * (omega * feq[i] + S[i]) / rho;
          }
          double gsum = 0.0, Gj = 0.0;
          for (int a = 0; a < D.dim; ++a) {
            gsum += G[a] * u[a];
            Gj += G[a] * j[a];
          }
          grad[idx] += gsum;
          const double Arho = E - dp * Gj / (rho * rho);
          for (int i = 0; i < q; ++i) {
            double s = (1.0 - omega) * mu[i] + Arho;
            for (int a = 0; a < D.dim; ++a) s += dp * G[a] / rho * D.c[i][a];
            lam_prev[i * N + idx] = s;
          }
        }
    double *tmp = lam; lam = lam_prev; lam_prev = tmp;
  }
  free(hist); free(lam); free(lam_prev);
  return ORC_OK;
}
