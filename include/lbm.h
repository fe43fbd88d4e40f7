/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann hot path: fused BGK
 * collide-and-stream on D2Q9 / D3Q19 lattices with halfway bounce-back walls,
 * moving-wall bounce-back, periodic wrap and Guo body-force forcing.
 *
 * Method: OpenLB User Guide, release 1.6 (arXiv:2307.11752).
 *   - collide and stream:      Introduction, section "Lattice Boltzmann Methods"
 *                              (collision equation, BGK operator, streaming equation)
 *   - BGK collision:           Core Concepts, "Collision Operators" (BGK listing)
 *   - descriptors:             Core Concepts, "Descriptor" (D2Q9 listing; D3Q19 figure)
 *   - Guo forcing:             Simulation Models, "Coupling Between Momentum and
 *                              Energy Equations" (velocity shift and forcing equations)
 *   - material numbers:        Geometry Creation, "Setting Material Numbers"
 *   - bounce-back dynamics:    Initial and Boundary Conditions, "Additional Options"
 *   - equilibrium initialisation: Initial and Boundary Conditions,
 *                              "Define Initial Conditions"
 *   - lattice statistics:      lesson "Extract Data From a Simulation"
 * All quantities are in lattice units (dx = dt = 1, c_s^2 = 1/3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Every call returns an lbm_status (0 = LBM_OK, negative = error).  No call
 *    throws or aborts; on error the handle keeps its previous state and
 *    lbm_last_error() describes the failure.  One exception: a HIP failure
 *    inside lbm_step (lbm_batch_step, lbm_batch_autotune) may leave some of
 *    the requested steps queued, so the lattice (every member of the batch)
 *    is then marked inconsistent: stepping and reading it return
 *    LBM_ERR_STATE until lbm_init_equilibrium or lbm_set_populations is
 *    called again.  Likewise a HIP failure while a batch uploads its work
 *    tables (lbm_batch_set_launch, lbm_batch_set_phase_launch,
 *    lbm_batch_autotune) makes lbm_batch_step return LBM_ERR_STATE until a
 *    launch shape is set successfully.
 *  * Cell index idx = x + nx*(y + ny*z), x fastest; N = nx*ny*nz.  D2Q9 needs nz == 1.
 *  * Device buffers are caller-owned (e.g. PyTorch tensors) and must outlive the
 *    handle.  The library never allocates device memory.
 *  * Work is enqueued on the stream given at creation (NULL = the null stream).
 *    Calls marked "async" return before the device finishes; calls marked
 *    "sync" wait for that stream.
 *  * A handle is not thread-safe; distinct handles are independent.
 *
 * Velocity ordering (needed only to read raw population buffers): D2Q9 follows
 * the guide's listing {(0,0),(-1,1),(-1,0),(-1,-1),(0,-1),(1,-1),(1,0),(1,1),(0,1)}.
 * D3Q19 is ordered as rest, then (-1,0,0),(0,-1,0),(0,0,-1),(-1,-1,0),(-1,1,0),
 * (-1,0,-1),(-1,0,1),(0,-1,-1),(0,-1,1), then the negatives of entries 1..9 in
 * the same order, so opposite(i) = i + 9 for 1 <= i <= 9 (the D2Q9 listing's
 * convention, with 4 in place of 9).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_lattice lbm_lattice; /* opaque handle */

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 } lbm_descriptor;

/* Population storage type.  F64 storage computes in double; every other type
 * is converted to float in registers and computes in float. */
typedef enum {
  LBM_STORE_F64 = 0,
  LBM_STORE_F32 = 1,
  LBM_STORE_F16 = 2,  /* IEEE binary16 holding the value times 2^12 (so that small
                         weight-shifted values stay normal); |value| < 16 */
  LBM_STORE_BF16 = 3  /* bfloat16 */
} lbm_storage;

/* Creation flags. */
#define LBM_FLAG_SHIFTED 1u /* store f_i - w_i instead of f_i (any storage type) */

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,         /* bad argument: size, pointer, tau <= 1/2, NaN input */
  LBM_ERR_GEOMETRY = -2,    /* material layout rejected (see lbm_set_geometry) */
  LBM_ERR_UNSUPPORTED = -3, /* material 4/5/>5, lattice too large */
  LBM_ERR_HIP = -4,         /* a HIP runtime call failed; text in lbm_last_error */
  LBM_ERR_STATE = -5,       /* call order violated (e.g. step before geometry/init) */
  LBM_ERR_NONFINITE = -6    /* NaN/Inf found in a reduction */
} lbm_status;

/* Sizes of the two caller-allocated device buffers for a lattice.
 * pop_bytes: the populations in the storage type.  With s bytes per value and
 * B = 32768 / s cells per chunk, a lattice of more than B cells whose buffer
 * stays below 2^32 bytes is blocked: N is rounded up to whole chunks, and
 * population i of cell idx sits at element
 *   (idx / B) * q * B + i * B + idx % B
 * (each chunk holds its q runs of B values back to back).  Otherwise the
 * buffer holds one array per population: element i * PS + idx, with PS = N
 * rounded up to a multiple of 64.  The value stored depends on the
 * propagation phase, so read populations with lbm_get_populations.
 * aux_bytes: per-cell link masks plus device scratch (the partial sums of
 * lbm_totals and the staging of lbm_moments: 32 bytes per cell, at least
 * 64 KiB and at most 1 MiB).  Host-only; needs no GPU. */
lbm_status lbm_required_bytes(lbm_descriptor d, int nx, int ny, int nz, lbm_storage s,
                              size_t* pop_bytes, size_t* aux_bytes);

/* Create a lattice on the current HIP device.  tau is the BGK relaxation time
 * (omega = 1/tau, collision equation of the guide's introduction); it must be
 * > 1/2 (the guide requires a relaxation time greater than 0.5), or +INFINITY
 * for omega = 0 (pure streaming, used for bit-exact tests).  dev_pop/dev_aux
 * must hold at least lbm_required_bytes() and be 256-byte aligned.  hip_stream
 * is a hipStream_t (NULL = null stream).  The lattice starts with no geometry,
 * g = 0 and u_w = 0.  Host-side argument checks run before any HIP call. */
lbm_status lbm_lattice_create(lbm_lattice** out, lbm_descriptor d, int nx, int ny, int nz,
                              double tau, lbm_storage s, unsigned flags, void* dev_pop,
                              size_t pop_bytes, void* dev_aux, size_t aux_bytes,
                              void* hip_stream);

/* Host-only geometry check (no GPU needed), the same rule lbm_set_geometry
 * applies.  material: host array of N bytes, material numbers of the guide
 * (0 = no dynamics, 1 = fluid, 2 = no-slip bounce-back wall, 3 = moving
 * bounce-back wall with the lattice's wall velocity).  periodic_mask: bit 0 =
 * x, bit 1 = y, bit 2 = z.  Returns LBM_ERR_UNSUPPORTED for a material > 3,
 * LBM_ERR_GEOMETRY if a fluid cell has, along some lattice velocity, a
 * material-0 neighbour or a neighbour outside the box on a non-periodic axis. */
lbm_status lbm_validate_geometry(lbm_descriptor d, int nx, int ny, int nz,
                                 const uint8_t* material, unsigned periodic_mask);

/* Install the material layout (host array of N bytes, copied) and the
 * periodic axes; validated as lbm_validate_geometry.  sync.  Invalidates the
 * populations: call lbm_init_equilibrium or lbm_set_populations next. */
lbm_status lbm_set_geometry(lbm_lattice* h, const uint8_t* material, unsigned periodic_mask);

/* Wall velocity u_w (3 doubles, host) of every material-3 cell.  Bounce-back
 * across a link (x, x+c_i) to a moving wall returns f*_i - 2 w_i rho(x) (c_i.u_w)/c_s^2. */
lbm_status lbm_set_wall_velocity(lbm_lattice* h, const double u_w[3]);

/* Uniform body acceleration g (3 doubles, host) for Guo forcing: the
 * collision uses u = j/rho + g/2 and adds the Guo term with force density
 * rho*g.  g = 0 gives plain BGK. */
lbm_status lbm_set_body_force(lbm_lattice* h, const double g[3]);

/* Change the relaxation time (same rule as at creation). */
lbm_status lbm_set_tau(lbm_lattice* h, double tau);

/* Set every fluid cell to the second-order equilibrium of (rho, u).
 * rho_dev: device double[N] or NULL (rho = 1); u_dev: device double[3*N]
 * (component a of cell idx at a*N + idx) or NULL (u = 0).  async.  Resets the
 * step counter and the propagation phase. */
lbm_status lbm_init_equilibrium(lbm_lattice* h, const double* rho_dev, const double* u_dev);

/* Overwrite the populations from device double[q*N] (natural layout: value of
 * f_i at cell idx at i*N + idx, not shifted), rounded to the storage type.
 * async.  Resets the step counter and the propagation phase. */
lbm_status lbm_set_populations(lbm_lattice* h, const double* f_dev);

/* Decode the current populations into device double[q*N] in the natural
 * layout of lbm_set_populations (unshifted; entries of non-fluid cells are 0).
 * async. */
lbm_status lbm_get_populations(lbm_lattice* h, double* f_dev);

/* Advance n >= 0 full time steps (collide + stream), enqueued on the lattice's
 * stream.  async.  After the call the stored state is the post-streaming,
 * pre-collision population set at time t0 + n. */
lbm_status lbm_step(lbm_lattice* h, int n);

/* Replay lbm_step in captured HIP graphs of `steps` time steps (even, > 0;
 * 0 = direct launches, the default).  lbm_step(n) then launches whole graphs
 * for as many full runs of `steps` as n holds and the rest directly.  Needs a
 * non-null stream (graph capture); the graph is rebuilt after any change of
 * tau, force, wall velocity or geometry.  Results are identical to direct
 * launches (same kernels, same arguments). */
lbm_status lbm_set_graph_steps(lbm_lattice* h, int steps);

/* Macroscopic fields of the current state (the guide's lesson "Extract Data
 * From a Simulation"): density rho and the force-shifted velocity
 * u = j/rho + g/2 of the guide's Guo velocity shift, decoded and accumulated
 * in double.  Non-fluid cells report 0.
 * lbm_moments: host buffers rho double[N] and u double[3*N] (component a of
 * cell idx at a*N + idx); either may be NULL.  sync: the cells are decoded in
 * chunks through the lattice's device scratch and copied to the host.
 * lbm_moments_device: device buffers rho_dev float[N] and u_dev float[3*N]
 * (same layout, values rounded to float once at the end); either may be
 * NULL.  async. */
lbm_status lbm_moments(lbm_lattice* h, double* rho, double* u);
lbm_status lbm_moments_device(lbm_lattice* h, float* rho_dev, float* u_dev);

/* Totals over fluid cells, reduced on the device in double: mass = sum rho,
 * momentum = sum_i c_i f_i (unshifted), stats = {average rho, average energy
 * (half the mean of |u|^2), max |u|} with the shifted u (may be NULL).  Host
 * outputs; sync.  LBM_ERR_NONFINITE if any result is NaN or Inf. */
lbm_status lbm_totals(lbm_lattice* h, double* mass, double momentum[3], double stats[3]);

/* lbm_totals for callers that cannot allocate device memory, e.g. code
 * under HIP graph capture, tight serving loops or harnesses that forbid it.
 * The same reduction and outputs as lbm_totals, bitwise, but the partial sums
 * and the result live in a library-owned static device array (64 KiB + 64 B
 * per GPU, held until the process ends) instead of the lattice's aux scratch;
 * that array is enough for a lattice of any size, so no size is refused.
 * Calls no allocating routine.  Every call on one GPU uses that GPU's copy:
 * calls that overlap on one GPU (other threads, other streams) race, and the
 * array keeps the last call's contents.  sync. */
lbm_status lbm_totals_noalloc(lbm_lattice* h, double* mass, double momentum[3],
                              double stats[3]);

/* Number of steps taken since the last initialisation, and fluid cell count. */
lbm_status lbm_get_info(const lbm_lattice* h, long long* steps, long long* fluid_cells);

/* Release the handle (not the caller's buffers).  Waits for its stream.
 * Lattices owned by a batch are released with the batch. */
lbm_status lbm_lattice_destroy(lbm_lattice* h);

/* ---------------------------------------------------------------------------
 * Batched ensembles.  `count` fully fluid lattices, periodic on every axis,
 * of uneven shapes dims[3*l .. 3*l+2] = (nx, ny, nz) and relaxation times
 * tau[l], share one population buffer and one aux buffer (both caller-owned,
 * sized by lbm_batch_required_bytes) and advance together: each time step
 * walks a work list of (lattice, cell range) items in one launch (one per
 * row width class in the second propagation phase), and runs of steps replay
 * as a captured HIP graph.  The update of every cell is the single-lattice
 * collide-and-stream (same cell arithmetic, same in-place AA layout).  No
 * body force, no walls.  With 16-bit storage, a member whose nx is odd keeps
 * one padding slot after every x-row in the population buffer (rows nx + 1
 * slots apart); the member calls below read and write cells only.
 *
 * Each member is also an ordinary lattice handle (lbm_batch_lattice): use
 * lbm_init_equilibrium / lbm_set_populations / lbm_get_populations /
 * lbm_moments / lbm_totals / lbm_get_info on it.  Calls that would advance
 * or reconfigure a member alone (lbm_step, lbm_set_geometry, lbm_set_tau,
 * lbm_set_body_force, lbm_set_wall_velocity, lbm_set_graph_steps,
 * lbm_lattice_destroy) return LBM_ERR_STATE.  Nearest guide analogue: many
 * cuboids (block lattices) per process (Core Concepts, "(Super,Block)Lattice").
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch; /* opaque handle */

/* Host-only sizes of the batch's population and aux buffers. */
lbm_status lbm_batch_required_bytes(lbm_descriptor d, int count, const int* dims, lbm_storage s,
                                    size_t* pop_bytes, size_t* aux_bytes);

/* Create the batch on the current device (sync: uploads the all-fluid
 * geometry of every member).  Arguments as lbm_lattice_create, per member. */
lbm_status lbm_batch_create(lbm_batch** out, lbm_descriptor d, int count, const int* dims,
                            const double* tau, lbm_storage s, unsigned flags, void* dev_pop,
                            size_t pop_bytes, void* dev_aux, size_t aux_bytes, void* hip_stream);

/* Borrow member `index` as a lattice handle (owned by the batch). */
lbm_status lbm_batch_lattice(lbm_batch* b, int index, lbm_lattice** view);

/* Advance every member by n steps.  async.  All members must be initialised
 * and in the same propagation phase (LBM_ERR_STATE otherwise). */
lbm_status lbm_batch_step(lbm_batch* b, int n);

/* As lbm_set_graph_steps, for the batch launch. */
lbm_status lbm_batch_set_graph_steps(lbm_batch* b, int steps);

/* Launch shape of both propagation phases: threads per block (128, 256 or
 * 512; a phase-0 item is a run of that many lanes of cells, a phase-1 item as
 * many whole x-rows as fit, so phase 1 needs at least the widest row's lanes)
 * and resident blocks per compute unit of the persistent grid (1..64), or 0
 * for one block per work item.  LBM_ERR_ARG for any other value. */
lbm_status lbm_batch_set_launch(lbm_batch* b, int threads, int blocks_per_cu);

/* The same for one phase (0 or 1) only; the other keeps its shape.  The two
 * phases are separate launches with different bodies (phase 0 local to each
 * cell, phase 1 over whole x-rows), and their fastest shapes differ. */
lbm_status lbm_batch_set_phase_launch(lbm_batch* b, int phase, int threads, int blocks_per_cu);

/* Current shape of one phase (0 or 1).  Host only. */
lbm_status lbm_batch_get_phase_launch(const lbm_batch* b, int phase, int* threads,
                                      int* blocks_per_cu);

/* Measure every launch shape in the built-in candidate set (threads 128 /
 * 256 / 512 x blocks per CU 0 / 2 / 4 / 8 / 16) for both phases over
 * trial_steps (even, 2..1000) timed steps each, timing the two phases'
 * launches apart;
 * then time each phase's fastest shape combined, and keep that combination if
 * it beats the fastest common shape, else the common shape (read the result
 * with lbm_batch_get_phase_launch).  Reports phase 1's shape in *threads /
 * *blocks_per_cu and the kept shapes' measured ms per step as
 * *best_ms_per_step (any output may be NULL).
 * Members must be initialised (any state will do); every trial (each
 * candidate, and the combination) advances them by trial_steps + 2 steps (the
 * propagation phase is kept), so initialise them again afterwards.  sync. */
lbm_status lbm_batch_autotune(lbm_batch* b, int trial_steps, int* threads, int* blocks_per_cu,
                              double* best_ms_per_step);

/* Member count, total cells, and phase 1's launch shape. */
lbm_status lbm_batch_get_info(const lbm_batch* b, int* count, long long* total_cells,
                              int* threads, int* blocks_per_cu);

/* Release the batch and its member handles (not the caller's buffers). */
lbm_status lbm_batch_destroy(lbm_batch* b);

const char* lbm_batch_last_error(const lbm_batch* b);

/* ---------------------------------------------------------------------------
 * Porous channel and its discrete adjoint (D3Q19, FP32 storage and arithmetic).
 *
 * Model: the guide's porous media model (Simulation Models, "Porous Media
 * Model"): a per-cell porosity d in [0, 1] (0 solid, 1 fluid) scales the
 * velocity of the Maxwellian.  The fused collision uses v = d u, u = j/rho +
 * g/2, in both the second-order equilibrium and the Guo term (d = 1 is the
 * plain BGK + Guo collision); resting bounce-back walls (material 2) and
 * periodic axes as for lbm_set_geometry; moving walls are refused.
 * Objective J: the mean force-shifted x-velocity over the fluid cells of the
 * plane x = plane_x after `steps` steps from rest (rho = 1, u = 0).
 * Gradient dJ/dd by the discrete adjoint of the scheme (the guide's adjoint
 * LBM option, Flow Control and Optimization, "Derivative Computation"),
 * reverse in time with the forward states recomputed from checkpoints taken
 * every `checkpoint_every` steps.  All device memory is one caller-owned
 * work buffer of lbm_porous_required_bytes: about (steps / checkpoint_every
 * + checkpoint_every + 4) states of 76 bytes per cell.  checkpoint_every = 1
 * keeps every forward state and recomputes none (the fastest gradient; about
 * 20 GB for a 128 x 64 x 64 channel over 500 steps).
 * ------------------------------------------------------------------------- */
typedef struct lbm_porous lbm_porous; /* opaque handle */

lbm_status lbm_porous_required_bytes(int nx, int ny, int nz, int steps, int checkpoint_every,
                                     size_t* work_bytes);

/* material: host, N bytes (copied); g: host body acceleration; plane_x: the
 * objective plane (0 <= plane_x < nx). */
lbm_status lbm_porous_create(lbm_porous** out, int nx, int ny, int nz, double tau,
                             const uint8_t* material, unsigned periodic_mask, const double g[3],
                             int steps, int checkpoint_every, int plane_x, void* dev_work,
                             size_t work_bytes, void* hip_stream);

/* Run the forward problem for porosity_dev (device float[N], copied) and
 * return J (host).  Keeps the checkpoints for lbm_porous_backward.  sync. */
lbm_status lbm_porous_forward(lbm_porous* h, const float* porosity_dev, double* J);

/* dJ/dd for the porosity of the last forward run into grad_dev (device
 * float[N]; zero on non-fluid cells).  sync.  LBM_ERR_STATE before any
 * successful forward run (or after a failed one, whose checkpoints are
 * incomplete). */
lbm_status lbm_porous_backward(lbm_porous* h, float* grad_dev);

/* Number of forward runs completed on h (0 before the first).  A caller that
 * keeps the value of a run can tell whether lbm_porous_backward still
 * differentiates that run: it does while the count is unchanged.  Host-only. */
lbm_status lbm_porous_generation(const lbm_porous* h, long long* generation);

/* Final populations of the last forward run, device double[19*N], natural
 * layout (f_i of cell idx at i*N + idx).  sync. */
lbm_status lbm_porous_get_final(lbm_porous* h, double* f_dev);

lbm_status lbm_porous_destroy(lbm_porous* h);
const char* lbm_porous_last_error(const lbm_porous* h);

const char* lbm_status_string(lbm_status st);
/* Message of the last failed call on h ("" if none); h may be NULL for
 * failures of lbm_lattice_create. */
const char* lbm_last_error(const lbm_lattice* h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
