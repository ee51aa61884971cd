/*
 * mpc.h -- C ABI of the MI355X (gfx950) multiparticle-collision-dynamics
 * library: one MPC-SRD time step on one GPU, for one periodic (or z-walled)
 * box or for a batch of independent boxes advanced together.
 *
 * The method is that of Westphal, Goh, Winkler and Gompper, "HTMPC",
 * arXiv:2406.15236, Sec. II:
 *   - streaming r <- r + h v                                   (Eq. 1)
 *   - random shift of the collision lattice before each collision
 *   - particles sorted into cubic cells of side a
 *   - per cell: centre-of-mass velocity v_cm, relative velocities rotated by a
 *     fixed angle alpha about an axis drawn at random per cell and step  (Eq. 2)
 *   - optional Maxwell-Boltzmann scaling thermostat: relative velocities scaled
 *     by kappa = sqrt(2 E_k / sum m v_c^2), E_k ~ Gamma(f/2, k_B T),
 *     f = 3 (N_c - 1)                                          (Thermostat)
 *   - optional no-slip walls at z = 0 and z = H (bounce-back + phantom
 *     particles filling wall-cut cells) and constant gravity (Boundary
 *     conditions, External fields)
 *   - particles periodically reordered by cell (Sec. III.B.3, reordering).
 *     Here the device keeps the particles in cell order every step; the
 *     reorder interval R decides when the order seen through mpc_get_state
 *     is renumbered to (cell, index) order: after every step t with
 *     (t + 1) mod R = 0 (R = 0: never).
 * The arguments follow the paper's statement of the method: box in cells,
 * cell size a, mean density <N_c>, time step h, rotation angle alpha, k_B T,
 * mass m, and a main random seed (Sec. III.E: the main seed may be given as
 * a parameter).
 *
 * Conventions for every call:
 *   - All calls are extern "C"; no C++ exception crosses this boundary.
 *   - Return value 0 on success, else a negative MPC_E* code; mpc_strerror()
 *     names it and mpc_last_error() gives the message of the handle.
 *   - Device pointers are hipMalloc'ed (or torch-allocated) memory on the
 *     current device; host pointers are ordinary host memory.
 *   - A handle belongs to one HIP stream and is not thread-safe.
 *   - mpc_step only enqueues work on the stream; errors detected inside
 *     kernels (a particle outside the box or not finite, more than
 *     MPC_MAX_CELL_PARTICLES particles in one cell) are sticky and reported by
 *     the next synchronising call (mpc_sync, mpc_observables, mpc_get_state,
 *     mpc_get_binning).
 */
#ifndef MPC355_MPC_H
#define MPC355_MPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage form of the particle state. */
typedef enum {
  MPC_FP64 = 0,    /* x, v in FP64 (48-byte record); every operation in FP64            */
  MPC_FP32 = 1,    /* x, v in FP32 (24-byte record); streamed in FP32, cell sums and
                      rotation in FP64                                                 */
  MPC_SPLIT32 = 2  /* packed int32 cell index + FP32 offset in [0,1) per axis, FP32
                      velocities and the particle's index in one 32-byte record;
                      streaming and rotation in FP32 with compensated FP32 momentum
                      sums per cell; thermostat energy and kappa in FP64               */
} mpc_form;

/* Feature flags (identical for all boxes of one handle). */
enum {
  MPC_MBS = 1u,     /* Maxwell-Boltzmann scaling thermostat (Sec. II, Thermostat)     */
  MPC_WALLS_Z = 2u, /* no-slip walls at z = 0 and z = L[2] = H: bounce-back streaming
                       and phantom particles in wall-cut cells (Sec. II, Boundary
                       conditions); x and y stay periodic                              */
  MPC_AMC = 4u,     /* angular-momentum-conserving collision SRD+a (Sec. II, Eqs. 3-4):
                       v_i' = v_cm + D u_i + omega x r_ic with omega = I^-1 dL, where
                       r_ic is the position relative to the cell's centre of mass in
                       the shifted cell's frame, frac(x/a + s), I the inertia tensor
                       and dL = m sum_i r_ic x (u_i - D u_i).  A cell of two uses the
                       pseudo-inverse of its singular I, omega = dL / (m |r_12|^2 / 2);
                       det I = 0 gives omega = 0.  With MPC_MBS the rotation is not
                       scaled; kappa scales the corrected relative velocities
                       D u_i + omega x r_ic so that their kinetic energy equals the
                       drawn E_k (angular momentum is then scaled by kappa).
                       Periodic boxes or slip walls: with MPC_WALLS_Z and without
                       MPC_SLIP -> MPC_EINVAL (phantoms carry no positions)       */
  MPC_SLIP = 16u,    /* with MPC_WALLS_Z: slip walls (Sec. II, Boundary conditions):
                       specular reflection (z and v_z mirrored, v_x, v_y kept) and no
                       phantom particles.  Without MPC_WALLS_Z -> MPC_EINVAL         */
  MPC_FIXED_SUMS = 8u /* reproducible cell sums (Sec. III.C): every sum over a cell's
                       fluid particles (momentum, kinetic energy, the SRD+a moments)
                       is exact in fixed point -- each FP64 term x becomes the
                       integer trunc(x 2^80) in 128 bits, the sum is rounded once
                       to FP64 -- so the trajectory does not depend on the order in
                       which particles are stored (caller's order, reorder interval,
                       tiling).  Terms must satisfy |x| < 2^37 in cell units (speeds
                       below 2^18.5 cells per unit time); otherwise the next
                       synchronising call returns MPC_ERANGE                        */
};

/* Error codes. */
enum {
  MPC_OK = 0,
  MPC_EINVAL = -1,   /* invalid argument (box, a, h, alpha, density, kT, m, form, flags) */
  MPC_ENOSPACE = -2, /* workspace smaller than mpc_workspace_bytes                       */
  MPC_ERANGE = -3,   /* N or cell count >= 2^31, box too large for the form, a cell
                        that held more than MPC_MAX_CELL_PARTICLES particles, or (with
                        MPC_FIXED_SUMS) a summand outside the fixed-point range       */
  MPC_EHIP = -4,     /* HIP runtime error (message kept in the handle)                  */
  MPC_ESTATE = -5    /* a particle left the box or became non-finite                    */
};

/* Largest number of particles one collision cell may hold in a step: a cell
 * is collided in one on-chip pass.  A fuller cell is streamed and re-binned
 * but not collided in that step, and the next synchronising call returns
 * MPC_ERANGE (the trajectory is then no longer the method's). */
#define MPC_MAX_CELL_PARTICLES 256
#define MPC_MAX_BOXES 4096

/* Parameters of one box.  Lengths are in units of the cell size a except a
 * itself; positions passed to or returned by the state calls are physical
 * (multiplied by a), velocities physical (length / time). */
typedef struct {
  int32_t  L[3];          /* box in cells; with MPC_WALLS_Z, L[2] = H                     */
  int32_t  form;          /* mpc_form (same for all boxes)                                 */
  uint32_t flags;         /* MPC_MBS | MPC_WALLS_Z | MPC_SLIP | MPC_AMC | MPC_FIXED_SUMS
                             (same for all boxes)                                         */
  int32_t  reorder_every; /* R: renumber particles in (cell, index) order after every
                             R-th step; 0 = never (same for all boxes)                    */
  double   a;             /* cell size, > 0                                                */
  double   density;       /* <N_c>: N = llround(density * L0 * L1 * L2), > 0              */
  double   dt;            /* MPC time step h, > 0                                          */
  double   alpha;         /* rotation angle in radians                                     */
  double   kT;            /* k_B T, > 0                                                    */
  double   mass;          /* particle mass m, > 0                                          */
  double   g[3];          /* constant acceleration; applied as v += g h after collision   */
  uint64_t seed;          /* key of the counter-based random streams                      */
  double   wall_u;        /* no-slip walls (MPC_WALLS_Z without MPC_SLIP): the wall at
                             z = H moves with velocity +wall_u along x and the wall at
                             z = 0 with -wall_u (shear flow); 0 otherwise            */
  double   le_u;          /* periodic box, Lees-Edwards shear flow (Sec. II, boundary
                             conditions): the periodic image above the box (z + L[2] a)
                             moves with +le_u along x and is displaced by
                             (le_u tau) mod (L[0] a) at time tau = t dt.  A particle
                             through a z face re-enters shifted by -/+ that offset
                             with v_x -/+ le_u; a collision cell across a z face is
                             formed with the image on the other side, in its velocity
                             frame (with MPC_AMC also with its image positions).
                             One step takes the offset once, so a particle should
                             not cross more than one z face per step
                             (|v_z| dt < L[2] a).
                             0 = plain periodic.  With MPC_WALLS_Z -> MPC_EINVAL  */
} mpc_params;

/* Observables of one box (FP64, compensated sums over the particles). */
typedef struct {
  uint64_t step;       /* number of completed steps                     */
  uint64_t n;          /* particles                                     */
  double   P[3];       /* total momentum sum m v                        */
  double   E;          /* kinetic energy sum m v^2 / 2                  */
  double   T;          /* sum m |v - P/M|^2 / (3 (n - 1))  (k_B T units) */
  double   mass_total; /* n m                                           */
} mpc_obs;

/* Per-kernel device time accumulated by mpc_step_profiled (milliseconds,
 * from HIP events recorded on the handle's stream around each launch):
 * scan = prefix sum of the cell counts, per-cell random draws and (walls)
 * phantom sums; scatter = the sort permutation; collide = the collision,
 * the next step's streaming and binning and the state write; prologue = the
 * binning of a state set from outside; other = the step-counter advance. */
typedef struct {
  double scan_ms, scatter_ms, collide_ms, prologue_ms, other_ms;
  uint64_t scan_launches, scatter_launches, collide_launches, prologue_launches;
} mpc_kernel_times;

typedef struct mpc_sim mpc_sim;

/* Bytes of device workspace needed for nbox boxes with parameters p[0..nbox).
 * The workspace holds the double-buffered particle state, keys, permutation,
 * cell histogram and offsets, and small tables.  Errors: MPC_EINVAL,
 * MPC_ERANGE. */
int mpc_workspace_bytes(const mpc_params* p, int32_t nbox, size_t* bytes);

/* Create a handle.  p[0..nbox) is copied.  workspace: device memory of at
 * least mpc_workspace_bytes bytes, 256-byte aligned, owned by the caller and
 * kept alive until mpc_destroy.  hip_stream: the hipStream_t all work is
 * enqueued on (NULL = default stream), owned by the caller.  The particle
 * state is undefined until mpc_init_state or mpc_set_state.  The step
 * counter starts at 0.  Errors: MPC_EINVAL, MPC_ENOSPACE, MPC_ERANGE, MPC_EHIP. */
int mpc_create(const mpc_params* p, int32_t nbox, void* workspace, size_t bytes,
               void* hip_stream, mpc_sim** out);

/* Fill every box on the device: positions uniform in the box, velocities
 * normal with standard deviation sqrt(kT/m) per component and the mean of
 * each box removed (counter-based stream keyed by init_seed and box). */
int mpc_init_state(mpc_sim* s, uint64_t init_seed);

/* Advance all boxes by nsteps steps (enqueue only). */
int mpc_step(mpc_sim* s, int64_t nsteps);

/* As mpc_step, launching kernel by kernel (no graph) with HIP events around
 * each launch; adds the device times to *acc (which the caller zeroes) after
 * synchronising the stream. */
int mpc_step_profiled(mpc_sim* s, int64_t nsteps, mpc_kernel_times* acc);

/* Captured hipGraphs for mpc_step: 0 = launch kernel by kernel; 1 = replay
 * a graph of one step per step (the default); K in 2..1000 = also capture K
 * consecutive steps in one graph, so that mpc_step(n) is floor(n / K)
 * launches of that graph plus one-step replays for the rest.  Results do
 * not depend on this choice.  A new K drops the captured graphs (they are
 * captured again at the next mpc_step; synchronises).  Errors: MPC_EINVAL
 * (enable outside 0..1000), MPC_EHIP. */
int mpc_set_graph(mpc_sim* s, int32_t enable);

/* Wait for the stream; report sticky kernel errors (MPC_ESTATE, MPC_ERANGE). */
int mpc_sync(mpc_sim* s);

/* Observables of box `box` (synchronises). */
int mpc_observables(mpc_sim* s, int32_t box, mpc_obs* out);

/* Particle count and cell count (including wall layers) of a box. */
int mpc_box_info(mpc_sim* s, int32_t box, int64_t* n, int64_t* ncell);

/* Step counter: get, or set (the random streams are keyed by it). */
int mpc_get_step(mpc_sim* s, uint64_t* step);
int mpc_set_step(mpc_sim* s, uint64_t step);

/* Copy the state of one box from / to host FP64 SoA arrays x[3][n], v[3][n]
 * (x[0..n) = x components, x[n..2n) y, x[2n..3n) z; physical units).  n must
 * equal the box's particle count.  Positions must lie in [0, L a) on periodic
 * axes and in [0, H a] on a walled z axis (MPC_EINVAL otherwise).
 * Conversions: FP64 exact; FP32 rounds to nearest; SPLIT32 stores
 * cell = floor(x/a), offset = (float)(x/a - cell) (an offset that rounds to 1
 * moves to the next cell).  get returns the exact FP64 value of what is
 * stored.  Both synchronise and move the box through host staging buffers a
 * few million particles at a time.  get returns MPC_ESTATE if the stored
 * logical indices are not a permutation of [0, n) (x and v then hold only
 * part of the state); set leaves the state unchanged on MPC_EINVAL (the
 * positions are checked before anything is copied). */
int mpc_set_state(mpc_sim* s, int32_t box, const double* x, const double* v, int64_t n);
int mpc_get_state(mpc_sim* s, int32_t box, double* x, double* v, int64_t n);

/* State of selected particles of one box, for sampling a box too large to
 * copy whole: for k in [0, m), x[k], x[m + k], x[2m + k] and v[k], v[m + k],
 * v[2m + k] receive the position and velocity of the particle with logical
 * index idx[k] -- the index at which mpc_get_state would return it -- with
 * the same conversion as mpc_get_state (exact FP64 of what is stored, times
 * a).  idx entries lie in [0, n) and may repeat; x and v hold 3m doubles
 * each, caller-owned.  Takes temporary device memory (4 n + 52 m bytes) for
 * the duration of the call.  Synchronises.  Errors: MPC_EINVAL (index
 * outside the box, NULL pointer with m > 0), MPC_EHIP, and sticky kernel
 * errors (MPC_ESTATE, MPC_ERANGE). */
int mpc_get_particles(mpc_sim* s, int32_t box, const int64_t* idx, int64_t m, double* x,
                      double* v);

/* Binning of the last completed step of one box (synchronises):
 *   offset[ncell+1]: exclusive prefix of particles per cell;
 *   perm[n]: index (in the particle order of mpc_get_state before that step)
 *            of the j-th particle in (cell key, index) order;
 *   key[n]:  cell key of each particle, indexed by that same order.
 * Keys are x-fastest: ((c_z' * L1) + c_y) * L0 + c_x with c_z' = c_z (periodic)
 * or c_z + 1 (walls).  Any pointer may be NULL.  MPC_EINVAL if no step has
 * run since the state was set. */
int mpc_get_binning(mpc_sim* s, int32_t box, uint32_t* key, uint32_t* perm, uint32_t* offset);

/* Autotuner: choose the collide tiling (cells per tile, persistent grid size,
 * rows per block of the tile order) by timing trial_steps steps (1..1000) of
 * each candidate from the current state (a candidate counts with its fastest
 * step), in a coordinate search (tile size,
 * then grid, then row block, then the x-segment-major order with each row
 * block).  Before every trial and at the end the state
 * and step counter are restored from a copy, so the random streams and all
 * later results are exactly those of an untuned handle (results do not depend
 * on the tiling).  The copy is one state buffer, in temporary device memory
 * (pinned host memory if the device has no room).  Synchronises.  Returns the
 * chosen tile size (0 = automatic per box) and grid in *tile_cells and *grid
 * (either may be NULL).  Errors: MPC_EINVAL, MPC_EHIP, and sticky kernel
 * errors of the state (MPC_ESTATE, MPC_ERANGE). */
int mpc_autotune(mpc_sim* s, int32_t trial_steps, int32_t* tile_cells, int32_t* grid);

/* Override the collide tiling: cells per tile (4..32, 0 = automatic),
 * persistent grid size (0 = automatic), the number of rows per block of the
 * XCD-aware tile order (0 = automatic, 8) and the order inside a block
 * (0 = the tiles of one row after another; 1 = the same x segment of every
 * row of the block, then the next segment).  Results do not depend on the
 * tiling.  Errors: MPC_EINVAL (out of range), MPC_EHIP. */
int mpc_set_tiling(mpc_sim* s, int32_t tile_cells, int32_t grid, int32_t yblock, int32_t order);

/* Current collide tiling: tile_cells (0 = automatic per box), persistent grid
 * size, rows per block of the tile order, the order inside a block, and the
 * number of tiles.  Any pointer may be NULL. */
int mpc_get_tiling(mpc_sim* s, int32_t* tile_cells, int32_t* grid, int32_t* yblock,
                   int32_t* order, int64_t* ntiles);

/* Release the handle (not the workspace or the stream).  Synchronises. */
int mpc_destroy(mpc_sim* s);

/* Allocation-free run, for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc):
 * advances one FP64 box (p->form = MPC_FP64, any flags) in place by nsteps
 * steps, the first with step index `step` (the random streams are keyed by
 * it), exactly as mpc_create + mpc_set_state + mpc_set_step + mpc_step +
 * mpc_get_state would.  x[3][n], v[3][n]: caller-owned device arrays, FP64
 * SoA in physical units as in mpc_set_state; on return they hold the state
 * after the steps in the same particle order.  All working memory (both
 * state buffers, keys, permutation, cell counts, offsets, draws, tables) is
 * a static device array of 256 MiB inside the library, one per device, held
 * until the process ends; no device memory is allocated.  Boxes whose
 * workspace (mpc_workspace_bytes) exceeds 256 MiB -> MPC_ERANGE (about 2e6
 * particles at 10 per cell).  Every call on a device shares that device's
 * array: calls that overlap on one device (other threads, or a stream not
 * drained) race.  Launches kernel by kernel on hip_stream (NULL = default
 * stream) and synchronises it.  Errors: MPC_EINVAL (bad parameters, n not
 * the box's particle count, form not FP64, a position outside the box or a
 * non-finite value), MPC_ERANGE, MPC_EHIP, and the sticky kernel errors of
 * mpc_sync. */
int mpc_run_noalloc(const mpc_params* p, double* x, double* v, int64_t n, uint64_t step,
                    int64_t nsteps, void* hip_stream);

/* Bandwidth probes (measurement only; no MPC state): plain streaming kernels
 * that give the HBM bandwidth a kernel attains on this device, the
 * reference beside which the MPC kernels' byte rates are reported.
 * mpc_probe_copy copies `bytes` from src to dst (device pointers, 16-byte
 * aligned, bytes a multiple of 16, non-overlapping): every byte read and
 * written once.  mpc_probe_read reads `bytes` from src once and writes one
 * 32-bit XOR fold per thread to out (device memory of at least
 * grid * 256 * 4 bytes, out_bytes).  grid: workgroups of 256 threads,
 * 0 = 8 per compute unit.  Both only enqueue on hip_stream (NULL = default
 * stream).  Errors: MPC_EINVAL (alignment, size, out too small), MPC_EHIP. */
int mpc_probe_copy(void* dst, const void* src, size_t bytes, int32_t grid, void* hip_stream);
int mpc_probe_read(const void* src, size_t bytes, void* out, size_t out_bytes, int32_t grid,
                   void* hip_stream);

const char* mpc_strerror(int code);
const char* mpc_last_error(mpc_sim* s);

#ifdef __cplusplus
}
#endif
#endif
