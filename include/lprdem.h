/*
 * lprdem.h -- C ABI of the MI355X graded-bed DEM stepper.
 *
 * The library steps the contact pipeline of the paper "Local particle
 * refinement in terramechanical simulations" (arXiv 2501.05300) for
 * polydisperse spheres whose radius grows with depth:
 *
 *   broad phase  : multi-level cell lists, one grid per radius band, over a
 *                  Morton-ordered particle store;
 *   narrow phase : exact FP64 sphere-sphere and sphere-wall predicates;
 *   contact law  : section "Nonsmooth DEM and multibody dynamics" --
 *                  Hertz gap g_n = delta^{e_H} (e_H = 5/4), compliance e_H/k_n,
 *                  k_n = E* sqrt(d*) / 3 with E* and d* as defined there,
 *                  damping gamma_n = 4.5 dt (eq:g_n, read as the compliant
 *                  force F_n = max(0, k_n (delta^{2e_H-1} + e_H gamma_n
 *                  delta^{2e_H-2} ddelta/dt))), Coulomb cone |F_t| <= mu_t F_n
 *                  (eq:G_t) and rolling cone |M_r| <= mu_r r* F_n (eq:G_r),
 *                  both realised as springs with per-contact history;
 *   accumulation : deterministic (no floating-point atomics), FP64 body
 *                  reactions;
 *   integration  : velocity then position (the ordering of the paper's
 *                  first-order stepper), explicit.
 *
 * Conventions
 *   - All entry points are synchronous with respect to their host arguments
 *     and return an lpr_status.  No C++ exception crosses this boundary.
 *   - Unless a parameter says "device", every pointer argument is a host
 *     pointer owned by the caller; inputs are copied, outputs are written.
 *   - Particle arrays are indexed by stable id (the order of the arrays
 *     passed at creation), 3 components interleaved (x0 y0 z0 x1 ...).
 *   - Work is enqueued on the HIP stream given at creation.  lpr_step returns
 *     after enqueueing; every read and lpr_sync wait for the stream.
 *   - Device faults found by kernels (history-slot overflow, non-finite
 *     values, a particle through a plane wall) latch.  The state then stays at the last complete step; reads
 *     and lpr_sync report the latched status; only lpr_get_state and
 *     lpr_bed_destroy remain usable.
 */
#ifndef LPRDEM_H
#define LPRDEM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LPR_OK = 0,
  LPR_E_INVAL = -1,     /* invalid argument or description */
  LPR_E_NOMEM = -2,     /* allocation failed */
  LPR_E_DEVICE = -3,    /* HIP runtime error */
  LPR_E_CAPACITY = -4,  /* output buffer too small, or a per-particle
                           history table overflowed (latched) */
  LPR_E_STATE = -5,     /* call not allowed in the current state (a latched
                           fault, or a broad-phase skin exceeded) */
  LPR_E_NUMERIC = -6,   /* non-finite force or state (latched) */
  LPR_E_DOMAIN = -7     /* a particle passed through a plane wall: its
                           centre lies beyond the plane by more than its
                           radius (latched) */
} lpr_status;

enum { LPR_WALL_PLANE = 0, LPR_WALL_DISK = 1, LPR_WALL_ANNULUS = 2, LPR_WALL_BOX = 3 };

/* Device-memory provider.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; release frees it.  A NULL allocator
 * makes the library use hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes);
  void (*release)(void* ctx, void* ptr);
  void* ctx;
} lpr_allocator;

/* Material and contact parameters of a bed (section "Generation of soil
 * samples": 2200 kg/m^3, 1 GPa, 0.15, mu_t 0.3, mu_r 0.02). */
typedef struct {
  double rho;           /* particle density [kg/m^3] */
  double E, nu;         /* Young's modulus [Pa], Poisson ratio */
  double mu_t, mu_r;    /* Coulomb and rolling-resistance coefficients */
  double dt;            /* time step [s] */
  double gamma_factor;  /* gamma_n = gamma_factor * dt (paper: 4.5) */
  double e_H;           /* gap exponent: 1.25 (Hertz) or 1 (linear) */
  double kappa_t;       /* tangential / normal spring stiffness ratio */
  double s_k;           /* multiplier on k_n */
  double g[3];          /* gravity [m/s^2] */
} lpr_params;

/* A wall primitive attached to a kinematic body.  Geometry is given in the
 * body frame (relative to the body origin, before its rotation about +z).
 *   PLANE   : point origin, unit normal axis toward the particles; contact
 *             when the signed distance (x - o).axis < r.
 *   DISK    : one-sided disk, centre origin, normal axis toward the
 *             particles, radius dims[0]; face and rim contacts.
 *   ANNULUS : like DISK with radii dims[0] (inner) .. dims[1] (outer); the
 *             first row of frame is its in-plane reference direction.
 *   BOX     : centre origin, local axes = rows of frame, half extents dims.
 * mu_t / mu_r < 0 means "the bed's value". */
typedef struct {
  int32_t kind;
  int32_t body;
  double origin[3];
  double axis[3];
  double frame[9];
  double dims[3];
  double mu_t, mu_r;
} lpr_wall;

/* A kinematic body: origin(t) = origin + lin_vel t, rotated by ang_vel t
 * about +z through its origin.  z_free = 1 makes z a dynamic degree of
 * freedom of mass `mass` under gravity and the particles' reaction. */
typedef struct {
  double origin[3];
  double lin_vel[3];
  double ang_vel;
  int32_t z_free;
  double mass;
} lpr_body;

typedef struct {
  int64_t n;               /* particle count (> 0) */
  double box[3];           /* periodic lengths in x, y (z unused) */
  uint32_t periodic;       /* bit0: x periodic, bit1: y periodic */
  const double* pos;       /* host, n*3 */
  const float* radius;     /* host, n, > 0 */
  const float* vel;        /* host, n*3 or NULL (zero) */
  const float* omega;      /* host, n*3 or NULL (zero) */
  int32_t n_walls;         /* <= LPR_MAX_WALLS */
  const lpr_wall* walls;
  int32_t n_bodies;        /* <= LPR_MAX_BODIES; body 0 is the static frame */
  const lpr_body* bodies;
  lpr_params params;
  /* broad-phase controls; they change how contacts are found, never which */
  int32_t rebuild_every;   /* 1: cell search every step; k > 1: candidate
                              lists with a skin, rebuilt every k steps */
  float skin;              /* [m], required > 0 when rebuild_every > 1 */
  float band_ratio;        /* radius ratio of one cell-list level (0: 2) */
  float cell_factor;       /* cell edge / (2 r_max(level) + skin), >= 1 (0: 1) */
  int32_t block;           /* threads per block of the step kernel: 64, 128
                              or 256 (0: 64) */
  int32_t record_forces;   /* 1: keep the last step's per-particle contact
                              forces and torques for lpr_read_forces and its
                              per-contact loads for lpr_read_contact_loads
                              (64 B per particle and owner slot, 32 B per
                              particle and wall) */
  int32_t persistent;      /* 1: the step kernel runs as one persistent grid
                              that fills the GPU (same results) */
  /* storage order (never changes results, only which particles share cache
     lines): particles are kept sorted by (level, Morton code of their cell),
     equal codes in their previous order.  At every sort_every-th rebuild a
     device radix sort re-sorts them and the state is gathered into the new
     order; 0: the default (every 16th rebuild with rebuild_every 1, every
     rebuild otherwise), < 0: never (the order of creation stays), at most
     4096 */
  int32_t sort_every;
  int32_t input_order;     /* 1: start from the caller's order instead of the
                              sorted one (to measure what the sort buys) */
  float level_cell_factor[16];  /* per radius band (cell-list level q, the
                                   q-th band from the finest): its cell
                                   factor, >= 1; 0 takes cell_factor */
} lpr_bed_desc;

#define LPR_MAX_WALLS 16
#define LPR_MAX_BODIES 4
#define LPR_SLOTS 16        /* sphere contacts per owner particle */

/* A contact of the last step: a < b are stable ids of two particles, or a is
 * a particle and b = -1 - w for wall w. */
typedef struct {
  int64_t a, b;
} lpr_contact;

/* One history record: owner stable id, partner code (stable id or -1 - w),
 * tangential spring (3) and rolling spring (3). */
typedef struct {
  int64_t owner, partner;
  float xi_t[3], xi_r[3];
} lpr_history;

typedef struct lpr_bed lpr_bed;

/* Creates a bed.  The description is validated (0 < n < 2^27, r > 0,
 * finite inputs, dt > 0, periodic length > 2 max(r_i + r_j + skin),
 * wall/body indices in range), particles are placed in Morton order per
 * radius band on the device (and re-sorted there as they move, see
 * sort_every), and the per-step kernel sequence is captured in a HIP graph
 * on `hip_stream` (NULL = the default stream).  *out receives
 * the bed; on error *out is NULL.  A sphere owns its contacts with spheres
 * of larger radius (equal radii: larger stable id) in 16 slots; a 17th
 * latches LPR_E_CAPACITY, reported at the next lpr_sync. */
lpr_status lpr_bed_create(const lpr_bed_desc* desc, const lpr_allocator* alloc, void* hip_stream,
                          lpr_bed** out);
lpr_status lpr_bed_destroy(lpr_bed* bed);

/* Enqueues n_steps >= 0 steps.  Asynchronous. */
lpr_status lpr_step(lpr_bed* bed, int64_t n_steps);
/* Like lpr_step, but launches the kernels directly (no graph) with HIP
 * events on the bed's stream around each kernel group, then waits.
 * out[0]: summed ms of the broad-phase rebuild kernels, out[1]: summed ms of
 * the fused contact/integration kernel, out[2]: summed ms of the body
 * reduction kernel, out[3]: ms from the first to the last event.  Used to
 * measure per-kernel durations for the roofline. */
lpr_status lpr_step_profiled(lpr_bed* bed, int64_t n_steps, double out[4]);
/* Like lpr_step_profiled with finer phases, HIP events on the bed's stream
 * at each phase boundary of every step, then waits.  Summed milliseconds:
 * out[0] binning (counter clearing, cell binning and the cell-range scan),
 * out[1] re-sort of the storage order (radix sort and gather; 0 in steps
 * without one), out[2] cell lists, out[3] owner-side search, out[4] reverse
 * lists, out[5] the contact step (the fused kernel, or the implicit step's
 * kernels), out[6] body reduction, out[7] ms from the first to the last
 * event.  Phases 0-4 are 0 in steps that reuse candidate lists. */
lpr_status lpr_step_phases(lpr_bed* bed, int64_t n_steps, double out[8]);
/* Waits for the bed's stream and reports any latched device status. */
lpr_status lpr_sync(lpr_bed* bed);

/* Particle state in stable-id order (host buffers, n*3 each; any may be NULL). */
lpr_status lpr_get_state(lpr_bed* bed, double* pos, float* vel, float* omega);
/* Replaces the particle state (NULL leaves a field unchanged); history of
 * contacts is kept. */
lpr_status lpr_set_state(lpr_bed* bed, const double* pos, const float* vel, const float* omega);

/* Contact history.  lpr_get_history writes up to `capacity` records and sets
 * *n_total; LPR_E_CAPACITY (nothing written) when capacity < *n_total.
 * lpr_set_history replaces all history; records for pairs that are not in
 * the current candidate lists are dropped (they would be dropped by the
 * next step anyway). */
lpr_status lpr_get_history(lpr_bed* bed, lpr_history* out, int64_t capacity, int64_t* n_total);
lpr_status lpr_set_history(lpr_bed* bed, const lpr_history* rec, int64_t count);

/* The last step's contacts, ascending (a, b); LPR_E_CAPACITY with *n_total
 * set and nothing written when capacity is too small. */
lpr_status lpr_read_contacts(lpr_bed* bed, lpr_contact* out, int64_t capacity, int64_t* n_total);
/* The last step's contact-only force and torque per particle (requires
 * record_forces; host buffers n*3, stable-id order). */
lpr_status lpr_read_forces(lpr_bed* bed, float* force, float* torque);
/* Loads of one contact of the last step (section "Nonsmooth DEM and
 * multibody dynamics", eq:g_n, eq:G_t, eq:G_r): a and b as in lpr_contact;
 * force = the contact force on particle a (normal and tangential parts),
 * moment = the rolling-resistance moment on particle a (the torque on a is
 * (p - x_a) x force + moment, p the contact point), fn = the normal force
 * magnitude F_n >= 0.  For a wall contact (b = -1 - w) they act on the
 * particle. */
typedef struct {
  int64_t a, b;
  float force[3];
  float moment[3];
  float fn;
  float reserved;
} lpr_contact_load;

/* The last step's per-contact loads in lpr_read_contacts order (requires
 * record_forces and the explicit stepper, else LPR_E_STATE); LPR_E_CAPACITY
 * with *n_total set and nothing written when capacity is too small. */
lpr_status lpr_read_contact_loads(lpr_bed* bed, lpr_contact_load* out, int64_t capacity, int64_t* n_total);
/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid allocation): lpr_read_contact_loads without any allocation.
 * Its workspace is a static device array of LPR_NOALLOC_SCRATCH_BYTES that
 * each GPU the library runs on holds until the process ends; it must hold
 * about 8 bytes per particle (n rounded up to 256) plus 48 bytes per
 * contact, else LPR_E_CAPACITY (nothing written).  The bed must have no
 * pending device status (call lpr_sync after stepping; else LPR_E_STATE).
 * Calls that overlap on one GPU share the array and race: serialise them.
 * Same output and errors as lpr_read_contact_loads otherwise. */
#define LPR_NOALLOC_SCRATCH_BYTES (32u << 20)
lpr_status lpr_read_contact_loads_noalloc(lpr_bed* bed, lpr_contact_load* out, int64_t capacity, int64_t* n_total);
/* World pose of wall `wall` at the current clock (the pose the next step
 * uses): origin (3), unit normal `axis` after the body's motion (3), and the
 * three rows of its frame (9).  The body rotation angle is ang_vel * k dt
 * in FP64 (cos and sin of the device math library). */
lpr_status lpr_read_wall_pose(lpr_bed* bed, int32_t wall, double out15[15]);
/* Reaction of the last step on a body: force from the particles (3) and
 * torque about the body origin (3), FP64. */
lpr_status lpr_read_reaction(lpr_bed* bed, int32_t body, double out6[6]);
/* Sum over steps of the body reaction since the last reset and the number
 * of steps summed; reset = 1 clears the sums after reading. */
lpr_status lpr_reaction_window(lpr_bed* bed, int32_t body, double sum6[6], int64_t* steps, int32_t reset);
/* Current pose of a body: origin and translation velocity. */
lpr_status lpr_read_body(lpr_bed* bed, int32_t body, double origin[3], double vel[3]);

/* Time step index k (t = k dt) and dynamic-body state. */
lpr_status lpr_set_clock(lpr_bed* bed, int64_t step);
lpr_status lpr_get_clock(lpr_bed* bed, int64_t* step);
lpr_status lpr_set_body_state(lpr_bed* bed, int32_t body, double z, double vz);

typedef struct {
  int64_t steps;            /* completed steps */
  int64_t contacts;         /* contacts of the last step (sphere + wall) */
  int64_t candidates;       /* owner-side candidate pairs in the lists */
  int64_t rebuilds;         /* broad-phase rebuilds performed */
  int32_t levels;           /* cell-list levels */
  int64_t cells;            /* cells over all levels */
  int32_t max_owner_slots;  /* largest per-owner candidate count seen */
  int64_t skin_trips;       /* times a skin was exceeded between rebuilds
                               (those steps were rebuilt and repeated) */
  int32_t adjoint_interval; /* checkpoint interval of the last adjoint window
                               (0 before the first) */
  int64_t sorts;            /* device re-sorts of the storage order */
  int64_t outside_grid;     /* binnings of a particle outside its level's
                               grid on a bounded axis since creation (it is
                               then binned into the edge cell and its
                               contacts are still found; a growing count
                               means the bed left its planned extent) */
} lpr_stats;
lpr_status lpr_get_stats(lpr_bed* bed, lpr_stats* out);

/* ---- batched beds ----------------------------------------------------
 * Many beds (uneven sizes and grading) stepped together: every kernel of a
 * step covers all beds in one launch, and the steady cycle is one captured
 * HIP graph.  Beds are independent (no contacts across beds); each keeps its
 * own parameters, walls, bodies, clock and cell-list layout (band_ratio,
 * cell_factor).  rebuild_every, skin, block, persistent and record_forces
 * must agree across the descriptions.  lpr_step, lpr_step_profiled,
 * lpr_sync, lpr_get_stats and lpr_bed_destroy take the batch handle; the
 * per-bed reads below take a bed index (the single-bed functions address
 * bed 0). */
lpr_status lpr_batch_create(const lpr_bed_desc* const* descs, int32_t n_beds, const lpr_allocator* alloc,
                            void* hip_stream, lpr_bed** out);
lpr_status lpr_batch_size(lpr_bed* batch, int32_t* n_beds);
lpr_status lpr_batch_get_state(lpr_bed* batch, int32_t bed, double* pos, float* vel, float* omega);
lpr_status lpr_batch_set_state(lpr_bed* batch, int32_t bed, const double* pos, const float* vel,
                               const float* omega);
lpr_status lpr_batch_get_history(lpr_bed* batch, int32_t bed, lpr_history* out, int64_t capacity,
                                 int64_t* n_total);
lpr_status lpr_batch_set_history(lpr_bed* batch, int32_t bed, const lpr_history* rec, int64_t count);
lpr_status lpr_batch_read_contacts(lpr_bed* batch, int32_t bed, lpr_contact* out, int64_t capacity,
                                   int64_t* n_total);
lpr_status lpr_batch_read_forces(lpr_bed* batch, int32_t bed, float* force, float* torque);
lpr_status lpr_batch_read_contact_loads(lpr_bed* batch, int32_t bed, lpr_contact_load* out, int64_t capacity,
                                        int64_t* n_total);
lpr_status lpr_batch_read_wall_pose(lpr_bed* batch, int32_t bed, int32_t wall, double out15[15]);
lpr_status lpr_batch_read_reaction(lpr_bed* batch, int32_t bed, int32_t body, double out6[6]);
lpr_status lpr_batch_reaction_window(lpr_bed* batch, int32_t bed, int32_t body, double sum6[6], int64_t* steps,
                                     int32_t reset);
lpr_status lpr_batch_read_body(lpr_bed* batch, int32_t bed, int32_t body, double origin[3], double vel[3]);
lpr_status lpr_batch_set_clock(lpr_bed* batch, int32_t bed, int64_t step);
lpr_status lpr_batch_get_clock(lpr_bed* batch, int32_t bed, int64_t* step);
lpr_status lpr_batch_set_body_state(lpr_bed* batch, int32_t bed, int32_t body, double z, double vz);

/* Changes the step kernel's launch shape (64/128/256 threads, persistent
 * grid or not) of a bed or batch; results are unchanged. */
lpr_status lpr_set_launch(lpr_bed* bed, int32_t block, int32_t persistent);

/* Autotuner.  Times `trial_steps` steps of throwaway copies of the beds
 * for each cell-list layout (band_ratio in {1.5, 2, 3} x cell_factor in
 * {1, 1.25}), then each launch shape (block 64/128/256, persistent or not)
 * on the fastest layout, then, radius band by radius band (cell-list level
 * q of every bed, finest first), cell factors 1.25 and 1.5 for that band
 * alone, keeping each that is faster; returns the fastest setting in *best
 * (and every trial in `trials`, up to `capacity`; *n_trials gets the count).
 * None of these choices changes the contacts found or the results. */
typedef struct {
  float band_ratio;
  float cell_factor;
  int32_t block;
  int32_t persistent;
  double ms_per_step;
  float level_cell_factor[16];  /* per radius band; 0: cell_factor */
} lpr_tuning;
lpr_status lpr_autotune(const lpr_bed_desc* const* descs, int32_t n_beds, const lpr_allocator* alloc,
                        void* hip_stream, int32_t trial_steps, lpr_tuning* best, lpr_tuning* trials,
                        int32_t capacity, int32_t* n_trials);

/* ---- adjoint --------------------------------------------------------
 * Calibration needs the sensitivity of bulk responses to the contact
 * parameters (the paper's introduction: scaled DEM models must be
 * calibrated; parameters k_n, mu_t, mu_r of its contact model).
 *
 * lpr_set_contact_params replaces (s_k, mu_t, mu_r) of every bed.
 *
 * lpr_adjoint_window steps a single bed n_steps steps from its current
 * state and returns J = (1/n_steps) sum_k R_z(k), the mean z reaction on
 * `body`, and dJ/d(s_k, mu_t, mu_r) by reverse mode: the window runs forward
 * with a checkpoint every ckpt_every steps.  Candidate lists are rebuilt at
 * each checkpoint and kept for its segment, with the bed's skin or, for a
 * bed without one, min(r_min/4, what its cell plan covers); a bed with
 * neither (rebuild_every 1 and cell_factor 1) gives LPR_E_INVAL.  If a
 * particle moves more than skin/2 within a segment, the forward restarts
 * from the window start with half the interval (one-step segments rebuild
 * every step and cannot trip); lpr_stats.adjoint_interval reports the
 * interval used.  Then, segment by segment in reverse, the
 * checkpoint is restored, the segment recomputed with its per-step inputs
 * recorded, and the hand-written vector-Jacobian products of integration,
 * accumulation, contact law and geometry run step by step, holding the
 * contact set and the Coulomb / rolling / clamp branches as the forward took
 * them.  State adjoints are FP32; parameter adjoints are summed in FP64.
 * mu_t / mu_r act on particle-particle contacts and on walls whose mu is
 * negative (they follow the bed).  The bed is left in its state after the
 * window.  Bodies must be prescribed and non-rotating (LPR_E_INVAL).
 * Device memory: about (ckpt_every + n_steps / ckpt_every) * 600 bytes per
 * particle. */
lpr_status lpr_set_contact_params(lpr_bed* bed, double s_k, double mu_t, double mu_r);
lpr_status lpr_adjoint_window(lpr_bed* bed, int64_t n_steps, int32_t ckpt_every, int32_t body, double* J,
                              double grad[3]);

/* ---- time-implicit step ----------------------------------------------
 * Section "Nonsmooth DEM and multibody dynamics": the paper steps its
 * contact laws (eq:g_n, eq:G_t, eq:G_r) with the SPOOK integrator and a
 * projected iterative solver, which lets the step exceed the contact period.
 *
 * lpr_set_stepper selects the stepper of a bed or batch:
 *   LPR_STEPPER_EXPLICIT (default): the explicit compliant step.
 *   LPR_STEPPER_SPOOK: one SPOOK step of length params.dt per call step.
 *     The gap -delta^e_H with compliance e_H / k_n and damping time
 *     tau = gamma_factor dt gives each contact a normal row on its normal
 *     impulse P >= 0; the tangential impulse lies in the Coulomb disc
 *     |p_t| <= mu_t P and the rolling impulse in |p_r| <= mu_r r* P, each
 *     removing its relative motion inside the bound and opposing it at the
 *     bound.  The rows are solved by n_iter projected block-Jacobi sweeps
 *     with mass splitting (every contact solves its own rows against masses
 *     divided by its bodies' contact counts; velocities are rebuilt from
 *     all impulses in a fixed order), in FP64; n_iter is the paper's N_it
 *     (eq:Nit).  Contacts are the pairs overlapping at the start of the
 *     step.  The history record of a contact is then its impulse on the
 *     owner over the step (xi_t) and its rolling impulse (xi_r), the warm
 *     start of the next step; lpr_read_forces gives impulses / dt, and body
 *     reactions are impulses / dt.
 *   Returns LPR_E_INVAL for an unknown kind, n_iter outside [1, 100000], a
 *   bed with candidate lists (rebuild_every > 1 or skin > 0: the implicit
 *   step searches every step) or a body with a dynamic z.  The first SPOOK
 *   selection allocates about 2.3 kB per particle (rows and impulses of 16
 *   owner slots and the walls); lpr_set_contact_params also updates the
 *   implicit step.  The adjoint window refuses an implicit bed (LPR_E_STATE). */
enum { LPR_STEPPER_EXPLICIT = 0, LPR_STEPPER_SPOOK = 1 };
lpr_status lpr_set_stepper(lpr_bed* bed, int32_t kind, int32_t n_iter);

const char* lpr_status_str(lpr_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* lpr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
