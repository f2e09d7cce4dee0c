/*
 * lpr_oracle.h -- C interface of the plain FP64 CPU oracle for the graded-bed
 * DEM contact pipeline (test infrastructure only).
 *
 * The oracle is the slow, obviously correct reference that the HIP path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or constant with
 * the HIP library under paper_2501_05300_amd/.
 *
 * What it computes (paper section "Nonsmooth DEM and multibody dynamics",
 * equations eq:momentum and eq:g_n .. eq:G_r, read as an explicit compliant
 * step):
 *   - the contact set {(i,j): |x_j - x_i|_minimum-image < r_i + r_j} plus
 *     sphere-wall contacts, each pair owned by the particle with the smaller
 *     (radius, stable id);
 *   - Hertz normal force with the paper's stiffness k_n = E* sqrt(d*) / 3 and
 *     damping gamma_n = 4.5 dt, Coulomb-capped tangential spring with history,
 *     rolling-resistance spring with history capped at mu_r r* F_n;
 *   - force/torque accumulation and semi-implicit Euler (velocity, then
 *     position, as the paper's first-order stepper orders them);
 *   - FP64 reaction force/torque on kinematic bodies (plate, ring);
 *   - a forward-mode (dual number) derivative of the mean plate reaction with
 *     respect to (stiffness scale, mu_t, mu_r).
 *
 * All arithmetic is IEEE FP64.  Particle arrays are in stable-id order.
 * Every function returns 0 on success and a negative code on error.
 */
#ifndef LPR_ORACLE_H
#define LPR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_WALL_PLANE = 0, ORC_WALL_DISK = 1, ORC_WALL_ANNULUS = 2, ORC_WALL_BOX = 3 };

typedef struct {
  double rho;          /* particle density [kg/m^3] */
  double E, nu;        /* Young's modulus [Pa], Poisson ratio */
  double mu_t, mu_r;   /* Coulomb and rolling-resistance coefficients */
  double dt;           /* time step [s] */
  double gamma_factor; /* gamma_n = gamma_factor * dt (paper: 4.5) */
  double e_H;          /* Hertz exponent of the gap function (5/4; 1 = linear) */
  double kappa_t;      /* tangential / normal stiffness ratio */
  double s_k;          /* multiplier on k_n */
  double g[3];         /* gravity [m/s^2] */
} orc_params;

typedef struct {
  int32_t kind;        /* ORC_WALL_* */
  int32_t body;        /* index of the kinematic body the wall is attached to */
  double origin[3];    /* in body coordinates (relative to the body origin) */
  double axis[3];      /* unit normal toward the particle side (plane, disk, annulus) */
  double frame[9];     /* box: three orthonormal local axes, row-major */
  double dims[3];      /* disk: R; annulus: R_in, R_out; box: half extents */
  double mu_t, mu_r;   /* friction with particles; negative = use the bed's value */
} orc_wall;

typedef struct {
  double origin[3];    /* body origin at t = 0 (world) */
  double lin_vel[3];   /* prescribed translation velocity */
  double ang_vel;      /* prescribed rotation rate about +z through the origin */
  int32_t z_free;      /* 1: z is a dynamic degree of freedom (dead weight) */
  double mass;         /* mass of a z_free body */
} orc_body;

typedef struct orc_bed orc_bed;

/* Creates an oracle bed.  pos: n*3 doubles, rad: n floats, vel/omg: n*3
 * floats (may be NULL = zero).  box: periodic lengths in x, y (z unused);
 * periodic: bit0 x, bit1 y.  Returns NULL on invalid input. */
orc_bed* orc_create(int64_t n, const double* pos, const float* rad,
                    const float* vel, const float* omg, const double box[3],
                    uint32_t periodic, const orc_params* prm, int32_t n_walls,
                    const orc_wall* walls, int32_t n_bodies, const orc_body* bodies);
void orc_destroy(orc_bed* b);

/* Overwrites positions / velocities / angular velocities (doubles, n*3). */
int orc_set_state(orc_bed* b, const double* pos, const double* vel, const double* omg);
int orc_get_state(const orc_bed* b, double* pos, double* vel, double* omg);
/* Sets the time step index k (t = k dt) and, for z_free bodies, their z and v_z. */
int orc_set_clock(orc_bed* b, int64_t step);
int orc_set_body_state(orc_bed* b, int32_t body, double z, double vz);
int orc_get_body_state(const orc_bed* b, int32_t body, double* origin3, double* vel3);

/* History records: key (owner stable id, partner code) where partner code is
 * the partner's stable id, or -1-w for wall w; value (xi_t[3], xi_r[3]). */
int64_t orc_history_count(const orc_bed* b);
int orc_get_history(const orc_bed* b, int64_t* keys2, double* vals6, int64_t cap);
int orc_set_history(orc_bed* b, int64_t count, const int64_t* keys2, const double* vals6);

/* Advances n_steps steps with the bed's stepper. */
int orc_step(orc_bed* b, int64_t n_steps);

/* Chooses the stepper: kind 0 = explicit compliant step (default); kind 1 =
 * the time-implicit SPOOK step (section "Nonsmooth DEM and multibody
 * dynamics") solved with n_iter projected block-Jacobi iterations with mass
 * splitting.  Under kind 1 the history value of a contact is the impulse on
 * its owner over the step (3 doubles) and the rolling impulse (3 doubles),
 * the last-step forces are impulses / dt, and dt is the implicit step.
 * Returns -3 for kind 1 when a body has a dynamic z, -1 for a bad kind or
 * n_iter < 1. */
int orc_set_stepper(orc_bed* b, int32_t kind, int32_t n_iter);

/* Contact set at the current state (does not step).  method 0 = O(N^2)
 * brute force, 1 = uniform grid.  Pairs (owner sid, partner code) sorted
 * ascending; *n_total receives the count. */
int orc_contact_set(const orc_bed* b, int32_t method, int64_t* pairs2, int64_t cap, int64_t* n_total);

/* Results of the last step: its contact set (sorted), the contact-only force
 * and torque on every particle, and each body's reaction (force on the body
 * from the particles, torque about the body origin). */
int orc_last_contacts(const orc_bed* b, int64_t* pairs2, int64_t cap, int64_t* n_total);
int orc_last_forces(const orc_bed* b, double* force3, double* torque3);
int orc_last_reaction(const orc_bed* b, int32_t body, double out6[6]);
/* Per contact of the last step, in orc_last_contacts order: the contact
 * force on the owner (3 doubles each), the rolling-resistance moment on the
 * owner (3) and the normal force magnitude F_n >= 0 (1).  Under the implicit
 * stepper these are impulses / dt.  Any pointer may be NULL. */
int orc_last_contact_loads(const orc_bed* b, double* force3, double* moment3, double* fn);
/* Per contact of the last explicit step, in orc_last_contacts order: the
 * summed magnitudes of the contact law's force terms (elastic and damping
 * normal terms, tangential spring and damping terms) and of its moment
 * terms (rolling spring and damping), before they combine and are capped:
 * the scales that rounding in an evaluation of the law is relative to.
 * Either pointer may be NULL. */
int orc_last_contact_scales(const orc_bed* b, double* force_terms, double* moment_terms);
/* World pose of wall `wall` at the current clock (the pose the next step
 * uses): origin (3), normal (3), the three rows of its frame (9). */
int orc_wall_pose(const orc_bed* b, int32_t wall, double out15[15]);

/* Steps n_steps with forward-mode derivatives.  J = mean over the window of
 * one reaction component on `body` (component 0-2 force x,y,z; 3-5 torque
 * x,y,z; the plate-sinkage objective is component 2); grad = dJ/d(s_k, mu_t,
 * mu_r), with mu_t and mu_r those of the bed (walls whose mu is negative
 * follow the bed).  The bed state advances as in orc_step.  Returns -3 when
 * a body has a dynamic z (derivatives through it are not provided) or the
 * bed uses the implicit stepper. */
int orc_tangent_window(orc_bed* b, int64_t n_steps, int32_t body, int32_t component, double* J,
                       double grad3[3]);

/* Number of threads the oracle's loops may use (OpenMP); returns the count in effect. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
