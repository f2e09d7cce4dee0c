// lpr_spook.h -- the time-implicit step (host side of its kernels).
//
// Section "Nonsmooth DEM and multibody dynamics": the SPOOK discretisation of
// eq:momentum with the contact laws eq:g_n, eq:G_t and eq:G_r, solved by
// projected block-Jacobi iterations with mass splitting.  The contact set,
// the owner slots and the reverse lists are the explicit step's; each contact
// keeps its impulse over the step in its history slot (the next step's warm
// start).  Every quantity of the solve is FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpr_kernels.h"

namespace lpr {

// Per-bed constants of the implicit step.
struct SpConst {
  double rho;     // particle density
  double kfac;    // s_k E* / 3 (k_n = kfac sqrt(d*))
  double eH;      // Hertz exponent of the gap
  double h;       // step
  double ups;     // 1 / (1 + 4 tau / h), tau = gamma_n
  double mu_t, mu_r;
  double g[3];
};

// Rows of one sphere-sphere contact (owner slot): unit normal owner ->
// partner, lever arms, the normal row's regularisation S and constant C,
// and the rolling bound per unit normal impulse mu_r r*.
struct SpRow {
  double nx, ny, nz, la;
  double lb, S, C, mrr;
};

// Rows of one sphere-wall contact, with the wall's velocity at the contact
// point, its spin about z and the contact point.
struct SpWRow {
  double nx, ny, nz, la;
  double S, C, mut, mrr;
  double ux, uy, uz, wz;
  double px, py, pz, pad;
};

// Impulses of one contact: normal impulse P, tangential impulse on the owner
// and rolling impulse on the owner.
struct SpImp {
  double P, tx, ty, tz;
  double rx, ry, rz, pad;
};

// Velocity iterate of one particle with its split inverse mass and inertia
// (contact count / m, contact count / I): one 64-byte read per partner.
struct SpVel {
  double vx, vy, vz, ima;
  double wx, wy, wz, iIa;
};

// Sum of impulses (force part, moment part) on one particle, or the part a
// contact gives its partner.
struct SpSum {
  double fx, fy, fz, tx, ty, tz;
};

struct SpBufs {
  SpConst* sc;      // [nbeds]
  SpRow* row;       // [K][N]
  SpImp* imp;       // [K][N]
  SpWRow* wrow;     // [nwall_max][N]
  SpImp* wimp;      // [nwall_max][N]
  SpVel* vel;       // [N]
  double2* sinv;    // [N] contact count / m, contact count / I (split inverse mass and inertia)
  SpSum* own;       // [N] impulses of a particle's owner-side contacts (slots and walls), one sweep
  SpSum* cb;        // [K][N] what each owner slot's contact gives its partner, one sweep (zero out of contact)
  uint32_t* flag;   // [N] owner slots (bits 0-15) and walls (bits 16-31) in contact
  int32_t nwall_max;
};

// Rows and warm starts of every contact at state s; reads history parity h.
void launch_sp_rows(const DevBufs& d, const SpBufs& sp, int s, int h, int l, hipStream_t st);
// Velocities from the free velocities and all impulses.  first = 1 reads
// the impulses themselves and stores the split inverse masses; later sweeps
// add the owner-side sums and the partner parts the contacts kernel wrote.
void launch_sp_vel(const DevBufs& d, const SpBufs& sp, int s, int l, int first, hipStream_t st);
// One projected block-Jacobi sweep over every contact; also writes the
// owner-side sums and the partner parts the next velocity rebuild adds.
void launch_sp_contacts(const DevBufs& d, const SpBufs& sp, int l, hipStream_t st);
// New state, history (parity h ^ 1), contact flags, force records and body
// reaction partials (blocks of SP_BS particles).
void launch_sp_finish(const DevBufs& d, const SpBufs& sp, int s, int h, int l, int record, hipStream_t st);

constexpr int SP_BS = 256;

}  // namespace lpr
