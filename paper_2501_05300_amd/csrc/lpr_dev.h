// lpr_dev.h -- device data layout, geometry and contact law of the HIP stepper.
//
// Layout in HBM (all arrays in storage order = beds back to back, each bed
// padded to a multiple of PAD particles, Morton order per radius band):
//   st[2][N]   PState (64 B)  position and radius (double4), velocity and
//              1/m (float4), angular velocity and 1/I (float4), one aligned
//              record per particle (ping-pong by step parity)
//   sid[N]     int32    stable id inside the bed
//   meta[N]    uint32   bed << 8 | level, INACTIVE for padding
//   own_idx[2][K][N] int32   owner-side candidate partners (slot-major)
//   own_cnt[2][N]    int32
//   hist[2][K][N] HRec (xi_t, xi_r); zero for a slot out of contact
//   wA[2][W][N], wB[2][W][N]  the same for walls, indexed by wall
//   cflag[2][N] uint32 bit k: owner slot k in contact; bit 16+w: wall w
//   rev_start[N+1], rev_ent[*]  reverse (partner-side) entries, packed
//                              owner << 4 | slot, per partner in ascending
//                              owner stable id
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpr {

// State of one particle: one 64-byte record, so a partner's state is a
// single aligned read.
struct PState {
  double4 x;  // x, y, z, r
  float4 v;   // velocity, 1/m
  float4 w;   // angular velocity, 1/I
};

// A search candidate in cell-list order: position (FP64), radius (the FP32
// value it was created with) and stable id, 32 bytes read as one.
struct CRec {
  double x, y, z;
  float r;
  int32_t sid;
};

// Spring history of one contact slot, 32 bytes so that the partner side of
// a contact reads it as one sector.
struct HRec {
  float4 t;  // tangential spring xi_t (w unused)
  float4 r;  // rolling spring xi_r (w unused)
};


constexpr int K = 16;            // sphere contacts per owner
constexpr int MAXW = 16;         // walls per bed
constexpr int MAXB = 4;          // bodies per bed
constexpr int PAD = 256;         // per-bed particle range alignment
constexpr int MAXLEV = 16;       // cell-list levels per bed
constexpr int ADV_CH = 32;       // chunks of the two-level reaction reduction per bed
constexpr int CPF_PAD = 8;       // readable entries past the end of the cell-ordered FP32 copy
constexpr uint32_t INACTIVE = 0xffffffffu;
constexpr int WALL_BIT = 16;

// error latch bits
constexpr uint32_t ERR_CAPACITY = 1u;
constexpr uint32_t ERR_NUMERIC = 2u;
constexpr uint32_t ERR_SKIN = 4u;
constexpr uint32_t ERR_WALL = 8u;   // a particle's centre lies beyond a plane wall by more than its radius

enum { WPLANE = 0, WDISK = 1, WANNULUS = 2, WBOX = 3 };

// One cell-list level of one bed: a dense grid over the level's slab.
struct LevelGrid {
  double lo[3];      // origin (0 on periodic axes)
  double inv_w[3];   // 1 / cell width
  double w[3];       // cell width
  int32_t n[3];      // cells per axis
  int32_t per[3];    // axis wraps
  int64_t base;      // first global cell id
  double rmax;       // largest radius binned at this level
};

// Per-bed constants.
struct BedConst {
  double L[2];
  uint32_t periodic;
  int32_t lev0, nlev;
  int32_t wall0, nwall;
  int32_t body0, nbody;
  int32_t p0, p1;        // padded particle range [p0, p1)
  float skin;
  float s_k;             // stiffness multiplier (part of kfac)
  // contact law (FP32) and integration
  float kfac;            // s_k E* / 3  (k_n = kfac sqrt(d*))
  float gn;              // gamma_n = gamma_factor dt
  float eH, kappa_t;
  float mu_t, mu_r;
  float dt;
  float g[3];
  int32_t law;           // 0: e_H = 5/4, 1: e_H = 1, 2: general
  int32_t sort_off;      // storage index of a particle minus its rank in the sorted order of all beds
  double dt_d;
};

// A wall in world coordinates at the current step.
struct WallPose {
  double o[3];
  double nu[3];
  double e[3][3];
  double dims[3];
  double c[3];       // body origin
  double vel[3];     // body translation velocity
  double omega;      // body rotation rate about +z
  float mu_t, mu_r;  // < 0: bed value
  int32_t kind;
  int32_t body;      // local body index in the bed
};

// A wall in body coordinates (as given at creation).
struct WallDef {
  double origin[3], axis[3], frame[9], dims[3];
  double mu_t, mu_r;
  int32_t kind, body;
};

// A kinematic body of a bed.
struct BodyDef {
  double origin[3], lin_vel[3], ang_vel, mass;
  int32_t z_free;
};

// Dynamic state per body.
struct BodyDyn {
  double z, vz;        // z_free bodies
  double last[6];      // reaction of the last step
  double wsum[6];      // window sums
  int64_t wsteps;
};

// Per-bed clock.
struct BedDyn {
  int64_t k;           // step index of the next step (t = k dt)
  int64_t completed;   // completed steps since creation
};

// Number of cells of an n[0] x n[1] x n[2] grid whose Morton code (bits of
// x, y, z interleaved, x lowest) is below that of cell c: the cell's rank in
// the Morton order of the grid, dense in [0, cells).  For every bit of c's
// code that is set, the cells sharing the code above that bit and having 0
// there are counted axis by axis: each axis then has some high bits fixed and
// its low bits free, and the count is the part of that range inside the grid.
// Every count is at most the grid's cell total (< 2^31), so 32-bit
// arithmetic is exact; the terms are formed for every bit and kept or not
// without branching.
__host__ __device__ inline uint32_t morton_rank(const int32_t c[3], const int32_t n[3]) {
  const uint32_t m = (uint32_t)(n[0] > n[1] ? (n[0] > n[2] ? n[0] : n[2]) : (n[1] > n[2] ? n[1] : n[2]));
  int nb = 0;
  while ((1u << nb) < m) ++nb;
  const uint32_t cx[3] = {(uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]};
  const uint32_t nx[3] = {(uint32_t)n[0], (uint32_t)n[1], (uint32_t)n[2]};
  uint32_t rank = 0;
  for (int k = nb - 1; k >= 0; --k)
    for (int a = 2; a >= 0; --a) {
      uint32_t prod = 1;
      for (int b = 0; b < 3; ++b) {
        // axes below a keep bit k free, axes above it have it fixed, axis a
        // has it fixed to 0
        const int sh = (b > a) ? k : k + 1;
        const int w = (b < a) ? k + 1 : k;
        const uint32_t lo = (cx[b] >> sh) << sh;
        const uint32_t cnt = nx[b] > lo ? nx[b] - lo : 0u;
        const uint32_t cap = 1u << w;
        prod *= cnt < cap ? cnt : cap;
      }
      rank += ((cx[a] >> k) & 1u) ? prod : 0u;
    }
  return rank;
}

// ---------------------------------------------------------------------------
// Exact FP64 geometry.  These expressions are the contact-set definition;
// contraction into FMA is disabled so that every product and sum is rounded
// as written.

__device__ __forceinline__ double image(double d, double L, bool per) {
#pragma clang fp contract(off)
  if (per) {
    const double h = 0.5 * L;
    if (d > h) return d - L;
    if (d < -h) return d + L;
  }
  return d;
}

__device__ __forceinline__ double dot3d(double ax, double ay, double az, double bx, double by, double bz) {
#pragma clang fp contract(off)
  return (ax * bx + ay * by) + az * bz;
}

// Separation owner -> partner (minimum image) and its squared length.
__device__ __forceinline__ double pair_sep(const BedConst& bc, const double4& a, const double4& b, double& dx,
                                           double& dy, double& dz) {
#pragma clang fp contract(off)
  dx = image(b.x - a.x, bc.L[0], (bc.periodic & 1u) != 0);
  dy = image(b.y - a.y, bc.L[1], (bc.periodic & 2u) != 0);
  dz = b.z - a.z;
  return (dx * dx + dy * dy) + dz * dz;
}

// Candidate test of the broad phase: d < r_a + r_b + skin.  With skin = 0 it
// is exactly sphere_touch ((ra + rb) + 0 == ra + rb).
__device__ __forceinline__ bool within_skin(double d2, double ra, double rb, double skin) {
#pragma clang fp contract(off)
  const double R = (ra + rb) + skin;
  return d2 < R * R;
}

__device__ __forceinline__ bool sphere_touch(double d2, double ra, double rb) {
#pragma clang fp contract(off)
  const double R = ra + rb;
  return d2 < R * R;
}

// Sphere-wall test: returns true on contact, with overlap delta and the unit
// normal n from the particle centre toward the wall (FP64).
__device__ __forceinline__ bool wall_geom(const WallPose& W, double x, double y, double z, double r,
                                          double& delta, double& nx, double& ny, double& nz) {
#pragma clang fp contract(off)
  const double rx = x - W.o[0], ry = y - W.o[1], rz = z - W.o[2];
  if (W.kind == WPLANE) {
    const double s = dot3d(rx, ry, rz, W.nu[0], W.nu[1], W.nu[2]);
    if (!(s < r)) return false;
    delta = r - s;
    nx = -W.nu[0]; ny = -W.nu[1]; nz = -W.nu[2];
    return true;
  }
  if (W.kind == WDISK || W.kind == WANNULUS) {
    const double s = dot3d(rx, ry, rz, W.nu[0], W.nu[1], W.nu[2]);
    if (!(s > 0.0)) return false;
    const double qx = x - s * W.nu[0], qy = y - s * W.nu[1], qz = z - s * W.nu[2];
    const double vx = qx - W.o[0], vy = qy - W.o[1], vz = qz - W.o[2];
    const double rho2 = dot3d(vx, vy, vz, vx, vy, vz);
    const double Rin = (W.kind == WDISK) ? 0.0 : W.dims[0];
    const double Rout = (W.kind == WDISK) ? W.dims[0] : W.dims[1];
    if (rho2 <= Rout * Rout && rho2 >= Rin * Rin) {
      if (!(s < r)) return false;
      delta = r - s;
      nx = -W.nu[0]; ny = -W.nu[1]; nz = -W.nu[2];
      return true;
    }
    const double Rc = (rho2 > Rout * Rout) ? Rout : Rin;
    double cx, cy, cz;
    if (rho2 > 0.0) {
      const double f = Rc / sqrt(rho2);
      cx = W.o[0] + f * vx; cy = W.o[1] + f * vy; cz = W.o[2] + f * vz;
    } else {
      cx = W.o[0] + Rc * W.e[0][0]; cy = W.o[1] + Rc * W.e[0][1]; cz = W.o[2] + Rc * W.e[0][2];
    }
    const double Dx = cx - x, Dy = cy - y, Dz = cz - z;
    const double d2 = dot3d(Dx, Dy, Dz, Dx, Dy, Dz);
    if (!(d2 < r * r)) return false;
    const double d = sqrt(d2);
    delta = r - d;
    const double id = 1.0 / d;
    nx = id * Dx; ny = id * Dy; nz = id * Dz;
    return true;
  }
  // box
  double l[3];
  bool inside = true;
  for (int a = 0; a < 3; ++a) {
    l[a] = dot3d(rx, ry, rz, W.e[a][0], W.e[a][1], W.e[a][2]);
    if (!(fabs(l[a]) < W.dims[a])) inside = false;
  }
  if (inside) {
    int best = 0;
    double bestgap = W.dims[0] - fabs(l[0]);
    for (int a = 1; a < 3; ++a) {
      const double gp = W.dims[a] - fabs(l[a]);
      if (gp < bestgap) { bestgap = gp; best = a; }
    }
    const double sg = (l[best] >= 0.0) ? 1.0 : -1.0;
    const double absl = (sg > 0.0) ? l[best] : -l[best];
    delta = r + (W.dims[best] - absl);
    nx = -sg * W.e[best][0]; ny = -sg * W.e[best][1]; nz = -sg * W.e[best][2];
    return true;
  }
  double cl[3];
  for (int a = 0; a < 3; ++a) cl[a] = (l[a] > W.dims[a]) ? W.dims[a] : ((l[a] < -W.dims[a]) ? -W.dims[a] : l[a]);
  double cx = W.o[0] + cl[0] * W.e[0][0], cy = W.o[1] + cl[0] * W.e[0][1], cz = W.o[2] + cl[0] * W.e[0][2];
  cx = cx + cl[1] * W.e[1][0]; cy = cy + cl[1] * W.e[1][1]; cz = cz + cl[1] * W.e[1][2];
  cx = cx + cl[2] * W.e[2][0]; cy = cy + cl[2] * W.e[2][1]; cz = cz + cl[2] * W.e[2][2];
  const double Dx = cx - x, Dy = cy - y, Dz = cz - z;
  const double d2 = dot3d(Dx, Dy, Dz, Dx, Dy, Dz);
  if (!(d2 < r * r)) return false;
  const double d = sqrt(d2);
  delta = r - d;
  const double id = 1.0 / d;
  nx = id * Dx; ny = id * Dy; nz = id * Dz;
  return true;
}

// ---------------------------------------------------------------------------
// Contact law (FP32), evaluated from the owner's side.

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross(float3 a, float3 b) {
  return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

struct LawIn {
  float delta;       // overlap (> 0)
  float3 n;          // unit normal owner -> partner
  float3 u;          // owner velocity relative to the partner at the contact point
  float3 wrel;       // owner angular velocity relative to the partner
  float dstar;       // effective diameter
  float mu_t, mu_r;
  float3 xt, xr;     // stored springs
};

struct LawOut {
  float3 F;          // force on the owner
  float3 Ft;         // its tangential part
  float3 M;          // rolling moment on the owner
  float3 xt, xr;     // updated springs
  float Fn;          // normal force magnitude (after the clamp at zero)
};

// Intermediates of one law evaluation: everything its vector-Jacobian
// product needs, including the branch taken at each cap and clamp.
struct LawTape {
  float kn, rstar, dd, a0, a1, Fn, kt, ct;
  bool on;            // normal force before the clamp was positive
  float3 vt;
  float xn, lp2, sc;
  float3 xp0;
  bool rot;           // stored spring was rotated into the tangent plane
  float3 xt1, Ftr;
  float capt, Ft2;
  bool slip;          // Coulomb cap active
  float kr, cr;
  float3 xr1, Mtr;
  float capr, M2;
  bool roll;          // rolling cap active
};

__device__ __forceinline__ void law_forward(const BedConst& bc, const LawIn& in, LawTape& t, LawOut& o) {
  t.kn = bc.kfac * sqrtf(in.dstar);
  t.rstar = 0.5f * in.dstar;
  t.dd = dot(in.u, in.n);
  if (bc.law == 0) {
    t.a0 = sqrtf(in.delta);
    t.a1 = in.delta * t.a0;
  } else if (bc.law == 1) {
    t.a0 = 1.0f;
    t.a1 = in.delta;
  } else {
    t.a0 = powf(in.delta, 2.0f * bc.eH - 2.0f);
    t.a1 = powf(in.delta, 2.0f * bc.eH - 1.0f);
  }
  const float Fr = t.kn * (t.a1 + bc.eH * bc.gn * t.a0 * t.dd);
  t.on = Fr > 0.0f;
  t.Fn = t.on ? Fr : 0.0f;
  // tangential spring with history, Coulomb cap
  t.kt = bc.kappa_t * (2.0f * bc.eH - 1.0f) * t.kn * t.a0;
  t.ct = bc.gn * t.kt;
  t.vt = in.u - t.dd * in.n;
  t.xn = dot(in.xt, in.n);
  t.xp0 = in.xt - t.xn * in.n;
  t.lp2 = dot(t.xp0, t.xp0);
  t.rot = t.lp2 > 0.0f;
  t.sc = t.rot ? sqrtf(dot(in.xt, in.xt) / t.lp2) : 1.0f;
  const float3 xp = t.rot ? t.sc * t.xp0 : t.xp0;
  t.xt1 = xp + bc.dt * t.vt;
  t.Ftr = (-t.kt) * t.xt1 - t.ct * t.vt;
  t.capt = in.mu_t * t.Fn;
  t.Ft2 = dot(t.Ftr, t.Ftr);
  t.slip = t.Ft2 > t.capt * t.capt;
  if (t.slip) {
    o.Ft = (t.capt * rsqrtf(t.Ft2)) * t.Ftr;
    o.xt = (-1.0f / t.kt) * (o.Ft + t.ct * t.vt);
  } else {
    o.Ft = t.Ftr;
    o.xt = t.xt1;
  }
  // rolling spring with history, rolling-resistance cap
  t.kr = t.kt * t.rstar * t.rstar;
  t.cr = bc.gn * t.kr;
  t.xr1 = in.xr + bc.dt * in.wrel;
  t.Mtr = (-t.kr) * t.xr1 - t.cr * in.wrel;
  t.capr = in.mu_r * t.rstar * t.Fn;
  t.M2 = dot(t.Mtr, t.Mtr);
  t.roll = t.M2 > t.capr * t.capr;
  if (t.roll) {
    o.M = (t.capr * rsqrtf(t.M2)) * t.Mtr;
    o.xr = (-1.0f / t.kr) * (o.M + t.cr * in.wrel);
  } else {
    o.M = t.Mtr;
    o.xr = t.xr1;
  }
  o.F = o.Ft - t.Fn * in.n;
  o.Fn = t.Fn;
}

__device__ __forceinline__ void contact_law(const BedConst& bc, const LawIn& in, LawOut& o) {
  LawTape t;
  law_forward(bc, in, t, o);
}

// Adjoints of the law's inputs.
struct LawBar {
  float delta;
  float3 n, u, wrel, xt, xr;
  float kn, mu_t, mu_r;
};

__device__ __forceinline__ float3 zero3() { return make_float3(0.f, 0.f, 0.f); }

// Vector-Jacobian product of law_forward, the branches held as taped.
// Fb, Ftb, Mb: adjoints of the outputs F, Ft, M; xtb, xrb: of the new springs.
__device__ __forceinline__ void law_vjp(const BedConst& bc, const LawIn& in, const LawTape& t, const LawOut& o,
                                        float3 Fb, float3 Ftb, float3 Mb, float3 xtb, float3 xrb, LawBar& r) {
  // F = Ft - Fn n
  Ftb = Ftb + Fb;
  float Fnb = -dot(Fb, in.n);
  float3 nb = (-t.Fn) * Fb;
  float3 ub = zero3(), wb = zero3(), vtb = zero3(), xt1b = zero3(), xr1b = zero3(), Ftrb = zero3(), Mtrb = zero3();
  float ktb = 0.f, ctb = 0.f, krb = 0.f, crb = 0.f, captb = 0.f, caprb = 0.f;
  // rolling
  if (t.roll) {
    const float ikr = 1.0f / t.kr;
    Mb = Mb - ikr * xrb;
    crb += -dot(xrb, in.wrel) * ikr;
    wb = wb + (-t.cr * ikr) * xrb;
    krb += -dot(xrb, o.xr) * ikr;
    const float Mn = sqrtf(t.M2);
    const float3 m = (1.0f / Mn) * t.Mtr;
    const float mb = dot(Mb, m);
    caprb += mb;
    Mtrb = Mtrb + (t.capr / Mn) * (Mb - mb * m);
  } else {
    xr1b = xr1b + xrb;
    Mtrb = Mtrb + Mb;
  }
  krb += -dot(Mtrb, t.xr1);
  xr1b = xr1b + (-t.kr) * Mtrb;
  crb += -dot(Mtrb, in.wrel);
  wb = wb + (-t.cr) * Mtrb;
  r.xr = xr1b;
  wb = wb + bc.dt * xr1b;
  r.mu_r = caprb * t.rstar * t.Fn;
  Fnb += caprb * in.mu_r * t.rstar;
  krb += bc.gn * crb;
  ktb += krb * t.rstar * t.rstar;
  // tangential
  if (t.slip) {
    const float ikt = 1.0f / t.kt;
    Ftb = Ftb - ikt * xtb;
    ctb += -dot(xtb, t.vt) * ikt;
    vtb = vtb + (-t.ct * ikt) * xtb;
    ktb += -dot(xtb, o.xt) * ikt;
    const float Fnrm = sqrtf(t.Ft2);
    const float3 f = (1.0f / Fnrm) * t.Ftr;
    const float fb = dot(Ftb, f);
    captb += fb;
    Ftrb = Ftrb + (t.capt / Fnrm) * (Ftb - fb * f);
  } else {
    xt1b = xt1b + xtb;
    Ftrb = Ftrb + Ftb;
  }
  ktb += -dot(Ftrb, t.xt1);
  xt1b = xt1b + (-t.kt) * Ftrb;
  ctb += -dot(Ftrb, t.vt);
  vtb = vtb + (-t.ct) * Ftrb;
  r.mu_t = captb * t.Fn;
  Fnb += captb * in.mu_t;
  const float3 xpb = xt1b;
  vtb = vtb + bc.dt * xt1b;
  float3 xp0b, xob = zero3();
  if (t.rot) {
    xp0b = t.sc * xpb;
    const float scb = dot(xpb, t.xp0);
    const float lo2b = scb / (2.0f * t.sc * t.lp2);
    const float lp2b = -scb * t.sc / (2.0f * t.lp2);
    xp0b = xp0b + (2.0f * lp2b) * t.xp0;
    xob = xob + (2.0f * lo2b) * in.xt;
  } else {
    xp0b = xpb;
  }
  xob = xob + xp0b;
  const float xnb = -dot(xp0b, in.n);
  nb = nb + (-t.xn) * xp0b;
  xob = xob + xnb * in.n;
  nb = nb + xnb * in.xt;
  r.xt = xob;
  // vt = u - dd n
  ub = ub + vtb;
  float ddb = -dot(vtb, in.n);
  nb = nb + (-t.dd) * vtb;
  ktb += bc.gn * ctb;
  const float kfe = bc.kappa_t * (2.0f * bc.eH - 1.0f);
  float knb = ktb * kfe * t.a0;
  float a0b = ktb * kfe * t.kn;
  // normal
  const float Frb = t.on ? Fnb : 0.0f;
  knb += Frb * (t.a1 + bc.eH * bc.gn * t.a0 * t.dd);
  const float a1b = Frb * t.kn;
  a0b += Frb * t.kn * bc.eH * bc.gn * t.dd;
  ddb += Frb * t.kn * bc.eH * bc.gn * t.a0;
  ub = ub + ddb * in.n;
  nb = nb + ddb * in.u;
  // a1 = delta^(2e-1), a0 = delta^(2e-2)
  r.delta = (a1b * (2.0f * bc.eH - 1.0f) * t.a1 + a0b * (2.0f * bc.eH - 2.0f) * t.a0) / in.delta;
  r.n = nb;
  r.u = ub;
  r.wrel = wb;
  r.kn = knb;
}

__device__ __forceinline__ bool owner_rule(float ri, int si, float rj, int sj) {
  return (ri < rj) || (ri == rj && si < sj);
}

}  // namespace lpr
