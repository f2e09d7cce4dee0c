// lpr_dev.h -- device data layout, geometry and contact law of the HIP stepper.
//
// Layout in HBM (all arrays in storage order = beds back to back, each bed
// padded to a multiple of PAD particles, Morton order per radius band):
//   pos[2][N]  double4  x, y, z, r             (ping-pong by step parity)
//   vel[2][N]  float4   v, 1/m
//   omg[2][N]  float4   omega, 1/I
//   sid[N]     int32    stable id inside the bed
//   meta[N]    uint32   bed << 8 | level, INACTIVE for padding
//   own_idx[2][K][N] int32   owner-side candidate partners (slot-major)
//   own_cnt[2][N]    int32
//   hA[2][K][N] float4 (xi_t, xi_r.x), hB[2][K][N] float2 (xi_r.y, xi_r.z)
//   wA[2][W][N], wB[2][W][N]  the same for walls, indexed by wall
//   cflag[2][N] uint32 bit k: owner slot k in contact; bit 16+w: wall w
//   rev_start[N+1], rev_ent[*]  reverse (partner-side) entries, packed
//                              owner << 4 | slot, ascending per partner
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpr {

constexpr int K = 16;            // sphere contacts per owner
constexpr int MAXW = 16;         // walls per bed
constexpr int MAXB = 4;          // bodies per bed
constexpr int PAD = 256;         // per-bed particle range alignment
constexpr int MAXLEV = 16;       // cell-list levels per bed
constexpr uint32_t INACTIVE = 0xffffffffu;
constexpr int WALL_BIT = 16;

// error latch bits
constexpr uint32_t ERR_CAPACITY = 1u;
constexpr uint32_t ERR_NUMERIC = 2u;
constexpr uint32_t ERR_SKIN = 4u;

enum { WPLANE = 0, WDISK = 1, WANNULUS = 2, WBOX = 3 };

// One cell-list level of one bed: a dense grid over the level's slab.
struct LevelGrid {
  double lo[3];      // origin (0 on periodic axes)
  double inv_w[3];   // 1 / cell width
  int32_t n[3];      // cells per axis
  int32_t per[3];    // axis wraps
  int64_t base;      // first global cell id
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
  float bp_tol;          // FP32 broad-phase pre-test margin [m]
  // contact law (FP32) and integration
  float kfac;            // s_k E* / 3  (k_n = kfac sqrt(d*))
  float gn;              // gamma_n = gamma_factor dt
  float eH, kappa_t;
  float mu_t, mu_r;
  float dt;
  float g[3];
  int32_t law;           // 0: e_H = 5/4, 1: e_H = 1, 2: general
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
};

__device__ __forceinline__ void contact_law(const BedConst& bc, const LawIn& in, LawOut& o) {
  const float kn = bc.kfac * sqrtf(in.dstar);
  const float rstar = 0.5f * in.dstar;
  const float dd = dot(in.u, in.n);
  float a1, a0;
  if (bc.law == 0) {
    a0 = sqrtf(in.delta);
    a1 = in.delta * a0;
  } else if (bc.law == 1) {
    a0 = 1.0f;
    a1 = in.delta;
  } else {
    a0 = powf(in.delta, 2.0f * bc.eH - 2.0f);
    a1 = powf(in.delta, 2.0f * bc.eH - 1.0f);
  }
  float Fn = kn * (a1 + bc.eH * bc.gn * a0 * dd);
  Fn = fmaxf(Fn, 0.0f);
  // tangential spring with history, Coulomb cap
  const float kt = bc.kappa_t * (2.0f * bc.eH - 1.0f) * kn * a0;
  const float ct = bc.gn * kt;
  const float3 vt = in.u - dd * in.n;
  float3 xt = in.xt;
  const float xn = dot(xt, in.n);
  float3 xp = xt - xn * in.n;
  const float lp2 = dot(xp, xp);
  if (lp2 > 0.0f) xp = sqrtf(dot(xt, xt) / lp2) * xp;
  xt = xp + bc.dt * vt;
  float3 Ft = (-kt) * xt - ct * vt;
  const float capt = in.mu_t * Fn;
  const float Ft2 = dot(Ft, Ft);
  if (Ft2 > capt * capt) {
    Ft = (capt * rsqrtf(Ft2)) * Ft;
    xt = (-1.0f / kt) * (Ft + ct * vt);
  }
  // rolling spring with history, rolling-resistance cap
  const float kr = kt * rstar * rstar;
  const float cr = bc.gn * kr;
  float3 xr = in.xr + bc.dt * in.wrel;
  float3 M = (-kr) * xr - cr * in.wrel;
  const float capr = in.mu_r * rstar * Fn;
  const float M2 = dot(M, M);
  if (M2 > capr * capr) {
    M = (capr * rsqrtf(M2)) * M;
    xr = (-1.0f / kr) * (M + cr * in.wrel);
  }
  o.F = Ft - Fn * in.n;
  o.Ft = Ft;
  o.M = M;
  o.xt = xt;
  o.xr = xr;
}

__device__ __forceinline__ bool owner_rule(float ri, int si, float rj, int sj) {
  return (ri < rj) || (ri == rj && si < sj);
}

}  // namespace lpr
