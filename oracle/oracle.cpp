// oracle.cpp -- plain FP64 CPU oracle of the graded-bed DEM step.
//
// TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
// benchmark's CPU-baseline leg are the only users.  Nothing here is shared
// with the HIP library: no header, helper, table or constant generator.
//
// The step follows the paper's model in the order the paper presents it:
//   * the contact set is recomputed every step by collision detection
//     (section "Nonsmooth DEM and multibody dynamics", text after eq:G_r);
//   * normal law from the gap function g_n = delta^{e_H}, compliance
//     e_H / k_n with k_n = E* sqrt(d*) / 3, E* and d* as defined there, and
//     damping gamma_n = 4.5 dt, read as the compliant (regularised) form of
//     eq:g_n:  F_n = max(0, k_n (delta^{2e_H-1} + e_H gamma_n delta^{2e_H-2} ddelta/dt));
//   * Coulomb cone |F_t| <= mu_t F_n (eq:G_t) and rolling cone
//     |M_r| <= mu_r r* F_n (eq:G_r), realised as springs with history
//     capped by the cones (the paper fixes the limits, not the stick law);
//   * Newton-Euler update (eq:momentum), velocity first, then position, as
//     in the paper's first-order SPOOK stepper.
// Compile with -ffp-contract=off: the contact predicate must be the plain
// IEEE expression (dx*dx + dy*dy) + dz*dz < (r_i + r_j)^2.
#include "lpr_oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Scalar types: double for the plain step, Dual for forward-mode derivatives
// with respect to (s_k, mu_t, mu_r).  Dual's value part is computed with
// exactly the operations the double path uses, so both take the same
// branches (contact set, Coulomb and rolling caps, max(0, .)).
struct Dual {
  double v;
  double d[3];
  Dual() : v(0.0), d{0.0, 0.0, 0.0} {}
  Dual(double x) : v(x), d{0.0, 0.0, 0.0} {}  // implicit on purpose
};
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int k = 0; k < 3; ++k) r.d[k] = -a.d[k];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < 3; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

inline double tsqrt(double x) { return std::sqrt(x); }
inline Dual tsqrt(const Dual& a) {
  Dual r(std::sqrt(a.v));
  for (int k = 0; k < 3; ++k) r.d[k] = (r.v > 0.0) ? a.d[k] / (2.0 * r.v) : 0.0;
  return r;
}
// a^e for a > 0
inline double tpow(double a, double e) { return std::pow(a, e); }
inline Dual tpow(const Dual& a, double e) {
  Dual r(std::pow(a.v, e));
  const double s = e * std::pow(a.v, e - 1.0);
  for (int k = 0; k < 3; ++k) r.d[k] = s * a.d[k];
  return r;
}

template <class T>
struct V3 {
  T x, y, z;
};
template <class T> inline V3<T> add(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> inline V3<T> scl(const T& s, const V3<T>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> inline T dot(const V3<T>& a, const V3<T>& b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
template <class T> inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> inline T norm(const V3<T>& a) { return tsqrt(dot(a, a)); }
template <class T> inline V3<T> neg(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T> inline V3<double> vals(const V3<T>& a) { return {val(a.x), val(a.y), val(a.z)}; }
template <class T> inline V3<T> lift(const V3<double>& a) { return {T(a.x), T(a.y), T(a.z)}; }

// World pose of one wall at the current time (values only).
struct WallPose {
  int kind;
  int body;
  V3<double> o;     // world origin
  V3<double> nu;    // world normal (plane / disk / annulus)
  V3<double> e[3];  // world axes (box; row 0 doubles as the in-plane
                    // reference direction of an annulus)
  double dims[3];
  double mu_t, mu_r;  // < 0: the bed's value
};

// World pose of a kinematic body at the current time.
struct BodyPose {
  V3<double> c;    // origin
  V3<double> vel;  // translation velocity
  double omega;    // rotation rate about +z
  double theta;    // rotation angle about +z
};

struct Contact {
  int64_t owner;    // particle index (= stable id)
  int64_t partner;  // particle index, or -1-w for wall w
};

using Hist = std::array<double, 6>;

template <class T>
struct State {
  std::vector<V3<T>> x, v, w;
  std::vector<std::vector<int64_t>> hkey;         // per owner, partner codes ascending
  std::vector<std::vector<std::array<T, 6>>> hval;  // per owner, (xi_t, xi_r)
  T s_k, mu_t, mu_r;
};

}  // namespace

struct orc_bed {
  int64_t n = 0;
  double L[2] = {0.0, 0.0};
  uint32_t periodic = 0;
  orc_params p{};
  std::vector<orc_wall> walls;
  std::vector<orc_body> bodies;
  std::vector<double> r, m, I;
  State<double> st;
  int64_t k = 0;                // step index, t = k dt
  std::vector<double> bz, bvz;  // z_free bodies: origin z and v_z
  std::vector<Contact> last_contacts;
  std::vector<double> lastF, lastT, lastR;
  // per contact of the last step, in last_contacts order: force on the
  // owner (3), rolling moment on the owner (3), normal force magnitude
  std::vector<double> lastCF, lastCM, lastCN;
  // per contact of the last step: the summed magnitudes of the law's force
  // terms (elastic, damping, tangential spring and damping) and of its
  // moment terms (rolling spring and damping) before they combine
  std::vector<double> lastCSF, lastCSM;
  int stepper = 0;      // 0: explicit compliant step, 1: SPOOK with projected iterations
  int n_iter = 0;       // projected iterations per SPOOK step
};

namespace {

// ---------------------------------------------------------------------------
// Geometry.

// Owner rule: the pair belongs to the particle with the smaller (radius, id).
inline bool owns(const orc_bed& b, int64_t i, int64_t j) {
  return (b.r[i] < b.r[j]) || (b.r[i] == b.r[j] && i < j);
}

// Minimum-image shift decision: shift by -L when d > L/2, +L when d < -L/2.
inline double image_shift(double d, double L) {
  const double h = 0.5 * L;
  if (d > h) return -L;
  if (d < -h) return L;
  return 0.0;
}

// Sphere-sphere predicate on FP64 values (the contact-set definition).
inline bool sphere_contact(const orc_bed& b, const V3<double>& xi, double ri,
                           const V3<double>& xj, double rj) {
  double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
  if (b.periodic & 1u) dx = dx + image_shift(dx, b.L[0]);
  if (b.periodic & 2u) dy = dy + image_shift(dy, b.L[1]);
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double R = ri + rj;
  return d2 < R * R;
}

V3<double> rot_z(const V3<double>& a, double c, double s) {
  return {a.x * c - a.y * s, a.x * s + a.y * c, a.z};
}

std::vector<BodyPose> body_poses(const orc_bed& b, double t) {
  std::vector<BodyPose> out(b.bodies.size());
  for (size_t q = 0; q < b.bodies.size(); ++q) {
    const orc_body& B = b.bodies[q];
    BodyPose P;
    P.c = {B.origin[0] + B.lin_vel[0] * t, B.origin[1] + B.lin_vel[1] * t, B.origin[2] + B.lin_vel[2] * t};
    P.vel = {B.lin_vel[0], B.lin_vel[1], B.lin_vel[2]};
    if (B.z_free) {
      P.c.z = b.bz[q];
      P.vel.z = b.bvz[q];
    }
    P.omega = B.ang_vel;
    P.theta = B.ang_vel * t;
    out[q] = P;
  }
  return out;
}

std::vector<WallPose> wall_poses(const orc_bed& b, const std::vector<BodyPose>& bp) {
  std::vector<WallPose> out(b.walls.size());
  for (size_t q = 0; q < b.walls.size(); ++q) {
    const orc_wall& W = b.walls[q];
    const BodyPose& P = bp[W.body];
    const double c = std::cos(P.theta), s = std::sin(P.theta);
    WallPose o;
    o.kind = W.kind;
    o.body = W.body;
    o.o = add(P.c, rot_z({W.origin[0], W.origin[1], W.origin[2]}, c, s));
    o.nu = rot_z({W.axis[0], W.axis[1], W.axis[2]}, c, s);
    for (int a = 0; a < 3; ++a)
      o.e[a] = rot_z({W.frame[3 * a + 0], W.frame[3 * a + 1], W.frame[3 * a + 2]}, c, s);
    for (int a = 0; a < 3; ++a) o.dims[a] = W.dims[a];
    o.mu_t = W.mu_t;
    o.mu_r = W.mu_r;
    out[q] = o;
  }
  return out;
}

// Sphere-wall geometry: contact flag (decided on values), overlap delta and
// unit normal n pointing from the particle centre toward the wall.
template <class T>
bool wall_geom(const WallPose& W, const V3<T>& x, double r, T* delta, V3<T>* n) {
  const V3<T> o = lift<T>(W.o);
  if (W.kind == ORC_WALL_PLANE) {
    const T s = dot(sub(x, o), lift<T>(W.nu));
    if (!(val(s) < r)) return false;
    *delta = T(r) - s;
    *n = lift<T>(neg(W.nu));
    return true;
  }
  if (W.kind == ORC_WALL_DISK || W.kind == ORC_WALL_ANNULUS) {
    const V3<T> nu = lift<T>(W.nu);
    const T s = dot(sub(x, o), nu);
    if (!(val(s) > 0.0)) return false;  // one-sided: centre must be in front
    const V3<T> q = sub(x, scl(s, nu));
    const V3<T> rv = sub(q, o);
    const T rho2 = dot(rv, rv);
    const double Rin = (W.kind == ORC_WALL_DISK) ? 0.0 : W.dims[0];
    const double Rout = (W.kind == ORC_WALL_DISK) ? W.dims[0] : W.dims[1];
    if (val(rho2) <= Rout * Rout && val(rho2) >= Rin * Rin) {  // face
      if (!(val(s) < r)) return false;
      *delta = T(r) - s;
      *n = lift<T>(neg(W.nu));
      return true;
    }
    const double Rc = (val(rho2) > Rout * Rout) ? Rout : Rin;  // rim circle
    V3<T> c;
    if (val(rho2) > 0.0) {
      const T rho = tsqrt(rho2);
      c = add(o, scl(T(Rc) / rho, rv));
    } else {
      c = add(o, scl(T(Rc), lift<T>(W.e[0])));
    }
    const V3<T> D = sub(c, x);
    const T d2 = dot(D, D);
    if (!(val(d2) < r * r)) return false;
    const T d = tsqrt(d2);
    *delta = T(r) - d;
    *n = scl(T(1.0) / d, D);
    return true;
  }
  // box
  const V3<T> rel = sub(x, o);
  T l[3];
  bool inside = true;
  for (int a = 0; a < 3; ++a) {
    l[a] = dot(rel, lift<T>(W.e[a]));
    if (!(std::fabs(val(l[a])) < W.dims[a])) inside = false;
  }
  if (inside) {
    int best = 0;
    double bestgap = W.dims[0] - std::fabs(val(l[0]));
    for (int a = 1; a < 3; ++a) {
      const double g = W.dims[a] - std::fabs(val(l[a]));
      if (g < bestgap) { bestgap = g; best = a; }
    }
    const double sg = (val(l[best]) >= 0.0) ? 1.0 : -1.0;
    const T absl = (sg > 0.0) ? l[best] : -l[best];
    *delta = T(r) + (T(W.dims[best]) - absl);
    *n = lift<T>(scl(-sg, W.e[best]));
    return true;
  }
  T cl[3];
  for (int a = 0; a < 3; ++a) {
    if (val(l[a]) > W.dims[a]) cl[a] = T(W.dims[a]);
    else if (val(l[a]) < -W.dims[a]) cl[a] = T(-W.dims[a]);
    else cl[a] = l[a];
  }
  V3<T> c = add(o, scl(cl[0], lift<T>(W.e[0])));
  c = add(c, scl(cl[1], lift<T>(W.e[1])));
  c = add(c, scl(cl[2], lift<T>(W.e[2])));
  const V3<T> D = sub(c, x);
  const T d2 = dot(D, D);
  if (!(val(d2) < r * r)) return false;
  const T d = tsqrt(d2);
  *delta = T(r) - d;
  *n = scl(T(1.0) / d, D);
  return true;
}

// ---------------------------------------------------------------------------
// Contact detection on FP64 values.

void brute_pairs(const orc_bed& b, const std::vector<V3<double>>& x, std::vector<Contact>* out) {
  for (int64_t i = 0; i < b.n; ++i)
    for (int64_t j = i + 1; j < b.n; ++j) {
      if (!sphere_contact(b, x[i], b.r[i], x[j], b.r[j])) continue;
      if (owns(b, i, j)) out->push_back({i, j});
      else out->push_back({j, i});
    }
}

// Uniform grid, cell edge >= 2 r_max, 27-cell search with de-duplicated
// periodic neighbours.
void grid_pairs(const orc_bed& b, const std::vector<V3<double>>& x, std::vector<Contact>* out) {
  double rmax = 0.0;
  for (int64_t i = 0; i < b.n; ++i) rmax = std::max(rmax, b.r[i]);
  const double h = 2.0 * rmax;
  int64_t nc[3];
  double w[3], lo[3];
  bool per[3] = {(b.periodic & 1u) != 0, (b.periodic & 2u) != 0, false};
  for (int a = 0; a < 3; ++a) {
    if (per[a]) {
      nc[a] = std::max<int64_t>(1, (int64_t)std::floor(b.L[a] / h));
      w[a] = b.L[a] / (double)nc[a];
      lo[a] = 0.0;
    } else {
      double mn = 1e300, mx = -1e300;
      for (int64_t i = 0; i < b.n; ++i) {
        const double c = (a == 0) ? x[i].x : (a == 1) ? x[i].y : x[i].z;
        mn = std::min(mn, c);
        mx = std::max(mx, c);
      }
      lo[a] = mn;
      w[a] = h;
      nc[a] = (int64_t)std::floor((mx - mn) / h) + 1;
    }
  }
  auto cell_of = [&](const V3<double>& p, int a) {
    const double c = (a == 0) ? p.x : (a == 1) ? p.y : p.z;
    int64_t k = (int64_t)std::floor((c - lo[a]) / w[a]);
    if (k < 0) k = 0;
    if (k > nc[a] - 1) k = nc[a] - 1;
    return k;
  };
  const int64_t ncell = nc[0] * nc[1] * nc[2];
  std::vector<std::vector<int64_t>> cells((size_t)ncell);
  std::vector<int64_t> cid((size_t)b.n);
  for (int64_t i = 0; i < b.n; ++i) {
    const int64_t c = (cell_of(x[i], 2) * nc[1] + cell_of(x[i], 1)) * nc[0] + cell_of(x[i], 0);
    cid[i] = c;
    cells[c].push_back(i);
  }
  std::vector<std::vector<Contact>> per_owner((size_t)b.n);
#pragma omp parallel for schedule(dynamic, 256) if (b.n > 4096)
  for (int64_t i = 0; i < b.n; ++i) {
    int64_t ci[3] = {cell_of(x[i], 0), cell_of(x[i], 1), cell_of(x[i], 2)};
    std::vector<int64_t> nb[3];
    for (int a = 0; a < 3; ++a) {
      for (int d = -1; d <= 1; ++d) {
        int64_t c = ci[a] + d;
        if (per[a]) c = ((c % nc[a]) + nc[a]) % nc[a];
        else if (c < 0 || c >= nc[a]) continue;
        if (std::find(nb[a].begin(), nb[a].end(), c) == nb[a].end()) nb[a].push_back(c);
      }
    }
    for (int64_t cz : nb[2])
      for (int64_t cy : nb[1])
        for (int64_t cx : nb[0])
          for (int64_t j : cells[(cz * nc[1] + cy) * nc[0] + cx]) {
            if (j == i || !owns(b, i, j)) continue;
            if (sphere_contact(b, x[i], b.r[i], x[j], b.r[j])) per_owner[i].push_back({i, j});
          }
  }
  for (auto& v : per_owner) out->insert(out->end(), v.begin(), v.end());
}

void wall_contacts(const orc_bed& b, const std::vector<V3<double>>& x, const std::vector<WallPose>& wp,
                   std::vector<Contact>* out) {
  for (int64_t i = 0; i < b.n; ++i)
    for (size_t q = 0; q < wp.size(); ++q) {
      double dl;
      V3<double> nn;
      if (wall_geom<double>(wp[q], x[i], b.r[i], &dl, &nn)) out->push_back({i, -1 - (int64_t)q});
    }
}

bool contact_less(const Contact& a, const Contact& c) {
  return (a.owner < c.owner) || (a.owner == c.owner && a.partner < c.partner);
}

std::vector<Contact> detect(const orc_bed& b, const std::vector<V3<double>>& x, const std::vector<WallPose>& wp,
                            int method) {
  std::vector<Contact> cs;
  if (method == 0) brute_pairs(b, x, &cs);
  else grid_pairs(b, x, &cs);
  wall_contacts(b, x, wp, &cs);
  std::sort(cs.begin(), cs.end(), contact_less);
  return cs;
}

// ---------------------------------------------------------------------------
// Contact law for one contact, evaluated from the owner's side.

template <class T>
struct LawOut {
  V3<T> Fi;        // force on the owner
  V3<T> Ti;        // torque on the owner
  V3<T> Tj;        // torque on the partner particle (sphere-sphere)
  V3<T> Mr;        // rolling-resistance moment on the owner
  V3<T> p;         // contact point (world, owner's image frame)
  T Fn;            // normal force magnitude (after the clamp at zero)
  double sF, sM;   // magnitudes of the law's force and moment terms
  std::array<T, 6> xi;
};

template <class T>
struct LawIn {
  T delta;          // overlap
  V3<T> n;          // unit normal owner -> partner
  V3<T> u;          // velocity of owner relative to partner at the contact point
  V3<T> wrel;       // angular velocity of owner relative to partner
  double dstar;     // effective diameter
  T mu_t, mu_r;
  std::array<T, 6> xi_old;
};

template <class T>
void contact_law(const orc_params& p, const T& s_k, const LawIn<T>& in, V3<T>* F_out, V3<T>* M_out,
                 std::array<T, 6>* xi_new, T* Fn_out, double* scale_F, double* scale_M) {
  const double eH = p.e_H;
  const double Estar = 1.0 / ((1.0 - p.nu * p.nu) / p.E + (1.0 - p.nu * p.nu) / p.E);
  const double rstar = 0.5 * in.dstar;
  const T kn = s_k * T(Estar * std::sqrt(in.dstar) / 3.0);
  const double gn = p.gamma_factor * p.dt;
  const T ddelta = dot(in.u, in.n);
  // normal: F_n = max(0, k_n (delta^{2e-1} + e gamma_n delta^{2e-2} ddelta))
  const T a1 = tpow(in.delta, 2.0 * eH - 1.0);
  const T a0 = (eH == 1.0) ? T(1.0) : tpow(in.delta, 2.0 * eH - 2.0);
  T Fn = kn * (a1 + T(eH * gn) * a0 * ddelta);
  if (val(Fn) < 0.0) Fn = T(0.0);
  // tangential spring: k_t = kappa_t dF_n/ddelta (elastic part), c_t = gamma_n k_t
  const T Kn = T(2.0 * eH - 1.0) * kn * a0;
  const T kt = T(p.kappa_t) * Kn;
  const T ct = T(gn) * kt;
  const V3<T> vt = sub(in.u, scl(ddelta, in.n));
  V3<T> xt = {in.xi_old[0], in.xi_old[1], in.xi_old[2]};
  // rotate the stored spring into the current tangent plane, keep its length
  const T xn = dot(xt, in.n);
  V3<T> xp = sub(xt, scl(xn, in.n));
  const T len_old = norm(xt), len_p = norm(xp);
  if (val(len_p) > 0.0) xp = scl(len_old / len_p, xp);
  xt = add(xp, scl(T(p.dt), vt));
  V3<T> Ft = sub(scl(-kt, xt), scl(ct, vt));
  *scale_F = std::fabs(val(kn * a1)) + std::fabs(val(kn * T(eH * gn) * a0 * ddelta)) + val(kt) * val(norm(xt)) +
             val(ct) * val(norm(vt));
  const T Ftn = norm(Ft);
  const T capt = in.mu_t * Fn;
  if (val(Ftn) > val(capt)) {
    Ft = scl(capt / Ftn, Ft);
    xt = scl(T(-1.0) / kt, add(Ft, scl(ct, vt)));
  }
  // rolling spring: k_r = k_t r*^2, c_r = gamma_n k_r, cap mu_r r* F_n
  const T kr = kt * T(rstar * rstar);
  const T cr = T(gn) * kr;
  V3<T> xr = {in.xi_old[3], in.xi_old[4], in.xi_old[5]};
  xr = add(xr, scl(T(p.dt), in.wrel));
  V3<T> Mr = sub(scl(-kr, xr), scl(cr, in.wrel));
  *scale_M = val(kr) * val(norm(xr)) + val(cr) * val(norm(in.wrel));
  const T Mrn = norm(Mr);
  const T capr = in.mu_r * T(rstar) * Fn;
  if (val(Mrn) > val(capr)) {
    Mr = scl(capr / Mrn, Mr);
    xr = scl(T(-1.0) / kr, add(Mr, scl(cr, in.wrel)));
  }
  *F_out = add(scl(-Fn, in.n), Ft);
  *M_out = Mr;
  *xi_new = {xt.x, xt.y, xt.z, xr.x, xr.y, xr.z};
  *Fn_out = Fn;
}

template <class T>
std::array<T, 6> lookup_hist(const State<T>& S, int64_t owner, int64_t code) {
  const auto& keys = S.hkey[owner];
  auto it = std::lower_bound(keys.begin(), keys.end(), code);
  if (it != keys.end() && *it == code) return S.hval[owner][it - keys.begin()];
  return {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
}

template <class T>
LawOut<T> eval_contact(const orc_bed& b, const State<T>& S, const std::vector<WallPose>& wp,
                       const std::vector<BodyPose>& bp, const Contact& c) {
  const int64_t i = c.owner;
  const double ri = b.r[i];
  LawIn<T> in;
  LawOut<T> out;
  in.xi_old = lookup_hist(S, i, c.partner);
  if (c.partner >= 0) {
    const int64_t j = c.partner;
    const double rj = b.r[j];
    // separation to the nearest periodic image of j
    V3<T> D = sub(S.x[j], S.x[i]);
    if (b.periodic & 1u) D.x = D.x + T(image_shift(val(D.x), b.L[0]));
    if (b.periodic & 2u) D.y = D.y + T(image_shift(val(D.y), b.L[1]));
    const T d2 = dot(D, D);
    T d = tsqrt(d2);
    V3<T> n;
    if (val(d2) > 0.0) n = scl(T(1.0) / d, D);
    else n = {T(0.0), T(0.0), T(1.0)};
    in.delta = T(ri + rj) - d;
    in.n = n;
    const V3<T> ai = scl(T(ri) - T(0.5) * in.delta, n);  // contact point - x_i
    const V3<T> aj = sub(ai, D);                         // contact point - x_j (image)
    const V3<T> ui = add(S.v[i], cross(S.w[i], ai));
    const V3<T> uj = add(S.v[j], cross(S.w[j], aj));
    in.u = sub(ui, uj);
    in.wrel = sub(S.w[i], S.w[j]);
    in.dstar = 2.0 * ri * rj / (ri + rj);
    in.mu_t = S.mu_t;
    in.mu_r = S.mu_r;
    V3<T> F, M;
    contact_law(b.p, S.s_k, in, &F, &M, &out.xi, &out.Fn, &out.sF, &out.sM);
    out.Fi = F;
    out.Mr = M;
    out.Ti = add(cross(ai, F), M);
    out.Tj = sub(cross(aj, neg(F)), M);
    out.p = add(S.x[i], ai);
    return out;
  }
  const int64_t wq = -1 - c.partner;
  const WallPose& W = wp[wq];
  const BodyPose& P = bp[W.body];
  T delta;
  V3<T> n;
  wall_geom<T>(W, S.x[i], ri, &delta, &n);
  in.delta = delta;
  in.n = n;
  const V3<T> ai = scl(T(ri) - T(0.5) * delta, n);
  const V3<T> pnt = add(S.x[i], ai);
  const V3<T> Omega = {T(0.0), T(0.0), T(P.omega)};
  const V3<T> uw = add(lift<T>(P.vel), cross(Omega, sub(pnt, lift<T>(P.c))));
  in.u = sub(add(S.v[i], cross(S.w[i], ai)), uw);
  in.wrel = sub(S.w[i], Omega);
  in.dstar = 2.0 * ri;
  in.mu_t = (W.mu_t < 0.0) ? S.mu_t : T(W.mu_t);
  in.mu_r = (W.mu_r < 0.0) ? S.mu_r : T(W.mu_r);
  V3<T> F, M;
  contact_law(b.p, S.s_k, in, &F, &M, &out.xi, &out.Fn, &out.sF, &out.sM);
  out.Fi = F;
  out.Mr = M;
  out.Ti = add(cross(ai, F), M);
  out.Tj = {T(0.0), T(0.0), T(0.0)};
  out.p = pnt;
  return out;
}

// One step.  Fills the bed's last_* records.  Returns component `comp`
// (0-2 force, 3-5 torque) of the reaction on `rbody` (zero when rbody < 0).
template <class T>
T step_once(orc_bed& b, State<T>& S, int rbody, int comp = 2) {
  const double t = (double)b.k * b.p.dt;
  const std::vector<BodyPose> bp = body_poses(b, t);
  const std::vector<WallPose> wp = wall_poses(b, bp);
  std::vector<V3<double>> xv((size_t)b.n);
  for (int64_t i = 0; i < b.n; ++i) xv[i] = vals(S.x[i]);
  std::vector<Contact> cs = detect(b, xv, wp, b.n <= 4096 ? 0 : 1);

  const int64_t nc = (int64_t)cs.size();
  std::vector<LawOut<T>> lo((size_t)nc);
#pragma omp parallel for schedule(dynamic, 1024) if (nc > 4096)
  for (int64_t q = 0; q < nc; ++q) lo[q] = eval_contact(b, S, wp, bp, cs[q]);

  const V3<T> zero = {T(0.0), T(0.0), T(0.0)};
  std::vector<V3<T>> F((size_t)b.n, zero), Tq((size_t)b.n, zero);
  const size_t nb = b.bodies.size();
  std::vector<V3<T>> RF(nb, zero), RT(nb, zero);
  for (int64_t q = 0; q < nc; ++q) {
    const Contact& c = cs[q];
    F[c.owner] = add(F[c.owner], lo[q].Fi);
    Tq[c.owner] = add(Tq[c.owner], lo[q].Ti);
    if (c.partner >= 0) {
      F[c.partner] = sub(F[c.partner], lo[q].Fi);
      Tq[c.partner] = add(Tq[c.partner], lo[q].Tj);
    } else {
      const int body = wp[-1 - c.partner].body;
      const V3<T> Fw = neg(lo[q].Fi);
      RF[body] = add(RF[body], Fw);
      RT[body] = add(RT[body], sub(cross(sub(lo[q].p, lift<T>(bp[body].c)), Fw), lo[q].Mr));
    }
  }
  // new history: only contacts found this step survive
  std::vector<std::vector<int64_t>> nk((size_t)b.n);
  std::vector<std::vector<std::array<T, 6>>> nv((size_t)b.n);
  for (int64_t q = 0; q < nc; ++q) {
    nk[cs[q].owner].push_back(cs[q].partner);
    nv[cs[q].owner].push_back(lo[q].xi);
  }
  S.hkey.swap(nk);
  S.hval.swap(nv);
  // record
  b.last_contacts = cs;
  b.lastF.assign((size_t)(3 * b.n), 0.0);
  b.lastT.assign((size_t)(3 * b.n), 0.0);
  for (int64_t i = 0; i < b.n; ++i) {
    b.lastF[3 * i + 0] = val(F[i].x); b.lastF[3 * i + 1] = val(F[i].y); b.lastF[3 * i + 2] = val(F[i].z);
    b.lastT[3 * i + 0] = val(Tq[i].x); b.lastT[3 * i + 1] = val(Tq[i].y); b.lastT[3 * i + 2] = val(Tq[i].z);
  }
  b.lastCF.assign((size_t)(3 * nc), 0.0);
  b.lastCM.assign((size_t)(3 * nc), 0.0);
  b.lastCN.assign((size_t)nc, 0.0);
  b.lastCSF.assign((size_t)nc, 0.0);
  b.lastCSM.assign((size_t)nc, 0.0);
  for (int64_t q = 0; q < nc; ++q) {
    b.lastCSF[q] = lo[q].sF;
    b.lastCSM[q] = lo[q].sM;
    b.lastCF[3 * q + 0] = val(lo[q].Fi.x); b.lastCF[3 * q + 1] = val(lo[q].Fi.y); b.lastCF[3 * q + 2] = val(lo[q].Fi.z);
    b.lastCM[3 * q + 0] = val(lo[q].Mr.x); b.lastCM[3 * q + 1] = val(lo[q].Mr.y); b.lastCM[3 * q + 2] = val(lo[q].Mr.z);
    b.lastCN[q] = val(lo[q].Fn);
  }
  b.lastR.assign(6 * nb, 0.0);
  for (size_t q = 0; q < nb; ++q) {
    b.lastR[6 * q + 0] = val(RF[q].x); b.lastR[6 * q + 1] = val(RF[q].y); b.lastR[6 * q + 2] = val(RF[q].z);
    b.lastR[6 * q + 3] = val(RT[q].x); b.lastR[6 * q + 4] = val(RT[q].y); b.lastR[6 * q + 5] = val(RT[q].z);
  }
  // semi-implicit Euler: v first, then x with the new v; wrap periodic axes
  const double dt = b.p.dt;
  const V3<T> g = {T(b.p.g[0]), T(b.p.g[1]), T(b.p.g[2])};
#pragma omp parallel for schedule(static) if (b.n > 4096)
  for (int64_t i = 0; i < b.n; ++i) {
    const V3<T> a = add(scl(T(1.0 / b.m[i]), F[i]), g);
    S.v[i] = add(S.v[i], scl(T(dt), a));
    S.w[i] = add(S.w[i], scl(T(dt / b.I[i]), Tq[i]));
    S.x[i] = add(S.x[i], scl(T(dt), S.v[i]));
    if (b.periodic & 1u) {
      if (val(S.x[i].x) >= b.L[0]) S.x[i].x = S.x[i].x - T(b.L[0]);
      else if (val(S.x[i].x) < 0.0) S.x[i].x = S.x[i].x + T(b.L[0]);
    }
    if (b.periodic & 2u) {
      if (val(S.x[i].y) >= b.L[1]) S.x[i].y = S.x[i].y - T(b.L[1]);
      else if (val(S.x[i].y) < 0.0) S.x[i].y = S.x[i].y + T(b.L[1]);
    }
  }
  // dead-weight bodies: m z'' = R_z + m g_z (semi-implicit)
  for (size_t q = 0; q < nb; ++q) {
    if (!b.bodies[q].z_free) continue;
    b.bvz[q] = b.bvz[q] + dt * (val(RF[q].z) / b.bodies[q].mass + b.p.g[2]);
    b.bz[q] = b.bz[q] + dt * b.bvz[q];
  }
  b.k += 1;
  if (rbody < 0) return T(0.0);
  const V3<T>& R = (comp < 3) ? RF[rbody] : RT[rbody];
  const int c = comp % 3;
  return (c == 0) ? R.x : (c == 1) ? R.y : R.z;
}

// ---------------------------------------------------------------------------
// Time-implicit stepper (section "Nonsmooth DEM and multibody dynamics"): the
// SPOOK discretisation of eq:momentum with the contact laws eq:g_n, eq:G_t and
// eq:G_r, solved by projected block-Jacobi iterations with mass splitting.
//
// Step of length h.  Start velocities v0, free velocities v* = v0 + h g; the
// new velocities are v+ = v* + M^-1 (sum of contact impulses).  A contact
// between a and b (b may be a wall) has unit normal n (a toward b), overlap
// delta > 0 and lever arms l_a = r_a - delta/2, l_b = r_b - delta/2; u is the
// velocity of a relative to b at the contact point and u_n = u . n.
//   normal:  0 <= -u_n(v+) + S P + C  perp  P >= 0, with
//            S = 4 / (k_n e_H h^2 (1 + 4 tau/h) delta^(2 e_H - 2)),
//            C = (u_n(v0) - 4 delta / (e_H h)) / (1 + 4 tau/h), tau = gamma_n.
//            This is the SPOOK row of the gap -delta^e_H with compliance
//            e_H / k_n, divided by its Jacobian scale e_H delta^(e_H - 1) so
//            that the multiplier P is the normal impulse.
//   tangent: u_t(v+) = 0 while |p_t| < mu_t P; at |p_t| = mu_t P, p_t opposes u_t.
//   rolling: w_a - w_b = 0 while |p_r| < mu_r r* P; at the bound p_r opposes it.
// The impulse on a is -P n + p_t at the contact point plus the moment p_r; b
// receives the opposite.
//
// Iteration: every contact, from the velocities of the previous iteration,
// solves its own rows one after another (normal, tangent, rolling) against
// its two bodies with masses and inertias divided by their contact counts,
// then the velocities are rebuilt from v* and all impulses.  Fixed points
// satisfy the conditions above.  The history of a contact is its impulse on
// a (-P n + p_t) and p_r, the warm start of the next step.

struct SpC {
  int64_t a, b;            // b < 0: wall -1-b
  V3<double> n;
  double la, lb;
  double S, C;
  double mu_t, mrr;        // mu_t and mu_r r*
  V3<double> uw, ww;       // wall: velocity at the contact point, angular velocity
  V3<double> pc;           // contact point
  int body;
  double P;
  V3<double> pt, pr;
};

inline V3<double> rel_vel(const SpC& c, const V3<double>& va, const V3<double>& wa, const V3<double>& vb,
                          const V3<double>& wb) {
  const V3<double> ua = add(va, scl(c.la, cross(wa, c.n)));
  if (c.b < 0) return sub(ua, c.uw);
  return add(sub(ua, vb), scl(c.lb, cross(wb, c.n)));
}

void spook_step(orc_bed& b) {
  State<double>& S = b.st;
  const double h = b.p.dt;
  const double t = (double)b.k * h;
  const std::vector<BodyPose> bp = body_poses(b, t);
  const std::vector<WallPose> wp = wall_poses(b, bp);
  std::vector<Contact> cs = detect(b, S.x, wp, b.n <= 4096 ? 0 : 1);
  const int64_t nc = (int64_t)cs.size();
  const double eH = b.p.e_H;
  const double Estar = 1.0 / ((1.0 - b.p.nu * b.p.nu) / b.p.E + (1.0 - b.p.nu * b.p.nu) / b.p.E);
  const double tau = b.p.gamma_factor * h;
  const double ups = 1.0 / (1.0 + 4.0 * tau / h);
  std::vector<int64_t> deg((size_t)b.n, 0);
  std::vector<SpC> C((size_t)nc);
  for (int64_t q = 0; q < nc; ++q) {
    const Contact& ct = cs[q];
    SpC& c = C[q];
    const int64_t i = ct.owner;
    c.a = i;
    c.b = ct.partner;
    const double ri = b.r[i];
    double delta, dstar;
    if (ct.partner >= 0) {
      const int64_t j = ct.partner;
      V3<double> D = sub(S.x[j], S.x[i]);
      if (b.periodic & 1u) D.x = D.x + image_shift(D.x, b.L[0]);
      if (b.periodic & 2u) D.y = D.y + image_shift(D.y, b.L[1]);
      const double dd = norm(D);
      c.n = (dd > 0.0) ? scl(1.0 / dd, D) : V3<double>{0.0, 0.0, 1.0};
      delta = (ri + b.r[j]) - dd;
      dstar = 2.0 * ri * b.r[j] / (ri + b.r[j]);
      c.la = ri - 0.5 * delta;
      c.lb = b.r[j] - 0.5 * delta;
      c.mu_t = S.mu_t;
      c.mrr = S.mu_r * 0.5 * dstar;
      c.body = -1;
      deg[j] += 1;
    } else {
      const WallPose& W = wp[-1 - ct.partner];
      const BodyPose& Pb = bp[W.body];
      wall_geom<double>(W, S.x[i], ri, &delta, &c.n);
      dstar = 2.0 * ri;
      c.la = ri - 0.5 * delta;
      c.lb = 0.0;
      c.pc = add(S.x[i], scl(c.la, c.n));
      const V3<double> Om = {0.0, 0.0, Pb.omega};
      c.uw = add(Pb.vel, cross(Om, sub(c.pc, Pb.c)));
      c.ww = Om;
      c.mu_t = (W.mu_t < 0.0) ? S.mu_t : W.mu_t;
      c.mrr = ((W.mu_r < 0.0) ? S.mu_r : W.mu_r) * 0.5 * dstar;
      c.body = W.body;
    }
    deg[i] += 1;
    const double kn = S.s_k * Estar * std::sqrt(dstar) / 3.0;
    // an overlap that rounds to zero has no stiffness: its row cannot push
    c.S = (delta > 0.0) ? 4.0 / (kn * eH * h * h * (1.0 + 4.0 * tau / h) * std::pow(delta, 2.0 * eH - 2.0))
                        : 1e300;
    const V3<double> vb0 = (c.b >= 0) ? S.v[c.b] : V3<double>{0, 0, 0};
    const V3<double> wb0 = (c.b >= 0) ? S.w[c.b] : V3<double>{0, 0, 0};
    const double un0 = dot(rel_vel(c, S.v[i], S.w[i], vb0, wb0), c.n);
    c.C = ups * (un0 - 4.0 * delta / (eH * h));
    // warm start from the stored impulse, re-expressed in the new frame
    const Hist hs = lookup_hist(S, i, ct.partner);
    const V3<double> J = {hs[0], hs[1], hs[2]};
    const double Jn = dot(J, c.n);
    c.P = std::max(0.0, -Jn);
    c.pt = sub(J, scl(Jn, c.n));
    c.pr = {hs[3], hs[4], hs[5]};
  }
  const V3<double> g = {b.p.g[0], b.p.g[1], b.p.g[2]};
  std::vector<V3<double>> vs((size_t)b.n), V((size_t)b.n), W((size_t)b.n);
  for (int64_t i = 0; i < b.n; ++i) vs[i] = add(S.v[i], scl(h, g));
  const V3<double> zero = {0.0, 0.0, 0.0};
  // velocities from v*, the start spins and the current impulses
  auto rebuild = [&]() {
    std::vector<V3<double>> dv((size_t)b.n, zero), dw((size_t)b.n, zero);
    for (int64_t q = 0; q < nc; ++q) {
      const SpC& c = C[q];
      const V3<double> Ja = add(scl(-c.P, c.n), c.pt);
      dv[c.a] = add(dv[c.a], Ja);
      dw[c.a] = add(dw[c.a], add(scl(c.la, cross(c.n, c.pt)), c.pr));
      if (c.b >= 0) {
        dv[c.b] = sub(dv[c.b], Ja);
        dw[c.b] = add(dw[c.b], sub(scl(c.lb, cross(c.n, c.pt)), c.pr));
      }
    }
    for (int64_t i = 0; i < b.n; ++i) {
      V[i] = add(vs[i], scl(1.0 / b.m[i], dv[i]));
      W[i] = add(S.w[i], scl(1.0 / b.I[i], dw[i]));
    }
  };
  rebuild();
  for (int it = 0; it < b.n_iter; ++it) {
#pragma omp parallel for schedule(static) if (nc > 4096)
    for (int64_t q = 0; q < nc; ++q) {
      SpC& c = C[q];
      const int64_t i = c.a;
      V3<double> va = V[i], wa = W[i], vb = zero, wb = c.ww;
      const double ima = (double)deg[i] / b.m[i], iIa = (double)deg[i] / b.I[i];
      double imb = 0.0, iIb = 0.0;
      if (c.b >= 0) {
        vb = V[c.b];
        wb = W[c.b];
        imb = (double)deg[c.b] / b.m[c.b];
        iIb = (double)deg[c.b] / b.I[c.b];
      }
      // normal row
      const double un = dot(rel_vel(c, va, wa, vb, wb), c.n);
      const double Pn = std::max(0.0, c.P - (-un + c.S * c.P + c.C) / (ima + imb + c.S));
      const double dP = Pn - c.P;
      c.P = Pn;
      va = sub(va, scl(ima * dP, c.n));
      vb = add(vb, scl(imb * dP, c.n));
      // tangent rows, Coulomb disc
      const V3<double> u = rel_vel(c, va, wa, vb, wb);
      const V3<double> ut = sub(u, scl(dot(u, c.n), c.n));
      const double Dt = ima + imb + c.la * c.la * iIa + c.lb * c.lb * iIb;
      V3<double> pt = sub(c.pt, scl(1.0 / Dt, ut));
      const double capt = c.mu_t * Pn, lt = norm(pt);
      if (lt > capt) pt = (lt > 0.0) ? scl(capt / lt, pt) : zero;
      const V3<double> dpt = sub(pt, c.pt);
      c.pt = pt;
      va = add(va, scl(ima, dpt));
      wa = add(wa, scl(iIa * c.la, cross(c.n, dpt)));
      vb = sub(vb, scl(imb, dpt));
      wb = add(wb, scl(iIb * c.lb, cross(c.n, dpt)));
      // rolling rows, rolling-resistance ball
      const V3<double> wr = sub(wa, wb);
      V3<double> pr = sub(c.pr, scl(1.0 / (iIa + iIb), wr));
      const double capr = c.mrr * Pn, lr = norm(pr);
      if (lr > capr) pr = (lr > 0.0) ? scl(capr / lr, pr) : zero;
      c.pr = pr;
    }
    rebuild();
  }
  // records: contact forces and torques over the step, body reactions
  const size_t nb = b.bodies.size();
  b.last_contacts = cs;
  b.lastF.assign((size_t)(3 * b.n), 0.0);
  b.lastT.assign((size_t)(3 * b.n), 0.0);
  b.lastR.assign(6 * nb, 0.0);
  b.lastCF.assign((size_t)(3 * nc), 0.0);
  b.lastCM.assign((size_t)(3 * nc), 0.0);
  b.lastCN.assign((size_t)nc, 0.0);
  b.lastCSF.clear();  // the explicit law's term scales do not apply
  b.lastCSM.clear();
  std::vector<std::vector<int64_t>> nk((size_t)b.n);
  std::vector<std::vector<Hist>> nv((size_t)b.n);
  for (int64_t q = 0; q < nc; ++q) {
    const SpC& c = C[q];
    const V3<double> Ja = add(scl(-c.P, c.n), c.pt);
    const V3<double> Fa = scl(1.0 / h, Ja);
    b.lastCF[3 * q + 0] = Fa.x; b.lastCF[3 * q + 1] = Fa.y; b.lastCF[3 * q + 2] = Fa.z;
    b.lastCM[3 * q + 0] = c.pr.x / h; b.lastCM[3 * q + 1] = c.pr.y / h; b.lastCM[3 * q + 2] = c.pr.z / h;
    b.lastCN[q] = c.P / h;
    const V3<double> Ta = scl(1.0 / h, add(scl(c.la, cross(c.n, c.pt)), c.pr));
    double* F = &b.lastF[3 * c.a];
    double* T = &b.lastT[3 * c.a];
    F[0] += Fa.x; F[1] += Fa.y; F[2] += Fa.z;
    T[0] += Ta.x; T[1] += Ta.y; T[2] += Ta.z;
    if (c.b >= 0) {
      const V3<double> Tb = scl(1.0 / h, sub(scl(c.lb, cross(c.n, c.pt)), c.pr));
      double* Fb = &b.lastF[3 * c.b];
      double* Tbp = &b.lastT[3 * c.b];
      Fb[0] -= Fa.x; Fb[1] -= Fa.y; Fb[2] -= Fa.z;
      Tbp[0] += Tb.x; Tbp[1] += Tb.y; Tbp[2] += Tb.z;
    } else {
      const V3<double> Fw = neg(Fa);
      const V3<double> Tw = sub(cross(sub(c.pc, bp[c.body].c), Fw), scl(1.0 / h, c.pr));
      double* R = &b.lastR[6 * c.body];
      R[0] += Fw.x; R[1] += Fw.y; R[2] += Fw.z;
      R[3] += Tw.x; R[4] += Tw.y; R[5] += Tw.z;
    }
    nk[c.a].push_back(cs[q].partner);
    nv[c.a].push_back({Ja.x, Ja.y, Ja.z, c.pr.x, c.pr.y, c.pr.z});
  }
  S.hkey.swap(nk);
  S.hval.swap(nv);
  // positions with the new velocities; wrap periodic axes
  for (int64_t i = 0; i < b.n; ++i) {
    S.v[i] = V[i];
    S.w[i] = W[i];
    S.x[i] = add(S.x[i], scl(h, V[i]));
    if (b.periodic & 1u) {
      if (S.x[i].x >= b.L[0]) S.x[i].x -= b.L[0];
      else if (S.x[i].x < 0.0) S.x[i].x += b.L[0];
    }
    if (b.periodic & 2u) {
      if (S.x[i].y >= b.L[1]) S.x[i].y -= b.L[1];
      else if (S.x[i].y < 0.0) S.x[i].y += b.L[1];
    }
  }
  b.k += 1;
}

bool finite3(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

extern "C" {

orc_bed* orc_create(int64_t n, const double* pos, const float* rad, const float* vel, const float* omg,
                    const double box[3], uint32_t periodic, const orc_params* prm, int32_t n_walls,
                    const orc_wall* walls, int32_t n_bodies, const orc_body* bodies) {
  if (n <= 0 || !pos || !rad || !prm || !box) return nullptr;
  if (!(prm->dt > 0.0) || !(prm->rho > 0.0) || !(prm->E > 0.0)) return nullptr;
  if (n_walls < 0 || n_bodies < 0 || (n_walls > 0 && (!walls || n_bodies == 0))) return nullptr;
  if (!finite3(pos, 3 * n)) return nullptr;
  orc_bed* b = new orc_bed();
  b->n = n;
  b->L[0] = box[0];
  b->L[1] = box[1];
  b->periodic = periodic;
  b->p = *prm;
  b->walls.assign(walls, walls + n_walls);
  b->bodies.assign(bodies, bodies + n_bodies);
  for (const orc_wall& W : b->walls)
    if (W.body < 0 || W.body >= n_bodies || W.kind < 0 || W.kind > 3) { delete b; return nullptr; }
  b->r.resize(n);
  b->m.resize(n);
  b->I.resize(n);
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double r = (double)rad[i];
    if (!(r > 0.0) || !std::isfinite(r)) { delete b; return nullptr; }
    b->r[i] = r;
    b->m[i] = prm->rho * (4.0 / 3.0) * M_PI * r * r * r;
    b->I[i] = 0.4 * b->m[i] * r * r;
    rmax = std::max(rmax, r);
  }
  for (int a = 0; a < 2; ++a)
    if ((periodic >> a) & 1u)
      if (!(box[a] > 4.0 * rmax)) { delete b; return nullptr; }
  State<double>& S = b->st;
  S.x.resize(n);
  S.v.resize(n);
  S.w.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    S.x[i] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    S.v[i] = vel ? V3<double>{vel[3 * i], vel[3 * i + 1], vel[3 * i + 2]} : V3<double>{0, 0, 0};
    S.w[i] = omg ? V3<double>{omg[3 * i], omg[3 * i + 1], omg[3 * i + 2]} : V3<double>{0, 0, 0};
  }
  S.hkey.assign(n, {});
  S.hval.assign(n, {});
  S.s_k = prm->s_k;
  S.mu_t = prm->mu_t;
  S.mu_r = prm->mu_r;
  b->bz.resize(n_bodies);
  b->bvz.resize(n_bodies);
  for (int q = 0; q < n_bodies; ++q) {
    b->bz[q] = bodies[q].origin[2];
    b->bvz[q] = bodies[q].lin_vel[2];
  }
  b->lastR.assign(6 * (size_t)n_bodies, 0.0);
  return b;
}

void orc_destroy(orc_bed* b) { delete b; }

int orc_set_state(orc_bed* b, const double* pos, const double* vel, const double* omg) {
  if (!b) return -1;
  for (int64_t i = 0; i < b->n; ++i) {
    if (pos) b->st.x[i] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    if (vel) b->st.v[i] = {vel[3 * i], vel[3 * i + 1], vel[3 * i + 2]};
    if (omg) b->st.w[i] = {omg[3 * i], omg[3 * i + 1], omg[3 * i + 2]};
  }
  return 0;
}

int orc_get_state(const orc_bed* b, double* pos, double* vel, double* omg) {
  if (!b) return -1;
  for (int64_t i = 0; i < b->n; ++i) {
    if (pos) { pos[3 * i] = b->st.x[i].x; pos[3 * i + 1] = b->st.x[i].y; pos[3 * i + 2] = b->st.x[i].z; }
    if (vel) { vel[3 * i] = b->st.v[i].x; vel[3 * i + 1] = b->st.v[i].y; vel[3 * i + 2] = b->st.v[i].z; }
    if (omg) { omg[3 * i] = b->st.w[i].x; omg[3 * i + 1] = b->st.w[i].y; omg[3 * i + 2] = b->st.w[i].z; }
  }
  return 0;
}

int orc_set_clock(orc_bed* b, int64_t step) {
  if (!b || step < 0) return -1;
  b->k = step;
  return 0;
}

int orc_set_body_state(orc_bed* b, int32_t body, double z, double vz) {
  if (!b || body < 0 || body >= (int32_t)b->bodies.size()) return -1;
  b->bz[body] = z;
  b->bvz[body] = vz;
  return 0;
}

int orc_get_body_state(const orc_bed* b, int32_t body, double* origin3, double* vel3) {
  if (!b || body < 0 || body >= (int32_t)b->bodies.size()) return -1;
  const std::vector<BodyPose> bp = body_poses(*b, (double)b->k * b->p.dt);
  if (origin3) { origin3[0] = bp[body].c.x; origin3[1] = bp[body].c.y; origin3[2] = bp[body].c.z; }
  if (vel3) { vel3[0] = bp[body].vel.x; vel3[1] = bp[body].vel.y; vel3[2] = bp[body].vel.z; }
  return 0;
}

int64_t orc_history_count(const orc_bed* b) {
  if (!b) return -1;
  int64_t c = 0;
  for (const auto& v : b->st.hkey) c += (int64_t)v.size();
  return c;
}

int orc_get_history(const orc_bed* b, int64_t* keys2, double* vals6, int64_t cap) {
  if (!b) return -1;
  int64_t q = 0;
  for (int64_t i = 0; i < b->n; ++i)
    for (size_t s = 0; s < b->st.hkey[i].size(); ++s) {
      if (q >= cap) return -2;
      keys2[2 * q] = i;
      keys2[2 * q + 1] = b->st.hkey[i][s];
      for (int a = 0; a < 6; ++a) vals6[6 * q + a] = b->st.hval[i][s][a];
      ++q;
    }
  return 0;
}

int orc_set_history(orc_bed* b, int64_t count, const int64_t* keys2, const double* vals6) {
  if (!b || count < 0) return -1;
  std::vector<std::vector<std::pair<int64_t, Hist>>> tmp((size_t)b->n);
  for (int64_t q = 0; q < count; ++q) {
    const int64_t o = keys2[2 * q];
    if (o < 0 || o >= b->n) return -1;
    Hist h;
    for (int a = 0; a < 6; ++a) h[a] = vals6[6 * q + a];
    tmp[o].push_back({keys2[2 * q + 1], h});
  }
  for (int64_t i = 0; i < b->n; ++i) {
    std::sort(tmp[i].begin(), tmp[i].end(),
              [](const std::pair<int64_t, Hist>& a, const std::pair<int64_t, Hist>& c) { return a.first < c.first; });
    b->st.hkey[i].clear();
    b->st.hval[i].clear();
    for (auto& e : tmp[i]) {
      b->st.hkey[i].push_back(e.first);
      b->st.hval[i].push_back(e.second);
    }
  }
  return 0;
}

int orc_step(orc_bed* b, int64_t n_steps) {
  if (!b || n_steps < 0) return -1;
  for (int64_t s = 0; s < n_steps; ++s) {
    if (b->stepper == 1) spook_step(*b);
    else step_once<double>(*b, b->st, -1);
  }
  return 0;
}

int orc_set_stepper(orc_bed* b, int32_t kind, int32_t n_iter) {
  if (!b || kind < 0 || kind > 1) return -1;
  if (kind == 1) {
    if (n_iter < 1) return -1;
    for (const orc_body& B : b->bodies)
      if (B.z_free) return -3;  // dynamic bodies are not part of the implicit solve
  }
  b->stepper = kind;
  b->n_iter = n_iter;
  return 0;
}

static int copy_pairs(const std::vector<Contact>& cs, int64_t* pairs2, int64_t cap, int64_t* n_total) {
  if (n_total) *n_total = (int64_t)cs.size();
  if ((int64_t)cs.size() > cap) return -2;
  for (size_t q = 0; q < cs.size(); ++q) {
    pairs2[2 * q] = cs[q].owner;
    pairs2[2 * q + 1] = cs[q].partner;
  }
  return 0;
}

int orc_contact_set(const orc_bed* b, int32_t method, int64_t* pairs2, int64_t cap, int64_t* n_total) {
  if (!b) return -1;
  const std::vector<BodyPose> bp = body_poses(*b, (double)b->k * b->p.dt);
  const std::vector<WallPose> wp = wall_poses(*b, bp);
  std::vector<Contact> cs = detect(*b, b->st.x, wp, method);
  return copy_pairs(cs, pairs2, cap, n_total);
}

int orc_last_contacts(const orc_bed* b, int64_t* pairs2, int64_t cap, int64_t* n_total) {
  if (!b) return -1;
  return copy_pairs(b->last_contacts, pairs2, cap, n_total);
}

int orc_last_forces(const orc_bed* b, double* force3, double* torque3) {
  if (!b || b->lastF.size() != (size_t)(3 * b->n)) return -1;
  if (force3) std::memcpy(force3, b->lastF.data(), sizeof(double) * 3 * b->n);
  if (torque3) std::memcpy(torque3, b->lastT.data(), sizeof(double) * 3 * b->n);
  return 0;
}

int orc_last_contact_loads(const orc_bed* b, double* force3, double* moment3, double* fn) {
  if (!b || b->lastCN.size() != b->last_contacts.size()) return -1;
  const size_t nc = b->last_contacts.size();
  if (force3 && nc) std::memcpy(force3, b->lastCF.data(), sizeof(double) * 3 * nc);
  if (moment3 && nc) std::memcpy(moment3, b->lastCM.data(), sizeof(double) * 3 * nc);
  if (fn && nc) std::memcpy(fn, b->lastCN.data(), sizeof(double) * nc);
  return 0;
}

int orc_last_contact_scales(const orc_bed* b, double* force_terms, double* moment_terms) {
  if (!b || b->lastCSF.size() != b->last_contacts.size()) return -1;
  const size_t nc = b->last_contacts.size();
  if (force_terms && nc) std::memcpy(force_terms, b->lastCSF.data(), sizeof(double) * nc);
  if (moment_terms && nc) std::memcpy(moment_terms, b->lastCSM.data(), sizeof(double) * nc);
  return 0;
}

int orc_wall_pose(const orc_bed* b, int32_t wall, double out15[15]) {
  if (!b || wall < 0 || wall >= (int32_t)b->walls.size()) return -1;
  const std::vector<BodyPose> bp = body_poses(*b, (double)b->k * b->p.dt);
  const std::vector<WallPose> wp = wall_poses(*b, bp);
  const WallPose& W = wp[wall];
  const V3<double> v[5] = {W.o, W.nu, W.e[0], W.e[1], W.e[2]};
  for (int q = 0; q < 5; ++q) {
    out15[3 * q + 0] = v[q].x;
    out15[3 * q + 1] = v[q].y;
    out15[3 * q + 2] = v[q].z;
  }
  return 0;
}

int orc_last_reaction(const orc_bed* b, int32_t body, double out6[6]) {
  if (!b || body < 0 || body >= (int32_t)b->bodies.size()) return -1;
  for (int a = 0; a < 6; ++a) out6[a] = b->lastR[6 * body + a];
  return 0;
}

int orc_tangent_window(orc_bed* b, int64_t n_steps, int32_t body, int32_t component, double* J,
                       double grad3[3]) {
  if (!b || n_steps <= 0 || body < 0 || body >= (int32_t)b->bodies.size()) return -1;
  if (component < 0 || component > 5) return -1;
  for (const orc_body& B : b->bodies)
    if (B.z_free) return -3;  // derivative through a dynamic body is not provided
  if (b->stepper != 0) return -3;  // derivatives of the explicit step only
  State<Dual> S;
  const State<double>& D = b->st;
  S.x.resize(b->n);
  S.v.resize(b->n);
  S.w.resize(b->n);
  for (int64_t i = 0; i < b->n; ++i) {
    S.x[i] = lift<Dual>(D.x[i]);
    S.v[i] = lift<Dual>(D.v[i]);
    S.w[i] = lift<Dual>(D.w[i]);
  }
  S.hkey = D.hkey;
  S.hval.resize(b->n);
  for (int64_t i = 0; i < b->n; ++i)
    for (const auto& h : D.hval[i]) {
      std::array<Dual, 6> hd;
      for (int a = 0; a < 6; ++a) hd[a] = Dual(h[a]);
      S.hval[i].push_back(hd);
    }
  S.s_k = Dual(D.s_k);
  S.s_k.d[0] = 1.0;
  S.mu_t = Dual(D.mu_t);
  S.mu_t.d[1] = 1.0;
  S.mu_r = Dual(D.mu_r);
  S.mu_r.d[2] = 1.0;
  Dual acc(0.0);
  for (int64_t s = 0; s < n_steps; ++s) acc = acc + step_once<Dual>(*b, S, body, component);
  const Dual Jd = acc / Dual((double)n_steps);
  *J = Jd.v;
  for (int a = 0; a < 3; ++a) grad3[a] = Jd.d[a];
  // the bed advances exactly as orc_step would have advanced it
  State<double>& O = b->st;
  for (int64_t i = 0; i < b->n; ++i) {
    O.x[i] = vals(S.x[i]);
    O.v[i] = vals(S.v[i]);
    O.w[i] = vals(S.w[i]);
  }
  O.hkey = S.hkey;
  for (int64_t i = 0; i < b->n; ++i) {
    O.hval[i].clear();
    for (const auto& h : S.hval[i]) {
      Hist hv;
      for (int a = 0; a < 6; ++a) hv[a] = h[a].v;
      O.hval[i].push_back(hv);
    }
  }
  return 0;
}

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // extern "C"
