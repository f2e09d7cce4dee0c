// lpr_spook.hip -- kernels of the time-implicit step.
//
// Section "Nonsmooth DEM and multibody dynamics": one SPOOK step of length h
// (eq:momentum, eq:g_n, eq:G_t, eq:G_r).  Start velocities v0, free velocities
// v* = v0 + h g; new velocities v+ = v* + M^-1 (sum of contact impulses).  A
// contact between owner a and partner b (a sphere or a wall) has unit normal
// n (a toward b), overlap delta > 0, lever arms l_a = r_a - delta/2,
// l_b = r_b - delta/2, and relative velocity u of a with respect to b at the
// contact point.  Its rows:
//   normal   0 <= -u.n(v+) + S P + C  perp  P >= 0, where
//            S = 4 / (k_n e_H h^2 (1 + 4 tau/h) delta^(2 e_H - 2)) and
//            C = (u.n(v0) - 4 delta / (e_H h)) / (1 + 4 tau/h), tau = gamma_n:
//            the SPOOK row of the gap -delta^e_H with compliance e_H / k_n,
//            scaled by 1 / (e_H delta^(e_H - 1)) so that P is the normal impulse;
//   tangent  the tangential slip vanishes while |p_t| < mu_t P; at the bound
//            p_t opposes it (maximal dissipation);
//   rolling  w_a - w_b vanishes while |p_r| < mu_r r* P; at the bound p_r opposes it.
// The impulse on a is -P n + p_t at the contact point plus the moment p_r.
//
// Solver: projected block-Jacobi with mass splitting.  Each sweep, every
// contact solves its own rows in turn (normal, tangent, rolling) from the
// previous sweep's velocities, against its bodies' masses and inertias
// divided by their contact counts; the velocities are then rebuilt from v*
// and every impulse, per particle in a fixed order (owner slots, reverse
// list, walls).  To read each contact once per sweep, the contacts kernel
// also writes every particle's owner-side sum and, per owner slot, the part
// of the impulse its partner receives; the velocity kernel adds those.
// Fixed points satisfy the rows above; the result does not depend on thread
// scheduling.
#include "lpr_spook.h"

#include <hip/hip_runtime.h>

namespace lpr {
namespace {

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 mk(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ D3 add(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 sub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 scl(double s, D3 a) { return D3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
  return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double nrm(D3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ D3 from4f(float4 a) { return D3{(double)a.x, (double)a.y, (double)a.z}; }

// Launch block -> work block: the blocks the hardware places on one XCD
// take one contiguous range of particles (g work blocks, grid rounded up to 8).
__device__ __forceinline__ int64_t sp_block(int64_t b, int64_t g) {
  const int64_t chunk = (g + 7) / 8;
  const int64_t w = (b & 7) * chunk + (b >> 3);
  return w < g ? w : -1;
}

__device__ __forceinline__ bool sp_latched(const uint32_t* err) { return *(const volatile uint32_t*)err != 0u; }

__device__ __forceinline__ double sphere_mass(double rho, double r) { return rho * (4.0 / 3.0) * M_PI * r * r * r; }

// velocity of a relative to b at the contact point (b a sphere)
__device__ __forceinline__ D3 rel_pair(D3 n, double la, double lb, D3 va, D3 wa, D3 vb, D3 wb) {
  return add(add(sub(va, vb), scl(la, cross(wa, n))), scl(lb, cross(wb, n)));
}

// Normal row, warm start from the stored impulse on the owner J and p_r.
__device__ __forceinline__ void warm(D3 n, D3 J, D3 pr, SpImp& o) {
  const double Jn = dot(J, n);
  o.P = Jn < 0.0 ? -Jn : 0.0;
  o.tx = J.x - Jn * n.x;
  o.ty = J.y - Jn * n.y;
  o.tz = J.z - Jn * n.z;
  o.rx = pr.x;
  o.ry = pr.y;
  o.rz = pr.z;
  o.pad = 0.0;
}

// An overlap that rounds to zero (the predicate holds by less than the
// rounding of the distance) has no stiffness: its row cannot push.
__device__ __forceinline__ double row_S(const SpConst& c, double dstar, double delta) {
  if (!(delta > 0.0)) return 1e300;
  const double kn = c.kfac * sqrt(dstar);
  const double dp = (c.eH == 1.25) ? sqrt(delta) : pow(delta, 2.0 * c.eH - 2.0);
  return 4.0 * c.ups / (kn * c.eH * c.h * c.h * dp);
}

__global__ __launch_bounds__(SP_BS) void k_sp_rows(DevBufs d, SpBufs sp, int s, int h, int l) {
  if (sp_latched(d.err)) return;
  const int64_t N = d.N;
  const int64_t blk = sp_block(blockIdx.x, N / SP_BS);
  if (blk < 0) return;
  const int64_t i = blk * SP_BS + threadIdx.x;
  if (d.meta[i] == INACTIVE) {
    sp.flag[i] = 0u;
    return;
  }
  const int bed = d.chunk_bed32[i >> 8];
  const BedConst bc = d.beds[bed];
  const SpConst c = sp.sc[bed];
  const PState me = d.st[s][i];
  const double ri = me.x.w;
  const D3 va = from4f(me.v), wa = from4f(me.w);
  uint32_t fl = 0u;
  const int n_own = d.own_cnt[l][i];
  for (int k = 0; k < n_own; ++k) {
    const int64_t q = (int64_t)k * N + i;
    const int64_t j = d.own_idx[l][q];
    const PState ot = d.st[s][j];
    double dx, dy, dz;
    const double d2 = pair_sep(bc, me.x, ot.x, dx, dy, dz);
    if (!sphere_touch(d2, me.x.w, ot.x.w)) {
      sp.cb[q] = SpSum{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // the partner's sweeps add nothing from this slot
      continue;
    }
    const double rj = ot.x.w;
    const double dist = sqrt(d2);
    const D3 n = (d2 > 0.0) ? mk(dx / dist, dy / dist, dz / dist) : mk(0.0, 0.0, 1.0);
    const double delta = (ri + rj) - dist;
    const double dstar = 2.0 * ri * rj / (ri + rj);
    SpRow r;
    r.nx = n.x; r.ny = n.y; r.nz = n.z;
    r.la = ri - 0.5 * delta;
    r.lb = rj - 0.5 * delta;
    r.S = row_S(c, dstar, delta);
    const double un0 = dot(rel_pair(n, r.la, r.lb, va, wa, from4f(ot.v), from4f(ot.w)), n);
    r.C = c.ups * (un0 - 4.0 * delta / (c.eH * c.h));
    r.mrr = c.mu_r * 0.5 * dstar;
    sp.row[q] = r;
    const HRec hr = d.hist[h][q];
    SpImp o;
    warm(n, from4f(hr.t), from4f(hr.r), o);
    sp.imp[q] = o;
    fl |= 1u << k;
  }
  const uint32_t fold = d.cflag[h][i];
  for (int w = 0; w < bc.nwall; ++w) {
    const WallPose& W = d.walls[bc.wall0 + w];
    double delta, nx, ny, nz;
    if (!wall_geom(W, me.x.x, me.x.y, me.x.z, ri, delta, nx, ny, nz)) continue;
    if (W.kind == WPLANE && delta > 2.0 * ri) atomicOr(d.err, ERR_WALL);  // tunnelled through a plane
    const int64_t q = (int64_t)w * N + i;
    const D3 n = mk(nx, ny, nz);
    SpWRow r;
    r.nx = nx; r.ny = ny; r.nz = nz;
    r.la = ri - 0.5 * delta;
    r.S = row_S(c, 2.0 * ri, delta);
    r.px = me.x.x + r.la * nx;
    r.py = me.x.y + r.la * ny;
    r.pz = me.x.z + r.la * nz;
    const double rx = r.px - W.c[0], ry = r.py - W.c[1];
    r.ux = W.vel[0] - W.omega * ry;
    r.uy = W.vel[1] + W.omega * rx;
    r.uz = W.vel[2];
    r.wz = W.omega;
    r.pad = 0.0;
    const D3 u0 = sub(add(va, scl(r.la, cross(wa, n))), mk(r.ux, r.uy, r.uz));
    r.C = c.ups * (dot(u0, n) - 4.0 * delta / (c.eH * c.h));
    r.mut = (W.mu_t < 0.f) ? c.mu_t : (double)W.mu_t;
    r.mrr = ((W.mu_r < 0.f) ? c.mu_r : (double)W.mu_r) * ri;
    sp.wrow[q] = r;
    D3 J = mk(0.0, 0.0, 0.0), pr = mk(0.0, 0.0, 0.0);
    if ((fold >> (WALL_BIT + w)) & 1u) {
      const float4 a4 = d.wA[h][q];
      const float2 b2 = d.wB[h][q];
      J = mk(a4.x, a4.y, a4.z);
      pr = mk(a4.w, b2.x, b2.y);
    }
    SpImp o;
    warm(n, J, pr, o);
    sp.wimp[q] = o;
    fl |= 1u << (WALL_BIT + w);
  }
  sp.flag[i] = fl;
}

// Sum of the impulses on particle i (force part, moment part) in the fixed
// order owner slots, reverse list, walls; returns the contact count.
__device__ __forceinline__ int impulse_sums(const DevBufs& d, const SpBufs& sp, int l, int64_t i, uint32_t fl,
                                            D3& dv, D3& dw) {
  const int64_t N = d.N;
  int cnt = 0;
  dv = mk(0.0, 0.0, 0.0);
  dw = mk(0.0, 0.0, 0.0);
  uint32_t own = fl & 0xffffu;
  while (own) {
    const int k = __builtin_ctz(own);
    own &= own - 1u;
    const int64_t q = (int64_t)k * N + i;
    const SpRow r = sp.row[q];
    const SpImp o = sp.imp[q];
    const D3 n = mk(r.nx, r.ny, r.nz), pt = mk(o.tx, o.ty, o.tz);
    dv = add(dv, sub(pt, scl(o.P, n)));
    dw = add(dw, add(scl(r.la, cross(n, pt)), mk(o.rx, o.ry, o.rz)));
    ++cnt;
  }
  const uint32_t e0 = d.rev_start[i], e1 = d.rev_start[i + 1];
  for (uint32_t e = e0; e < e1; ++e) {
    const uint32_t pk = d.rev_ent[e];
    const int64_t o_i = pk >> 4;
    const int k = (int)(pk & 15u);
    if (!((sp.flag[o_i] >> k) & 1u)) continue;
    const int64_t q = (int64_t)k * N + o_i;
    const SpRow r = sp.row[q];
    const SpImp o = sp.imp[q];
    const D3 n = mk(r.nx, r.ny, r.nz), pt = mk(o.tx, o.ty, o.tz);
    dv = sub(dv, sub(pt, scl(o.P, n)));
    dw = add(dw, sub(scl(r.lb, cross(n, pt)), mk(o.rx, o.ry, o.rz)));
    ++cnt;
  }
  uint32_t wl = fl >> WALL_BIT;
  while (wl) {
    const int w = __builtin_ctz(wl);
    wl &= wl - 1u;
    const int64_t q = (int64_t)w * N + i;
    const SpWRow r = sp.wrow[q];
    const SpImp o = sp.wimp[q];
    const D3 n = mk(r.nx, r.ny, r.nz), pt = mk(o.tx, o.ty, o.tz);
    dv = add(dv, sub(pt, scl(o.P, n)));
    dw = add(dw, add(scl(r.la, cross(n, pt)), mk(o.rx, o.ry, o.rz)));
    ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(SP_BS) void k_sp_vel(DevBufs d, SpBufs sp, int s, int l, int first) {
  if (sp_latched(d.err)) return;
  const int64_t N = d.N;
  const int64_t blk = sp_block(blockIdx.x, N / SP_BS);
  if (blk < 0) return;
  const int64_t i = blk * SP_BS + threadIdx.x;
  if (d.meta[i] == INACTIVE) return;
  const SpConst c = sp.sc[d.chunk_bed32[i >> 8]];
  const PState me = d.st[s][i];
  const double r = me.x.w;
  const double m = sphere_mass(c.rho, r), I = 0.4 * m * r * r;
  D3 dv, dw;
  double2 si;
  if (first) {
    const int cnt = impulse_sums(d, sp, l, i, sp.flag[i], dv, dw);
    si = make_double2((double)cnt / m, (double)cnt / I);
    sp.sinv[i] = si;
  } else {
    si = sp.sinv[i];
    const SpSum o = sp.own[i];
    dv = mk(o.fx, o.fy, o.fz);
    dw = mk(o.tx, o.ty, o.tz);
    const uint32_t e0 = d.rev_start[i], e1 = d.rev_start[i + 1];
    for (uint32_t e = e0; e < e1; ++e) {
      const uint32_t pk = d.rev_ent[e];
      const SpSum b = sp.cb[(int64_t)(pk & 15u) * N + (pk >> 4)];
      dv = add(dv, mk(b.fx, b.fy, b.fz));
      dw = add(dw, mk(b.tx, b.ty, b.tz));
    }
  }
  SpVel V;
  V.vx = (double)me.v.x + c.h * c.g[0] + dv.x / m;
  V.vy = (double)me.v.y + c.h * c.g[1] + dv.y / m;
  V.vz = (double)me.v.z + c.h * c.g[2] + dv.z / m;
  V.wx = (double)me.w.x + dw.x / I;
  V.wy = (double)me.w.y + dw.y / I;
  V.wz = (double)me.w.z + dw.z / I;
  V.ima = si.x;
  V.iIa = si.y;
  sp.vel[i] = V;
}

// One contact's rows, solved in turn against split masses (b a sphere when
// ib >= 0, a wall moving with (ub, wb) otherwise).
__device__ __forceinline__ void solve_block(D3 n, double la, double lb, double S, double C, double mut,
                                            double mrr, double ima, double iIa, double imb, double iIb, D3 va,
                                            D3 wa, D3 vb, D3 wb, bool wall, SpImp& o) {
  // normal
  const D3 u1 = wall ? sub(add(va, scl(la, cross(wa, n))), vb) : rel_pair(n, la, lb, va, wa, vb, wb);
  const double un = dot(u1, n);
  double P = o.P - (-un + S * o.P + C) / (ima + imb + S);
  P = P > 0.0 ? P : 0.0;
  const double dP = P - o.P;
  o.P = P;
  va = sub(va, scl(ima * dP, n));
  vb = add(vb, scl(imb * dP, n));
  // tangent, Coulomb disc
  const D3 u2 = wall ? sub(add(va, scl(la, cross(wa, n))), vb) : rel_pair(n, la, lb, va, wa, vb, wb);
  const D3 ut = sub(u2, scl(dot(u2, n), n));
  const double Dt = ima + imb + la * la * iIa + lb * lb * iIb;
  const D3 pt0 = mk(o.tx, o.ty, o.tz);
  D3 pt = sub(pt0, scl(1.0 / Dt, ut));
  const double capt = mut * P, lt = nrm(pt);
  if (lt > capt) pt = (lt > 0.0) ? scl(capt / lt, pt) : mk(0.0, 0.0, 0.0);
  const D3 dpt = sub(pt, pt0);
  o.tx = pt.x; o.ty = pt.y; o.tz = pt.z;
  wa = add(wa, scl(iIa * la, cross(n, dpt)));
  wb = add(wb, scl(iIb * lb, cross(n, dpt)));
  // rolling, rolling-resistance ball
  const D3 wr = sub(wa, wb);
  D3 pr = sub(mk(o.rx, o.ry, o.rz), scl(1.0 / (iIa + iIb), wr));
  const double capr = mrr * P, lr = nrm(pr);
  if (lr > capr) pr = (lr > 0.0) ? scl(capr / lr, pr) : mk(0.0, 0.0, 0.0);
  o.rx = pr.x; o.ry = pr.y; o.rz = pr.z;
}

__global__ __launch_bounds__(SP_BS) void k_sp_contacts(DevBufs d, SpBufs sp, int l) {
  if (sp_latched(d.err)) return;
  const int64_t N = d.N;
  const int64_t blk = sp_block(blockIdx.x, N / SP_BS);
  if (blk < 0) return;
  const int64_t i = blk * SP_BS + threadIdx.x;
  const uint32_t fl = sp.flag[i];   // 0 for padding
  if (fl == 0u) {
    sp.own[i] = SpSum{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    return;
  }
  const SpConst c = sp.sc[d.chunk_bed32[i >> 8]];
  const SpVel Vi = sp.vel[i];
  const D3 va = mk(Vi.vx, Vi.vy, Vi.vz), wa = mk(Vi.wx, Vi.wy, Vi.wz);
  D3 fo = mk(0.0, 0.0, 0.0), to = mk(0.0, 0.0, 0.0);
  uint32_t own = fl & 0xffffu;
  while (own) {
    const int k = __builtin_ctz(own);
    own &= own - 1u;
    const int64_t q = (int64_t)k * N + i;
    const int64_t j = d.own_idx[l][q];
    const SpVel Vj = sp.vel[j];
    const SpRow r = sp.row[q];
    SpImp o = sp.imp[q];
    const D3 n = mk(r.nx, r.ny, r.nz);
    solve_block(n, r.la, r.lb, r.S, r.C, c.mu_t, r.mrr, Vi.ima, Vi.iIa, Vj.ima, Vj.iIa, va, wa,
                mk(Vj.vx, Vj.vy, Vj.vz), mk(Vj.wx, Vj.wy, Vj.wz), false, o);
    sp.imp[q] = o;
    // impulse on the owner -P n + p_t at the contact point, rolling impulse p_r
    const D3 pt = mk(o.tx, o.ty, o.tz), pr = mk(o.rx, o.ry, o.rz);
    const D3 J = sub(pt, scl(o.P, n));
    const D3 npt = cross(n, pt);
    fo = add(fo, J);
    to = add(to, add(scl(r.la, npt), pr));
    const D3 tb = sub(scl(r.lb, npt), pr);
    sp.cb[q] = SpSum{-J.x, -J.y, -J.z, tb.x, tb.y, tb.z};
  }
  uint32_t wl = fl >> WALL_BIT;
  while (wl) {
    const int w = __builtin_ctz(wl);
    wl &= wl - 1u;
    const int64_t q = (int64_t)w * N + i;
    const SpWRow r = sp.wrow[q];
    SpImp o = sp.wimp[q];
    const D3 n = mk(r.nx, r.ny, r.nz);
    solve_block(n, r.la, 0.0, r.S, r.C, r.mut, r.mrr, Vi.ima, Vi.iIa, 0.0, 0.0, va, wa,
                mk(r.ux, r.uy, r.uz), mk(0.0, 0.0, r.wz), true, o);
    sp.wimp[q] = o;
    const D3 pt = mk(o.tx, o.ty, o.tz);
    fo = add(fo, sub(pt, scl(o.P, n)));
    to = add(to, add(scl(r.la, cross(n, pt)), mk(o.rx, o.ry, o.rz)));
  }
  sp.own[i] = SpSum{fo.x, fo.y, fo.z, to.x, to.y, to.z};
}

__device__ __forceinline__ double sp_wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(SP_BS) void k_sp_finish(DevBufs d, SpBufs sp, int s, int h, int l, int record) {
  __shared__ double red[SP_BS / 64][6];
  if (__syncthreads_or(sp_latched(d.err) ? 1 : 0)) return;  // uniform per block
  const int64_t N = d.N;
  const int64_t blk = sp_block(blockIdx.x, N / SP_BS);
  if (blk < 0) return;  // whole launch block idle
  const int64_t i = blk * SP_BS + threadIdx.x;
  const int bed = d.chunk_bed32[(blk * SP_BS) >> 8];
  const BedConst bc = d.beds[bed];
  const SpConst c = sp.sc[bed];
  const bool active = d.meta[i] != INACTIVE;
  const int hn = h ^ 1, sn = s ^ 1;
  const uint32_t fl = active ? sp.flag[i] : 0u;
  PState me{};
  if (active) {
    me = d.st[s][i];
    // history: impulse on the owner and rolling impulse; other slots zero
    const int n_own = d.own_cnt[l][i];
    for (int k = 0; k < n_own; ++k) {
      const int64_t q = (int64_t)k * N + i;
      HRec hr;
      if ((fl >> k) & 1u) {
        const SpRow r = sp.row[q];
        const SpImp o = sp.imp[q];
        hr.t = make_float4((float)(o.tx - o.P * r.nx), (float)(o.ty - o.P * r.ny), (float)(o.tz - o.P * r.nz), 0.f);
        hr.r = make_float4((float)o.rx, (float)o.ry, (float)o.rz, 0.f);
      } else {
        hr.t = make_float4(0.f, 0.f, 0.f, 0.f);
        hr.r = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      d.hist[hn][q] = hr;
    }
  }
  // walls, body by body, with an ordered FP64 block reduction per body
  for (int b = 0; b < bc.nbody; ++b) {
    double r6[6] = {0, 0, 0, 0, 0, 0};
    int hit = 0;
    if (active) {
      for (int w = 0; w < bc.nwall; ++w) {
        if (!((fl >> (WALL_BIT + w)) & 1u)) continue;
        const WallPose& W = d.walls[bc.wall0 + w];
        if (W.body != b) continue;
        hit = 1;
        const int64_t q = (int64_t)w * N + i;
        const SpWRow r = sp.wrow[q];
        const SpImp o = sp.wimp[q];
        const double Jx = o.tx - o.P * r.nx, Jy = o.ty - o.P * r.ny, Jz = o.tz - o.P * r.nz;
        d.wA[hn][q] = make_float4((float)Jx, (float)Jy, (float)Jz, (float)o.rx);
        d.wB[hn][q] = make_float2((float)o.ry, (float)o.rz);
        // reaction on the body: the opposite of the force on the particle at
        // the contact point, and the opposite rolling moment
        const double fx = -Jx / c.h, fy = -Jy / c.h, fz = -Jz / c.h;
        const double rx = r.px - W.c[0], ry = r.py - W.c[1], rz = r.pz - W.c[2];
        r6[0] += fx; r6[1] += fy; r6[2] += fz;
        r6[3] += (ry * fz - rz * fy) - o.rx / c.h;
        r6[4] += (rz * fx - rx * fz) - o.ry / c.h;
        r6[5] += (rx * fy - ry * fx) - o.rz / c.h;
      }
    }
    double* part = d.partial + (int64_t)(bc.body0 + b) * 6 * d.nblk + blk;
    if (__syncthreads_or(hit)) {
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      for (int cc = 0; cc < 6; ++cc) {
        const double sum = sp_wave_sum(r6[cc]);
        if (lane == 0) red[wv][cc] = sum;
      }
      __syncthreads();
      if (threadIdx.x < 6) {
        double acc = 0.0;
        for (int q = 0; q < SP_BS / 64; ++q) acc += red[q][threadIdx.x];
        part[(int64_t)threadIdx.x * d.nblk] = acc;
      }
      __syncthreads();
    } else if (threadIdx.x < 6) {
      part[(int64_t)threadIdx.x * d.nblk] = 0.0;
    }
  }
  if (!active) return;
  d.cflag[hn][i] = fl;
  if (record) {
    D3 dv, dw;
    impulse_sums(d, sp, l, i, fl, dv, dw);
    d.frc[i] = make_float4((float)(dv.x / c.h), (float)(dv.y / c.h), (float)(dv.z / c.h), 0.f);
    d.trq[i] = make_float4((float)(dw.x / c.h), (float)(dw.y / c.h), (float)(dw.z / c.h), 0.f);
  }
  // positions with the new velocities
  const SpVel V = sp.vel[i];
  double x = me.x.x + c.h * V.vx;
  double y = me.x.y + c.h * V.vy;
  const double z = me.x.z + c.h * V.vz;
  if (bc.periodic & 1u) {
    if (x >= bc.L[0]) x -= bc.L[0];
    else if (x < 0.0) x += bc.L[0];
  }
  if (bc.periodic & 2u) {
    if (y >= bc.L[1]) y -= bc.L[1];
    else if (y < 0.0) y += bc.L[1];
  }
  if (!(isfinite(V.vx) && isfinite(V.vy) && isfinite(V.vz) && isfinite(V.wx) && isfinite(V.wy) &&
        isfinite(V.wz) && isfinite(x) && isfinite(y) && isfinite(z)))
    atomicOr(d.err, ERR_NUMERIC);
  PState out;
  out.x = make_double4(x, y, z, me.x.w);
  out.v = make_float4((float)V.vx, (float)V.vy, (float)V.vz, me.v.w);
  out.w = make_float4((float)V.wx, (float)V.wy, (float)V.wz, me.w.w);
  d.st[sn][i] = out;
}

unsigned sp_grid(const DevBufs& d) {
  const int64_t g = d.N / SP_BS;
  return (unsigned)(((g + 7) / 8) * 8);
}

}  // namespace

void launch_sp_rows(const DevBufs& d, const SpBufs& sp, int s, int h, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_sp_rows, dim3(sp_grid(d)), dim3(SP_BS), 0, st, d, sp, s, h, l);
}

void launch_sp_vel(const DevBufs& d, const SpBufs& sp, int s, int l, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_sp_vel, dim3(sp_grid(d)), dim3(SP_BS), 0, st, d, sp, s, l, first);
}

void launch_sp_contacts(const DevBufs& d, const SpBufs& sp, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_sp_contacts, dim3(sp_grid(d)), dim3(SP_BS), 0, st, d, sp, l);
}

void launch_sp_finish(const DevBufs& d, const SpBufs& sp, int s, int h, int l, int record, hipStream_t st) {
  hipLaunchKernelGGL(k_sp_finish, dim3(sp_grid(d)), dim3(SP_BS), 0, st, d, sp, s, h, l, record);
}

}  // namespace lpr
