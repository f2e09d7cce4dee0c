// lpr_adjoint.hip -- reverse-mode (adjoint) kernels of the DEM step.
//
// Objective: J = (1/T) sum_k R_z(k), the mean z reaction on one body over a
// window of T steps; parameters theta = (s_k, mu_t, mu_r).  The host runs
// the window forward with checkpoints, then walks the segments backwards:
// it restores a checkpoint, recomputes the segment recording each step's
// input state and contact history, and runs these kernels step by step in
// reverse.  Per step (contact set and every cap/clamp branch held as the
// forward took them):
//   k_adj_pre    force/torque adjoints from the velocity adjoints
//                (v' = v + dt F/m, w' = w + dt T/I, x' = x + dt v')
//   k_adj_step   per particle, the vector-Jacobian product of every contact
//                it takes part in (as owner and as partner, one code path,
//                like the forward kernel), accumulated into its own state
//                adjoints; the owner side writes the adjoint of the old
//                springs and the parameter adjoints (FP64)
//   k_adj_remap  at a segment boundary, maps spring adjoints from the new
//                candidate lists to the old ones (transpose of the forward
//                carry-over)
#include "lpr_kernels.h"

namespace lpr {

#define ADJ_INLINE __device__ __forceinline__

ADJ_INLINE float3 ld3(const float4& v) { return make_float3(v.x, v.y, v.z); }

__global__ void k_adj_pre(DevBufs d, AdjBufs a, int q) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  const uint32_t m = d.meta[i];
  if (m == INACTIVE) return;
  const BedConst& bc = d.beds[m >> 8];
  const int64_t N = d.N;
  const float4 v = a.st[(int64_t)q * N + i].v;
  const float4 w = a.st[(int64_t)q * N + i].w;
  const float4 xb = a.xb[i], vb = a.vb[i], wb = a.wb[i];
  // x' = x + dt v'  ->  adjoint of v' gains dt xb
  const float vx = vb.x + bc.dt * xb.x, vy = vb.y + bc.dt * xb.y, vz = vb.z + bc.dt * xb.z;
  a.vb[i] = make_float4(vx, vy, vz, 0.f);
  const float fm = bc.dt * v.w, ti = bc.dt * w.w;
  a.Fb[i] = make_float4(fm * vx, fm * vy, fm * vz, 0.f);
  a.Tb[i] = make_float4(ti * wb.x, ti * wb.y, ti * wb.z, 0.f);
}

void launch_adj_pre(const DevBufs& d, const AdjBufs& a, int q, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_pre, dim3((unsigned)(d.N / 256)), dim3(256), 0, st, d, a, q);
}

// Wall geometry adjoint: adds to xb the effect of (delta_b, n_b) through the
// particle position.  Planes and disk/annulus faces have a fixed normal.
ADJ_INLINE void wall_geom_vjp(const WallPose& W, double x, double y, double z, double r, float deltab, float3 nb,
                              float3& xb) {
  const double rx = x - W.o[0], ry = y - W.o[1], rz = z - W.o[2];
  const float3 nu = f3((float)W.nu[0], (float)W.nu[1], (float)W.nu[2]);
  if (W.kind == WPLANE) {  // delta = r - (x - o).nu
    xb = xb - deltab * nu;
    return;
  }
  if (W.kind == WDISK || W.kind == WANNULUS) {
    const double s = dot3d(rx, ry, rz, W.nu[0], W.nu[1], W.nu[2]);
    const double vx = rx - s * W.nu[0], vy = ry - s * W.nu[1], vz = rz - s * W.nu[2];
    const double rho2 = dot3d(vx, vy, vz, vx, vy, vz);
    const double Rin = (W.kind == WDISK) ? 0.0 : W.dims[0];
    const double Rout = (W.kind == WDISK) ? W.dims[0] : W.dims[1];
    if (rho2 <= Rout * Rout && rho2 >= Rin * Rin) {
      xb = xb - deltab * nu;
      return;
    }
    // rim: D = c(x) - x, c on the circle of radius Rc
    const double Rc = (rho2 > Rout * Rout) ? Rout : Rin;
    const double rho = sqrt(rho2);
    const float3 rh = f3((float)(vx / rho), (float)(vy / rho), (float)(vz / rho));
    const double f = Rc / rho;
    const double cx = W.o[0] + f * vx, cy = W.o[1] + f * vy, cz = W.o[2] + f * vz;
    const float3 D = f3((float)(cx - x), (float)(cy - y), (float)(cz - z));
    const float dist = sqrtf(dot(D, D));
    const float3 n = (1.0f / dist) * D;
    const float3 Db = (1.0f / dist) * (nb - dot(nb, n) * n) - deltab * n;
    // dc/dx = (Rc/rho) (I - rh rh^T)(I - nu nu^T), symmetric
    float3 w = Db - dot(Db, nu) * nu;
    w = w - dot(w, rh) * rh;
    xb = xb + (float)f * w - Db;
    return;
  }
  // box
  double l[3];
  bool inside = true;
  for (int q = 0; q < 3; ++q) {
    l[q] = dot3d(rx, ry, rz, W.e[q][0], W.e[q][1], W.e[q][2]);
    if (!(fabs(l[q]) < W.dims[q])) inside = false;
  }
  if (inside) {
    int best = 0;
    double bestgap = W.dims[0] - fabs(l[0]);
    for (int q = 1; q < 3; ++q) {
      const double gp = W.dims[q] - fabs(l[q]);
      if (gp < bestgap) { bestgap = gp; best = q; }
    }
    const float sg = (l[best] >= 0.0) ? 1.0f : -1.0f;
    const float3 e = f3((float)W.e[best][0], (float)W.e[best][1], (float)W.e[best][2]);
    xb = xb - (sg * deltab) * e;
    return;
  }
  double cl[3];
  bool free_ax[3];
  for (int q = 0; q < 3; ++q) {
    free_ax[q] = !(l[q] > W.dims[q] || l[q] < -W.dims[q]);
    cl[q] = (l[q] > W.dims[q]) ? W.dims[q] : ((l[q] < -W.dims[q]) ? -W.dims[q] : l[q]);
  }
  double cx = W.o[0] + cl[0] * W.e[0][0], cy = W.o[1] + cl[0] * W.e[0][1], cz = W.o[2] + cl[0] * W.e[0][2];
  cx = cx + cl[1] * W.e[1][0]; cy = cy + cl[1] * W.e[1][1]; cz = cz + cl[1] * W.e[1][2];
  cx = cx + cl[2] * W.e[2][0]; cy = cy + cl[2] * W.e[2][1]; cz = cz + cl[2] * W.e[2][2];
  const float3 D = f3((float)(cx - x), (float)(cy - y), (float)(cz - z));
  const float dist = sqrtf(dot(D, D));
  const float3 n = (1.0f / dist) * D;
  const float3 Db = (1.0f / dist) * (nb - dot(nb, n) * n) - deltab * n;
  float3 w = zero3();
  for (int q = 0; q < 3; ++q)
    if (free_ax[q]) {
      const float3 e = f3((float)W.e[q][0], (float)W.e[q][1], (float)W.e[q][2]);
      w = w + dot(Db, e) * e;
    }
  xb = xb + w - Db;
}

constexpr int ADJ_BS = 128;

__global__ __launch_bounds__(ADJ_BS) void k_adj_step(DevBufs d, AdjBufs a, int q, int hp, int obj_body,
                                                     float invT) {
  const int64_t N = d.N;
  const int64_t i = blockIdx.x * (int64_t)ADJ_BS + threadIdx.x;
  if (i >= N) return;
  const uint32_t m = d.meta[i];
  if (m == INACTIVE) return;
  const BedConst bc = d.beds[m >> 8];
  const int hn = hp ^ 1;
  const PState* S = a.st + (int64_t)q * N;
  const uint32_t* CF = a.cflag + (int64_t)q * N;
  const HRec* HS = a.hist + (int64_t)q * K * N;
  const PState me = S[i];
  const double4 xi = me.x;
  const float4 vi = me.v, wi = me.w;
  const float3 Fbi = ld3(a.Fb[i]), Tbi = ld3(a.Tb[i]);
  float3 xba = zero3(), vba = zero3(), wba = zero3();
  double th0 = 0.0, th1 = 0.0, th2 = 0.0;
  const uint32_t fold = CF[i];
  const int n_own = a.own_cnt[i];
  const uint32_t rs = a.rev_start[i];
  const int n_tot = n_own + (int)(a.rev_start[i + 1] - rs);
  for (int e = 0; e < n_tot; ++e) {
    int64_t o, qq;
    int k;
    const bool mine = e < n_own;
    if (mine) {
      k = e;
      o = i;
      qq = a.own_idx[k * N + i];
    } else {
      const uint32_t pk = a.rev_ent[rs + (e - n_own)];
      o = pk >> 4;
      k = (int)(pk & 15u);
      qq = i;
    }
    const int64_t other = mine ? qq : o;
    const PState ot = S[other];
    const double4 xo_ = ot.x;
    const float4 vo_ = ot.v, wo_ = ot.w;
    const double4 xa = mine ? xi : xo_, xb = mine ? xo_ : xi;
    const float4 va = mine ? vi : vo_, vb = mine ? vo_ : vi;
    const float4 wa = mine ? wi : wo_, wb = mine ? wo_ : wi;
    double dx, dy, dz;
    const double d2 = pair_sep(bc, xa, xb, dx, dy, dz);
    if (!sphere_touch(d2, xa.w, xb.w)) {
      if (mine) {  // no contact: the spring is dropped, no adjoint flows back
        a.hbA[hn][k * N + i] = make_float4(0.f, 0.f, 0.f, 0.f);
        a.hbB[hn][k * N + i] = make_float2(0.f, 0.f);
      }
      continue;
    }
    const uint32_t fo = mine ? fold : CF[o];
    const bool valid = (fo >> k) & 1u;
    LawIn in;
    if (valid) {
      const HRec hr = HS[k * N + o];
      in.xt = f3(hr.t.x, hr.t.y, hr.t.z);
      in.xr = f3(hr.r.x, hr.r.y, hr.r.z);
    } else {
      in.xt = zero3();
      in.xr = zero3();
    }
    // the forward kernel's expressions, verbatim
    const double dist = sqrt(d2);
    const double dl = (xa.w + xb.w) - dist;
    const float ra = (float)xa.w, rb = (float)xb.w;
    in.delta = (float)dl;
    const float idist = (d2 > 0.0) ? 1.0f / (float)dist : 0.0f;
    if (d2 > 0.0) in.n = f3((float)dx * idist, (float)dy * idist, (float)dz * idist);
    else in.n = f3(0.f, 0.f, 1.f);
    const float la = ra - 0.5f * in.delta, lb = rb - 0.5f * in.delta;
    const float3 wa3 = ld3(wa), wb3 = ld3(wb);
    in.u = f3(va.x - vb.x, va.y - vb.y, va.z - vb.z) + la * cross(wa3, in.n) + lb * cross(wb3, in.n);
    in.wrel = wa3 - wb3;
    in.dstar = 2.0f * ra * rb / (ra + rb);
    in.mu_t = bc.mu_t;
    in.mu_r = bc.mu_r;
    LawTape tp;
    LawOut out;
    law_forward(bc, in, tp, out);
    // adjoints of the outputs: F_a += F, T_a += la (n x Ft) + M,
    // F_b -= F, T_b += lb (n x Ft) - M
    const float3 Fbo = ld3(a.Fb[other]), Tbo = ld3(a.Tb[other]);
    const float3 Fba = mine ? Fbi : Fbo, Fbb = mine ? Fbo : Fbi;
    const float3 Tba = mine ? Tbi : Tbo, Tbb = mine ? Tbo : Tbi;
    const float4 h4 = a.hbA[hp][k * N + o];
    const float2 h2 = a.hbB[hp][k * N + o];
    const float3 nft = cross(in.n, out.Ft);
    const float3 A = la * Tba + lb * Tbb;
    LawBar r;
    law_vjp(bc, in, tp, out, Fba - Fbb, cross(A, in.n), Tba - Tbb, f3(h4.x, h4.y, h4.z), f3(h4.w, h2.x, h2.y), r);
    float3 nb = r.n + cross(out.Ft, A);
    float lab = dot(Tba, nft) + dot(r.u, cross(wa3, in.n));
    float lbb = dot(Tbb, nft) + dot(r.u, cross(wb3, in.n));
    const float3 nxu = cross(in.n, r.u);
    const float3 wab = la * nxu + r.wrel, wbb = lb * nxu - r.wrel;
    nb = nb + la * cross(r.u, wa3) + lb * cross(r.u, wb3);
    const float deltab = r.delta - 0.5f * (lab + lbb);
    const float3 Db = idist * (nb - dot(nb, in.n) * in.n) - deltab * in.n;  // adjoint of x_b - x_a
    if (mine) {
      xba = xba - Db;
      vba = vba + r.u;
      wba = wba + wab;
      th0 += (double)(r.kn * tp.kn / bc.s_k);
      th1 += (double)r.mu_t;
      th2 += (double)r.mu_r;
      a.hbA[hn][k * N + i] = valid ? make_float4(r.xt.x, r.xt.y, r.xt.z, r.xr.x) : make_float4(0.f, 0.f, 0.f, 0.f);
      a.hbB[hn][k * N + i] = valid ? make_float2(r.xr.y, r.xr.z) : make_float2(0.f, 0.f);
    } else {
      xba = xba + Db;
      vba = vba - r.u;
      wba = wba + wbb;
    }
  }
  // walls
  const WallPose* WP = a.walls + (int64_t)q * a.nwall_total;
  for (int w = 0; w < bc.nwall; ++w) {
    const WallPose& W = WP[bc.wall0 + w];
    double dl, nx, ny, nz;
    const bool hit = wall_geom(W, xi.x, xi.y, xi.z, xi.w, dl, nx, ny, nz);
    if (!hit) {
      a.wbA[hn][w * N + i] = make_float4(0.f, 0.f, 0.f, 0.f);
      a.wbB[hn][w * N + i] = make_float2(0.f, 0.f);
      continue;
    }
    const bool valid = (fold >> (WALL_BIT + w)) & 1u;
    LawIn in;
    if (valid) {
      const float4 a4 = a.wA[((int64_t)q * a.nwall_max + w) * N + i];
      const float2 b2 = a.wB[((int64_t)q * a.nwall_max + w) * N + i];
      in.xt = f3(a4.x, a4.y, a4.z);
      in.xr = f3(a4.w, b2.x, b2.y);
    } else {
      in.xt = zero3();
      in.xr = zero3();
    }
    const float ra = (float)xi.w;
    in.delta = (float)dl;
    in.n = f3((float)nx, (float)ny, (float)nz);
    const float la = ra - 0.5f * in.delta;
    const double px = xi.x + (double)la * nx, py = xi.y + (double)la * ny;
    const double rx = px - W.c[0], ry = py - W.c[1];
    const float3 uw = f3((float)(W.vel[0] - W.omega * ry), (float)(W.vel[1] + W.omega * rx), (float)W.vel[2]);
    const float3 wa3 = ld3(wi);
    in.u = ld3(vi) + la * cross(wa3, in.n) - uw;
    in.wrel = f3(wi.x, wi.y, wi.z - (float)W.omega);
    in.dstar = 2.0f * ra;
    in.mu_t = (W.mu_t < 0.f) ? bc.mu_t : W.mu_t;
    in.mu_r = (W.mu_r < 0.f) ? bc.mu_r : W.mu_r;
    LawTape tp;
    LawOut out;
    law_forward(bc, in, tp, out);
    float3 Fb = Fbi;
    if (bc.body0 + W.body == obj_body) Fb.z -= invT;  // J gains -F_z / T for each contact with the body
    const float4 h4 = a.wbA[hp][w * N + i];
    const float2 h2 = a.wbB[hp][w * N + i];
    const float3 A = la * Tbi;
    LawBar r;
    law_vjp(bc, in, tp, out, Fb, cross(A, in.n), Tbi, f3(h4.x, h4.y, h4.z), f3(h4.w, h2.x, h2.y), r);
    const float3 nb = r.n + cross(out.Ft, A) + la * cross(r.u, wa3);
    const float lab = dot(Tbi, cross(in.n, out.Ft)) + dot(r.u, cross(wa3, in.n));
    vba = vba + r.u;
    wba = wba + la * cross(in.n, r.u) + r.wrel;
    wall_geom_vjp(W, xi.x, xi.y, xi.z, xi.w, r.delta - 0.5f * lab, nb, xba);
    th0 += (double)(r.kn * tp.kn / bc.s_k);
    if (W.mu_t < 0.f) th1 += (double)r.mu_t;
    if (W.mu_r < 0.f) th2 += (double)r.mu_r;
    a.wbA[hn][w * N + i] = valid ? make_float4(r.xt.x, r.xt.y, r.xt.z, r.xr.x) : make_float4(0.f, 0.f, 0.f, 0.f);
    a.wbB[hn][w * N + i] = valid ? make_float2(r.xr.y, r.xr.z) : make_float2(0.f, 0.f);
  }
  const float4 x0 = a.xb[i], v0 = a.vb[i], w0 = a.wb[i];
  a.xb[i] = make_float4(x0.x + xba.x, x0.y + xba.y, x0.z + xba.z, 0.f);
  a.vb[i] = make_float4(v0.x + vba.x, v0.y + vba.y, v0.z + vba.z, 0.f);
  a.wb[i] = make_float4(w0.x + wba.x, w0.y + wba.y, w0.z + wba.z, 0.f);
  a.theta[3 * i + 0] += th0;
  a.theta[3 * i + 1] += th1;
  a.theta[3 * i + 2] += th2;
}

void launch_adj_step(const DevBufs& d, const AdjBufs& a, int q, int hp, int obj_body, float invT, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_step, dim3((unsigned)(d.N / ADJ_BS)), dim3(ADJ_BS), 0, st, d, a, q, hp, obj_body, invT);
}

// Spring adjoints of the new lists (slot k, buffer hp) -> old lists (slot
// k', buffer hp^1): the forward copied old slot k' into new slot k when the
// partner matched and the old spring was live; otherwise the new spring
// started at zero and nothing flows back.
__global__ void k_adj_remap(DevBufs d, AdjBufs a, const int32_t* old_cnt, const int32_t* old_idx,
                            const uint32_t* old_flag, int hp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  const uint32_t m = d.meta[i];
  if (m == INACTIVE) return;
  const BedConst& bc = d.beds[m >> 8];
  const int64_t N = d.N;
  const int hn = hp ^ 1;
  const int cnt_old = old_cnt[i], cnt_new = a.own_cnt[i];
  const uint32_t fo = old_flag[i];
  for (int k2 = 0; k2 < cnt_old; ++k2) {
    float4 A4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 B2 = make_float2(0.f, 0.f);
    if ((fo >> k2) & 1u) {
      const int32_t j = old_idx[k2 * N + i];
      for (int k = 0; k < cnt_new; ++k)
        if (a.own_idx[k * N + i] == j) {
          A4 = a.hbA[hp][k * N + i];
          B2 = a.hbB[hp][k * N + i];
          break;
        }
    }
    a.hbA[hn][k2 * N + i] = A4;
    a.hbB[hn][k2 * N + i] = B2;
  }
  for (int w = 0; w < bc.nwall; ++w) {
    const bool live = (fo >> (WALL_BIT + w)) & 1u;
    a.wbA[hn][w * N + i] = live ? a.wbA[hp][w * N + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    a.wbB[hn][w * N + i] = live ? a.wbB[hp][w * N + i] : make_float2(0.f, 0.f);
  }
}

void launch_adj_remap(const DevBufs& d, const AdjBufs& a, const int32_t* old_cnt, const int32_t* old_idx,
                      const uint32_t* old_flag, int hp, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_remap, dim3((unsigned)(d.N / 256)), dim3(256), 0, st, d, a, old_cnt, old_idx, old_flag,
                     hp);
}

// Ordered FP64 sum of the per-particle parameter adjoints (one block).
__global__ void k_adj_theta(DevBufs d, AdjBufs a, double* out3) {
  __shared__ double red[256];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < d.N; i += 256) acc += a.theta[3 * i + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out3[c] = red[0];
    __syncthreads();
  }
}

void launch_adj_theta(const DevBufs& d, const AdjBufs& a, double* out3, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_theta, dim3(1), dim3(256), 0, st, d, a, out3);
}

}  // namespace lpr
