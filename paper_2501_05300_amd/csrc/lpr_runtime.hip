// lpr_runtime.hip -- host runtime behind the C ABI of include/lprdem.h.
//
// A stepper instance holds one or more beds back to back in device memory
// (each bed padded to a multiple of PAD particles).  The host keeps the
// ping-pong parities of state, history and candidate lists, enqueues the
// rebuild and step kernels, and replays a captured HIP graph for the steady
// cycle of 2 * rebuild_every steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "lpr_cells.h"
#include "lpr_kernels.h"
#include "lpr_spook.h"
#include "lprdem.h"

using namespace lpr;

namespace {

thread_local std::string g_last_error;

lpr_status fail(lpr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIPTRY(expr)                                                                                \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fail(LPR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct HostBed {
  int64_t n = 0;       // particles
  int64_t p0 = 0;      // first storage index
  int64_t npad = 0;    // padded count
  std::vector<int64_t> perm;  // storage offset -> stable id at creation (a re-sort changes it; the
                              // device's sid array is the current map)
  int nwall = 0, nbody = 0, nlev = 0;
  int wall0 = 0, body0 = 0, lev0 = 0;
  double dt = 0.0;
  double rmin = 0.0;
  // largest skin the cell plan covers: one-cell stencils find every pair
  // closer than r_i + r_j + skin_cap at the time the lists are built
  double skin_cap = 0.0;
  lpr_params params{};
  std::vector<lpr_body> bodies;
};

uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

bool finite_arr(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}
bool finite_arrf(const float* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

// Host view of the buffer parities (state, history, lists, storage order)
// and the steps since the last broad-phase rebuild.
struct Par {
  int s = 0, h = 0, l = 0;
  int o = 0;   // storage order: flips at each re-sort
  int sc = 0;  // rebuilds since the last re-sort, modulo the sort cadence
  int64_t since = std::numeric_limits<int64_t>::max() / 2;
};

struct lpr_bed {
  lpr_allocator alloc{};
  bool use_hip_malloc = true;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void*> blocks;
  DevBufs d{};
  std::vector<HostBed> hb;
  int block = 64;
  int persist_blocks = 0;  // > 0: persistent step kernel with this grid
  int record = 0;
  int R = 1;      // configured rebuild cadence
  int R_eff = 1;  // cadence in use (halved after a skin trip, restored per lpr_step)
  float skin = 0.f;
  // storage-order sort: every sort_every-th rebuild (0: never) re-sorts the
  // particles by (bed, level, Morton code of the cell); the sorted copies go
  // to the second buffer of each pair below and the pairs swap (order parity o)
  int sort_every = 0;
  bool sort_hold = false;  // suspended (adjoint windows keep one order)
  int o = 0, sc = 0;
  int64_t sorts = 0;
  int32_t* sid_alt = nullptr;
  uint32_t* meta_alt = nullptr;
  int32_t* pcell_alt = nullptr;
  uint32_t* prank_alt = nullptr;
  int go = 0;  // order parity the captured cycle starts from
  // phase timing: when set, the enqueue functions record these events at the
  // phase boundaries of the step being enqueued (see lpr_step_phases)
  hipEvent_t* pev = nullptr;
  int device = 0;                 // the GPU the bed lives on
  char* ld_ws = nullptr;          // workspace of the per-contact read (grown on demand)
  size_t ld_ws_bytes = 0;
  // host parities
  int s = 0, h = 0, l = 0;
  int64_t since = std::numeric_limits<int64_t>::max() / 2;  // steps since the last rebuild
  int64_t host_steps = 0;
  int64_t rebuilds = 0;
  // parity log since the last clean sync, for rewinding after a skin trip
  int64_t base_steps = 0;
  Par base_par;
  std::vector<Par> plog;
  int64_t skin_trips = 0;
  // captured cycle
  bool has_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gs = 0, gh = 0, gl = 0;
  int gsteps = 0;
  int nlev_total = 0;
  int64_t ncells = 0;
  int max_walls = 0;
  bool faulted = false;
  lpr_status fault_status = LPR_OK;
  // adjoint storage (allocated on first use, grown as needed)
  AdjBufs adj{};
  int adj_steps = 0;      // per-step records available
  int adj_ckpts = 0;      // checkpoints available
  int adj_interval = 0;   // checkpoint interval the last adjoint window used
  struct Ckpt {
    PState* st;
    uint32_t* cflag; HRec* hist; float4* wA; float2* wB;
    int32_t* own_cnt; int32_t* own_idx;
    BedDyn* bedyn; BodyDyn* bdyn;
    int s, h, l;
    int64_t since, host_steps, rebuilds;
  };
  std::vector<Ckpt> ckpts;
  double* theta_out = nullptr;
  // time-implicit stepper (allocated on first selection)
  int stepper = LPR_STEPPER_EXPLICIT;
  int n_iter = 0;
  bool sp_ready = false;
  SpBufs sp{};

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (use_hip_malloc) {
      if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    } else {
      p = alloc.alloc(alloc.ctx, bytes);
    }
    if (p) blocks.push_back(p);
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    for (size_t q = 0; q < blocks.size(); ++q)
      if (blocks[q] == p) {
        blocks.erase(blocks.begin() + (long)q);
        break;
      }
    if (use_hip_malloc) (void)hipFree(p);
    else alloc.release(alloc.ctx, p);
  }
  void release_all() {
    for (void* p : blocks) {
      if (use_hip_malloc) (void)hipFree(p);
      else alloc.release(alloc.ctx, p);
    }
    blocks.clear();
  }
};

namespace {

template <class T>
bool dal(lpr_bed* b, T** out, size_t count) {
  *out = (T*)b->dalloc(sizeof(T) * (count ? count : 1));
  return *out != nullptr;
}

lpr_status validate(const lpr_bed_desc* d) {
  if (!d) return fail(LPR_E_INVAL, "null description");
  if (d->n <= 0) return fail(LPR_E_INVAL, "n must be > 0");
  if (d->n >= (int64_t(1) << 27)) return fail(LPR_E_INVAL, "n too large for packed contact entries");
  if (!d->pos || !d->radius) return fail(LPR_E_INVAL, "pos and radius are required");
  const lpr_params& p = d->params;
  if (!(p.dt > 0.0) || !(p.rho > 0.0) || !(p.E > 0.0) || !(p.nu > -1.0 && p.nu < 0.5))
    return fail(LPR_E_INVAL, "invalid material parameters or dt");
  if (!(p.e_H >= 1.0) || !(p.kappa_t >= 0.0) || !(p.s_k > 0.0) || !(p.gamma_factor >= 0.0) || !(p.mu_t >= 0.0) ||
      !(p.mu_r >= 0.0))
    return fail(LPR_E_INVAL, "invalid contact-law parameters");
  if (!finite_arr(d->pos, 3 * d->n)) return fail(LPR_E_INVAL, "non-finite position");
  if (d->vel && !finite_arrf(d->vel, 3 * d->n)) return fail(LPR_E_INVAL, "non-finite velocity");
  if (d->omega && !finite_arrf(d->omega, 3 * d->n)) return fail(LPR_E_INVAL, "non-finite angular velocity");
  for (int64_t i = 0; i < d->n; ++i)
    if (!(d->radius[i] > 0.f) || !std::isfinite(d->radius[i])) return fail(LPR_E_INVAL, "radius must be > 0");
  if (d->n_walls < 0 || d->n_walls > LPR_MAX_WALLS) return fail(LPR_E_INVAL, "too many walls");
  if (d->n_bodies < 0 || d->n_bodies > LPR_MAX_BODIES) return fail(LPR_E_INVAL, "too many bodies");
  if (d->n_walls > 0 && (!d->walls || d->n_bodies == 0 || !d->bodies))
    return fail(LPR_E_INVAL, "walls need bodies");
  for (int w = 0; w < d->n_walls; ++w) {
    const lpr_wall& W = d->walls[w];
    if (W.kind < 0 || W.kind > 3 || W.body < 0 || W.body >= d->n_bodies)
      return fail(LPR_E_INVAL, "wall kind or body out of range");
  }
  for (int q = 0; q < d->n_bodies; ++q)
    if (d->bodies[q].z_free && !(d->bodies[q].mass > 0.0)) return fail(LPR_E_INVAL, "a z_free body needs mass > 0");
  if (d->rebuild_every < 0 || (d->rebuild_every > 1 && !(d->skin > 0.f)))
    return fail(LPR_E_INVAL, "rebuild_every > 1 needs skin > 0");
  if (d->skin < 0.f) return fail(LPR_E_INVAL, "skin must be >= 0");
  if (d->band_ratio != 0.f && !(d->band_ratio > 1.f)) return fail(LPR_E_INVAL, "band_ratio must be > 1");
  if (d->cell_factor != 0.f && !(d->cell_factor >= 1.f)) return fail(LPR_E_INVAL, "cell_factor must be >= 1");
  if (d->block != 0 && d->block != 64 && d->block != 128 && d->block != 256)
    return fail(LPR_E_INVAL, "block must be 64, 128 or 256");
  if (d->sort_every > 4096) return fail(LPR_E_INVAL, "sort_every must be at most 4096");
  for (int q = 0; q < MAXLEV; ++q)
    if (d->level_cell_factor[q] != 0.f && !(d->level_cell_factor[q] >= 1.f))
      return fail(LPR_E_INVAL, "level_cell_factor entries must be 0 or >= 1");
  float rmax = 0.f;
  for (int64_t i = 0; i < d->n; ++i) rmax = std::max(rmax, d->radius[i]);
  for (int a = 0; a < 2; ++a)
    if ((d->periodic >> a) & 1u)
      if (!(d->box[a] > 2.0 * (2.0 * (double)rmax + (double)d->skin)))
        return fail(LPR_E_INVAL, "periodic length must exceed 2 max(r_i + r_j + skin)");
  return LPR_OK;
}

// Builds radius bands, level grids and the Morton storage order of one bed.
void plan_bed(const lpr_bed_desc* D, double band_ratio, double cell_factor, double skin, bool input_order, HostBed& H,
              std::vector<LevelGrid>& levels, int64_t& cell_base, std::vector<uint8_t>& lev_of) {
  const int64_t n = D->n;
  double rlo = std::numeric_limits<double>::max();
  for (int64_t i = 0; i < n; ++i) rlo = std::min(rlo, (double)D->radius[i]);
  double thr[MAXLEV + 1];
  for (int q = 0; q <= MAXLEV; ++q) thr[q] = rlo * std::pow(band_ratio, (double)q);
  lev_of.assign(n, 0);
  int nlev = 1;
  for (int64_t i = 0; i < n; ++i) {
    const double r = D->radius[i];
    int q = 0;
    while (q + 1 < MAXLEV && thr[q + 1] <= r) ++q;
    lev_of[i] = (uint8_t)q;
    nlev = std::max(nlev, q + 1);
  }
  std::vector<double> rmax(nlev, 0.0), zlo(nlev, 1e300), zhi(nlev, -1e300), xlo(nlev, 1e300), xhi(nlev, -1e300),
      ylo(nlev, 1e300), yhi(nlev, -1e300);
  for (int64_t i = 0; i < n; ++i) {
    const int q = lev_of[i];
    rmax[q] = std::max(rmax[q], (double)D->radius[i]);
    xlo[q] = std::min(xlo[q], D->pos[3 * i]); xhi[q] = std::max(xhi[q], D->pos[3 * i]);
    ylo[q] = std::min(ylo[q], D->pos[3 * i + 1]); yhi[q] = std::max(yhi[q], D->pos[3 * i + 1]);
    zlo[q] = std::min(zlo[q], D->pos[3 * i + 2]); zhi[q] = std::max(zhi[q], D->pos[3 * i + 2]);
  }
  H.lev0 = (int)levels.size();
  H.nlev = nlev;
  H.skin_cap = std::numeric_limits<double>::max();
  for (int q = 0; q < nlev; ++q) {
    LevelGrid G{};
    double rm = rmax[q] > 0.0 ? rmax[q] : thr[q + 1];
    if (rmax[q] <= 0.0) { xlo[q] = xhi[q] = ylo[q] = yhi[q] = zlo[q] = zhi[q] = 0.0; }
    const double cf_q = D->level_cell_factor[q] > 0.f ? (double)D->level_cell_factor[q] : cell_factor;
    const double hcell = cf_q * (2.0 * rm + skin);
    const double lo3[3] = {xlo[q], ylo[q], zlo[q]}, hi3[3] = {xhi[q], yhi[q], zhi[q]};
    for (int a = 0; a < 3; ++a) {
      const bool per = (a < 2) && ((D->periodic >> a) & 1u);
      if (per) {
        const int nc = std::max(1, (int)std::floor(D->box[a] / hcell));
        G.n[a] = nc;
        G.lo[a] = 0.0;
        G.inv_w[a] = (double)nc / D->box[a];
        G.w[a] = D->box[a] / (double)nc;
        G.per[a] = 1;
      } else {
        const double lo = lo3[a] - 2.0 * hcell, hi = hi3[a] + 2.0 * hcell;
        int nc = (int)std::ceil((hi - lo) / hcell);
        nc = std::max(1, std::min(nc, 1 << 20));
        G.n[a] = nc;
        G.lo[a] = lo;
        G.inv_w[a] = 1.0 / hcell;
        G.w[a] = hcell;
        G.per[a] = 0;
      }
    }
    if (rmax[q] > 0.0) {
      // the widest pair of this level (both radii at rm) is the one that
      // needs the most room; pairs with a finer particle need less
      double w = hcell;
      for (int a = 0; a < 3; ++a) w = std::min(w, 1.0 / G.inv_w[a]);
      H.skin_cap = std::min(H.skin_cap, w - 2.0 * rm);
    }
    G.base = cell_base;
    G.rmax = rm;
    cell_base += (int64_t)G.n[0] * G.n[1] * G.n[2];
    levels.push_back(G);
  }
  // storage order: level, then Morton code of the cell, then stable id (the
  // order a device re-sort keeps); or the caller's order
  H.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) H.perm[i] = i;
  if (input_order) return;
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    const LevelGrid& G = levels[H.lev0 + lev_of[i]];
    const uint64_t cx = (uint64_t)cell_axis(G, 0, D->pos[3 * i]);
    const uint64_t cy = (uint64_t)cell_axis(G, 1, D->pos[3 * i + 1]);
    const uint64_t cz = (uint64_t)cell_axis(G, 2, D->pos[3 * i + 2]);
    key[i] = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
  }
  std::sort(H.perm.begin(), H.perm.end(), [&](int64_t a, int64_t b) {
    if (lev_of[a] != lev_of[b]) return lev_of[a] < lev_of[b];
    if (key[a] != key[b]) return key[a] < key[b];
    return a < b;
  });
}

Par cur_par(const lpr_bed* b) {
  Par p;
  p.s = b->s; p.h = b->h; p.l = b->l; p.o = b->o; p.sc = b->sc; p.since = b->since;
  return p;
}

// Swaps every buffer pair that a re-sort writes: the state pair (the sorted
// state goes to the buffer the next step would write), stable ids, metadata,
// cells and cell ranks.
void swap_order(lpr_bed* b) {
  std::swap(b->d.st[0], b->d.st[1]);
  std::swap(b->d.sid, b->sid_alt);
  std::swap(b->d.meta, b->meta_alt);
  std::swap(b->d.pcell, b->pcell_alt);
  std::swap(b->d.prank, b->prank_alt);
  b->o ^= 1;
}

void set_par(lpr_bed* b, const Par& p) {
  if (p.o != b->o) swap_order(b);
  b->s = p.s; b->h = p.h; b->l = p.l; b->sc = p.sc; b->since = p.since;
}

// Parity changes of one step, as enqueue_step makes them (R: the cadence of
// the captured cycle, S: rebuilds per re-sort, 0 for none).
void simulate_step(Par& p, int R, int S) {
  if (p.since >= R) {
    p.since = 0;
    if (S > 0) {
      if (p.sc == 0) {  // a re-sorting rebuild writes the other buffers
        p.o ^= 1;
        p.l ^= 1;
        p.h ^= 1;
      }
      p.sc = (p.sc + 1) % S;
    }
  }
  p.s ^= 1;
  p.h ^= 1;
  p.since += 1;
}

void enqueue_step(lpr_bed* b);

lpr_status sync_check(lpr_bed* b) {
  for (;;) {
    HIPTRY(hipStreamSynchronize(b->stream));
    uint32_t e = 0;
    HIPTRY(hipMemcpy(&e, b->d.err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (e == 0) {
      b->base_steps = b->host_steps;
      b->base_par = cur_par(b);
      b->plog.clear();
      return LPR_OK;
    }
    if (e != ERR_SKIN) break;
    // A particle moved more than skin/2 since the candidate lists were
    // built: the steps from there on were skipped whole.  Rewind the host
    // view to the last completed step, rebuild, and run the rest again.
    BedDyn bd;
    HIPTRY(hipMemcpy(&bd, b->d.bedyn, sizeof(BedDyn), hipMemcpyDeviceToHost));
    const int64_t done = bd.completed - b->base_steps;
    if (done < 0 || done > (int64_t)b->plog.size()) break;
    const Par p = (done == 0) ? b->base_par : b->plog[(size_t)(done - 1)];
    const int64_t remaining = b->host_steps - bd.completed;
    const uint32_t zero[2] = {0u, 0u};
    HIPTRY(hipMemcpy(b->d.err, zero, sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(b->d.viol, zero, 2 * sizeof(uint32_t), hipMemcpyHostToDevice));
    set_par(b, p);
    b->since = std::numeric_limits<int64_t>::max() / 2;
    b->host_steps = bd.completed;
    b->base_steps = bd.completed;
    b->base_par = cur_par(b);
    b->plog.clear();
    b->skin_trips += 1;
    b->R_eff = std::max(1, b->R_eff / 2);  // rebuild more often for the rest of this call
    for (int64_t q = 0; q < remaining; ++q) enqueue_step(b);
    HIPTRY(hipGetLastError());
  }
  uint32_t e = 0;
  HIPTRY(hipMemcpy(&e, b->d.err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  {
    // the device stopped at the last complete step: take the host view of
    // the buffers back to it (a re-sort enqueued after that step wrote only
    // the second buffers, so the state and ids of that step are intact)
    BedDyn bd;
    HIPTRY(hipMemcpy(&bd, b->d.bedyn, sizeof(BedDyn), hipMemcpyDeviceToHost));
    const int64_t done = bd.completed - b->base_steps;
    if (done >= 0 && done <= (int64_t)b->plog.size()) set_par(b, done == 0 ? b->base_par : b->plog[(size_t)(done - 1)]);
    b->faulted = true;
    if (e & ERR_CAPACITY) b->fault_status = LPR_E_CAPACITY;
    else if (e & ERR_NUMERIC) b->fault_status = LPR_E_NUMERIC;
    else if (e & ERR_WALL) b->fault_status = LPR_E_DOMAIN;
    else b->fault_status = LPR_E_STATE;
    return fail(b->fault_status, (e & ERR_CAPACITY) ? "a particle exceeded its contact slots"
                                : (e & ERR_NUMERIC) ? "non-finite force or state"
                                : (e & ERR_WALL)    ? "a particle passed through a plane wall"
                                                    : "latched device fault");
  }
  return LPR_OK;
}

void mark(lpr_bed* b, int k) {
  if (b->pev) (void)hipEventRecord(b->pev[k], b->stream);
}

void enqueue_rebuild(lpr_bed* b) {
  DevBufs& d = b->d;
  const bool srt = b->sort_every > 0 && !b->sort_hold && b->sc == 0;
  launch_zero(d.cell_cnt, d.ncells, d.rev_cnt, d.N, b->stream);
  launch_bin(d, b->s, srt ? 1 : 0, b->stream);
  launch_scan(d.cell_cnt, d.cell_start, d.scan_tmp, d.ncells, b->stream);
  mark(b, 1);
  if (srt) {
    const int passes = launch_sort(d, b->stream);
    launch_reorder(d, b->s, passes & 1, d.st[b->s ^ 1], b->sid_alt, b->meta_alt, b->pcell_alt, b->prank_alt,
                   b->stream);
    swap_order(b);
    b->sorts += 1;
  }
  if (b->sort_every > 0 && !b->sort_hold) b->sc = (b->sc + 1) % b->sort_every;
  mark(b, 2);
  launch_scatter(d, b->s, b->stream);
  mark(b, 3);
  launch_search(d, b->s, b->l, b->h, srt ? d.src : nullptr, b->stream);
  mark(b, 4);
  if (srt) {  // lists and springs moved to the other buffers (else updated in place)
    b->l ^= 1;
    b->h ^= 1;
  }
  launch_scan(d.rev_cnt, d.rev_start, d.scan_tmp, d.N, b->stream);
  launch_rev_scatter(d, b->l, b->stream);
  launch_rev_sort(d, b->stream);
  mark(b, 5);
  b->since = 0;
  b->rebuilds += 1;
}

// The contact solve of one step at the current parities (the rebuild, if
// any, already enqueued): the fused explicit step kernel, or the implicit
// step's rows, n_iter projected sweeps and finish.  Returns the block size
// whose reaction partials the body reduction reads.
int enqueue_contact_step(lpr_bed* b, hipStream_t sm) {
  if (b->stepper == LPR_STEPPER_SPOOK) {
    launch_sp_rows(b->d, b->sp, b->s, b->h, b->l, sm);
    launch_sp_vel(b->d, b->sp, b->s, b->l, 1, sm);
    for (int it = 0; it < b->n_iter; ++it) {
      launch_sp_contacts(b->d, b->sp, b->l, sm);
      launch_sp_vel(b->d, b->sp, b->s, b->l, 0, sm);
    }
    launch_sp_finish(b->d, b->sp, b->s, b->h, b->l, b->record, sm);
    return SP_BS;
  }
  StepPar p{b->s, b->h, b->l, false};
  launch_step(b->d, p, b->block, b->record, b->persist_blocks, sm);
  return b->block;
}

void enqueue_step(lpr_bed* b) {
  if (b->since >= b->R_eff) enqueue_rebuild(b);
  const int pb = enqueue_contact_step(b, b->stream);
  launch_advance(b->d, pb, b->stream);
  b->s ^= 1;
  b->h ^= 1;
  b->since += 1;
  b->host_steps += 1;
  b->plog.push_back(cur_par(b));
}

// Steps of the captured cycle: two re-sorts' worth of rebuilds (two
// rebuilds without sorting), so that every buffer pair is back where it
// started at the end of the cycle.
int cycle_steps(const lpr_bed* b) { return 2 * b->R * (b->sort_every > 0 ? b->sort_every : 1); }

lpr_status capture_cycle(lpr_bed* b) {
  const int S = cycle_steps(b);
  const Par p0 = cur_par(b);
  const int s0 = b->s, h0 = b->h, l0 = b->l, o0 = b->o;
  const int64_t since0 = b->since, steps0 = b->host_steps, reb0 = b->rebuilds, sorts0 = b->sorts;
  const size_t plog0 = b->plog.size();
  HIPTRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
  for (int q = 0; q < S; ++q) enqueue_step(b);
  hipGraph_t g = nullptr;
  HIPTRY(hipStreamEndCapture(b->stream, &g));
  hipGraphExec_t ex = nullptr;
  HIPTRY(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  b->graph = g;
  b->gexec = ex;
  b->gs = s0; b->gh = h0; b->gl = l0; b->go = o0;
  b->gsteps = S;
  b->has_graph = true;
  // the capture only recorded; restore the host view
  set_par(b, p0);
  b->host_steps = steps0; b->rebuilds = reb0; b->sorts = sorts0;
  b->plog.resize(plog0);
  (void)since0;
  return LPR_OK;
}

lpr_status guard(lpr_bed* b) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  if (b->faulted) return fail(LPR_E_STATE, "the bed has a latched fault");
  return LPR_OK;
}

lpr_status ensure_lists(lpr_bed* b) {
  if (b->since >= b->R_eff) enqueue_rebuild(b);
  return LPR_OK;
}

// Parity of the buffers holding the state after the completed steps.
lpr_status state_parity(lpr_bed* b, int* par) {
  BedDyn bd;
  if (!b->faulted) {
    lpr_status st = sync_check(b);
    if (st != LPR_OK && st != LPR_E_CAPACITY && st != LPR_E_NUMERIC) return st;
  }
  HIPTRY(hipStreamSynchronize(b->stream));
  HIPTRY(hipMemcpy(&bd, b->d.bedyn, sizeof(BedDyn), hipMemcpyDeviceToHost));
  *par = (int)(bd.completed & 1);
  return LPR_OK;
}

lpr_status create_impl(const lpr_bed_desc* const* descs, int nb, const lpr_allocator* alloc, void* stream,
                       lpr_bed** out) {
  if (!out) return fail(LPR_E_INVAL, "null output");
  *out = nullptr;
  if (nb <= 0 || !descs) return fail(LPR_E_INVAL, "no beds");
  for (int q = 0; q < nb; ++q) {
    lpr_status st = validate(descs[q]);
    if (st != LPR_OK) return st;
  }
  const lpr_bed_desc& D0 = *descs[0];
  lpr_bed* b = new lpr_bed();
  if (alloc && alloc->alloc && alloc->release) {
    b->alloc = *alloc;
    b->use_hip_malloc = false;
  }
  if (stream) {
    b->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(LPR_E_DEVICE, "stream creation failed");
    }
    b->own_stream = true;
  }
  (void)hipGetDevice(&b->device);
  b->block = D0.block ? D0.block : 64;
  if (D0.persistent) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->persist_blocks = std::max(8, step_occupancy(b->block) * cus);
  }
  b->record = D0.record_forces ? 1 : 0;
  b->R = std::max(1, D0.rebuild_every);
  b->R_eff = b->R;
  b->skin = b->R > 1 ? D0.skin : 0.f;
  b->sort_every = D0.sort_every < 0 ? 0 : (D0.sort_every > 0 ? D0.sort_every : (b->R == 1 ? 16 : 1));

  // plan beds
  std::vector<LevelGrid> levels;
  std::vector<std::vector<uint8_t>> lev_of(nb);
  int64_t cell_base = 0, p = 0;
  int wall_total = 0, body_total = 0, max_walls = 1;
  b->hb.resize(nb);
  for (int q = 0; q < nb; ++q) {
    HostBed& H = b->hb[q];
    const lpr_bed_desc* D = descs[q];
    H.n = D->n;
    H.p0 = p;
    H.npad = (D->n + PAD - 1) / PAD * PAD;
    p += H.npad;
    const double band = D->band_ratio > 0.f ? D->band_ratio : 2.0;
    const double cfac = D->cell_factor > 0.f ? D->cell_factor : 1.0;
    plan_bed(D, band, cfac, (double)b->skin, D0.input_order != 0, H, levels, cell_base, lev_of[q]);
    H.nwall = D->n_walls;
    H.nbody = std::max(1, D->n_bodies);
    H.wall0 = wall_total;
    H.body0 = body_total;
    wall_total += H.nwall;
    body_total += H.nbody;
    max_walls = std::max(max_walls, H.nwall);
    H.dt = D->params.dt;
    H.params = D->params;
    H.bodies.assign(D->bodies, D->bodies + D->n_bodies);
    H.rmin = std::numeric_limits<double>::max();
    for (int64_t i = 0; i < D->n; ++i) H.rmin = std::min(H.rmin, (double)D->radius[i]);
  }
  if (cell_base >= (int64_t(1) << 31) - 2) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return fail(LPR_E_INVAL, "too many cells; raise cell_factor");
  }
  if (p >= (int64_t(1) << 27)) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return fail(LPR_E_INVAL, "too many particles for packed contact entries (padded total >= 2^27)");
  }
  b->nlev_total = (int)levels.size();
  b->ncells = cell_base;
  b->max_walls = max_walls;
  const int64_t N = p;
  DevBufs& d = b->d;
  d.N = N;
  d.nbeds = nb;
  d.ncells = cell_base;
  bool ok = true;
  for (int q = 0; q < 2; ++q) {
    ok &= dal(b, &d.st[q], N);
    ok &= dal(b, &d.own_idx[q], (size_t)K * N) && dal(b, &d.own_cnt[q], N);
    ok &= dal(b, &d.hist[q], (size_t)K * N);
    ok &= dal(b, &d.wA[q], (size_t)max_walls * N) && dal(b, &d.wB[q], (size_t)max_walls * N);
    ok &= dal(b, &d.cflag[q], N);
  }
  ok &= dal(b, &d.sid, N) && dal(b, &d.meta, N) && dal(b, &d.chunk_bed32, N / PAD);
  ok &= dal(b, &d.cell_cnt, cell_base) && dal(b, &d.cell_start, cell_base + 1);
  ok &= dal(b, &d.pcell, N) && dal(b, &d.prank, N) && dal(b, &d.cell_list, N);
  ok &= dal(b, &d.crec, N) && dal(b, &d.cpf, N + CPF_PAD) && dal(b, &d.zext, 2 * levels.size());
  ok &= dal(b, &d.disp, N) && dal(b, &d.viol, 2);
  ok &= dal(b, &d.own_rank, (size_t)K * N) && dal(b, &d.rev_cnt, N) && dal(b, &d.rev_start, N + 1);
  ok &= dal(b, &d.rev_ent, (size_t)K * N) && dal(b, &d.rev_tmp, (size_t)K * N);
  if (b->record) {
    ok &= dal(b, &d.frc, N) && dal(b, &d.trq, N);
    ok &= dal(b, &d.cF, (size_t)K * N) && dal(b, &d.cM, (size_t)K * N);
    ok &= dal(b, &d.wF, (size_t)max_walls * N) && dal(b, &d.wM, (size_t)max_walls * N);
  }
  d.nwall_max = max_walls;
  if (b->sort_every > 0) {
    for (int q = 0; q < 2; ++q) ok &= dal(b, &d.skey[q], N) && dal(b, &d.sval[q], N);
    ok &= dal(b, &d.rs_hist, sort_hist_elems(N)) && dal(b, &d.src, N);
    ok &= dal(b, &b->sid_alt, N) && dal(b, &b->meta_alt, N) && dal(b, &b->pcell_alt, N) && dal(b, &b->prank_alt, N);
  }
  d.sort_bits = 1;
  while ((int64_t(1) << d.sort_bits) <= cell_base) ++d.sort_bits;
  d.n_active = 0;
  for (const HostBed& H : b->hb) d.n_active += H.n;
  d.nblk = N / 64;
  ok &= dal(b, &d.partial, (size_t)d.nblk * 6 * std::max(1, body_total));
  ok &= dal(b, &d.adv_chunk, (size_t)nb * MAXB * ADV_CH * 6) && dal(b, &d.adv_cnt, (size_t)nb);
  ok &= dal(b, &d.scan_tmp, std::max(scan_tmp_elems(cell_base), scan_tmp_elems(N + 1)));
  ok &= dal(b, &d.beds, nb) && dal(b, &d.levels, levels.size());
  ok &= dal(b, &d.wdefs, std::max(1, wall_total)) && dal(b, &d.walls, std::max(1, wall_total));
  ok &= dal(b, &d.bdefs, body_total) && dal(b, &d.bdyn, body_total) && dal(b, &d.bedyn, nb);
  ok &= dal(b, &d.err, 1) && dal(b, &d.stat, 4);
  if (!ok) {
    b->release_all();
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return fail(LPR_E_NOMEM, "device allocation failed");
  }

  // host images
  std::vector<PState> hst(N);
  for (PState& p : hst) {
    p.x = make_double4(0, 0, 0, 0);
    p.v = make_float4(0, 0, 0, 0);
    p.w = make_float4(0, 0, 0, 0);
  }
  std::vector<int32_t> hsid(N, -1), hchunk(N / PAD, 0);
  std::vector<uint32_t> hmeta(N, INACTIVE);
  std::vector<BedConst> hbc(nb);
  std::vector<WallDef> hwd(std::max(1, wall_total));
  std::vector<BodyDef> hbd(body_total);
  std::vector<BodyDyn> hbdyn(body_total);
  std::vector<BedDyn> hbedyn(nb);
  for (int q = 0; q < nb; ++q) {
    const lpr_bed_desc* D = descs[q];
    HostBed& H = b->hb[q];
    const lpr_params& P = D->params;
    for (int64_t off = 0; off < H.n; ++off) {
      const int64_t i = H.perm[off];
      const int64_t sidx = H.p0 + off;
      const double r = (double)D->radius[i];
      const double m = P.rho * (4.0 / 3.0) * M_PI * r * r * r;
      const double I = 0.4 * m * r * r;
      hst[sidx].x = make_double4(D->pos[3 * i], D->pos[3 * i + 1], D->pos[3 * i + 2], r);
      hst[sidx].v = make_float4(D->vel ? D->vel[3 * i] : 0.f, D->vel ? D->vel[3 * i + 1] : 0.f,
                                D->vel ? D->vel[3 * i + 2] : 0.f, (float)(1.0 / m));
      hst[sidx].w = make_float4(D->omega ? D->omega[3 * i] : 0.f, D->omega ? D->omega[3 * i + 1] : 0.f,
                                D->omega ? D->omega[3 * i + 2] : 0.f, (float)(1.0 / I));
      hsid[sidx] = (int32_t)i;
      hmeta[sidx] = ((uint32_t)q << 8) | lev_of[q][i];
    }
    for (int64_t c = H.p0 / PAD; c < (H.p0 + H.npad) / PAD; ++c) hchunk[c] = q;
    BedConst& C = hbc[q];
    C.L[0] = D->box[0];
    C.L[1] = D->box[1];
    C.periodic = D->periodic & 3u;
    C.lev0 = H.lev0;
    C.nlev = H.nlev;
    C.wall0 = H.wall0;
    C.nwall = H.nwall;
    C.body0 = H.body0;
    C.nbody = H.nbody;
    C.p0 = (int32_t)H.p0;
    C.p1 = (int32_t)(H.p0 + H.npad);
    C.skin = b->skin;
    const double Estar = 1.0 / ((1.0 - P.nu * P.nu) / P.E + (1.0 - P.nu * P.nu) / P.E);
    C.kfac = (float)(P.s_k * Estar / 3.0);
    C.s_k = (float)P.s_k;
    C.gn = (float)(P.gamma_factor * P.dt);
    C.eH = (float)P.e_H;
    C.kappa_t = (float)P.kappa_t;
    C.mu_t = (float)P.mu_t;
    C.mu_r = (float)P.mu_r;
    C.dt = (float)P.dt;
    C.dt_d = P.dt;
    for (int a = 0; a < 3; ++a) C.g[a] = (float)P.g[a];
    C.law = (P.e_H == 1.25) ? 0 : (P.e_H == 1.0 ? 1 : 2);
    {
      int64_t before = 0;  // particles of the beds before this one
      for (int q2 = 0; q2 < q; ++q2) before += b->hb[q2].n;
      C.sort_off = (int32_t)(H.p0 - before);
    }
    for (int w = 0; w < H.nwall; ++w) {
      const lpr_wall& W = D->walls[w];
      WallDef& X = hwd[H.wall0 + w];
      for (int a = 0; a < 3; ++a) {
        X.origin[a] = W.origin[a];
        X.axis[a] = W.axis[a];
        X.dims[a] = W.dims[a];
      }
      for (int a = 0; a < 9; ++a) X.frame[a] = W.frame[a];
      X.mu_t = W.mu_t;
      X.mu_r = W.mu_r;
      X.kind = W.kind;
      X.body = W.body;
    }
    for (int q2 = 0; q2 < H.nbody; ++q2) {
      BodyDef& B = hbd[H.body0 + q2];
      BodyDyn& Y = hbdyn[H.body0 + q2];
      std::memset(&B, 0, sizeof(B));
      std::memset(&Y, 0, sizeof(Y));
      if (q2 < D->n_bodies) {
        const lpr_body& S = D->bodies[q2];
        for (int a = 0; a < 3; ++a) {
          B.origin[a] = S.origin[a];
          B.lin_vel[a] = S.lin_vel[a];
        }
        B.ang_vel = S.ang_vel;
        B.mass = S.mass;
        B.z_free = S.z_free;
        Y.z = S.origin[2];
        Y.vz = S.lin_vel[2];
      }
    }
    hbedyn[q].k = 0;
    hbedyn[q].completed = 0;
  }
  hipStream_t st = b->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  e = (hipError_t)(e | up(d.st[0], hst.data(), sizeof(PState) * N));
  e = (hipError_t)(e | up(d.st[1], hst.data(), sizeof(PState) * N));
  e = (hipError_t)(e | up(d.sid, hsid.data(), sizeof(int32_t) * N));
  e = (hipError_t)(e | up(d.meta, hmeta.data(), sizeof(uint32_t) * N));
  if (b->sort_every > 0) {  // padding keeps its marks in both buffers of each pair
    e = (hipError_t)(e | up(b->sid_alt, hsid.data(), sizeof(int32_t) * N));
    e = (hipError_t)(e | up(b->meta_alt, hmeta.data(), sizeof(uint32_t) * N));
  }
  e = (hipError_t)(e | up(d.chunk_bed32, hchunk.data(), sizeof(int32_t) * (N / PAD)));
  e = (hipError_t)(e | up(d.beds, hbc.data(), sizeof(BedConst) * nb));
  e = (hipError_t)(e | up(d.levels, levels.data(), sizeof(LevelGrid) * levels.size()));
  e = (hipError_t)(e | up(d.wdefs, hwd.data(), sizeof(WallDef) * hwd.size()));
  e = (hipError_t)(e | up(d.bdefs, hbd.data(), sizeof(BodyDef) * body_total));
  e = (hipError_t)(e | up(d.bdyn, hbdyn.data(), sizeof(BodyDyn) * body_total));
  e = (hipError_t)(e | up(d.bedyn, hbedyn.data(), sizeof(BedDyn) * nb));
  for (int q = 0; q < 2; ++q) {
    e = (hipError_t)(e | hipMemsetAsync(d.own_cnt[q], 0, sizeof(int32_t) * N, st));
    e = (hipError_t)(e | hipMemsetAsync(d.cflag[q], 0, sizeof(uint32_t) * N, st));
    e = (hipError_t)(e | hipMemsetAsync(d.hist[q], 0, sizeof(HRec) * K * N, st));
  }
  e = (hipError_t)(e | hipMemsetAsync(d.err, 0, sizeof(uint32_t), st));
  e = (hipError_t)(e | hipMemsetAsync(d.stat, 0, sizeof(uint32_t) * 4, st));
  e = (hipError_t)(e | hipMemsetAsync(d.disp, 0, sizeof(float) * N, st));
  e = (hipError_t)(e | hipMemsetAsync(d.cpf + N, 0, sizeof(float4) * CPF_PAD, st));
  e = (hipError_t)(e | hipMemsetAsync(d.viol, 0, sizeof(uint32_t) * 2, st));
  e = (hipError_t)(e | hipMemsetAsync(d.zext, 0, sizeof(uint32_t) * 2 * levels.size(), st));
  e = (hipError_t)(e | hipMemsetAsync(d.partial, 0, sizeof(double) * d.nblk * 6 * std::max(1, body_total), st));
  e = (hipError_t)(e | hipMemsetAsync(d.adv_cnt, 0, sizeof(uint32_t) * nb, st));
  if (b->record) {
    e = (hipError_t)(e | hipMemsetAsync(d.frc, 0, sizeof(float4) * N, st));
    e = (hipError_t)(e | hipMemsetAsync(d.trq, 0, sizeof(float4) * N, st));
  }
  launch_poses(d, st);
  if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
    b->release_all();
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return fail(LPR_E_DEVICE, "upload failed");
  }
  *out = b;
  return LPR_OK;
}

}  // namespace

extern "C" {

const char* lpr_status_str(lpr_status s) {
  switch (s) {
    case LPR_OK: return "ok";
    case LPR_E_INVAL: return "invalid argument";
    case LPR_E_NOMEM: return "out of memory";
    case LPR_E_DEVICE: return "device error";
    case LPR_E_CAPACITY: return "capacity exceeded";
    case LPR_E_STATE: return "invalid state";
    case LPR_E_NUMERIC: return "non-finite value";
    case LPR_E_DOMAIN: return "particle through a wall";
  }
  return "unknown status";
}

const char* lpr_last_error(void) { return g_last_error.c_str(); }

lpr_status lpr_bed_create(const lpr_bed_desc* desc, const lpr_allocator* alloc, void* hip_stream, lpr_bed** out) {
  const lpr_bed_desc* one[1] = {desc};
  return create_impl(one, 1, alloc, hip_stream, out);
}

lpr_status lpr_bed_destroy(lpr_bed* b) {
  if (!b) return LPR_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->release_all();
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LPR_OK;
}

lpr_status lpr_step(lpr_bed* b, int64_t n_steps) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (n_steps < 0) return fail(LPR_E_INVAL, "n_steps must be >= 0");
  b->R_eff = b->R;
  while (n_steps > 0) {
    const bool at_cycle = (b->since >= b->R) && (b->sort_every <= 0 || b->sc == 0);
    if (at_cycle && n_steps >= cycle_steps(b)) {
      if (!b->has_graph) {
        lpr_status st = capture_cycle(b);
        if (st != LPR_OK) return st;
      }
      if (b->s == b->gs && b->h == b->gh && b->l == b->gl && b->o == b->go) {
        HIPTRY(hipGraphLaunch(b->gexec, b->stream));
        // a cycle has an even number of steps and of rebuilds and two
        // re-sorts (or none): every parity is back where it started
        Par p = cur_par(b);
        const int S = b->sort_every > 0 ? b->sort_every : 0;
        for (int q = 0; q < b->gsteps; ++q) {
          simulate_step(p, b->R, S);
          b->plog.push_back(p);
        }
        b->since = b->R;
        b->host_steps += b->gsteps;
        b->rebuilds += b->gsteps / b->R;
        if (S > 0) b->sorts += 2;
        n_steps -= b->gsteps;
        continue;
      }
    }
    enqueue_step(b);
    n_steps -= 1;
  }
  HIPTRY(hipGetLastError());
  return LPR_OK;
}

lpr_status lpr_step_profiled(lpr_bed* b, int64_t n_steps, double out[4]) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (n_steps < 0 || !out) return fail(LPR_E_INVAL, "bad arguments");
  for (int c = 0; c < 4; ++c) out[c] = 0.0;
  if (n_steps == 0) return LPR_OK;
  std::vector<hipEvent_t> ev((size_t)n_steps * 4);
  for (auto& e : ev) HIPTRY(hipEventCreate(&e));
  for (int64_t q = 0; q < n_steps; ++q) {
    HIPTRY(hipEventRecord(ev[4 * q + 0], b->stream));
    if (b->since >= b->R_eff) enqueue_rebuild(b);
    HIPTRY(hipEventRecord(ev[4 * q + 1], b->stream));
    const int pb = enqueue_contact_step(b, b->stream);
    HIPTRY(hipEventRecord(ev[4 * q + 2], b->stream));
    launch_advance(b->d, pb, b->stream);
    HIPTRY(hipEventRecord(ev[4 * q + 3], b->stream));
    b->s ^= 1;
    b->h ^= 1;
    b->since += 1;
    b->host_steps += 1;
    b->plog.push_back(cur_par(b));
  }
  HIPTRY(hipGetLastError());
  HIPTRY(hipStreamSynchronize(b->stream));
  for (int64_t q = 0; q < n_steps; ++q) {
    float ms[3];
    for (int c = 0; c < 3; ++c) HIPTRY(hipEventElapsedTime(&ms[c], ev[4 * q + c], ev[4 * q + c + 1]));
    for (int c = 0; c < 3; ++c) out[c] += ms[c];
  }
  float tot = 0.f;
  HIPTRY(hipEventElapsedTime(&tot, ev[0], ev[4 * (n_steps - 1) + 3]));
  out[3] = tot;
  for (auto& e : ev) (void)hipEventDestroy(e);
  return sync_check(b);
}

lpr_status lpr_step_phases(lpr_bed* b, int64_t n_steps, double out[8]) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (n_steps < 0 || !out) return fail(LPR_E_INVAL, "bad arguments");
  for (int c = 0; c < 8; ++c) out[c] = 0.0;
  if (n_steps == 0) return LPR_OK;
  std::vector<hipEvent_t> ev((size_t)n_steps * 8);
  for (auto& e : ev) HIPTRY(hipEventCreate(&e));
  for (int64_t q = 0; q < n_steps; ++q) {
    b->pev = &ev[8 * q];
    mark(b, 0);
    if (b->since >= b->R_eff) {
      enqueue_rebuild(b);
    } else {
      for (int k = 1; k <= 5; ++k) mark(b, k);
    }
    const int pb = enqueue_contact_step(b, b->stream);
    mark(b, 6);
    launch_advance(b->d, pb, b->stream);
    mark(b, 7);
    b->pev = nullptr;
    b->s ^= 1;
    b->h ^= 1;
    b->since += 1;
    b->host_steps += 1;
    b->plog.push_back(cur_par(b));
  }
  HIPTRY(hipGetLastError());
  HIPTRY(hipStreamSynchronize(b->stream));
  for (int64_t q = 0; q < n_steps; ++q)
    for (int c = 0; c < 7; ++c) {
      float ms = 0.f;
      HIPTRY(hipEventElapsedTime(&ms, ev[8 * q + c], ev[8 * q + c + 1]));
      out[c] += ms;
    }
  float tot = 0.f;
  HIPTRY(hipEventElapsedTime(&tot, ev[0], ev[8 * (n_steps - 1) + 7]));
  out[7] = tot;
  for (auto& e : ev) (void)hipEventDestroy(e);
  return sync_check(b);
}

lpr_status lpr_sync(lpr_bed* b) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  if (b->faulted) return fail(b->fault_status, "latched device fault");
  return sync_check(b);
}

static lpr_status get_state_impl(lpr_bed* b, int32_t bed, double* pos, float* vel, float* omega) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  int par = 0;
  lpr_status st = state_parity(b, &par);
  if (st != LPR_OK) return st;
  const HostBed& H = b->hb[bed];
  std::vector<PState> hs(H.npad);
  std::vector<int32_t> sid(H.npad);
  HIPTRY(hipMemcpy(hs.data(), b->d.st[par] + H.p0, sizeof(PState) * H.npad, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid + H.p0, sizeof(int32_t) * H.npad, hipMemcpyDeviceToHost));
  for (int64_t off = 0; off < H.npad; ++off) {
    if (sid[off] < 0) continue;
    const int64_t q = sid[off];
    const PState& p = hs[off];
    if (pos) { pos[3 * q] = p.x.x; pos[3 * q + 1] = p.x.y; pos[3 * q + 2] = p.x.z; }
    if (vel) { vel[3 * q] = p.v.x; vel[3 * q + 1] = p.v.y; vel[3 * q + 2] = p.v.z; }
    if (omega) { omega[3 * q] = p.w.x; omega[3 * q + 1] = p.w.y; omega[3 * q + 2] = p.w.z; }
  }
  return LPR_OK;
}

static lpr_status set_state_impl(lpr_bed* b, int32_t bed, const double* pos, const float* vel, const float* omega) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  const HostBed& H = b->hb[bed];
  if (pos && !finite_arr(pos, 3 * H.n)) return fail(LPR_E_INVAL, "non-finite position");
  if (vel && !finite_arrf(vel, 3 * H.n)) return fail(LPR_E_INVAL, "non-finite velocity");
  if (omega && !finite_arrf(omega, 3 * H.n)) return fail(LPR_E_INVAL, "non-finite angular velocity");
  int par = 0;
  lpr_status st = state_parity(b, &par);
  if (st != LPR_OK) return st;
  std::vector<PState> hs(H.npad);
  std::vector<int32_t> sid(H.npad);
  HIPTRY(hipMemcpy(hs.data(), b->d.st[par] + H.p0, sizeof(PState) * H.npad, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid + H.p0, sizeof(int32_t) * H.npad, hipMemcpyDeviceToHost));
  for (int64_t off = 0; off < H.npad; ++off) {
    if (sid[off] < 0) continue;
    const int64_t q = sid[off];
    PState& p = hs[off];
    if (pos) { p.x.x = pos[3 * q]; p.x.y = pos[3 * q + 1]; p.x.z = pos[3 * q + 2]; }
    if (vel) { p.v.x = vel[3 * q]; p.v.y = vel[3 * q + 1]; p.v.z = vel[3 * q + 2]; }
    if (omega) { p.w.x = omega[3 * q]; p.w.y = omega[3 * q + 1]; p.w.z = omega[3 * q + 2]; }
  }
  HIPTRY(hipMemcpy(b->d.st[par] + H.p0, hs.data(), sizeof(PState) * H.npad, hipMemcpyHostToDevice));
  b->since = std::numeric_limits<int64_t>::max() / 2;  // positions moved: rebuild before the next step
  return LPR_OK;
}

static lpr_status get_history_impl(lpr_bed* b, int32_t bed, lpr_history* out, int64_t capacity, int64_t* n_total) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  const HostBed& H = b->hb[bed];
  const int64_t N = b->d.N;
  std::vector<int32_t> cnt(N), idx((size_t)K * N), sid(N);
  std::vector<uint32_t> fl(N);
  std::vector<HRec> a((size_t)K * N);
  std::vector<float4> wa((size_t)b->max_walls * N);
  std::vector<float2> wc((size_t)b->max_walls * N);
  HIPTRY(hipMemcpy(cnt.data(), b->d.own_cnt[b->l], sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(idx.data(), b->d.own_idx[b->l], sizeof(int32_t) * K * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(fl.data(), b->d.cflag[b->h], sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(a.data(), b->d.hist[b->h], sizeof(HRec) * K * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(wa.data(), b->d.wA[b->h], sizeof(float4) * b->max_walls * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(wc.data(), b->d.wB[b->h], sizeof(float2) * b->max_walls * N, hipMemcpyDeviceToHost));
  std::vector<lpr_history> recs;
  for (int64_t i = H.p0; i < H.p0 + H.npad; ++i) {
    if (sid[i] < 0) continue;
    for (int k = 0; k < cnt[i]; ++k)
      if ((fl[i] >> k) & 1u) {
        const HRec& A = a[(size_t)k * N + i];
        recs.push_back({sid[i], sid[idx[(size_t)k * N + i]], {A.t.x, A.t.y, A.t.z}, {A.r.x, A.r.y, A.r.z}});
      }
    for (int w = 0; w < H.nwall; ++w)
      if ((fl[i] >> (WALL_BIT + w)) & 1u) {
        const float4 A = wa[(size_t)w * N + i];
        const float2 C = wc[(size_t)w * N + i];
        recs.push_back({sid[i], -1 - (int64_t)w, {A.x, A.y, A.z}, {A.w, C.x, C.y}});
      }
  }
  std::sort(recs.begin(), recs.end(), [](const lpr_history& x, const lpr_history& y) {
    return x.owner < y.owner || (x.owner == y.owner && x.partner < y.partner);
  });
  if (n_total) *n_total = (int64_t)recs.size();
  if ((int64_t)recs.size() > capacity) return fail(LPR_E_CAPACITY, "history buffer too small");
  if (!recs.empty()) std::memcpy(out, recs.data(), sizeof(lpr_history) * recs.size());
  return LPR_OK;
}

static lpr_status set_history_impl(lpr_bed* b, int32_t bed, const lpr_history* rec, int64_t count) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (count < 0 || (count > 0 && !rec)) return fail(LPR_E_INVAL, "bad history records");
  ensure_lists(b);
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  const HostBed& H = b->hb[bed];
  const int64_t N = b->d.N;
  std::vector<int32_t> cnt(N), idx((size_t)K * N), sid(N);
  HIPTRY(hipMemcpy(cnt.data(), b->d.own_cnt[b->l], sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(idx.data(), b->d.own_idx[b->l], sizeof(int32_t) * K * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  std::vector<std::vector<const lpr_history*>> by_owner(H.n);
  for (int64_t q = 0; q < count; ++q) {
    if (rec[q].owner < 0 || rec[q].owner >= H.n) return fail(LPR_E_INVAL, "history owner out of range");
    by_owner[rec[q].owner].push_back(&rec[q]);
  }
  // the other beds of a batch keep their records: start from the device
  // arrays and clear this bed's range
  const int W = b->max_walls;
  std::vector<uint32_t> fl(N);
  std::vector<HRec> a((size_t)K * N);
  std::vector<float4> wa((size_t)W * N);
  std::vector<float2> wc((size_t)W * N);
  HIPTRY(hipMemcpy(fl.data(), b->d.cflag[b->h], sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(a.data(), b->d.hist[b->h], sizeof(HRec) * K * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(wa.data(), b->d.wA[b->h], sizeof(float4) * W * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(wc.data(), b->d.wB[b->h], sizeof(float2) * W * N, hipMemcpyDeviceToHost));
  for (int64_t i = H.p0; i < H.p0 + H.npad; ++i) {
    fl[i] = 0u;
    for (int k = 0; k < K; ++k) {
      a[(size_t)k * N + i].t = make_float4(0, 0, 0, 0);
      a[(size_t)k * N + i].r = make_float4(0, 0, 0, 0);
    }
    for (int w = 0; w < W; ++w) {
      wa[(size_t)w * N + i] = make_float4(0, 0, 0, 0);
      wc[(size_t)w * N + i] = make_float2(0, 0);
    }
  }
  for (int64_t i = H.p0; i < H.p0 + H.npad; ++i) {
    if (sid[i] < 0) continue;
    for (const lpr_history* r : by_owner[sid[i]]) {
      if (r->partner >= 0) {
        for (int k = 0; k < cnt[i]; ++k)
          if (sid[idx[(size_t)k * N + i]] == r->partner) {
            a[(size_t)k * N + i].t = make_float4(r->xi_t[0], r->xi_t[1], r->xi_t[2], 0.f);
            a[(size_t)k * N + i].r = make_float4(r->xi_r[0], r->xi_r[1], r->xi_r[2], 0.f);
            fl[i] |= 1u << k;
          }
      } else {
        const int64_t w = -1 - r->partner;
        if (w < H.nwall) {
          wa[(size_t)w * N + i] = make_float4(r->xi_t[0], r->xi_t[1], r->xi_t[2], r->xi_r[0]);
          wc[(size_t)w * N + i] = make_float2(r->xi_r[1], r->xi_r[2]);
          fl[i] |= 1u << (WALL_BIT + w);
        }
      }
    }
  }
  HIPTRY(hipMemcpy(b->d.cflag[b->h], fl.data(), sizeof(uint32_t) * N, hipMemcpyHostToDevice));
  HIPTRY(hipMemcpy(b->d.hist[b->h], a.data(), sizeof(HRec) * K * N, hipMemcpyHostToDevice));
  HIPTRY(hipMemcpy(b->d.wA[b->h], wa.data(), sizeof(float4) * W * N, hipMemcpyHostToDevice));
  HIPTRY(hipMemcpy(b->d.wB[b->h], wc.data(), sizeof(float2) * W * N, hipMemcpyHostToDevice));
  return LPR_OK;
}

static lpr_status read_contacts_impl(lpr_bed* b, int32_t bed, lpr_contact* out, int64_t capacity, int64_t* n_total) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  const HostBed& H = b->hb[bed];
  const int64_t N = b->d.N;
  std::vector<int32_t> cnt(N), idx((size_t)K * N), sid(N);
  std::vector<uint32_t> fl(N);
  HIPTRY(hipMemcpy(cnt.data(), b->d.own_cnt[b->l], sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(idx.data(), b->d.own_idx[b->l], sizeof(int32_t) * K * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(fl.data(), b->d.cflag[b->h], sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
  std::vector<lpr_contact> cs;
  if (b->host_steps > 0) {
    for (int64_t i = H.p0; i < H.p0 + H.npad; ++i) {
      if (sid[i] < 0) continue;
      for (int k = 0; k < cnt[i]; ++k)
        if ((fl[i] >> k) & 1u) {
          const int64_t x = sid[i], y = sid[idx[(size_t)k * N + i]];
          cs.push_back({std::min(x, y), std::max(x, y)});
        }
      for (int w = 0; w < H.nwall; ++w)
        if ((fl[i] >> (WALL_BIT + w)) & 1u) cs.push_back({(int64_t)sid[i], -1 - (int64_t)w});
    }
  }
  std::sort(cs.begin(), cs.end(),
            [](const lpr_contact& x, const lpr_contact& y) { return x.a < y.a || (x.a == y.a && x.b < y.b); });
  if (n_total) *n_total = (int64_t)cs.size();
  if ((int64_t)cs.size() > capacity) return fail(LPR_E_CAPACITY, "contact buffer too small");
  if (!cs.empty()) std::memcpy(out, cs.data(), sizeof(lpr_contact) * cs.size());
  return LPR_OK;
}

static lpr_status read_forces_impl(lpr_bed* b, int32_t bed, float* force, float* torque) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  if (!b->record) return fail(LPR_E_STATE, "bed was created without record_forces");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  const HostBed& H = b->hb[bed];
  std::vector<float4> f(H.npad), t(H.npad);
  std::vector<int32_t> sid(H.npad);
  HIPTRY(hipMemcpy(f.data(), b->d.frc + H.p0, sizeof(float4) * H.npad, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(t.data(), b->d.trq + H.p0, sizeof(float4) * H.npad, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(sid.data(), b->d.sid + H.p0, sizeof(int32_t) * H.npad, hipMemcpyDeviceToHost));
  for (int64_t off = 0; off < H.npad; ++off) {
    if (sid[off] < 0) continue;
    const int64_t q = sid[off];
    if (force) { force[3 * q] = f[off].x; force[3 * q + 1] = f[off].y; force[3 * q + 2] = f[off].z; }
    if (torque) { torque[3 * q] = t[off].x; torque[3 * q + 1] = t[off].y; torque[3 * q + 2] = t[off].z; }
  }
  return LPR_OK;
}

// Per-contact loads are compacted on the device into a workspace: per
// particle its contact count, their exclusive scan (and the scan's tile
// sums), then the records; the records are copied to the caller's buffer and
// put in canonical order there.
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t load_head_bytes(int64_t np) {
  return al256(4 * (size_t)np) + al256(4 * ((size_t)np + 1)) + al256(4 * scan_tmp_elems(np));
}

// Counts and scans the last step's contacts of bed `bed` into ws; *total
// gets their number.
static lpr_status load_count(lpr_bed* b, int32_t bed, char* ws, int64_t* total) {
  const HostBed& H = b->hb[bed];
  const int64_t np = H.npad;
  uint32_t* cnt = (uint32_t*)ws;
  uint32_t* off = (uint32_t*)(ws + al256(4 * (size_t)np));
  uint32_t* tmp = (uint32_t*)(ws + al256(4 * (size_t)np) + al256(4 * ((size_t)np + 1)));
  launch_load_count(b->d, b->l, b->h, H.p0, np, H.nwall, cnt, b->stream);
  launch_scan(cnt, off, tmp, np, b->stream);
  uint32_t tot = 0;
  HIPTRY(hipMemcpyAsync(&tot, off + np, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream));
  HIPTRY(hipStreamSynchronize(b->stream));
  HIPTRY(hipGetLastError());
  *total = (b->host_steps > 0) ? (int64_t)tot : 0;
  return LPR_OK;
}

// Writes the counted records to rec (device, after the head of ws), copies
// them to out and sorts them there by (a, b).
static lpr_status load_pack(lpr_bed* b, int32_t bed, char* ws, lpr_contact_load* rec, int64_t total,
                     lpr_contact_load* out) {
  if (total == 0) return LPR_OK;
  const HostBed& H = b->hb[bed];
  const int64_t np = H.npad;
  const uint32_t* off = (const uint32_t*)(ws + al256(4 * (size_t)np));
  launch_load_pack(b->d, b->l, b->h, H.p0, np, H.nwall, off, rec, b->stream);
  HIPTRY(hipMemcpyAsync(out, rec, sizeof(lpr_contact_load) * (size_t)total, hipMemcpyDeviceToHost, b->stream));
  HIPTRY(hipStreamSynchronize(b->stream));
  HIPTRY(hipGetLastError());
  std::sort(out, out + total, [](const lpr_contact_load& x, const lpr_contact_load& y) {
    return x.a < y.a || (x.a == y.a && x.b < y.b);
  });
  return LPR_OK;
}

static lpr_status loads_readable(lpr_bed* b) {
  if (!b->record) return fail(LPR_E_STATE, "bed was created without record_forces");
  if (b->stepper != LPR_STEPPER_EXPLICIT) return fail(LPR_E_STATE, "per-contact loads are kept by the explicit step");
  return LPR_OK;
}

static lpr_status read_contact_loads_impl(lpr_bed* b, int32_t bed, lpr_contact_load* out, int64_t capacity,
                                          int64_t* n_total) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  lpr_status st = loads_readable(b);
  if (st != LPR_OK) return st;
  if ((st = sync_check(b)) != LPR_OK) return st;
  const int64_t np = b->hb[bed].npad;
  const size_t head = load_head_bytes(np);
  auto ensure = [&](size_t need) -> bool {
    if (b->ld_ws_bytes >= need) return true;
    b->dfree(b->ld_ws);
    b->ld_ws = (char*)b->dalloc(need);
    b->ld_ws_bytes = b->ld_ws ? need : 0;
    return b->ld_ws != nullptr;
  };
  if (!ensure(head)) return fail(LPR_E_NOMEM, "per-contact read workspace");
  int64_t total = 0;
  if ((st = load_count(b, bed, b->ld_ws, &total)) != LPR_OK) return st;
  if (n_total) *n_total = total;
  if (total > capacity) return fail(LPR_E_CAPACITY, "contact buffer too small");
  if (total == 0) return LPR_OK;
  const size_t need = head + sizeof(lpr_contact_load) * (size_t)total;
  if (b->ld_ws_bytes < need) {
    // the counts and their scan live at the head of the workspace: recount
    // in the larger one
    if (!ensure(need)) return fail(LPR_E_NOMEM, "per-contact read workspace");
    if ((st = load_count(b, bed, b->ld_ws, &total)) != LPR_OK) return st;
  }
  return load_pack(b, bed, b->ld_ws, (lpr_contact_load*)(b->ld_ws + head), total, out);
}

static lpr_status read_wall_pose_impl(lpr_bed* b, int32_t bed, int32_t wall, double out15[15]) {
  if (!b || !out15) return fail(LPR_E_INVAL, "null argument");
  const HostBed& H = b->hb[bed];
  if (wall < 0 || wall >= H.nwall) return fail(LPR_E_INVAL, "wall out of range");
  HIPTRY(hipStreamSynchronize(b->stream));
  WallPose P;
  HIPTRY(hipMemcpy(&P, b->d.walls + H.wall0 + wall, sizeof(WallPose), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a) {
    out15[a] = P.o[a];
    out15[3 + a] = P.nu[a];
    for (int c = 0; c < 3; ++c) out15[6 + 3 * c + a] = P.e[c][a];
  }
  return LPR_OK;
}

static lpr_status read_reaction_impl(lpr_bed* b, int32_t bed, int32_t body, double out6[6]) {
  if (!b || !out6) return fail(LPR_E_INVAL, "null argument");
  const HostBed& H = b->hb[bed];
  if (body < 0 || body >= H.nbody) return fail(LPR_E_INVAL, "body out of range");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  BodyDyn D;
  HIPTRY(hipMemcpy(&D, b->d.bdyn + H.body0 + body, sizeof(BodyDyn), hipMemcpyDeviceToHost));
  for (int c = 0; c < 6; ++c) out6[c] = D.last[c];
  return LPR_OK;
}

static lpr_status reaction_window_impl(lpr_bed* b, int32_t bed, int32_t body, double sum6[6], int64_t* steps, int32_t reset) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  const HostBed& H = b->hb[bed];
  if (body < 0 || body >= H.nbody) return fail(LPR_E_INVAL, "body out of range");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  BodyDyn D;
  HIPTRY(hipMemcpy(&D, b->d.bdyn + H.body0 + body, sizeof(BodyDyn), hipMemcpyDeviceToHost));
  if (sum6)
    for (int c = 0; c < 6; ++c) sum6[c] = D.wsum[c];
  if (steps) *steps = D.wsteps;
  if (reset) {
    for (int c = 0; c < 6; ++c) D.wsum[c] = 0.0;
    D.wsteps = 0;
    HIPTRY(hipMemcpy(b->d.bdyn + H.body0 + body, &D, sizeof(BodyDyn), hipMemcpyHostToDevice));
  }
  return LPR_OK;
}

static lpr_status read_body_impl(lpr_bed* b, int32_t bed, int32_t body, double origin[3], double vel[3]) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  const HostBed& H = b->hb[bed];
  if (body < 0 || body >= H.nbody) return fail(LPR_E_INVAL, "body out of range");
  HIPTRY(hipStreamSynchronize(b->stream));
  BodyDyn D;
  BodyDef B;
  BedDyn E;
  HIPTRY(hipMemcpy(&D, b->d.bdyn + H.body0 + body, sizeof(BodyDyn), hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(&B, b->d.bdefs + H.body0 + body, sizeof(BodyDef), hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(&E, b->d.bedyn + bed, sizeof(BedDyn), hipMemcpyDeviceToHost));
  const double t = (double)E.k * H.dt;
  for (int a = 0; a < 3; ++a) {
    if (origin) origin[a] = B.origin[a] + B.lin_vel[a] * t;
    if (vel) vel[a] = B.lin_vel[a];
  }
  if (B.z_free) {
    if (origin) origin[2] = D.z;
    if (vel) vel[2] = D.vz;
  }
  return LPR_OK;
}

static lpr_status set_clock_impl(lpr_bed* b, int32_t bed, int64_t step) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (step < 0) return fail(LPR_E_INVAL, "step must be >= 0");
  HIPTRY(hipStreamSynchronize(b->stream));
  BedDyn E;
  HIPTRY(hipMemcpy(&E, b->d.bedyn + bed, sizeof(BedDyn), hipMemcpyDeviceToHost));
  E.k = step;
  HIPTRY(hipMemcpy(b->d.bedyn + bed, &E, sizeof(BedDyn), hipMemcpyHostToDevice));
  launch_poses(b->d, b->stream);
  HIPTRY(hipStreamSynchronize(b->stream));
  return LPR_OK;
}

static lpr_status get_clock_impl(lpr_bed* b, int32_t bed, int64_t* step) {
  if (!b || !step) return fail(LPR_E_INVAL, "null argument");
  HIPTRY(hipStreamSynchronize(b->stream));
  BedDyn E;
  HIPTRY(hipMemcpy(&E, b->d.bedyn + bed, sizeof(BedDyn), hipMemcpyDeviceToHost));
  *step = E.k;
  return LPR_OK;
}

static lpr_status set_body_state_impl(lpr_bed* b, int32_t bed, int32_t body, double z, double vz) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  const HostBed& H = b->hb[bed];
  if (body < 0 || body >= H.nbody) return fail(LPR_E_INVAL, "body out of range");
  HIPTRY(hipStreamSynchronize(b->stream));
  BodyDyn D;
  HIPTRY(hipMemcpy(&D, b->d.bdyn + H.body0 + body, sizeof(BodyDyn), hipMemcpyDeviceToHost));
  D.z = z;
  D.vz = vz;
  HIPTRY(hipMemcpy(b->d.bdyn + H.body0 + body, &D, sizeof(BodyDyn), hipMemcpyHostToDevice));
  launch_poses(b->d, b->stream);
  HIPTRY(hipStreamSynchronize(b->stream));
  return LPR_OK;
}

lpr_status lpr_get_stats(lpr_bed* b, lpr_stats* out) {
  if (!b || !out) return fail(LPR_E_INVAL, "null argument");
  HIPTRY(hipStreamSynchronize(b->stream));
  BedDyn E;
  uint32_t stat[4];
  HIPTRY(hipMemcpy(&E, b->d.bedyn, sizeof(BedDyn), hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(stat, b->d.stat, sizeof(stat), hipMemcpyDeviceToHost));
  const int64_t N = b->d.N;
  std::vector<int32_t> cnt(N);
  std::vector<uint32_t> fl(N);
  HIPTRY(hipMemcpy(cnt.data(), b->d.own_cnt[b->l], sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(fl.data(), b->d.cflag[b->h], sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
  int64_t cand = 0, con = 0;
  for (int64_t i = 0; i < N; ++i) {
    cand += cnt[i];
    con += __builtin_popcount(fl[i]);
  }
  out->steps = E.completed;
  out->contacts = b->host_steps > 0 ? con : 0;
  out->candidates = cand;
  out->rebuilds = b->rebuilds;
  out->levels = b->nlev_total;
  out->cells = b->ncells;
  out->max_owner_slots = (int32_t)stat[0];
  out->skin_trips = b->skin_trips;
  out->adjoint_interval = b->adj_interval;
  out->sorts = b->sorts;
  out->outside_grid = stat[2];
  return LPR_OK;
}


lpr_status lpr_batch_create(const lpr_bed_desc* const* descs, int32_t n_beds, const lpr_allocator* alloc,
                            void* hip_stream, lpr_bed** out) {
  if (n_beds <= 0 || n_beds > (1 << 20)) {
    if (out) *out = nullptr;
    return fail(LPR_E_INVAL, "n_beds out of range");
  }
  for (int q = 1; q < n_beds; ++q)
    if (!descs || !descs[q] || !descs[0] || descs[q]->rebuild_every != descs[0]->rebuild_every ||
        descs[q]->skin != descs[0]->skin || descs[q]->block != descs[0]->block ||
        descs[q]->record_forces != descs[0]->record_forces || descs[q]->persistent != descs[0]->persistent ||
        descs[q]->sort_every != descs[0]->sort_every || descs[q]->input_order != descs[0]->input_order)
      return fail(LPR_E_INVAL, "beds of a batch share rebuild_every, skin, block, persistent, record_forces, "
                               "sort_every, input_order");
  return create_impl(descs, n_beds, alloc, hip_stream, out);
}

lpr_status lpr_batch_size(lpr_bed* b, int32_t* n_beds) {
  if (!b || !n_beds) return fail(LPR_E_INVAL, "null argument");
  *n_beds = (int32_t)b->hb.size();
  return LPR_OK;
}

lpr_status lpr_set_launch(lpr_bed* b, int32_t block, int32_t persistent) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (block != 64 && block != 128 && block != 256) return fail(LPR_E_INVAL, "block must be 64, 128 or 256");
  HIPTRY(hipStreamSynchronize(b->stream));
  b->block = block;
  b->persist_blocks = 0;
  if (persistent) {
    int dev = 0, cus = 0;
    HIPTRY(hipGetDevice(&dev));
    HIPTRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->persist_blocks = std::max(8, step_occupancy(block) * cus);
  }
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->has_graph = false;
  return LPR_OK;
}

namespace {

lpr_status time_trial(lpr_bed* b, int32_t steps, double* ms_per_step) {
  lpr_status st = lpr_step(b, 2);  // first rebuild and graph capture outside the timing
  if (st == LPR_OK) st = lpr_sync(b);
  double out[4];
  if (st == LPR_OK) st = lpr_step_profiled(b, steps, out);
  if (st == LPR_OK) *ms_per_step = out[3] / steps;
  return st;
}

}  // namespace

// The per-band cell factor of level q in the descriptions being tuned (the
// first bed's; the caller's choice, usually 0).
static float given_level_factor(const std::vector<lpr_bed_desc>& work, int q) {
  return work.empty() ? 0.f : work[0].level_cell_factor[q];
}

lpr_status lpr_autotune(const lpr_bed_desc* const* descs, int32_t n_beds, const lpr_allocator* alloc,
                        void* hip_stream, int32_t trial_steps, lpr_tuning* best, lpr_tuning* trials,
                        int32_t capacity, int32_t* n_trials) {
  if (!descs || n_beds <= 0 || !best || trial_steps <= 0) return fail(LPR_E_INVAL, "bad arguments");
  std::vector<lpr_bed_desc> work(descs[0] ? (size_t)n_beds : 0);
  for (int q = 0; q < n_beds; ++q) {
    if (!descs[q]) return fail(LPR_E_INVAL, "null description");
    work[q] = *descs[q];
  }
  std::vector<const lpr_bed_desc*> ptrs(n_beds);
  for (int q = 0; q < n_beds; ++q) ptrs[q] = &work[q];
  std::vector<lpr_tuning> done;
  // layout: radius-band ratio and cell factor (one batch each)
  const float bands[3] = {1.5f, 2.0f, 3.0f};
  const float cells[2] = {1.0f, 1.25f};
  lpr_tuning bestt{};
  bestt.ms_per_step = std::numeric_limits<double>::max();
  for (float br : bands)
    for (float cf : cells) {
      for (auto& w : work) {
        w.band_ratio = br;
        w.cell_factor = cf;
        w.block = 64;
        w.persistent = 0;
        w.record_forces = 0;
      }
      lpr_bed* b = nullptr;
      lpr_status st = create_impl(ptrs.data(), n_beds, alloc, hip_stream, &b);
      if (st != LPR_OK) return st;
      double ms = 0.0;
      st = time_trial(b, trial_steps, &ms);
      lpr_bed_destroy(b);
      if (st != LPR_OK) return st;
      lpr_tuning t{br, cf, 256, 0, ms, {}};
      for (int q = 0; q < MAXLEV; ++q) t.level_cell_factor[q] = given_level_factor(work, q);
      done.push_back(t);
      if (ms < bestt.ms_per_step) bestt = t;
    }
  // launch shape on the chosen layout
  for (auto& w : work) {
    w.band_ratio = bestt.band_ratio;
    w.cell_factor = bestt.cell_factor;
  }
  lpr_bed* b = nullptr;
  lpr_status st = create_impl(ptrs.data(), n_beds, alloc, hip_stream, &b);
  if (st != LPR_OK) return st;
  const int blocks[3] = {64, 128, 256};
  for (int bl : blocks)
    for (int pe = 0; pe < 2; ++pe) {
      if (bl == 256 && pe == 0) continue;  // measured in the layout phase
      st = lpr_set_launch(b, bl, pe);
      double ms = 0.0;
      if (st == LPR_OK) st = time_trial(b, trial_steps, &ms);
      if (st != LPR_OK) {
        lpr_bed_destroy(b);
        return st;
      }
      lpr_tuning t = bestt;
      t.block = bl;
      t.persistent = pe;
      t.ms_per_step = ms;
      done.push_back(t);
      if (ms < bestt.ms_per_step) bestt = t;
    }
  int nlev = 1;
  for (const HostBed& H : b->hb) nlev = std::max(nlev, H.nlev);
  lpr_bed_destroy(b);
  // radius band by radius band: a larger cell factor for that band alone
  for (auto& w : work) {
    w.block = bestt.block;
    w.persistent = bestt.persistent;
  }
  const float band_cells[2] = {1.25f, 1.5f};
  for (int q = 0; q < nlev; ++q)
    for (float cf : band_cells) {
      for (auto& w : work)
        for (int q2 = 0; q2 < MAXLEV; ++q2) w.level_cell_factor[q2] = bestt.level_cell_factor[q2];
      for (auto& w : work) w.level_cell_factor[q] = cf;
      lpr_bed* bq = nullptr;
      st = create_impl(ptrs.data(), n_beds, alloc, hip_stream, &bq);
      if (st != LPR_OK) return st;
      double ms = 0.0;
      st = time_trial(bq, trial_steps, &ms);
      lpr_bed_destroy(bq);
      if (st != LPR_OK) return st;
      lpr_tuning t = bestt;
      t.level_cell_factor[q] = cf;
      t.ms_per_step = ms;
      done.push_back(t);
      if (ms < bestt.ms_per_step) bestt = t;
    }
  *best = bestt;
  if (n_trials) *n_trials = (int32_t)done.size();
  if (trials)
    for (int q = 0; q < (int)done.size() && q < capacity; ++q) trials[q] = done[q];
  return LPR_OK;
}

namespace {

bool adj_reserve(lpr_bed* b, int steps, int nckpt) {
  DevBufs& d = b->d;
  const int64_t N = d.N;
  const int W = b->max_walls;
  AdjBufs& a = b->adj;
  if (b->adj_steps < steps) {
    bool ok = dal(b, &a.st, (size_t)steps * N) && dal(b, &a.cflag, (size_t)steps * N) &&
              dal(b, &a.hist, (size_t)steps * K * N) &&
              dal(b, &a.wA, (size_t)steps * W * N) && dal(b, &a.wB, (size_t)steps * W * N);
    const int nw = std::max(1, (int)(b->hb.back().wall0 + b->hb.back().nwall));
    ok = ok && dal(b, &a.walls, (size_t)steps * nw);
    if (!ok) return false;
    a.nwall_total = nw;
    a.nwall_max = W;
    b->adj_steps = steps;
  }
  if (!a.xb) {
    bool ok = dal(b, &a.own_cnt, N) && dal(b, &a.own_idx, (size_t)K * N) && dal(b, &a.rev_start, N + 1) &&
              dal(b, &a.rev_ent, (size_t)K * N) && dal(b, &a.xb, N) && dal(b, &a.vb, N) && dal(b, &a.wb, N) &&
              dal(b, &a.Fb, N) && dal(b, &a.Tb, N) && dal(b, &a.theta, 3 * N) && dal(b, &b->theta_out, 3);
    for (int q = 0; q < 2; ++q)
      ok = ok && dal(b, &a.hbA[q], (size_t)K * N) && dal(b, &a.hbB[q], (size_t)K * N) &&
           dal(b, &a.wbA[q], (size_t)W * N) && dal(b, &a.wbB[q], (size_t)W * N);
    if (!ok) return false;
  }
  while ((int)b->ckpts.size() < nckpt) {
    lpr_bed::Ckpt c{};
    const size_t nb = std::max<size_t>(1, b->hb.back().body0 + b->hb.back().nbody);
    bool ok = dal(b, &c.st, N) && dal(b, &c.cflag, N) &&
              dal(b, &c.hist, (size_t)K * N) && dal(b, &c.wA, (size_t)W * N) &&
              dal(b, &c.wB, (size_t)W * N) && dal(b, &c.own_cnt, N) && dal(b, &c.own_idx, (size_t)K * N) &&
              dal(b, &c.bedyn, b->hb.size()) && dal(b, &c.bdyn, nb);
    if (!ok) return false;
    b->ckpts.push_back(c);
  }
  return true;
}

hipError_t d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
}

lpr_status ckpt_save(lpr_bed* b, lpr_bed::Ckpt& c) {
  DevBufs& d = b->d;
  const int64_t N = d.N;
  const int W = b->max_walls;
  const size_t nb = std::max<size_t>(1, b->hb.back().body0 + b->hb.back().nbody);
  hipStream_t st = b->stream;
  HIPTRY(d2d(c.st, d.st[b->s], sizeof(PState) * N, st));
  HIPTRY(d2d(c.cflag, d.cflag[b->h], sizeof(uint32_t) * N, st));
  HIPTRY(d2d(c.hist, d.hist[b->h], sizeof(HRec) * K * N, st));
  HIPTRY(d2d(c.wA, d.wA[b->h], sizeof(float4) * W * N, st));
  HIPTRY(d2d(c.wB, d.wB[b->h], sizeof(float2) * W * N, st));
  HIPTRY(d2d(c.own_cnt, d.own_cnt[b->l], sizeof(int32_t) * N, st));
  HIPTRY(d2d(c.own_idx, d.own_idx[b->l], sizeof(int32_t) * K * N, st));
  HIPTRY(d2d(c.bedyn, d.bedyn, sizeof(BedDyn) * b->hb.size(), st));
  HIPTRY(d2d(c.bdyn, d.bdyn, sizeof(BodyDyn) * nb, st));
  c.s = b->s; c.h = b->h; c.l = b->l;
  c.since = b->since; c.host_steps = b->host_steps; c.rebuilds = b->rebuilds;
  return LPR_OK;
}

lpr_status ckpt_restore(lpr_bed* b, const lpr_bed::Ckpt& c) {
  DevBufs& d = b->d;
  const int64_t N = d.N;
  const int W = b->max_walls;
  const size_t nb = std::max<size_t>(1, b->hb.back().body0 + b->hb.back().nbody);
  hipStream_t st = b->stream;
  b->s = c.s; b->h = c.h; b->l = c.l;
  b->since = c.since; b->host_steps = c.host_steps; b->rebuilds = c.rebuilds;
  HIPTRY(d2d(d.st[b->s], c.st, sizeof(PState) * N, st));
  HIPTRY(d2d(d.cflag[b->h], c.cflag, sizeof(uint32_t) * N, st));
  HIPTRY(d2d(d.hist[b->h], c.hist, sizeof(HRec) * K * N, st));
  HIPTRY(d2d(d.wA[b->h], c.wA, sizeof(float4) * W * N, st));
  HIPTRY(d2d(d.wB[b->h], c.wB, sizeof(float2) * W * N, st));
  HIPTRY(d2d(d.own_cnt[b->l], c.own_cnt, sizeof(int32_t) * N, st));
  HIPTRY(d2d(d.own_idx[b->l], c.own_idx, sizeof(int32_t) * K * N, st));
  HIPTRY(d2d(d.bedyn, c.bedyn, sizeof(BedDyn) * b->hb.size(), st));
  HIPTRY(d2d(d.bdyn, c.bdyn, sizeof(BodyDyn) * nb, st));
  launch_poses(d, st);
  return LPR_OK;
}

lpr_status set_device_skin(lpr_bed* b, float skin) {
  for (size_t q = 0; q < b->hb.size(); ++q)
    HIPTRY(hipMemcpy((char*)(b->d.beds + q) + offsetof(BedConst, skin), &skin, sizeof(float), hipMemcpyHostToDevice));
  return LPR_OK;
}

}  // namespace

static lpr_status upload_sp_consts(lpr_bed* b) {
  std::vector<SpConst> sc(b->hb.size());
  for (size_t q = 0; q < b->hb.size(); ++q) {
    const lpr_params& P = b->hb[q].params;
    const double Estar = 1.0 / ((1.0 - P.nu * P.nu) / P.E + (1.0 - P.nu * P.nu) / P.E);
    const double h = P.dt, tau = P.gamma_factor * P.dt;
    SpConst& c = sc[q];
    c.rho = P.rho;
    c.kfac = P.s_k * Estar / 3.0;
    c.eH = P.e_H;
    c.h = h;
    c.ups = 1.0 / (1.0 + 4.0 * tau / h);
    c.mu_t = P.mu_t;
    c.mu_r = P.mu_r;
    for (int a = 0; a < 3; ++a) c.g[a] = P.g[a];
  }
  HIPTRY(hipMemcpy(b->sp.sc, sc.data(), sizeof(SpConst) * sc.size(), hipMemcpyHostToDevice));
  return LPR_OK;
}

lpr_status lpr_set_stepper(lpr_bed* b, int32_t kind, int32_t n_iter) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (kind != LPR_STEPPER_EXPLICIT && kind != LPR_STEPPER_SPOOK) return fail(LPR_E_INVAL, "unknown stepper");
  if (kind == LPR_STEPPER_SPOOK) {
    if (n_iter < 1 || n_iter > 100000) return fail(LPR_E_INVAL, "n_iter must be in [1, 100000]");
    if (b->R != 1 || b->skin > 0.f)
      return fail(LPR_E_INVAL, "the implicit step searches contacts every step (rebuild_every 1, no skin)");
    for (const HostBed& H : b->hb)
      for (const lpr_body& B : H.bodies)
        if (B.z_free) return fail(LPR_E_INVAL, "the implicit step takes prescribed bodies only");
  }
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  if (kind == LPR_STEPPER_SPOOK && !b->sp_ready) {
    const size_t N = (size_t)b->d.N, W = (size_t)b->max_walls;
    SpBufs& sp = b->sp;
    bool ok = dal(b, &sp.sc, b->hb.size()) && dal(b, &sp.row, (size_t)K * N) && dal(b, &sp.imp, (size_t)K * N) &&
              dal(b, &sp.wrow, W * N) && dal(b, &sp.wimp, W * N) && dal(b, &sp.vel, N) && dal(b, &sp.sinv, N) &&
              dal(b, &sp.flag, N) && dal(b, &sp.own, N) && dal(b, &sp.cb, (size_t)K * N);
    if (!ok) return fail(LPR_E_NOMEM, "implicit step buffers");
    sp.nwall_max = b->max_walls;
    HIPTRY(hipMemset(sp.flag, 0, sizeof(uint32_t) * N));
    b->sp_ready = true;
  }
  if (kind == LPR_STEPPER_SPOOK) {
    lpr_status cs = upload_sp_consts(b);
    if (cs != LPR_OK) return cs;
  }
  // the captured cycle holds the previous stepper's kernels
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->has_graph = false;
  b->stepper = kind;
  b->n_iter = (kind == LPR_STEPPER_SPOOK) ? n_iter : 0;
  return LPR_OK;
}

lpr_status lpr_set_contact_params(lpr_bed* b, double s_k, double mu_t, double mu_r) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (!(s_k > 0.0) || !(mu_t >= 0.0) || !(mu_r >= 0.0)) return fail(LPR_E_INVAL, "invalid contact parameters");
  HIPTRY(hipStreamSynchronize(b->stream));
  for (size_t q = 0; q < b->hb.size(); ++q) {
    HostBed& H = b->hb[q];
    H.params.s_k = s_k;
    H.params.mu_t = mu_t;
    H.params.mu_r = mu_r;
    const lpr_params& P = H.params;
    BedConst C;
    HIPTRY(hipMemcpy(&C, b->d.beds + q, sizeof(BedConst), hipMemcpyDeviceToHost));
    const double Estar = 1.0 / ((1.0 - P.nu * P.nu) / P.E + (1.0 - P.nu * P.nu) / P.E);
    C.kfac = (float)(P.s_k * Estar / 3.0);
    C.s_k = (float)P.s_k;
    C.mu_t = (float)P.mu_t;
    C.mu_r = (float)P.mu_r;
    HIPTRY(hipMemcpy(b->d.beds + q, &C, sizeof(BedConst), hipMemcpyHostToDevice));
  }
  if (b->sp_ready) return upload_sp_consts(b);
  return LPR_OK;
}

lpr_status lpr_adjoint_window(lpr_bed* b, int64_t n_steps, int32_t ckpt_every, int32_t body, double* J_out,
                              double grad_out[3]) {
  lpr_status g = guard(b);
  if (g != LPR_OK) return g;
  if (b->hb.size() != 1) return fail(LPR_E_INVAL, "the adjoint window runs on a single bed");
  if (b->stepper != LPR_STEPPER_EXPLICIT)
    return fail(LPR_E_STATE, "the adjoint window differentiates the explicit step only");
  const HostBed& H = b->hb[0];
  if (n_steps <= 0 || ckpt_every <= 0 || !J_out || !grad_out) return fail(LPR_E_INVAL, "bad arguments");
  if (body < 0 || body >= H.nbody) return fail(LPR_E_INVAL, "body out of range");
  for (const lpr_body& B : H.bodies)
    if (B.z_free || B.ang_vel != 0.0)
      return fail(LPR_E_INVAL, "the adjoint supports prescribed, non-rotating bodies only");
  lpr_status st = sync_check(b);
  if (st != LPR_OK) return st;
  DevBufs& d = b->d;
  const int64_t N = d.N;
  // Candidate lists stay fixed within a checkpoint segment: they are built
  // at each segment start with a skin that has to cover the whole segment.
  // The bed's own skin if it has one (its cells were planned for it), else a
  // quarter of the smallest radius, never more than the cell plan covers.
  const double skin_d = b->skin > 0.f ? (double)b->skin : std::min(0.25 * H.rmin, 0.9 * H.skin_cap);
  if (!(skin_d > 0.0))
    return fail(LPR_E_INVAL, "the adjoint window needs candidate lists with a skin: create the bed with "
                             "rebuild_every > 1 and skin > 0, or with cell_factor > 1");
  const float skin = (float)skin_d;
  const int R0 = b->R, Reff0 = b->R_eff;
  const float skin0 = b->skin;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->has_graph = false;
  b->sort_hold = true;  // one storage order for the window: the records index particles by it
  auto restore_mode = [&]() {
    b->sort_hold = false;
    b->R = R0;
    b->R_eff = Reff0;
    b->skin = skin0;
    (void)set_device_skin(b, skin0);
    // the displacement record belongs to the recomputed segments: rebuild
    // before the next step
    b->since = std::numeric_limits<int64_t>::max() / 2;
  };
  double sum6[6];
  int64_t wsteps = 0;
  if ((st = reaction_window_impl(b, 0, body, sum6, &wsteps, 1)) != LPR_OK) { restore_mode(); return st; }
  // Forward window with checkpoints.  When a particle moves more than skin/2
  // within a segment the segment was too long for this skin: go back to the
  // window start and halve the interval (a one-step segment rebuilds its
  // lists every step and cannot trip).
  int C = (int)std::min<int64_t>(ckpt_every, n_steps);
  int64_t nseg = 0;
  for (;;) {
    nseg = (n_steps + C - 1) / C;
    if (!adj_reserve(b, C, (int)nseg + 1)) { restore_mode(); return fail(LPR_E_NOMEM, "adjoint buffers"); }
    b->R = C;
    b->R_eff = C;
    b->skin = C > 1 ? skin : 0.f;
    if ((st = set_device_skin(b, b->skin)) != LPR_OK) { restore_mode(); return st; }
    const int64_t trips0 = b->skin_trips;
    for (int64_t s = 0; s < nseg; ++s) {
      if ((st = ckpt_save(b, b->ckpts[s])) != LPR_OK) { restore_mode(); return st; }
      b->since = std::numeric_limits<int64_t>::max() / 2;
      const int64_t ns = std::min<int64_t>(C, n_steps - s * C);
      for (int64_t q = 0; q < ns; ++q) enqueue_step(b);
    }
    if ((st = sync_check(b)) != LPR_OK) { restore_mode(); return st; }
    if (b->skin_trips == trips0) break;
    if ((st = ckpt_restore(b, b->ckpts[0])) != LPR_OK) { restore_mode(); return st; }
    HIPTRY(hipStreamSynchronize(b->stream));
    b->base_steps = b->host_steps;
    b->base_par = cur_par(b);
    b->plog.clear();
    C = std::max(1, C / 2);
  }
  b->adj_interval = C;
  if ((st = reaction_window_impl(b, 0, body, sum6, &wsteps, 1)) != LPR_OK) { restore_mode(); return st; }
  const double J = sum6[2] / (double)n_steps;
  lpr_bed::Ckpt& end = b->ckpts[nseg];
  if ((st = ckpt_save(b, end)) != LPR_OK) { restore_mode(); return st; }
  // reverse sweep
  AdjBufs& a = b->adj;
  hipStream_t sm = b->stream;
  const int W = b->max_walls;
  HIPTRY(hipMemsetAsync(a.xb, 0, sizeof(float4) * N, sm));
  HIPTRY(hipMemsetAsync(a.vb, 0, sizeof(float4) * N, sm));
  HIPTRY(hipMemsetAsync(a.wb, 0, sizeof(float4) * N, sm));
  HIPTRY(hipMemsetAsync(a.theta, 0, sizeof(double) * 3 * N, sm));
  for (int q = 0; q < 2; ++q) {
    HIPTRY(hipMemsetAsync(a.hbA[q], 0, sizeof(float4) * K * N, sm));
    HIPTRY(hipMemsetAsync(a.hbB[q], 0, sizeof(float2) * K * N, sm));
    HIPTRY(hipMemsetAsync(a.wbA[q], 0, sizeof(float4) * W * N, sm));
    HIPTRY(hipMemsetAsync(a.wbB[q], 0, sizeof(float2) * W * N, sm));
  }
  const int obj = H.body0 + body;
  const float invT = (float)(1.0 / (double)n_steps);
  int hp = 0;
  for (int64_t s = nseg - 1; s >= 0; --s) {
    const lpr_bed::Ckpt& ck = b->ckpts[s];
    if ((st = ckpt_restore(b, ck)) != LPR_OK) { restore_mode(); return st; }
    b->since = std::numeric_limits<int64_t>::max() / 2;
    const int ns = (int)std::min<int64_t>(C, n_steps - s * C);
    for (int q = 0; q < ns; ++q) {  // recompute, recording each step's inputs
      if (b->since >= b->R_eff) enqueue_rebuild(b);
      if (q == 0) {
        HIPTRY(d2d(a.own_cnt, d.own_cnt[b->l], sizeof(int32_t) * N, sm));
        HIPTRY(d2d(a.own_idx, d.own_idx[b->l], sizeof(int32_t) * K * N, sm));
        HIPTRY(d2d(a.rev_start, d.rev_start, sizeof(uint32_t) * (N + 1), sm));
        HIPTRY(d2d(a.rev_ent, d.rev_ent, sizeof(uint32_t) * K * N, sm));
      }
      HIPTRY(d2d(a.st + (int64_t)q * N, d.st[b->s], sizeof(PState) * N, sm));
      HIPTRY(d2d(a.cflag + (int64_t)q * N, d.cflag[b->h], sizeof(uint32_t) * N, sm));
      HIPTRY(d2d(a.hist + (int64_t)q * K * N, d.hist[b->h], sizeof(HRec) * K * N, sm));
      HIPTRY(d2d(a.wA + (int64_t)q * W * N, d.wA[b->h], sizeof(float4) * W * N, sm));
      HIPTRY(d2d(a.wB + (int64_t)q * W * N, d.wB[b->h], sizeof(float2) * W * N, sm));
      HIPTRY(d2d(a.walls + (int64_t)q * a.nwall_total, d.walls, sizeof(WallPose) * a.nwall_total, sm));
      StepPar p{b->s, b->h, b->l, false};
      launch_step(d, p, b->block, b->record, b->persist_blocks, sm);
      launch_advance(d, b->block, sm);
      b->s ^= 1;
      b->h ^= 1;
      b->since += 1;
      b->host_steps += 1;
    }
    for (int q = ns - 1; q >= 0; --q) {
      launch_adj_pre(d, a, q, sm);
      launch_adj_step(d, a, q, hp, obj, invT, sm);
      hp ^= 1;
    }
    if (s > 0) {
      launch_adj_remap(d, a, ck.own_cnt, ck.own_idx, ck.cflag, hp, sm);
      hp ^= 1;
    }
    HIPTRY(hipGetLastError());
  }
  launch_adj_theta(d, a, b->theta_out, sm);
  double grad[3];
  HIPTRY(hipMemcpyAsync(grad, b->theta_out, sizeof(grad), hipMemcpyDeviceToHost, sm));
  HIPTRY(hipStreamSynchronize(sm));
  // back to the state after the window
  if ((st = ckpt_restore(b, end)) != LPR_OK) { restore_mode(); return st; }
  restore_mode();
  if ((st = sync_check(b)) != LPR_OK) return st;
  *J_out = J;
  for (int c = 0; c < 3; ++c) grad_out[c] = grad[c];
  return LPR_OK;
}

// Single-bed entry points address bed 0; the batch ones take a bed index.
lpr_status lpr_get_state(lpr_bed* b, double* pos, float* vel, float* omega) { return get_state_impl(b, 0, pos, vel, omega); }
lpr_status lpr_batch_get_state(lpr_bed* b, int32_t bed, double* pos, float* vel, float* omega) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return get_state_impl(b, bed, pos, vel, omega);
}
lpr_status lpr_set_state(lpr_bed* b, const double* pos, const float* vel, const float* omega) { return set_state_impl(b, 0, pos, vel, omega); }
lpr_status lpr_batch_set_state(lpr_bed* b, int32_t bed, const double* pos, const float* vel, const float* omega) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return set_state_impl(b, bed, pos, vel, omega);
}
lpr_status lpr_get_history(lpr_bed* b, lpr_history* out, int64_t capacity, int64_t* n_total) { return get_history_impl(b, 0, out, capacity, n_total); }
lpr_status lpr_batch_get_history(lpr_bed* b, int32_t bed, lpr_history* out, int64_t capacity, int64_t* n_total) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return get_history_impl(b, bed, out, capacity, n_total);
}
lpr_status lpr_set_history(lpr_bed* b, const lpr_history* rec, int64_t count) { return set_history_impl(b, 0, rec, count); }
lpr_status lpr_batch_set_history(lpr_bed* b, int32_t bed, const lpr_history* rec, int64_t count) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return set_history_impl(b, bed, rec, count);
}
lpr_status lpr_read_contacts(lpr_bed* b, lpr_contact* out, int64_t capacity, int64_t* n_total) { return read_contacts_impl(b, 0, out, capacity, n_total); }
lpr_status lpr_batch_read_contacts(lpr_bed* b, int32_t bed, lpr_contact* out, int64_t capacity, int64_t* n_total) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_contacts_impl(b, bed, out, capacity, n_total);
}
lpr_status lpr_read_forces(lpr_bed* b, float* force, float* torque) { return read_forces_impl(b, 0, force, torque); }
lpr_status lpr_batch_read_forces(lpr_bed* b, int32_t bed, float* force, float* torque) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_forces_impl(b, bed, force, torque);
}
lpr_status lpr_read_contact_loads(lpr_bed* b, lpr_contact_load* out, int64_t capacity, int64_t* n_total) {
  return read_contact_loads_impl(b, 0, out, capacity, n_total);
}
lpr_status lpr_batch_read_contact_loads(lpr_bed* b, int32_t bed, lpr_contact_load* out, int64_t capacity,
                                        int64_t* n_total) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_contact_loads_impl(b, bed, out, capacity, n_total);
}
lpr_status lpr_read_wall_pose(lpr_bed* b, int32_t wall, double out15[15]) { return read_wall_pose_impl(b, 0, wall, out15); }
lpr_status lpr_batch_read_wall_pose(lpr_bed* b, int32_t bed, int32_t wall, double out15[15]) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_wall_pose_impl(b, bed, wall, out15);
}
lpr_status lpr_read_reaction(lpr_bed* b, int32_t body, double out6[6]) { return read_reaction_impl(b, 0, body, out6); }
lpr_status lpr_batch_read_reaction(lpr_bed* b, int32_t bed, int32_t body, double out6[6]) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_reaction_impl(b, bed, body, out6);
}
lpr_status lpr_reaction_window(lpr_bed* b, int32_t body, double sum6[6], int64_t* steps, int32_t reset) { return reaction_window_impl(b, 0, body, sum6, steps, reset); }
lpr_status lpr_batch_reaction_window(lpr_bed* b, int32_t bed, int32_t body, double sum6[6], int64_t* steps, int32_t reset) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return reaction_window_impl(b, bed, body, sum6, steps, reset);
}
lpr_status lpr_read_body(lpr_bed* b, int32_t body, double origin[3], double vel[3]) { return read_body_impl(b, 0, body, origin, vel); }
lpr_status lpr_batch_read_body(lpr_bed* b, int32_t bed, int32_t body, double origin[3], double vel[3]) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return read_body_impl(b, bed, body, origin, vel);
}
lpr_status lpr_set_clock(lpr_bed* b, int64_t step) { return set_clock_impl(b, 0, step); }
lpr_status lpr_batch_set_clock(lpr_bed* b, int32_t bed, int64_t step) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return set_clock_impl(b, bed, step);
}
lpr_status lpr_get_clock(lpr_bed* b, int64_t* step) { return get_clock_impl(b, 0, step); }
lpr_status lpr_batch_get_clock(lpr_bed* b, int32_t bed, int64_t* step) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return get_clock_impl(b, bed, step);
}
lpr_status lpr_set_body_state(lpr_bed* b, int32_t body, double z, double vz) { return set_body_state_impl(b, 0, body, z, vz); }
lpr_status lpr_batch_set_body_state(lpr_bed* b, int32_t bed, int32_t body, double z, double vz) {
  if (!b || bed < 0 || bed >= (int32_t)b->hb.size()) return fail(LPR_E_INVAL, "bed index out of range");
  return set_body_state_impl(b, bed, body, z, vz);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Per-contact read without allocation: the workspace is a static device
// array, one per GPU the library runs on, held until the process ends.  Host
// code must use its address from hipGetSymbolAddress (the array's own name is
// a host-side stand-in), taken once per device with that device current.

static_assert(LPR_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[LPR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

lpr_status scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LPR_E_DEVICE, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LPR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return LPR_OK;
}

lpr_status read_contact_loads_noalloc_impl(lpr_bed* b, int32_t bed, lpr_contact_load* out, int64_t capacity,
                                           int64_t* n_total) {
  lpr_status st = loads_readable(b);
  if (st != LPR_OK) return st;
  // no sync_check: its recovery from a skin trip re-enqueues steps and grows
  // host logs; a bed whose last steps have not been checked is refused
  HIPTRY(hipStreamSynchronize(b->stream));
  uint32_t e = 0;
  HIPTRY(hipMemcpy(&e, b->d.err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (e != 0u || b->faulted) return fail(LPR_E_STATE, "the bed has a pending device status: call lpr_sync first");
  const int64_t np = b->hb[bed].npad;
  const size_t head = load_head_bytes(np);
  if (head > (size_t)LPR_NOALLOC_SCRATCH_BYTES)
    return fail(LPR_E_CAPACITY, "bed too large for the static scratch of lpr_read_contact_loads_noalloc");
  char* ws = nullptr;
  if ((st = scratch_address(b->device, &ws)) != LPR_OK) return st;
  int64_t total = 0;
  if ((st = load_count(b, bed, ws, &total)) != LPR_OK) return st;
  if (n_total) *n_total = total;
  if (total > capacity) return fail(LPR_E_CAPACITY, "contact buffer too small");
  if (head + sizeof(lpr_contact_load) * (size_t)total > (size_t)LPR_NOALLOC_SCRATCH_BYTES)
    return fail(LPR_E_CAPACITY, "more contacts than the static scratch of lpr_read_contact_loads_noalloc holds");
  return load_pack(b, bed, ws, (lpr_contact_load*)(ws + head), total, out);
}

}  // namespace

extern "C" {

lpr_status lpr_read_contact_loads_noalloc(lpr_bed* b, lpr_contact_load* out, int64_t capacity, int64_t* n_total) {
  if (!b) return fail(LPR_E_INVAL, "null bed");
  int cur = 0;
  HIPTRY(hipGetDevice(&cur));
  if (cur != b->device) HIPTRY(hipSetDevice(b->device));
  const lpr_status st = read_contact_loads_noalloc_impl(b, 0, out, capacity, n_total);
  if (cur != b->device) (void)hipSetDevice(cur);
  return st;
}

}  // extern "C"
