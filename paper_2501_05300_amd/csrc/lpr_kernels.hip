// lpr_kernels.hip -- HIP kernels of the graded-bed DEM step (gfx950).
//
// One step with the broad phase rebuilt (per step when rebuild_every = 1):
//   k_zero      clear cell and reverse counters
//   k_bin       per particle: cell of its own radius-band level, rank in cell
//   scan        exclusive scan of cell counts -> cell ranges
//   k_scatter   cell lists
//   k_search    owner-side candidates: same level with larger (r, id), and
//               every coarser level within reach, in the neighbour cells
//               whose box lies within reach; sorted by partner id; lists and
//               springs updated in place (or moved after a re-sort);
//               reverse counts
//   scan        reverse ranges;  k_rev_scatter / k_rev_sort: partner-side
//               entries in ascending owner stable id
// then every step:
//   k_step      fused narrow phase + contact law + accumulation + walls +
//               integration; each particle evaluates all of its contacts
//               (as owner and as partner) through one code path, so the two
//               sides of a pair are bitwise opposite; FP64 reaction partials
//   k_advance   ordered FP64 reduction of reactions, dynamic bodies, next
//               wall poses, clock
#include "lpr_cells.h"
#include "lpr_kernels.h"

namespace lpr {

#define LPR_DEV_INLINE __device__ __forceinline__

LPR_DEV_INLINE bool latched(const uint32_t* err) { return *(const volatile uint32_t*)err != 0u; }

// ---------------------------------------------------------------------------
// helpers

// Clears two arrays in one launch (the rebuild's cell and reverse counters):
// 16-byte stores over each array's whole groups of four words when both are
// 16-byte aligned (vec), single words otherwise and for the last few.
__global__ void k_zero(uint32_t* p, int64_t n, uint32_t* q, int64_t m, int vec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n4 = vec ? n / 4 : 0, m4 = vec ? m / 4 : 0;
  for (int64_t i = t0; i < n4 + m4; i += stride) {
    if (i < n4)
      reinterpret_cast<uint4*>(p)[i] = make_uint4(0u, 0u, 0u, 0u);
    else
      reinterpret_cast<uint4*>(q)[i - n4] = make_uint4(0u, 0u, 0u, 0u);
  }
  const int64_t rn = n - 4 * n4, rm = m - 4 * m4;
  for (int64_t i = t0; i < rn + rm; i += stride) {
    if (i < rn)
      p[4 * n4 + i] = 0u;
    else
      q[4 * m4 + (i - rn)] = 0u;
  }
}

void launch_zero(uint32_t* p, int64_t n, uint32_t* q, int64_t m, hipStream_t st) {
  if (n + m <= 0) return;
  const int vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(q)) & 15u) == 0u ? 1 : 0;
  const int64_t work = vec ? (n + m) / 4 + 8 : n + m;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n, q, m, vec);
}

// Work block handled by launch block b of a grid of g blocks: the blocks
// that the hardware places on one XCD (b mod 8) take one contiguous range of
// particles, so neighbours they gather share that XCD's L2.
LPR_DEV_INLINE int64_t xcd_block(int64_t b, int64_t g) {
  const int64_t chunk = (g + 7) / 8;
  const int64_t x = b & 7, q = b >> 3;
  const int64_t w = x * chunk + q;
  return w < g ? w : -1;
}

// ---------------------------------------------------------------------------
// binning

// FP32 value <-> unsigned key with the same order (0 lies below every
// finite value), for extents kept with integer atomicMax.
LPR_DEV_INLINE uint32_t ord_key(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
LPR_DEV_INLINE float ord_val(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Bins every particle into the grid of its own level and widens the level's
// recorded range of centre heights (monotone, so a stale range is still a
// superset; one atomic per wave and bound, and only when the wave's value
// extends it).
// Consecutive particles mostly share cells: the lanes of a wave that fall in
// one cell take their ranks from a single atomic (ballot, prefix count), and
// the wave's atomics for all its cells go out in one instruction.
//
// SORT also writes the particle's sort key, its level's first cell id plus
// the Morton rank of its cell in the level grid (so keys order particles by
// bed, level and Morton code of the cell), and its storage index; padding
// gets a key above every cell.
template <bool SORT>
__global__ void k_bin(DevBufs d, int s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d.N || latched(d.err)) return;
  const uint32_t m = d.meta[i];
  if (m == INACTIVE) {
    if (SORT) {
      d.skey[0][i] = (1u << d.sort_bits) - 1u;
      d.sval[0][i] = (int32_t)i;
    }
    return;
  }
  const BedConst& bc = d.beds[m >> 8];
  const int gl = bc.lev0 + (int)(m & 0xffu);
  const LevelGrid& G = d.levels[gl];
  const double4 p = d.st[s][i].x;
  const int cx = cell_axis(G, 0, p.x), cy = cell_axis(G, 1, p.y), cz = cell_axis(G, 2, p.z);
  const int32_t c = (int32_t)(G.base + ((int64_t)cz * G.n[1] + cy) * G.n[0] + cx);
  d.pcell[i] = c;
  {
    // outside the level's grid on a bounded axis the particle is binned into
    // the edge cell (the search covers it there); count such binnings
#pragma clang fp contract(off)
    bool out = false;
    const double q[3] = {p.x, p.y, p.z};
    for (int a = 0; a < 3; ++a)
      if (!G.per[a]) {
        const double f = (q[a] - G.lo[a]) * G.inv_w[a];
        out = out || !(f >= 0.0 && f < (double)G.n[a]);
      }
    if (out) atomicAdd(&d.stat[2], 1u);
  }
  if (SORT) {
    const int32_t cc[3] = {cx, cy, cz};
    d.skey[0][i] = (uint32_t)(G.base + morton_rank(cc, G.n));
    d.sval[0][i] = (int32_t)i;
  }
  // group the wave's lanes by cell (votes only), then one atomic per group,
  // all groups' atomics issued together
  const int lane = (int)(threadIdx.x & 63u);
  uint64_t todo = __ballot(1);  // the wave's active lanes
  int leader_of = lane;
  uint32_t off = 0u, gsize = 0u;
  while (todo != 0ull) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int32_t key = __shfl(c, leader, 64);
    const uint64_t grp = __ballot(c == key) & todo;
    if ((grp >> lane) & 1ull) {
      leader_of = leader;
      off = (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
    }
    if (lane == leader) gsize = (uint32_t)__popcll(grp);
    todo &= ~grp;
  }
  uint32_t base = 0u;
  if (lane == leader_of) base = atomicAdd(&d.cell_cnt[c], gsize);
  d.prank[i] = __shfl(base, leader_of, 64) + off;
  uint32_t khi = ord_key((float)p.z), klo = ord_key(-(float)p.z);
  // a full wave whose lanes share one level (nearly every wave) reduces first
  const int gl0 = __shfl(gl, __ffsll((unsigned long long)__ballot(1)) - 1, 64);
  if (__ballot(1) == ~0ull && __all(gl == gl0)) {
    for (int o = 32; o >= 1; o >>= 1) {
      khi = max(khi, (uint32_t)__shfl_xor((int)khi, o, 64));
      klo = max(klo, (uint32_t)__shfl_xor((int)klo, o, 64));
    }
  }
  if (khi > *(const volatile uint32_t*)&d.zext[2 * gl]) atomicMax(&d.zext[2 * gl], khi);
  if (klo > *(const volatile uint32_t*)&d.zext[2 * gl + 1]) atomicMax(&d.zext[2 * gl + 1], klo);
}

void launch_bin(const DevBufs& d, int s, int sort, hipStream_t st) {
  if (sort) hipLaunchKernelGGL(k_bin<true>, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, d, s);
  else hipLaunchKernelGGL(k_bin<false>, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, d, s);
}

// Fills the cell lists, with the position, radius and stable id copied
// alongside so that the search reads each cell's candidates contiguously.
__global__ void k_scatter(DevBufs d, int s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d.N || latched(d.err)) return;
  if (d.meta[i] == INACTIVE) return;
  const int32_t c = d.pcell[i];
  const uint32_t q = d.cell_start[c] + d.prank[i];
  d.cell_list[q] = (int32_t)i;
  const double4 p = d.st[s][i].x;
  CRec cr;
  cr.x = p.x;
  cr.y = p.y;
  cr.z = p.z;
  cr.r = (float)p.w;  // radii are FP32 values, so this is exact
  cr.sid = d.sid[i];
  d.crec[q] = cr;
  d.cpf[q] = make_float4((float)p.x, (float)p.y, (float)p.z, (float)p.w);
}

void launch_scatter(const DevBufs& d, int s, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, d, s);
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 counts: tiles of 2048 (256 threads x 8)

constexpr int SB = 256, SIPT = 8, STILE = SB * SIPT;

LPR_DEV_INLINE uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[SB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int q = 0; q < SB / 64; ++q) {
    if (q < wv) off += wsum[q];
    tot += wsum[q];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// A thread's eight counts: two 16-byte reads where all eight lie inside and
// the array is 16-byte aligned (base is a multiple of eight).
LPR_DEV_INLINE void load8(const uint32_t* in, int64_t base, int64_t n, bool vec, uint32_t v[SIPT]) {
  if (vec && base + SIPT <= n) {
    const uint4 a = *reinterpret_cast<const uint4*>(in + base), b = *reinterpret_cast<const uint4*>(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    for (int q = 0; q < SIPT; ++q) v[q] = (base + q < n) ? in[base + q] : 0u;
  }
}

__global__ void k_scan_tiles(const uint32_t* in, uint32_t* tsum, int64_t n, int vec) {
  const int64_t base = blockIdx.x * (int64_t)STILE + threadIdx.x * SIPT;
  uint32_t v[SIPT];
  load8(in, base, n, vec != 0, v);
  uint32_t s = 0;
  for (int q = 0; q < SIPT; ++q) s += v[q];
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// Each tile's offset is the sum of the earlier tiles' sums, added up by the
// tile's own block (a few coalesced reads per thread: the sums of a few
// thousand tiles), then the tile is scanned.
__global__ void k_scan_apply(const uint32_t* in, uint32_t* out, const uint32_t* tsum, int64_t n, int vec) {
  uint32_t pre = 0;
  for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += SB) pre += tsum[t];
  uint32_t toff;
  block_excl_scan(pre, &toff);
  const int64_t base = blockIdx.x * (int64_t)STILE + threadIdx.x * SIPT;
  uint32_t v[SIPT];
  load8(in, base, n, vec != 0, v);
  uint32_t s = 0;
  for (int q = 0; q < SIPT; ++q) s += v[q];
  uint32_t tot;
  uint32_t off = block_excl_scan(s, &tot) + toff;
  uint32_t o[SIPT];
  for (int q = 0; q < SIPT; ++q) {
    o[q] = off;
    off += v[q];
  }
  if (vec && base + SIPT <= n) {
    *reinterpret_cast<uint4*>(out + base) = make_uint4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<uint4*>(out + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    if (base + SIPT == n) out[n] = off;
  } else {
    for (int q = 0; q < SIPT; ++q) {
      if (base + q < n) out[base + q] = o[q];
      if (base + q == n - 1) out[n] = o[q] + v[q];
    }
  }
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + STILE - 1) / STILE) + 1; }

void launch_scan(uint32_t* cnt, uint32_t* start, uint32_t* tmp, int64_t n, hipStream_t st) {
  const int64_t tiles = (n + STILE - 1) / STILE;
  const int vec = ((reinterpret_cast<uintptr_t>(cnt) | reinterpret_cast<uintptr_t>(start)) & 15u) == 0u ? 1 : 0;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SB), 0, st, cnt, tmp, n, vec);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(SB), 0, st, cnt, start, tmp, n, vec);
}

// ---------------------------------------------------------------------------
// storage-order sort: stable LSD radix sort of 32-bit keys, 8-bit digits
//
// Each pass: every tile of RS_TILE consecutive entries counts its digits
// (k_rs_hist, digit-major table), the table is scanned (digit d of tile t
// starts after every smaller digit and after digit d of earlier tiles), and
// k_rs_scatter moves each entry to its place.  Within a tile the entries are
// taken in order, a wave at a time: the lanes holding one digit are found by
// eight ballots, a lane's rank among them is the count of lower lanes, the
// lowest lane records the group's size, and one thread per digit turns the
// waves' sizes into offsets.  Equal keys keep their order, so the sorted
// order is (key, previous storage index) whatever the scheduling.

constexpr int RS_BS = 256, RS_ROUNDS = 8, RS_TILE = RS_BS * RS_ROUNDS, RS_BINS = 256;
static_assert(RS_BS == RS_BINS, "one thread per digit");

__global__ __launch_bounds__(RS_BS) void k_rs_hist(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                 uint32_t* __restrict__ hist, int64_t ntiles) {
  __shared__ uint32_t h[RS_BINS];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = blockIdx.x * (int64_t)RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t q = base + r * RS_BS + threadIdx.x;
    if (q < n) atomicAdd(&h[(key[q] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_BS) void k_rs_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                                    int shift, const uint32_t* __restrict__ hoff, int64_t ntiles) {
  __shared__ uint32_t wofs[RS_BS / 64][RS_BINS];  // per wave: group size, then the group's first position
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int dig = threadIdx.x;                    // the digit this thread keeps the running position of
  uint32_t run = hoff[(int64_t)dig * ntiles + blockIdx.x];
  const int64_t base = blockIdx.x * (int64_t)RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int w = 0; w < RS_BS / 64; ++w) wofs[w][dig] = 0u;
    __syncthreads();
    const int64_t q = base + r * RS_BS + threadIdx.x;
    const bool ok = q < n;
    const uint32_t k = ok ? kin[q] : 0u;
    const int32_t v = ok ? vin[q] : 0;
    const uint32_t dg = (k >> shift) & 255u;
    uint64_t same = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t set = __ballot((dg >> b) & 1u);
      same &= ((dg >> b) & 1u) ? set : ~set;
    }
    const uint32_t rk = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    if (ok && rk == 0u) wofs[wv][dg] = (uint32_t)__popcll(same);
    __syncthreads();
#pragma unroll
    for (int w = 0; w < RS_BS / 64; ++w) {
      const uint32_t c = wofs[w][dig];
      wofs[w][dig] = run;
      run += c;
    }
    __syncthreads();
    if (ok) {
      const uint32_t at = wofs[wv][dg] + rk;
      kout[at] = k;
      vout[at] = v;
    }
    __syncthreads();
  }
}

size_t sort_hist_elems(int64_t n) { return (size_t)RS_BINS * (size_t)((n + RS_TILE - 1) / RS_TILE) + 1; }

int launch_sort(const DevBufs& d, hipStream_t st) {
  const int64_t n = d.N, ntiles = (n + RS_TILE - 1) / RS_TILE;
  const int passes = (d.sort_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int a = p & 1;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_BS), 0, st, d.skey[a], n, 8 * p, d.rs_hist, ntiles);
    launch_scan(d.rs_hist, d.rs_hist, d.scan_tmp, RS_BINS * ntiles, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_BS), 0, st, d.skey[a], d.sval[a], d.skey[a ^ 1],
                       d.sval[a ^ 1], n, 8 * p, d.rs_hist, ntiles);
  }
  return passes;
}

// Sorted rank r holds a particle of some bed; its new storage index is r plus
// that bed's offset (beds keep their padded ranges, their particles come
// first in them).  Reads are gathers, writes are in storage order.
__global__ void k_reorder(DevBufs d, int s, int buf, PState* __restrict__ st_out, int32_t* __restrict__ sid_out,
                          uint32_t* __restrict__ meta_out, int32_t* __restrict__ pcell_out,
                          uint32_t* __restrict__ prank_out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= d.n_active || latched(d.err)) return;
  const int32_t o = d.sval[buf][r];
  const uint32_t m = d.meta[o];
  const int64_t i = r + d.beds[m >> 8].sort_off;
  st_out[i] = d.st[s][o];
  sid_out[i] = d.sid[o];
  meta_out[i] = m;
  pcell_out[i] = d.pcell[o];
  prank_out[i] = d.prank[o];
  d.src[i] = o;
}

void launch_reorder(const DevBufs& d, int s, int buf, PState* st_out, int32_t* sid_out, uint32_t* meta_out,
                    int32_t* pcell_out, uint32_t* prank_out, hipStream_t st) {
  if (d.n_active <= 0) return;
  hipLaunchKernelGGL(k_reorder, dim3((unsigned)((d.n_active + 255) / 256)), dim3(256), 0, st, d, s, buf, st_out,
                     sid_out, meta_out, pcell_out, prank_out);
}

// ---------------------------------------------------------------------------
// owner-side search with history carry-over
//
// Each thread walks the neighbourhood of its particle at its own level and
// every coarser one (a coarser level only when its recorded centre heights
// lie within reach): along each axis the particle's cell and those of its
// two neighbours that lie within r_i + r_max(level) + skin of it.  That is at
// most 3 x 3 rows of up to 3 cells; the cells of a row are consecutive in
// the cell order, so the row is one range of the cell lists (two where the x
// axis wraps).  The bounds of a piece's nine rows are read together and the
// non-empty rows packed into a per-lane LDS table.  A first pass reads the
// 16-byte FP32 copy of each candidate, eight per round in one stream over
// the table's rows, and keeps the ones within a conservative FP32 distance
// bound (and not owned by the partner); a second pass reads the kept
// candidates' FP64 records, four at a time, and applies the owner rule and
// the exact predicate.  Accepted partners are put in ascending stable id and
// inherit their spring history from the previous lists.

constexpr int SBS = 64;   // threads per search block
// One LDS array of LROWS rows per lane, used in three ways:
//   first pass: rows [0, RT) the row table, rows [RT, LROWS - 1) the kept
//   list and row LROWS - 1 a sink for the writes that keep nothing;
//   exact walk (kept list full): rows [LROWS - K, LROWS) its partners;
//   accepted partners: positions compacted in place in the kept rows, stable
//   ids in rows [0, K) for the slot sort, then each slot's previous slot.
constexpr int LROWS = 32;
constexpr int RT = 18;             // a level has at most 9 rows in each of two x pieces
constexpr int PCAP = LROWS - RT - 1;  // first-pass candidates kept per particle (more: exact walk)
static_assert(RT >= K && LROWS - K >= K, "sort ids must not overlap a kept list");

// a if c, else b, as bit masks (a plain conditional here would be turned into
// control flow)
LPR_DEV_INLINE uint32_t pick(bool c, uint32_t a, uint32_t b) {
  const uint32_t m = 0u - (uint32_t)c;
  return (a & m) | (b & ~m);
}

// First pass over one level's rows (the row table holds nr packed rows):
// each lane walks its rows as one stream, eight positions per round, so its
// rounds follow its own candidate count, and keeps the candidates that pass
// a conservative FP32 distance bound and are not owned by the partner (a
// larger radius owns nothing here).  WRAP takes the minimum image on the
// periodic axes; a wave whose lanes have no cell across a periodic edge
// skips it, since then every separation is already the nearest image.
// The FP32 copy is read through a buffer resource: 32-bit byte offsets (one
// shift per address) and a hardware range check (reads past the resource
// return zeros).  Word 3 is the data format field of CDNA buffer resources
// for plain dword reads.
LPR_DEV_INLINE __amdgpu_buffer_rsrc_t cand_rsrc(const float4* cpf, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)cpf, (short)0, (int)((n + CPF_PAD) * 16), 0x00020000);
}

LPR_DEV_INLINE float4 cand_load(__amdgpu_buffer_rsrc_t rs, uint32_t q) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(q << 4), 0, 0);
  return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

template <bool WRAP>
LPR_DEV_INLINE void walk_rows(__amdgpu_buffer_rsrc_t cpf, const uint32_t (*rtab)[SBS], int32_t (*c_idx)[SBS], int t,
                              int nr, float pfx, float pfy, float pfz, float rif, float reach, bool perx, bool pery,
                              float Lx, float Ly, int& np) {
  if (nr <= 0) return;
  // rows ri, ri + 1, ri + 2 as packed entries; row ri's unread part is
  // [qa0, qa0 + la), never empty.  Entries past nr are read (they lie inside
  // the LDS array) but never used.
  int ri = 0;
  uint32_t wb = rtab[1][t], wc = rtab[2][t];
  uint32_t qa0, la;
  {
    const uint32_t wa = rtab[0][t];
    qa0 = wa >> 6;
    la = wa & 63u;
  }
  while (ri < nr) {
    float4 c[8];
    uint32_t qa[8];
    bool ok[8];
    // positions of the round: the rest of row ri, then rows ri + 1 and
    // ri + 2 (a round ends early where it would need a fourth row).
    // Position u lies in row A below sB (= avA), in row B below sC, else in
    // row C, at u plus that row's offset.  Positions past the three rows
    // (ok false) are read all the same: they lie within seven of a row's
    // start, which the copy's padding covers, and are never kept.
    const int avA = (int)la;
    const int avB = (ri + 1 < nr) ? (int)(wb & 63u) : 0;
    const int avC = (ri + 2 < nr) ? (int)(wc & 63u) : 0;
    const uint32_t qb0 = (ri + 1 < nr) ? wb >> 6 : qa0, qc0 = (ri + 2 < nr) ? wc >> 6 : qa0;
    const int sB = avA, sC = avA + avB, sE = sC + avC;
    const uint32_t oB = qb0 - (uint32_t)sB, oC = qc0 - (uint32_t)sC;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      qa[u] = (uint32_t)u + (u < sB ? qa0 : (u < sC ? oB : oC));
      ok[u] = u < sE;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = cand_load(cpf, qa[u]);
    {
      // move past the rows this round used up (their LDS entries are read
      // while the candidates are in flight)
      const int s1 = avA, s2 = avA + avB, s3 = s2 + avC;
      const int used = min(8, s3);
      const int k = (used >= s1 ? 1 : 0) + (used >= s2 && ri + 1 < nr ? 1 : 0) + (used >= s3 && ri + 2 < nr ? 1 : 0);
      if (k == 0) {
        qa0 += (uint32_t)used;
        la -= (uint32_t)used;
      } else {
        const int off = used - (k == 1 ? s1 : (k == 2 ? s2 : s3));
        ri += k;
        const uint32_t wa = rtab[ri][t];
        wb = rtab[ri + 1][t];
        wc = rtab[ri + 2][t];
        qa0 = (wa >> 6) + (uint32_t)off;
        la = (wa & 63u) - (uint32_t)off;
      }
    }
    // the test is evaluated for all eight without branching, so each
    // candidate stays one 16-byte read (a branch on the radius first would
    // let the compiler fetch the position only after it)
    bool keep[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      float fx = c[u].x - pfx, fy = c[u].y - pfy;
      const float fz = c[u].z - pfz;
      if (WRAP) {
        if (perx) fx = (fx > 0.5f * Lx) ? fx - Lx : ((fx < -0.5f * Lx) ? fx + Lx : fx);
        if (pery) fy = (fy > 0.5f * Ly) ? fy - Ly : ((fy < -0.5f * Ly) ? fy + Ly : fy);
      }
      const float Rf = reach + c[u].w;
      // j owns pairs with a smaller radius (bitwise and: no short circuit)
      keep[u] = ok[u] & !(c[u].w < rif) & (fx * fx + fy * fy + fz * fz < Rf * Rf);
    }
    // every slot writes (no branches): a slot that keeps nothing writes the
    // next free entry, which a kept one overwrites, or the sink row once the
    // list is full
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c_idx[min(np, PCAP)][t] = (int32_t)qa[u];
      np += keep[u] ? 1 : 0;
    }
  }
}

// Whether a coarser level has a centre within `reach` of the particle's
// height (its extents are FP32 roundings: widened by one FP32 ulp).
LPR_DEV_INLINE bool level_in_reach(const DevBufs& d, int gl, const double4& pi, double reach) {
  const uint32_t khi = d.zext[2 * gl], klo = d.zext[2 * gl + 1];
  if (khi == 0u) return false;  // no particle at this level
  const float fhi = ord_val(khi), flo = -ord_val(klo);
  const double zhi = (double)fhi + ((double)fabsf(fhi) * 0x1p-23 + 0x1p-126);
  const double zlo = (double)flo - ((double)fabsf(flo) * 0x1p-23 + 0x1p-126);
  return pi.z - zhi < reach && zlo - pi.z < reach;
}

// Owner rule (the smaller radius owns; equal radii, the smaller stable id)
// and the exact FP64 predicate d < r_i + r_j + skin.
LPR_DEV_INLINE bool owner_candidate(const BedConst& bc, const double4& pi, int32_t si, double skin, const CRec& c) {
  const float rif = (float)pi.w;
  if (c.r < rif) return false;
  if (c.r == rif && c.sid <= si) return false;
  const double4 pj = make_double4(c.x, c.y, c.z, (double)c.r);
  double dx, dy, dz;
  const double d2 = pair_sep(bc, pi, pj, dx, dy, dz);
  return within_skin(d2, pi.w, pj.w, skin);
}

// Five waves per SIMD: 8 KB of LDS per 64-lane block and at most 96 VGPRs
// (the previous lists' partners are read after the walk to stay within them).
// src (after a re-sort of the storage order): the index each particle had
// when the previous lists were built; their partners are matched through it.
__global__ __launch_bounds__(SBS) __attribute__((amdgpu_waves_per_eu(5))) void k_search(DevBufs d, int s, int lo, int ho,
                                                                                       const int32_t* __restrict__ src) {
  // rows of the level being walked are packed as (first cell-list position
  // << 6 | length); the rows' layout over the array is described at LROWS
  __shared__ int32_t lds[LROWS][SBS];
  uint32_t (*const rtab)[SBS] = reinterpret_cast<uint32_t (*)[SBS]>(lds);
  int32_t (*const c_sid)[SBS] = lds;
  int32_t (*c_idx)[SBS] = lds + RT;  // kept candidates, then the accepted ones
  const int t = threadIdx.x;
  // each XCD takes one contiguous range of particles, so the neighbour rows
  // its blocks read overlap in that XCD's L2
  const int64_t blk = xcd_block(blockIdx.x, (d.N + SBS - 1) / SBS);
  if (blk < 0) return;
  const int64_t i = blk * SBS + t;
  if (i >= d.N || latched(d.err)) return;
  // after a re-sort of the storage order (src given) the lists and springs
  // are written to the other buffers; otherwise they are updated in place
  const bool moved = src != nullptr;
  const int ln = moved ? lo ^ 1 : lo, hn = moved ? ho ^ 1 : ho;
  const int64_t N = d.N;
  if (i == 0) {  // fresh lists: no displacement since they were built
    d.viol[0] = 0u;
    d.viol[1] = 0u;
  }
  const uint32_t m = d.meta[i];
  if (m == INACTIVE) {
    d.own_cnt[ln][i] = 0;
    d.cflag[hn][i] = 0u;
    return;
  }
  // a wave holds particles of one bed (beds are padded to PAD particles, a
  // multiple of the wave size), so the bed's constants and level grids are
  // read once per wave, as scalars
  const int bed = __builtin_amdgcn_readfirstlane((int)(m >> 8));
  const BedConst bc = d.beds[bed];
  const int lev_i = (int)(m & 0xffu);
  const double4 pi = d.st[s][i].x;
  // the previous lists' flags and count, read now so that their latency
  // hides behind the walk
  const int64_t io = moved ? (int64_t)src[i] : i;
  const uint32_t fo = d.cflag[ho][io];
  const int cnt_old = d.own_cnt[lo][io];
  const float rif = (float)pi.w;
  const int32_t si = d.sid[i];
  const double skin = (double)bc.skin;
  const float pfx = (float)pi.x, pfy = (float)pi.y, pfz = (float)pi.z;
  const float Lx = (float)bc.L[0], Ly = (float)bc.L[1];
  const bool perx = (bc.periodic & 1u) != 0, pery = (bc.periodic & 2u) != 0;
  // FP32 bound: rounding the coordinates to FP32 and forming their (wrapped)
  // differences errs by a few ulp of the largest magnitude involved (the
  // candidate lies within the particle's magnitude plus one period);
  // 2^-19 of it is 16 ulp
  const float mag = fmaxf(fmaxf(fabsf(pfx), fabsf(pfy)), fmaxf(fabsf(pfz), fmaxf(Lx, Ly)));
  const float reach = rif + bc.skin + mag * 0x1p-19f;
  const __amdgpu_buffer_rsrc_t crs = cand_rsrc(d.cpf, N);
  int np = 0;
  // levels in a loop that is the same for the whole wave (so each level's
  // grid is a scalar read); a lane takes part from its own level on, in the
  // coarser ones when their centres are within reach, and while its kept
  // list has room
  for (int lev = 0; lev < bc.nlev; ++lev) {
    const int gl = bc.lev0 + lev;
    const LevelGrid G = d.levels[gl];
    const double rch = pi.w + G.rmax + skin;
    const bool want = lev >= lev_i && np <= PCAP && (lev == lev_i || level_in_reach(d, gl, pi, rch));
    if (!__any(want)) continue;
    int nr = 0;
    bool wide = false;
    RowSet R;
    R.across = false;
    if (want) {
      row_set(G, pi, rch, R);
#pragma unroll
      for (int p = 0; p < 2; ++p) {  // compile-time piece index (registers, not scratch)
        if (p >= R.nxp) break;
        uint32_t q0[9], q1[9];
        row_piece(d.cell_start, G, R, p, q0, q1);
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const uint32_t len = q1[r] - q0[r];
          if (len > 0u) {
            wide = wide || len > 63u || q0[r] >= (1u << 26);
            rtab[nr][t] = (q0[r] << 6) | (len & 63u);
            ++nr;
          }
        }
      }
    }
    if (wide) {  // a row too long (or a list too large) for the packed table
      np = PCAP + 1;
      nr = 0;
    }
    if (__any(R.across))
      walk_rows<true>(crs, rtab, c_idx, t, nr, pfx, pfy, pfz, rif, reach, perx, pery, Lx, Ly, np);
    else
      walk_rows<false>(crs, rtab, c_idx, t, nr, pfx, pfy, pfz, rif, reach, perx, pery, Lx, Ly, np);
  }
  const bool exact = np > PCAP;
  if (exact) {
    // more kept candidates than the list holds: exact walk from the FP64
    // records into K rows (a dense cluster; the capacity check below still
    // applies)
    c_idx = lds + (LROWS - K);
    np = 0;
    for (int lev = lev_i; lev < bc.nlev; ++lev) {
      const int gl = bc.lev0 + lev;
      const LevelGrid G = d.levels[gl];
      if (lev > lev_i && !level_in_reach(d, gl, pi, pi.w + G.rmax + skin)) continue;
      RowSet R;
      row_set(G, pi, pi.w + G.rmax + skin, R);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (p >= R.nxp) break;
        uint32_t q0[9], q1[9];
        row_piece(d.cell_start, G, R, p, q0, q1);
        for (int r = 0; r < 9; ++r)
          for (uint32_t q = q0[r]; q < q1[r]; ++q)
            if (owner_candidate(bc, pi, si, skin, d.crec[q])) {
              if (np < K) c_idx[np][t] = (int32_t)q;
              ++np;
            }
      }
    }
  }
  // the previous lists' partners, read alongside the exact pass
  int32_t old_j[K];
#pragma unroll
  for (int k2 = 0; k2 < K; ++k2) old_j[k2] = (k2 < cnt_old) ? d.own_idx[lo][k2 * N + io] : -1;
  // exact pass over the kept candidates, reads four at a time; accepted ones
  // are compacted in place
  int cnt = 0;
  const int nk = min(np, exact ? K : PCAP);
  for (int a = 0; a < nk; a += 4) {
    CRec c[4];
    int32_t qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qv[u] = c_idx[(a + u < nk) ? a + u : a][t];
      c[u] = d.crec[qv[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (a + u < nk && owner_candidate(bc, pi, si, skin, c[u])) {
        if (cnt < K) {
          c_idx[cnt][t] = qv[u];
          c_sid[cnt][t] = c[u].sid;
        }
        ++cnt;
      }
  }
  if (exact && np > K) cnt = max(cnt, K + 1);  // more partners than slots
  if (cnt > K) {
    atomicOr(d.err, ERR_CAPACITY);
    cnt = K;
  }
  // canonical slot order: ascending partner stable id
  for (int a = 1; a < cnt; ++a) {
    const int32_t ks = c_sid[a][t], kj = c_idx[a][t];
    int b = a - 1;
    while (b >= 0 && c_sid[b][t] > ks) {
      c_sid[b + 1][t] = c_sid[b][t];
      c_idx[b + 1][t] = c_idx[b][t];
      --b;
    }
    c_sid[b + 1][t] = ks;
    c_idx[b + 1][t] = kj;
  }
  // slots four at a time, with every read and atomic of a group in flight
  // together: storage index of the partner, its reverse-list rank and the
  // slot it held in the previous lists.  A slot whose pair was not in contact
  // holds zero history, so readers need not consult the contact flags.
  uint32_t fn = fo & 0xffff0000u;
  for (int k0 = 0; k0 < cnt; k0 += 4) {
    int32_t jj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) jj[u] = (k0 + u < cnt) ? d.cell_list[c_idx[k0 + u][t]] : -2;
    uint32_t rk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) rk[u] = (k0 + u < cnt) ? atomicAdd(&d.rev_cnt[jj[u]], 1u) : 0u;
    int32_t jo[4];  // the partner's index in the previous lists
#pragma unroll
    for (int u = 0; u < 4; ++u) jo[u] = (moved && k0 + u < cnt) ? src[jj[u]] : jj[u];
    int mk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      mk[u] = -1;
#pragma unroll
      for (int k2 = K - 1; k2 >= 0; --k2)
        if (old_j[k2] == jo[u]) mk[u] = k2;
      if (k0 + u < cnt && mk[u] >= 0 && ((fo >> mk[u]) & 1u)) fn |= 1u << (k0 + u);
    }
    if (moved) {
      // new storage order: the lists and springs move to the other buffers
      HRec hr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        hr[u].t = make_float4(0.f, 0.f, 0.f, 0.f);
        hr[u].r = make_float4(0.f, 0.f, 0.f, 0.f);
        if (mk[u] >= 0 && ((fo >> mk[u]) & 1u)) hr[u] = d.hist[ho][(int64_t)mk[u] * N + io];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k0 + u < cnt) {
          const int64_t o = (int64_t)(k0 + u) * N + i;
          d.own_idx[ln][o] = jj[u];
          d.own_rank[o] = rk[u];
          d.hist[hn][o] = hr[u];
        }
    } else {
      // same storage order: the lists are rewritten in place where a slot
      // changed, and the previous slot of each is kept for the springs
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k0 + u < cnt) {
          const int64_t o = (int64_t)(k0 + u) * N + i;
          if (mk[u] != k0 + u) d.own_idx[ln][o] = jj[u];
          d.own_rank[o] = rk[u];
          c_sid[k0 + u][t] = mk[u];
        }
    }
  }
  if (!moved) {
    // springs in place: slot k takes the spring of its previous slot m (or
    // zero).  Both lists ascend in partner id, so m grows with k: copies to
    // a lower slot, taken in ascending order, and copies to a higher slot,
    // in descending order, never read a slot already written, and zeros go
    // last.  An unchanged slot (m == k) is not touched, nor is a slot that
    // already holds zero (a previous slot out of contact).
    HRec* const H = d.hist[ho];
    for (int k = 0; k < cnt; ++k) {
      const int m = c_sid[k][t];
      if (m > k && ((fo >> m) & 1u)) H[(int64_t)k * N + i] = H[(int64_t)m * N + i];
    }
    for (int k = cnt - 1; k >= 0; --k) {
      const int m = c_sid[k][t];
      if (m >= 0 && m < k && ((fo >> m) & 1u)) H[(int64_t)k * N + i] = H[(int64_t)m * N + i];
    }
    for (int k = 0; k < cnt; ++k) {
      const int m = c_sid[k][t];
      const bool live = m >= 0 && ((fo >> m) & 1u);
      const bool zero_now = k < cnt_old && !((fo >> k) & 1u);
      if (m != k && !live && !zero_now) {
        HRec z;
        z.t = make_float4(0.f, 0.f, 0.f, 0.f);
        z.r = make_float4(0.f, 0.f, 0.f, 0.f);
        H[(int64_t)k * N + i] = z;
      }
    }
  } else {
    for (int w = 0; w < bc.nwall; ++w)
      if ((fo >> (WALL_BIT + w)) & 1u) {
        d.wA[hn][w * N + i] = d.wA[ho][w * N + io];
        d.wB[hn][w * N + i] = d.wB[ho][w * N + io];
      }
  }
  d.own_cnt[ln][i] = cnt;
  d.cflag[hn][i] = fn;
  d.disp[i] = 0.f;
  // largest owner count seen: an atomic only when this count raises it
  if ((uint32_t)cnt > *(const volatile uint32_t*)&d.stat[0]) atomicMax(&d.stat[0], (uint32_t)cnt);
}

void launch_search(const DevBufs& d, int s, int lo, int ho, const int32_t* src, hipStream_t st) {
  const int64_t g = (d.N + SBS - 1) / SBS;
  hipLaunchKernelGGL(k_search, dim3((unsigned)((g + 7) / 8 * 8)), dim3(SBS), 0, st, d, s, lo, ho, src);
}

__global__ void k_rev_scatter(DevBufs d, int l) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d.N || latched(d.err)) return;
  const int cnt = d.own_cnt[l][i];
  // each entry is written with its sort key (the owner's stable id) in the
  // high word, one 8-byte write, so that the sort that follows reads no ids
  const uint64_t key = (uint64_t)(uint32_t)d.sid[i] << 32;
  // slots four at a time, their reads in flight together
  for (int k0 = 0; k0 < cnt; k0 += 4) {
    int32_t j[4];
    uint32_t rk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      j[u] = (k0 + u < cnt) ? d.own_idx[l][(int64_t)(k0 + u) * d.N + i] : 0;
      rk[u] = (k0 + u < cnt) ? d.own_rank[(int64_t)(k0 + u) * d.N + i] : 0u;
    }
    uint32_t at[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) at[u] = (k0 + u < cnt) ? d.rev_start[j[u]] + rk[u] : 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u < cnt) d.rev_tmp[at[u]] = key | (((uint32_t)i << 4) | (uint32_t)(k0 + u));
  }
}

void launch_rev_scatter(const DevBufs& d, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_rev_scatter, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, d, l);
}

// Partner-side entries of a particle in ascending stable id of the owner, so
// that the order in which its forces are summed does not depend on the
// storage order (and so on the cell layout); an owner holds a given partner
// in one slot at most, so the keys are distinct.  The scatter left each
// entry beside its key (key << 32 | entry); the sorted entries are written
// to the list the step reads.
__global__ void k_rev_sort(DevBufs d) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= d.N || latched(d.err)) return;
  const uint32_t a = d.rev_start[j], b = d.rev_start[j + 1];
  if (b - a <= 8u) {
    // short lists (nearly all): sorted in registers by an odd-even
    // transposition network (the key decides, being in the high word)
    uint64_t e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = (a + u < b) ? d.rev_tmp[a + u] : ~0ull;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int u = r & 1; u + 1 < 8; u += 2)
        if (e[u + 1] < e[u]) {
          const uint64_t te = e[u];
          e[u] = e[u + 1];
          e[u + 1] = te;
        }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (a + u < b) d.rev_ent[a + u] = (uint32_t)e[u];
    return;
  }
  // long lists: insertion sort in place over the keyed entries, then copied
  for (uint32_t q = a + 1; q < b; ++q) {
    const uint64_t e = d.rev_tmp[q];
    uint32_t p = q;
    while (p > a) {
      const uint64_t prev = d.rev_tmp[p - 1];
      if (prev <= e) break;
      d.rev_tmp[p] = prev;
      --p;
    }
    d.rev_tmp[p] = e;
  }
  for (uint32_t q = a; q < b; ++q) d.rev_ent[q] = (uint32_t)d.rev_tmp[q];
}

void launch_rev_sort(const DevBufs& d, hipStream_t st) {
  hipLaunchKernelGGL(k_rev_sort, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, d);
}

// ---------------------------------------------------------------------------
// the fused step

LPR_DEV_INLINE double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One work block of the fused step (all threads of the launch block).
template <int BS>
__device__ __forceinline__ void step_block(const DevBufs& d, const StepPar& p, int record, int64_t blk) {
  __shared__ double red[BS / 64][6];
  if (__syncthreads_or(latched(d.err) ? 1 : 0)) return;  // uniform per block
  const int64_t N = d.N;
  const int64_t i = blk * BS + threadIdx.x;
  const int bed = d.chunk_bed32[(blk * BS) >> 8];
  const BedConst bc = d.beds[bed];
  if (bc.skin > 0.f) {
    // candidate lists with a skin are complete only while every particle
    // has moved less than skin/2 since they were built; otherwise stop
    // before using them (the host rebuilds and repeats the step).  The flag
    // read here was raised by the previous step (flags alternate with the
    // state parity, so this step's own raises go to the other flag).
    if (*(const volatile uint32_t*)&d.viol[p.s] != 0u) {
      if (threadIdx.x == 0) atomicOr(d.err, ERR_SKIN);
      return;
    }
  }
  const uint32_t m = d.meta[i];
  const bool active = (m != INACTIVE);
  const int s = p.s, sn = p.s ^ 1, h = p.h, hn = p.h ^ 1, l = p.l;

  // the block's own states in LDS: storage follows the cell order, so most
  // partners lie in the same block and are read from here
  __shared__ PState sst[BS];
  const int64_t b0 = blk * BS;
  const PState me = d.st[s][i];
  sst[threadIdx.x] = me;
  __syncthreads();
  auto state_of = [&](int64_t j) -> PState {
    PState o;
    if ((uint64_t)(j - b0) < (uint64_t)BS)
      o = sst[j - b0];
    else
      o = d.st[s][j];
    return o;
  };

  double4 xi = make_double4(0, 0, 0, 0);
  float4 vi = make_float4(0, 0, 0, 0), wi = make_float4(0, 0, 0, 0);
  float3 F = f3(0.f, 0.f, 0.f), T = f3(0.f, 0.f, 0.f);
  uint32_t fnew = 0u;
  if (active) {
    xi = me.x;
    vi = me.v;
    wi = me.w;
    const int n_own = d.own_cnt[l][i];
    const uint32_t rs = d.rev_start[i];
    const int n_tot = n_own + (int)(d.rev_start[i + 1] - rs);
    // contact e + 1's partner state and history are read while contact e is
    // evaluated
    int64_t o_n = 0, oth_n = 0;
    int k_n = 0;
    PState ot_n{};
    HRec hr_n{};
    // the first PRE slot partners and partner-side entries are read together
    // before the loop (most particles have no more), so that a contact's
    // partner state is requested without first waiting for its index
    constexpr int PRE = 8;
    const int n_rev = n_tot - n_own;
    int32_t pre_o[PRE];
    uint32_t pre_r[PRE];
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      pre_o[u] = (u < n_own) ? d.own_idx[l][(int64_t)u * N + i] : 0;
      pre_r[u] = (u < n_rev) ? d.rev_ent[rs + u] : 0u;
    }
    auto own_at = [&](int k2) -> int64_t {
      int32_t v = 0;
      bool hit = false;
#pragma unroll
      for (int u = 0; u < PRE; ++u)
        if (k2 == u) { v = pre_o[u]; hit = true; }
      return hit ? (int64_t)v : (int64_t)d.own_idx[l][(int64_t)k2 * N + i];
    };
    auto rev_at = [&](int q) -> uint32_t {
      uint32_t v = 0u;
      bool hit = false;
#pragma unroll
      for (int u = 0; u < PRE; ++u)
        if (q == u) { v = pre_r[u]; hit = true; }
      return hit ? v : d.rev_ent[rs + q];
    };
    if (n_tot > 0) {
      if (n_own > 0) {
        k_n = 0;
        o_n = i;
        oth_n = own_at(0);
      } else {
        const uint32_t pk = rev_at(0);
        o_n = pk >> 4;
        k_n = (int)(pk & 15u);
        oth_n = o_n;
      }
      ot_n = state_of(oth_n);
      hr_n = d.hist[h][k_n * N + o_n];
    }
    // not unrolled or peeled: one copy of the law evaluates both sides of
    // every pair, so their forces are exactly opposite
#pragma clang loop unroll(disable)
    for (int e = 0; e < n_tot; ++e) {
      const int64_t o = o_n;
      const int k = k_n;
      const PState ot = ot_n;
      const HRec hr_pf = hr_n;
      const bool mine = e < n_own;
      if (e + 1 < n_tot) {
        if (e + 1 < n_own) {
          k_n = e + 1;
          o_n = i;
          oth_n = own_at(k_n);
        } else {
          const uint32_t pk = rev_at(e + 1 - n_own);
          o_n = pk >> 4;
          k_n = (int)(pk & 15u);
          oth_n = o_n;
        }
        ot_n = state_of(oth_n);
        hr_n = d.hist[h][k_n * N + o_n];
      }
      const double4 xo_ = ot.x;
      const float4 vo_ = ot.v;
      const float4 wo_ = ot.w;
      const double4 xa = mine ? xi : xo_, xb = mine ? xo_ : xi;   // owner a, partner b
      const float4 va = mine ? vi : vo_, vb = mine ? vo_ : vi;
      const float4 wa = mine ? wi : wo_, wb = mine ? wo_ : wi;
      double dx, dy, dz;
      const double d2 = pair_sep(bc, xa, xb, dx, dy, dz);
      if (!sphere_touch(d2, xa.w, xb.w)) {
        if (mine) {  // out of contact: the slot keeps no history
          HRec z;
          z.t = make_float4(0.f, 0.f, 0.f, 0.f);
          z.r = make_float4(0.f, 0.f, 0.f, 0.f);
          d.hist[hn][k * N + i] = z;
        }
        continue;
      }
      // slots out of contact hold zeros, so the history is read as it is
      LawIn in;
      {
        const HRec hr = hr_pf;
        in.xt = f3(hr.t.x, hr.t.y, hr.t.z);
        in.xr = f3(hr.r.x, hr.r.y, hr.r.z);
      }
      // overlap in FP64 (it is a small difference of large numbers); the
      // unit normal only needs FP32
      const double dist = sqrt(d2);
      const double dl = (xa.w + xb.w) - dist;
      const float ra = (float)xa.w, rb = (float)xb.w;
      in.delta = (float)dl;
      if (d2 > 0.0) {
        const float id = 1.0f / (float)dist;
        in.n = f3((float)dx * id, (float)dy * id, (float)dz * id);
      } else {
        in.n = f3(0.f, 0.f, 1.f);
      }
      const float la = ra - 0.5f * in.delta, lb = rb - 0.5f * in.delta;   // lever arms
      const float3 wa3 = f3(wa.x, wa.y, wa.z), wb3 = f3(wb.x, wb.y, wb.z);
      in.u = f3(va.x - vb.x, va.y - vb.y, va.z - vb.z) + la * cross(wa3, in.n) + lb * cross(wb3, in.n);
      in.wrel = wa3 - wb3;
      in.dstar = 2.0f * ra * rb / (ra + rb);
      in.mu_t = bc.mu_t;
      in.mu_r = bc.mu_r;
      LawOut out;
      contact_law(bc, in, out);
      const float3 nft = cross(in.n, out.Ft);
      if (mine) {
        F = F + out.F;
        T = T + (la * nft + out.M);
        HRec hr;
        hr.t = make_float4(out.xt.x, out.xt.y, out.xt.z, 0.f);
        hr.r = make_float4(out.xr.x, out.xr.y, out.xr.z, 0.f);
        d.hist[hn][k * N + i] = hr;
        fnew |= 1u << k;
        if (record) {
          d.cF[k * N + i] = make_float4(out.F.x, out.F.y, out.F.z, out.Fn);
          d.cM[k * N + i] = make_float4(out.M.x, out.M.y, out.M.z, 0.f);
        }
      } else {
        F = F - out.F;
        T = T + (lb * nft - out.M);
      }
    }
  }

  // walls, body by body, with an ordered FP64 block reduction per body
  for (int b = 0; b < bc.nbody; ++b) {
    double r6[6] = {0, 0, 0, 0, 0, 0};
    int hit = 0;
    if (active) {
      const uint32_t fold = d.cflag[h][i];
      for (int w = 0; w < bc.nwall; ++w) {
        const WallPose& W = d.walls[bc.wall0 + w];
        if (W.body != b) continue;
        double dl, nx, ny, nz;
        if (!wall_geom(W, xi.x, xi.y, xi.z, xi.w, dl, nx, ny, nz)) continue;
        // a sphere wholly through a plane has tunnelled: a failed run
        if (W.kind == WPLANE && dl > 2.0 * xi.w) atomicOr(d.err, ERR_WALL);
        hit = 1;
        LawIn in;
        if ((fold >> (WALL_BIT + w)) & 1u) {
          const float4 a4 = d.wA[h][w * N + i];
          const float2 b2 = d.wB[h][w * N + i];
          in.xt = f3(a4.x, a4.y, a4.z);
          in.xr = f3(a4.w, b2.x, b2.y);
        } else {
          in.xt = f3(0.f, 0.f, 0.f);
          in.xr = f3(0.f, 0.f, 0.f);
        }
        const float ra = (float)xi.w;
        in.delta = (float)dl;
        in.n = f3((float)nx, (float)ny, (float)nz);
        const float la = ra - 0.5f * in.delta;
        // contact point (FP64) and wall velocity there
        const double px = xi.x + (double)la * nx, py = xi.y + (double)la * ny, pz = xi.z + (double)la * nz;
        const double rx = px - W.c[0], ry = py - W.c[1], rz = pz - W.c[2];
        const float3 uw = f3((float)(W.vel[0] - W.omega * ry), (float)(W.vel[1] + W.omega * rx), (float)W.vel[2]);
        const float3 wa3 = f3(wi.x, wi.y, wi.z);
        in.u = f3(vi.x, vi.y, vi.z) + la * cross(wa3, in.n) - uw;
        in.wrel = f3(wi.x, wi.y, wi.z - (float)W.omega);
        in.dstar = 2.0f * ra;
        in.mu_t = (W.mu_t < 0.f) ? bc.mu_t : W.mu_t;
        in.mu_r = (W.mu_r < 0.f) ? bc.mu_r : W.mu_r;
        LawOut out;
        contact_law(bc, in, out);
        F = F + out.F;
        T = T + (la * cross(in.n, out.Ft) + out.M);
        d.wA[hn][w * N + i] = make_float4(out.xt.x, out.xt.y, out.xt.z, out.xr.x);
        d.wB[hn][w * N + i] = make_float2(out.xr.y, out.xr.z);
        fnew |= 1u << (WALL_BIT + w);
        if (record) {
          d.wF[w * N + i] = make_float4(out.F.x, out.F.y, out.F.z, out.Fn);
          d.wM[w * N + i] = make_float4(out.M.x, out.M.y, out.M.z, 0.f);
        }
        // reaction on the body: -F at p, and -M
        const double fx = -(double)out.F.x, fy = -(double)out.F.y, fz = -(double)out.F.z;
        r6[0] += fx; r6[1] += fy; r6[2] += fz;
        r6[3] += (ry * fz - rz * fy) - (double)out.M.x;
        r6[4] += (rz * fx - rx * fz) - (double)out.M.y;
        r6[5] += (rx * fy - ry * fx) - (double)out.M.z;
      }
    }
    // partial sums are component-major: [bed body][component][block]
    double* part = d.partial + (int64_t)(bc.body0 + b) * 6 * d.nblk + blk;
    if (__syncthreads_or(hit)) {
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      for (int c = 0; c < 6; ++c) {
        const double sum = wave_sum(r6[c]);
        if (lane == 0) red[wv][c] = sum;
      }
      __syncthreads();
      if (threadIdx.x < 6) {
        double acc = 0.0;
        for (int q = 0; q < BS / 64; ++q) acc += red[q][threadIdx.x];
        part[(int64_t)threadIdx.x * d.nblk] = acc;
      }
      __syncthreads();
    } else if (threadIdx.x < 6) {
      part[(int64_t)threadIdx.x * d.nblk] = 0.0;
    }
  }
  if (!active) return;
  d.cflag[hn][i] = fnew;
  if (record) {
    d.frc[i] = make_float4(F.x, F.y, F.z, 0.f);
    d.trq[i] = make_float4(T.x, T.y, T.z, 0.f);
  }
  // semi-implicit Euler: velocity first, then position with the new velocity
  const float vx = vi.x + bc.dt * (F.x * vi.w + bc.g[0]);
  const float vy = vi.y + bc.dt * (F.y * vi.w + bc.g[1]);
  const float vz = vi.z + bc.dt * (F.z * vi.w + bc.g[2]);
  const float ox = wi.x + bc.dt * (T.x * wi.w);
  const float oy = wi.y + bc.dt * (T.y * wi.w);
  const float oz = wi.z + bc.dt * (T.z * wi.w);
  double x = xi.x + bc.dt_d * (double)vx;
  double y = xi.y + bc.dt_d * (double)vy;
  const double z = xi.z + bc.dt_d * (double)vz;
  if (bc.periodic & 1u) {
    if (x >= bc.L[0]) x -= bc.L[0];
    else if (x < 0.0) x += bc.L[0];
  }
  if (bc.periodic & 2u) {
    if (y >= bc.L[1]) y -= bc.L[1];
    else if (y < 0.0) y += bc.L[1];
  }
  if (!(isfinite(vx) && isfinite(vy) && isfinite(vz) && isfinite(ox) && isfinite(oy) && isfinite(oz) &&
        isfinite(x) && isfinite(y) && isfinite(z)))
    atomicOr(d.err, ERR_NUMERIC);
  if (bc.skin > 0.f) {
    // bound on the distance moved since the lists were built: |dx| = dt |v|
    const float moved = d.disp[i] + bc.dt * sqrtf(vx * vx + vy * vy + vz * vz);
    d.disp[i] = moved;
    if (moved > 0.45f * bc.skin) atomicOr(&d.viol[sn], 1u);
  }
  PState out;
  out.x = make_double4(x, y, z, xi.w);
  out.v = make_float4(vx, vy, vz, vi.w);
  out.w = make_float4(ox, oy, oz, wi.w);
  d.st[sn][i] = out;
}

// One launch block per work block, XCD-aware placement.
template <int BS>
__global__ __launch_bounds__(BS) void k_step(DevBufs d, StepPar p, int record) {
  const int64_t g = d.N / BS;
  const int64_t blk = xcd_block(blockIdx.x, g);
  if (blk < 0) return;  // whole launch block idle (grid rounded up to 8)
  step_block<BS>(d, p, record, blk);
}

// Persistent form: a grid that fills the GPU once; each launch block walks
// the work blocks of its XCD's contiguous range with a fixed stride, so the
// assignment (and every result) is deterministic.
template <int BS>
__global__ __launch_bounds__(BS) void k_step_persist(DevBufs d, StepPar p, int record) {
  const int64_t g = d.N / BS;
  const int64_t chunk = (g + 7) / 8;
  const int64_t x = blockIdx.x & 7, lanes = gridDim.x >> 3;  // launch blocks per XCD
  const int64_t end = (x + 1) * chunk < g ? (x + 1) * chunk : g;
  for (int64_t blk = x * chunk + (blockIdx.x >> 3); blk < end; blk += lanes) step_block<BS>(d, p, record, blk);
}

template <int BS>
void launch_step_t(const DevBufs& d, const StepPar& p, int record, int persist_blocks, hipStream_t st) {
  const int64_t g = d.N / BS;
  if (persist_blocks > 0) {
    const int64_t grid = ((int64_t)persist_blocks + 7) / 8 * 8;
    hipLaunchKernelGGL(k_step_persist<BS>, dim3((unsigned)grid), dim3(BS), 0, st, d, p, record);
  } else {
    const int64_t grid = (g + 7) / 8 * 8;
    hipLaunchKernelGGL(k_step<BS>, dim3((unsigned)grid), dim3(BS), 0, st, d, p, record);
  }
}

void launch_step(const DevBufs& d, const StepPar& p, int block, int record, int persist_blocks, hipStream_t st) {
  if (block == 64) launch_step_t<64>(d, p, record, persist_blocks, st);
  else if (block == 128) launch_step_t<128>(d, p, record, persist_blocks, st);
  else launch_step_t<256>(d, p, record, persist_blocks, st);
}

int step_occupancy(int block) {
  int n = 0;
  hipError_t e;
  if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_persist<64>, 64, 0);
  else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_persist<128>, 128, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_persist<256>, 256, 0);
  return e == hipSuccess ? n : 0;
}

// ---------------------------------------------------------------------------
// body reduction, dynamic bodies, wall poses, clock

LPR_DEV_INLINE void rot_z(const double* a, double c, double s, double* o) {
#pragma clang fp contract(off)
  o[0] = a[0] * c - a[1] * s;
  o[1] = a[0] * s + a[1] * c;
  o[2] = a[2];
}

LPR_DEV_INLINE void make_pose(const WallDef& W, const BodyDef& B, const BodyDyn& D, double t, WallPose& P) {
#pragma clang fp contract(off)
  double c[3] = {B.origin[0] + B.lin_vel[0] * t, B.origin[1] + B.lin_vel[1] * t, B.origin[2] + B.lin_vel[2] * t};
  double v[3] = {B.lin_vel[0], B.lin_vel[1], B.lin_vel[2]};
  if (B.z_free) {
    c[2] = D.z;
    v[2] = D.vz;
  }
  const double th = B.ang_vel * t;
  const double cs = cos(th), sn = sin(th);
  double ro[3];
  rot_z(W.origin, cs, sn, ro);
  P.o[0] = c[0] + ro[0]; P.o[1] = c[1] + ro[1]; P.o[2] = c[2] + ro[2];
  rot_z(W.axis, cs, sn, P.nu);
  for (int a = 0; a < 3; ++a) rot_z(&W.frame[3 * a], cs, sn, P.e[a]);
  for (int a = 0; a < 3; ++a) {
    P.dims[a] = W.dims[a];
    P.c[a] = c[a];
    P.vel[a] = v[a];
  }
  P.omega = B.ang_vel;
  P.mu_t = (float)W.mu_t;
  P.mu_r = (float)W.mu_r;
  P.kind = W.kind;
  P.body = W.body;
}

// Ordered reduction of the reaction partials in two levels: ADV_CH blocks
// per bed each sum one contiguous chunk of the block partials (a fixed
// order: strided per thread, a shuffle tree per wave, waves ascending) and
// store the chunk's sums; the block that finishes last (a counter per bed)
// adds the chunk sums in chunk order, advances the bed's bodies and poses
// and clears the counter.  Every sum has the same terms in the same order
// whatever the timing.
constexpr int ADV_BS = 256;

__global__ __launch_bounds__(ADV_BS) void k_advance(DevBufs d, int step_block) {
  __shared__ double red[ADV_BS / 64][6];
  __shared__ double tot_s[MAXB][6];
  __shared__ int last_s;
  if (__syncthreads_or(latched(d.err) ? 1 : 0)) return;  // uniform over the launch
  const int bed = blockIdx.x / ADV_CH, ch = blockIdx.x % ADV_CH;
  const BedConst bc = d.beds[bed];
  const int64_t blk0 = bc.p0 / step_block, blk1 = bc.p1 / step_block;
  const int64_t len = (blk1 - blk0 + ADV_CH - 1) / ADV_CH;
  const int64_t c0 = blk0 + ch * len, c1 = (c0 + len < blk1) ? c0 + len : blk1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int b = 0; b < bc.nbody; ++b) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double* part = d.partial + (int64_t)(bc.body0 + b) * 6 * d.nblk;
    for (int64_t q0 = c0 + threadIdx.x; q0 < c1; q0 += 2 * ADV_BS) {
      double v[2][6];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t q = q0 + (int64_t)u * ADV_BS;
#pragma unroll
        for (int c = 0; c < 6; ++c) v[u][c] = (q < c1) ? part[(int64_t)c * d.nblk + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += v[u][c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double sw = wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = sw;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      double sc = 0.0;
      for (int q = 0; q < ADV_BS / 64; ++q) sc += red[q][threadIdx.x];
      d.adv_chunk[(((int64_t)bed * MAXB + b) * ADV_CH + ch) * 6 + threadIdx.x] = sc;
    }
    __syncthreads();
  }
  // the chunk sums are visible to every XCD before the count is raised
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last_s = (atomicAdd(&d.adv_cnt[bed], 1u) == (uint32_t)(ADV_CH - 1)) ? 1 : 0;
  __syncthreads();
  if (!last_s) return;
  __threadfence();
  if (threadIdx.x < 6 * bc.nbody) {
    const int b = threadIdx.x / 6, c = threadIdx.x % 6;
    const double* cs = d.adv_chunk + ((int64_t)bed * MAXB + b) * ADV_CH * 6;
    double sc = 0.0;
    for (int q = 0; q < ADV_CH; ++q) sc += __hip_atomic_load(&cs[q * 6 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tot_s[b][c] = sc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int b = 0; b < bc.nbody; ++b) {
      BodyDyn& D = d.bdyn[bc.body0 + b];
      const BodyDef& B = d.bdefs[bc.body0 + b];
      for (int c = 0; c < 6; ++c) {
        D.last[c] = tot_s[b][c];
        D.wsum[c] += tot_s[b][c];
      }
      D.wsteps += 1;
      if (B.z_free) {
        D.vz = D.vz + bc.dt_d * (tot_s[b][2] / B.mass + (double)bc.g[2]);
        D.z = D.z + bc.dt_d * D.vz;
      }
    }
    d.adv_cnt[bed] = 0u;
  }
  __syncthreads();
  // poses for the next step
  const int64_t k_next = d.bedyn[bed].k + 1;
  const double t = (double)k_next * bc.dt_d;
  for (int w = threadIdx.x; w < bc.nwall; w += ADV_BS) {
    const WallDef& W = d.wdefs[bc.wall0 + w];
    make_pose(W, d.bdefs[bc.body0 + W.body], d.bdyn[bc.body0 + W.body], t, d.walls[bc.wall0 + w]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d.bedyn[bed].k = k_next;
    d.bedyn[bed].completed += 1;
  }
}

void launch_advance(const DevBufs& d, int step_block, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3((unsigned)(d.nbeds * ADV_CH)), dim3(ADV_BS), 0, st, d, step_block);
}

__global__ void k_poses(DevBufs d) {
  const int bed = blockIdx.x;
  const BedConst bc = d.beds[bed];
  const double t = (double)d.bedyn[bed].k * bc.dt_d;
  for (int w = threadIdx.x; w < bc.nwall; w += blockDim.x) {
    const WallDef& W = d.wdefs[bc.wall0 + w];
    make_pose(W, d.bdefs[bc.body0 + W.body], d.bdyn[bc.body0 + W.body], t, d.walls[bc.wall0 + w]);
  }
}

void launch_poses(const DevBufs& d, hipStream_t st) {
  hipLaunchKernelGGL(k_poses, dim3((unsigned)d.nbeds), dim3(64), 0, st, d);
}

// ---------------------------------------------------------------------------
// per-contact loads of the last step, compacted on the device

LPR_DEV_INLINE uint32_t contact_bits(const DevBufs& d, int l, int h, int64_t i, int nwall) {
  const uint32_t fl = d.cflag[h][i];
  const int own = d.own_cnt[l][i];
  const uint32_t slots = fl & ((1u << own) - 1u) & 0xffffu;
  const uint32_t walls = (fl >> WALL_BIT) & ((1u << nwall) - 1u);
  return slots | (walls << WALL_BIT);
}

__global__ void k_load_count(DevBufs d, int l, int h, int64_t p0, int64_t np, int nwall, uint32_t* cnt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int64_t i = p0 + t;
  cnt[t] = (d.sid[i] < 0) ? 0u : (uint32_t)__popc(contact_bits(d, l, h, i, nwall));
}

__global__ void k_load_pack(DevBufs d, int l, int h, int64_t p0, int64_t np, int nwall, const uint32_t* off,
                            lpr_contact_load* out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int64_t i = p0 + t, N = d.N;
  const int32_t a = d.sid[i];
  if (a < 0) return;
  uint32_t q = off[t];
  const uint32_t bits = contact_bits(d, l, h, i, nwall);
  for (int k = 0; k < K; ++k) {
    if (!((bits >> k) & 1u)) continue;
    const int32_t b = d.sid[d.own_idx[l][(int64_t)k * N + i]];
    const float4 F = d.cF[(int64_t)k * N + i], M = d.cM[(int64_t)k * N + i];
    // loads are kept for the owner; a pair is reported on its smaller id
    const float sg = (a < b) ? 1.f : -1.f;
    lpr_contact_load r;
    r.a = (a < b) ? a : b;
    r.b = (a < b) ? b : a;
    r.force[0] = sg * F.x; r.force[1] = sg * F.y; r.force[2] = sg * F.z;
    r.moment[0] = sg * M.x; r.moment[1] = sg * M.y; r.moment[2] = sg * M.z;
    r.fn = F.w;
    r.reserved = 0.f;
    out[q++] = r;
  }
  for (int w = 0; w < nwall; ++w) {
    if (!((bits >> (WALL_BIT + w)) & 1u)) continue;
    const float4 F = d.wF[(int64_t)w * N + i], M = d.wM[(int64_t)w * N + i];
    lpr_contact_load r;
    r.a = a;
    r.b = -1 - (int64_t)w;
    r.force[0] = F.x; r.force[1] = F.y; r.force[2] = F.z;
    r.moment[0] = M.x; r.moment[1] = M.y; r.moment[2] = M.z;
    r.fn = F.w;
    r.reserved = 0.f;
    out[q++] = r;
  }
}

void launch_load_count(const DevBufs& d, int l, int h, int64_t p0, int64_t np, int nwall, uint32_t* cnt,
                       hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_load_count, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, d, l, h, p0, np, nwall, cnt);
}

void launch_load_pack(const DevBufs& d, int l, int h, int64_t p0, int64_t np, int nwall, const uint32_t* off,
                      lpr_contact_load* out, hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_load_pack, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, d, l, h, p0, np, nwall, off,
                     out);
}

}  // namespace lpr
