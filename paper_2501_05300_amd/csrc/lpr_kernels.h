// lpr_kernels.h -- launch wrappers of the stepper's kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpr_dev.h"
#include "lprdem.h"

namespace lpr {

// Device pointers of one stepper instance (one bed or a batch of beds).
struct DevBufs {
  int64_t N;            // padded particle count
  int32_t nbeds;
  int64_t ncells;
  // state
  PState* st[2];
  int32_t* sid;
  uint32_t* meta;
  uint8_t* chunk_bed;   // bed of each PAD-chunk of particles (as int32 below)
  int32_t* chunk_bed32;
  // cells
  uint32_t* cell_cnt;
  uint32_t* cell_start;  // ncells + 1
  int32_t* pcell;
  uint32_t* prank;
  int32_t* cell_list;
  // lists
  int32_t* own_idx[2];   // [K][N]
  int32_t* own_cnt[2];   // [N]
  uint32_t* own_rank;    // [K][N]
  uint32_t* rev_cnt;     // [N]
  uint32_t* rev_start;   // [N+1]
  uint32_t* rev_ent;     // [K*N]
  uint64_t* rev_tmp;     // [K*N] entries with their sort key, between the reverse scatter and sort
  // history
  HRec* hist[2];         // [K][N]
  float4* wA[2];         // [MAXW][N]
  float2* wB[2];
  uint32_t* cflag[2];
  // records
  float4* frc;           // optional
  float4* trq;
  float4* cF;            // optional, [K][N]: per owner slot in contact, force on the owner and F_n
  float4* cM;            // optional, [K][N]: rolling moment on the owner
  float4* wF;            // optional, [nwall_max][N]: the same per wall contact
  float4* wM;
  int32_t nwall_max;
  double* partial;       // [bodies][6][nblk] block partial sums of reactions
  int64_t nblk;          // blocks of the smallest step-kernel block size (N / 64)
  double* adv_chunk;     // [beds][MAXB][ADV_CH][6] chunk sums of the reaction partials
  uint32_t* adv_cnt;     // [beds] chunks summed this step (cleared by the last)
  // scan scratch
  uint32_t* scan_tmp;
  CRec* crec;            // position, radius and stable id in cell-list order (rebuild)
  float4* cpf;           // FP32 (x, y, z, r) in cell-list order (rebuild), CPF_PAD entries past N
  uint32_t* zext;        // [levels][2] highest z and highest -z of the level's centres seen
                         // (order-preserving FP32 bits, 0 = none; monotone)
  // storage-order sort (radix sort of (level, Morton) keys)
  uint32_t* skey[2];     // [N] keys, ping-pong over the passes
  int32_t* sval[2];      // [N] storage indices carried with the keys
  uint32_t* rs_hist;     // [256 * tiles + 1] digit counts per tile, then their scan
  int32_t* src;          // [N] after a sort: previous storage index of each particle
  int32_t sort_bits;     // key bits (keys are < 2^sort_bits)
  int64_t n_active;      // particles of all beds (the sorted ranks that are real)
  float* disp;           // distance bound moved since the last rebuild
  uint32_t* viol;        // [2] skin-exceeded flags, by state parity
  // tables
  BedConst* beds;
  LevelGrid* levels;
  WallDef* wdefs;
  WallPose* walls;
  BodyDef* bdefs;
  BodyDyn* bdyn;
  BedDyn* bedyn;
  uint32_t* err;
  uint32_t* stat;        // [0] max owner count at last rebuild, [1] rebuilds
};

// Adjoint work buffers: per-step records of one checkpoint segment (the
// state, springs and wall poses each step read), the segment's fixed
// candidate lists, the running adjoints and per-particle FP64 parameter
// adjoints.
struct AdjBufs {
  PState* st;            // [steps][N]
  uint32_t* cflag;       // [steps][N]
  HRec* hist;            // [steps][K][N]
  float4* wA;            // [steps][nwall_max][N]
  float2* wB;
  WallPose* walls;       // [steps][nwall_total]
  int32_t nwall_total, nwall_max;
  int32_t* own_cnt;      // lists of the segment
  int32_t* own_idx;
  uint32_t* rev_start;
  uint32_t* rev_ent;
  float4* xb;            // adjoints of position, velocity, angular velocity
  float4* vb;
  float4* wb;
  float4* Fb;            // adjoints of the accumulated force and torque
  float4* Tb;
  float4* hbA[2];        // spring adjoints by owner slot (ping-pong)
  float2* hbB[2];
  float4* wbA[2];        // wall spring adjoints
  float2* wbB[2];
  double* theta;         // [N][3] adjoints of (s_k, mu_t, mu_r)
};

// Parities of one step, known on the host.
struct StepPar {
  int s;     // state buffer read this step
  int h;     // history buffer read by the step kernel
  int l;     // list buffer used by the step kernel
  bool rebuild;
};

void launch_zero(uint32_t* p, int64_t n, uint32_t* q, int64_t m, hipStream_t st);
// sort = 1 also writes each particle's sort key (level base + Morton rank
// of its cell) and storage index.
void launch_bin(const DevBufs& d, int s, int sort, hipStream_t st);
// Stable LSD radix sort of (skey[0], sval[0]) in 8-bit digits; the result is
// in buffer (passes & 1).  Returns the number of passes.
int launch_sort(const DevBufs& d, hipStream_t st);
size_t sort_hist_elems(int64_t n);
// Gathers the particles into sorted order: state s into st_out, stable id,
// metadata, cell and cell rank into the *_out arrays, and src.
void launch_reorder(const DevBufs& d, int s, int buf, PState* st_out, int32_t* sid_out, uint32_t* meta_out,
                    int32_t* pcell_out, uint32_t* prank_out, hipStream_t st);
void launch_scan(uint32_t* in_out_cnt, uint32_t* start, uint32_t* tmp, int64_t n, hipStream_t st);
void launch_scatter(const DevBufs& d, int s, hipStream_t st);
// Owner-side search at state s; reads list/history parity (l_old, h_old) and
// writes (1-l_old, 1-h_old).  src: NULL, or (after a re-sort) the index each
// particle had when the previous lists were built.
void launch_search(const DevBufs& d, int s, int l_old, int h_old, const int32_t* src, hipStream_t st);
void launch_rev_scatter(const DevBufs& d, int l, hipStream_t st);
void launch_rev_sort(const DevBufs& d, hipStream_t st);
// persist_blocks > 0: persistent grid of that many launch blocks.
void launch_step(const DevBufs& d, const StepPar& p, int block, int record, int persist_blocks, hipStream_t st);
int step_occupancy(int block);
void launch_advance(const DevBufs& d, int block, hipStream_t st);
void launch_poses(const DevBufs& d, hipStream_t st);
// Per-contact loads of the last step for the particles [p0, p0 + np) of one
// bed: cnt[t] = contacts of particle p0 + t (owner slots in contact and
// walls), then, with off the exclusive scan of cnt, one record per contact
// at out[off[t] ...] in slot order, walls last (not yet in canonical order).
void launch_load_count(const DevBufs& d, int l, int h, int64_t p0, int64_t np, int nwall, uint32_t* cnt,
                       hipStream_t st);
void launch_load_pack(const DevBufs& d, int l, int h, int64_t p0, int64_t np, int nwall, const uint32_t* off,
                      lpr_contact_load* out, hipStream_t st);
size_t scan_tmp_elems(int64_t n);
void launch_adj_pre(const DevBufs& d, const AdjBufs& a, int q, hipStream_t st);
void launch_adj_step(const DevBufs& d, const AdjBufs& a, int q, int hp, int obj_body, float invT, hipStream_t st);
void launch_adj_remap(const DevBufs& d, const AdjBufs& a, const int32_t* old_cnt, const int32_t* old_idx,
                      const uint32_t* old_flag, int hp, hipStream_t st);
void launch_adj_theta(const DevBufs& d, const AdjBufs& a, double* out3, hipStream_t st);

}  // namespace lpr
