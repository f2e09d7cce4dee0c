// lpr_cells.h -- cell coordinates and the neighbour rows of a particle at
// one cell-list level (host and device: the kernels' broad phase and a host
// check of its bounds and coverage).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpr_dev.h"

namespace lpr {

#define LPR_HD __host__ __device__ inline

LPR_HD int imin(int a, int b) { return a < b ? a : b; }
LPR_HD int imax(int a, int b) { return a > b ? a : b; }

// Cell of coordinate x along axis a as binning assigns it: the floor of the
// cell coordinate, wrapped on a periodic axis and clamped to the grid.
LPR_HD int cell_axis(const LevelGrid& G, int a, double x) {
#pragma clang fp contract(off)
  double f = (x - G.lo[a]) * G.inv_w[a];
  f = fmin(fmax(f, -1.0), (double)G.n[a]);
  int c = (int)floor(f);
  if (G.per[a]) {
    if (c >= G.n[a]) c -= G.n[a];
    if (c < 0) c += G.n[a];
  }
  c = c < 0 ? 0 : (c >= G.n[a] ? G.n[a] - 1 : c);
  return c;
}

// Cells along axis a that can hold a partner closer than `reach` to the
// coordinate x: the range [c + lo, c + hi] around the particle's cell c, with
// lo, hi in {-1, 0, 1} (a cell is at least `reach` wide, so one neighbour on
// either side is the most that is ever needed).  The bounds come from the
// cell coordinate of x -+ reach with a slack of 1e-9 cell, far above the
// rounding of the cell coordinates, so no cell that holds such a partner is
// dropped.
LPR_HD void axis_span(const LevelGrid& G, int a, double x, double reach, int& c, int& lo, int& hi, float& glo,
                              float& ghi) {
#pragma clang fp contract(off)
  const int n = G.n[a];
  c = cell_axis(G, a, x);
  const double dr = reach * G.inv_w[a] + 1e-9;
  double f, fc;
  if (G.per[a]) {
    // offsets from the cell coordinate as cell_axis clamps it, so they are
    // relative to c
    f = fmin(fmax((x - G.lo[a]) * G.inv_w[a], -1.0), (double)n);
    fc = floor(f);
    lo = (floor(f - dr) < fc) ? -1 : 0;
    hi = (floor(f + dr) > fc) ? 1 : 0;
  } else {
    // binning clamps a cell index to the grid, so the span's ends are
    // clamped the same way (particles beyond an edge sit in the edge cell)
    f = fmin(fmax((x - G.lo[a]) * G.inv_w[a], -1073741824.0), 1073741824.0);
    fc = (double)c;
    const int a0 = imin(imax((int)floor(f - dr), 0), n - 1), b0 = imin(imax((int)floor(f + dr), 0), n - 1);
    lo = imax(a0, c - 1) - c;
    hi = imin(b0, c + 1) - c;
  }
  // distances from the particle to the faces of its cell below and above,
  // less the same slack (zero where it lies outside the cell: a particle
  // beyond a grid edge, whose neighbour cells on the far side are then
  // farther than these bounds say)
  glo = (float)(fmax(f - fc - 1e-9, 0.0) * G.w[a]);
  ghi = (float)(fmax(fc + 1.0 - f - 1e-9, 0.0) * G.w[a]);
}

// The particle's neighbour rows at one level: rows along x of the needed
// (y, z) cells (the cells of a row are consecutive in the cell order), each
// in one piece, or two where the x range wraps.  Short periodic axes (three
// cells or fewer) take every cell once.  Within that box, a row whose (y, z)
// cells lie wholly out of reach is dropped, and so is a row's cell on either
// side in x that lies wholly out of reach: a cell is kept while the nearest
// point of its box is closer than the reach.
struct RowSet {
  int y0, nyl;          // rows y0 .. y0 + nyl - 1 (wrapped on a periodic axis)
  int z0, nzl;          // rows z0 .. z0 + nzl - 1
  int xa0, xb0, xa1, xb1, nxp;  // x pieces [xa, xb)
  int xl, xh;           // x offsets of the box's first and last cell (-1, 0 or 1)
  int wrap;             // 0; 1: piece 1 is the cell at x offset -1; 2: at +1
  uint32_t keep;        // row r: bit 3r row kept, 3r + 1 its x - 1 cell, 3r + 2 its x + 1 cell
  bool across;  // a cell lies across a periodic edge from the particle (only
                // then can a separation need the minimum image)
};

LPR_HD void row_set(const LevelGrid& G, const double4& pi, double reach, RowSet& R) {
  int cx, xl, xh, cy, yl, yh, cz, zl, zh;
  float gxl, gxh, gyl, gyh, gzl, gzh;
  axis_span(G, 0, pi.x, reach, cx, xl, xh, gxl, gxh);
  axis_span(G, 1, pi.y, reach, cy, yl, yh, gyl, gyh);
  axis_span(G, 2, pi.z, reach, cz, zl, zh, gzl, gzh);
  const bool yall = G.per[1] && G.n[1] <= 3;
  if (yall) {
    R.y0 = 0;
    R.nyl = G.n[1];
  } else {
    R.y0 = cy + yl;
    R.nyl = imax(0, yh - yl + 1);
  }
  R.across = G.per[1] && (G.n[1] <= 3 || cy + yl < 0 || cy + yh >= G.n[1]);
  R.z0 = cz + zl;  // z never wraps
  R.nzl = imax(0, zh - zl + 1);
  const int n = G.n[0];
  R.xa0 = R.xb0 = R.xa1 = R.xb1 = 0;
  R.nxp = 0;
  R.wrap = 0;
  R.xl = xl;
  R.xh = xh;
  if (G.per[0] && n <= 3) {
    R.xb0 = n;
    R.nxp = 1;
    R.across = true;
    R.xl = R.xh = 0;  // every cell once, none dropped
  } else if (xh >= xl) {
    const int a0 = cx + xl, b0 = cx + xh + 1;  // [a0, b0), may leave [0, n) on a periodic axis
    if (a0 < 0) {
      R.xa0 = 0; R.xb0 = b0; R.xa1 = a0 + n; R.xb1 = n; R.nxp = 2; R.wrap = 1;
      R.across = true;
    } else if (b0 > n) {
      R.xa0 = a0; R.xb0 = n; R.xa1 = 0; R.xb1 = b0 - n; R.nxp = 2; R.wrap = 2;
      R.across = true;
    } else {
      R.xa0 = a0; R.xb0 = b0; R.nxp = 1;
    }
  }
  // the box tests in FP32: the distances above are FP64 roundings, and a
  // relative margin of 2^-16 on the squared reach, far above their rounding,
  // keeps every test on the side of keeping a cell
  const float R2 = (float)(reach * reach) * (1.0f + 0x1p-16f);
  const float x2l = gxl * gxl, x2h = gxh * gxh;
  uint32_t keep = 0u;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int dz = zl + r / 3, dy = yl + r % 3;
    const float ez = dz < 0 ? gzl : (dz > 0 ? gzh : 0.f);
    const float ey = yall ? 0.f : (dy < 0 ? gyl : (dy > 0 ? gyh : 0.f));
    const float e2 = ey * ey + ez * ez;
    keep |= (e2 < R2 ? 1u : 0u) << (3 * r);
    keep |= (e2 + x2l < R2 ? 1u : 0u) << (3 * r + 1);
    keep |= (e2 + x2h < R2 ? 1u : 0u) << (3 * r + 2);
  }
  R.keep = keep;
}

// Cell-list bounds [q0, q1) of the nine rows of x piece p (empty rows
// [0, 0)).  Every cell id is below 2^31 (checked when the grids are laid
// out), so row offsets are 32-bit.
LPR_HD void row_piece(const uint32_t* __restrict__ cell_start, const LevelGrid& G, const RowSet& R, int p,
                      uint32_t q0[9], uint32_t q1[9]) {
  const uint32_t n0 = (uint32_t)G.n[0], plane = n0 * (uint32_t)G.n[1];
  const uint32_t zb = (uint32_t)G.base + (uint32_t)R.z0 * plane;
  uint32_t yb[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int y = R.y0 + b;
    if (G.per[1]) y = (y < 0) ? y + G.n[1] : (y >= G.n[1] ? y - G.n[1] : y);
    yb[b] = (uint32_t)y * n0;
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int a = r / 3, b = r % 3;
    q0[r] = 0u;
    q1[r] = 0u;
    // the row's x cells on this piece, less those out of reach
    const bool dlo = R.xl < 0 && !((R.keep >> (3 * r + 1)) & 1u);
    const bool dhi = R.xh > 0 && !((R.keep >> (3 * r + 2)) & 1u);
    int xa = p ? R.xa1 : R.xa0, xb = p ? R.xb1 : R.xb0;
    if (p == 0) {
      xa += (dlo && R.wrap != 1) ? 1 : 0;
      xb -= (dhi && R.wrap != 2) ? 1 : 0;
    } else if ((R.wrap == 1 && dlo) || (R.wrap == 2 && dhi)) {
      xb = xa;
    }
    if (a < R.nzl && b < R.nyl && p < R.nxp && ((R.keep >> (3 * r)) & 1u) && xa < xb) {
      const uint32_t rb = zb + (uint32_t)a * plane + yb[b];
      q0[r] = cell_start[rb + (uint32_t)xa];
      q1[r] = cell_start[rb + (uint32_t)xb];
    }
  }
}


}  // namespace lpr
