// Host check of the broad phase's neighbour rows (lpr_cells.h, host-and-device
// functions).  Random level grids -- periodic and bounded axes, short
// periodic axes of one to three cells, particles inside and beyond the grid
// -- are binned the way the kernels bin them, cell lists are built by a
// counting sort, and for random query points and reaches up to one cell
// width the rows of both x pieces are checked against brute force:
//   every read of the cell ranges stays inside the level's cells (the
//   ranges sit between poisoned guards),
//   no cell-list position is covered twice,
//   every particle closer than the reach (minimum image on periodic axes)
//   is covered.
// Then, with one entry per cell, for points inside the grid: the covered
// cells are exactly those whose box lies closer than the reach (up to the
// margins of the FP32 box tests).  Prints the counts and the coverage of
// the trimmed rows against the whole box of cells, then "ok".
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "lpr_cells.h"

using namespace lpr;

static double wrap_d(double d, double L) {
  if (d > 0.5 * L) d -= L;
  if (d < -0.5 * L) d += L;
  return d;
}

int main() {
  std::mt19937_64 g(11);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  long long covered = 0, boxed = 0;
  for (int t = 0; t < 400; ++t) {
    LevelGrid G{};
    const bool perx = (t % 3) != 0, pery = (t % 5) != 0;
    const double w = 0.5 + U(g);
    double L[2];
    for (int a = 0; a < 3; ++a) {
      const bool per = (a == 0 && perx) || (a == 1 && pery);
      int n = 1 + (int)(g() % 9);
      if (t % 7 == 0 && a < 2) n = 1 + (int)(g() % 3);  // short axes
      G.n[a] = n;
      G.per[a] = per ? 1 : 0;
      if (per) {
        const double box = n * w * (1.0 + 0.3 * U(g));  // cells at least w wide
        G.lo[a] = 0.0;
        G.inv_w[a] = n / box;
        G.w[a] = box / n;
        L[a] = box;
      } else {
        G.lo[a] = -0.5 * n * w + 0.1 * U(g);
        G.inv_w[a] = 1.0 / w;
        G.w[a] = w;
        if (a < 2) L[a] = 0.0;
      }
    }
    G.base = (int64_t)(g() % 5);
    const int64_t ncell = (int64_t)G.n[0] * G.n[1] * G.n[2];
    // particles: inside the grid, some beyond a bounded edge
    const int np = 50 + (int)(g() % 400);
    std::vector<double> P(3 * np);
    for (int i = 0; i < np; ++i)
      for (int a = 0; a < 3; ++a) {
        if (G.per[a]) {
          P[3 * i + a] = U(g) * (G.n[a] / G.inv_w[a]);
        } else {
          const double span = G.n[a] * G.w[a];
          P[3 * i + a] = G.lo[a] + (U(g) * 1.4 - 0.2) * span;
        }
      }
    // binning and cell lists (cell ids relative to the level, then offset
    // by base as the kernels' global ids are)
    std::vector<int64_t> cid(np);
    // cell ranges with poison around them: a read outside the level's cells
    // returns a bound far beyond the particle count
    const int64_t GUARD = 64;
    std::vector<uint32_t> guarded(GUARD + G.base + ncell + 1 + GUARD, 0xfffffff0u), cnt(ncell, 0u);
    uint32_t* start = guarded.data() + GUARD;
    for (int i = 0; i < np; ++i) {
      const int cx = cell_axis(G, 0, P[3 * i]), cy = cell_axis(G, 1, P[3 * i + 1]), cz = cell_axis(G, 2, P[3 * i + 2]);
      cid[i] = ((int64_t)cz * G.n[1] + cy) * G.n[0] + cx;
      cnt[cid[i]]++;
    }
    uint32_t acc = 0;
    for (int64_t c = 0; c < ncell; ++c) {
      start[G.base + c] = acc;
      acc += cnt[c];
    }
    start[G.base + ncell] = acc;
    std::vector<int> list(np), pos(np);
    {
      std::vector<uint32_t> fill(ncell, 0u);
      for (int i = 0; i < np; ++i) {
        pos[i] = (int)(start[G.base + cid[i]] + fill[cid[i]]++);
        list[pos[i]] = i;
      }
    }
    for (int q = 0; q < 60; ++q) {
      const int i = (int)(g() % np);
      double4 pi = make_double4(P[3 * i], P[3 * i + 1], P[3 * i + 2], 0.0);
      if (q % 2) {  // a query point anywhere, also beyond the grid
        for (int a = 0; a < 3; ++a) {
          const double span = G.n[a] / G.inv_w[a];
          const double v = G.per[a] ? U(g) * span : G.lo[a] + (U(g) * 1.4 - 0.2) * span;
          (a == 0 ? pi.x : (a == 1 ? pi.y : pi.z)) = v;
        }
      }
      double wmin = G.w[0];
      for (int a = 1; a < 3; ++a) wmin = std::fmin(wmin, G.w[a]);
      const double reach = wmin * (q % 5 == 0 ? 1.0 : U(g));
      RowSet R;
      row_set(G, pi, reach, R);
      std::vector<int> hit(np, 0);
      int nrow_box = 0;
      for (int p = 0; p < 2; ++p) {
        uint32_t q0[9], q1[9];
        row_piece(start, G, R, p, q0, q1);
        for (int r = 0; r < 9; ++r) {
          if (q1[r] < q0[r] || q1[r] > (uint32_t)np) {
            std::printf("bad row bounds t=%d q=%d r=%d\n", t, q, r);
            return 1;
          }
          for (uint32_t k = q0[r]; k < q1[r]; ++k) hit[list[k]]++;
        }
        // the untrimmed box: same pieces without the cuts
        RowSet B = R;
        B.keep = 0x7ffffffu;
        row_piece(start, G, B, p, q0, q1);
        for (int r = 0; r < 9; ++r) {
          if (q1[r] < q0[r] || q1[r] > (uint32_t)np) {
            std::printf("bad box row bounds t=%d q=%d r=%d\n", t, q, r);
            return 1;
          }
          nrow_box += (int)(q1[r] - q0[r]);
        }
      }
      int nhit = 0;
      for (int j = 0; j < np; ++j) {
        if (hit[j] > 1) {
          std::printf("particle covered twice t=%d q=%d j=%d\n", t, q, j);
          return 1;
        }
        nhit += hit[j];
        double dx = P[3 * j] - pi.x, dy = P[3 * j + 1] - pi.y, dz = P[3 * j + 2] - pi.z;
        if (G.per[0]) dx = wrap_d(dx, L[0]);
        if (G.per[1]) dy = wrap_d(dy, L[1]);
        if (std::sqrt(dx * dx + dy * dy + dz * dz) < reach && !hit[j]) {
          std::printf("missed particle t=%d q=%d j=%d d=%.17g reach=%.17g\n", t, q, j,
                      std::sqrt(dx * dx + dy * dy + dz * dz), reach);
          return 1;
        }
      }
      covered += nhit;
      boxed += nrow_box;
    }
  }
  // cell-level coverage: every cell holds one entry (cell_start[c] = c), so
  // the rows' ranges are cell ranges; for query points inside the grid each
  // cell whose box lies closer than the reach (minimum image on periodic
  // axes) must be covered exactly once, and one farther than the reach by
  // more than the test margins must not be
  long long must = 0, extra = 0, far = 0;
  for (int t = 0; t < 300; ++t) {
    LevelGrid G{};
    double L[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      const bool per = a < 2 && ((t >> a) & 1);
      const int n = per ? 4 + (int)(g() % 6) : 3 + (int)(g() % 6);
      const double w = 0.5 + U(g);
      G.n[a] = n;
      G.per[a] = per ? 1 : 0;
      G.lo[a] = per ? 0.0 : -U(g);
      G.inv_w[a] = 1.0 / w;
      G.w[a] = w;
      L[a] = n * w;
    }
    G.base = 3;
    const int64_t ncell = (int64_t)G.n[0] * G.n[1] * G.n[2];
    const int64_t GUARD = 64;
    std::vector<uint32_t> guarded(GUARD + G.base + ncell + 1 + GUARD, 0xfffffff0u);
    uint32_t* start = guarded.data() + GUARD;
    for (int64_t c = 0; c <= ncell; ++c) start[G.base + c] = (uint32_t)c;
    double wmin = std::fmin(G.w[0], std::fmin(G.w[1], G.w[2]));
    for (int q = 0; q < 200; ++q) {
      double x[3];
      for (int a = 0; a < 3; ++a) x[a] = G.lo[a] + U(g) * L[a];
      // a point near a cell face or corner now and then
      if (q % 3 == 0)
        for (int a = 0; a < 3; ++a) {
          const double f = (x[a] - G.lo[a]) * G.inv_w[a];
          const double fl = std::floor(f);
          if (U(g) < 0.5 && fl >= 0 && fl < G.n[a]) x[a] = G.lo[a] + (fl + 1e-7 * U(g)) * G.w[a];
        }
      const double reach = wmin * (q % 4 == 0 ? 1.0 : (0.3 + 0.7 * U(g)));
      RowSet R;
      row_set(G, make_double4(x[0], x[1], x[2], 0.0), reach, R);
      std::vector<int> hit(ncell, 0);
      for (int p = 0; p < 2; ++p) {
        uint32_t q0[9], q1[9];
        row_piece(start, G, R, p, q0, q1);
        for (int r = 0; r < 9; ++r) {
          if (q1[r] < q0[r] || q1[r] > (uint32_t)ncell) {
            std::printf("bad cell bounds t=%d q=%d r=%d\n", t, q, r);
            return 1;
          }
          for (uint32_t k = q0[r]; k < q1[r]; ++k) hit[k]++;
        }
      }
      for (int64_t c = 0; c < ncell; ++c) {
        const int cc[3] = {(int)(c % G.n[0]), (int)((c / G.n[0]) % G.n[1]), (int)(c / ((int64_t)G.n[0] * G.n[1]))};
        double e2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          const double c0 = G.lo[a] + cc[a] * G.w[a], c1 = c0 + G.w[a];
          double best = 1e300;
          for (int img = -1; img <= 1; ++img) {
            if (!G.per[a] && img != 0) continue;
            const double sh = img * L[a];
            const double d = x[a] < c0 + sh ? c0 + sh - x[a] : (x[a] > c1 + sh ? x[a] - c1 - sh : 0.0);
            best = std::fmin(best, d);
          }
          e2 += best * best;
        }
        const double e = std::sqrt(e2);
        if (hit[c] > 1) {
          std::printf("cell covered twice t=%d q=%d c=%lld\n", t, q, (long long)c);
          return 1;
        }
        if (e < reach * (1.0 - 1e-12)) {
          ++must;
          if (!hit[c]) {
            std::printf("missed cell t=%d q=%d c=%lld e=%.17g reach=%.17g\n", t, q, (long long)c, e, reach);
            return 1;
          }
        } else if (hit[c]) {
          ++extra;
          if (e > reach * (1.0 + 1e-4)) ++far;
        }
      }
    }
  }
  if (far > 0) {
    std::printf("cells beyond the reach covered: %lld\n", far);
    return 1;
  }
  std::printf("cells within reach %lld, covered at the margin %lld\n", must, extra);
  std::printf("trimmed/box %.3f\n", (double)covered / (double)boxed);
  std::printf("ok\n");
  return 0;
}
