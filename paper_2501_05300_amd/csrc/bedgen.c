/*
 * bedgen.c -- seeded input generation: vertical drop placement of sphere
 * rafts onto a periodic bed.
 *
 * Input only.  This file holds no contact mechanics: it places each sphere at
 * the lowest height where it touches (without overlapping) the spheres
 * already placed below it or the floor z = 0, which is how the generators
 * build dense, overlap-free graded beds that a short settle turns into a
 * static packing.
 *
 * Spheres arrive grouped in rafts (a raft is one horizontal lattice layer of
 * similar-size spheres that do not touch one another).  A sphere of raft R
 * is tested against the spheres of rafts R-1 .. R-depth.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t* head;  /* first sphere per cell, -1 = empty */
  int64_t* next;  /* next sphere in the same cell */
  int64_t nx, ny;
  double cx, cy;
} grid2;

static int64_t wrapi(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

/* Places spheres raft by raft.  x, y, r: per-sphere inputs ordered by raft;
 * raft_start[0..n_rafts]: index ranges.  Lx, Ly: periodic lengths.  depth:
 * how many earlier rafts to test against.  z: output heights.
 * Returns 0, or -1 on bad input / allocation failure. */
int bedgen_drop(int64_t n, const double* x, const double* y, const double* r, int64_t n_rafts,
                const int64_t* raft_start, double Lx, double Ly, int32_t depth, double* z) {
  if (n <= 0 || n_rafts <= 0 || !(Lx > 0.0) || !(Ly > 0.0) || depth < 1) return -1;
  if (raft_start[0] != 0 || raft_start[n_rafts] != n) return -1;
  grid2 g;
  g.next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!g.next) return -1;
  int64_t cap_cells = 0;
  g.head = NULL;
  for (int64_t R = 0; R < n_rafts; ++R) {
    const int64_t a0 = raft_start[R], a1 = raft_start[R + 1];
    const int64_t p0 = raft_start[R - depth < 0 ? 0 : R - depth];
    /* cell edge >= r_i + r_j for any tested pair */
    double rc = 0.0, rp = 0.0;
    for (int64_t i = a0; i < a1; ++i) rc = fmax(rc, r[i]);
    for (int64_t i = p0; i < a0; ++i) rp = fmax(rp, r[i]);
    const double h = rc + rp;
    int64_t nx = 1, ny = 1;
    if (h > 0.0) {
      nx = (int64_t)floor(Lx / h);
      ny = (int64_t)floor(Ly / h);
      if (nx < 1) nx = 1;
      if (ny < 1) ny = 1;
    }
    if (nx * ny > cap_cells) {
      free(g.head);
      cap_cells = nx * ny;
      g.head = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap_cells);
      if (!g.head) { free(g.next); return -1; }
    }
    g.nx = nx;
    g.ny = ny;
    g.cx = Lx / (double)nx;
    g.cy = Ly / (double)ny;
    for (int64_t c = 0; c < nx * ny; ++c) g.head[c] = -1;
    for (int64_t j = p0; j < a0; ++j) {
      int64_t ix = (int64_t)floor(x[j] / g.cx), iy = (int64_t)floor(y[j] / g.cy);
      ix = wrapi(ix, nx);
      iy = wrapi(iy, ny);
      const int64_t c = iy * nx + ix;
      g.next[j] = g.head[c];
      g.head[c] = j;
    }
    for (int64_t i = a0; i < a1; ++i) {
      double zi = r[i];
      int64_t ix = (int64_t)floor(x[i] / g.cx), iy = (int64_t)floor(y[i] / g.cy);
      int64_t seenx[3], seeny[3];
      int nsx = 0, nsy = 0;
      for (int d = -1; d <= 1; ++d) {
        const int64_t cx = wrapi(ix + d, nx), cy = wrapi(iy + d, ny);
        int dup = 0;
        for (int q = 0; q < nsx; ++q) dup |= (seenx[q] == cx);
        if (!dup) seenx[nsx++] = cx;
        dup = 0;
        for (int q = 0; q < nsy; ++q) dup |= (seeny[q] == cy);
        if (!dup) seeny[nsy++] = cy;
      }
      for (int b = 0; b < nsy; ++b)
        for (int a = 0; a < nsx; ++a)
          for (int64_t j = g.head[seeny[b] * nx + seenx[a]]; j >= 0; j = g.next[j]) {
            double dx = x[i] - x[j], dy = y[i] - y[j];
            if (dx > 0.5 * Lx) dx -= Lx;
            else if (dx < -0.5 * Lx) dx += Lx;
            if (dy > 0.5 * Ly) dy -= Ly;
            else if (dy < -0.5 * Ly) dy += Ly;
            const double R = r[i] + r[j];
            const double rho2 = dx * dx + dy * dy;
            if (rho2 >= R * R) continue;
            /* rest just above contact; the tiny lift keeps the pair apart
             * after rounding */
            const double zt = z[j] + sqrt(R * R - rho2) + 1e-9 * R;
            if (zt > zi) zi = zt;
          }
      z[i] = zi;
    }
  }
  free(g.head);
  free(g.next);
  return 0;
}
