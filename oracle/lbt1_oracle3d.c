/*
 * Plain FP64 CPU oracle for the three-dimensional LBMTau1 step (D3Q19 and
 * D3Q27).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; it shares no code, table or constant with the GPU library.
 *
 * Source: M. Matyka and M. Dzikowski, arXiv:1912.09327.  The method is the
 * one of section 2 and Algorithm 1 with the lattice of the memory analysis of
 * section 4 (D3Q19, D3Q27): at tau = 1 the populations leaving a node are
 * the equilibria of its moments (Eq. LBMTau1), so a fluid node's new density
 * and momentum are sums over the Q lattice directions of the equilibrium the
 * upwind neighbour x - e_q sends along e_q (Eq. rhotau1, Eq. utau1 read as
 * momentum sums).  Eq. maxwellboltzmann carries over unchanged with the 3-D
 * weights; body force, the two wall rules and FIXED nodes as in the 2-D
 * oracle (a neighbour outside a non-periodic axis is a wall).
 *
 * The paper prints no 3-D direction order.  This oracle enumerates the
 * velocities with e_z outermost, then e_y, then e_x, each over -1, 0, 1,
 * keeping |e|^2 <= 2 for D3Q19; the weights follow from |e|^2:
 *   D3Q19: 1/3 (rest), 1/18 (|e|^2 = 1), 1/36 (|e|^2 = 2)
 *   D3Q27: 8/27, 2/27, 1/54, 1/216 (|e|^2 = 0, 1, 2, 3)
 * Build with -ffp-contract=off.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { O3_FLUID = 0, O3_SOLID = 1, O3_FIXED = 2 };
enum { O3_WALL_PAPER = 0, O3_WALL_HALFWAY = 1 };

typedef struct {
  int q;
  int e[27][3];
  int inv[27];
  double w[27];
} lattice3;

static int make_lattice(int q, lattice3 *L) {
  if (q != 19 && q != 27) return -1;
  static const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
  static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  int n = 0;
  for (int ez = -1; ez <= 1; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        int m = ex * ex + ey * ey + ez * ez;
        if (q == 19 && m > 2) continue;
        L->e[n][0] = ex;
        L->e[n][1] = ey;
        L->e[n][2] = ez;
        L->w[n] = q == 19 ? w19[m] : w27[m];
        ++n;
      }
  L->q = n;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (L->e[b][0] == -L->e[a][0] && L->e[b][1] == -L->e[a][1] && L->e[b][2] == -L->e[a][2]) L->inv[a] = b;
  return 0;
}

/* Velocities (q x 3, row-major) and weights of the oracle's lattice. */
int oracle3_tables(int q, int *e, double *w) {
  lattice3 L;
  if (make_lattice(q, &L)) return -1;
  for (int k = 0; k < L.q; ++k) {
    if (e)
      for (int a = 0; a < 3; ++a) e[3 * k + a] = L.e[k][a];
    if (w) w[k] = L.w[k];
  }
  return L.q;
}

static double feq3(const lattice3 *L, int k, double r, double u, double v, double w) {
  double eu = L->e[k][0] * u + L->e[k][1] * v + L->e[k][2] * w;
  return L->w[k] * r * (1.0 - 1.5 * (u * u + v * v + w * w) + 3.0 * eu + 4.5 * eu * eu);
}

static long nb3(int nx, int ny, int nz, unsigned per, int i, int j, int k, const int *e) {
  int a = i + e[0], b = j + e[1], c = k + e[2];
  if (a < 0 || a >= nx) {
    if (!(per & 1u)) return -1;
    a = (a + nx) % nx;
  }
  if (b < 0 || b >= ny) {
    if (!(per & 2u)) return -1;
    b = (b + ny) % ny;
  }
  if (c < 0 || c >= nz) {
    if (!(per & 4u)) return -1;
    c = (c + nz) % nz;
  }
  return ((long)c * ny + b) * nx + a;
}

static int o3_threads = 1;
void oracle3_set_threads(int n) { o3_threads = n > 0 ? n : 1; }

/*
 * One 3-D LBMTau1 step.  Arrays are nz*ny*nx, x fastest; state (R, U, V, W):
 * density and momentum.  flags NULL: all FLUID.  periodic: bit 0 x, 1 y, 2 z.
 */
int oracle3_step(int q, int nx, int ny, int nz, unsigned periodic, const uint8_t *flags, double fx, double fy,
                 double fz, int wall, const double *R, const double *U, const double *V, const double *W,
                 double *Rn, double *Un, double *Vn, double *Wn) {
  lattice3 L;
  if (make_lattice(q, &L) || nx < 1 || ny < 1 || nz < 1) return -1;
  if (wall != O3_WALL_PAPER && wall != O3_WALL_HALFWAY) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(o3_threads)
#endif
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long x = ((long)k * ny + j) * nx + i;
        int fl = flags ? flags[x] : O3_FLUID;
        if (fl != O3_FLUID) {
          Rn[x] = R[x];
          Un[x] = U[x];
          Vn[x] = V[x];
          Wn[x] = W[x];
          continue;
        }
        double rs = 0.0, us = 0.0, vs = 0.0, ws = 0.0;
        for (int d = 0; d < L.q; ++d) {
          /* the population arriving along e_d comes from x - e_d = x + e_inv(d) */
          int id = L.inv[d];
          long s = nb3(nx, ny, nz, periodic, i, j, k, L.e[id]);
          int solid = s < 0 || (flags && flags[s] == O3_SOLID);
          double f;
          if (!solid) {
            double r = R[s];
            f = feq3(&L, d, r, (U[s] + fx) / r, (V[s] + fy) / r, (W[s] + fz) / r);
          } else if (wall == O3_WALL_PAPER) {
            f = L.w[d] * R[x];
          } else {
            double r = R[x];
            f = feq3(&L, id, r, (U[x] + fx) / r, (V[x] + fy) / r, (W[x] + fz) / r);
          }
          rs += f;
          us += L.e[d][0] * f;
          vs += L.e[d][1] * f;
          ws += L.e[d][2] * f;
        }
        Rn[x] = rs;
        Un[x] = us;
        Vn[x] = vs;
        Wn[x] = ws;
      }
  return 0;
}

int oracle3_run(int q, int nx, int ny, int nz, unsigned periodic, const uint8_t *flags, double fx, double fy,
                double fz, int wall, long nsteps, double *R, double *U, double *V, double *W) {
  if (nsteps < 0) return -1;
  size_t n = (size_t)nx * ny * nz;
  double *buf = (double *)malloc(4 * n * sizeof(double));
  if (!buf) return -2;
  double *a[4] = {R, U, V, W};
  double *b[4] = {buf, buf + n, buf + 2 * n, buf + 3 * n};
  for (long t = 0; t < nsteps; ++t) {
    int rc = oracle3_step(q, nx, ny, nz, periodic, flags, fx, fy, fz, wall, a[0], a[1], a[2], a[3], b[0], b[1],
                          b[2], b[3]);
    if (rc) {
      free(buf);
      return rc;
    }
    for (int m = 0; m < 4; ++m) {
      double *tmp = a[m];
      a[m] = b[m];
      b[m] = tmp;
    }
  }
  if (a[0] != R)
    for (int m = 0; m < 4; ++m) memcpy(m == 0 ? R : m == 1 ? U : m == 2 ? V : W, a[m], n * sizeof(double));
  free(buf);
  return 0;
}
