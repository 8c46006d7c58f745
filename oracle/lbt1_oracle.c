/*
 * Plain FP64 CPU oracle for the LBMTau1 D2Q9 time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, table or constant with the GPU
 * library.
 *
 * Source: M. Matyka and M. Dzikowski, "Memory-efficient Lattice Boltzmann
 * Method for low Reynolds number flows" (arXiv:1912.09327).
 *
 * What it computes (section 2, "The Model", and the LBMTau1 algorithm of
 * section 2.1, Algorithm 1, with the lid-driven cavity program of Appendix A
 * as the behavioural reference):
 *
 *   state per node: density R and momentum (U, V) = sum_k e_k f_k
 *                   (Eq. rho1, Eq. u1; the algorithm divides U, V by R to get
 *                   the velocity, so the stored U, V are momenta)
 *   with tau = 1 the post-collision populations are the equilibria
 *   (Eq. LBMTau1), so the new moments of a fluid node x are sums over the
 *   nine neighbours x + e_k of the equilibrium that travels from the
 *   neighbour back to x, i.e. in direction inv(k) (Eq. rhotau1, Eq. utau1,
 *   read as momentum sums, see Algorithm 1).
 *   body force: added to the momentum before the velocity used in the
 *   equilibrium is formed (text after Eq. maxwellboltzmann; Algorithm 1).
 *   no-slip wall: if x + e_k is solid, the term is the zero-velocity
 *   equilibrium of x itself, w * R(x) (Eq. feqnoslip) -- the default rule
 *   ("paper" rule).  The "halfway" rule (standard half-way bounce-back of BGK
 *   at tau = 1: the equilibrium that x sends into the wall, f^eq_k(x), comes
 *   back reversed) is provided as the alternative reading.
 *   nodes flagged FIXED (the moving lid of Appendix A) act as sources with
 *   their stored moments and are never updated.
 *   multiphase (section "Moments-only multirelaxation time LBMTau1"): the
 *   Shan-Chen interaction force of Eq. f_sc, F(x) = psi(x) sum_k alpha_k
 *   psi(x + e_k) G(e_k), read with alpha_k = w_k and G(e_k) = -G e_k and the
 *   pseudopotential psi(rho) = rho0 (1 - exp(-rho / rho0)) of the Shan-Chen
 *   model the paper cites; at tau = 1 it enters the equilibrium of its node
 *   exactly like the body force.  A SOLID neighbour contributes the psi of
 *   its stored density; a neighbour outside a non-periodic axis that of the
 *   node itself.
 *
 * Summation follows the paper's direction order k = 0..8 and its arithmetic
 * form w * r * (1 - 3/2 |u|^2 + 3 e.u + 9/2 (e.u)^2).  Build with
 * -ffp-contract=off so the rounding is that of the written expression.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_FLUID = 0, OR_SOLID = 1, OR_FIXED = 2 };
enum { OR_WALL_PAPER = 0, OR_WALL_HALFWAY = 1 };

/* D2Q9 lattice of section 2: velocities in the order printed after
 * Eq. utau1, their inverses, and the weights 4/9, 1/9 (axes), 1/36 (diagonals). */
static const int OR_EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int OR_EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OR_INV[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double OR_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                               1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

void oracle_tables(int *ex, int *ey, int *inv, double *w) {
  for (int k = 0; k < 9; ++k) {
    if (ex) ex[k] = OR_EX[k];
    if (ey) ey[k] = OR_EY[k];
    if (inv) inv[k] = OR_INV[k];
    if (w) w[k] = OR_W[k];
  }
}

/* Eq. maxwellboltzmann for direction k at density r and velocity (u, v). */
double oracle_feq(int k, double r, double u, double v) {
  double eu = OR_EX[k] * u + OR_EY[k] * v;
  return OR_W[k] * r * (1.0 - 1.5 * (u * u + v * v) + 3.0 * eu + 4.5 * eu * eu);
}

/* Neighbour index of (i, j) in direction k; -1 when it leaves a
 * non-periodic axis (such a neighbour counts as a solid wall). */
static long neighbour(int nx, int ny, unsigned periodic, int i, int j, int k) {
  int ip = i + OR_EX[k];
  int jp = j + OR_EY[k];
  if (ip < 0 || ip >= nx) {
    if (!(periodic & 1u)) return -1;
    ip = (ip + nx) % nx;
  }
  if (jp < 0 || jp >= ny) {
    if (!(periodic & 2u)) return -1;
    jp = (jp + ny) % ny;
  }
  return (long)jp * nx + ip;
}

static int oracle_threads = 1;

void oracle_set_threads(int n) { oracle_threads = n > 0 ? n : 1; }

int oracle_get_threads(void) { return oracle_threads; }

/*
 * One LBMTau1 step (Algorithm 1).  Arrays are ny*nx, x fastest.
 * flags == NULL means every node is FLUID.  Non-FLUID nodes are copied.
 * FX, FY (optional, ny*nx): a force per node added to the uniform (fx, fy)
 * of the source node.  Returns 0, or -1 on bad arguments.
 */
static int step_forced(int nx, int ny, unsigned periodic, const uint8_t *flags,
                       double fx, double fy, const double *FX, const double *FY,
                       int wall, const double *R, const double *U,
                       const double *V, double *Rn, double *Un, double *Vn) {
  if (nx < 1 || ny < 1 || !R || !U || !V || !Rn || !Un || !Vn) return -1;
  if (wall != OR_WALL_PAPER && wall != OR_WALL_HALFWAY) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(oracle_threads)
#endif
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      long x = (long)j * nx + i;
      int fl = flags ? flags[x] : OR_FLUID;
      if (fl != OR_FLUID) {
        Rn[x] = R[x];
        Un[x] = U[x];
        Vn[x] = V[x];
        continue;
      }
      double rs = 0.0, us = 0.0, vs = 0.0;
      for (int k = 0; k < 9; ++k) {
        long s = neighbour(nx, ny, periodic, i, j, k);
        int ik = OR_INV[k];
        int solid = (s < 0) || (flags && flags[s] == OR_SOLID);
        double f;
        if (!solid) {
          double gx = FX ? fx + FX[s] : fx;
          double gy = FY ? fy + FY[s] : fy;
          double r = R[s];
          double u = (U[s] + gx) / r;
          double v = (V[s] + gy) / r;
          f = oracle_feq(ik, r, u, v);
        } else if (wall == OR_WALL_PAPER) {
          f = OR_W[ik] * R[x];
        } else {
          double gx = FX ? fx + FX[x] : fx;
          double gy = FY ? fy + FY[x] : fy;
          double r = R[x];
          double u = (U[x] + gx) / r;
          double v = (V[x] + gy) / r;
          f = oracle_feq(k, r, u, v);
        }
        rs += f;
        us += OR_EX[ik] * f;
        vs += OR_EY[ik] * f;
      }
      Rn[x] = rs;
      Un[x] = us;
      Vn[x] = vs;
    }
  }
  return 0;
}

int oracle_step(int nx, int ny, unsigned periodic, const uint8_t *flags,
                double fx, double fy, int wall, const double *R,
                const double *U, const double *V, double *Rn, double *Un,
                double *Vn) {
  return step_forced(nx, ny, periodic, flags, fx, fy, NULL, NULL, wall, R, U,
                     V, Rn, Un, Vn);
}

/* Shan-Chen pseudopotential. */
double oracle_sc_psi(double r, double rho0) { return rho0 * (1.0 - exp(-r / rho0)); }

/*
 * Shan-Chen force of every FLUID and FIXED node (Eq. f_sc with alpha_k = w_k,
 * G(e_k) = -G e_k):  F(x) = -G psi(x) sum_{k=1..8} w_k psi(x + e_k) e_k.
 * FX, FY receive ny*nx values (0 at SOLID nodes).  Returns 0 or -1.
 */
int oracle_sc_force(int nx, int ny, unsigned periodic, const uint8_t *flags,
                    double G, double rho0, const double *R, double *FX,
                    double *FY) {
  if (nx < 1 || ny < 1 || !R || !FX || !FY || !(rho0 > 0.0)) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(oracle_threads)
#endif
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      long x = (long)j * nx + i;
      if (flags && flags[x] == OR_SOLID) {
        FX[x] = 0.0;
        FY[x] = 0.0;
        continue;
      }
      double px = oracle_sc_psi(R[x], rho0);
      double sx = 0.0, sy = 0.0;
      for (int k = 1; k < 9; ++k) {
        long s = neighbour(nx, ny, periodic, i, j, k);
        double pk = s < 0 ? px : oracle_sc_psi(R[s], rho0);
        sx += OR_W[k] * pk * OR_EX[k];
        sy += OR_W[k] * pk * OR_EY[k];
      }
      FX[x] = -G * px * sx;
      FY[x] = -G * px * sy;
    }
  }
  return 0;
}

/* One multiphase step: the Shan-Chen force of the current state, then the
 * LBMTau1 step with it added to the uniform force. */
int oracle_step_sc(int nx, int ny, unsigned periodic, const uint8_t *flags,
                   double fx, double fy, double G, double rho0, int wall,
                   const double *R, const double *U, const double *V,
                   double *Rn, double *Un, double *Vn) {
  size_t n = (size_t)nx * (size_t)ny;
  double *F = (double *)malloc(2 * n * sizeof(double));
  if (!F) return -2;
  int rc = oracle_sc_force(nx, ny, periodic, flags, G, rho0, R, F, F + n);
  if (!rc)
    rc = step_forced(nx, ny, periodic, flags, fx, fy, F, F + n, wall, R, U, V,
                     Rn, Un, Vn);
  free(F);
  return rc;
}

/*
 * n steps in place on (R, U, V), ping-ponging through a scratch copy
 * (the two grids of Algorithm 1).  Returns 0, -1 on bad arguments,
 * -2 when scratch memory cannot be had.
 */
static int run_impl(int nx, int ny, unsigned periodic, const uint8_t *flags,
                    double fx, double fy, int sc, double G, double rho0,
                    int wall, long nsteps, double *R, double *U, double *V) {
  if (nsteps < 0) return -1;
  if (nsteps == 0) return 0;
  size_t n = (size_t)nx * (size_t)ny;
  double *buf = (double *)malloc(3 * n * sizeof(double));
  if (!buf) return -2;
  double *a[3] = {R, U, V};
  double *b[3] = {buf, buf + n, buf + 2 * n};
  for (long t = 0; t < nsteps; ++t) {
    int rc = sc ? oracle_step_sc(nx, ny, periodic, flags, fx, fy, G, rho0,
                                 wall, a[0], a[1], a[2], b[0], b[1], b[2])
                : oracle_step(nx, ny, periodic, flags, fx, fy, wall, a[0],
                              a[1], a[2], b[0], b[1], b[2]);
    if (rc) {
      free(buf);
      return rc;
    }
    for (int q = 0; q < 3; ++q) {
      double *tmp = a[q];
      a[q] = b[q];
      b[q] = tmp;
    }
  }
  if (a[0] != R) {
    memcpy(R, a[0], n * sizeof(double));
    memcpy(U, a[1], n * sizeof(double));
    memcpy(V, a[2], n * sizeof(double));
  }
  free(buf);
  return 0;
}

int oracle_run(int nx, int ny, unsigned periodic, const uint8_t *flags,
               double fx, double fy, int wall, long nsteps, double *R,
               double *U, double *V) {
  return run_impl(nx, ny, periodic, flags, fx, fy, 0, 0.0, 1.0, wall, nsteps,
                  R, U, V);
}

int oracle_run_sc(int nx, int ny, unsigned periodic, const uint8_t *flags,
                  double fx, double fy, double G, double rho0, int wall,
                  long nsteps, double *R, double *U, double *V) {
  return run_impl(nx, ny, periodic, flags, fx, fy, 1, G, rho0, wall, nsteps, R,
                  U, V);
}

/*
 * Diagnostics over FLUID nodes, all in FP64:
 *   out[0] mass          sum R                       (Eq. rho1 summed)
 *   out[1] momentum x    sum U
 *   out[2] momentum y    sum V
 *   out[3] residual      max over nodes and components of |u - u_snap|,
 *                        u = (U, V) / R  (0 when snap arrays are NULL)
 *   out[4] non-finite    count of nodes with a non-finite R, U or V
 *   out[5] fluid nodes   count
 */
int oracle_reduce(int nx, int ny, const uint8_t *flags, const double *R,
                  const double *U, const double *V, const double *Rs,
                  const double *Us, const double *Vs, double *out) {
  if (nx < 1 || ny < 1 || !R || !U || !V || !out) return -1;
  double m = 0.0, px = 0.0, py = 0.0, res = 0.0, bad = 0.0, cnt = 0.0;
  size_t n = (size_t)nx * (size_t)ny;
  for (size_t x = 0; x < n; ++x) {
    if (flags && flags[x] != OR_FLUID) continue;
    cnt += 1.0;
    if (!isfinite(R[x]) || !isfinite(U[x]) || !isfinite(V[x])) bad += 1.0;
    m += R[x];
    px += U[x];
    py += V[x];
    if (Rs && Us && Vs) {
      double du = fabs(U[x] / R[x] - Us[x] / Rs[x]);
      double dv = fabs(V[x] / R[x] - Vs[x] / Rs[x]);
      if (du > res) res = du;
      if (dv > res) res = dv;
    }
  }
  out[0] = m;
  out[1] = px;
  out[2] = py;
  out[3] = res;
  out[4] = bad;
  out[5] = cnt;
  return 0;
}
