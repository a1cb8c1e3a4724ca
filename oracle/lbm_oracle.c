/*
 * FP64 reference ("oracle") of the vectorial D2Q4^5 lattice Boltzmann scheme
 * for 2D linear elastodynamics (Boolakee, Geier, De Lorenzis, arXiv 2408.01081).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct C in double
 * precision.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code with the HIP library.
 *
 * Everything is in the paper's dimensionless variables (Section 2.3) with the
 * lattice speed c = dx/dt.  The flux matrices enter only through
 *   Phi_hat_x(U) = Phi_x(U)/c,  Phi_hat_y(U) = Phi_y(U)/c,
 * i.e. through the Courant numbers kK = c_K/c and km = c_mu/c.
 *
 * Array layouts (row-major, x fastest):
 *   populations f[q][c][ny][nx], q = 0..3 in the paper's order
 *     (1,0), (0,1), (-1,0), (0,-1)  (Eq. index_vel), c = 0..4 the components
 *     of U = (v_x, v_y, j_s, j_d, j_xy) (Eq. system);
 *   fields U[c][ny][nx]; body load Bhat[2][ny][nx] = dt * (b_x, b_y);
 *   wall data w[L][2], L = 2(nx+ny), in link order left, right, bottom, top
 *     (see orc_wall_link).
 *
 * Node (k,l) sits at ((k+1/2)dx, (l+1/2)dx).  For Dirichlet problems the
 * physical boundary lies half a spacing outside the outermost nodes
 * (q_ij = 1/2, Eq. bc_q).
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define NQ 4
#define NC 5

static const int EI[NQ] = {1, 0, -1, 0};
static const int EJ[NQ] = {0, 1, 0, -1};

/* index of the opposite direction (-i,-j) */
static int opposite(int q) { return (q + 2) % NQ; }

static size_t at(int c, int l, int k, int nx, int ny) {
  return ((size_t)c * ny + l) * nx + k;
}
static size_t atq(int q, int c, int l, int k, int nx, int ny) {
  return (((size_t)q * NC + c) * ny + l) * nx + k;
}

/* Flux functions of Eq. system divided by c (lattice units). */
static void phi_hat_x(double kK, double km, const double U[NC], double out[NC]) {
  out[0] = kK * U[2] + km * U[3];
  out[1] = km * U[4];
  out[2] = kK * U[0];
  out[3] = km * U[0];
  out[4] = km * U[1];
}
static void phi_hat_y(double kK, double km, const double U[NC], double out[NC]) {
  out[0] = km * U[4];
  out[1] = kK * U[2] - km * U[3];
  out[2] = kK * U[1];
  out[3] = -km * U[1];
  out[4] = km * U[0];
}

/* Equilibrium of Eq. feq:  f_eq_ij = 1/4 [ U + (2/c)(i Phi_x(U) + j Phi_y(U)) ]. */
static void equilibrium(double kK, double km, int q, const double U[NC], double feq[NC]) {
  double px[NC], py[NC];
  phi_hat_x(kK, km, U, px);
  phi_hat_y(kK, km, U, py);
  for (int c = 0; c < NC; ++c)
    feq[c] = 0.25 * (U[c] + 2.0 * (EI[q] * px[c] + EJ[q] * py[c]));
}

/* Zeroth moment plus half the forcing (Eq. cond_eq):
   U_num = sum_ij f_ij + dt/2 B.  Bhat = dt*B may be NULL (B = 0). */
static void zeroth_moment(const double* f, const double* Bhat, int k, int l, int nx, int ny,
                          double U[NC]) {
  for (int c = 0; c < NC; ++c) {
    double s = 0.0;
    for (int q = 0; q < NQ; ++q) s += f[atq(q, c, l, k, nx, ny)];
    U[c] = s;
  }
  if (Bhat) {
    U[0] += 0.5 * Bhat[at(0, l, k, nx, ny)];
    U[1] += 0.5 * Bhat[at(1, l, k, nx, ny)];
  }
}

/* ---------------------------------------------------------------------------
 * Wall links for the Dirichlet rule (Section 3.4.2).
 * For a boundary node x and a missing incoming direction q in D_x, the link
 * index into the wall data array:
 *   q = 0 (from the left)  at k = 0      -> l
 *   q = 2 (from the right) at k = nx-1   -> ny + l
 *   q = 1 (from below)     at l = 0      -> 2 ny + k
 *   q = 3 (from above)     at l = ny-1   -> 2 ny + nx + k
 * ------------------------------------------------------------------------- */
int orc_wall_link(int q, int k, int l, int nx, int ny) {
  switch (q) {
    case 0: return l;
    case 2: return ny + l;
    case 1: return 2 * ny + k;
    case 3: return 2 * ny + nx + k;
  }
  return -1;
}

/* Source term of Eq. bc_s for link direction (i,j) and wall velocity
 * du_D/dt = (a, b).  Rows 3-5 carry the Courant numbers kK = c_K/c and
 * km = c_mu/c: the leading-order bounce-back balance (Eq. bb0) reads
 * (1/c)(i Phi_x + j Phi_y) of the wall state, so the printed wave speeds are
 * divided by the lattice speed c (they coincide only for c = 1). */
/* Test-only ablation switch: when nonzero, rows 3-5 use the wave speeds
   c_K, c_mu themselves (kK*c, km*c) as printed, instead of kK, km. */
static double printed_source_c = 0.0;
void orc_set_printed_wall_source(double c) { printed_source_c = c; }

static void wall_source(double kK, double km, int q, double a, double b, double S[NC]) {
  const int i = EI[q], j = EJ[q];
  if (printed_source_c > 0.0) {
    kK *= printed_source_c;
    km *= printed_source_c;
  }
  S[0] = 0.5 * a;
  S[1] = 0.5 * b;
  S[2] = kK * (i * a + j * b);
  S[3] = km * (i * a - j * b);
  S[4] = km * (j * a + i * b);
}

/* ---------------------------------------------------------------------------
 * One time step (Section 3.6):
 *  1. collision: (a) U_num = sum f + dt/2 B(t_n); (b) displacement hook;
 *     (c) f_eq via Eq. feq; (d) f* = omega f_eq + (1 - omega) f, omega = 2
 *     (the forcing term of Eq. collision vanishes at omega = 2);
 *  2. streaming: f_ij(x + c_ij dt) = f*_ij(x) (Eq. streaming) with periodic
 *     wrap (Section 3.4.1) or, for missing links at boundary nodes,
 *     Eq. bc_ansatz  f_ij(x, t+dt) = D f*_{-i-j}(x, t) + S_ij(x_b, t + dt/2);
 *     (c) u* = u + dt/2 v.
 *
 * f      : pre-collision populations at t_n (input)
 * fnext  : pre-collision populations at t_{n+1} (output, may not alias f)
 * Bhat   : dt*(b_x, b_y) at t_n, or NULL
 * wall   : du_D/dt at the wall midpoints at t_n + dt/2, [L][2], or NULL (zero)
 * ustar  : u* (in/out, [2][ny][nx]) or NULL; uout receives u(t_n) or NULL
 * Uout   : receives U_num(t_n) [5][ny][nx] or NULL
 * dt     : physical time step (only used by the displacement hook)
 * fstar  : scratch [4][5][ny][nx]
 * ------------------------------------------------------------------------- */
void orc_step(int nx, int ny, int bc, double kK, double km, double dt,
              const double* f, double* fnext, const double* Bhat, const double* wall,
              double* ustar, double* uout, double* Uout, double* fstar) {
  const double omega = 2.0;
  /* 1. collision */
#pragma omp parallel for schedule(static)
  for (int l = 0; l < ny; ++l) {
    for (int k = 0; k < nx; ++k) {
      double U[NC];
      zeroth_moment(f, Bhat, k, l, nx, ny, U);
      if (Uout)
        for (int c = 0; c < NC; ++c) Uout[at(c, l, k, nx, ny)] = U[c];
      if (ustar) {
        for (int d = 0; d < 2; ++d) {
          double u = ustar[at(d, l, k, nx, ny)] + 0.5 * dt * U[d];
          if (uout) uout[at(d, l, k, nx, ny)] = u;
          /* 2(c): prepared here because v_num(t_n) is at hand */
          ustar[at(d, l, k, nx, ny)] = u + 0.5 * dt * U[d];
        }
      }
      for (int q = 0; q < NQ; ++q) {
        double feq[NC];
        equilibrium(kK, km, q, U, feq);
        for (int c = 0; c < NC; ++c) {
          size_t id = atq(q, c, l, k, nx, ny);
          fstar[id] = omega * feq[c] + (1.0 - omega) * f[id];
        }
      }
    }
  }
  /* 2. streaming, pulled: the population arriving at node (k,l) along q left
        node (k - i, l - j). */
#pragma omp parallel for schedule(static)
  for (int l = 0; l < ny; ++l) {
    for (int k = 0; k < nx; ++k) {
      for (int q = 0; q < NQ; ++q) {
        int ks = k - EI[q], ls = l - EJ[q];
        int inside = ks >= 0 && ks < nx && ls >= 0 && ls < ny;
        if (inside || bc == 0) {
          ks = (ks + nx) % nx;
          ls = (ls + ny) % ny;
          for (int c = 0; c < NC; ++c)
            fnext[atq(q, c, l, k, nx, ny)] = fstar[atq(q, c, ls, ks, nx, ny)];
        } else {
          /* Dirichlet: anti-bounce-back on (v_x, v_y), bounce-back on the rest
             (D = diag(-1,-1,1,1,1), Eq. bc_d), plus the source S_ij. */
          const int qb = opposite(q);
          double S[NC] = {0, 0, 0, 0, 0};
          if (wall) {
            int L = orc_wall_link(q, k, l, nx, ny);
            wall_source(kK, km, q, wall[2 * L], wall[2 * L + 1], S);
          }
          static const double D[NC] = {-1.0, -1.0, 1.0, 1.0, 1.0};
          for (int c = 0; c < NC; ++c)
            fnext[atq(q, c, l, k, nx, ny)] = D[c] * fstar[atq(qb, c, l, k, nx, ny)] + S[c];
        }
      }
    }
  }
}

/* U_num = sum f + dt/2 B for the whole grid (Eq. cond_eq). */
void orc_moments(int nx, int ny, const double* f, const double* Bhat, double* Uout) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < ny; ++l)
    for (int k = 0; k < nx; ++k) {
      double U[NC];
      zeroth_moment(f, Bhat, k, l, nx, ny, U);
      for (int c = 0; c < NC; ++c) Uout[at(c, l, k, nx, ny)] = U[c];
    }
}

/* ---------------------------------------------------------------------------
 * Second-order initialisation, Eq. ic_second, in lattice units:
 *   f_ij(x,0) = 1/4 [U0 + 2(i Ph_x(U0) + j Ph_y(U0))]
 *     - 1/8 { [Bh + 2(i Ph_x(Bh) + j Ph_y(Bh))]
 *           + [ i UX + (2i^2-1) Ph_x(UX) - 2(i Ph_x(Ph_x(UX)) + j Ph_y(Ph_x(UX))) ]
 *           + [ j UY + (2j^2-1) Ph_y(UY) - 2(i Ph_x(Ph_y(UY)) + j Ph_y(Ph_y(UY))) ] }
 * with Ph = Phi/c, Bh = dt*B(0), UX = dx * dU0/dx, UY = dx * dU0/dy
 * (the paper's factors dt*c = dx and dt/c * c^2 = dx absorbed).
 *
 * UX/UY may be NULL: they are then taken from second-order central
 * differences of U0 on the lattice (periodic wrap; at Dirichlet walls the
 * one-sided second-order formula (-3U0 + 4U1 - U2)/2, first order on a grid
 * two nodes wide, zero on a grid one node wide).
 * ------------------------------------------------------------------------- */
static double lattice_derivative(const double* U0, int c, int k, int l, int nx, int ny, int bc,
                                 int axis) {
  const int n = axis == 0 ? nx : ny;
  const int m = axis == 0 ? k : l;
#define U0AT(mm) (axis == 0 ? U0[at(c, l, (mm), nx, ny)] : U0[at(c, (mm), k, nx, ny)])
  if (bc == 0) {
    if (n == 1) return 0.0;
    return 0.5 * (U0AT((m + 1) % n) - U0AT((m - 1 + n) % n));
  }
  if (n == 1) return 0.0;
  if (n == 2) return U0AT(1) - U0AT(0);
  if (m == 0) return 0.5 * (-3.0 * U0AT(0) + 4.0 * U0AT(1) - U0AT(2));
  if (m == n - 1) return 0.5 * (3.0 * U0AT(n - 1) - 4.0 * U0AT(n - 2) + U0AT(n - 3));
  return 0.5 * (U0AT(m + 1) - U0AT(m - 1));
#undef U0AT
}

void orc_init(int nx, int ny, int bc, double kK, double km, const double* U0, const double* UX,
              const double* UY, const double* Bhat0, double* f) {
#pragma omp parallel for schedule(static)
  for (int l = 0; l < ny; ++l) {
    for (int k = 0; k < nx; ++k) {
      double u[NC], ux[NC], uy[NC], bh[NC] = {0, 0, 0, 0, 0};
      for (int c = 0; c < NC; ++c) {
        u[c] = U0[at(c, l, k, nx, ny)];
        ux[c] = UX ? UX[at(c, l, k, nx, ny)] : lattice_derivative(U0, c, k, l, nx, ny, bc, 0);
        uy[c] = UY ? UY[at(c, l, k, nx, ny)] : lattice_derivative(U0, c, k, l, nx, ny, bc, 1);
      }
      if (Bhat0) {
        bh[0] = Bhat0[at(0, l, k, nx, ny)];
        bh[1] = Bhat0[at(1, l, k, nx, ny)];
      }
      double pxU[NC], pyU[NC], pxB[NC], pyB[NC], pxX[NC], pyY[NC];
      double pxpxX[NC], pypxX[NC], pxpyY[NC], pypyY[NC];
      phi_hat_x(kK, km, u, pxU);
      phi_hat_y(kK, km, u, pyU);
      phi_hat_x(kK, km, bh, pxB);
      phi_hat_y(kK, km, bh, pyB);
      phi_hat_x(kK, km, ux, pxX);
      phi_hat_y(kK, km, uy, pyY);
      phi_hat_x(kK, km, pxX, pxpxX);
      phi_hat_y(kK, km, pxX, pypxX);
      phi_hat_x(kK, km, pyY, pxpyY);
      phi_hat_y(kK, km, pyY, pypyY);
      for (int q = 0; q < NQ; ++q) {
        const double i = EI[q], j = EJ[q];
        for (int c = 0; c < NC; ++c) {
          double eq = 0.25 * (u[c] + 2.0 * (i * pxU[c] + j * pyU[c]));
          double force = bh[c] + 2.0 * (i * pxB[c] + j * pyB[c]);
          double xpart = i * ux[c] + (2.0 * i * i - 1.0) * pxX[c] -
                         2.0 * (i * pxpxX[c] + j * pypxX[c]);
          double ypart = j * uy[c] + (2.0 * j * j - 1.0) * pyY[c] -
                         2.0 * (i * pxpyY[c] + j * pypyY[c]);
          f[atq(q, c, l, k, nx, ny)] = eq - 0.125 * (force + xpart + ypart);
        }
      }
    }
  }
}

/* ---------------------------------------------------------------------------
 * Weighted L2 grid norm squared (Definition grid_norm with Eq. def_symmetrizer):
 *   ||f||_P^2 = sum_x sum_ij f_ij^T k_ij f_ij,  k_ij = g_ij^{-1},
 *   g_ij = 1/4 I + 1/(2c) (i A_x + j A_y)   (Eq. stability_linear).
 * The inverse is formed by Gauss-Jordan elimination with partial pivoting.
 * Returns -1 if some g_ij is singular.
 * ------------------------------------------------------------------------- */
static void flux_matrices(double kK, double km, double Ax[NC][NC], double Ay[NC][NC]) {
  /* columns are Phi_hat applied to unit vectors */
  for (int c = 0; c < NC; ++c) {
    double e[NC] = {0, 0, 0, 0, 0}, px[NC], py[NC];
    e[c] = 1.0;
    phi_hat_x(kK, km, e, px);
    phi_hat_y(kK, km, e, py);
    for (int r = 0; r < NC; ++r) {
      Ax[r][c] = px[r];
      Ay[r][c] = py[r];
    }
  }
}

static int invert5(double a[NC][NC], double inv[NC][NC]) {
  double m[NC][2 * NC];
  for (int r = 0; r < NC; ++r)
    for (int c = 0; c < 2 * NC; ++c) m[r][c] = c < NC ? a[r][c] : (c - NC == r ? 1.0 : 0.0);
  for (int col = 0; col < NC; ++col) {
    int piv = col;
    for (int r = col + 1; r < NC; ++r)
      if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
    if (fabs(m[piv][col]) < 1e-300) return -1;
    if (piv != col)
      for (int c = 0; c < 2 * NC; ++c) {
        double t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    double d = m[col][col];
    for (int c = 0; c < 2 * NC; ++c) m[col][c] /= d;
    for (int r = 0; r < NC; ++r)
      if (r != col) {
        double fct = m[r][col];
        for (int c = 0; c < 2 * NC; ++c) m[r][c] -= fct * m[col][c];
      }
  }
  for (int r = 0; r < NC; ++r)
    for (int c = 0; c < NC; ++c) inv[r][c] = m[r][c + NC];
  return 0;
}

/* k_ij matrices, out[q][5][5] */
int orc_norm_weights(double kK, double km, double* out) {
  double Ax[NC][NC], Ay[NC][NC];
  flux_matrices(kK, km, Ax, Ay);
  for (int q = 0; q < NQ; ++q) {
    double g[NC][NC], kq[NC][NC];
    for (int r = 0; r < NC; ++r)
      for (int c = 0; c < NC; ++c)
        g[r][c] = (r == c ? 0.25 : 0.0) + 0.5 * (EI[q] * Ax[r][c] + EJ[q] * Ay[r][c]);
    if (invert5(g, kq)) return -1;
    for (int r = 0; r < NC; ++r)
      for (int c = 0; c < NC; ++c) out[(q * NC + r) * NC + c] = kq[r][c];
  }
  return 0;
}

double orc_energy(int nx, int ny, double kK, double km, const double* f) {
  double kw[NQ * NC * NC];
  if (orc_norm_weights(kK, km, kw)) return -1.0;
  /* one partial sum per row, then the rows in order: the value does not
     depend on the number of threads */
  double* rows = (double*)malloc(sizeof(double) * (size_t)ny);
  if (!rows) return -1.0;
#pragma omp parallel for schedule(static)
  for (int l = 0; l < ny; ++l) {
    double row = 0.0;
    for (int k = 0; k < nx; ++k)
      for (int q = 0; q < NQ; ++q) {
        double v[NC];
        for (int c = 0; c < NC; ++c) v[c] = f[atq(q, c, l, k, nx, ny)];
        for (int r = 0; r < NC; ++r)
          for (int c = 0; c < NC; ++c) row += v[r] * kw[(q * NC + r) * NC + c] * v[c];
      }
    rows[l] = row;
  }
  double total = 0.0;
  for (int l = 0; l < ny; ++l) total += rows[l];
  free(rows);
  return total;
}

/* Run n steps with zero body load and a fixed (possibly NULL) wall array;
   the pre-collision state is advanced in place.  Used for timing. */
void orc_run(int nx, int ny, int bc, double kK, double km, double* f, double* work,
             double* fstar, long nsteps) {
  double* a = f;
  double* b = work;
  for (long s = 0; s < nsteps; ++s) {
    orc_step(nx, ny, bc, kK, km, 0.0, a, b, NULL, NULL, NULL, NULL, NULL, fstar);
    double* t = a;
    a = b;
    b = t;
  }
  if (a != f) memcpy(f, a, sizeof(double) * (size_t)NQ * NC * nx * ny);
}

/* Number of OpenMP threads a parallel region of the oracle uses. */
int orc_threads(void) { return omp_get_max_threads(); }
