// Host-side helpers shared by the single-lattice and batched entry points:
// error reporting, parameter validation (Eq. stab_cond), lattice layout and
// the norm weights k_ij = g_ij^{-1} (Eq. def_symmetrizer).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <string>

#include "lbm.h"
#include "lbm_kernels.hpp"

namespace lbmh {

using lbmk::Grid;
using lbmk::NC;
using lbmk::NP;
using lbmk::NQ;

extern thread_local std::string g_err;

inline lbm_status fail(lbm_status s, const std::string& m) {
  g_err = m;
  return s;
}

inline lbm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(LBM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

inline lbm_status launch_check(const char* what) { return hip_check(hipGetLastError(), what); }

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Inverse of a symmetric positive definite 5x5 matrix by Cholesky
// factorisation; returns false if the matrix is not positive definite.
inline bool spd_inverse5(const double A[NC][NC], double inv[NC][NC]) {
  double Lm[NC][NC] = {};
  for (int i = 0; i < NC; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= Lm[i][k] * Lm[j][k];
      if (i == j) {
        if (s <= 0.0) return false;
        Lm[i][i] = sqrt(s);
      } else {
        Lm[i][j] = s / Lm[j][j];
      }
    }
  // solve A x = e_k column by column
  for (int k = 0; k < NC; ++k) {
    double z[NC], xk[NC];
    for (int i = 0; i < NC; ++i) {
      double s = (i == k) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) s -= Lm[i][j] * z[j];
      z[i] = s / Lm[i][i];
    }
    for (int i = NC - 1; i >= 0; --i) {
      double s = z[i];
      for (int j = i + 1; j < NC; ++j) s -= Lm[j][i] * xk[j];
      xk[i] = s / Lm[i][i];
    }
    for (int i = 0; i < NC; ++i) inv[i][k] = xk[i];
  }
  return true;
}


struct Derived {
  double cK, cmu, c, kK, km;
};

inline lbm_status derive(const lbm_params* p, Derived* d) {
  if (!p) return fail(LBM_E_ARG, "null params");
  if (p->nx < 1 || p->ny < 1) return fail(LBM_E_ARG, "nx, ny must be >= 1");
  if (p->bc != LBM_PERIODIC && p->bc != LBM_DIRICHLET) return fail(LBM_E_ARG, "bad bc");
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(LBM_E_ARG, "grid too large");
  // mu = 0 (c_mu = 0, the limit of Section 6.1's material list) is admitted;
  // such a lattice is initialised from the displacement gradient
  // (lbm_init_from_gradient), since the stress form divides by c_mu
  if (!(p->dx > 0) || !(p->dt > 0) || !(p->rho > 0) || !(p->mu >= 0))
    return fail(LBM_E_ARG, "dx, dt, rho must be positive and mu non-negative");
  if (p->flags & ~(uint32_t)(LBM_F_PLANE_LAYOUT | LBM_F_DISPLACEMENT | LBM_F_ALLOW_UNSTABLE))
    return fail(LBM_E_ARG, "unknown flags");
  double lam = p->lambda;
  if (p->model == LBM_PLANE_STRESS) {
    if (!(lam + 2.0 * p->mu > 0)) return fail(LBM_E_ARG, "lambda + 2 mu must be positive");
    lam = 2.0 * lam * p->mu / (lam + 2.0 * p->mu);
  } else if (p->model != LBM_PLANE_STRAIN && p->model != LBM_CONTINUUM_2D) {
    return fail(LBM_E_ARG, "bad model");
  }
  const double cK2 = (lam + p->mu) / p->rho;
  if (!(cK2 > 0)) return fail(LBM_E_ARG, "lambda + mu must be positive");
  d->cK = sqrt(cK2);
  d->cmu = sqrt(p->mu / p->rho);
  d->c = p->dx / p->dt;
  d->kK = d->cK / d->c;
  d->km = d->cmu / d->c;
  const double ratio = 2.0 * sqrt(d->kK * d->kK + d->km * d->km);
  if (!(ratio < 1.0) && !(p->flags & LBM_F_ALLOW_UNSTABLE)) {
    char b[160];
    snprintf(b, sizeof b, "CFL-like condition violated: 2 sqrt(cK^2+cmu^2)/c = %.6f >= 1", ratio);
    return fail(LBM_E_CFL, b);
  }
  return LBM_OK;
}

inline Grid make_grid(const lbm_params* p) {
  Grid g;
  g.nx = p->nx;
  g.ny = p->ny;
  const int64_t rowlen = round_up(p->nx, 64);  // floats of one plane row, 256-byte aligned
  if (p->flags & LBM_F_PLANE_LAYOUT) {
    // [plane][y][x]; plane starts staggered by 256 bytes modulo 16 KiB so the
    // 40 concurrent streams of a step do not start on the same channel
    g.pitch = rowlen;
    g.plane = round_up(rowlen * p->ny, 4096) + 64;
  } else {
    // [y][plane][x]: the 20 plane rows of one lattice row are contiguous, so a
    // workgroup's reads come from three contiguous 20-row blocks and its writes
    // go to one (measured 6.0 vs 5.45 TB/s on a 4096^2 step)
    g.plane = rowlen;
    g.pitch = rowlen * NP;
  }
  return g;
}

inline size_t state_bytes(const Grid& g) {
  const int64_t floats = g.plane * NP > g.pitch * g.ny ? g.plane * NP : g.pitch * g.ny;
  return (size_t)round_up(floats * 4, 256);
}


// k_ij = g_ij^{-1} with g_ij = 1/4 I + (1/2)(i A_x + j A_y)/c (Eq. stability_linear)
inline bool norm_weights(double kK, double km, double out[NQ][NC][NC]) {
  const int I[NQ] = {1, 0, -1, 0}, J[NQ] = {0, 1, 0, -1};
  double Ax[NC][NC] = {}, Ay[NC][NC] = {};
  Ax[0][2] = Ax[2][0] = kK;
  Ax[0][3] = Ax[3][0] = km;
  Ax[1][4] = Ax[4][1] = km;
  Ay[0][4] = Ay[4][0] = km;
  Ay[1][2] = Ay[2][1] = kK;
  Ay[1][3] = Ay[3][1] = -km;
  for (int q = 0; q < NQ; ++q) {
    double gq[NC][NC];
    for (int r = 0; r < NC; ++r)
      for (int c = 0; c < NC; ++c)
        gq[r][c] = (r == c ? 0.25 : 0.0) + 0.5 * (I[q] * Ax[r][c] + J[q] * Ay[r][c]);
    if (!spd_inverse5(gq, out[q])) return false;
  }
  return true;
}

}  // namespace lbmh
