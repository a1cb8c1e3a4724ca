// FP64 second-order initialisation (Eq. ic_second) shared by the single-lattice
// and batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"

namespace lbmk {

// What the two field arrays of an initialisation hold: (v0, Cauchy stress)
// or (v0, displacement gradient of u0)
constexpr int INIT_FROM_STRESS = 0;
constexpr int INIT_FROM_GRADIENT = 1;

struct InitConst {
  double kK, km, cK, cmu, rho, dx;
  int bc;
  int src = INIT_FROM_STRESS;
};

// Phi_x(V)/c and Phi_y(V)/c in double precision
__device__ inline void flux_x(const InitConst& k, const double V[NC], double o[NC]) {
  o[0] = k.kK * V[2] + k.km * V[3];
  o[1] = k.km * V[4];
  o[2] = k.kK * V[0];
  o[3] = k.km * V[0];
  o[4] = k.km * V[1];
}
__device__ inline void flux_y(const InitConst& k, const double V[NC], double o[NC]) {
  o[0] = k.km * V[4];
  o[1] = k.kK * V[2] - k.km * V[3];
  o[2] = k.kK * V[1];
  o[3] = -k.km * V[1];
  o[4] = k.km * V[0];
}

// U = (v, j) from velocity and Cauchy stress at a node (inverse of Eq. sigma_num)
__device__ inline void to_U(const InitConst& k, double vx, double vy, double sxx, double syy,
                            double sxy, double U[NC]) {
  const double r = 1.0 / k.rho;
  U[0] = vx;
  U[1] = vy;
  U[2] = -(sxx + syy) * r / (2.0 * k.cK);
  U[3] = -(sxx - syy) * r / (2.0 * k.cmu);
  U[4] = -sxy * r / k.cmu;
}

// U0 at a node from the initial data: with INIT_FROM_STRESS s0 is the Cauchy
// stress [3][ny][nx]; with INIT_FROM_GRADIENT it is the displacement
// gradient [4][ny][nx] (du_x/dx, du_x/dy, du_y/dx, du_y/dy) and U0 follows
// Eq. ic_vector directly, j = -c (derivatives of u0), with no division by
// c_mu (so c_mu = 0 is allowed)
// Eq. ic_vector: U from v and the displacement gradient (uxx = du_x/dx,
// uxy = du_x/dy, uyx = du_y/dx, uyy = du_y/dy); linear, so it also maps
// derivatives of these fields to derivatives of U
__device__ inline void from_gradient(const InitConst& k, double vx, double vy, double uxx,
                                     double uxy, double uyx, double uyy, double U[NC]) {
  U[0] = vx;
  U[1] = vy;
  U[2] = -k.cK * (uxx + uyy);
  U[3] = -k.cmu * (uxx - uyy);
  U[4] = -k.cmu * (uyx + uxy);
}

template <typename T>
__device__ inline void node_U(const InitConst& k, const T* v0, const T* s0, int64_t n, int64_t id,
                              double U[NC]) {
  if (k.src == INIT_FROM_GRADIENT) {
    from_gradient(k, v0[id], v0[n + id], s0[id], s0[n + id], s0[2 * n + id], s0[3 * n + id], U);
    return;
  }
  to_U(k, (double)v0[id], (double)v0[n + id], (double)s0[id], (double)s0[n + id],
       (double)s0[2 * n + id], U);
}

// lattice derivative dx * dU/dx along one axis by central differences
template <typename T>
__device__ inline void lattice_grad(const InitConst& k, const T* v0, const T* s0,
                                    int nx, int ny, int x, int y, int axis, double G[NC]) {
  const int64_t n = (int64_t)nx * ny;
  const int m = axis == 0 ? x : y, len = axis == 0 ? nx : ny;
  auto id_of = [&](int mm) -> int64_t {
    return axis == 0 ? (int64_t)y * nx + mm : (int64_t)mm * nx + x;
  };
  double A[NC], B[NC], C[NC];
  if (len == 1) {
    for (int c = 0; c < NC; ++c) G[c] = 0.0;
    return;
  }
  if (k.bc == LBM_PERIODIC || (m > 0 && m < len - 1)) {
    const int mp = m + 1 == len ? 0 : m + 1, mm = m == 0 ? len - 1 : m - 1;
    node_U(k, v0, s0, n, id_of(mp), A);
    node_U(k, v0, s0, n, id_of(mm), B);
    for (int c = 0; c < NC; ++c) G[c] = 0.5 * (A[c] - B[c]);
    return;
  }
  if (len == 2) {
    node_U(k, v0, s0, n, id_of(1), A);
    node_U(k, v0, s0, n, id_of(0), B);
    for (int c = 0; c < NC; ++c) G[c] = A[c] - B[c];
    return;
  }
  // one-sided second order at a wall
  const int s = m == 0 ? 1 : -1;
  node_U(k, v0, s0, n, id_of(m), A);
  node_U(k, v0, s0, n, id_of(m + s), B);
  node_U(k, v0, s0, n, id_of(m + 2 * s), C);
  for (int c = 0; c < NC; ++c) G[c] = s * 0.5 * (-3.0 * A[c] + 4.0 * B[c] - C[c]);
}

// B_hat(x, y, t_0) = (dt / rho) b_bar in FP64 from the separable tables (zero
// without a load)
__device__ inline void body_hat0(const Force& F, int x, int y, double& bx, double& by) {
  double a = 0.0, b = 0.0;
  for (int r = 0; r < F.rank; ++r) {
    const double yt = (double)F.Y[(int64_t)r * F.ny + y] * (double)F.Trow[r];
    const float* X = F.X + (int64_t)r * 2 * F.nx;
    a += (double)X[x] * yt;
    b += (double)X[F.nx + x] * yt;
  }
  bx = (double)F.scale * a;
  by = (double)F.scale * b;
}

// Populations f*(0) of one node (x, y): Eq. ic_second in FP64 followed by the
// first omega = 2 collision, rounded once to FP32.  v0 [2][ny][nx] and s0
// (Cauchy stress [3][ny][nx], or the displacement gradient [4][ny][nx] with
// INIT_FROM_GRADIENT) are the instance's fields (double or float); grad is
// nullable FP64 physical derivatives d/dx, d/dy of the input fields:
// [2][5][ny][nx] of (v, sigma_bar), or [2][6][ny][nx] of (v, grad u0) with
// INIT_FROM_GRADIENT; F the body load at t_0 (rank 0: none).
template <typename T>
__device__ inline void init_node(const T* __restrict__ v0, const T* __restrict__ s0,
                                 const double* __restrict__ grad, float* __restrict__ dst,
                                 const Grid& g, const InitConst& k, int x, int y,
                                 const Force& F = Force{}) {
  const int64_t n = (int64_t)g.nx * g.ny;
  const int64_t id = (int64_t)y * g.nx + x;
  double U[NC], UX[NC], UY[NC];
  node_U(k, v0, s0, n, id, U);
  if (grad) {
    // physical derivatives of the input fields -> lattice derivatives of U
    if (k.src == INIT_FROM_GRADIENT) {
      const double* gx = grad;
      const double* gy = grad + 6 * n;
      from_gradient(k, gx[id], gx[n + id], gx[2 * n + id], gx[3 * n + id], gx[4 * n + id],
                    gx[5 * n + id], UX);
      from_gradient(k, gy[id], gy[n + id], gy[2 * n + id], gy[3 * n + id], gy[4 * n + id],
                    gy[5 * n + id], UY);
    } else {
      const double* gx = grad;
      const double* gy = grad + 5 * n;
      to_U(k, gx[id], gx[n + id], gx[2 * n + id], gx[3 * n + id], gx[4 * n + id], UX);
      to_U(k, gy[id], gy[n + id], gy[2 * n + id], gy[3 * n + id], gy[4 * n + id], UY);
    }
    for (int c = 0; c < NC; ++c) {
      UX[c] *= k.dx;
      UY[c] *= k.dx;
    }
  } else {
    lattice_grad(k, v0, s0, g.nx, g.ny, x, y, 0, UX);
    lattice_grad(k, v0, s0, g.nx, g.ny, x, y, 1, UY);
  }

  // Eq. ic_second in lattice units (c dt = dx absorbed into UX, UY):
  // f_q = 1/4 [U + 2 C_q U]
  //   - 1/8 { B + 2 C_q B + i UX + (2i^2-1) X(UX) - 2 C_q X(UX)
  //           + j UY + (2j^2-1) Y(UY) - 2 C_q Y(UY) },  B = (B_hat_x, B_hat_y, 0, 0, 0)
  double Bh[NC] = {0.0, 0.0, 0.0, 0.0, 0.0}, XB[NC], YB[NC];
  if (F.rank > 0) body_hat0(F, x, y, Bh[0], Bh[1]);
  flux_x(k, Bh, XB);
  flux_y(k, Bh, YB);
  double XU[NC], YU[NC], XUX[NC], YUY[NC], XXUX[NC], YXUX[NC], XYUY[NC], YYUY[NC];
  flux_x(k, U, XU);
  flux_y(k, U, YU);
  flux_x(k, UX, XUX);
  flux_y(k, UY, YUY);
  flux_x(k, XUX, XXUX);
  flux_y(k, XUX, YXUX);
  flux_x(k, YUY, XYUY);
  flux_y(k, YUY, YYUY);
  const int I[NQ] = {1, 0, -1, 0}, J[NQ] = {0, 1, 0, -1};
  double f[NQ][NC];
  for (int q = 0; q < NQ; ++q) {
    const double i = I[q], j = J[q];
    for (int c = 0; c < NC; ++c) {
      const double eq = 0.25 * (U[c] + 2.0 * (i * XU[c] + j * YU[c]));
      const double cb = Bh[c] + 2.0 * (i * XB[c] + j * YB[c]);
      const double cx = i * UX[c] + (2.0 * i * i - 1.0) * XUX[c] - 2.0 * (i * XXUX[c] + j * YXUX[c]);
      const double cy = j * UY[c] + (2.0 * j * j - 1.0) * YUY[c] - 2.0 * (i * XYUY[c] + j * YYUY[c]);
      f[q][c] = eq - 0.125 * (cb + cx + cy);
    }
  }
  // first collision in FP64 (omega = 2): f* = 2 f_eq(U_num) - f, U_num = sum f
  double Un[NC], Xn[NC], Yn[NC];
  for (int c = 0; c < NC; ++c) Un[c] = (f[0][c] + f[1][c]) + (f[2][c] + f[3][c]) + 0.5 * Bh[c];
  flux_x(k, Un, Xn);
  flux_y(k, Un, Yn);
  for (int q = 0; q < NQ; ++q) {
    const double i = I[q], j = J[q];
    for (int c = 0; c < NC; ++c) {
      const double fs = 0.5 * Un[c] + (i * Xn[c] + j * Yn[c]) - f[q][c];
      dst[pidx(g, q * NC + c, y, x)] = (float)fs;
    }
  }
}


}  // namespace lbmk
