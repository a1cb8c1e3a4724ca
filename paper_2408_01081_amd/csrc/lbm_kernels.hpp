// Device kernels of the vectorial D2Q4^5 lattice Boltzmann scheme for 2D
// linear elastodynamics (arXiv 2408.01081) on gfx950.
//
// State convention.  The buffer holds the *post-collision* populations f*(t_n)
// in FP32, structure of arrays: 20 planes p = 5 q + c (q in the paper's order
// (1,0),(0,1),(-1,0),(0,-1), c over U = (v_x, v_y, j_s, j_d, j_xy)), each plane
// ny rows of `pitch` floats.  One time step pulls f_q(x, t_{n+1}) = f*_q(x - e_q)
// (Eq. streaming, periodic wrap or the Dirichlet rule Eq. bc_ansatz), forms
// U = sum_q f_q (Eq. cond_eq) and writes f*_q = 1/2 U + C_q U - f_q, which is
// the omega = 2 collision 2 f_eq - f with f_eq of Eq. feq in Courant-number form
// (C_q U = i Phi_x(U)/c + j Phi_y(U)/c).  Because sum_q f*_q = U + dt B/2 and
// the collision is an involution, U(t_n) and the pre-collision populations are
// recovered locally from the stored f*(t_n).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

constexpr int NQ = 4;
constexpr int NC = 5;
constexpr int NP = NQ * NC;

struct Grid {
  int nx, ny;
  int64_t pitch;  // floats per row
  int64_t plane;  // floats per plane
};

struct Wall {
  const float* W;     // [rank][L][2]
  const float* Trow;  // [rank] time functions of this step
  int rank;
  int L;              // 2 (nx + ny)
  // [L][2] velocities of this step already summed over the rank (nullptr: sum
  // W and Trow here); the sum is wall_series below in both cases
  const float* V = nullptr;
};

// Wall velocity du_D/dt at link `link` (Eq. bc_ansatz data), separable form
// sum_r W[r][link] T[r], accumulated in rank order with FMA.
__device__ inline void wall_series(const Wall& w, int link, float& a, float& b) {
  a = 0.f;
  b = 0.f;
  for (int r = 0; r < w.rank; ++r) {
    const float t = w.Trow[r];
    const float* p = w.W + ((int64_t)r * w.L + link) * 2;
    a = fmaf(p[0], t, a);
    b = fmaf(p[1], t, b);
  }
}

__device__ inline void wall_velocity(const Wall& w, int link, float& a, float& b) {
  if (w.V) {
    a = w.V[2 * link];
    b = w.V[2 * link + 1];
    return;
  }
  wall_series(w, link, a, b);
}

// Dirichlet rule for a missing population q (direction (i,j)):
//   f_q = D f*_{qbar}(x) + S_q,  D = diag(-1,-1,1,1,1)  (Eq. bc_d),
//   S_q = (a/2, b/2, kK (i a + j b), km (i a - j b), km (j a + i b))  (Eq. bc_s
//   in Courant-number form).
__device__ inline void wall_rule(int i, int j, float kK, float km, float a, float b,
                                 const float fb[NC], float out[NC]) {
  out[0] = 0.5f * a - fb[0];
  out[1] = 0.5f * b - fb[1];
  out[2] = fb[2] + kK * (float)(i) * a + kK * (float)(j) * b;
  out[3] = fb[3] + km * (float)(i) * a - km * (float)(j) * b;
  out[4] = fb[4] + km * (float)(j) * a + km * (float)(i) * b;
}

// Zeroth moment sum_q f_q of one node (the scheme's U without the load term),
// summed as f_2 + (f_0 + (f_1 + f_3)): the y neighbours first, then one x
// neighbour at a time, the order in which the blocked kernel's cross-lane
// adds can consume them.
__device__ inline void moment0(const float f[NQ][NC], float U[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) U[c] = f[2][c] + (f[0][c] + (f[1][c] + f[3][c]));
}

// omega = 2 collision of one node for a given moment U:
// f*_q = 2 f_eq,q(U) - f_q = (U/2 + s_q C U) - f_q (Eq. feq), the first
// bracket as one fused multiply-add (U/2 is exact, so this rounds as the sum
// of h = U/2 and s_q C U would).  Written once so every kernel variant
// rounds identically.
__device__ inline void collide_with(float kK, float km, const float U[NC], float f[NQ][NC]) {
  // X = Phi_x(U)/c, Y = Phi_y(U)/c
  const float X0 = fmaf(kK, U[2], km * U[3]);
  const float X1 = km * U[4];
  const float X2 = kK * U[0];
  const float X3 = km * U[0];
  const float X4 = km * U[1];
  const float Y0 = km * U[4];
  const float Y1 = fmaf(kK, U[2], -(km * U[3]));
  const float Y2 = kK * U[1];
  const float Y3 = -(km * U[1]);
  const float Y4 = km * U[0];
  const float X[NC] = {X0, X1, X2, X3, X4};
  const float Y[NC] = {Y0, Y1, Y2, Y3, Y4};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    f[0][c] = fmaf(0.5f, U[c], X[c]) - f[0][c];
    f[1][c] = fmaf(0.5f, U[c], Y[c]) - f[1][c];
    f[2][c] = fmaf(0.5f, U[c], -X[c]) - f[2][c];
    f[3][c] = fmaf(0.5f, U[c], -Y[c]) - f[3][c];
  }
}

// Collision without body load (U = sum_q f_q).
__device__ inline void collide(float kK, float km, float f[NQ][NC]) {
  float U[NC];
  moment0(f, U);
  collide_with(kK, km, U, f);
}

// Separable physical body load b_bar_c(x_k, y_l, t) = sum_r X[r][c][k] Y[r][l] T_r(t)
// of one time level; the scheme uses B_hat = dt b = (dt / rho) b_bar on the
// velocity components (Eq. cond_eq: U_num = sum_q f_q + B_hat / 2).
struct Force {
  const float* X;     // [rank][2][nx]
  const float* Y;     // [rank][ny]
  const float* Trow;  // [rank] time functions of this time level
  int rank, nx, ny;
  float scale;        // dt / rho
};

__device__ inline void body_hat(const Force& F, int x, int y, float& bx, float& by) {
  float a = 0.f, b = 0.f;
  for (int r = 0; r < F.rank; ++r) {
    const float yt = F.Y[(int64_t)r * F.ny + y] * F.Trow[r];
    const float* X = F.X + (int64_t)r * 2 * F.nx;
    a = fmaf(X[x], yt, a);
    b = fmaf(X[F.nx + x], yt, b);
  }
  bx = F.scale * a;
  by = F.scale * b;
}

}  // namespace lbmk
