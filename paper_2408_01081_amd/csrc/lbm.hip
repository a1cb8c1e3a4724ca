// HIP implementation (gfx950) of the C ABI in include/lbm.h: the vectorial
// D2Q4^5 lattice Boltzmann scheme for 2D linear elastodynamics
// (Boolakee, Geier, De Lorenzis, arXiv 2408.01081).
//
// Kernels
//   k_init       FP64 second-order initialisation (Eq. ic_second) + first
//                collision, rounded once to FP32 (one pass, 40 B in/80 B out).
//   k_step       fused pull-stream + collide, FP32, memory bound
//                (80 B read + 80 B written per node and step).
//   k_moments    U(t_n) = sum_q f*_q  and the outputs of Section 3.5.
//   k_reduce_*   FP64 block reductions (energy, rel-L2), deterministic order.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"

using namespace lbmk;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const std::string& m) {
  g_err = m;
  return s;
}

lbm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(LBM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------

// ---- FP64 initialisation ---------------------------------------------------
struct InitConst {
  double kK, km, cK, cmu, rho, dx;
  int bc;
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

__device__ inline void node_U(const InitConst& k, const double* v0, const double* s0,
                              int64_t n, int64_t id, double U[NC]) {
  to_U(k, v0[id], v0[n + id], s0[id], s0[n + id], s0[2 * n + id], U);
}

// lattice derivative dx * dU/dx along one axis by central differences
__device__ inline void lattice_grad(const InitConst& k, const double* v0, const double* s0,
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

__global__ __launch_bounds__(256) void k_init(const double* __restrict__ v0,
                                              const double* __restrict__ s0,
                                              const double* __restrict__ grad,
                                              float* __restrict__ dst, Grid g, InitConst k) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);

  double U[NC], UX[NC], UY[NC];
  node_U(k, v0, s0, n, id, U);
  if (grad) {
    // physical derivatives of (v, sigma_bar) -> lattice derivatives of U
    const double* gx = grad;
    const double* gy = grad + 5 * n;
    to_U(k, gx[id], gx[n + id], gx[2 * n + id], gx[3 * n + id], gx[4 * n + id], UX);
    to_U(k, gy[id], gy[n + id], gy[2 * n + id], gy[3 * n + id], gy[4 * n + id], UY);
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
  //   - 1/8 { i UX + (2i^2-1) X(UX) - 2 C_q X(UX) + j UY + (2j^2-1) Y(UY) - 2 C_q Y(UY) }
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
      const double cx = i * UX[c] + (2.0 * i * i - 1.0) * XUX[c] - 2.0 * (i * XXUX[c] + j * YXUX[c]);
      const double cy = j * UY[c] + (2.0 * j * j - 1.0) * YUY[c] - 2.0 * (i * XYUY[c] + j * YYUY[c]);
      f[q][c] = eq - 0.125 * (cx + cy);
    }
  }
  // first collision in FP64 (omega = 2): f* = 2 f_eq(U_num) - f, U_num = sum f
  double Un[NC], Xn[NC], Yn[NC];
  for (int c = 0; c < NC; ++c) Un[c] = (f[0][c] + f[1][c]) + (f[2][c] + f[3][c]);
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

// load pre-collision FP32 populations [4][5][ny][nx] and collide (FP32)
__global__ __launch_bounds__(256) void k_set_populations(const float* __restrict__ fin,
                                                         float* __restrict__ dst, Grid g,
                                                         float kK, float km) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = fin[(q * NC + c) * n + id];
  collide(kK, km, f);
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) dst[pidx(g, q * NC + c, y, x)] = f[q][c];
}

// mode 0: physical moments (v, sigma_bar); 1: U; 2: pre-collision populations
struct MomConst {
  float cK, cmu, rho, kK, km;
  int mode;
};

__global__ __launch_bounds__(256) void k_moments(const float* __restrict__ src,
                                                 float* __restrict__ out, Grid g, MomConst m) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(g, q * NC + c, y, x)];
  if (m.mode == 2) {
    collide(m.kK, m.km, f);  // the omega = 2 collision is an involution
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) out[(q * NC + c) * n + id] = f[q][c];
    return;
  }
  float U[NC];
  for (int c = 0; c < NC; ++c) U[c] = (f[0][c] + f[1][c]) + (f[2][c] + f[3][c]);
  if (m.mode == 1) {
    for (int c = 0; c < NC; ++c) out[c * n + id] = U[c];
    return;
  }
  out[id] = U[0];
  out[n + id] = U[1];
  out[2 * n + id] = -m.rho * (m.cK * U[2] + m.cmu * U[3]);
  out[3 * n + id] = -m.rho * (m.cK * U[2] - m.cmu * U[3]);
  out[4 * n + id] = -m.rho * (m.cmu * U[4]);
}

struct NormConst {
  double k[NQ][NC][NC];
};

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// mode 0: energy sum_q f*^T k_q f* ; mode 1: rel-L2 partial sums vs ref
__global__ __launch_bounds__(RED_THREADS) void k_reduce(const float* __restrict__ src,
                                                        const double* __restrict__ ref, Grid g,
                                                        NormConst nc, int mode,
                                                        double* __restrict__ partial) {
  __shared__ double sh[RED_THREADS];
  const int64_t n = (int64_t)g.nx * g.ny;
  double a = 0.0, b = 0.0;
  for (int64_t id = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * RED_THREADS) {
    const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
    double f[NQ][NC];
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) f[q][c] = (double)src[pidx(g, q * NC + c, y, x)];
    if (mode == 0) {
      for (int q = 0; q < NQ; ++q)
        for (int r = 0; r < NC; ++r) {
          double t = 0.0;
          for (int c = 0; c < NC; ++c) t += nc.k[q][r][c] * f[q][c];
          a += f[q][r] * t;
        }
    } else {
      for (int c = 0; c < NC; ++c) {
        // U from the stored post-collision state, summed in FP32 like the
        // moments kernel, then widened
        const float u32 = ((float)f[0][c] + (float)f[1][c]) + ((float)f[2][c] + (float)f[3][c]);
        const double d = (double)u32 - ref[c * n + id];
        a += d * d;
        b += ref[c * n + id] * ref[c * n + id];
      }
    }
  }
  const double sa = block_sum(a, sh);
  const double sb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa;
    partial[2 * blockIdx.x + 1] = sb;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const double* __restrict__ partial,
                                                              int nblocks,
                                                              double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += RED_THREADS) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  const double sa = block_sum(a, sh);
  const double sb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    out[0] = sa;
    out[1] = sb;
  }
}

// plain streaming copy, 16 bytes per lane and access, nontemporal stores
// (bandwidth and memory-counter reference)
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src,
                                              float4* __restrict__ dst, int64_t n4) {
  typedef float V __attribute__((ext_vector_type(4)));
  const V* s = reinterpret_cast<const V*>(src);
  V* d = reinterpret_cast<V*>(dst);
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  V v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + 256 * k < n4) v[k] = s[i + 256 * k];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i + 256 * k < n4) __builtin_nontemporal_store(v[k], d + i + 256 * k);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Inverse of a symmetric positive definite 5x5 matrix by Cholesky
// factorisation; returns false if the matrix is not positive definite.
bool spd_inverse5(const double A[NC][NC], double inv[NC][NC]) {
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

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Grid g;
  hipStream_t stream;
  float* buf[2];
  double* partial;  // [RED_BLOCKS][2] + [2] result
  int cur;          // buffer holding f*(t_n)
  bool initialised;
  int64_t nstep;
  double cK, cmu, c, kK, km;
  NormConst norm;
  // wall data
  int wall_rank;
  const float* wall_W;
  const float* wall_T;
  int64_t wall_nsteps;
  int device;
  int step_cfg;  // index into kStepConfigs
};

namespace {

struct Derived {
  double cK, cmu, c, kK, km;
};

lbm_status derive(const lbm_params* p, Derived* d) {
  if (!p) return fail(LBM_E_ARG, "null params");
  if (p->nx < 1 || p->ny < 1) return fail(LBM_E_ARG, "nx, ny must be >= 1");
  if (p->bc != LBM_PERIODIC && p->bc != LBM_DIRICHLET) return fail(LBM_E_ARG, "bad bc");
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(LBM_E_ARG, "grid too large");
  if (!(p->dx > 0) || !(p->dt > 0) || !(p->rho > 0) || !(p->mu > 0))
    return fail(LBM_E_ARG, "dx, dt, rho, mu must be positive");
  if (p->flags & ~(uint32_t)LBM_F_PLANE_LAYOUT) return fail(LBM_E_ARG, "unknown flags");
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
  if (!(ratio < 1.0)) {
    char b[160];
    snprintf(b, sizeof b, "CFL-like condition violated: 2 sqrt(cK^2+cmu^2)/c = %.6f >= 1", ratio);
    return fail(LBM_E_CFL, b);
  }
  return LBM_OK;
}

Grid make_grid(const lbm_params* p) {
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

size_t state_bytes(const Grid& g) {
  const int64_t floats = g.plane * NP > g.pitch * g.ny ? g.plane * NP : g.pitch * g.ny;
  return (size_t)round_up(floats * 4, 256);
}

size_t ws_bytes(const Grid& g) {
  return 2 * state_bytes(g) + (size_t)round_up((2 * RED_BLOCKS + 2) * 8, 256);
}

lbm_status launch_check(const char* what) { return hip_check(hipGetLastError(), what); }

lbm_status reduce(lbm_ctx* c, int mode, const double* ref, double out[2]) {
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  int nb = (int)((n + RED_THREADS - 1) / RED_THREADS);
  nb = nb > RED_BLOCKS ? RED_BLOCKS : nb;
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(RED_THREADS), 0, c->stream, c->buf[c->cur], ref,
                     c->g, c->norm, mode, c->partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c->stream, c->partial, nb,
                     c->partial + 2 * RED_BLOCKS);
  lbm_status s = launch_check("reduce launch");
  if (s) return s;
  s = hip_check(hipMemcpyAsync(out, c->partial + 2 * RED_BLOCKS, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream),
                "reduce copy");
  if (s) return s;
  return hip_check(hipStreamSynchronize(c->stream), "reduce sync");
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

size_t lbm_workspace_bytes(const lbm_params* p) {
  Derived d;
  if (derive(p, &d) != LBM_OK) return 0;
  return ws_bytes(make_grid(p));
}

lbm_status lbm_create(const lbm_params* p, void* d_ws, size_t ws_size, void* hip_stream,
                      lbm_ctx** out) {
  if (!out) return fail(LBM_E_ARG, "null out");
  Derived d;
  lbm_status s = derive(p, &d);
  if (s) return s;
  if (!d_ws) return fail(LBM_E_ARG, "null workspace");
  if (((uintptr_t)d_ws & 255) != 0) return fail(LBM_E_ARG, "workspace not 256-byte aligned");
  const Grid g = make_grid(p);
  if (ws_size < ws_bytes(g)) return fail(LBM_E_SPACE, "workspace too small");
  NormConst nc;
  for (int q = 0; q < NQ; ++q) {
    // g_q = 1/4 I + (1/2)(i A_x + j A_y)/c  (Eq. stability_linear), inverted
    const int I[NQ] = {1, 0, -1, 0}, J[NQ] = {0, 1, 0, -1};
    double Ax[NC][NC] = {}, Ay[NC][NC] = {}, gq[NC][NC];
    Ax[0][2] = Ax[2][0] = d.kK;
    Ax[0][3] = Ax[3][0] = d.km;
    Ax[1][4] = Ax[4][1] = d.km;
    Ay[0][4] = Ay[4][0] = d.km;
    Ay[1][2] = Ay[2][1] = d.kK;
    Ay[1][3] = Ay[3][1] = -d.km;
    for (int r = 0; r < NC; ++r)
      for (int c = 0; c < NC; ++c)
        gq[r][c] = (r == c ? 0.25 : 0.0) + 0.5 * (I[q] * Ax[r][c] + J[q] * Ay[r][c]);
    if (!spd_inverse5(gq, nc.k[q])) return fail(LBM_E_CFL, "g_ij not positive definite");
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_E_ARG, "out of host memory");
  c->p = *p;
  c->g = g;
  c->stream = (hipStream_t)hip_stream;
  c->buf[0] = (float*)d_ws;
  c->buf[1] = (float*)((char*)d_ws + state_bytes(g));
  c->partial = (double*)((char*)d_ws + 2 * state_bytes(g));
  c->cur = 0;
  c->initialised = false;
  c->nstep = 0;
  c->cK = d.cK;
  c->cmu = d.cmu;
  c->c = d.c;
  c->kK = d.kK;
  c->km = d.km;
  c->norm = nc;
  c->wall_rank = 0;
  c->wall_W = c->wall_T = nullptr;
  c->wall_nsteps = 0;
  hipGetDevice(&c->device);
  c->step_cfg = default_step_config(g.nx);
  *out = c;
  g_err.clear();
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
  delete c;
  return LBM_OK;
}

lbm_status lbm_lattice_constants(const lbm_ctx* c, double* kK, double* km, double* cc) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (kK) *kK = c->kK;
  if (km) *km = c->km;
  if (cc) *cc = c->c;
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* c, const double* d_v0, const double* d_sigma0, const double* d_grad) {
  if (!c || !d_v0 || !d_sigma0) return fail(LBM_E_ARG, "null argument");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  InitConst k{c->kK, c->km, c->cK, c->cmu, c->p.rho, c->p.dx, c->p.bc};
  hipLaunchKernelGGL(k_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, d_v0,
                     d_sigma0, d_grad, c->buf[0], c->g, k);
  lbm_status s = launch_check("k_init launch");
  if (s) return s;
  c->cur = 0;
  c->nstep = 0;
  c->initialised = true;
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* d_f) {
  if (!c || !d_f) return fail(LBM_E_ARG, "null argument");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  hipLaunchKernelGGL(k_set_populations, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     c->stream, d_f, c->buf[0], c->g, (float)c->kK, (float)c->km);
  lbm_status s = launch_check("k_set_populations launch");
  if (s) return s;
  c->cur = 0;
  c->nstep = 0;
  c->initialised = true;
  return LBM_OK;
}

lbm_status lbm_set_wall_velocity(lbm_ctx* c, int32_t rank, const float* d_W, const float* d_T,
                                 int64_t nsteps) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (rank < 0 || rank > 4096) return fail(LBM_E_ARG, "rank out of range");
  if (rank > 0 && (!d_W || !d_T || nsteps < 0)) return fail(LBM_E_ARG, "null wall table");
  if (rank > 0 && c->p.bc != LBM_DIRICHLET)
    return fail(LBM_E_ARG, "wall data need a Dirichlet problem");
  c->wall_rank = rank;
  c->wall_W = rank ? d_W : nullptr;
  c->wall_T = rank ? d_T : nullptr;
  c->wall_nsteps = rank ? nsteps : 0;
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->nstep : -1; }

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (!c->initialised) return fail(LBM_E_STATE, "lbm_step before lbm_init");
  if (nsteps < 0) return fail(LBM_E_ARG, "negative step count");
  if (c->wall_rank > 0 && c->nstep + nsteps > c->wall_nsteps)
    return fail(LBM_E_ARG, "wall table too short for the requested steps");
  const Grid& g = c->g;
  const StepConfig& cfg = kStepConfigs[c->step_cfg];
  const StepConst sc = step_const(cfg, g, (float)c->kK, (float)c->km);
  const StepFn fn = cfg.fn[c->p.bc];
  for (int64_t s = 0; s < nsteps; ++s) {
    Wall w;
    w.rank = c->wall_rank;
    w.W = c->wall_W;
    w.Trow = c->wall_rank ? c->wall_T + (c->nstep + s) * c->wall_rank : nullptr;
    w.L = 2 * (g.nx + g.ny);
    hipLaunchKernelGGL(fn, dim3(sc.ntiles), dim3(cfg.threads), 0, c->stream,
                       (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], g, sc, w);
    c->cur ^= 1;
  }
  c->nstep += nsteps;
  return launch_check("k_step launch");
}

// ---- launch configurations and the autotuner ------------------------------
namespace {

struct TuneKey {
  int nx, ny, bc;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, bc) < std::tie(o.nx, o.ny, o.bc);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune_cache;
bool g_tune_file_loaded = false;

int find_config(int vec, int threads, int nt, int xmode) {
  for (int i = 0; i < kNumStepConfigs; ++i) {
    const StepConfig& k = kStepConfigs[i];
    if (k.vec == vec && k.threads == threads && k.nt == nt && k.xmode == xmode) return i;
  }
  return -1;
}

// Cache file (path in LBM_AUTOTUNE_CACHE): one line per tuned shape,
// "nx ny bc vec threads nt xmode ms".  Caller holds g_tune_mu.
void load_tune_file() {
  if (g_tune_file_loaded) return;
  g_tune_file_loaded = true;
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  int nx, ny, bc, vec, th, nt, xm;
  double ms;
  while (fscanf(f, "%d %d %d %d %d %d %d %lf", &nx, &ny, &bc, &vec, &th, &nt, &xm, &ms) == 8) {
    const int i = find_config(vec, th, nt, xm);
    if (i >= 0 && step_config_valid(i, nx)) g_tune_cache[TuneKey{nx, ny, bc}] = i;
  }
  fclose(f);
}

void append_tune_file(const TuneKey& k, int i, double ms) {
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  const StepConfig& c = kStepConfigs[i];
  fprintf(f, "%d %d %d %d %d %d %d %.6f\n", k.nx, k.ny, k.bc, c.vec, c.threads, c.nt, c.xmode,
          ms);
  fclose(f);
}

}  // namespace

int32_t lbm_step_config_count(void) { return kNumStepConfigs; }

lbm_status lbm_step_config_info(int32_t index, int32_t* vec, int32_t* threads, int32_t* nt,
                                int32_t* xmode) {
  if (index < 0 || index >= kNumStepConfigs) return fail(LBM_E_ARG, "config index out of range");
  const StepConfig& k = kStepConfigs[index];
  if (vec) *vec = k.vec;
  if (threads) *threads = k.threads;
  if (nt) *nt = k.nt;
  if (xmode) *xmode = k.xmode;
  return LBM_OK;
}

lbm_status lbm_get_step_config(const lbm_ctx* c, int32_t* index) {
  if (!c || !index) return fail(LBM_E_ARG, "null argument");
  *index = c->step_cfg;
  return LBM_OK;
}

lbm_status lbm_set_step_config(lbm_ctx* c, int32_t index) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (!step_config_valid(index, c->g.nx))
    return fail(LBM_E_ARG, "launch configuration not valid for this grid");
  c->step_cfg = index;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t reps, int32_t use_cache, int32_t* h_index,
                        double* h_ms) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (!c->initialised) return fail(LBM_E_STATE, "autotune needs an initialised lattice");
  if (reps < 1) return fail(LBM_E_ARG, "reps must be >= 1");
  const TuneKey key{c->g.nx, c->g.ny, c->p.bc};
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c->step_cfg = it->second;
      if (h_index) *h_index = it->second;
      if (h_ms) *h_ms = -1.0;
      return LBM_OK;
    }
  }
  // Time every valid variant on the live state without changing it: each
  // timed launch reads the current buffer and writes the other one.
  hipEvent_t e0, e1;
  lbm_status s = hip_check(hipEventCreate(&e0), "event");
  if (s) return s;
  s = hip_check(hipEventCreate(&e1), "event");
  if (s) {
    hipEventDestroy(e0);
    return s;
  }
  Wall w;
  w.rank = 0;
  w.W = nullptr;
  w.Trow = nullptr;
  w.L = 2 * (c->g.nx + c->g.ny);
  int best = -1;
  double best_ms = 1e300;
  for (int i = 0; i < kNumStepConfigs && s == LBM_OK; ++i) {
    if (!step_config_valid(i, c->g.nx)) continue;
    const StepConfig& cfg = kStepConfigs[i];
    const StepConst sc = step_const(cfg, c->g, (float)c->kK, (float)c->km);
    for (int r = 0; r < reps + 2; ++r) {
      if (r == 2) hipEventRecord(e0, c->stream);
      hipLaunchKernelGGL(cfg.fn[c->p.bc], dim3(sc.ntiles), dim3(cfg.threads), 0, c->stream,
                         (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], c->g, sc, w);
    }
    hipEventRecord(e1, c->stream);
    s = hip_check(hipEventSynchronize(e1), "autotune sync");
    float ms = 0.f;
    if (s == LBM_OK) s = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing");
    if (s == LBM_OK && ms / reps < best_ms) {
      best_ms = ms / reps;
      best = i;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s) return s;
  if (best < 0) return fail(LBM_E_ARG, "no valid launch configuration");
  c->step_cfg = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    g_tune_cache[key] = best;
    append_tune_file(key, best, best_ms);
  }
  if (h_index) *h_index = best;
  if (h_ms) *h_ms = best_ms;
  return LBM_OK;
}

lbm_status lbm_time_step_config(lbm_ctx* c, int32_t index, int32_t reps, double* h_ms) {
  if (!c || !h_ms) return fail(LBM_E_ARG, "null argument");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  if (!step_config_valid(index, c->g.nx)) return fail(LBM_E_ARG, "invalid configuration");
  if (reps < 1) return fail(LBM_E_ARG, "reps must be >= 1");
  hipEvent_t e0, e1;
  lbm_status s = hip_check(hipEventCreate(&e0), "event");
  if (s) return s;
  s = hip_check(hipEventCreate(&e1), "event");
  if (s) {
    hipEventDestroy(e0);
    return s;
  }
  Wall w;
  w.rank = 0;
  w.W = nullptr;
  w.Trow = nullptr;
  w.L = 2 * (c->g.nx + c->g.ny);
  const StepConfig& cfg = kStepConfigs[index];
  const StepConst sc = step_const(cfg, c->g, (float)c->kK, (float)c->km);
  for (int r = 0; r < reps + 2; ++r) {
    if (r == 2) hipEventRecord(e0, c->stream);
    hipLaunchKernelGGL(cfg.fn[c->p.bc], dim3(sc.ntiles), dim3(cfg.threads), 0, c->stream,
                       (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], c->g, sc, w);
  }
  hipEventRecord(e1, c->stream);
  s = hip_check(hipEventSynchronize(e1), "timing sync");
  float ms = 0.f;
  if (s == LBM_OK) s = hip_check(hipEventElapsedTime(&ms, e0, e1), "timing");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s) return s;
  *h_ms = ms / reps;
  return LBM_OK;
}

static lbm_status moments_mode(lbm_ctx* c, float* out, int mode) {
  if (!c || !out) return fail(LBM_E_ARG, "null argument");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  MomConst m{(float)c->cK, (float)c->cmu, (float)c->p.rho, (float)c->kK, (float)c->km, mode};
  hipLaunchKernelGGL(k_moments, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     c->buf[c->cur], out, c->g, m);
  return launch_check("k_moments launch");
}

lbm_status lbm_moments(lbm_ctx* c, float* d_out) { return moments_mode(c, d_out, 0); }
lbm_status lbm_moments_U(lbm_ctx* c, float* d_U) { return moments_mode(c, d_U, 1); }
lbm_status lbm_populations(lbm_ctx* c, float* d_f) { return moments_mode(c, d_f, 2); }

lbm_status lbm_energy(lbm_ctx* c, double* h_out) {
  if (!c || !h_out) return fail(LBM_E_ARG, "null argument");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  double r[2];
  lbm_status s = reduce(c, 0, nullptr, r);
  if (s) return s;
  *h_out = r[0];
  return LBM_OK;
}

lbm_status lbm_copy_f32(float* d_dst, const float* d_src, int64_t n, void* hip_stream) {
  if (!d_dst || !d_src || n < 0) return fail(LBM_E_ARG, "bad copy arguments");
  if (n % 4 != 0 || ((uintptr_t)d_dst & 15) || ((uintptr_t)d_src & 15))
    return fail(LBM_E_ARG, "copy needs 16-byte aligned buffers and n % 4 == 0");
  if (n == 0) return LBM_OK;
  const int64_t n4 = n / 4;
  const int64_t blocks = (n4 + 1023) / 1024;
  if (blocks > 0x7fffffff) return fail(LBM_E_ARG, "copy too large");
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (const float4*)d_src, (float4*)d_dst, n4);
  return launch_check("k_copy launch");
}

lbm_status lbm_rel_l2(lbm_ctx* c, const double* d_ref, double* h_out) {
  if (!c || !d_ref || !h_out) return fail(LBM_E_ARG, "null argument");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  double r[2];
  lbm_status s = reduce(c, 1, d_ref, r);
  if (s) return s;
  *h_out = r[1] > 0 ? sqrt(r[0] / r[1]) : sqrt(r[0]);
  return LBM_OK;
}

}  // extern "C"
