// HIP implementation (gfx950) of the C ABI in include/lbm.h: the vectorial
// D2Q4^5 lattice Boltzmann scheme for 2D linear elastodynamics
// (Boolakee, Geier, De Lorenzis, arXiv 2408.01081).
//
// Kernels
//   k_init       FP64 second-order initialisation (Eq. ic_second) + first
//                collision, rounded once to FP32 (one pass, 40 B in/80 B out).
//   k_step       fused pull-stream + collide, FP32, memory bound
//                (80 B read + 80 B written per node and step).
//   k_moments    U(t_n) = sum_q f*_q - B_hat(t_n)/2 and the outputs of Section 3.5.
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
#include "lbm_tblock.hpp"
#include "lbm_tb_tables.hpp"
#include "lbm_init.hpp"
#include "lbm_host.hpp"

thread_local std::string lbmh::g_err;
using namespace lbmh;

using namespace lbmk;

namespace {

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;



// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_init(const double* __restrict__ v0,
                                              const double* __restrict__ s0,
                                              const double* __restrict__ grad,
                                              float* __restrict__ dst, Grid g, InitConst k,
                                              Force F) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  init_node<double>(v0, s0, grad, dst, g, k, x, y, F);
}

// U_num(t_n) of a node from its stored post-collision populations:
// sum_q f*_q = U_num + B_hat / 2, so U_num = sum_q f*_q - B_hat / 2
__device__ inline void node_moment(const float f[NQ][NC], const Force& F, int x, int y,
                                   float U[NC]) {
  moment0(f, U);
  if (F.rank > 0) {
    float bx, by;
    body_hat(F, x, y, bx, by);
    U[0] -= 0.5f * bx;
    U[1] -= 0.5f * by;
  }
}

// Displacement state after initialisation: D = u0 + dt/2 v_num(t_0)
__global__ __launch_bounds__(256) void k_init_disp(const float* __restrict__ src,
                                                   const double* __restrict__ u0,
                                                   double* __restrict__ D, Grid g, Force F,
                                                   double half_dt) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC], U[NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(g, q * NC + c, y, x)];
  node_moment(f, F, x, y, U);
  for (int d = 0; d < 2; ++d) D[d * n + id] = u0[d * n + id] + half_dt * (double)U[d];
}

// Displacement output u(t_n) = D - dt/2 v_num(t_n) (D holds u(t_n) + dt/2 v_num(t_n))
__global__ __launch_bounds__(256) void k_displacement(const float* __restrict__ src,
                                                      const double* __restrict__ D,
                                                      float* __restrict__ out, Grid g, Force F,
                                                      double half_dt) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC], U[NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(g, q * NC + c, y, x)];
  node_moment(f, F, x, y, U);
  for (int d = 0; d < 2; ++d) out[d * n + id] = (float)(D[d * n + id] - half_dt * (double)U[d]);
}

// load pre-collision FP32 populations [4][5][ny][nx] and collide (FP32)
__global__ __launch_bounds__(256) void k_set_populations(const float* __restrict__ fin,
                                                         float* __restrict__ dst, Grid g,
                                                         float kK, float km, Force F) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = fin[(q * NC + c) * n + id];
  if (F.rank > 0) {
    float U[NC];
    moment0(f, U);
    float bx, by;
    body_hat(F, x, y, bx, by);
    U[0] += 0.5f * bx;
    U[1] += 0.5f * by;
    collide_with(kK, km, U, f);
  } else {
    collide(kK, km, f);
  }
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) dst[pidx(g, q * NC + c, y, x)] = f[q][c];
}

// mode 0: physical moments (v, sigma_bar); 1: U; 2: pre-collision populations
struct MomConst {
  float cK, cmu, rho, kK, km;
  int mode;
};

__global__ __launch_bounds__(256) void k_moments(const float* __restrict__ src,
                                                 float* __restrict__ out, Grid g, MomConst m,
                                                 Force F) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)g.nx * g.ny;
  if (id >= n) return;
  const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
  float f[NQ][NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(g, q * NC + c, y, x)];
  if (m.mode == 2) {
    // f = 2 f_eq(U_num) - f*: without a load the collision is an involution
    if (F.rank > 0) {
      float U[NC];
      node_moment(f, F, x, y, U);
      collide_with(m.kK, m.km, U, f);
    } else {
      collide(m.kK, m.km, f);
    }
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) out[(q * NC + c) * n + id] = f[q][c];
    return;
  }
  float U[NC];
  node_moment(f, F, x, y, U);
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

// mode 0: energy sum_q f^T k_q f of the pre-collision populations (without
// a load the collision is an isometry of this norm, so f* serves); mode 1:
// rel-L2 partial sums of U_num vs ref
__global__ __launch_bounds__(RED_THREADS) void k_reduce(const float* __restrict__ src,
                                                        const double* __restrict__ ref, Grid g,
                                                        NormConst nc, int mode,
                                                        double* __restrict__ partial, Force F,
                                                        float kK, float km) {
  __shared__ double sh[RED_THREADS];
  const int64_t n = (int64_t)g.nx * g.ny;
  double a = 0.0, b = 0.0;
  for (int64_t id = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * RED_THREADS) {
    const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
    double f[NQ][NC];
    float fs[NQ][NC];
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) fs[q][c] = src[pidx(g, q * NC + c, y, x)];
    if (F.rank > 0 && mode == 0) {
      float U[NC];
      node_moment(fs, F, x, y, U);
      collide_with(kK, km, U, fs);
    }
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) f[q][c] = (double)fs[q][c];
    if (mode == 0) {
      for (int q = 0; q < NQ; ++q)
        for (int r = 0; r < NC; ++r) {
          double t = 0.0;
          for (int c = 0; c < NC; ++c) t += nc.k[q][r][c] * f[q][c];
          a += f[q][r] * t;
        }
    } else {
      // U from the stored post-collision state, in FP32 like the moments
      // kernel, then widened
      float U[NC];
      node_moment(fs, F, x, y, U);
      for (int c = 0; c < NC; ++c) {
        const double d = (double)U[c] - ref[c * n + id];
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

// ---- space-time error norms against an exact solution (Section 6.1) -------
// Exact fields of the outputs in separable form, FP64:
//   phi_c(x_k, y_l, t_n) = sum_r X[r][c][k] Y[r][l] T[n][r],
// c = u_x, u_y, v_x, v_y, sigma_bar_xx, sigma_bar_yy, sigma_bar_xy.
struct RefTable {
  const double* X;     // [rank][ERR_C][nx]
  const double* Y;     // [rank][ny]
  const double* Trow;  // [rank] of this time level
  int rank, nx, ny;
};
constexpr int ERR_C = 7;
// per group (0: u, 1: v, 2: sigma_bar): sum |e|^2, sum |exact|^2, max |e|_inf
constexpr int ERR_VALS = 9;
constexpr int ERR_ACC = ERR_VALS + 1;  // + number of levels added

__device__ inline double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per-block error sums of one time level: numerical outputs formed exactly as
// the moments and displacement kernels form them (U in FP32, u in FP64),
// compared in FP64 with the exact fields.
__global__ __launch_bounds__(RED_THREADS) void k_err_partial(const float* __restrict__ src,
                                                             const double* __restrict__ D,
                                                             Grid g, Force F, RefTable R,
                                                             MomConst m, double half_dt,
                                                             double* __restrict__ partial) {
  __shared__ double sh[RED_THREADS];
  const int64_t n = (int64_t)g.nx * g.ny;
  double e2[3] = {0, 0, 0}, x2[3] = {0, 0, 0}, em[3] = {0, 0, 0};
  for (int64_t id = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * RED_THREADS) {
    const int y = (int)(id / g.nx), x = (int)(id - (int64_t)y * g.nx);
    float f[NQ][NC], U[NC];
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(g, q * NC + c, y, x)];
    node_moment(f, F, x, y, U);
    double num[ERR_C];
    num[0] = D ? D[id] - half_dt * (double)U[0] : 0.0;
    num[1] = D ? D[n + id] - half_dt * (double)U[1] : 0.0;
    num[2] = U[0];
    num[3] = U[1];
    num[4] = -m.rho * (m.cK * U[2] + m.cmu * U[3]);
    num[5] = -m.rho * (m.cK * U[2] - m.cmu * U[3]);
    num[6] = -m.rho * (m.cmu * U[4]);
    double ex[ERR_C] = {0, 0, 0, 0, 0, 0, 0};
    for (int r = 0; r < R.rank; ++r) {
      const double yt = R.Y[(int64_t)r * R.ny + y] * R.Trow[r];
      const double* X = R.X + (int64_t)r * ERR_C * R.nx + x;
      for (int c = 0; c < ERR_C; ++c) ex[c] = fma(X[(int64_t)c * R.nx], yt, ex[c]);
    }
    for (int c = D ? 0 : 2; c < ERR_C; ++c) {
      const int grp = c < 2 ? 0 : (c < 4 ? 1 : 2);
      const double d = num[c] - ex[c];
      e2[grp] += d * d;
      x2[grp] += ex[c] * ex[c];
      em[grp] = fmax(em[grp], fabs(d));
    }
  }
  for (int k = 0; k < 3; ++k) {
    const double a = block_sum(e2[k], sh);
    const double b = block_sum(x2[k], sh);
    const double c = block_max(em[k], sh);
    if (threadIdx.x == 0) {
      partial[ERR_VALS * blockIdx.x + 3 * k] = a;
      partial[ERR_VALS * blockIdx.x + 3 * k + 1] = b;
      partial[ERR_VALS * blockIdx.x + 3 * k + 2] = c;
    }
  }
}

// Adds one level's block partials (fixed order) to the running sums.
__global__ __launch_bounds__(RED_THREADS) void k_err_final(const double* __restrict__ partial,
                                                           int nblocks, double* __restrict__ acc) {
  __shared__ double sh[RED_THREADS];
  for (int k = 0; k < ERR_VALS; ++k) {
    const bool is_max = k % 3 == 2;
    double v = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += RED_THREADS) {
      const double p = partial[ERR_VALS * i + k];
      v = is_max ? fmax(v, p) : v + p;
    }
    const double r = is_max ? block_max(v, sh) : block_sum(v, sh);
    if (threadIdx.x == 0) acc[k] = is_max ? fmax(acc[k], r) : acc[k] + r;
  }
  if (threadIdx.x == 0) acc[ERR_VALS] += 1.0;
}

__global__ void k_err_zero(double* acc) {
  if (threadIdx.x < ERR_ACC) acc[threadIdx.x] = 0.0;
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
  int step_cfg;   // index into kStepConfigs
  int tb_cfg;         // index into kTBVariants, or -1 (single steps only)
  int tb_slots[64];   // resident waves of a blocked variant on this device (0: not known)
  int tbf_slots[48];  // the same for the variants with a load / displacement (3 per variant)
  int tb_rem[TB_MAX_STEPS + 1];  // variant for the last r = 2 .. 10 steps of a run (-1: nearest shape)
  // launch times the autotuner measured for this shape (ms; -1: not timed):
  // every blocked variant, and the best single-step configuration
  double tb_launch_ms[kNumTBVariants];
  double step_launch_ms;
  // split Dirichlet blocked launches (mode -1, the default, or 1: wherever a
  // split kernel exists and the lattice allows; 0: never): the wall band
  // with the Dirichlet rule and the interior with the periodic kernel's
  // code, in one launch
  int tb_split;
  int tbs_slots[8];  // resident waves of a split kernel on this device (0: not known)
  float* wall_v;        // [WALL_CHUNK][2 (nx + ny)][2] wall velocities of upcoming steps
  // separable body load (rank 0: none); row n of force_T belongs to t_n
  const float* force_X;
  const float* force_Y;
  const float* force_T;
  int force_rank;
  int64_t force_nsteps;
  float* force_rows;  // [8][ny][TB_MAXR] row factors of a blocked launch with a load
  double* disp;  // [2][ny][nx] FP64 displacement state D, or null (LBM_F_DISPLACEMENT)
  bool disp_ready;
  // exact solution for the error norms (rank 0: none)
  const double* ref_X;
  const double* ref_Y;
  const double* ref_T;
  int ref_rank;
  int64_t ref_nsteps;
  bool err_on;
  double* err_part;  // [RED_BLOCKS][ERR_VALS] block partials
  double* err_acc;   // [ERR_ACC] running sums
};

namespace {

// most steps whose wall velocities are summed ahead in one launch; a lattice
// stepping T per blocked launch uses chunks of floor(WALL_CHUNK / T) T steps
// so that blocked launches fill every chunk
constexpr int WALL_CHUNK = 420;

// the wall-velocity table exists for Dirichlet lattices only
size_t wall_table_bytes(const Grid& g, int bc) {
  if (bc != LBM_DIRICHLET) return 0;
  return (size_t)round_up((int64_t)WALL_CHUNK * 2 * (g.nx + g.ny) * 2 * 4, 256);
}

size_t disp_bytes(const Grid& g, uint32_t flags) {
  if (!(flags & LBM_F_DISPLACEMENT)) return 0;
  return (size_t)round_up((int64_t)2 * g.nx * g.ny * 8, 256);
}

constexpr size_t ERR_BYTES = (size_t)(RED_BLOCKS * ERR_VALS + 16) * 8;

size_t force_rows_bytes(const Grid& g) {
  return (size_t)round_up((int64_t)8 * g.ny * TB_MAXR * 4, 256);
}

size_t ws_bytes(const Grid& g, int bc, uint32_t flags) {
  return 2 * state_bytes(g) + (size_t)round_up((2 * RED_BLOCKS + 2) * 8, 256) +
         wall_table_bytes(g, bc) + disp_bytes(g, flags) + round_up(ERR_BYTES, 256) +
         force_rows_bytes(g);
}

RefTable ref_at(const lbm_ctx* c, int64_t n) {
  RefTable R;
  R.X = c->ref_X;
  R.Y = c->ref_Y;
  R.Trow = c->ref_T + n * c->ref_rank;
  R.rank = c->ref_rank;
  R.nx = c->g.nx;
  R.ny = c->g.ny;
  return R;
}


// body load of time level n (rank 0 without load data)
Force force_at(const lbm_ctx* c, int64_t n) {
  Force F;
  F.rank = c->force_rank;
  F.X = c->force_X;
  F.Y = c->force_Y;
  F.Trow = c->force_rank ? c->force_T + n * c->force_rank : nullptr;
  F.nx = c->g.nx;
  F.ny = c->g.ny;
  F.scale = (float)(c->p.dt / c->p.rho);
  return F;
}

// add the errors of the state in the current buffer (time level `level`)
// to the running sums
void err_accumulate(lbm_ctx* c, int64_t level) {
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  int nb = (int)((n + RED_THREADS - 1) / RED_THREADS);
  nb = nb > RED_BLOCKS ? RED_BLOCKS : nb;
  MomConst m{(float)c->cK, (float)c->cmu, (float)c->p.rho, (float)c->kK, (float)c->km, 0};
  hipLaunchKernelGGL(k_err_partial, dim3(nb), dim3(RED_THREADS), 0, c->stream,
                     (const float*)c->buf[c->cur], (const double*)(c->disp_ready ? c->disp : nullptr),
                     c->g, force_at(c, level), ref_at(c, level), m, 0.5 * c->p.dt,
                     c->err_part);
  hipLaunchKernelGGL(k_err_final, dim3(1), dim3(RED_THREADS), 0, c->stream,
                     (const double*)c->err_part, nb, c->err_acc);
}

// V[s][link][2] = wall velocity of step `step0 + s` at every link
__global__ void k_wall_eval(const float* __restrict__ W, const float* __restrict__ T, int rank,
                            int L, int nsteps, float* __restrict__ V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsteps * L) return;
  const int s = (int)(i / L), link = (int)(i - (int64_t)s * L);
  Wall w;
  w.W = W;
  w.Trow = T + (int64_t)s * rank;
  w.rank = rank;
  w.L = L;
  float a, b;
  wall_series(w, link, a, b);
  V[2 * i] = a;
  V[2 * i + 1] = b;
}

lbm_status reduce(lbm_ctx* c, int mode, const double* ref, double out[2]) {
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  int nb = (int)((n + RED_THREADS - 1) / RED_THREADS);
  nb = nb > RED_BLOCKS ? RED_BLOCKS : nb;
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(RED_THREADS), 0, c->stream, c->buf[c->cur], ref,
                     c->g, c->norm, mode, c->partial, force_at(c, c->nstep), (float)c->kK,
                     (float)c->km);
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
  return ws_bytes(make_grid(p), p->bc, p->flags);
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
  if (ws_size < ws_bytes(g, p->bc, p->flags)) return fail(LBM_E_SPACE, "workspace too small");
  NormConst nc;
  if (!norm_weights(d.kK, d.km, nc.k)) {
    if (!(p->flags & LBM_F_ALLOW_UNSTABLE)) return fail(LBM_E_CFL, "g_ij not positive definite");
    // above the limit the weighted norm does not exist: plain sum of squares
    for (int q = 0; q < NQ; ++q)
      for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) nc.k[q][a][b] = a == b ? 1.0 : 0.0;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_E_ARG, "out of host memory");
  c->p = *p;
  c->g = g;
  c->stream = (hipStream_t)hip_stream;
  c->buf[0] = (float*)d_ws;
  c->buf[1] = (float*)((char*)d_ws + state_bytes(g));
  c->partial = (double*)((char*)d_ws + 2 * state_bytes(g));
  c->wall_v = p->bc == LBM_DIRICHLET
                  ? (float*)((char*)d_ws + 2 * state_bytes(g) +
                             (size_t)round_up((2 * RED_BLOCKS + 2) * 8, 256))
                  : nullptr;
  c->disp = (p->flags & LBM_F_DISPLACEMENT)
                ? (double*)((char*)d_ws + 2 * state_bytes(g) +
                           (size_t)round_up((2 * RED_BLOCKS + 2) * 8, 256) +
                           wall_table_bytes(g, p->bc))
                : nullptr;
  c->disp_ready = false;
  c->err_part = (double*)((char*)d_ws + 2 * state_bytes(g) +
                          (size_t)round_up((2 * RED_BLOCKS + 2) * 8, 256) +
                          wall_table_bytes(g, p->bc) + disp_bytes(g, p->flags));
  c->err_acc = c->err_part + (size_t)RED_BLOCKS * ERR_VALS;
  c->force_rows = (float*)((char*)c->err_part + round_up(ERR_BYTES, 256));
  c->err_on = false;
  c->ref_X = c->ref_Y = c->ref_T = nullptr;
  c->ref_rank = 0;
  c->ref_nsteps = 0;
  c->force_X = c->force_Y = c->force_T = nullptr;
  c->force_rank = 0;
  c->force_nsteps = 0;
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
  c->tb_cfg = -1;
  for (int r = 0; r <= TB_MAX_STEPS; ++r) c->tb_rem[r] = -1;
  c->tb_split = -1;
  for (int i = 0; i < kNumTBVariants; ++i) c->tb_launch_ms[i] = -1.0;
  c->step_launch_ms = -1.0;
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

static lbm_status init_from(lbm_ctx* c, const double* d_v0, const double* d_s0,
                            const double* d_grad, int src) {
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  InitConst k{c->kK, c->km, c->cK, c->cmu, c->p.rho, c->p.dx, c->p.bc, src};
  hipLaunchKernelGGL(k_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, d_v0,
                     d_s0, d_grad, c->buf[0], c->g, k, force_at(c, 0));
  lbm_status s = launch_check("k_init launch");
  if (s) return s;
  c->cur = 0;
  c->nstep = 0;
  c->initialised = true;
  c->disp_ready = false;
  c->err_on = false;
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* c, const double* d_v0, const double* d_sigma0, const double* d_grad) {
  if (!c || !d_v0 || !d_sigma0) return fail(LBM_E_ARG, "null argument");
  if (!(c->cmu > 0))
    return fail(LBM_E_ARG,
                "mu = 0: the stress does not determine j_d, j_xy; use lbm_init_from_gradient");
  return init_from(c, d_v0, d_sigma0, d_grad, INIT_FROM_STRESS);
}

lbm_status lbm_init_from_gradient(lbm_ctx* c, const double* d_v0, const double* d_gradu0,
                                  const double* d_grad) {
  if (!c || !d_v0 || !d_gradu0) return fail(LBM_E_ARG, "null argument");
  return init_from(c, d_v0, d_gradu0, d_grad, INIT_FROM_GRADIENT);
}

lbm_status lbm_set_body_force(lbm_ctx* c, int32_t rank, const float* d_X, const float* d_Y,
                              const float* d_T, int64_t nsteps) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (rank < 0 || rank > 4096) return fail(LBM_E_ARG, "rank out of range");
  if (rank > 0 && (!d_X || !d_Y || !d_T || nsteps < 0)) return fail(LBM_E_ARG, "null load table");
  c->force_rank = rank;
  c->force_X = rank ? d_X : nullptr;
  c->force_Y = rank ? d_Y : nullptr;
  c->force_T = rank ? d_T : nullptr;
  c->force_nsteps = rank ? nsteps : 0;
  return LBM_OK;
}

lbm_status lbm_init_displacement(lbm_ctx* c, const double* d_u0) {
  if (!c || !d_u0) return fail(LBM_E_ARG, "null argument");
  if (!c->disp) return fail(LBM_E_STATE, "context created without LBM_F_DISPLACEMENT");
  if (!c->initialised || c->nstep != 0)
    return fail(LBM_E_STATE, "lbm_init_displacement needs a freshly initialised lattice");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  hipLaunchKernelGGL(k_init_disp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     (const float*)c->buf[c->cur], d_u0, c->disp, c->g, force_at(c, 0),
                     0.5 * c->p.dt);
  lbm_status s = launch_check("k_init_disp launch");
  if (s) return s;
  c->disp_ready = true;
  return LBM_OK;
}

lbm_status lbm_displacement(lbm_ctx* c, float* d_u) {
  if (!c || !d_u) return fail(LBM_E_ARG, "null argument");
  if (!c->disp || !c->disp_ready)
    return fail(LBM_E_STATE, "no displacement: LBM_F_DISPLACEMENT and lbm_init_displacement");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  hipLaunchKernelGGL(k_displacement, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     (const float*)c->buf[c->cur], (const double*)c->disp, d_u, c->g,
                     force_at(c, c->nstep), 0.5 * c->p.dt);
  return launch_check("k_displacement launch");
}

lbm_status lbm_set_reference(lbm_ctx* c, int32_t rank, const double* d_X, const double* d_Y,
                             const double* d_T, int64_t nsteps) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (rank < 0 || rank > 4096) return fail(LBM_E_ARG, "rank out of range");
  if (rank > 0 && (!d_X || !d_Y || !d_T || nsteps < 0))
    return fail(LBM_E_ARG, "null reference table");
  c->ref_rank = rank;
  c->ref_X = rank ? d_X : nullptr;
  c->ref_Y = rank ? d_Y : nullptr;
  c->ref_T = rank ? d_T : nullptr;
  c->ref_nsteps = rank ? nsteps : 0;
  if (!rank) c->err_on = false;
  return LBM_OK;
}

lbm_status lbm_error_track(lbm_ctx* c, int32_t on) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (!on) {
    c->err_on = false;
    return LBM_OK;
  }
  if (c->ref_rank == 0) return fail(LBM_E_STATE, "no reference solution (lbm_set_reference)");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  if (c->nstep > c->ref_nsteps) return fail(LBM_E_ARG, "reference table too short");
  hipLaunchKernelGGL(k_err_zero, dim3(1), dim3(64), 0, c->stream, c->err_acc);
  err_accumulate(c, c->nstep);
  lbm_status s = launch_check("error accumulation launch");
  if (s) return s;
  c->err_on = true;
  return LBM_OK;
}

lbm_status lbm_error_sums(lbm_ctx* c, double* h_out) {
  if (!c || !h_out) return fail(LBM_E_ARG, "null argument");
  lbm_status s = hip_check(hipMemcpyAsync(h_out, c->err_acc, ERR_ACC * sizeof(double),
                                          hipMemcpyDeviceToHost, c->stream),
                           "error sums copy");
  if (s) return s;
  return hip_check(hipStreamSynchronize(c->stream), "error sums sync");
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* d_f) {
  if (!c || !d_f) return fail(LBM_E_ARG, "null argument");
  const int64_t n = (int64_t)c->g.nx * c->g.ny;
  hipLaunchKernelGGL(k_set_populations, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     c->stream, d_f, c->buf[0], c->g, (float)c->kK, (float)c->km,
                     force_at(c, 0));
  lbm_status s = launch_check("k_set_populations launch");
  if (s) return s;
  c->cur = 0;
  c->nstep = 0;
  c->initialised = true;
  c->disp_ready = false;
  c->err_on = false;
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

}  // extern "C"

namespace {

// Kernel handles of the blocked variants (lbm_tb_tables.hpp), filled once
// from the translation units that instantiate them.
struct TBTables {
  TBFn fn[kNumTBVariants][2];       // load-free, [variant][bc]
  TBExtFns xfn[kNumTBExtVariants];  // with extras, [variant][extras][bc]
  TBSplitFn sfn[kNumTBSplitVariants];  // split Dirichlet launches
};

const TBTables& tb_tables() {
  static const TBTables t = [] {
    TBTables r;
    TBFn p[kNumTBVariants], d[kNumTBVariants];
    tb_fill_periodic_a(p);
    tb_fill_periodic_b(p);
    tb_fill_dirichlet_a(d);
    tb_fill_dirichlet_b(d);
    for (int i = 0; i < kNumTBVariants; ++i) {
      r.fn[i][LBM_PERIODIC] = p[i];
      r.fn[i][LBM_DIRICHLET] = d[i];
    }
    tb_fill_extra_a(r.xfn);
    tb_fill_extra_b(r.xfn);
    tb_fill_split(r.sfn);
    return r;
  }();
  return t;
}

static_assert(kNumTBVariants <= 64, "tb_slots size");
static_assert(kNumTBExtVariants * 3 <= 48, "tbf_slots size");
static_assert(kNumTBSplitVariants <= 8, "tbs_slots size");


// Sum the wall velocities of steps step0 .. step0 + n - 1 (n <= WALL_CHUNK)
// into the context's table; no-op without wall data.
void eval_walls(lbm_ctx* c, int64_t step0, int n) {
  if (c->wall_rank == 0 || n <= 0) return;
  const int L = 2 * (c->g.nx + c->g.ny);
  const int64_t total = (int64_t)n * L;
  hipLaunchKernelGGL(k_wall_eval, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                     c->wall_W, c->wall_T + step0 * c->wall_rank, c->wall_rank, L, n, c->wall_v);
}

Wall zero_wall(const lbm_ctx* c) {
  Wall w;
  w.rank = 0;
  w.W = nullptr;
  w.Trow = nullptr;
  w.L = 2 * (c->g.nx + c->g.ny);
  return w;
}

// For timing launches: sum the walls of the next `n` steps (the most steps a
// blocked launch takes) into the table when the context has wall data for
// them.
bool timing_walls(lbm_ctx* c, int n = 8) {
  if (c->wall_rank == 0 || c->nstep + n > c->wall_nsteps) return false;
  eval_walls(c, c->nstep, n);
  return true;
}

// walls of table entry s (summed by eval_walls); zero velocity without data
Wall wall_at(const lbm_ctx* c, int s) {
  Wall w;
  w.rank = 0;
  w.W = nullptr;
  w.Trow = nullptr;
  w.L = 2 * (c->g.nx + c->g.ny);
  w.V = c->wall_rank ? c->wall_v + (int64_t)s * w.L * 2 : nullptr;
  return w;
}

WallSeq walls_from(const lbm_ctx* c, int s, bool with_walls) {
  WallSeq ws;
  ws.L = 2 * (c->g.nx + c->g.ny);
  ws.V = with_walls && c->wall_rank ? c->wall_v + (int64_t)s * ws.L * 2 : nullptr;
  return ws;
}

// Rows per segment of blocked variant k: its seg_rows, or for seg_rows <= 0 as
// many as give one wave per resident slot (times -seg_rows; for TB_SEG_SIMD
// one per SIMD whatever the occupancy) across the grid, rounded up to the
// ring length (*slots caches the device's resident waves).
int seg_rows_of(lbm_ctx* c, int steps, int seg_rows, int pf, TBFn fn, int* slots) {
  if (seg_rows > 0) return seg_rows;
  if (*slots == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, 256, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess ||
        per_cu < 1 || cus < 1) {
      (void)hipGetLastError();
      per_cu = 2;
      cus = 256;
    }
    *slots = (seg_rows == TB_SEG_SIMD ? 1 : per_cu) * 4 * cus;
  }
  const int ring = 3 + pf;
  const int valid = TB_LANES - 2 * steps;
  const int nstrips = (c->g.nx + valid - 1) / valid;
  const int rounds = seg_rows < 0 && seg_rows != TB_SEG_SIMD ? -seg_rows : 1;
  int nseg = *slots * rounds / nstrips;
  if (nseg < 1) nseg = 1;
  int rows = (c->g.ny + nseg - 1) / nseg;
  rows = (rows + ring - 1) / ring * ring;
  return rows;
}

int tb_seg_rows(lbm_ctx* c, int index) {
  const TBVariant& k = kTBVariants[index];
  return seg_rows_of(c, k.steps, k.seg_rows, k.pf, tb_tables().fn[index][c->p.bc],
                     &c->tb_slots[index]);
}

// ---- split Dirichlet launches ---------------------------------------------
// The Dirichlet rule changes a node's update only at the walls, and a change
// travels one node per step, so after T steps every node at least T nodes
// from each wall holds what periodic arithmetic on the same rows gives (the
// same operations in the same order: bitwise equal).  A split launch
// (k_tblock_split) sweeps the interior strips [lo, hi) (stores in
// [T, nx - T)) over rows [SPLIT_ROWS, ny - SPLIT_ROWS) with the periodic
// kernel's code, whose registers the wall code does not take, and the band
// along the walls (the other strips, all rows; the first and last SPLIT_ROWS
// rows of the interior strips) with the Dirichlet rule as short segments, in
// one grid.  The interior's segments leave as many resident wave slots to
// the band as it has tiles, so both run in one round.  16 rows for the band
// at the top and bottom walls and per segment of the side-wall strips
// (2048 x 1024, T = 7: 151 GLUPS; 8 or 24 rows: 142, 32: 106 to 147).
constexpr int SPLIT_ROWS = 16;

struct SplitPlan {
  int kernel;  // index into kTBSplitVariants
  TBConst in, band;
  int ntiles;
};

// the split kernel of load-free variant `index`, or -1
int split_kernel(int index) {
  const TBVariant& k = kTBVariants[index];
  for (int i = 0; i < kNumTBSplitVariants; ++i) {
    const TBSplitVariant& s = kTBSplitVariants[i];
    if (s.steps == k.steps && s.nt == k.nt && s.pf == k.pf) return i;
  }
  return -1;
}

int split_slots(lbm_ctx* c, int kernel) {
  int& slots = c->tbs_slots[kernel];
  if (slots == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void*)tb_tables().sfn[kernel], 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess ||
        per_cu < 1 || cus < 1) {
      (void)hipGetLastError();
      per_cu = 1;
      cus = 256;
    }
    slots = per_cu * 4 * cus;
  }
  return slots;
}

bool split_plan(lbm_ctx* c, int index, SplitPlan& sp) {
  if (c->p.bc != LBM_DIRICHLET || c->tb_split == 0) return false;
  const TBVariant& k = kTBVariants[index];
  const int T = k.steps;
  sp.kernel = split_kernel(index);
  if (sp.kernel < 0) return false;
  const Grid& g = c->g;
  const int valid = TB_LANES - 2 * T;
  const int lo = 1, hi = (g.nx - T) / valid;
  if (hi - lo < 1 || g.ny < 2 * SPLIT_ROWS + 1) return false;
  sp.band = tblock_const(g, (float)c->kK, (float)c->km, SPLIT_ROWS, T);
  sp.band.band_lo = lo;
  sp.band.band_hi = hi;
  sp.band.band_rows = SPLIT_ROWS;
  const int nband = (sp.band.nstrips - (hi - lo)) * sp.band.nseg + 2 * (hi - lo);
  const int rows = g.ny - 2 * SPLIT_ROWS;
  int seg = k.seg_rows;
  if (seg <= 0) {
    const int rounds = seg < 0 && seg != TB_SEG_SIMD ? -seg : 1;
    int nseg = (split_slots(c, sp.kernel) * rounds - nband) / (hi - lo);
    if (nseg < 1) nseg = 1;
    const int ring = 3 + k.pf;
    seg = (rows + nseg - 1) / nseg;
    seg = (seg + ring - 1) / ring * ring;
  }
  sp.in = tblock_const(g, (float)c->kK, (float)c->km, seg, T);
  sp.in.strip_first = lo;
  sp.in.nstrips = hi - lo;
  sp.in.y_first = SPLIT_ROWS;
  sp.in.y_end = g.ny - SPLIT_ROWS;
  sp.in.nseg = (rows + seg - 1) / seg;
  sp.ntiles = nband + sp.in.nstrips * sp.in.nseg;
  return true;
}

// one launch of variant `index`: kTBVariants[index].steps steps, level l with
// the walls of table entry s0 + l - 1
void launch_tb(lbm_ctx* c, int index, const float* src, float* dst, const WallSeq& ws) {
  const TBVariant& k = kTBVariants[index];
  SplitPlan sp;
  if (split_plan(c, index, sp)) {
    hipLaunchKernelGGL(tb_tables().sfn[sp.kernel], dim3((unsigned)((sp.ntiles + 3) / 4)),
                       dim3(256), 0, c->stream, src, dst, c->g, sp.band, sp.in, ws);
    return;
  }
  const TBConst sc = tblock_const(c->g, (float)c->kK, (float)c->km, tb_seg_rows(c, index), k.steps);
  const int ntiles = sc.nstrips * sc.nseg;
  hipLaunchKernelGGL(tb_tables().fn[index][c->p.bc], dim3((unsigned)((ntiles + 3) / 4)),
                     dim3(256), 0, c->stream, src, dst, c->g, sc, ws,
                     TBExtra{nullptr, nullptr, 0, 0.f, nullptr, 0.0});
}

// The variant that takes the last r (2 <= r < T) steps of a run in one
// launch after full launches of variant `shape`: the autotuner's fastest
// r-step variant when it has timed them, else the r-step variant nearest to
// that shape (same rows per segment, store type and prefetch, then the same
// rows per segment and prefetch, then the same rows per segment, then the
// first); -1 if none, or if `shape` is not a blocked variant.
int remainder_variant(const lbm_ctx* c, int r, int shape) {
  if (r < 2 || r > TB_MAX_STEPS || shape < 0 || shape >= kNumTBVariants) return -1;
  if (c->tb_rem[r] >= 0) return c->tb_rem[r];
  const TBVariant& t = kTBVariants[shape];
  int best = -1, best_score = -1;
  for (int i = 0; i < kNumTBVariants; ++i) {
    const TBVariant& k = kTBVariants[i];
    if (k.steps != r) continue;
    const int score = (k.seg_rows == t.seg_rows ? 4 : 0) + (k.pf == t.pf ? 2 : 0) +
                      (k.nt == t.nt ? 1 : 0);
    if (score > best_score) {
      best_score = score;
      best = i;
    }
  }
  return best;
}

// rows[l][y][r] = Y[r][y] T_{n1 + l}[r] for r < R, -0 for R <= r < MR (the
// factors of body_hat, one per level of a blocked launch whose first level
// is n1)
__global__ void k_force_rows(const float* __restrict__ Y, const float* __restrict__ T1, int R,
                             int ny, int T, int MR, float* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)T * ny * MR) return;
  const int r = (int)(i % MR);
  const int64_t ly = i / MR;
  const int y = (int)(ly % ny), l = (int)(ly / ny);
  rows[i] = r < R ? Y[(int64_t)r * ny + y] * T1[(int64_t)l * R + r] : -0.f;
}

// whether extras variant i has the kernel for extras m on this lattice (load
// ranks, and one wrap of a load row at most)
bool extra_usable(const lbm_ctx* c, int i, int m) {
  const TBExtVariant& k = kTBExtVariants[i];
  if (!tb_tables().xfn[i][m][c->p.bc]) return false;
  const int mr = c->force_rank > 16 ? 32 : 16;  // the narrowest rank width that holds the load
  if (m != 1 && k.mr != mr) return false;
  return c->g.ny >= k.steps + 3 + k.pf;
}

// the whole-run variant with extras m (0 load, 1 displacement, 2 both) for a
// lattice whose blocked variant is tb_cfg: the same launch shape if there is
// one, else the same T, else the first for its boundary type; -1 if none
// applies
int extra_variant(const lbm_ctx* c, int m) {
  if (c->tb_cfg < 0 || c->force_rank > TB_MAXR || !tblock_fits(c->g)) return -1;
  const TBVariant& t = kTBVariants[c->tb_cfg];
  int same_t = -1, first = -1;
  for (int i = 0; i < kNumTBExtVariants; ++i) {
    const TBExtVariant& k = kTBExtVariants[i];
    if (!k.main || !extra_usable(c, i, m)) continue;
    if (k.steps == t.steps && k.seg_rows == t.seg_rows && k.nt == t.nt && k.pf == t.pf) return i;
    if (k.steps == t.steps && same_t < 0) same_t = i;
    if (first < 0) first = i;
  }
  return same_t >= 0 ? same_t : first;
}

// the variant with extras m for the last steps of a run: the one with the
// most steps, at most r, for this lattice (-1: none, r < 2)
int extra_remainder_variant(const lbm_ctx* c, int m, int r) {
  int best = -1;
  for (int i = 0; i < kNumTBExtVariants; ++i) {
    const TBExtVariant& k = kTBExtVariants[i];
    if (k.steps > r || k.steps < 2 || !extra_usable(c, i, m)) continue;
    if (best < 0 || k.steps > kTBExtVariants[best].steps) best = i;
  }
  return best;
}

}  // namespace
extern "C" {

// Steps with a body load and/or the displacement state: one step per launch
// of the one-node-per-thread kernel.  Step n -> n+1 collides at t_{n+1} with
// the load row of that level.
static lbm_status step_ext(lbm_ctx* c, int64_t nsteps) {
  typedef void (*ExtFn)(const float*, float*, Grid, StepConst, Wall, StepExtra);
  static const ExtFn fns[2][2][2] = {
      {{&k_step_ext<LBM_PERIODIC, false, false>, &k_step_ext<LBM_PERIODIC, false, true>},
       {&k_step_ext<LBM_PERIODIC, true, false>, &k_step_ext<LBM_PERIODIC, true, true>}},
      {{&k_step_ext<LBM_DIRICHLET, false, false>, &k_step_ext<LBM_DIRICHLET, false, true>},
       {&k_step_ext<LBM_DIRICHLET, true, false>, &k_step_ext<LBM_DIRICHLET, true, true>}}};
  const Grid& g = c->g;
  const bool force = c->force_rank > 0, disp = c->disp != nullptr;
  const ExtFn fn = fns[c->p.bc][force][disp];
  StepConst sc;
  sc.kK = (float)c->kK;
  sc.km = (float)c->km;
  sc.tiles_x = (g.nx + 255) / 256;
  sc.ntiles = sc.tiles_x * g.ny;
  StepExtra ex;
  ex.D = c->disp;
  ex.half_dt = 0.5 * c->p.dt;
  const int64_t base = c->nstep;
  for (int64_t s0 = 0; s0 < nsteps; s0 += WALL_CHUNK) {
    const int m = (int)(nsteps - s0 < WALL_CHUNK ? nsteps - s0 : WALL_CHUNK);
    eval_walls(c, base + s0, m);
    for (int k = 0; k < m; ++k) {
      const int64_t level = base + s0 + k + 1;  // the level this step forms
      ex.F = force_at(c, level);
      hipLaunchKernelGGL(fn, dim3(sc.ntiles), dim3(256), 0, c->stream,
                         (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], g, sc, wall_at(c, k),
                         ex);
      c->cur ^= 1;
      if (c->err_on) err_accumulate(c, level);
    }
  }
  c->nstep = base + nsteps;
  return launch_check("k_step_ext launch");
}

// One launch of extras variant vi (extras m): kTBExtVariants[vi].steps steps
// from the current step, walls from table entry s; with a load the row
// factors of its levels are formed first.
static void launch_tbx(lbm_ctx* c, int vi, int m, int s) {
  const TBExtVariant& k = kTBExtVariants[vi];
  const TBFn fn = tb_tables().xfn[vi][m][c->p.bc];
  const int T = k.steps, R = c->force_rank;
  const TBConst sc = tblock_const(c->g, (float)c->kK, (float)c->km,
                                  seg_rows_of(c, T, k.seg_rows, k.pf, fn, &c->tbf_slots[vi * 3 + m]),
                                  T);
  const int ntiles = sc.nstrips * sc.nseg;
  const TBExtra F{c->force_X, c->force_rows, R, (float)(c->p.dt / c->p.rho), c->disp,
                  0.5 * c->p.dt};
  const int64_t nrows = (int64_t)T * c->g.ny * k.mr;
  if (R > 0)
    hipLaunchKernelGGL(k_force_rows, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0,
                       c->stream, c->force_Y, c->force_T + (c->nstep + 1) * R, R, c->g.ny, T,
                       k.mr, c->force_rows);
  hipLaunchKernelGGL(fn, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, c->stream,
                     (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], c->g, sc,
                     walls_from(c, s, true), F);
  c->cur ^= 1;
  c->nstep += T;
}

// Steps with a body load and/or the displacement state (no error norms), T
// per launch with variant vi, extras m.  The steps after the last full launch
// run in as few launches of shorter variants as exist (the longest that fits
// first); a single step left runs one launch of the one-step kernel.
static lbm_status step_extra_blocked(lbm_ctx* c, int64_t nsteps, int vi, int m) {
  const int T = kTBExtVariants[vi].steps;
  const int chunk = WALL_CHUNK / T * T;
  for (int64_t done = 0; done < nsteps;) {
    const int n = (int)(nsteps - done < chunk ? nsteps - done : chunk);
    eval_walls(c, c->nstep, n);
    int j = 0;
    for (; j + T <= n; j += T) launch_tbx(c, vi, m, j);
    for (int r = n - j; r >= 2; r = n - j) {
      const int ri = extra_remainder_variant(c, m, r);
      if (ri < 0) break;
      launch_tbx(c, ri, m, j);
      j += kTBExtVariants[ri].steps;
    }
    done += j;
    if (j < n) {
      // fewer than two steps left, or no shorter variant: one launch per step
      lbm_status s = launch_check("k_tblock launch (load / displacement)");
      if (s) return s;
      s = step_ext(c, n - j);
      if (s) return s;
      done += n - j;
    }
  }
  return launch_check("k_tblock launch (load / displacement)");
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (!c->initialised) return fail(LBM_E_STATE, "lbm_step before lbm_init");
  if (nsteps < 0) return fail(LBM_E_ARG, "negative step count");
  if (c->wall_rank > 0 && c->nstep + nsteps > c->wall_nsteps)
    return fail(LBM_E_ARG, "wall table too short for the requested steps");
  if (c->force_rank > 0 && c->nstep + nsteps > c->force_nsteps)
    return fail(LBM_E_ARG, "body load table too short for the requested steps");
  if (c->disp && !c->disp_ready)
    return fail(LBM_E_STATE, "LBM_F_DISPLACEMENT: lbm_init_displacement before lbm_step");
  if (c->err_on && c->nstep + nsteps > c->ref_nsteps)
    return fail(LBM_E_ARG, "reference table too short for the requested steps");
  if ((c->force_rank > 0 || c->disp) && !c->err_on) {
    const int m = c->force_rank > 0 ? (c->disp ? 2 : 0) : 1;
    const int vi = extra_variant(c, m);
    if (vi >= 0) return step_extra_blocked(c, nsteps, vi, m);
  }
  if (c->force_rank > 0 || c->disp || c->err_on) return step_ext(c, nsteps);
  const Grid& g = c->g;
  const StepConfig& cfg = kStepConfigs[c->step_cfg];
  const StepConst sc = step_const(cfg, g, (float)c->kK, (float)c->km);
  const StepFn fn = cfg.fn[c->p.bc];
  // chunks of a multiple of T steps (at most WALL_CHUNK): the chunk's wall
  // velocities are summed first, then its steps run, T per launch with a
  // blocked variant; the r < T steps after the last full launch of a run take
  // one launch of an r-step variant (r >= 2) or of the single-step kernel
  const int T = c->tb_cfg >= 0 ? kTBVariants[c->tb_cfg].steps : 1;
  const int chunk = WALL_CHUNK / T * T;
  for (int64_t s0 = 0; s0 < nsteps; s0 += chunk) {
    const int m = (int)(nsteps - s0 < chunk ? nsteps - s0 : chunk);
    eval_walls(c, c->nstep + s0, m);
    int k = 0;
    if (T > 1) {
      for (; k + T <= m; k += T) {
        launch_tb(c, c->tb_cfg, c->buf[c->cur], c->buf[c->cur ^ 1], walls_from(c, k, true));
        c->cur ^= 1;
      }
      const int ri = remainder_variant(c, m - k, c->tb_cfg);
      if (ri >= 0) {
        launch_tb(c, ri, c->buf[c->cur], c->buf[c->cur ^ 1], walls_from(c, k, true));
        c->cur ^= 1;
        k = m;
      }
    }
    for (; k < m; ++k) {
      hipLaunchKernelGGL(fn, dim3(sc.ntiles), dim3(cfg.threads), 0, c->stream,
                         (const float*)c->buf[c->cur], c->buf[c->cur ^ 1], g, sc, wall_at(c, k));
      c->cur ^= 1;
    }
  }
  c->nstep += nsteps;
  return launch_check("k_step launch");
}

// ---- launch configurations and the autotuner ------------------------------
}  // extern "C"

namespace {

struct TuneKey {
  int nx, ny, bc;
  int split;  // split mode of Dirichlet lattices (-1, the default, for periodic ones)
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, bc, split) < std::tie(o.nx, o.ny, o.bc, o.split);
  }
};

// single-step configuration, blocked variant (-1: none) and the variants for
// the last r steps of a run (-1: nearest shape)
struct TuneVal {
  int cfg, cfg2;
  int rem[TB_MAX_STEPS + 1];
  double launch_ms[kNumTBVariants];  // in this process only (-1: not timed)
  double step_ms;
};

TuneVal tune_val(int cfg, int cfg2, const int* rem, const lbm_ctx* timed = nullptr) {
  TuneVal v;
  v.cfg = cfg;
  v.cfg2 = cfg2;
  for (int r = 0; r <= TB_MAX_STEPS; ++r) v.rem[r] = rem ? rem[r] : -1;
  for (int i = 0; i < kNumTBVariants; ++i) v.launch_ms[i] = timed ? timed->tb_launch_ms[i] : -1.0;
  v.step_ms = timed ? timed->step_launch_ms : -1.0;
  return v;
}

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;
bool g_tune_file_loaded = false;

int find_config(int vec, int threads, int nt, int xmode) {
  for (int i = 0; i < kNumStepConfigs; ++i) {
    const StepConfig& k = kStepConfigs[i];
    if (k.vec == vec && k.threads == threads && k.nt == nt && k.xmode == xmode) return i;
  }
  return -1;
}

// Cache file (path in LBM_AUTOTUNE_CACHE): one line per tuned shape,
// "nx ny bc vec threads nt xmode tb ms r2 .. r10" (tb = blocked variant or -1,
// r = the variant for the last r steps of a run or -1; lines without the r
// fields are read with none), for the default split mode only.
// Caller holds g_tune_mu.
void load_tune_file() {
  if (g_tune_file_loaded) return;
  g_tune_file_loaded = true;
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    int nx, ny, bc, vec, th, nt, xm, s2, rem[TB_MAX_STEPS + 1];
    double ms;
    for (int r = 0; r <= TB_MAX_STEPS; ++r) rem[r] = -1;
    static_assert(TB_MAX_STEPS == 10, "the line format below lists r = 2 .. 10");
    const int n = sscanf(line, "%d %d %d %d %d %d %d %d %lf %d %d %d %d %d %d %d %d %d", &nx,
                         &ny, &bc, &vec, &th, &nt, &xm, &s2, &ms, &rem[2], &rem[3], &rem[4],
                         &rem[5], &rem[6], &rem[7], &rem[8], &rem[9], &rem[10]);
    if (n != 9 && n != 18) continue;
    for (int r = 2; r <= TB_MAX_STEPS; ++r)
      if (rem[r] < -1 || rem[r] >= kNumTBVariants || (rem[r] >= 0 && kTBVariants[rem[r]].steps != r))
        rem[r] = -1;
    const int i = find_config(vec, th, nt, xm);
    if (i >= 0 && step_config_valid(i, nx) && s2 >= -1 && s2 < kNumTBVariants)
      g_tune_cache[TuneKey{nx, ny, bc, -1}] = tune_val(i, s2, s2 >= 0 ? rem : nullptr);
  }
  fclose(f);
}

void append_tune_file(const TuneKey& k, const TuneVal& v, double ms) {
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path || k.split != -1) return;  // the file holds the default mode's choices
  FILE* f = fopen(path, "a");
  if (!f) return;
  const StepConfig& c = kStepConfigs[v.cfg];
  fprintf(f, "%d %d %d %d %d %d %d %d %.6f", k.nx, k.ny, k.bc, c.vec, c.threads, c.nt, c.xmode,
          v.cfg2, ms);
  for (int r = 2; r <= TB_MAX_STEPS; ++r) fprintf(f, " %d", v.rem[r]);
  fprintf(f, "\n");
  fclose(f);
}

}  // namespace
extern "C" {

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
  const TuneKey key{c->g.nx, c->g.ny, c->p.bc, c->p.bc == LBM_DIRICHLET ? c->tb_split : -1};
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c->step_cfg = it->second.cfg;
      c->tb_cfg = it->second.cfg2 < kNumTBVariants && tblock_fits(c->g) ? it->second.cfg2 : -1;
      for (int r = 0; r <= TB_MAX_STEPS; ++r) c->tb_rem[r] = c->tb_cfg >= 0 ? it->second.rem[r] : -1;
      for (int i = 0; i < kNumTBVariants; ++i) c->tb_launch_ms[i] = it->second.launch_ms[i];
      c->step_launch_ms = it->second.step_ms;
      if (h_index) *h_index = it->second.cfg;
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
  // timed with this context's walls at the current step when it has them
  const bool tw = timing_walls(c);
  const Wall w = tw ? wall_at(c, 0) : zero_wall(c);
  const WallSeq ws = walls_from(c, 0, tw);
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
  // blocked variants: time per step = time per launch / steps per launch
  int best2 = -1;
  double best2_ms = 1e300;
  int rem[TB_MAX_STEPS + 1];
  double rem_ms[TB_MAX_STEPS + 1];
  for (int r = 0; r <= TB_MAX_STEPS; ++r) {
    rem[r] = -1;
    rem_ms[r] = 1e300;
  }
  for (int i = 0; i < kNumTBVariants && s == LBM_OK && tblock_fits(c->g); ++i) {
    for (int r = 0; r < reps + 2; ++r) {
      if (r == 2) hipEventRecord(e0, c->stream);
      launch_tb(c, i, c->buf[c->cur], c->buf[c->cur ^ 1], ws);
    }
    hipEventRecord(e1, c->stream);
    s = hip_check(hipEventSynchronize(e1), "autotune sync");
    float ms = 0.f;
    if (s == LBM_OK) s = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing");
    const int steps = kTBVariants[i].steps;
    const double per = (double)ms / reps / steps;
    if (s == LBM_OK) c->tb_launch_ms[i] = (double)ms / reps;
    if (s == LBM_OK && per < best2_ms) {
      best2_ms = per;
      best2 = i;
    }
    // the fastest launch of each step count, for the last steps of a run
    if (s == LBM_OK && (double)ms / reps < rem_ms[steps]) {
      rem_ms[steps] = (double)ms / reps;
      rem[steps] = i;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s) return s;
  if (best < 0) return fail(LBM_E_ARG, "no valid launch configuration");
  c->step_cfg = best;
  c->step_launch_ms = best_ms;
  c->tb_cfg = best2_ms < best_ms ? best2 : -1;
  for (int r = 0; r <= TB_MAX_STEPS; ++r) c->tb_rem[r] = rem[r];
  const double per_step = best2_ms < best_ms ? best2_ms : best_ms;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    g_tune_cache[key] = tune_val(best, c->tb_cfg, rem, c);
    append_tune_file(key, g_tune_cache[key], per_step);
  }
  if (h_index) *h_index = best;
  if (h_ms) *h_ms = per_step;
  return LBM_OK;
}

int32_t lbm_tblock_config_count(void) { return kNumTBVariants; }

lbm_status lbm_tblock_config_info(int32_t index, int32_t* steps, int32_t* seg_rows, int32_t* nt,
                                  int32_t* pf) {
  if (index < 0 || index >= kNumTBVariants) return fail(LBM_E_ARG, "config index out of range");
  const TBVariant& k = kTBVariants[index];
  if (steps) *steps = k.steps;
  if (seg_rows) *seg_rows = k.seg_rows;
  if (nt) *nt = k.nt;
  if (pf) *pf = k.pf;
  return LBM_OK;
}

int32_t lbm_steps_per_launch(const lbm_ctx* c) {
  if (!c) return -1;
  if (c->err_on) return 1;
  if (c->force_rank > 0 || c->disp) {
    const int m = c->force_rank > 0 ? (c->disp ? 2 : 0) : 1;
    const int vi = extra_variant(c, m);
    return vi >= 0 ? kTBExtVariants[vi].steps : 1;
  }
  return c->tb_cfg >= 0 && tblock_fits(c->g) ? kTBVariants[c->tb_cfg].steps : 1;
}

lbm_status lbm_get_tblock_config(const lbm_ctx* c, int32_t* index) {
  if (!c || !index) return fail(LBM_E_ARG, "null argument");
  *index = c->tb_cfg;
  return LBM_OK;
}

lbm_status lbm_set_tblock_config(lbm_ctx* c, int32_t index) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (index < -1 || index >= kNumTBVariants) return fail(LBM_E_ARG, "config index out of range");
  if (index >= 0 && !tblock_fits(c->g))
    return fail(LBM_E_ARG, "grid too wide for the blocked kernel (row offsets exceed 2^31 B)");
  c->tb_cfg = index;
  return LBM_OK;
}

lbm_status lbm_select_for_steps(lbm_ctx* c, int64_t nsteps, int32_t* h_index) {
  if (!c || !h_index || nsteps < 1) return fail(LBM_E_ARG, "null argument or no steps");
  *h_index = c->tb_cfg;
  if (c->step_launch_ms <= 0.0) return LBM_OK;  // no launch times: selection unchanged
  // predicted time of a run of nsteps steps with variant v (-1: single steps):
  // its full launches, then the launch lbm_step takes for the steps left
  auto cost = [&](int v) {
    const int T = v >= 0 ? kTBVariants[v].steps : 1;
    const double full = v >= 0 ? c->tb_launch_ms[v] : c->step_launch_ms;
    if (full <= 0.0) return 1e300;
    const int r = (int)(nsteps % T);
    double rest = 0.0;
    if (r == 1) {
      rest = c->step_launch_ms;
    } else if (r > 1) {
      const int ri = remainder_variant(c, r, v);
      rest = ri >= 0 && c->tb_launch_ms[ri] > 0.0 ? c->tb_launch_ms[ri] : r * c->step_launch_ms;
    }
    return (double)(nsteps / T) * full + rest;
  };
  int best = -1;
  double best_cost = cost(-1);
  for (int v = 0; v < kNumTBVariants; ++v) {
    const double cv = cost(v);
    if (cv < best_cost) {
      best_cost = cv;
      best = v;
    }
  }
  c->tb_cfg = best;
  *h_index = best;
  return LBM_OK;
}

lbm_status lbm_get_tblock_remainder(const lbm_ctx* c, int32_t r, int32_t* h_index) {
  if (!c || !h_index) return fail(LBM_E_ARG, "null argument");
  *h_index = remainder_variant(c, r, c->tb_cfg);
  return LBM_OK;
}

lbm_status lbm_set_tblock_split(lbm_ctx* c, int32_t mode) {
  if (!c) return fail(LBM_E_ARG, "null ctx");
  if (mode < -1 || mode > 1) return fail(LBM_E_ARG, "split mode must be -1, 0 or 1");
  c->tb_split = mode;
  return LBM_OK;
}

int32_t lbm_tblock_split_active(lbm_ctx* c, int32_t index) {
  if (!c || index < 0 || index >= kNumTBVariants) return -1;
  SplitPlan sp;
  return split_plan(c, index, sp) ? 1 : 0;
}

lbm_status lbm_time_tblock_config(lbm_ctx* c, int32_t index, int32_t reps, double* h_ms) {
  if (!c || !h_ms) return fail(LBM_E_ARG, "null argument");
  if (!c->initialised) return fail(LBM_E_STATE, "not initialised");
  if (index < 0 || index >= kNumTBVariants) return fail(LBM_E_ARG, "invalid configuration");
  if (!tblock_fits(c->g))
    return fail(LBM_E_ARG, "grid too wide for the blocked kernel (row offsets exceed 2^31 B)");
  if (reps < 1) return fail(LBM_E_ARG, "reps must be >= 1");
  hipEvent_t e0, e1;
  lbm_status s = hip_check(hipEventCreate(&e0), "event");
  if (s) return s;
  s = hip_check(hipEventCreate(&e1), "event");
  if (s) {
    hipEventDestroy(e0);
    return s;
  }
  // timed with this context's walls at the current step when it has them
  const WallSeq ws = walls_from(c, 0, timing_walls(c));
  for (int r = 0; r < reps + 2; ++r) {
    if (r == 2) hipEventRecord(e0, c->stream);
    launch_tb(c, index, c->buf[c->cur], c->buf[c->cur ^ 1], ws);
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
  // timed with this context's walls at the current step when it has them
  const bool tw = timing_walls(c);
  const Wall w = tw ? wall_at(c, 0) : zero_wall(c);
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
                     c->buf[c->cur], out, c->g, m, force_at(c, c->nstep));
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
