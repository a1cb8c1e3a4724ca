// Fused pull-stream + collide step kernel and its launch configurations.
//
// One workgroup covers one row segment of THREADS * VEC nodes; each thread
// owns VEC consecutive nodes and touches every plane with VEC-wide (8- or
// 16-byte) accesses.  The x-shifted pulls (directions (1,0) and (-1,0)) need
// one element beyond the thread's own vector on each side:
//   XMODE 0  an extra 4-byte load (hits L1/L2: the neighbour lane fetched it)
//   XMODE 1  the neighbour lane's value by a lane shuffle; the two wave-edge
//            elements of all ten shifted planes come from one load per wave
//            (lanes 0..9) broadcast with readlane.  Needs nx % (64 VEC) == 0.
// NT = 1 writes with nontemporal stores.  Every variant performs the same
// FP32 operations per node (collide()), so all produce bitwise-identical
// states; the autotuner only chooses among them by measured time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_kernels.hpp"

namespace lbmk {

struct StepConst {
  float kK, km;
  int tiles_x;  // workgroups per row
  int ntiles;   // workgroups in the launch
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap the dispatch index so every XCD owns one contiguous run of tiles
// (rows): the y-halo rows and the x-halo cache lines of neighbouring tiles are
// then fetched into the same L2.
__device__ inline int xcd_tile(int bid, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

__device__ inline int64_t pidx(const Grid& g, int p, int y, int x) {
  return (int64_t)p * g.plane + (int64_t)y * g.pitch + x;
}

template <int VEC>
struct VecT;
template <>
struct VecT<1> {
  typedef float T;
};
template <>
struct VecT<2> {
  typedef float T __attribute__((ext_vector_type(2)));
};
template <>
struct VecT<4> {
  typedef float T __attribute__((ext_vector_type(4)));
};

template <int VEC>
__device__ inline void vload(const float* p, float out[VEC]) {
  if constexpr (VEC == 1) {
    out[0] = *p;
  } else {
    typedef typename VecT<VEC>::T T;
    const T v = *reinterpret_cast<const T*>(p);
#pragma unroll
    for (int k = 0; k < VEC; ++k) out[k] = v[k];
  }
}

template <int VEC, int NT>
__device__ inline void vstore(float* p, const float in[VEC]) {
  typedef typename VecT<VEC>::T T;
  T v;
  if constexpr (VEC == 1) {
    v = in[0];
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) v[k] = in[k];
  }
  if constexpr (NT)
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(p));
  else
    *reinterpret_cast<T*>(p) = v;
}

// Optional per-node work of a step: body load of the new time level and the
// trapezoidal displacement update (Section 3.5): with v = v_num of the new
// level, u = D + dt/2 v is the displacement at that level and D <- u + dt/2 v
// is kept for the next (D [2][ny][nx], updated in place).
struct StepExtra {
  Force F;
  double* D;       // displacement state u + dt/2 v, FP64 [2][ny][nx]
  double half_dt;
};

// One row segment (row y, segment tx) of one lattice: the body shared by the
// single-lattice and the batched step kernels.
template <int BC, int VEC, int THREADS, int NT, int XMODE, bool FORCE = false, bool DISP = false>
__device__ inline void step_segment(const float* __restrict__ src, float* __restrict__ dst,
                                    const Grid& g, float kK, float km, const Wall& w, int y,
                                    int tx, const StepExtra& ex = StepExtra{}) {
  StepConst sc;
  sc.kK = kK;
  sc.km = km;
  const int x0 = (tx * THREADS + (int)threadIdx.x) * VEC;
  const int nx = g.nx, ny = g.ny;
  if (x0 >= nx) return;  // XMODE 1: nx % (64 VEC) == 0, so whole waves exit together

  auto wrapx = [&](int x) -> int {
    if (BC == LBM_PERIODIC) return x < 0 ? x + nx : (x >= nx ? x - nx : x);
    return x < 0 ? 0 : (x >= nx ? nx - 1 : x);
  };
  int yb = y - 1, yt = y + 1;
  if (BC == LBM_PERIODIC) {
    yb = yb < 0 ? ny - 1 : yb;
    yt = yt >= ny ? 0 : yt;
  } else {
    yb = yb < 0 ? 0 : yb;
    yt = yt >= ny ? ny - 1 : yt;
  }

  float f[VEC][NQ][NC];
  float halo = 0.f;
  if constexpr (XMODE == 1) {
    const int lane = (int)threadIdx.x & 63;
    const int wx0 = x0 - lane * VEC;  // first node of this wave
    if (lane < NC)
      halo = src[pidx(g, 0 * NC + lane, y, wrapx(wx0 - 1))];
    else if (lane < 2 * NC)
      halo = src[pidx(g, 2 * NC + lane - NC, y, wrapx(wx0 + 64 * VEC))];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float a[VEC], b[VEC], d[VEC], e[VEC];
    vload<VEC>(src + pidx(g, 0 * NC + c, y, x0), a);
    vload<VEC>(src + pidx(g, 2 * NC + c, y, x0), b);
    vload<VEC>(src + pidx(g, 1 * NC + c, yb, x0), d);
    vload<VEC>(src + pidx(g, 3 * NC + c, yt, x0), e);
    float al, br;
    if constexpr (XMODE == 0) {
      al = src[pidx(g, 0 * NC + c, y, wrapx(x0 - 1))];
      br = src[pidx(g, 2 * NC + c, y, wrapx(x0 + VEC))];
    } else {
      const int lane = (int)threadIdx.x & 63;
      const float hl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(halo), c));
      const float hr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(halo), NC + c));
      const float up = __shfl_up(a[VEC - 1], 1, 64);
      const float dn = __shfl_down(b[0], 1, 64);
      al = lane == 0 ? hl : up;
      br = lane == 63 ? hr : dn;
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      f[k][0][c] = k == 0 ? al : a[k - 1];
      f[k][2][c] = k == VEC - 1 ? br : b[k + 1];
      f[k][1][c] = d[k];
      f[k][3][c] = e[k];
    }
  }

  if (BC == LBM_DIRICHLET) {
    // Eq. bc_ansatz for links that cross a wall (corner nodes: both links)
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const int x = x0 + k;
      float fb[NC], va, vb;
      if (x == 0) {
        for (int c = 0; c < NC; ++c) fb[c] = src[pidx(g, 2 * NC + c, y, x)];
        wall_velocity(w, y, va, vb);
        wall_rule(1, 0, sc.kK, sc.km, va, vb, fb, f[k][0]);
      }
      if (x == nx - 1) {
        for (int c = 0; c < NC; ++c) fb[c] = src[pidx(g, 0 * NC + c, y, x)];
        wall_velocity(w, ny + y, va, vb);
        wall_rule(-1, 0, sc.kK, sc.km, va, vb, fb, f[k][2]);
      }
      if (y == 0) {
        for (int c = 0; c < NC; ++c) fb[c] = src[pidx(g, 3 * NC + c, y, x)];
        wall_velocity(w, 2 * ny + x, va, vb);
        wall_rule(0, 1, sc.kK, sc.km, va, vb, fb, f[k][1]);
      }
      if (y == ny - 1) {
        for (int c = 0; c < NC; ++c) fb[c] = src[pidx(g, 1 * NC + c, y, x)];
        wall_velocity(w, 2 * ny + nx + x, va, vb);
        wall_rule(0, -1, sc.kK, sc.km, va, vb, fb, f[k][3]);
      }
    }
  }

#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    if constexpr (FORCE || DISP) {
      // U_num = sum_q f_q + B_hat / 2 (Eq. cond_eq)
      float U[NC];
      moment0(f[k], U);
      if constexpr (FORCE) {
        float bx, by;
        body_hat(ex.F, x0 + k, y, bx, by);
        U[0] += 0.5f * bx;
        U[1] += 0.5f * by;
      }
      if constexpr (DISP) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          // FP64 running sum: FP32 would add a rounding of the full
          // displacement at every half step
          double* p = ex.D + ((int64_t)d * ny + y) * nx + x0 + k;
          const double u = *p + ex.half_dt * (double)U[d];
          *p = u + ex.half_dt * (double)U[d];
        }
      }
      collide_with(sc.kK, sc.km, U, f[k]);
    } else {
      collide(sc.kK, sc.km, f[k]);
    }
  }

#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      float o[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) o[k] = f[k][q][c];
      vstore<VEC, NT>(dst + pidx(g, q * NC + c, y, x0), o);
    }
}

template <int BC, int VEC, int THREADS, int NT, int XMODE>
__global__ __launch_bounds__(THREADS) void k_step(const float* __restrict__ src,
                                                  float* __restrict__ dst, Grid g, StepConst sc,
                                                  Wall w) {
  const int tile = xcd_tile(blockIdx.x, sc.ntiles);
  const int y = tile / sc.tiles_x;
  const int tx = tile - y * sc.tiles_x;
  step_segment<BC, VEC, THREADS, NT, XMODE>(src, dst, g, sc.kK, sc.km, w, y, tx);
}

// Steps with a body load and/or displacement output: one node per thread,
// 256 threads, plain loads and stores.
template <int BC, bool FORCE, bool DISP>
__global__ __launch_bounds__(256) void k_step_ext(const float* __restrict__ src,
                                                  float* __restrict__ dst, Grid g, StepConst sc,
                                                  Wall w, StepExtra ex) {
  const int tile = xcd_tile(blockIdx.x, sc.ntiles);
  const int y = tile / sc.tiles_x;
  const int tx = tile - y * sc.tiles_x;
  step_segment<BC, 1, 256, 0, 0, FORCE, DISP>(src, dst, g, sc.kK, sc.km, w, y, tx, ex);
}

// ---------------------------------------------------------------------------
// Launch configurations
// ---------------------------------------------------------------------------
typedef void (*StepFn)(const float*, float*, Grid, StepConst, Wall);

struct StepConfig {
  int vec, threads, nt, xmode;
  StepFn fn[2];  // [bc]
};

#define LBM_CFG(V, T, N, X) \
  {V, T, N, X, {&k_step<LBM_PERIODIC, V, T, N, X>, &k_step<LBM_DIRICHLET, V, T, N, X>}}

// Index 0 is the default for grids with nx % 4 == 0.
static const StepConfig kStepConfigs[] = {
    LBM_CFG(4, 256, 0, 0), LBM_CFG(4, 256, 1, 0), LBM_CFG(4, 256, 0, 1), LBM_CFG(4, 256, 1, 1),
    LBM_CFG(4, 128, 0, 0), LBM_CFG(4, 128, 1, 0), LBM_CFG(4, 128, 0, 1), LBM_CFG(4, 128, 1, 1),
    LBM_CFG(4, 512, 0, 0), LBM_CFG(4, 512, 1, 0), LBM_CFG(4, 512, 0, 1), LBM_CFG(4, 512, 1, 1),
    LBM_CFG(4, 64, 0, 0),  LBM_CFG(4, 64, 1, 0),  LBM_CFG(4, 64, 0, 1),  LBM_CFG(4, 64, 1, 1),
    LBM_CFG(2, 256, 0, 0), LBM_CFG(2, 256, 1, 0), LBM_CFG(2, 256, 0, 1), LBM_CFG(2, 256, 1, 1),
    LBM_CFG(2, 128, 0, 0), LBM_CFG(2, 128, 1, 0), LBM_CFG(2, 128, 0, 1), LBM_CFG(2, 128, 1, 1),
    LBM_CFG(2, 512, 0, 0), LBM_CFG(2, 512, 1, 0), LBM_CFG(2, 64, 0, 1),  LBM_CFG(2, 64, 1, 1),
    LBM_CFG(1, 256, 0, 0), LBM_CFG(1, 256, 1, 0), LBM_CFG(1, 64, 0, 0),  LBM_CFG(1, 64, 1, 0),
    LBM_CFG(1, 128, 0, 1), LBM_CFG(1, 256, 0, 1),
};
#undef LBM_CFG

constexpr int kNumStepConfigs = (int)(sizeof(kStepConfigs) / sizeof(kStepConfigs[0]));

inline bool step_config_valid(int i, int nx) {
  if (i < 0 || i >= kNumStepConfigs) return false;
  const StepConfig& c = kStepConfigs[i];
  if (nx % c.vec != 0) return false;
  if (c.xmode == 1 && nx % (64 * c.vec) != 0) return false;
  return true;
}

inline int default_step_config(int nx) {
  for (int i = 0; i < kNumStepConfigs; ++i) {
    const StepConfig& c = kStepConfigs[i];
    if (c.threads == 256 && c.nt == 0 && c.xmode == 0 && step_config_valid(i, nx)) return i;
  }
  return -1;
}

inline StepConst step_const(const StepConfig& c, const Grid& g, float kK, float km) {
  StepConst sc;
  sc.kK = kK;
  sc.km = km;
  const int per = c.threads * c.vec;
  sc.tiles_x = (g.nx + per - 1) / per;
  sc.ntiles = sc.tiles_x * g.ny;
  return sc;
}

}  // namespace lbmk
