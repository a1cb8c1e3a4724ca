// Two time steps per pass over HBM (temporal blocking in registers).
//
// One wave owns a strip of 64 consecutive columns and sweeps a segment of
// rows.  For every row it loads the post-collision populations f*(t_n) of
// one row ahead, forms the intermediate level f*(t_{n+1}) of the row above
// the output row, then the output level f*(t_{n+2}) of the output row, and
// stores only that: 80 B read + 80 B written per node for two updates.
//   x neighbours: lane shuffles; the two edge lanes of the strip cannot see
//     beyond it, so level n+1 is exact on lanes 1..62 and level n+2 on lanes
//     2..61: strips overlap by 4 columns and store 60 columns each;
//   y neighbours: the previous and next rows of the sweep, kept in registers;
//     a segment starts with two rows of warm-up.
// Walls (Dirichlet) are applied at both levels with their own time rows.
// Every node update is collide() on the same inputs as the single-step
// kernel, so the result is bitwise identical to two launches of it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"

namespace lbmk {

constexpr int S2_LANES = 64;
constexpr int S2_VALID = S2_LANES - 4;  // stored columns per strip

struct Step2Const {
  float kK, km;
  int nstrips;   // strips across a row
  int seg_rows;  // output rows per segment
  int nseg;      // segments along y
};

__device__ inline int wrap_mod(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}

template <int BC>
__device__ inline int row_index(int y, int ny) {
  if (BC == LBM_PERIODIC) return wrap_mod(y, ny);
  return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// one level-update of row y at this lane's column x from the rows below,
// at and above (post-collision values of the previous level)
template <int BC>
__device__ inline void level_update(const float below[NP], const float at[NP],
                                    const float above[NP], int x, int y, int nx, int ny,
                                    float kK, float km, const Wall& w, float out[NP]) {
  float f[NQ][NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const float l = __shfl_up(at[0 * NC + c], 1, 64);    // f*_0 from x - 1
    const float r = __shfl_down(at[2 * NC + c], 1, 64);  // f*_2 from x + 1
    f[0][c] = l;
    f[1][c] = below[1 * NC + c];
    f[2][c] = r;
    f[3][c] = above[3 * NC + c];
  }
  if (BC == LBM_DIRICHLET) {
    float fb[NC], va, vb;
    if (x == 0) {
      for (int c = 0; c < NC; ++c) fb[c] = at[2 * NC + c];
      wall_velocity(w, y, va, vb);
      wall_rule(1, 0, kK, km, va, vb, fb, f[0]);
    }
    if (x == nx - 1) {
      for (int c = 0; c < NC; ++c) fb[c] = at[0 * NC + c];
      wall_velocity(w, ny + y, va, vb);
      wall_rule(-1, 0, kK, km, va, vb, fb, f[2]);
    }
    if (y == 0) {
      for (int c = 0; c < NC; ++c) fb[c] = at[3 * NC + c];
      wall_velocity(w, 2 * ny + x, va, vb);
      wall_rule(0, 1, kK, km, va, vb, fb, f[1]);
    }
    if (y == ny - 1) {
      for (int c = 0; c < NC; ++c) fb[c] = at[1 * NC + c];
      wall_velocity(w, 2 * ny + nx + x, va, vb);
      wall_rule(0, -1, kK, km, va, vb, fb, f[3]);
    }
  }
  collide(kK, km, f);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) out[q * NC + c] = f[q][c];
}

template <int BC, int NT, int PF>
__global__ __launch_bounds__(256) void k_step2(const float* __restrict__ src,
                                               float* __restrict__ dst, Grid g, Step2Const sc,
                                               Wall w0, Wall w1) {
  const int lane = threadIdx.x & 63;
  const int ntiles = sc.nstrips * sc.nseg;
  const int nwg = (ntiles + 3) / 4;
  const int wid = xcd_tile(blockIdx.x, nwg) * 4 + (threadIdx.x >> 6);
  if (wid >= ntiles) return;  // whole waves exit together
  const int strip = wid % sc.nstrips, seg = wid / sc.nstrips;
  const int nx = g.nx, ny = g.ny;
  const int x = strip * S2_VALID - 2 + lane;  // unwrapped column of this lane
  const int xc = BC == LBM_PERIODIC ? wrap_mod(x, nx) : (x < 0 ? 0 : (x >= nx ? nx - 1 : x));
  // column for the wall tests: out-of-range lanes never match a wall column
  const int xw = (x >= 0 && x < nx) ? x : -2;
  const bool store = lane >= 2 && lane < S2_LANES - 2 && x >= 0 && x < nx;
  const int y0 = seg * sc.seg_rows;
  const int y1 = y0 + sc.seg_rows < ny ? y0 + sc.seg_rows : ny;

  auto load = [&](int y, float v[NP]) {
    const float* p = src + (int64_t)row_index<BC>(y, ny) * g.pitch + xc;
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = p[(int64_t)k * g.plane];
  };

  float n0[NP], n1[NP], n2[NP], m0[NP], m1[NP], m2[NP], o[NP];
  // warm-up: level n rows y0-2 .. y0+1, level n+1 rows y0-1, y0
  float nm2[NP], nm1[NP];
  load(y0 - 2, nm2);
  load(y0 - 1, nm1);
  load(y0, n0);
  load(y0 + 1, n1);
  level_update<BC>(nm2, nm1, n0, xw, y0 - 1, nx, ny, sc.kK, sc.km, w0, m0);
  level_update<BC>(nm1, n0, n1, xw, y0, nx, ny, sc.kK, sc.km, w0, m1);
  // m0 = level n+1 row r-1, m1 = row r; n0 = level n row r, n1 = row r+1.
  // PF rows are prefetched ahead of their use (pre[0] = row r+2, ...).
  float pre[PF][NP];
#pragma unroll
  for (int k = 0; k < PF; ++k) load(y0 + 2 + k, pre[k]);
  for (int r = y0; r < y1; ++r) {
#pragma unroll
    for (int k = 0; k < NP; ++k) n2[k] = pre[0][k];
#pragma unroll
    for (int j = 0; j + 1 < PF; ++j)
#pragma unroll
      for (int k = 0; k < NP; ++k) pre[j][k] = pre[j + 1][k];
    if (r + PF < y1) load(r + 2 + PF, pre[PF - 1]);  // prefetch
    level_update<BC>(n0, n1, n2, xw, r + 1, nx, ny, sc.kK, sc.km, w0, m2);  // n+1, row r+1
    level_update<BC>(m0, m1, m2, xw, r, nx, ny, sc.kK, sc.km, w1, o);       // n+2, row r
    if (store) {
      float* p = dst + (int64_t)r * g.pitch + x;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        if (NT)
          __builtin_nontemporal_store(o[k], p + (int64_t)k * g.plane);
        else
          p[(int64_t)k * g.plane] = o[k];
      }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      n0[k] = n1[k];
      n1[k] = n2[k];
      m0[k] = m1[k];
      m1[k] = m2[k];
    }
  }
}

inline Step2Const step2_const(const Grid& g, float kK, float km, int seg_rows) {
  Step2Const sc;
  sc.kK = kK;
  sc.km = km;
  sc.nstrips = (g.nx + S2_VALID - 1) / S2_VALID;
  sc.seg_rows = seg_rows;
  sc.nseg = (g.ny + seg_rows - 1) / seg_rows;
  return sc;
}

}  // namespace lbmk
