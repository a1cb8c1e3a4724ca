// Two time steps per pass over HBM (temporal blocking in registers).
//
// One wave owns a strip of 64 consecutive columns and sweeps a segment of
// rows.  For every row it loads the post-collision populations f*(t_n) of
// one row ahead, forms the intermediate level f*(t_{n+1}) of the row above
// the output row, then the output level f*(t_{n+2}) of the output row, and
// stores only that: 80 B read + 80 B written per node for two updates.
//   x neighbours: one-lane DPP wave shifts; the two edge lanes of the strip
//     cannot see beyond it, so level n+1 is exact on lanes 1..62 and level
//     n+2 on lanes 2..61: strips overlap by 4 columns and store 60 columns;
//   y neighbours: the previous and next rows of the sweep, kept in registers;
//     a segment starts with two rows of warm-up.
// Row buffers form rings whose slots rotate by renaming (the sweep is unrolled
// by the ring length), so a prefetched row is never copied between registers
// and the wait for it sits at its first use, PF rows after its load; the
// stores of earlier rows stay in flight meanwhile.  Rows are addressed with
// buffer instructions: a wave-uniform resource per row (scalar registers), the
// plane offset as scalar offset and the column as 32-bit lane offset.  Lanes
// that must not store give an offset beyond the resource's range, which the
// hardware drops: the stores need no branch, so the wait counts stay exact.
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
  int plane4;    // bytes between planes
  int extent;    // bytes one row's resource covers: (NP - 1) planes + one row
};

constexpr int S2_RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer access (gfx9 family)
constexpr int S2_DROP = (int)0x80000000u;  // lane offset beyond every row's range

__device__ inline int wrap_mod(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}

// row actually read for sweep row y (uniform): periodic wrap or wall clamp
template <int BC>
__device__ inline int row_index(int y, int ny) {
  if (BC == LBM_PERIODIC) {
    while (y < 0) y += ny;
    while (y >= ny) y -= ny;
    return y;
  }
  return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// value held by lane - 1 (wave_shr:1) and by lane + 1 (wave_shl:1); the
// lane without a source reads 0, and its result is never stored
__device__ inline float from_lane_below(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ inline float from_lane_above(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
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
    f[0][c] = from_lane_below(at[0 * NC + c]);  // f*_0 from x - 1
    f[1][c] = below[1 * NC + c];
    f[2][c] = from_lane_above(at[2 * NC + c]);  // f*_2 from x + 1
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

// Per-lane constants of one wave's strip.
struct Strip {
  int xw;       // column for the wall tests (-2 for lanes outside the grid)
  int xr4;      // byte offset of the column this lane reads
  int xs4;      // byte offset of the column this lane stores, or S2_DROP
};

template <int BC>
__device__ inline void load_row(const float* __restrict__ src, const Grid& g,
                                const Step2Const& sc, const Strip& st, int y, float v[NP]) {
  const float* rp = src + (int64_t)row_index<BC>(y, g.ny) * g.pitch;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)rp, (short)0, sc.extent, S2_RSRC_WORD3);
#pragma unroll
  for (int k = 0; k < NP; ++k)
    v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, st.xr4, k * sc.plane4, 0));
}

// update of row y from the rows below, at and above it; rows off the grid
// (computed only to be dropped or replaced by a wall) use any valid row for
// their wall lookups
template <int BC>
__device__ inline void row_update(const float below[NP], const float at[NP],
                                  const float above[NP], int xw, int y, const Grid& g,
                                  const Step2Const& sc, const Wall& w, float out[NP]) {
  const int yc = y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y);
  level_update<BC>(below, at, above, xw, yc, g.nx, g.ny, sc.kK, sc.km, w, out);
}

// One wave's sweep over output rows y0 .. y1-1: output row r needs level n+1
// rows r-1 .. r+1 and level n rows r-2 .. r+2.
template <int BC, int NT, int PF>
__device__ inline void sweep(const float* __restrict__ src, float* __restrict__ dst,
                             const Grid& g, const Step2Const& sc, const Strip& st, int y0, int y1,
                             const Wall& w0, const Wall& w1) {
  constexpr int NB = 3 + PF;  // ring length
  const int count = y1 - y0;
  const int last_in = y1 + 1;  // last level-n row the sweep needs

  // level-n ring: row y0 + i in slot i % NB; level-n+1 ring: row y0 + i - 1
  // in slot i % NB
  float nb[NB][NP], mb[NB][NP], o[NP];
  {
    float t0[NP], t1[NP];
    load_row<BC>(src, g, sc, st, y0 - 2, t0);
    load_row<BC>(src, g, sc, st, y0 - 1, t1);
    load_row<BC>(src, g, sc, st, y0, nb[0]);
    load_row<BC>(src, g, sc, st, y0 + 1, nb[1]);
    row_update<BC>(t0, t1, nb[0], st.xw, y0 - 1, g, sc, w0, mb[0]);
    row_update<BC>(t1, nb[0], nb[1], st.xw, y0, g, sc, w0, mb[1]);
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) load_row<BC>(src, g, sc, st, y0 + 2 + k, nb[2 + k]);

  // The sweep runs in whole rings of NB rows; rows past the segment end are
  // computed from valid (wrapped or clamped) rows and their stores dropped.
  // No early exit inside a ring: a conditional exit would let the compiler
  // sink each prefetch past it, next to its first use.
  for (int i0 = 0; i0 < count; i0 += NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = i0 + j;
      const int rr = y0 + i;
      // prefetch level-n row rr + 2 + PF into the slot of row rr - 1 (no
      // longer read); unconditional, so the wait counts are the same on every
      // path.  Past the last needed row it re-reads that row (a cache hit)
      // instead of fetching one more from memory.
      const int yl = rr + 2 + PF < last_in ? rr + 2 + PF : last_in;
      load_row<BC>(src, g, sc, st, yl, nb[(j + NB - 1) % NB]);
      // keep the prefetch at the head of the row: the scheduler would sink it
      // towards its first use and shorten the distance it hides
      __builtin_amdgcn_sched_barrier(0);
      // level n+1, row rr + 1
      row_update<BC>(nb[j], nb[(j + 1) % NB], nb[(j + 2) % NB], st.xw, rr + 1, g, sc, w0,
                     mb[(j + 2) % NB]);
      // level n+2, row rr
      row_update<BC>(mb[j], mb[(j + 1) % NB], mb[(j + 2) % NB], st.xw, rr, g, sc, w1, o);
      {
        const int off = i < count ? st.xs4 : S2_DROP;
        const int yo = rr < 0 ? 0 : (rr >= g.ny ? g.ny - 1 : rr);
        float* rp = dst + (int64_t)yo * g.pitch;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)rp, (short)0, sc.extent, S2_RSRC_WORD3);
#pragma unroll
        for (int k = 0; k < NP; ++k)  // aux 2: nontemporal
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[k]), rs, off, k * sc.plane4,
                                                NT ? 2 : 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int BC, int NT, int PF>
__global__ __launch_bounds__(256) void k_step2(const float* __restrict__ src,
                                               float* __restrict__ dst, Grid g, Step2Const sc,
                                               Wall w0, Wall w1) {
  const int lane = threadIdx.x & 63;
  const int ntiles = sc.nstrips * sc.nseg;
  const int nwg = (ntiles + 3) / 4;
  // wave index: uniform by construction, stated to the compiler
  const int wid = xcd_tile(blockIdx.x, nwg) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wid >= ntiles) return;  // whole waves exit together
  const int strip = wid % sc.nstrips, seg = wid / sc.nstrips;
  const int nx = g.nx, ny = g.ny;
  const int x = strip * S2_VALID - 2 + lane;  // unwrapped column of this lane
  const int xc = BC == LBM_PERIODIC ? wrap_mod(x, nx) : (x < 0 ? 0 : (x >= nx ? nx - 1 : x));
  const bool store = lane >= 2 && lane < S2_LANES - 2 && x >= 0 && x < nx;
  Strip st;
  st.xw = (x >= 0 && x < nx) ? x : -2;
  st.xr4 = (int)((uint32_t)xc * 4u);
  st.xs4 = store ? (int)((uint32_t)x * 4u) : S2_DROP;
  const int y0 = seg * sc.seg_rows;
  const int y1 = y0 + sc.seg_rows < ny ? y0 + sc.seg_rows : ny;
  sweep<BC, NT, PF>(src, dst, g, sc, st, y0, y1, w0, w1);
}

inline Step2Const step2_const(const Grid& g, float kK, float km, int seg_rows) {
  Step2Const sc;
  sc.kK = kK;
  sc.km = km;
  sc.nstrips = (g.nx + S2_VALID - 1) / S2_VALID;
  sc.seg_rows = seg_rows;
  sc.nseg = (g.ny + seg_rows - 1) / seg_rows;
  sc.plane4 = (int)(g.plane * 4);
  sc.extent = (int)(((NP - 1) * g.plane + g.nx) * 4);
  return sc;
}

// the byte offsets of a row's resource must stay below 2^31
inline bool step2_fits(const Grid& g) {
  return ((NP - 1) * g.plane + g.pitch) * 4 < ((int64_t)1 << 31);
}

}  // namespace lbmk
