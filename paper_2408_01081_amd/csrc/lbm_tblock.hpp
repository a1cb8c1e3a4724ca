// T time steps per pass over HBM (temporal blocking in registers).
//
// One wave owns a strip of 64 consecutive columns and sweeps a segment of
// output rows.  Level 0 is the post-collision state f*(t_n) read from memory;
// level l (1 <= l <= T) is f*(t_{n+l}).  At sub-iteration i of the sweep
// (output row y0 + i) the wave
//   loads   level 0 row y0 + i + T + PF      (PF rows ahead of its use),
//   forms   level l row y0 + i + T - l       (l = 1 .. T) from level l-1 rows
//           y0 + i + T - l - 1 .. y0 + i + T - l + 1,
//   stores  level T row y0 + i.
// Only level T goes back to memory: 80 B read + 80 B written per node for T
// node updates.
//   x neighbours: one-lane DPP wave shifts; lane edges lose one exact column
//     per level, so level T is exact on lanes T .. 63-T: strips overlap by 2T
//     columns and store 64 - 2T columns;
//   y neighbours: rows kept in registers.  Level l needs rows from
//     sub-iterations i-2 .. i of level l-1, so every level is a ring of
//     3 + PF slots holding the row of sub-iteration i in slot i mod (3 + PF);
//     the sweep is unrolled by the ring length, so slots rotate by renaming
//     and a row is never copied between registers (the wait for a prefetched
//     row sits at its first use).  Before the first output row, 2T
//     sub-iterations fill the pipeline, each computing only the levels whose
//     rows the segment needs.
// Rows are addressed with buffer instructions: a wave-uniform resource per row
// (scalar registers), the plane offset as scalar offset and the column as
// 32-bit lane offset.  Lanes that must not store give an offset beyond the
// resource's range, which the hardware drops: stores need no branch, so the
// wait counts stay exact.
// Walls (Dirichlet) are applied at every level with the velocities of that
// level's step.  Every node update is the single-step kernel's moment and
// collision on the same inputs, so the result is bitwise identical to T
// launches of it.  Optional extras per launch: a separable body load (row
// factors staged through LDS) and the FP64 displacement state (the rows a
// wave owns kept in LDS), each added in the single-step kernel's order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"

namespace lbmk {

constexpr int TB_LANES = 64;

struct TBConst {
  float kK, km;
  int nstrips;   // strips across a row (of the launch)
  int seg_rows;  // output rows per segment
  int nseg;      // segments along y
  int plane4;    // bytes between planes
  int extent;    // bytes one row's resource covers: (NP - 1) planes + one row
  // the launch's tiles: strips strip_first .. + nstrips - 1, segment k holds
  // output rows y_first + k seg_rows .. (up to y_end - 1); or, when band_hi >
  // band_lo (the wall band of a split Dirichlet step), every segment of the
  // strips outside [band_lo, band_hi) and only the first and last seg_rows
  // rows of the strips inside (see band_tile)
  int strip_first, y_first, y_end;
  int band_lo, band_hi;
  int band_rows;  // wall band: rows at the top and at the bottom of the strips inside
};

// Wall velocities of the launch's steps: level l (step n + l - 1) reads the
// summed table V + (l-1) 2L (nullptr: walls at rest).
struct WallSeq {
  const float* V;
  int L;  // 2 (nx + ny)
};

// Body load of a blocked launch (Eq. cond_eq: U_num = sum f + B_hat / 2),
// the separable sum of the single-step kernel's body_hat: each lane keeps its
// column's coefficients X[r][c][x] (ranks >= rank padded with +0) and the
// launch's row factors rows[l][y][r] = Y[r][y] T_{n+l+1}[r] (padded with -0)
// are staged through LDS (fac_request, fac_stage, fac_read below).  A padded term adds +0 * -0 = -0, which
// leaves every sum unchanged in round-to-nearest, so the result is bitwise
// the single-step kernel's.
constexpr int TB_MAXR = 32;  // largest rank the blocked kernel takes (variants of 16 and 32)
struct TBExtra {
  const float* X;     // [rank][2][nx]
  const float* rows;  // [T][ny][MR], written before the launch (MR: the variant's ranks)
  int rank;
  float scale;        // dt / rho
  double* D;          // [2][ny][nx] FP64 displacement state (launches that keep it)
  double half_dt;     // dt / 2
};

// FP64 displacement state D = u + dt/2 v_num of a blocked launch: every step
// adds dt/2 v_num twice, u = D + dt/2 U, D = u + dt/2 U (the single-step
// kernel's operations), so each row is updated at its T levels in order.  A
// wave keeps the rows it owns in an LDS ring of TB_DSLOTS rows (16 B per
// lane: both components), requested two sub-iterations before their first
// level, staged one before, and written back after their last level.
constexpr int TB_DSLOTS = 16;
template <int MR>
struct LaneLoad {
  float x[2][MR];
};

// B_hat (c = 0, 1) of this lane's node from the row factors yt
template <int MR>
__device__ __forceinline__ void load_terms(const LaneLoad<MR>& ll, const float (&yt)[MR],
                                           float scale, float& bx, float& by) {
  float a = 0.f, b = 0.f;
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    a = fmaf(ll.x[0][r], yt[r], a);
    b = fmaf(ll.x[1][r], yt[r], b);
  }
  bx = scale * a;
  by = scale * b;
}

constexpr int TB_RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer access (gfx9 family)
constexpr int TB_DROP = (int)0x80000000u;  // lane offset beyond every row's range

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
// lane without a source reads 0 (bound control), and its result is never
// stored
__device__ inline float from_lane_below(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_lane_above(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Shifted operands folded into the add / subtract that consumes them (DPP
// source operand, wave_shr:1 reads lane - 1, wave_shl:1 lane + 1, bound
// control as in the shifts above).  The compiler folds a separate shift only
// when all its uses follow within a few instructions, which the blocked
// kernel's long sub-iterations defeat, so the two blocks below are assembler.
// A DPP instruction must not read a register that one of the two VALU
// instructions before it wrote; the compiler's hazard check does not look
// inside an assembler block, so each block opens with five or more plain VALU
// instructions that write none of the registers its DPP instructions read
// from outside, and every in-block value is read three or more instructions
// after it is written.  Outputs are early-clobber: no input register is
// overwritten before the block has read it.

// U_c = f2_c(lane + 1) + (f0_c(lane - 1) + (f1_c + f3_c)), c = 0 .. 4 (the
// association of moment0); s is scratch.
__device__ __forceinline__ void moment_shifted(const float f0[NC], const float f1[NC],
                                               const float f2[NC], const float f3[NC],
                                               float U[NC]) {
  float s[NC];
  asm volatile(
      "v_add_f32 %5, %15, %25\n\t"
      "v_add_f32 %6, %16, %26\n\t"
      "v_add_f32 %7, %17, %27\n\t"
      "v_add_f32 %8, %18, %28\n\t"
      "v_add_f32 %9, %19, %29\n\t"
      "v_add_f32_dpp %5, %10, %5 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %6, %11, %6 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %7, %12, %7 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %8, %13, %8 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %9, %14, %9 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %0, %20, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %1, %21, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %2, %22, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %3, %23, %8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %4, %24, %9 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=&v"(U[0]), "=&v"(U[1]), "=&v"(U[2]), "=&v"(U[3]), "=&v"(U[4]), "=&v"(s[0]),
        "=&v"(s[1]), "=&v"(s[2]), "=&v"(s[3]), "=&v"(s[4])
      : "v"(f0[0]), "v"(f0[1]), "v"(f0[2]), "v"(f0[3]), "v"(f0[4]), "v"(f1[0]), "v"(f1[1]),
        "v"(f1[2]), "v"(f1[3]), "v"(f1[4]), "v"(f2[0]), "v"(f2[1]), "v"(f2[2]), "v"(f2[3]),
        "v"(f2[4]), "v"(f3[0]), "v"(f3[1]), "v"(f3[2]), "v"(f3[3]), "v"(f3[4]));
}

// o0_c = fma(U_c, 1/2, X_c) - f0_c(lane - 1) and o2_c = fma(U_c, 1/2, -X_c)
// - f2_c(lane + 1): the collision of populations 0 and 2 (collide_with).
__device__ __forceinline__ void collide_shifted(const float U[NC], const float X[NC],
                                                const float f0[NC], const float f2[NC],
                                                float o0[NC], float o2[NC]) {
  asm volatile(
      "v_fma_f32 %0, %10, 0.5, %15\n\t"
      "v_fma_f32 %1, %11, 0.5, %16\n\t"
      "v_fma_f32 %2, %12, 0.5, %17\n\t"
      "v_fma_f32 %3, %13, 0.5, %18\n\t"
      "v_fma_f32 %4, %14, 0.5, %19\n\t"
      "v_fma_f32 %5, %10, 0.5, -%15\n\t"
      "v_fma_f32 %6, %11, 0.5, -%16\n\t"
      "v_fma_f32 %7, %12, 0.5, -%17\n\t"
      "v_fma_f32 %8, %13, 0.5, -%18\n\t"
      "v_fma_f32 %9, %14, 0.5, -%19\n\t"
      "v_subrev_f32_dpp %0, %20, %0 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %1, %21, %1 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %2, %22, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %3, %23, %3 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %4, %24, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %5, %25, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %6, %26, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %7, %27, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %8, %28, %8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_subrev_f32_dpp %9, %29, %9 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=&v"(o0[0]), "=&v"(o0[1]), "=&v"(o0[2]), "=&v"(o0[3]), "=&v"(o0[4]), "=&v"(o2[0]),
        "=&v"(o2[1]), "=&v"(o2[2]), "=&v"(o2[3]), "=&v"(o2[4])
      : "v"(U[0]), "v"(U[1]), "v"(U[2]), "v"(U[3]), "v"(U[4]), "v"(X[0]), "v"(X[1]),
        "v"(X[2]), "v"(X[3]), "v"(X[4]), "v"(f0[0]), "v"(f0[1]), "v"(f0[2]), "v"(f0[3]),
        "v"(f0[4]), "v"(f2[0]), "v"(f2[1]), "v"(f2[2]), "v"(f2[3]), "v"(f2[4]));
}

// one level-update of row y at this lane's column x from the rows below,
// at and above (post-collision values of the previous level).  EDGE: the
// wave's columns include a Dirichlet wall column (x = 0 or nx - 1), whose
// lanes replace a shifted population by the wall rule; other waves of a
// Dirichlet lattice meet walls only in rows 0 and ny - 1, a branch uniform
// across the wave.
template <int BC, bool EDGE, bool FORCE, int MR>
__device__ __forceinline__ void level_update(const float below[NP], const float at[NP],
                                    const float above[NP], int x, int y, int nx, int ny,
                                    float kK, float km, const Wall& w, const LaneLoad<MR>& ll,
                                    const float (&yt)[MR], float scale, float out[NP],
                                    float (&Uo)[2]) {
  // the load terms first: they do not depend on the populations
  float bx = 0.f, by = 0.f;
  if constexpr (FORCE) load_terms(ll, yt, scale, bx, by);
  if constexpr (BC == LBM_PERIODIC || !EDGE) {
    // collide() on f_0 = f*_0(x - 1), f_1 = f*_1(y - 1), f_2 = f*_2(x + 1),
    // f_3 = f*_3(y + 1) (or the wall rule in the rows next to a wall) with
    // the same operations in the same order
    float f1[NC], f3[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      f1[c] = below[1 * NC + c];
      f3[c] = above[3 * NC + c];
    }
    if constexpr (BC == LBM_DIRICHLET) {
      float va, vb;
      if (y == 0) {
        wall_velocity(w, 2 * ny + x, va, vb);
        wall_rule(0, 1, kK, km, va, vb, at + 3 * NC, f1);
      }
      if (y == ny - 1) {
        wall_velocity(w, 2 * ny + nx + x, va, vb);
        wall_rule(0, -1, kK, km, va, vb, at + 1 * NC, f3);
      }
    }
    float U[NC];
    moment_shifted(at + 0 * NC, f1, at + 2 * NC, f3, U);
    if constexpr (FORCE) {
      U[0] += 0.5f * bx;
      U[1] += 0.5f * by;
    }
    Uo[0] = U[0];
    Uo[1] = U[1];
    float X[NC], Y[NC];
    X[0] = fmaf(kK, U[2], km * U[3]);
    X[1] = km * U[4];
    X[2] = kK * U[0];
    X[3] = km * U[0];
    X[4] = km * U[1];
    Y[0] = km * U[4];
    Y[1] = fmaf(kK, U[2], -(km * U[3]));
    Y[2] = kK * U[1];
    Y[3] = -(km * U[1]);
    Y[4] = km * U[0];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      out[1 * NC + c] = fmaf(0.5f, U[c], Y[c]) - f1[c];
      out[3 * NC + c] = fmaf(0.5f, U[c], -Y[c]) - f3[c];
    }
    collide_shifted(U, X, at + 0 * NC, at + 2 * NC, out + 0 * NC, out + 2 * NC);
    return;
  }
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
    // the side walls' velocities of this row are the same in every lane:
    // read them through the scalar cache before the lanes diverge (a vector
    // load inside the branch would wait for every prefetched row as well)
    float la = 0.f, lb = 0.f, ra = 0.f, rb = 0.f;
    if (w.V) {
      typedef const __attribute__((address_space(4))) float* ConstV;
      const ConstV v = (ConstV)w.V;
      la = v[2 * y];
      lb = v[2 * y + 1];
      ra = v[2 * (ny + y)];
      rb = v[2 * (ny + y) + 1];
    }
    if (x == 0) {
      for (int c = 0; c < NC; ++c) fb[c] = at[2 * NC + c];
      wall_rule(1, 0, kK, km, la, lb, fb, f[0]);
    }
    if (x == nx - 1) {
      for (int c = 0; c < NC; ++c) fb[c] = at[0 * NC + c];
      wall_rule(-1, 0, kK, km, ra, rb, fb, f[2]);
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
  float U[NC];
  moment0(f, U);
  if constexpr (FORCE) {
    U[0] += 0.5f * bx;
    U[1] += 0.5f * by;
  }
  Uo[0] = U[0];
  Uo[1] = U[1];
  collide_with(kK, km, U, f);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) out[q * NC + c] = f[q][c];
}

// Per-lane constants of one wave's strip.
struct Strip {
  int xw;   // column for the wall tests (-2 for lanes outside the grid)
  int xr4;  // byte offset of the column this lane reads
  int xs4;  // byte offset of the column this lane stores, or TB_DROP
};

// Level-0 rows are read in sweep order y0 - T, y0 - T + 1, ... up to the last
// row the segment needs and then that row again; the cursor holds the sweep
// row and the row it reads (periodic wrap or wall clamp) and advances by one
// compare and add instead of a wrap per row.  A row's base address is formed
// in 64 bits (scalar), so lattices of any size the workspace holds are
// addressed correctly; within a row the plane and column offsets fit in 32
// bits (tblock_fits).
struct RowCursor {
  int y;     // sweep row of the next load
  int r;     // row it reads
  int last;  // last level-0 row the segment needs
};

template <int BC>
__device__ __forceinline__ void cursor_advance(RowCursor& c, int ny) {
  if (c.y < c.last) {
    ++c.y;
    if (BC == LBM_PERIODIC) {
      c.r = c.r + 1 == ny ? 0 : c.r + 1;
    } else {
      c.r = c.y < 0 ? 0 : (c.y >= ny ? ny - 1 : c.y);
    }
  }
}

__device__ __forceinline__ void load_row(const float* __restrict__ src, int pitch4,
                                         const TBConst& sc, const Strip& st, int r, float v[NP]) {
  const char* rp = (const char*)src + (int64_t)r * pitch4;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)rp, (short)0, sc.extent, TB_RSRC_WORD3);
#pragma unroll
  for (int k = 0; k < NP; ++k)
    v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, st.xr4, k * sc.plane4, 0));
}

// update of row y of level l from the rows below, at and above it; rows off
// the grid (computed only to be dropped or replaced by a wall) use any valid
// row for their wall lookups
template <int BC, bool EDGE, bool FORCE, int MR>
__device__ __forceinline__ void row_update(const float below[NP], const float at[NP],
                                           const float above[NP], int xw, int y, int level,
                                           const Grid& g, const TBConst& sc, const WallSeq& ws,
                                           const TBExtra& F, const LaneLoad<MR>& ll,
                                           const float (&yt)[MR], float out[NP],
                                           float (&Uo)[2]) {
  const int yc = y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y);
  Wall w;
  w.L = ws.L;
  w.V = ws.V ? ws.V + (int64_t)(level - 1) * 2 * ws.L : nullptr;
  w.W = nullptr;
  w.rank = 0;
  w.Trow = nullptr;
  level_update<BC, EDGE, FORCE, MR>(below, at, above, xw, yc, g.nx, g.ny, sc.kK, sc.km, w, ll,
                                    yt, F.scale, out, Uo);
}

// Row factors through LDS.  A sub-iteration j needs the factors of its T
// level rows, the table f[e], e = 16 (l - 1) + r (level l, rank r): lane k
// holds elements k and k + 64.  At sub-iteration i the wave requests them for
// sub-iteration i + 2 (vector loads, before the population prefetch), writes
// those of i + 1 (requested at i - 1) into that sub-iteration's LDS slot, and
// its level updates read their 16 factors from slot i (the same address in
// every lane: broadcast reads).  The node a row stands for: on a periodic
// lattice the rows beyond the grid are the wrapped rows (one wrap suffices:
// the host takes this path only for ny >= T + ring length); on a Dirichlet
// lattice their loads are never used (clamped).
template <int BC, int T, int MR>
__device__ __forceinline__ void fac_request(const TBExtra& F, const Grid& g, int y0, int j,
                                            float (&v)[(MR * T + 63) / 64]) {
  constexpr int FE = (MR * T + 63) / 64;  // factors per lane
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < FE; ++k) {
    const int e = lane + 64 * k;
    v[k] = 0.f;
    if (e < MR * T) {
      const int l = e / MR + 1, r = e % MR;
      const int y = y0 + j + T - l;
      int yl = y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y);
      if (BC == LBM_PERIODIC) yl = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
      v[k] = F.rows[((int64_t)(l - 1) * g.ny + yl) * MR + r];
    }
  }
}

template <int T, int MR>
__device__ __forceinline__ void fac_stage(float* slot, const float (&v)[(MR * T + 63) / 64]) {
  constexpr int FE = (MR * T + 63) / 64;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < FE; ++k)
    if (lane + 64 * k < MR * T) slot[lane + 64 * k] = v[k];
  // the wave's later reads of the slot see these writes (LDS operations of
  // a wave complete in order); keep the compiler from moving them
  __builtin_amdgcn_wave_barrier();
}

template <int MR>
__device__ __forceinline__ void fac_read(const float* slot, int level, float (&yt)[MR]) {
  const float4* p = reinterpret_cast<const float4*>(slot + (level - 1) * MR);
#pragma unroll
  for (int q = 0; q < MR / 4; ++q) {
    const float4 v = p[q];
    yt[4 * q] = v.x;
    yt[4 * q + 1] = v.y;
    yt[4 * q + 2] = v.z;
    yt[4 * q + 3] = v.w;
  }
}

// displacement rows: request (global loads of this lane's read column),
// stage into the LDS ring, update at one level, write back (lanes that own
// their column; the others get an offset beyond the row's range)
__device__ __forceinline__ void d_request(const TBExtra& F, const Grid& g, const Strip& st, int y,
                                          double (&v)[2]) {
  const int xc = st.xr4 >> 2;
#pragma unroll
  for (int c = 0; c < 2; ++c) v[c] = F.D[((int64_t)c * g.ny + y) * g.nx + xc];
}

__device__ __forceinline__ double* d_slot(double* dring, int y) {
  return dring + ((y & (TB_DSLOTS - 1)) * TB_LANES + (threadIdx.x & 63)) * 2;
}

__device__ __forceinline__ void d_stage(double* dring, int y, const double (&v)[2]) {
  double* p = d_slot(dring, y);
  p[0] = v[0];
  p[1] = v[1];
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void d_update(double (&d)[2], const float (&U)[2], double h) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double u = d[c] + h * (double)U[c];
    d[c] = u + h * (double)U[c];
  }
}

__device__ __forceinline__ void d_store(const TBExtra& F, const Grid& g, int doff, int y,
                                        const double (&d)[2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double* rp = F.D + ((int64_t)c * g.ny + y) * g.nx;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)rp, (short)0, (int)(g.nx * 8), TB_RSRC_WORD3);
    const uint64_t bits = (uint64_t)__double_as_longlong(d[c]);
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)bits, rs, doff, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(bits >> 32), rs, doff, 4, 0);
  }
}

// One level update of a row inside a sub-iteration, with the displacement
// rows when the launch keeps them (rows the wave owns: y0 <= y < y1)
template <int BC, bool EDGE, bool FORCE, bool DISP, int MR>
__device__ __forceinline__ void level_step(const float below[NP], const float at[NP],
                                           const float above[NP], int xw, int y, int level,
                                           const Grid& g, const TBConst& sc, const WallSeq& ws,
                                           const TBExtra& F, const LaneLoad<MR>& ll,
                                           const float (&yt)[MR], float out[NP],
                                           double* dring, int y0, int y1, int doff, bool last) {
  float Uo[2];
  if constexpr (DISP) {
    if (y >= y0 && y < y1) {
      double* p = d_slot(dring, y);
      double d[2] = {p[0], p[1]};
      row_update<BC, EDGE, FORCE, MR>(below, at, above, xw, y, level, g, sc, ws, F, ll, yt, out,
                                      Uo);
      d_update(d, Uo, F.half_dt);
      p[0] = d[0];
      p[1] = d[1];
      if (last) d_store(F, g, doff, y, d);
      return;
    }
  }
  row_update<BC, EDGE, FORCE, MR>(below, at, above, xw, y, level, g, sc, ws, F, ll, yt, out, Uo);
}

// One sub-iteration i of the sweep (PRE: a pipeline-filling sub-iteration
// before the first output row, I = i then; slot = i mod NB, known at compile
// time in both cases).
template <int BC, int NT, int PF, int T, bool EDGE, bool FORCE, bool DISP, int MR, bool PRE>
__device__ __forceinline__ void sub_iteration(const float* __restrict__ src, float* __restrict__ dst,
                                     const Grid& g, const TBConst& sc, const Strip& st,
                                     const WallSeq& ws, const TBExtra& F, const LaneLoad<MR>& ll,
                                     float* fac, float (&fv)[3 + PF][(MR * T + 63) / 64],
                                     double* dring,
                                     double (&dv)[3 + PF][2], int doff,
                                     int pitch4, RowCursor& cur, int y0,
                                     int y1, int i, int I, int slot, float (&lv0)[3 + PF][NP],
                                     float (&lv)[T - 1][3 + PF][NP]) {
  constexpr int NB = 3 + PF;
  constexpr int FS = MR * T;  // floats of one LDS factor slot
  const int s = slot, s1 = (slot + NB - 1) % NB, s2 = (slot + NB - 2) % NB;
  if constexpr (FORCE) fac_request<BC, T, MR>(F, g, y0, i + 2, fv[(s + 2) % NB]);
  // displacement row whose first level comes two sub-iterations on
  if constexpr (DISP) {
    const int yq = y0 + i + 2 + T - 1;
    if (yq >= y0 && yq < y1) d_request(F, g, st, yq, dv[(s + 2) % NB]);
  }
  // prefetch level-0 row y0 + i + T + PF (the cursor's row) into slot
  // (i + PF) mod NB, which held the row of sub-iteration i + PF - NB = i - 3
  // (no longer read).  Past the last needed row it re-reads that row (a
  // cache hit).
  load_row(src, pitch4, sc, st, cur.r, lv0[(slot + PF) % NB]);
  cursor_advance<BC>(cur, g.ny);
  // keep the prefetch at the head of the sub-iteration: the scheduler would
  // sink it towards its first use and shorten the distance it hides
  __builtin_amdgcn_sched_barrier(0);
  // level 1 .. T-1: level l row y0 + i + T - l; during the pipeline fill only
  // the levels whose rows the segment needs (I >= -2 (T - l)).  With a load
  // the factors of level l + 1 are read from LDS before level l is formed
  // (yt[l mod 2] holds level l's).
  float yt[2][MR];
  if constexpr (FORCE) {
    fac_stage<T, MR>(fac + ((s + 1) % NB) * FS, fv[(s + 1) % NB]);
    fac_read(fac + s * FS, 1, yt[1]);
    fac_read(fac + s * FS, 2, yt[0]);
  }
  if constexpr (DISP) {
    const int yq = y0 + i + 1 + T - 1;
    if (yq >= y0 && yq < y1) d_stage(dring, yq, dv[(s + 1) % NB]);
  }
  if (!PRE || I >= -2 * (T - 1))
    level_step<BC, EDGE, FORCE, DISP, MR>(lv0[s2], lv0[s1], lv0[s], st.xw, y0 + i + T - 1, 1, g, sc,
                                      ws, F, ll, yt[1], lv[0][s], dring, y0, y1, doff, false);
#pragma unroll
  for (int l = 2; l < T; ++l) {
    if constexpr (FORCE) fac_read(fac + s * FS, l + 1, yt[(l + 1) & 1]);
    if (PRE && I < -2 * (T - l)) continue;
    level_step<BC, EDGE, FORCE, DISP, MR>(lv[l - 2][s2], lv[l - 2][s1], lv[l - 2][s], st.xw,
                                      y0 + i + T - l, l, g, sc, ws, F, ll, yt[l & 1],
                                      lv[l - 1][s], dring, y0, y1, doff, false);
  }
  if (!PRE) {
    // level T, output row y0 + i
    float o[NP];
    const int rr = y0 + i;
    level_step<BC, EDGE, FORCE, DISP, MR>(lv[T - 2][s2], lv[T - 2][s1], lv[T - 2][s], st.xw, rr, T,
                                      g, sc, ws, F, ll, yt[T & 1], o, dring, y0, y1, doff, true);
    const int off = rr < y1 ? st.xs4 : TB_DROP;
    const int yo = rr < g.ny ? rr : g.ny - 1;
    char* rp = (char*)dst + (int64_t)yo * pitch4;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)rp, (short)0, sc.extent, TB_RSRC_WORD3);
#pragma unroll
    for (int k = 0; k < NP; ++k)  // aux 2: nontemporal
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[k]), rs, off, k * sc.plane4,
                                            NT ? 2 : 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// The sweep of one wave over output rows y0 .. y1 - 1 (EDGE: see level_update).
template <int BC, int NT, int PF, int T, bool EDGE, bool FORCE, bool DISP, int MR>
__device__ __forceinline__ void tblock_sweep(const float* __restrict__ src,
                                             float* __restrict__ dst, const Grid& g,
                                             const TBConst& sc, const Strip& st,
                                             const WallSeq& ws, const TBExtra& F,
                                             const LaneLoad<MR>& ll, float* fac, double* dring,
                                             int doff, int pitch4, RowCursor& cur, int y0,
                                             int y1) {
  constexpr int NB = 3 + PF;
  const int ny = g.ny;
  // displacement rows requested two sub-iterations ahead (dv), staged one
  // ahead; the first row with a level in the pipeline fill is y0 at
  // sub-iteration 1 - T, requested in the fill itself
  double dv[NB][2];
  // load factors: requested two sub-iterations ahead (fv), staged in LDS one
  // ahead; the first sub-iteration's are staged here
  float fv[NB][(MR * T + 63) / 64];
  if constexpr (FORCE) {
    constexpr int first = -2 * T;
    fac_request<BC, T, MR>(F, g, y0, first, fv[((first % NB) + NB) % NB]);
    fac_request<BC, T, MR>(F, g, y0, first + 1, fv[(((first + 1) % NB) + NB) % NB]);
    fac_stage<T, MR>(fac + (((first % NB) + NB) % NB) * MR * T, fv[((first % NB) + NB) % NB]);
  }
  float lv0[NB][NP];        // level 0: row of sub-iteration i is y0 + i + T
  float lv[T - 1][NB][NP];  // level l: row of sub-iteration i is y0 + i + T - l
  // level-0 rows of the first PF sub-iterations of the pipeline fill
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    constexpr int first = -2 * T;
    load_row(src, pitch4, sc, st, cur.r, lv0[((first + k) % NB + NB) % NB]);
    cursor_advance<BC>(cur, ny);
  }
  // pipeline fill: sub-iterations -2T .. -1
#pragma unroll
  for (int p = 0; p < 2 * T; ++p) {
    const int I = p - 2 * T;
    sub_iteration<BC, NT, PF, T, EDGE, FORCE, DISP, MR, true>(src, dst, g, sc, st, ws, F, ll, fac, fv,
                                                          dring, dv, doff, pitch4, cur, y0, y1, I,
                                                          I, (I % NB + NB) % NB, lv0, lv);
  }
  // The sweep runs in whole rings of NB rows; rows past the segment end are
  // computed from valid (wrapped or clamped) rows and their stores dropped.
  // No early exit inside a ring: a conditional exit would let the compiler
  // sink each prefetch past it, next to its first use.
  for (int i0 = 0; i0 < y1 - y0; i0 += NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      sub_iteration<BC, NT, PF, T, EDGE, FORCE, DISP, MR, false>(src, dst, g, sc, st, ws, F, ll, fac,
                                                             fv, dring, dv, doff, pitch4, cur, y0,
                                                             y1, i0 + j, 0, j, lv0, lv);
  }
}

// One wave's work: strip `strip`, output rows y0 .. y1 - 1.
template <int BC, int NT, int PF, int T, bool FORCE = false, bool DISP = false, int MR = 16>
__device__ __forceinline__ void tblock_wave(const float* __restrict__ src, float* __restrict__ dst,
                                   const Grid& g, const TBConst& sc, const WallSeq& ws,
                                   int strip, int y0, int y1, const TBExtra& F = TBExtra{},
                                   float* fac = nullptr, double* dring = nullptr) {
  static_assert(T >= 2 && T <= 10, "2 to 10 time levels per launch");
  constexpr int VALID = TB_LANES - 2 * T;  // stored columns per strip
  const int lane = threadIdx.x & 63;
  const int nx = g.nx, ny = g.ny;
  const int x = strip * VALID - T + lane;  // unwrapped column of this lane
  const int xc = BC == LBM_PERIODIC ? wrap_mod(x, nx) : (x < 0 ? 0 : (x >= nx ? nx - 1 : x));
  const bool store = lane >= T && lane < TB_LANES - T && x >= 0 && x < nx;
  Strip st;
  st.xw = (x >= 0 && x < nx) ? x : -2;
  st.xr4 = (int)((uint32_t)xc * 4u);
  st.xs4 = store ? (int)((uint32_t)x * 4u) : TB_DROP;
  const int pitch4 = (int)(g.pitch * 4);
  RowCursor cur;
  cur.y = y0 - T;
  cur.r = row_index<BC>(cur.y, ny);
  cur.last = y1 - 1 + T;
  // byte offset of this lane's column in a displacement row (doubles), or
  // beyond the row for lanes that do not own their column
  const int doff = store ? (int)((uint32_t)x * 8u) : TB_DROP;
  // this lane's load coefficients (the column it reads)
  LaneLoad<MR> ll;
  if constexpr (FORCE) {
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        ll.x[c][r] = r < F.rank ? F.X[((int64_t)r * 2 + c) * nx + xc] : 0.f;
  }
  if constexpr (BC == LBM_DIRICHLET) {
    // a Dirichlet wave meets the side walls only if its columns include one
    const int x_first = strip * VALID - T;
    if (x_first <= 0 || x_first + TB_LANES - 1 >= nx - 1) {
      tblock_sweep<BC, NT, PF, T, true, FORCE, DISP, MR>(src, dst, g, sc, st, ws, F, ll, fac, dring,
                                                     doff, pitch4, cur, y0, y1);
      return;
    }
  }
  tblock_sweep<BC, NT, PF, T, false, FORCE, DISP, MR>(src, dst, g, sc, st, ws, F, ll, fac, dring, doff,
                                                  pitch4, cur, y0, y1);
}

// Tiles of a launch (see TBConst): their number, and strip and output rows
// of tile `wid`.  The wall band of a split Dirichlet step lists the
// segments of the strips outside [band_lo, band_hi) first, then the top and
// bottom band_rows rows of each strip inside.
__device__ __forceinline__ int tile_count(const TBConst& sc) {
  const int inner = sc.band_hi - sc.band_lo;
  return inner > 0 ? (sc.nstrips - inner) * sc.nseg + 2 * inner : sc.nstrips * sc.nseg;
}
__device__ __forceinline__ void tile_of(const TBConst& sc, int ny, int wid, int& strip, int& y0,
                                        int& y1) {
  const int inner = sc.band_hi - sc.band_lo;
  if (inner <= 0) {
    const int seg = wid / sc.nstrips;
    strip = sc.strip_first + (wid - seg * sc.nstrips);
    y0 = sc.y_first + seg * sc.seg_rows;
    y1 = y0 + sc.seg_rows < sc.y_end ? y0 + sc.seg_rows : sc.y_end;
    return;
  }
  const int wside = (sc.nstrips - inner) * sc.nseg;
  if (wid < wside) {
    const int k = wid / sc.nseg, seg = wid - k * sc.nseg;
    strip = k < sc.band_lo ? k : sc.band_hi + (k - sc.band_lo);
    y0 = seg * sc.seg_rows;
    y1 = y0 + sc.seg_rows < ny ? y0 + sc.seg_rows : ny;
  } else {
    const int k = wid - wside;
    strip = sc.band_lo + (k >> 1);
    y0 = (k & 1) ? ny - sc.band_rows : 0;
    y1 = y0 + sc.band_rows;
  }
}

template <int BC, int NT, int PF, int T, bool FORCE = false, bool DISP = false, int MR = 16>
__global__ __launch_bounds__(256) void k_tblock(const float* __restrict__ src,
                                                float* __restrict__ dst, Grid g, TBConst sc,
                                                WallSeq ws, TBExtra F) {
  const int ntiles = tile_count(sc);
  const int nwg = (ntiles + 3) / 4;
  // wave index: uniform by construction, stated to the compiler
  const int wid = xcd_tile(blockIdx.x, nwg) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wid >= ntiles) return;  // whole waves exit together
  // per wave: one slot of load factors per ring row (unused without a load)
  __shared__ __attribute__((aligned(16))) float fac[FORCE ? 4 * (3 + PF) * MR * T : 4];
  float* mine = FORCE ? fac + (threadIdx.x >> 6) * (3 + PF) * MR * T : nullptr;
  // per wave: the displacement rows in flight (unused without them)
  __shared__ __attribute__((aligned(16))) double dring[DISP ? 4 * TB_DSLOTS * TB_LANES * 2 : 2];
  double* dmine = DISP ? dring + (threadIdx.x >> 6) * TB_DSLOTS * TB_LANES * 2 : nullptr;
  int strip, y0, y1;
  tile_of(sc, g.ny, wid, strip, y0, y1);
  tblock_wave<BC, NT, PF, T, FORCE, DISP, MR>(src, dst, g, sc, ws, strip, y0, y1, F, mine, dmine);
}

// A split Dirichlet launch in one grid: waves 0 .. (band tiles - 1) sweep the
// wall band (`band`, a band launch's tiles) with the Dirichlet rule, the
// others the interior (`in`) with the periodic kernel's code, which the
// Dirichlet rule never reaches there (the branch is uniform per wave; each
// path keeps its own register assignment).
template <int NT, int PF, int T>
__global__ __launch_bounds__(256) void k_tblock_split(const float* __restrict__ src,
                                                      float* __restrict__ dst, Grid g,
                                                      TBConst band, TBConst in, WallSeq ws) {
  const int nb = tile_count(band);
  const int ntiles = nb + tile_count(in);
  const int nwg = (ntiles + 3) / 4;
  const int wid = xcd_tile(blockIdx.x, nwg) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wid >= ntiles) return;
  int strip, y0, y1;
  if (wid < nb) {
    tile_of(band, g.ny, wid, strip, y0, y1);
    tblock_wave<LBM_DIRICHLET, NT, PF, T>(src, dst, g, band, ws, strip, y0, y1);
  } else {
    tile_of(in, g.ny, wid - nb, strip, y0, y1);
    tblock_wave<LBM_PERIODIC, NT, PF, T>(src, dst, g, in, ws, strip, y0, y1);
  }
}

inline TBConst tblock_const(const Grid& g, float kK, float km, int seg_rows, int T) {
  TBConst sc;
  sc.kK = kK;
  sc.km = km;
  sc.nstrips = (g.nx + (TB_LANES - 2 * T) - 1) / (TB_LANES - 2 * T);
  sc.seg_rows = seg_rows;
  sc.nseg = (g.ny + seg_rows - 1) / seg_rows;
  sc.plane4 = (int)(g.plane * 4);
  sc.extent = (int)(((NP - 1) * g.plane + g.nx) * 4);
  sc.strip_first = 0;
  sc.y_first = 0;
  sc.y_end = g.ny;
  sc.band_lo = sc.band_hi = 0;
  sc.band_rows = 0;
  return sc;
}

// the byte offsets inside one row's resource (19 plane strides + one row)
// must stay below 2^31; row base addresses are 64-bit
inline bool tblock_fits(const Grid& g) {
  return ((NP - 1) * g.plane + g.pitch) * 4 < ((int64_t)1 << 31);
}

}  // namespace lbmk
