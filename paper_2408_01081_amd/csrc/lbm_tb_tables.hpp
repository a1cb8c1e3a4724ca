// Launch variants of the blocked kernel (k_tblock, several time steps per
// launch) and the tables of their kernels.  The kernels are instantiated in
// several translation units (lbm_tb_*.hip) that compile in parallel; each
// fills its part of a table of host-side kernel handles, which the entry
// points launch.
#pragma once

#include <utility>

#include "lbm_tblock.hpp"

namespace lbmk {

typedef void (*TBFn)(const float*, float*, Grid, TBConst, WallSeq, TBExtra);

// T steps per launch, output rows per segment (0: as many as give one wave per
// resident slot across the grid, -k: k waves per slot, TB_SEG_SIMD: one wave
// per SIMD whatever the occupancy), nontemporal stores, level-0 rows
// prefetched ahead.
struct TBVariant {
  int steps, seg_rows, nt, pf;
};
constexpr int TB_SEG_SIMD = -100;
constexpr int TB_MAX_STEPS = 10;  // most steps of a launch

// Load-free variants; the index is the public variant number
// (lbm_tblock_config_info), so entries are only ever appended.
constexpr TBVariant kTBVariants[] = {
    {2, 4, 0, 1},  {2, 4, 1, 1},  {2, 8, 0, 1},  {2, 0, 0, 1},  {3, 4, 0, 1},  {3, 5, 0, 2},
    {3, 4, 1, 1},  {3, 8, 1, 1},  {4, 4, 0, 1},  {4, 8, 0, 1},  {4, 4, 1, 1},  {4, 8, 1, 1},
    {4, 12, 1, 1}, {5, 16, 0, 1}, {5, 32, 0, 1}, {5, 16, 1, 1}, {6, 16, 0, 1}, {6, 32, 0, 1},
    {6, 48, 0, 1}, {6, 16, 1, 1}, {7, 32, 0, 1}, {7, 48, 0, 1}, {7, 64, 0, 1}, {7, 32, 1, 1},
    {7, 0, 0, 1},  {7, -2, 0, 1}, {6, 0, 0, 1},  {5, 0, 0, 1},  {7, 16, 0, 1}, {7, 24, 0, 1},
    {7, 20, 0, 2}, {7, 30, 0, 2}, {6, 8, 0, 1},  {6, 12, 0, 1}, {6, 20, 0, 2}, {6, 30, 0, 2},
    {8, 20, 0, 2}, {8, 30, 0, 2}, {8, 24, 0, 1}, {8, 32, 0, 1}, {8, 0, 0, 2},  {8, -2, 0, 2},
    {8, 0, 0, 1},  {7, 0, 0, 2},  {4, 0, 0, 1},  {3, 0, 0, 1},  {4, 375, 0, 2}, {5, 375, 0, 2},
    {4, TB_SEG_SIMD, 0, 3}, {5, TB_SEG_SIMD, 0, 3}, {3, TB_SEG_SIMD, 0, 3}, {2, TB_SEG_SIMD, 0, 3},
    {10, -2, 0, 2}, {10, 0, 0, 2}, {9, 0, 0, 2}};
constexpr int kNumTBVariants = (int)(sizeof(kTBVariants) / sizeof(kTBVariants[0]));
constexpr bool tb_steps_in_range() {
  for (const TBVariant& v : kTBVariants)
    if (v.steps < 2 || v.steps > TB_MAX_STEPS) return false;
  return true;
}
static_assert(tb_steps_in_range(), "steps per launch in 2 .. TB_MAX_STEPS");
// the load-free tables are filled in two halves per boundary type
constexpr int kTBSplit = 24;

// Variants with a body load and/or the FP64 displacement state.  mr: load
// ranks the kernels take (16 or 32); mask: bit 2 m + bc is set when the
// kernel for extras m (0 load, 1 displacement, 2 both) and boundary type bc
// exists (at T = 8 only the periodic kernel with a load fits in registers, at
// T = 7 the periodic kernel with the displacement state alone); main: the
// variant serves whole runs (the others, T = 2 .. 5, take the steps left over
// after the last full launch).
struct TBExtVariant {
  int steps, seg_rows, nt, pf, mr;
  unsigned mask;
  bool main;
};
constexpr unsigned kTBXAll16 = 0x3f;  // every extras kind, both boundary types
constexpr unsigned kTBXLoad32 = 0x33; // load and load + displacement, both types
constexpr TBExtVariant kTBExtVariants[] = {
    {8, 0, 0, 2, 16, 0x01, true},       {7, 0, 0, 2, 16, 0x04, true},
    {6, 0, 0, 2, 16, 0x14, true},       {6, 16, 1, 1, 16, kTBXAll16, true},
    {6, 0, 0, 2, 32, 0x01, true},       {6, 0, 0, 1, 32, 0x10, true},
    {6, 16, 1, 1, 32, kTBXLoad32, true},
    {5, 16, 1, 1, 16, kTBXAll16, false}, {4, 16, 1, 1, 16, kTBXAll16, false},
    {3, 16, 1, 1, 16, kTBXAll16, false}, {2, 16, 1, 1, 16, kTBXAll16, false},
    {5, 16, 1, 1, 32, kTBXLoad32, false}, {4, 16, 1, 1, 32, kTBXLoad32, false},
    {3, 16, 1, 1, 32, kTBXLoad32, false}, {2, 16, 1, 1, 32, kTBXLoad32, false}};
constexpr int kNumTBExtVariants = (int)(sizeof(kTBExtVariants) / sizeof(kTBExtVariants[0]));
constexpr int kTBExtSplit = 7;

typedef TBFn TBExtFns[3][2];

// ---- instantiation helpers (used by the lbm_tb_*.hip units) ---------------
template <int BC, int LO, int... K>
void tb_fill_range(TBFn* out, std::integer_sequence<int, K...>) {
  ((out[LO + K] = &k_tblock<BC, kTBVariants[LO + K].nt, kTBVariants[LO + K].pf,
                            kTBVariants[LO + K].steps>),
   ...);
}

template <int I, int M, int BC>
void tbx_put(TBExtFns* out) {
  constexpr TBExtVariant v = kTBExtVariants[I];
  if constexpr ((v.mask >> (2 * M + BC)) & 1u)
    out[I][M][BC] = &k_tblock<BC, v.nt, v.pf, v.steps, M != 1, M != 0, v.mr>;
  else
    out[I][M][BC] = nullptr;
}

template <int I>
void tbx_put_all(TBExtFns* out) {
  tbx_put<I, 0, 0>(out);
  tbx_put<I, 0, 1>(out);
  tbx_put<I, 1, 0>(out);
  tbx_put<I, 1, 1>(out);
  tbx_put<I, 2, 0>(out);
  tbx_put<I, 2, 1>(out);
}

template <int LO, int... K>
void tbx_fill_range(TBExtFns* out, std::integer_sequence<int, K...>) {
  (tbx_put_all<LO + K>(out), ...);
}

// Kernels of split Dirichlet launches (k_tblock_split): T, nontemporal
// stores, rows prefetched.  A load-free variant with the same three runs
// split.  (At T = 8 the Dirichlet path keeps scratch spills, which make the
// wall band slower than the unsplit launch.)
struct TBSplitVariant {
  int steps, nt, pf;
};
constexpr TBSplitVariant kTBSplitVariants[] = {{7, 0, 1}, {7, 0, 2}, {6, 0, 1},
                                               {6, 0, 2}, {5, 0, 1}};
constexpr int kNumTBSplitVariants =
    (int)(sizeof(kTBSplitVariants) / sizeof(kTBSplitVariants[0]));
typedef void (*TBSplitFn)(const float*, float*, Grid, TBConst, TBConst, WallSeq);

template <int... K>
void tbs_fill(TBSplitFn* out, std::integer_sequence<int, K...>) {
  ((out[K] = &k_tblock_split<kTBSplitVariants[K].nt, kTBSplitVariants[K].pf,
                             kTBSplitVariants[K].steps>),
   ...);
}

// ---- the parts, one per translation unit ----------------------------------
void tb_fill_periodic_a(TBFn* out);   // lbm_tb_pa.hip: periodic, [0, kTBSplit)
void tb_fill_periodic_b(TBFn* out);   // lbm_tb_pb.hip: periodic, [kTBSplit, n)
void tb_fill_dirichlet_a(TBFn* out);  // lbm_tb_da.hip
void tb_fill_dirichlet_b(TBFn* out);  // lbm_tb_db.hip
void tb_fill_extra_a(TBExtFns* out);  // lbm_tb_xa.hip: [0, kTBExtSplit)
void tb_fill_extra_b(TBExtFns* out);  // lbm_tb_xb.hip: [kTBExtSplit, n)
void tb_fill_split(TBSplitFn* out);   // lbm_tb_sp.hip: the split kernels

}  // namespace lbmk
