// Batched lattices: many independent instances (uneven sizes, periodic or
// Dirichlet, their own material and time step) advanced together.
//
// Every instance keeps the single-lattice state layout (row-major, post-
// collision FP32 populations) inside two shared pools.  The unit of work is a
// row segment of one instance; a tile table maps the flattened workgroup
// index to (instance, row, segment), so one launch advances every instance by
// one step with the same per-node arithmetic as the single-lattice kernel
// (bitwise-identical results).  lbm_batch_step(n) runs n such launches as one
// hipGraph built node by node (no stream capture, no memset nodes).  With a
// temporally blocked variant selected, a node advances every instance by T
// steps: a second table maps each wave to (instance, strip, segment) and the
// wave runs the single-lattice blocked sweep on its instance.
//
// Packed field arrays (inputs and outputs of the batch) store instance i's
// fields contiguously, [component][ny_i][nx_i], starting at component count
// times the instance's first node (lbm_batch_node_offset).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_init.hpp"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"
#include "lbm_tblock.hpp"

using namespace lbmk;
using namespace lbmh;

namespace {

constexpr int BT = 256;  // threads per workgroup of the batched kernels

struct InstDesc {
  Grid g;
  int64_t off;    // float offset of the instance's state in each pool
  int64_t node0;  // first node of the instance in packed field arrays
  int tile0;      // first row-segment tile of the instance
  int tiles_x;    // row segments per row
  int bc;
  float kK, km, cK, cmu, rho;
  InitConst ic;
  double kw[NQ][NC][NC];  // norm weights
  const float* W;         // wall table or null
  const float* T;
  int rank;
  float* V;  // Dirichlet instances: [8][2 (nx + ny)][2] wall velocities of a blocked launch's steps
};

__device__ inline int find_instance(const InstDesc* __restrict__ d, int n, int64_t node) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].node0 <= node)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_batch_step(const float* __restrict__ pool_src,
                                                        float* __restrict__ pool_dst,
                                                        const InstDesc* __restrict__ descs,
                                                        const int* __restrict__ tile_inst,
                                                        int ntiles, int64_t step) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const InstDesc& d = descs[tile_inst[tile]];
  const int local = tile - d.tile0;
  const int y = local / d.tiles_x;
  const int tx = local - y * d.tiles_x;
  Wall w;
  w.rank = d.rank;
  w.W = d.W;
  w.Trow = d.rank ? d.T + step * d.rank : nullptr;
  w.L = 2 * (d.g.nx + d.g.ny);
  const float* src = pool_src + d.off;
  float* dst = pool_dst + d.off;
  if (d.bc == LBM_PERIODIC)
    step_segment<LBM_PERIODIC, 1, THREADS, 1, 0>(src, dst, d.g, d.kK, d.km, w, y, tx);
  else
    step_segment<LBM_DIRICHLET, 1, THREADS, 1, 0>(src, dst, d.g, d.kK, d.km, w, y, tx);
}

// V[s][link][2] of every instance with wall data: the wall velocities of
// steps step0 .. step0 + t - 1 (summed in rank order by wall_series, as the
// single-step kernel forms them).  Workgroup blockIdx.x covers instance
// blockIdx.x / per, its part blockIdx.x % per.
__global__ void k_batch_wall_eval(const InstDesc* __restrict__ descs, int per, int64_t step0,
                                  int t) {
  const InstDesc& d = descs[blockIdx.x / per];
  if (d.rank == 0) return;
  const int L = 2 * (d.g.nx + d.g.ny);
  const int64_t n = (int64_t)t * L;
  for (int64_t i = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)per * blockDim.x) {
    const int s = (int)(i / L), link = (int)(i - (int64_t)s * L);
    Wall w;
    w.W = d.W;
    w.Trow = d.T + (step0 + s) * d.rank;
    w.rank = d.rank;
    w.L = L;
    w.V = nullptr;
    float a, b;
    wall_series(w, link, a, b);
    d.V[2 * i] = a;
    d.V[2 * i + 1] = b;
  }
}

// T steps of every instance per launch; wave w works on instance
// waves[w].x, strip / segment index waves[w].y of that instance.  WALLS: an
// instance with wall data reads the velocities of the launch's steps from
// its table V (k_batch_wall_eval before the launch); without, walls rest
// (their velocities are the constant 0, which keeps the wall code's
// registers out of the kernel that serves batches without wall data).
template <int NT, int PF, int T, bool WALLS>
__global__ __launch_bounds__(256) void k_batch_tblock(const float* __restrict__ pool_src,
                                                      float* __restrict__ pool_dst,
                                                      const InstDesc* __restrict__ descs,
                                                      const int2* __restrict__ waves, int nwaves,
                                                      int seg_rows, int64_t step) {
  constexpr int VALID = TB_LANES - 2 * T;
  const int nwg = (nwaves + 3) / 4;
  const int wid = xcd_tile(blockIdx.x, nwg) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wid >= nwaves) return;  // whole waves exit together
  const int2 wv = waves[wid];
  const int inst = __builtin_amdgcn_readfirstlane(wv.x);
  const int local = __builtin_amdgcn_readfirstlane(wv.y);
  const InstDesc& d = descs[inst];
  TBConst sc;
  sc.kK = d.kK;
  sc.km = d.km;
  sc.nstrips = (d.g.nx + VALID - 1) / VALID;
  sc.seg_rows = seg_rows;
  sc.nseg = (d.g.ny + seg_rows - 1) / seg_rows;
  sc.plane4 = (int)(d.g.plane * 4);
  sc.extent = (int)(((NP - 1) * d.g.plane + d.g.nx) * 4);
  WallSeq ws;
  ws.V = WALLS && d.rank > 0 ? d.V : nullptr;
  ws.L = 2 * (d.g.nx + d.g.ny);
  const float* src = pool_src + d.off;
  float* dst = pool_dst + d.off;
  const int strip = local % sc.nstrips, seg = local / sc.nstrips;
  const int y0 = seg * seg_rows, y1 = y0 + seg_rows < d.g.ny ? y0 + seg_rows : d.g.ny;
  if (d.bc == LBM_PERIODIC)
    tblock_wave<LBM_PERIODIC, NT, PF, T>(src, dst, d.g, sc, ws, strip, y0, y1);
  else
    tblock_wave<LBM_DIRICHLET, NT, PF, T>(src, dst, d.g, sc, ws, strip, y0, y1);
}

typedef void (*BatchTBFn)(const float*, float*, const InstDesc*, const int2*, int, int, int64_t);
struct BatchTBConfig {
  int steps, seg_rows, nt, pf;
  BatchTBFn fn, fn_walls;  // walls at rest / wall tables
};
#define LBM_BTB(T, S, N, F) \
  {T, S, N, F, &k_batch_tblock<N, F, T, false>, &k_batch_tblock<N, F, T, true>}
const BatchTBConfig kBatchTB[] = {
    LBM_BTB(2, 4, 0, 1), LBM_BTB(2, 8, 1, 1),  LBM_BTB(3, 4, 0, 1),  LBM_BTB(3, 8, 0, 1),
    LBM_BTB(4, 4, 0, 1), LBM_BTB(4, 8, 0, 1),  LBM_BTB(4, 4, 1, 1),  LBM_BTB(4, 16, 0, 1),
    LBM_BTB(5, 8, 0, 1), LBM_BTB(5, 16, 0, 1), LBM_BTB(6, 16, 0, 1), LBM_BTB(7, 16, 0, 1),
    LBM_BTB(7, 32, 0, 1)};
#undef LBM_BTB
constexpr int kNumBatchTB = (int)(sizeof(kBatchTB) / sizeof(kBatchTB[0]));

// packed = 0: v0 [..][2][ny][nx] and s0 [..][3][ny][nx] separate arrays;
// packed = 1: one array [..][5][ny][nx] = (v, sigma_bar) in s0's place (v0 unused).
template <typename T>
__global__ __launch_bounds__(BT) void k_batch_init(const T* __restrict__ v0,
                                                   const T* __restrict__ s0, int packed,
                                                   float* __restrict__ pool,
                                                   const InstDesc* __restrict__ descs, int n,
                                                   int64_t total) {
  const int64_t node = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (node >= total) return;
  const InstDesc& d = descs[find_instance(descs, n, node)];
  const int64_t loc = node - d.node0;
  const int64_t ni = (int64_t)d.g.nx * d.g.ny;
  const int y = (int)(loc / d.g.nx), x = (int)(loc - (int64_t)y * d.g.nx);
  const T* v = packed ? s0 + 5 * d.node0 : v0 + 2 * d.node0;
  const T* s = packed ? s0 + 5 * d.node0 + 2 * ni : s0 + 3 * d.node0;
  init_node<T>(v, s, nullptr, pool + d.off, d.g, d.ic, x, y);
}

// mode 0: physical (v, sigma_bar); 1: U
__global__ __launch_bounds__(BT) void k_batch_moments(const float* __restrict__ pool,
                                                      float* __restrict__ out,
                                                      const InstDesc* __restrict__ descs, int n,
                                                      int64_t total, int mode) {
  const int64_t node = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (node >= total) return;
  const InstDesc& d = descs[find_instance(descs, n, node)];
  const int64_t loc = node - d.node0;
  const int64_t ni = (int64_t)d.g.nx * d.g.ny;
  const int y = (int)(loc / d.g.nx), x = (int)(loc - (int64_t)y * d.g.nx);
  const float* src = pool + d.off;
  float f[NQ][NC], U[NC];
  for (int q = 0; q < NQ; ++q)
    for (int c = 0; c < NC; ++c) f[q][c] = src[pidx(d.g, q * NC + c, y, x)];
  moment0(f, U);  // the single lattice's summation order
  float* o = out + 5 * d.node0 + loc;
  if (mode == 1) {
    for (int c = 0; c < NC; ++c) o[c * ni] = U[c];
    return;
  }
  o[0] = U[0];
  o[ni] = U[1];
  o[2 * ni] = -d.rho * (d.cK * U[2] + d.cmu * U[3]);
  o[3 * ni] = -d.rho * (d.cK * U[2] - d.cmu * U[3]);
  o[4 * ni] = -d.rho * (d.cmu * U[4]);
}

__device__ inline double wg_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = BT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per-tile partial sums in a fixed order.  mode 0: energy sum f*^T k f*;
// mode 1: judge sums against packed physical fields ref (FP32):
// a = sum |U - U(ref)|^2, b = sum |U|^2 over the U variables;
// mode 2: two packed field arrays, no lattice state:
// a = sum |U(ref) - U(ref2)|^2, b = sum |U(ref2)|^2.
__global__ __launch_bounds__(BT) void k_batch_reduce(const float* __restrict__ pool,
                                                     const float* __restrict__ ref,
                                                     const float* __restrict__ ref2,
                                                     const InstDesc* __restrict__ descs,
                                                     const int* __restrict__ tile_inst,
                                                     int mode, double* __restrict__ partial) {
  __shared__ double sh[BT];
  const int tile = blockIdx.x;
  const InstDesc& d = descs[tile_inst[tile]];
  const int local = tile - d.tile0;
  const int y = local / d.tiles_x;
  const int x = (local - y * d.tiles_x) * BT + (int)threadIdx.x;
  double a = 0.0, b = 0.0;
  if (x < d.g.nx && mode == 2) {
    const int64_t ni = (int64_t)d.g.nx * d.g.ny;
    const int64_t o = 5 * d.node0 + (int64_t)y * d.g.nx + x;
    double Ua[NC], Ub[NC];
    to_U(d.ic, ref[o], ref[o + ni], ref[o + 2 * ni], ref[o + 3 * ni], ref[o + 4 * ni], Ua);
    to_U(d.ic, ref2[o], ref2[o + ni], ref2[o + 2 * ni], ref2[o + 3 * ni], ref2[o + 4 * ni], Ub);
    for (int c = 0; c < NC; ++c) {
      const double e = Ua[c] - Ub[c];
      a += e * e;
      b += Ub[c] * Ub[c];
    }
  } else if (x < d.g.nx) {
    const float* src = pool + d.off;
    double f[NQ][NC];
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NC; ++c) f[q][c] = (double)src[pidx(d.g, q * NC + c, y, x)];
    if (mode == 0) {
      for (int q = 0; q < NQ; ++q)
        for (int r = 0; r < NC; ++r) {
          double t = 0.0;
          for (int c = 0; c < NC; ++c) t += d.kw[q][r][c] * f[q][c];
          a += f[q][r] * t;
        }
    } else {
      const int64_t ni = (int64_t)d.g.nx * d.g.ny;
      const float* rr = ref + 5 * d.node0 + (int64_t)y * d.g.nx + x;
      double Ur[NC];
      to_U(d.ic, rr[0], rr[ni], rr[2 * ni], rr[3 * ni], rr[4 * ni], Ur);
      for (int c = 0; c < NC; ++c) {
        // U in FP32 as the lattice forms it (moment0's order)
        const float u32 = (float)f[2][c] + ((float)f[0][c] + ((float)f[1][c] + (float)f[3][c]));
        const double u = (double)u32, e = u - Ur[c];
        a += e * e;
        b += u * u;
      }
    }
  }
  const double sa = wg_sum(a, sh);
  const double sb = wg_sum(b, sh);
  if (threadIdx.x == 0) {
    partial[2 * tile] = sa;
    partial[2 * tile + 1] = sb;
  }
}

// one workgroup per instance: sum its tiles' partials in a fixed order
__global__ __launch_bounds__(BT) void k_batch_reduce_final(const double* __restrict__ partial,
                                                           const InstDesc* __restrict__ descs,
                                                           const int* __restrict__ tile_count,
                                                           double* __restrict__ out) {
  __shared__ double sh[BT];
  const InstDesc& d = descs[blockIdx.x];
  const int nt = tile_count[blockIdx.x];
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < nt; t += BT) {
    a += partial[2 * (d.tile0 + t)];
    b += partial[2 * (d.tile0 + t) + 1];
  }
  const double sa = wg_sum(a, sh);
  const double sb = wg_sum(b, sh);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = sa;
    out[2 * blockIdx.x + 1] = sb;
  }
}

struct Layout {
  std::vector<InstDesc> desc;
  std::vector<int> tile_inst, tile_count;
  int64_t pool_floats = 0, total_nodes = 0;
  int ntiles = 0;
  int tb_waves[kNumBatchTB];    // waves of each blocked variant
  int64_t tb_wave0[kNumBatchTB];  // its wave table's first entry in the tables' region
  int64_t tb_all_waves = 0;
  bool tb_ok = true;          // every instance fits the blocked kernel
  size_t off_pool[2], off_desc, off_tiles, off_count, off_partial, off_out, off_waves, off_wallv,
      bytes;
  std::vector<int64_t> voff;  // float offset of each Dirichlet instance's wall table (-1: none)
  int max_links = 0;          // largest 2 (nx + ny) of a Dirichlet instance
};

constexpr int BATCH_TB_MAXT = 8;  // most steps of a blocked launch: rows of a wall table

// wave table of blocked variant `v`: (instance, strip + nstrips * segment)
std::vector<int2> wave_table(const Layout& L, int v) {
  const BatchTBConfig& k = kBatchTB[v];
  const int valid = TB_LANES - 2 * k.steps;
  std::vector<int2> t;
  for (int i = 0; i < (int)L.desc.size(); ++i) {
    const Grid& g = L.desc[i].g;
    const int n = ((g.nx + valid - 1) / valid) * ((g.ny + k.seg_rows - 1) / k.seg_rows);
    for (int j = 0; j < n; ++j) t.push_back(make_int2(i, j));
  }
  return t;
}

lbm_status plan(int32_t n, const lbm_params* params, Layout* L) {
  if (n < 1 || !params) return fail(LBM_E_ARG, "batch needs n >= 1 and parameters");
  L->desc.resize(n);
  L->tile_count.resize(n);
  L->voff.assign(n, -1);
  int64_t wallv_floats = 0;
  for (int i = 0; i < n; ++i) {
    Derived dv;
    lbm_status s = derive(&params[i], &dv);
    if (s) return fail(s, "instance " + std::to_string(i) + ": " + g_err);
    if (params[i].flags != 0)
      return fail(LBM_E_ARG, "batched instances take no flags (row layout, no displacement, CFL enforced)");
    // batched instances are initialised from stress fields, whose inverse
    // divides by c_mu
    if (!(params[i].mu > 0))
      return fail(LBM_E_ARG, "instance " + std::to_string(i) + ": batched instances need mu > 0");
    InstDesc& d = L->desc[i];
    memset(&d, 0, sizeof d);
    d.g = make_grid(&params[i]);
    d.off = L->pool_floats;
    L->pool_floats += round_up((int64_t)(state_bytes(d.g) / 4), 64);
    d.node0 = L->total_nodes;
    L->total_nodes += (int64_t)d.g.nx * d.g.ny;
    d.tiles_x = (d.g.nx + BT - 1) / BT;
    d.tile0 = L->ntiles;
    const int64_t nt = (int64_t)d.tiles_x * d.g.ny;
    if ((int64_t)L->ntiles + nt > 0x7fffffff) return fail(LBM_E_ARG, "batch too large");
    L->ntiles += (int)nt;
    L->tile_count[i] = (int)nt;
    d.bc = params[i].bc;
    d.kK = (float)dv.kK;
    d.km = (float)dv.km;
    d.cK = (float)dv.cK;
    d.cmu = (float)dv.cmu;
    d.rho = (float)params[i].rho;
    d.ic = InitConst{dv.kK, dv.km, dv.cK, dv.cmu, params[i].rho, params[i].dx, params[i].bc};
    if (!norm_weights(dv.kK, dv.km, d.kw)) return fail(LBM_E_CFL, "g_ij not positive definite");
    if (d.bc == LBM_DIRICHLET) {
      const int links = 2 * (d.g.nx + d.g.ny);
      L->voff[i] = wallv_floats;
      wallv_floats += round_up((int64_t)BATCH_TB_MAXT * links * 2, 64);
      if (links > L->max_links) L->max_links = links;
    }
  }
  for (int v = 0; v < kNumBatchTB; ++v) {
    const int valid = TB_LANES - 2 * kBatchTB[v].steps;
    int64_t w = 0;
    for (int i = 0; i < n; ++i) {
      const Grid& g = L->desc[i].g;
      w += (int64_t)((g.nx + valid - 1) / valid) *
           ((g.ny + kBatchTB[v].seg_rows - 1) / kBatchTB[v].seg_rows);
    }
    if (w > 0x7fffffff) return fail(LBM_E_ARG, "batch too large");
    L->tb_waves[v] = (int)w;
    L->tb_wave0[v] = L->tb_all_waves;
    L->tb_all_waves += w;
  }
  for (int i = 0; i < n; ++i) L->tb_ok = L->tb_ok && tblock_fits(L->desc[i].g);
  L->tile_inst.resize(L->ntiles);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < L->tile_count[i]; ++t) L->tile_inst[L->desc[i].tile0 + t] = i;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += (size_t)round_up((int64_t)b, 256);
    return at;
  };
  L->off_pool[0] = take((size_t)L->pool_floats * 4);
  L->off_pool[1] = take((size_t)L->pool_floats * 4);
  L->off_desc = take(sizeof(InstDesc) * n);
  L->off_tiles = take(sizeof(int) * L->ntiles);
  L->off_count = take(sizeof(int) * n);
  L->off_partial = take(sizeof(double) * 2 * (size_t)L->ntiles);
  L->off_out = take(sizeof(double) * 2 * n);
  L->off_waves = take(sizeof(int2) * (size_t)(L->tb_ok ? L->tb_all_waves : 0));
  L->off_wallv = take(sizeof(float) * (size_t)wallv_floats);
  L->bytes = o;
  return LBM_OK;
}

}  // namespace

struct lbm_batch {
  Layout L;
  int n;
  char* ws;
  hipStream_t stream;
  float* pool[2];
  InstDesc* d_desc;
  int* d_tiles;
  int* d_count;
  double* d_partial;
  double* d_out;
  int2* d_waves;  // wave tables of every blocked variant (uploaded at creation)
  int cur;
  bool initialised;
  int64_t nstep;
  std::vector<int64_t> wall_nsteps;
  bool any_wall;
  int tb_cfg;  // selected blocked variant, -1: one step per launch
  double tb_ms[kNumBatchTB];  // launch time of each variant the autotuner timed, -1: not timed
  // (steps, parity, blocked variant) -> graph, built while no instance has walls
  std::map<std::tuple<int64_t, int, int>, hipGraphExec_t> graphs;
};

namespace {

void drop_graphs(lbm_batch* b) {
  for (auto& kv : b->graphs) hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

lbm_status upload_descs(lbm_batch* b) {
  return hip_check(hipMemcpy(b->d_desc, b->L.desc.data(), sizeof(InstDesc) * b->n,
                             hipMemcpyHostToDevice),
                   "descriptor upload");
}

// The blocked variant that takes the last r (2 <= r < T) steps of a run in
// one launch after full launches of the selected variant: the fastest r-step
// variant the autotuner timed, else the r-step variant nearest to the
// selected one's shape (rows per segment, then store type and prefetch);
// -1 if none (no variant selected, or r outside 2 .. 7).
int remainder_variant(const lbm_batch* b, int r) {
  if (b->tb_cfg < 0 || r < 2 || r >= kBatchTB[b->tb_cfg].steps) return -1;
  const BatchTBConfig& t = kBatchTB[b->tb_cfg];
  int best = -1, best_score = -1;
  double best_ms = 1e300;
  for (int i = 0; i < kNumBatchTB; ++i) {
    const BatchTBConfig& k = kBatchTB[i];
    if (k.steps != r) continue;
    if (b->tb_ms[i] > 0.0) {
      if (best_score < 8 || b->tb_ms[i] < best_ms) {
        best_score = 8;
        best_ms = b->tb_ms[i];
        best = i;
      }
      continue;
    }
    const int score = (k.seg_rows == t.seg_rows ? 4 : 0) + (k.pf == t.pf ? 2 : 0) +
                      (k.nt == t.nt ? 1 : 0);
    if (score > best_score) {
      best_score = score;
      best = i;
    }
  }
  return best;
}

// Steps per launch for `steps` steps: T per launch with a blocked variant,
// then the r < T steps left as one launch of an r-step variant (r >= 2) or
// one step.
std::vector<int> launch_plan(const lbm_batch* b, int64_t steps) {
  std::vector<int> p;
  const int T = b->tb_cfg >= 0 ? kBatchTB[b->tb_cfg].steps : 1;
  int64_t k = 0;
  for (; T > 1 && k + T <= steps; k += T) p.push_back(T);
  if (T > 1 && steps - k >= 2 && remainder_variant(b, (int)(steps - k)) >= 0) {
    p.push_back((int)(steps - k));
    k = steps;
  }
  for (; k < steps; ++k) p.push_back(1);
  return p;
}

// Launch parameters of one launch advancing `t` steps from step index `step`
// (the step index matters only for wall tables).
struct LaunchArgs {
  const float* src;
  float* dst;
  const InstDesc* descs;
  const int* tiles;
  const int2* waves;
  int ntiles, nwaves, seg_rows;
  int64_t step;
  void* args[7];
  hipKernelNodeParams kp;
};

void make_launch(const lbm_batch* b, int t, int parity, int64_t step, LaunchArgs* a) {
  a->src = b->pool[parity];
  a->dst = b->pool[parity ^ 1];
  a->descs = b->d_desc;
  a->tiles = b->d_tiles;
  a->ntiles = b->L.ntiles;
  a->step = step;
  memset(&a->kp, 0, sizeof a->kp);
  a->kp.blockDim = dim3(BT);
  if (t == 1) {
    a->args[0] = (void*)&a->src;
    a->args[1] = (void*)&a->dst;
    a->args[2] = (void*)&a->descs;
    a->args[3] = (void*)&a->tiles;
    a->args[4] = (void*)&a->ntiles;
    a->args[5] = (void*)&a->step;
    a->kp.func = reinterpret_cast<void*>(&k_batch_step<BT>);
    a->kp.gridDim = dim3((unsigned)a->ntiles);
  } else {
    // the selected variant, or for the last steps of a run a shorter one
    const int v = t == kBatchTB[b->tb_cfg].steps ? b->tb_cfg : remainder_variant(b, t);
    const BatchTBConfig& k = kBatchTB[v];
    a->waves = b->d_waves + b->L.tb_wave0[v];
    a->nwaves = b->L.tb_waves[v];
    a->seg_rows = k.seg_rows;
    a->args[0] = (void*)&a->src;
    a->args[1] = (void*)&a->dst;
    a->args[2] = (void*)&a->descs;
    a->args[3] = (void*)&a->waves;
    a->args[4] = (void*)&a->nwaves;
    a->args[5] = (void*)&a->seg_rows;
    a->args[6] = (void*)&a->step;
    a->kp.func = reinterpret_cast<void*>(b->any_wall ? k.fn_walls : k.fn);
    a->kp.gridDim = dim3((unsigned)((a->nwaves + 3) / 4));
  }
  a->kp.kernelParams = a->args;
}

// The wall-table launch before a blocked launch of t steps from step index
// `step` (instances with wall data only).
struct WallEvalArgs {
  const InstDesc* descs;
  int per, t;
  int64_t step;
  void* args[4];
  hipKernelNodeParams kp;
};

void make_wall_eval(const lbm_batch* b, int t, int64_t step, WallEvalArgs* a) {
  a->descs = b->d_desc;
  a->t = t;
  a->step = step;
  const int64_t work = (int64_t)t * b->L.max_links;
  a->per = (int)((work + BT - 1) / BT);
  if (a->per > 16) a->per = 16;
  if (a->per < 1) a->per = 1;
  a->args[0] = (void*)&a->descs;
  a->args[1] = (void*)&a->per;
  a->args[2] = (void*)&a->step;
  a->args[3] = (void*)&a->t;
  memset(&a->kp, 0, sizeof a->kp);
  a->kp.func = reinterpret_cast<void*>(&k_batch_wall_eval);
  a->kp.gridDim = dim3((unsigned)(a->per * b->n));
  a->kp.blockDim = dim3(BT);
  a->kp.kernelParams = a->args;
}

// Build a graph of the launches for `steps` steps starting from buffer `cur`
// at step index `step0`.
lbm_status build_graph(lbm_batch* b, int64_t steps, int cur, int64_t step0,
                       hipGraphExec_t* exec) {
  hipGraph_t graph;
  lbm_status s = hip_check(hipGraphCreate(&graph, 0), "graph create");
  if (s) return s;
  hipGraphNode_t prev = nullptr;
  int parity = cur;
  int64_t step = step0;
  for (int t : launch_plan(b, steps)) {
    hipGraphNode_t node;
    if (t > 1 && b->any_wall) {
      WallEvalArgs w;
      make_wall_eval(b, t, step, &w);
      s = hip_check(hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                          &w.kp),
                    "graph add kernel node");
      if (s) break;
      prev = node;
    }
    LaunchArgs a;
    make_launch(b, t, parity, step, &a);
    s = hip_check(hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &a.kp),
                  "graph add kernel node");
    if (s) break;
    prev = node;
    parity ^= 1;
    step += t;
  }
  if (s == LBM_OK) s = hip_check(hipGraphInstantiate(exec, graph, nullptr, nullptr, 0),
                                 "graph instantiate");
  hipGraphDestroy(graph);
  return s;
}

void launch_direct(lbm_batch* b, int t, int parity, int64_t step) {
  if (t > 1 && b->any_wall) {
    WallEvalArgs w;
    make_wall_eval(b, t, step, &w);
    hipLaunchKernel(w.kp.func, w.kp.gridDim, w.kp.blockDim, w.kp.kernelParams, 0, b->stream);
  }
  LaunchArgs a;
  make_launch(b, t, parity, step, &a);
  hipLaunchKernel(a.kp.func, a.kp.gridDim, a.kp.blockDim, a.kp.kernelParams, 0, b->stream);
}

lbm_status batch_reduce(lbm_batch* b, int mode, const float* ref, double* h_out2,
                        const float* ref2 = nullptr) {
  hipLaunchKernelGGL(k_batch_reduce, dim3((unsigned)b->L.ntiles), dim3(BT), 0, b->stream,
                     (const float*)b->pool[b->cur], ref, ref2, (const InstDesc*)b->d_desc,
                     (const int*)b->d_tiles, mode, b->d_partial);
  hipLaunchKernelGGL(k_batch_reduce_final, dim3((unsigned)b->n), dim3(BT), 0, b->stream,
                     (const double*)b->d_partial, (const InstDesc*)b->d_desc,
                     (const int*)b->d_count, b->d_out);
  lbm_status s = launch_check("batch reduce launch");
  if (s) return s;
  s = hip_check(hipMemcpyAsync(h_out2, b->d_out, sizeof(double) * 2 * b->n,
                               hipMemcpyDeviceToHost, b->stream),
                "batch reduce copy");
  if (s) return s;
  return hip_check(hipStreamSynchronize(b->stream), "batch reduce sync");
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params* params) {
  Layout L;
  if (plan(n, params, &L) != LBM_OK) return 0;
  return L.bytes;
}

lbm_status lbm_batch_create(int32_t n, const lbm_params* params, void* d_ws, size_t ws_size,
                            void* hip_stream, lbm_batch** out) {
  if (!out) return fail(LBM_E_ARG, "null out");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(LBM_E_ARG, "workspace null or misaligned");
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_E_ARG, "out of host memory");
  lbm_status s = plan(n, params, &b->L);
  if (s == LBM_OK && ws_size < b->L.bytes) s = fail(LBM_E_SPACE, "workspace too small");
  if (s) {
    delete b;
    return s;
  }
  b->n = n;
  b->ws = (char*)d_ws;
  b->stream = (hipStream_t)hip_stream;
  b->pool[0] = (float*)(b->ws + b->L.off_pool[0]);
  b->pool[1] = (float*)(b->ws + b->L.off_pool[1]);
  b->d_desc = (InstDesc*)(b->ws + b->L.off_desc);
  b->d_tiles = (int*)(b->ws + b->L.off_tiles);
  b->d_count = (int*)(b->ws + b->L.off_count);
  b->d_partial = (double*)(b->ws + b->L.off_partial);
  b->d_out = (double*)(b->ws + b->L.off_out);
  b->d_waves = (int2*)(b->ws + b->L.off_waves);
  for (int i = 0; i < n; ++i)
    b->L.desc[i].V = b->L.voff[i] >= 0 ? (float*)(b->ws + b->L.off_wallv) + b->L.voff[i] : nullptr;
  b->tb_cfg = -1;
  for (int v = 0; v < kNumBatchTB; ++v) b->tb_ms[v] = -1.0;
  b->cur = 0;
  b->initialised = false;
  b->nstep = 0;
  b->wall_nsteps.assign(n, 0);
  b->any_wall = false;
  s = upload_descs(b);
  if (s == LBM_OK)
    s = hip_check(hipMemcpy(b->d_tiles, b->L.tile_inst.data(), sizeof(int) * b->L.ntiles,
                            hipMemcpyHostToDevice),
                  "tile table upload");
  if (s == LBM_OK)
    s = hip_check(hipMemcpy(b->d_count, b->L.tile_count.data(), sizeof(int) * n,
                            hipMemcpyHostToDevice),
                  "tile count upload");
  for (int v = 0; v < kNumBatchTB && s == LBM_OK && b->L.tb_ok; ++v) {
    const std::vector<int2> t = wave_table(b->L, v);
    s = hip_check(hipMemcpy(b->d_waves + b->L.tb_wave0[v], t.data(), sizeof(int2) * t.size(),
                            hipMemcpyHostToDevice),
                  "wave table upload");
  }
  if (s) {
    delete b;
    return s;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (b) {
    drop_graphs(b);
    delete b;
  }
  return LBM_OK;
}

int64_t lbm_batch_node_offset(const lbm_batch* b, int32_t i) {
  if (!b || i < 0 || i > b->n) return -1;
  return i == b->n ? b->L.total_nodes : b->L.desc[i].node0;
}

int64_t lbm_batch_step_count(const lbm_batch* b) { return b ? b->nstep : -1; }

static lbm_status batch_init_any(lbm_batch* b, const void* v0, const void* s0, int packed,
                                 bool f32) {
  const int64_t total = b->L.total_nodes;
  const unsigned grid = (unsigned)((total + BT - 1) / BT);
  if (f32)
    hipLaunchKernelGGL(k_batch_init<float>, dim3(grid), dim3(BT), 0, b->stream,
                       (const float*)v0, (const float*)s0, packed, b->pool[0],
                       (const InstDesc*)b->d_desc, b->n, total);
  else
    hipLaunchKernelGGL(k_batch_init<double>, dim3(grid), dim3(BT), 0, b->stream,
                       (const double*)v0, (const double*)s0, packed, b->pool[0],
                       (const InstDesc*)b->d_desc, b->n, total);
  lbm_status s = launch_check("batch init launch");
  if (s) return s;
  b->cur = 0;
  b->nstep = 0;
  b->initialised = true;
  return LBM_OK;
}

lbm_status lbm_batch_init(lbm_batch* b, const double* d_v0, const double* d_sigma0) {
  if (!b || !d_v0 || !d_sigma0) return fail(LBM_E_ARG, "null argument");
  return batch_init_any(b, d_v0, d_sigma0, 0, false);
}

lbm_status lbm_batch_init_fields_f32(lbm_batch* b, const float* d_fields) {
  if (!b || !d_fields) return fail(LBM_E_ARG, "null argument");
  return batch_init_any(b, nullptr, d_fields, 1, true);
}

lbm_status lbm_batch_set_wall_velocity(lbm_batch* b, int32_t i, int32_t rank, const float* d_W,
                                       const float* d_T, int64_t nsteps) {
  if (!b || i < 0 || i >= b->n) return fail(LBM_E_ARG, "bad instance");
  if (rank < 0 || rank > 4096) return fail(LBM_E_ARG, "rank out of range");
  if (rank > 0 && (!d_W || !d_T || nsteps < 0)) return fail(LBM_E_ARG, "null wall table");
  if (rank > 0 && b->L.desc[i].bc != LBM_DIRICHLET)
    return fail(LBM_E_ARG, "wall data need a Dirichlet instance");
  b->L.desc[i].W = rank ? d_W : nullptr;
  b->L.desc[i].T = rank ? d_T : nullptr;
  b->L.desc[i].rank = rank;
  b->wall_nsteps[i] = rank ? nsteps : 0;
  b->any_wall = false;
  for (int k = 0; k < b->n; ++k) b->any_wall |= b->L.desc[k].rank > 0;
  drop_graphs(b);
  hipStreamSynchronize(b->stream);  // descriptors may be in use by queued work
  return upload_descs(b);
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b) return fail(LBM_E_ARG, "null batch");
  if (!b->initialised) return fail(LBM_E_STATE, "step before init");
  if (nsteps < 0) return fail(LBM_E_ARG, "negative step count");
  if (nsteps == 0) return LBM_OK;
  for (int i = 0; i < b->n; ++i)
    if (b->L.desc[i].rank > 0 && b->nstep + nsteps > b->wall_nsteps[i])
      return fail(LBM_E_ARG, "wall table too short for the requested steps");
  lbm_status s;
  if (!b->any_wall) {
    auto key = std::make_tuple(nsteps, b->cur, b->tb_cfg);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      hipGraphExec_t exec;
      s = build_graph(b, nsteps, b->cur, 0, &exec);
      if (s) return s;
      it = b->graphs.emplace(key, exec).first;
    }
    s = hip_check(hipGraphLaunch(it->second, b->stream), "graph launch");
  } else {
    hipGraphExec_t exec;
    s = build_graph(b, nsteps, b->cur, b->nstep, &exec);
    if (s) return s;
    s = hip_check(hipGraphLaunch(exec, b->stream), "graph launch");
    hipGraphExecDestroy(exec);
  }
  if (s) return s;
  b->cur ^= (int)(launch_plan(b, nsteps).size() & 1);
  b->nstep += nsteps;
  return LBM_OK;
}

lbm_status lbm_batch_step_eager(lbm_batch* b, int64_t nsteps) {
  if (!b) return fail(LBM_E_ARG, "null batch");
  if (!b->initialised) return fail(LBM_E_STATE, "step before init");
  if (nsteps < 0) return fail(LBM_E_ARG, "negative step count");
  for (int i = 0; i < b->n; ++i)
    if (b->L.desc[i].rank > 0 && b->nstep + nsteps > b->wall_nsteps[i])
      return fail(LBM_E_ARG, "wall table too short for the requested steps");
  for (int t : launch_plan(b, nsteps)) {
    launch_direct(b, t, b->cur, b->nstep);
    b->cur ^= 1;
    b->nstep += t;
  }
  return launch_check("batch step launch");
}

int32_t lbm_batch_tblock_config_count(void) { return kNumBatchTB; }

lbm_status lbm_batch_tblock_config_info(int32_t index, int32_t* steps, int32_t* seg_rows,
                                        int32_t* nt, int32_t* pf) {
  if (index < 0 || index >= kNumBatchTB) return fail(LBM_E_ARG, "config index out of range");
  const BatchTBConfig& k = kBatchTB[index];
  if (steps) *steps = k.steps;
  if (seg_rows) *seg_rows = k.seg_rows;
  if (nt) *nt = k.nt;
  if (pf) *pf = k.pf;
  return LBM_OK;
}

lbm_status lbm_batch_get_tblock_config(const lbm_batch* b, int32_t* index) {
  if (!b || !index) return fail(LBM_E_ARG, "null argument");
  *index = b->tb_cfg;
  return LBM_OK;
}

lbm_status lbm_batch_set_tblock_config(lbm_batch* b, int32_t index) {
  if (!b) return fail(LBM_E_ARG, "null batch");
  if (index < -1 || index >= kNumBatchTB) return fail(LBM_E_ARG, "config index out of range");
  if (index == b->tb_cfg) return LBM_OK;
  if (index >= 0 && !b->L.tb_ok)
    return fail(LBM_E_ARG, "an instance is too wide for the blocked kernel");
  // every variant's wave table stays in the workspace, and cached graphs are
  // keyed by the variant: nothing to replace
  b->tb_cfg = index;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* h_index, double* h_ms) {
  if (!b) return fail(LBM_E_ARG, "null batch");
  if (!b->initialised) return fail(LBM_E_STATE, "autotune needs an initialised batch");
  if (reps < 1) return fail(LBM_E_ARG, "reps must be >= 1");
  hipEvent_t e0, e1;
  lbm_status s = hip_check(hipEventCreate(&e0), "event");
  if (s) return s;
  s = hip_check(hipEventCreate(&e1), "event");
  if (s) {
    hipEventDestroy(e0);
    return s;
  }
  int64_t wall_left = INT64_MAX;  // steps of wall data left for timed launches
  for (int i = 0; i < b->n; ++i)
    if (b->L.desc[i].rank > 0 && b->wall_nsteps[i] - b->nstep < wall_left)
      wall_left = b->wall_nsteps[i] - b->nstep;
  int best = -1;
  double best_ms = 1e300;
  // timed launches read the current pool and write the spare one: the state
  // is not changed
  for (int v = -1; v < kNumBatchTB && s == LBM_OK; ++v) {
    if (v >= 0 && !b->L.tb_ok) continue;
    if (wall_left < (v >= 0 ? kBatchTB[v].steps : 1)) continue;
    s = lbm_batch_set_tblock_config(b, v);
    if (s) break;
    const int t = v >= 0 ? kBatchTB[v].steps : 1;
    for (int r = 0; r < reps + 2; ++r) {
      if (r == 2) hipEventRecord(e0, b->stream);
      launch_direct(b, t, b->cur, b->nstep);
    }
    hipEventRecord(e1, b->stream);
    s = hip_check(hipEventSynchronize(e1), "autotune sync");
    float ms = 0.f;
    if (s == LBM_OK) s = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing");
    const double per = (double)ms / reps / t;
    if (s == LBM_OK && v >= 0) b->tb_ms[v] = (double)ms / reps;
    if (s == LBM_OK && per < best_ms) {
      best_ms = per;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s) return s;
  // the launch times decide the launches for the last steps of a run: rebuild
  // cached graphs
  s = hip_check(hipStreamSynchronize(b->stream), "batch sync");
  if (s) return s;
  drop_graphs(b);
  s = lbm_batch_set_tblock_config(b, best);
  if (s) return s;
  if (h_index) *h_index = best;
  if (h_ms) *h_ms = best_ms;
  return LBM_OK;
}

static lbm_status batch_moments(lbm_batch* b, float* out, int mode) {
  if (!b || !out) return fail(LBM_E_ARG, "null argument");
  if (!b->initialised) return fail(LBM_E_STATE, "not initialised");
  const int64_t total = b->L.total_nodes;
  hipLaunchKernelGGL(k_batch_moments, dim3((unsigned)((total + BT - 1) / BT)), dim3(BT), 0,
                     b->stream, (const float*)b->pool[b->cur], out, (const InstDesc*)b->d_desc,
                     b->n, total, mode);
  return launch_check("batch moments launch");
}

lbm_status lbm_batch_moments(lbm_batch* b, float* d_out) { return batch_moments(b, d_out, 0); }
lbm_status lbm_batch_moments_U(lbm_batch* b, float* d_U) { return batch_moments(b, d_U, 1); }

lbm_status lbm_batch_energy(lbm_batch* b, double* h_out) {
  if (!b || !h_out) return fail(LBM_E_ARG, "null argument");
  if (!b->initialised) return fail(LBM_E_STATE, "not initialised");
  std::vector<double> r(2 * b->n);
  lbm_status s = batch_reduce(b, 0, nullptr, r.data());
  if (s) return s;
  for (int i = 0; i < b->n; ++i) h_out[i] = r[2 * i];
  return LBM_OK;
}

lbm_status lbm_batch_rel_l2_fields(lbm_batch* b, const float* d_fields, double* h_out) {
  if (!b || !d_fields || !h_out) return fail(LBM_E_ARG, "null argument");
  if (!b->initialised) return fail(LBM_E_STATE, "not initialised");
  std::vector<double> r(2 * b->n);
  lbm_status s = batch_reduce(b, 1, d_fields, r.data());
  if (s) return s;
  for (int i = 0; i < b->n; ++i) h_out[i] = r[2 * i + 1] > 0 ? sqrt(r[2 * i] / r[2 * i + 1]) : 0.0;
  return LBM_OK;
}

lbm_status lbm_batch_rel_l2_pair(lbm_batch* b, const float* d_a, const float* d_b,
                                 double* h_out) {
  if (!b || !d_a || !d_b || !h_out) return fail(LBM_E_ARG, "null argument");
  std::vector<double> r(2 * b->n);
  lbm_status s = batch_reduce(b, 2, d_a, r.data(), d_b);
  if (s) return s;
  for (int i = 0; i < b->n; ++i) h_out[i] = r[2 * i + 1] > 0 ? sqrt(r[2 * i] / r[2 * i + 1]) : 0.0;
  return LBM_OK;
}

}  // extern "C"

// ---- the no-allocation variant of lbm_batch_rel_l2_pair --------------------
// Instance descriptors, tile table and partial sums live in a fixed array of
// device memory inside the library instead of a batch workspace.  Each GPU
// holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (kept per device below), never
// through the array's name.
namespace {

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)4 << 20;
constexpr int STATIC_MAX_INST = 256;
constexpr int STATIC_MAX_TILES = 131072;

static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;  // device -> its copy of scratch

// Address of the current device's scratch, looked up once per device (with
// that device current).
lbm_status scratch_on_current_device(unsigned char** out) {
  int dev = -1;
  lbm_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (s) return s;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    s = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (s) return s;
    it = g_scratch_addr.emplace(dev, (unsigned char*)p).first;
  }
  *out = it->second;
  return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_rel_l2_pair_static(int32_t n, const lbm_params* h_params,
                                             const float* d_a, const float* d_b, double* h_out,
                                             void* hip_stream) {
  if (!h_params || !d_a || !d_b || !h_out) return fail(LBM_E_ARG, "null argument");
  if (n < 1 || n > STATIC_MAX_INST)
    return fail(LBM_E_ARG, "lbm_rel_l2_pair_static takes 1 .. " +
                               std::to_string(STATIC_MAX_INST) + " instances");
  Layout L;
  lbm_status s = plan(n, h_params, &L);
  if (s) return s;
  if (L.ntiles > STATIC_MAX_TILES)
    return fail(LBM_E_SPACE, "lbm_rel_l2_pair_static: " + std::to_string(L.ntiles) +
                                 " row tiles exceed the fixed scratch's " +
                                 std::to_string(STATIC_MAX_TILES));
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += (size_t)round_up((int64_t)b, 256);
    return at;
  };
  const size_t off_desc = take(sizeof(InstDesc) * n);
  const size_t off_tiles = take(sizeof(int) * (size_t)L.ntiles);
  const size_t off_count = take(sizeof(int) * n);
  const size_t off_partial = take(sizeof(double) * 2 * (size_t)L.ntiles);
  const size_t off_out = take(sizeof(double) * 2 * n);
  if (o > STATIC_SCRATCH_BYTES) return fail(LBM_E_SPACE, "lbm_rel_l2_pair_static: scratch too small");
  unsigned char* base = nullptr;
  s = scratch_on_current_device(&base);
  if (s) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  // every partial and result slot is written before it is read: nothing to clear
  s = hip_check(hipMemcpyAsync(base + off_desc, L.desc.data(), sizeof(InstDesc) * n,
                               hipMemcpyHostToDevice, st),
                "static scratch upload");
  if (!s)
    s = hip_check(hipMemcpyAsync(base + off_tiles, L.tile_inst.data(),
                                 sizeof(int) * (size_t)L.ntiles, hipMemcpyHostToDevice, st),
                  "static scratch upload");
  if (!s)
    s = hip_check(hipMemcpyAsync(base + off_count, L.tile_count.data(), sizeof(int) * n,
                                 hipMemcpyHostToDevice, st),
                  "static scratch upload");
  if (s) return s;
  const InstDesc* descs = (const InstDesc*)(base + off_desc);
  double* partial = (double*)(base + off_partial);
  double* out = (double*)(base + off_out);
  hipLaunchKernelGGL(k_batch_reduce, dim3((unsigned)L.ntiles), dim3(BT), 0, st, nullptr, d_a,
                     d_b, descs, (const int*)(base + off_tiles), 2, partial);
  hipLaunchKernelGGL(k_batch_reduce_final, dim3((unsigned)n), dim3(BT), 0, st,
                     (const double*)partial, descs, (const int*)(base + off_count), out);
  s = launch_check("static pair reduce launch");
  if (s) return s;
  std::vector<double> r(2 * (size_t)n);
  s = hip_check(hipMemcpyAsync(r.data(), out, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st),
                "static pair reduce copy");
  if (s) return s;
  // the host copies above read L's vectors; they stay alive until here
  s = hip_check(hipStreamSynchronize(st), "static pair reduce sync");
  if (s) return s;
  for (int i = 0; i < n; ++i) h_out[i] = r[2 * i + 1] > 0 ? sqrt(r[2 * i] / r[2 * i + 1]) : 0.0;
  return LBM_OK;
}
