// Batched lattices: many independent instances (uneven sizes, periodic or
// Dirichlet, their own material and time step) advanced together.
//
// Every instance keeps the single-lattice state layout (row-major, post-
// collision FP32 populations) inside two shared pools.  The unit of work is a
// row segment of one instance; a tile table maps the flattened workgroup
// index to (instance, row, segment), so one launch advances every instance by
// one step with the same per-node arithmetic as the single-lattice kernel
// (bitwise-identical results).  lbm_batch_step(n) runs n such launches as one
// hipGraph built node by node (no stream capture, no memset nodes).
//
// Packed field arrays (inputs and outputs of the batch) store instance i's
// fields contiguously, [component][ny_i][nx_i], starting at component count
// times the instance's first node (lbm_batch_node_offset).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <new>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_init.hpp"
#include "lbm_kernels.hpp"
#include "lbm_step.hpp"

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
  float U[NC];
  for (int c = 0; c < NC; ++c)
    U[c] = (src[pidx(d.g, 0 * NC + c, y, x)] + src[pidx(d.g, 1 * NC + c, y, x)]) +
           (src[pidx(d.g, 2 * NC + c, y, x)] + src[pidx(d.g, 3 * NC + c, y, x)]);
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
// a = sum |U - U(ref)|^2, b = sum |U|^2 over the U variables.
__global__ __launch_bounds__(BT) void k_batch_reduce(const float* __restrict__ pool,
                                                     const float* __restrict__ ref,
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
  if (x < d.g.nx) {
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
        const float u32 = ((float)f[0][c] + (float)f[1][c]) + ((float)f[2][c] + (float)f[3][c]);
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
  size_t off_pool[2], off_desc, off_tiles, off_count, off_partial, off_out, bytes;
};

lbm_status plan(int32_t n, const lbm_params* params, Layout* L) {
  if (n < 1 || !params) return fail(LBM_E_ARG, "batch needs n >= 1 and parameters");
  L->desc.resize(n);
  L->tile_count.resize(n);
  for (int i = 0; i < n; ++i) {
    Derived dv;
    lbm_status s = derive(&params[i], &dv);
    if (s) return fail(s, "instance " + std::to_string(i) + ": " + g_err);
    if (params[i].flags != 0) return fail(LBM_E_ARG, "batched instances use the row layout");
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
  }
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
  int cur;
  bool initialised;
  int64_t nstep;
  std::vector<int64_t> wall_nsteps;
  bool any_wall;
  std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;  // (steps, parity), wall-free
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

// Build a graph of `steps` step launches starting from buffer `cur` at step
// index `step0` (the step index matters only for wall tables).
lbm_status build_graph(lbm_batch* b, int64_t steps, int cur, int64_t step0,
                       hipGraphExec_t* exec) {
  hipGraph_t graph;
  lbm_status s = hip_check(hipGraphCreate(&graph, 0), "graph create");
  if (s) return s;
  hipGraphNode_t prev = nullptr;
  for (int64_t k = 0; k < steps && s == LBM_OK; ++k) {
    const float* src = b->pool[(cur + k) & 1];
    float* dst = b->pool[(cur + k + 1) & 1];
    const InstDesc* descs = b->d_desc;
    const int* tiles = b->d_tiles;
    int ntiles = b->L.ntiles;
    int64_t step = step0 + k;
    void* args[] = {(void*)&src, (void*)&dst, (void*)&descs, (void*)&tiles, (void*)&ntiles,
                    (void*)&step};
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    kp.func = reinterpret_cast<void*>(&k_batch_step<BT>);
    kp.gridDim = dim3((unsigned)ntiles);
    kp.blockDim = dim3(BT);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    s = hip_check(hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                  "graph add kernel node");
    prev = node;
  }
  if (s == LBM_OK) s = hip_check(hipGraphInstantiate(exec, graph, nullptr, nullptr, 0),
                                 "graph instantiate");
  hipGraphDestroy(graph);
  return s;
}

lbm_status batch_reduce(lbm_batch* b, int mode, const float* ref, double* h_out2) {
  hipLaunchKernelGGL(k_batch_reduce, dim3((unsigned)b->L.ntiles), dim3(BT), 0, b->stream,
                     (const float*)b->pool[b->cur], ref, (const InstDesc*)b->d_desc,
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
    auto key = std::make_pair(nsteps, b->cur);
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
  b->cur = (int)((b->cur + nsteps) & 1);
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
  for (int64_t k = 0; k < nsteps; ++k) {
    hipLaunchKernelGGL(k_batch_step<BT>, dim3((unsigned)b->L.ntiles), dim3(BT), 0, b->stream,
                       (const float*)b->pool[b->cur], b->pool[b->cur ^ 1],
                       (const InstDesc*)b->d_desc, (const int*)b->d_tiles, b->L.ntiles,
                       b->nstep + k);
    b->cur ^= 1;
  }
  b->nstep += nsteps;
  return launch_check("batch step launch");
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

}  // extern "C"
