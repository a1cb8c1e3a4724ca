// The exact linear window operator of a periodic lattice (C ABI in
// include/lbm.h, lbm_wop_*).
//
// On a periodic lattice with a fixed material the window map
//   U -> moments(16 steps from the second-order initialisation of U)
// (Eq. ic_second with central-difference gradients, then Section 3.6's
// collision and streaming, then the zeroth moment) is linear and commutes
// with lattice shifts: it is a convolution whose taps G[d] (5 x 5 matrices,
// d = output - input offset) are the responses to unit deltas.  Information
// moves one node per step along an axis and the central differences reach
// one node, so G vanishes outside the diamond |dx| + |dy| <= 17.
//
//   lbm_wop_build   runs the library's own initialisation and 16 FP32 steps on
//                   a unit delta in each component (a 40 x 40 periodic lattice
//                   on the caller's scratch), gathers the taps and folds the
//                   field conversions (fields -> U on input, U -> fields on
//                   output) into them, packed as the matrix-core operand;
//   k_wop_apply     the convolution as FP32 matrix-core products
//                   (v_mfma_f32_16x16x4_f32): per wave a tile of 16 output
//                   columns x 3 output rows, M = 16 pixels, N = 3 rows x 5
//                   output fields (15 of 16), K = (input field, input row,
//                   input column) over the union of the three rows' diamonds,
//                   4 columns per product; the input tile of a workgroup
//                   (4 waves side by side, periodic wrap) is staged in LDS.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_host.hpp"
#include "lbm_kernels.hpp"

using namespace lbmk;
using namespace lbmh;

namespace {

constexpr int WOP_R = LBM_WOP_STEPS + 1;            // support radius
constexpr int WOP_SIDE = 2 * WOP_R + 1;             // taps per side
constexpr int WOP_GEN = 2 * WOP_R + 6;              // side of the generating lattice
constexpr int WOP_TR = 3;                           // output rows per wave tile
constexpr int WOP_RY = WOP_TR + 2 * WOP_R;          // input rows of a tile
constexpr int WOP_WAVES = 4;
constexpr int WOP_COLS = 16 * WOP_WAVES;            // output columns per workgroup
constexpr int WOP_PITCH = WOP_COLS + 2 * WOP_R + 3; // input columns X0 - R .. X0 + 63 + R + 3
constexpr int WOP_PLANE = WOP_RY * WOP_PITCH;

// input row ri of a tile (row Y0 - R + ri): half-width of the columns any of
// the tile's output rows Y0 .. Y0 + 2 reaches there, and the 4-column
// products covering them
__host__ __device__ constexpr int wop_half(int ri) {
  return WOP_R - (ri < WOP_R ? WOP_R - ri : (ri > WOP_R + WOP_TR - 1 ? ri - (WOP_R + WOP_TR - 1) : 0));
}
__host__ __device__ constexpr int wop_chunks(int ri) { return (2 * wop_half(ri) + 1 + 3) / 4; }
__host__ __device__ constexpr int wop_steps_per_field() {
  int s = 0;
  for (int ri = 0; ri < WOP_RY; ++ri) s += wop_chunks(ri);
  return s;
}
constexpr int WOP_STEPS_F = wop_steps_per_field();     // products per input field
constexpr int WOP_STEPS = NC * WOP_STEPS_F;            // products per tile
constexpr int WOP_GROUPS = (WOP_STEPS + 3) / 4;        // groups of 4 products
static_assert(WOP_GROUPS * 4 * (64 * 4 + 4) <= LBM_WOP_OPERAND_BYTES, "operand size");

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The packed operator: for product s (k = 4 input columns of one input row
// and field), lane l holds B[k = 4 s + l / 16][n = l % 16] in group s / 4,
// slot s % 4; then the wave-uniform LDS offset of each product's A operand.
struct WopOperand {
  float4 b[WOP_GROUPS][64];
  int4 aoff[WOP_GROUPS];
};
static_assert(sizeof(WopOperand) <= LBM_WOP_OPERAND_BYTES, "operand size");

// unit delta in component ci of U at the centre of the generating lattice,
// as physical fields (v, sigma_bar) through Eq. sigma_num
__global__ void k_wop_delta(double* __restrict__ v0, double* __restrict__ s0, int ci, double cK,
                            double cmu, double rho) {
  const int n = WOP_GEN * WOP_GEN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = WOP_GEN / 2;
  double U[NC] = {0, 0, 0, 0, 0};
  if (i == c0 * WOP_GEN + c0) U[ci] = 1.0;
  v0[i] = U[0];
  v0[n + i] = U[1];
  s0[i] = -rho * (cK * U[2] + cmu * U[3]);
  s0[n + i] = -rho * (cK * U[2] - cmu * U[3]);
  s0[2 * n + i] = -rho * (cmu * U[4]);
}

// G[dy + R][dx + R][co][ci] from the response U [5][GEN][GEN] to component ci
__global__ void k_wop_gather(const float* __restrict__ resp, float* __restrict__ G, int ci) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= WOP_SIDE * WOP_SIDE * NC) return;
  const int co = i % NC;
  const int d = i / NC;
  const int iy = d / WOP_SIDE, ix = d % WOP_SIDE;
  const int c0 = WOP_GEN / 2;
  const int n = WOP_GEN * WOP_GEN;
  G[(d * NC + co) * NC + ci] =
      resp[co * n + (c0 + iy - WOP_R) * WOP_GEN + (c0 + ix - WOP_R)];
}

// the packed operand in the physical fields: taps Tout G[d] Tin (FP64), with
// Tin: fields -> U (inverse of Eq. sigma_num), Tout: U -> fields
// (Eq. sigma_num times rho)
__global__ void k_wop_pack(const float* __restrict__ G, WopOperand* __restrict__ op, double cK,
                           double cmu, double rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= WOP_GROUPS * 4 * 64) return;
  const int lane = i & 63;
  const int s = i >> 6;  // product
  const int g = lane >> 4, nn = lane & 15;
  float val = 0.f;
  int aoff = 0;
  if (s < WOP_STEPS) {
    const int ci = s / WOP_STEPS_F;
    int rem = s - ci * WOP_STEPS_F, ri = 0;
    while (rem >= wop_chunks(ri)) rem -= wop_chunks(ri++);
    const int j = rem, a = wop_half(ri);
    aoff = ci * WOP_PLANE + ri * WOP_PITCH + (WOP_R - a + 4 * j);
    const int dx = -a + 4 * j + g;       // input column offset
    const int ry = ri - WOP_R;            // input row offset from the tile's first output row
    if (nn < NC * WOP_TR && dx <= a) {
      const int t = nn / NC, co = nn % NC;
      const int dyo = t - ry, dxo = -dx;  // output - input
      if (abs(dxo) + abs(dyo) <= WOP_R) {
        const float* Gd = G + ((dyo + WOP_R) * WOP_SIDE + (dxo + WOP_R)) * NC * NC;
        double Tin[NC][NC] = {};
        Tin[0][0] = 1.0;
        Tin[1][1] = 1.0;
        Tin[2][2] = Tin[2][3] = -1.0 / (2.0 * rho * cK);
        Tin[3][2] = -1.0 / (2.0 * rho * cmu);
        Tin[3][3] = 1.0 / (2.0 * rho * cmu);
        Tin[4][4] = -1.0 / (rho * cmu);
        double Tout[NC][NC] = {};
        Tout[0][0] = 1.0;
        Tout[1][1] = 1.0;
        Tout[2][2] = -rho * cK;
        Tout[2][3] = -rho * cmu;
        Tout[3][2] = -rho * cK;
        Tout[3][3] = rho * cmu;
        Tout[4][4] = -rho * cmu;
        double acc = 0.0;
        for (int p = 0; p < NC; ++p)
          for (int q = 0; q < NC; ++q)
            acc += Tout[co][p] * (double)Gd[p * NC + q] * Tin[q][ci];
        val = (float)acc;
      }
    }
  }
  reinterpret_cast<float*>(&op->b[s >> 2][lane])[s & 3] = val;
  if (lane == 0) reinterpret_cast<int*>(&op->aoff[s >> 2])[s & 3] = aoff;
}

__device__ inline int wrap_index(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// One workgroup: output columns X0 .. X0 + 63 of rows Y0 .. Y0 + 2 of window b.
__global__ __launch_bounds__(256) void k_wop_apply(const float* __restrict__ in,
                                                   float* __restrict__ out,
                                                   const WopOperand* __restrict__ op, int nx,
                                                   int ny, int tiles_x) {
  __shared__ float tile[NC * WOP_PLANE];
  __shared__ int rowy[WOP_RY];
  const int tid = threadIdx.x;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int X0 = tx * WOP_COLS, Y0 = ty * WOP_TR;
  const int64_t nn = (int64_t)nx * ny;
  const float* src = in + (int64_t)blockIdx.y * NC * nn;
  float* dst = out + (int64_t)blockIdx.y * NC * nn;
  // periodic wrap of the tile's rows (any lattice size)
  for (int i = tid; i < WOP_RY; i += 256) rowy[i] = wrap_index(Y0 - WOP_R + i, ny);
  const int w = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  // the two columns of the tile this lane fills (the second for lanes < 37)
  constexpr int C2 = WOP_PITCH - 64;
  const int cx0 = wrap_index(X0 - WOP_R + lane, nx);
  const int cx1 = lane < C2 ? wrap_index(X0 - WOP_R + 64 + lane, nx) : cx0;
  __syncthreads();
  // fill: wave w takes the (field, row) lines w, w + 4, w + 8, ..., four
  // lines per round so that eight loads per lane are in flight
  constexpr int LINES = NC * WOP_RY;
  for (int l0 = w; l0 < LINES; l0 += 16) {  // lines l0, l0 + 4, l0 + 8, l0 + 12
    float v0[4], v1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ln = l0 + 4 * k;
      if (ln < LINES) {
        const int c = ln / WOP_RY, r = ln - c * WOP_RY;
        const float* rp = src + c * nn + (int64_t)rowy[r] * nx;
        v0[k] = rp[cx0];
        v1[k] = rp[cx1];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ln = l0 + 4 * k;
      if (ln < LINES) {
        tile[ln * WOP_PITCH + lane] = v0[k];
        if (lane < C2) tile[ln * WOP_PITCH + 64 + lane] = v1[k];
      }
    }
  }
  __syncthreads();
  // this lane's A element of product s: tile[abase + aoff(s)]; the next
  // group's A and B are read while the current group's products run
  const float* abase = tile + 16 * w + m + g;
  const float4* bq = &op->b[0][lane];
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float4 b = bq[0];
  int4 ao = op->aoff[0];  // wave-uniform
  float a0 = abase[ao.x], a1 = abase[ao.y], a2 = abase[ao.z], a3 = abase[ao.w];
  for (int q = 0; q < WOP_GROUPS; ++q) {
    const int qn = q + 1 < WOP_GROUPS ? q + 1 : q;
    const float4 bn = bq[qn * 64];
    const int4 an = op->aoff[qn];
    const float n0 = abase[an.x], n1 = abase[an.y], n2 = abase[an.z], n3 = abase[an.w];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b.w, acc, 0, 0, 0);
    b = bn;
    a0 = n0;
    a1 = n1;
    a2 = n2;
    a3 = n3;
  }
  // D[i][n]: lane holds n = lane % 16 = 5 t + co for pixels i = 4 g + v
  const int n = lane & 15;
  if (n >= NC * WOP_TR) return;
  const int t = n / NC, co = n % NC;
  const int y = Y0 + t;
  if (y >= ny) return;
  float* row = dst + co * nn + (int64_t)y * nx;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = X0 + 16 * w + 4 * g + v;
    if (x < nx) row[x] = acc[v];
  }
}

// scratch of lbm_wop_build: the generating lattice's workspace, its initial
// fields and one response
size_t gen_ws_bytes(const lbm_params* p) {
  lbm_params q = *p;
  q.nx = q.ny = WOP_GEN;
  q.bc = LBM_PERIODIC;
  q.flags = 0;
  return lbm_workspace_bytes(&q);
}
constexpr size_t WOP_FIELDS_BYTES = (size_t)(2 + 3) * WOP_GEN * WOP_GEN * 8;
constexpr size_t WOP_RESP_BYTES = (size_t)NC * WOP_GEN * WOP_GEN * 4;
constexpr size_t WOP_G_BYTES = (size_t)WOP_SIDE * WOP_SIDE * NC * NC * 4;

lbm_status check_window_params(const lbm_params* p) {
  if (!p) return fail(LBM_E_ARG, "null params");
  if (p->bc != LBM_PERIODIC)
    return fail(LBM_E_ARG, "the window operator is that of a periodic lattice");
  Derived d;
  lbm_status s = derive(p, &d);
  if (s) return s;
  if (!(d.cmu > 0)) return fail(LBM_E_ARG, "the window operator needs mu > 0");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_wop_scratch_bytes(const lbm_params* p) {
  if (check_window_params(p) != LBM_OK) return 0;
  const size_t ws = gen_ws_bytes(p);
  if (ws == 0) return 0;
  return (size_t)round_up((int64_t)ws, 256) + (size_t)round_up(WOP_FIELDS_BYTES, 256) +
         (size_t)round_up(WOP_RESP_BYTES, 256) + (size_t)round_up(WOP_G_BYTES, 256);
}

size_t lbm_wop_operand_bytes(void) { return LBM_WOP_OPERAND_BYTES; }

lbm_status lbm_wop_build(const lbm_params* p, float* d_G, void* d_op, void* d_scratch,
                         size_t scratch_bytes, void* hip_stream) {
  lbm_status s = check_window_params(p);
  if (s) return s;
  if (!d_op || !d_scratch) return fail(LBM_E_ARG, "null argument");
  if (((uintptr_t)d_scratch & 255) || ((uintptr_t)d_op & 15))
    return fail(LBM_E_ARG, "scratch must be 256-byte and the operand 16-byte aligned");
  if (scratch_bytes < lbm_wop_scratch_bytes(p)) return fail(LBM_E_SPACE, "scratch too small");
  hipStream_t st = (hipStream_t)hip_stream;
  lbm_params q = *p;
  q.nx = q.ny = WOP_GEN;
  q.flags = 0;
  const size_t ws = (size_t)round_up((int64_t)gen_ws_bytes(p), 256);
  char* base = (char*)d_scratch;
  double* v0 = (double*)(base + ws);
  double* s0 = v0 + 2 * WOP_GEN * WOP_GEN;
  float* resp = (float*)(base + ws + round_up(WOP_FIELDS_BYTES, 256));
  float* G = d_G ? d_G
                 : (float*)(base + ws + round_up(WOP_FIELDS_BYTES, 256) +
                            round_up(WOP_RESP_BYTES, 256));
  lbm_ctx* ctx = nullptr;
  s = lbm_create(&q, d_scratch, ws, hip_stream, &ctx);
  if (s) return s;
  double kK, km, c;
  lbm_lattice_constants(ctx, &kK, &km, &c);
  const double cK = kK * c, cmu = km * c;
  const int n = WOP_GEN * WOP_GEN;
  for (int ci = 0; ci < NC && s == LBM_OK; ++ci) {
    hipLaunchKernelGGL(k_wop_delta, dim3((n + 255) / 256), dim3(256), 0, st, v0, s0, ci, cK, cmu,
                       p->rho);
    s = launch_check("k_wop_delta launch");
    if (!s) s = lbm_init(ctx, v0, s0, nullptr);
    if (!s) s = lbm_step(ctx, LBM_WOP_STEPS);
    if (!s) s = lbm_moments_U(ctx, resp);
    if (!s) {
      const int m = WOP_SIDE * WOP_SIDE * NC;
      hipLaunchKernelGGL(k_wop_gather, dim3((m + 255) / 256), dim3(256), 0, st, resp, G, ci);
      s = launch_check("k_wop_gather launch");
    }
  }
  lbm_destroy(ctx);
  if (s) return s;
  const int m = WOP_GROUPS * 4 * 64;
  hipLaunchKernelGGL(k_wop_pack, dim3((m + 255) / 256), dim3(256), 0, st, (const float*)G,
                     (WopOperand*)d_op, cK, cmu, p->rho);
  return launch_check("k_wop_pack launch");
}

lbm_status lbm_wop_apply(const lbm_params* p, const void* d_op, const float* d_in, float* d_out,
                         int32_t batch, void* hip_stream) {
  if (!p || !d_op || !d_in || !d_out) return fail(LBM_E_ARG, "null argument");
  if (p->bc != LBM_PERIODIC)
    return fail(LBM_E_ARG, "the window operator is that of a periodic lattice");
  if (p->nx < 1 || p->ny < 1 || batch < 1 || batch > 65535)
    return fail(LBM_E_ARG, "bad window size or batch");
  if ((uintptr_t)d_op & 15) return fail(LBM_E_ARG, "operand must be 16-byte aligned");
  const int64_t nb = (int64_t)NC * p->nx * p->ny * 4 * batch;
  const char *a = (const char*)d_in, *b = (const char*)d_out;
  if (a < b + nb && b < a + nb) return fail(LBM_E_ARG, "input and output overlap");
  const int tiles_x = (p->nx + WOP_COLS - 1) / WOP_COLS;
  const int tiles_y = (p->ny + WOP_TR - 1) / WOP_TR;
  if ((int64_t)tiles_x * tiles_y > 0x7fffffff) return fail(LBM_E_ARG, "window too large");
  hipLaunchKernelGGL(k_wop_apply, dim3((unsigned)(tiles_x * tiles_y), (unsigned)batch), dim3(256),
                     0, (hipStream_t)hip_stream, d_in, d_out, (const WopOperand*)d_op, p->nx,
                     p->ny, tiles_x);
  return launch_check("k_wop_apply launch");
}

}  // extern "C"
