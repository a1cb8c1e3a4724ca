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
//                   (v_mfma_f32_16x16x4_f32): per wave MT tiles of 16 output
//                   columns x 3 output rows, each M = 16 pixels, N = 3 rows x
//                   5 output fields (15 of 16), K = (input field, input row,
//                   input column) over the union of the three rows' diamonds,
//                   4 columns per product, every B operand shared by the MT
//                   tiles; the input tile of a workgroup (NCT column tiles
//                   side by side, periodic wrap) is staged in LDS, and 4
//                   waves per column tile take a quarter of the K range each
//                   (more waves per SIMD to cover the operand's L2 latency).
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
constexpr int WOP_GF = (WOP_STEPS_F + 3) / 4;          // groups of 4 products per field
constexpr int WOP_GROUPS = NC * WOP_GF;
constexpr int WOP_BPF = 2;                             // B groups read ahead
constexpr int WOP_KS = 4;                              // parts of the K range, one wave each

// Offset of product sl of a field (sl < 4 WOP_GF) in a tile row of pitch P
// relative to the field's plane: input row ri, first column R - half + 4 j
// of the 4 the product covers (past the field's products: 0, with zero taps)
template <int P>
struct WopOffsets {
  int o[4 * WOP_GF];
  constexpr WopOffsets() : o() {
    int sl = 0;
    for (int ri = 0; ri < WOP_RY; ++ri)
      for (int j = 0; j < wop_chunks(ri); ++j) o[sl++] = ri * P + (WOP_R - wop_half(ri) + 4 * j);
  }
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The packed operator: for product s = 4 WOP_GF ci + sl (input field ci, sl
// as above; k = 4 input columns of one input row), lane l holds
// B[k = l / 16][n = l % 16] in group s / 4, slot s % 4.
struct WopOperand {
  float4 b[WOP_GROUPS][64];
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
  const int ci = s / (4 * WOP_GF), sl = s - ci * 4 * WOP_GF;
  float val = 0.f;
  if (ci < NC && sl < WOP_STEPS_F) {
    int rem = sl, ri = 0;
    while (rem >= wop_chunks(ri)) rem -= wop_chunks(ri++);
    const int j = rem, a = wop_half(ri);
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
}

__device__ inline int wrap_index(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Tile geometry of k_wop_apply with MT 16-column matrix tiles per wave and
// NCT column tiles (of 16 MT columns) per workgroup: a workgroup covers COLS
// output columns of three rows, and stages input columns X0 - R .. X0 + COLS
// + R + 2 of every input row and field in LDS; WOP_KS waves per column tile.
__host__ __device__ constexpr int wop_threads(int nct) { return 64 * nct * WOP_KS; }
template <int MT, int NCT>
struct WopTile {
  static constexpr int COLS = 16 * MT * NCT;
  static constexpr int PITCH = COLS + 2 * WOP_R + 3;
  static constexpr int PLANE = WOP_RY * PITCH;
  static constexpr int THREADS = wop_threads(NCT);
};

// The products of groups Q0 .. Q0 + NQ - 1 of every input field into acc:
// this lane's A element of product sl of field ci for tile t is
// abase[ci PLANE + kOff.o[sl] + 16 t] (compile-time offsets once the group
// loop is unrolled); A is read one group ahead and B WOP_BPF groups ahead
// (in this wave's order: fields in turn, groups Q0 .. Q0 + NQ - 1 of each)
// while the current group's products run.
template <int MT, int PITCH, int PLANE, int Q0, int NQ>
__device__ __forceinline__ void wop_products(const float* abase, const f32x4* bq,
                                             f32x4 (&acc)[MT]) {
  static_assert(WOP_BPF <= NQ, "read-ahead within one field's part");
  constexpr WopOffsets<PITCH> kOff{};
  float a[MT][4];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) a[t][k] = abase[kOff.o[4 * Q0 + k] + 16 * t];
  f32x4 b[WOP_BPF];
#pragma unroll
  for (int d = 0; d < WOP_BPF; ++d) b[d] = bq[64 * (Q0 + d)];
  for (int ci = 0; ci < NC; ++ci) {
    const float* af = abase + ci * PLANE;
    const float* an = ci + 1 < NC ? af + PLANE : af;
    // the read-ahead past the last field re-reads a group of it
    const int gcur = ci * WOP_GF, gnext = (ci + 1 < NC ? ci + 1 : ci) * WOP_GF;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int jt = j + WOP_BPF;
      const f32x4 bnew = jt < NQ ? bq[64 * (gcur + Q0 + jt)] : bq[64 * (gnext + Q0 + jt - NQ)];
      const float* ap = j + 1 < NQ ? af : an;
      const int qn = j + 1 < NQ ? Q0 + j + 1 : Q0;
      float na[MT][4];
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) na[t][k] = ap[kOff.o[4 * qn + k] + 16 * t];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int t = 0; t < MT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][k], b[0][k], acc[t], 0, 0, 0);
#pragma unroll
      for (int d = 0; d + 1 < WOP_BPF; ++d) b[d] = b[d + 1];
      b[WOP_BPF - 1] = bnew;
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) a[t][k] = na[t][k];
    }
  }
}

// part kh of the K range: groups kh NQ .. (kh + 1) NQ - 1 of every field
template <int MT, int PITCH, int PLANE, int K>
__device__ __forceinline__ void wop_part(int kh, const float* abase, const f32x4* bq,
                                         f32x4 (&acc)[MT]) {
  constexpr int NQ = WOP_GF / WOP_KS;
  if (kh == K)
    wop_products<MT, PITCH, PLANE, K * NQ, NQ>(abase, bq, acc);
  else if constexpr (K + 1 < WOP_KS)
    wop_part<MT, PITCH, PLANE, K + 1>(kh, abase, bq, acc);
}

// One workgroup: output columns X0 .. X0 + COLS - 1 of rows Y0 .. Y0 + 2 of
// window blockIdx.y.  Wave w computes columns X0 + 16 MT (w % NCT) .. + 16 MT
// - 1 as MT matrix tiles that share every B operand, over part w / NCT of
// the K range; the parts' sums are added in order at the end.
template <int MT, int NCT>
__global__ __launch_bounds__(wop_threads(NCT)) void k_wop_apply(
    const float* __restrict__ in, float* __restrict__ out, const WopOperand* __restrict__ op,
    int nx, int ny, int tiles_x) {
  using TL = WopTile<MT, NCT>;
  constexpr int PITCH = TL::PITCH, PLANE = TL::PLANE, NT = TL::THREADS;
  constexpr int NW = NT / 64;
  static_assert(WOP_KS * NCT * MT * 64 * 16 <= NC * PLANE * 4, "partial sums fit the tile");
  __shared__ float tile[NC * PLANE];
  __shared__ int rowy[WOP_RY];
  const int tid = threadIdx.x;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int X0 = tx * TL::COLS, Y0 = ty * WOP_TR;
  const int64_t nn = (int64_t)nx * ny;
  const float* src = in + (int64_t)blockIdx.y * NC * nn;
  float* dst = out + (int64_t)blockIdx.y * NC * nn;
  // periodic wrap of the tile's rows and of this lane's columns (any
  // lattice size): lane fills tile columns lane + 64 c, c < CPL, the last
  // one for lanes < CLAST only
  for (int i = tid; i < WOP_RY; i += NT) rowy[i] = wrap_index(Y0 - WOP_R + i, ny);
  const int w = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  const int wc = w % NCT, kh = w / NCT;
  constexpr int CPL = (PITCH + 63) / 64;
  constexpr int CLAST = PITCH - 64 * (CPL - 1);
  int cx[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    cx[c] = (c + 1 < CPL || lane < CLAST) ? wrap_index(X0 - WOP_R + 64 * c + lane, nx) : 0;
  __syncthreads();
  // fill: wave w takes the (field, row) lines w, w + NW, w + 2 NW, ..., LPR
  // lines per round so that LPR CPL loads per lane are in flight (the
  // registers of the products are not live yet)
  constexpr int LINES = NC * WOP_RY;
  constexpr int LPR = 16 / CPL > 4 ? 16 / CPL : 4;
  for (int l0 = w; l0 < LINES; l0 += LPR * NW) {
    float v[LPR][CPL];
#pragma unroll
    for (int k = 0; k < LPR; ++k) {
      const int ln = l0 + NW * k;
      if (ln < LINES) {
        const int c = ln / WOP_RY, r = ln - c * WOP_RY;
        const float* rp = src + c * nn + (int64_t)rowy[r] * nx;
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) v[k][cc] = rp[cx[cc]];
      }
    }
#pragma unroll
    for (int k = 0; k < LPR; ++k) {
      const int ln = l0 + NW * k;
      if (ln < LINES) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc)
          if (cc + 1 < CPL || lane < CLAST) tile[ln * PITCH + 64 * cc + lane] = v[k][cc];
      }
    }
  }
  __syncthreads();
  const float* abase = tile + 16 * MT * wc + m + g;
  const f32x4* bq = reinterpret_cast<const f32x4*>(&op->b[0][lane]);
  f32x4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  wop_part<MT, PITCH, PLANE, 0>(kh, abase, bq, acc);
  // partial sums of parts 1 .. KS - 1 through LDS (the tile is no longer read)
  __syncthreads();
  f32x4* part = reinterpret_cast<f32x4*>(tile);
  if (kh > 0)
#pragma unroll
    for (int t = 0; t < MT; ++t) part[(((kh - 1) * NCT + wc) * MT + t) * 64 + lane] = acc[t];
  __syncthreads();
  if (kh > 0) return;
#pragma unroll
  for (int k = 1; k < WOP_KS; ++k)
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] += part[(((k - 1) * NCT + wc) * MT + t) * 64 + lane];
  // D[i][n]: lane holds n = lane % 16 = 5 t + co for pixels i = 4 g + v
  const int n = lane & 15;
  if (n >= NC * WOP_TR) return;
  const int t = n / NC, co = n % NC;
  const int y = Y0 + t;
  if (y >= ny) return;
  float* row = dst + co * nn + (int64_t)y * nx;
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int x = X0 + 16 * MT * wc + 16 * tt + 4 * g + v;
      if (x < nx) row[x] = acc[tt][v];
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

template <int MT, int NCT>
void launch_wop(const lbm_params* p, const WopOperand* op, const float* in, float* out, int batch,
                hipStream_t st) {
  using TL = WopTile<MT, NCT>;
  const int tiles_x = (p->nx + TL::COLS - 1) / TL::COLS;
  const int tiles_y = (p->ny + WOP_TR - 1) / WOP_TR;
  hipLaunchKernelGGL((k_wop_apply<MT, NCT>), dim3((unsigned)(tiles_x * tiles_y), (unsigned)batch),
                     dim3(TL::THREADS), 0, st, in, out, op, p->nx, p->ny, tiles_x);
}

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
  // Tile shape by the launch's size (measured on 64^2 .. 512^2, batches 1
  // to 32): two 16-column matrix tiles per wave (half the B traffic per
  // product) and two column tiles per workgroup where that gives 512 or
  // more workgroups, else one column tile per workgroup (more, smaller
  // workgroups spread over the CUs), else one matrix tile per wave; each
  // only while it computes at most 15% more columns than 16-column
  // granularity would.
  const int64_t ty64 = (p->ny + WOP_TR - 1) / WOP_TR;
  if ((p->nx / 16 + 1) * ty64 > 0x7fffffff) return fail(LBM_E_ARG, "window too large");
  const int64_t c16 = ((int64_t)p->nx + 15) / 16 * 16;
  auto ok = [&](int64_t cols, int64_t min_wgs) {
    const int64_t n = (p->nx + cols - 1) / cols;
    return n * cols * 100 <= c16 * 115 && n * ty64 * batch >= min_wgs;
  };
  const WopOperand* o = (const WopOperand*)d_op;
  hipStream_t st = (hipStream_t)hip_stream;
  if (ok(64, 512))
    launch_wop<2, 2>(p, o, d_in, d_out, batch, st);
  else if (ok(32, 512))
    launch_wop<2, 1>(p, o, d_in, d_out, batch, st);
  else if (ok(32, 0))
    launch_wop<1, 2>(p, o, d_in, d_out, batch, st);
  else
    launch_wop<1, 1>(p, o, d_in, d_out, batch, st);
  return launch_check("k_wop_apply launch");
}

}  // extern "C"
