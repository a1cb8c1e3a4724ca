// Learned window surrogate (C ABI in include/sg.h): a linear U-Net on the
// first-order system's variables with FiLM gains, trained on windows of the
// lattice Boltzmann scheme and checked by it.  Forward, loss, backward and
// Adam all run in this file's kernels and sg_kernels.hpp's matrix-core
// convolutions; the host code only sequences launches.
//
// Input per sample: 8 physical channels [8][H][W] (v_x, v_y, sigma_xx,
// sigma_yy, sigma_xy, lambda, mu, rho).  pre: U = (v, j) through the inverse
// of Eq. sigma_num with the pixel's material, divided by the per-sample RMS s
// of U, channels 5..31 zero.  Conditioning t in [-1, 1] from theta =
// atan2(mean c_mu, mean c_K) (time step at half the CFL-like limit, so theta
// fixes both Courant numbers); FiLM gain of conv layer l, output channel c:
// gamma[b][c] = sum_m a_l[c][m] T_m(t_b), Chebyshev T_0..T_3.  post:
// U' = U + s * gamma_out * z_out[0..4], back to physical fields.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "lbm_host.hpp"
#include "sg.h"
#include "sg_kernels.hpp"

using namespace sgk;
using lbmh::fail;
using lbmh::hip_check;
using lbmh::launch_check;
using lbmh::round_up;

namespace {

constexpr int NBASIS = 4;
constexpr int CP = 32;  // padded input/output channels
constexpr double THETA_LO = 8.0 * M_PI / 180.0;
constexpr double THETA_HI = 45.0 * M_PI / 180.0;

struct LayerSpec {
  const char* name;
  int cin, cout, level;
};
// two convolutions per level, four levels; order = parameter order
const LayerSpec kLayers[] = {
    {"in", 32, 32, 0},    {"e0a", 32, 32, 0},   {"e0b", 32, 32, 0},   {"e1a", 32, 64, 1},
    {"e1b", 64, 64, 1},   {"e2a", 64, 128, 2},  {"e2b", 128, 128, 2}, {"e3a", 128, 128, 3},
    {"e3b", 128, 128, 3}, {"d2a", 128, 128, 2}, {"d2b", 128, 64, 2},  {"d1a", 64, 64, 1},
    {"d1b", 64, 32, 1},   {"d0a", 32, 32, 0},   {"d0b", 32, 32, 0},   {"out", 32, 32, 0}};
constexpr int NL = (int)(sizeof(kLayers) / sizeof(kLayers[0]));
enum { L_IN, L_E0A, L_E0B, L_E1A, L_E1B, L_E2A, L_E2B, L_E3A, L_E3B, L_D2A, L_D2B, L_D1A,
       L_D1B, L_D0A, L_D0B, L_OUT };

constexpr int RT = 256;

// ---- per-sample statistics and pre/post -------------------------------------
struct Mat {
  float cK, cm, rho;
};
__device__ inline Mat material(const float* in, int64_t HW, int64_t p) {
  const float lam = in[5 * HW + p], mu = in[6 * HW + p], rho = in[7 * HW + p];
  Mat m;
  m.cK = sqrtf((lam + mu) / rho);
  m.cm = sqrtf(mu / rho);
  m.rho = rho;
  return m;
}
__device__ inline void phys_to_U(const float* f, int64_t HW, int64_t p, const Mat& m,
                                 float U[5]) {
  const float sxx = f[2 * HW + p] / m.rho, syy = f[3 * HW + p] / m.rho,
              sxy = f[4 * HW + p] / m.rho;
  U[0] = f[p];
  U[1] = f[HW + p];
  U[2] = -(sxx + syy) / (2.f * m.cK);
  U[3] = -(sxx - syy) / (2.f * m.cm);
  U[4] = -sxy / m.cm;
}

__device__ inline double wg_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = RT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per-sample statistics in two passes: SB workgroups per sample sum |U|^2,
// c_K and c_mu over their pixels (FP64), then one workgroup per sample adds
// the SB partial sums in a fixed order and forms s_b and the Chebyshev values
// T[b][m].
constexpr int SB = 64;  // workgroups per sample in the first pass

__global__ __launch_bounds__(RT) void k_stats_partial(const float* __restrict__ in, int HW,
                                                      double* __restrict__ part) {
  __shared__ double sh[RT];
  const int b = blockIdx.y;
  const float* f = in + (int64_t)b * 8 * HW;
  double u2 = 0.0, ck = 0.0, cm = 0.0;
  for (int p = blockIdx.x * RT + threadIdx.x; p < HW; p += SB * RT) {
    const Mat m = material(f, HW, p);
    float U[5];
    phys_to_U(f, HW, p, m, U);
    for (int c = 0; c < 5; ++c) u2 += (double)U[c] * U[c];
    ck += m.cK;
    cm += m.cm;
  }
  u2 = wg_sum(u2, sh);
  ck = wg_sum(ck, sh);
  cm = wg_sum(cm, sh);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)b * SB + blockIdx.x) * 3;
    o[0] = u2;
    o[1] = ck;
    o[2] = cm;
  }
}

// the FiLM gains of every layer, gamma[l][b][c] = sum_k a_l[c][k] T[b][k]
struct GammaArgs {
  const float* a[NL];
  float* g[NL];
  int cout[NL];
  int total;  // sum of cout
};

__global__ __launch_bounds__(RT) void k_stats(const double* __restrict__ part, int HW,
                                              float* __restrict__ sv, float* __restrict__ T) {
  __shared__ double sh[RT];
  const int b = blockIdx.x;
  const double* q = part + (int64_t)b * SB * 3;
  const bool mine = (int)threadIdx.x < SB;
  const double u2 = wg_sum(mine ? q[3 * threadIdx.x] : 0.0, sh);
  const double ck = wg_sum(mine ? q[3 * threadIdx.x + 1] : 0.0, sh);
  const double cm = wg_sum(mine ? q[3 * threadIdx.x + 2] : 0.0, sh);
  if (threadIdx.x == 0) {
    const double s = sqrt(u2 / (5.0 * HW));
    sv[b] = (float)(s > 0 ? s : 1.0);
    const double th = atan2(cm, ck);
    const double t = 2.0 * (th - THETA_LO) / (THETA_HI - THETA_LO) - 1.0;
    double Tm[NBASIS];
    Tm[0] = 1.0;
    Tm[1] = t;
    for (int k = 2; k < NBASIS; ++k) Tm[k] = 2.0 * t * Tm[k - 1] - Tm[k - 2];
    for (int k = 0; k < NBASIS; ++k) T[b * NBASIS + k] = (float)Tm[k];
  }
}

// x0[b][p][c] = U_c / s_b for c < 5, 0 otherwise; threads e < B * total
// also form the FiLM gain of one (sample, layer, channel)
__global__ __launch_bounds__(RT) void k_pre(const float* __restrict__ in, int B, int HW,
                                            const float* __restrict__ sv,
                                            float* __restrict__ x0, GammaArgs ga,
                                            const float* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (e < (int64_t)B * ga.total) {
    const int b = (int)(e / ga.total);
    int c = (int)(e - (int64_t)b * ga.total), l = 0;
    while (c >= ga.cout[l]) c -= ga.cout[l++];
    float s = 0.f;
    for (int k = 0; k < NBASIS; ++k) s = fmaf(ga.a[l][c * NBASIS + k], T[b * NBASIS + k], s);
    ga.g[l][b * ga.cout[l] + c] = s;
  }
  if (e >= (int64_t)B * HW) return;
  const int b = (int)(e / HW);
  const int64_t p = e - (int64_t)b * HW;
  const float* f = in + (int64_t)b * 8 * HW;
  const Mat m = material(f, HW, p);
  float U[5];
  phys_to_U(f, HW, p, m, U);
  const float r = 1.f / sv[b];
  float* o = x0 + e * CP;
  for (int c = 0; c < 5; ++c) o[c] = U[c] * r;
  for (int c = 5; c < CP; ++c) o[c] = 0.f;
}

// out[b][5][H][W] physical = fields of U + s gamma z_out[0..4]
__global__ __launch_bounds__(RT) void k_post(const float* __restrict__ in,
                                             const float* __restrict__ zout,
                                             const float* __restrict__ gout,
                                             const float* __restrict__ sv, int B, int HW,
                                             float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (e >= (int64_t)B * HW) return;
  const int b = (int)(e / HW);
  const int64_t p = e - (int64_t)b * HW;
  const float* f = in + (int64_t)b * 8 * HW;
  const Mat m = material(f, HW, p);
  float U[5];
  phys_to_U(f, HW, p, m, U);
  const float* z = zout + e * CP;
  const float* g = gout + (int64_t)b * CP;
  for (int c = 0; c < 5; ++c) U[c] = U[c] + sv[b] * (g[c] * z[c]);
  float* o = out + (int64_t)b * 5 * HW;
  o[p] = U[0];
  o[HW + p] = U[1];
  o[2 * HW + p] = -m.rho * (m.cK * U[2] + m.cm * U[3]);
  o[3 * HW + p] = -m.rho * (m.cK * U[2] - m.cm * U[3]);
  o[4 * HW + p] = -m.rho * (m.cm * U[4]);
}

// loss = mean (gamma z_out[0..4] - (U_target - U)/s)^2, gradient w.r.t. y_out
// (NHWC, 32 channels, zero beyond 5); per-workgroup partial sums
__global__ __launch_bounds__(RT) void k_loss(const float* __restrict__ in,
                                             const float* __restrict__ target,
                                             const float* __restrict__ zout,
                                             const float* __restrict__ gout,
                                             const float* __restrict__ sv, int B, int HW,
                                             float inv_n, float* __restrict__ gy,
                                             double* __restrict__ partial) {
  __shared__ double sh[RT];
  const int64_t e = (int64_t)blockIdx.x * RT + threadIdx.x;
  double l = 0.0;
  if (e < (int64_t)B * HW) {
    const int b = (int)(e / HW);
    const int64_t p = e - (int64_t)b * HW;
    const float* f = in + (int64_t)b * 8 * HW;
    const Mat m = material(f, HW, p);
    float U[5], Ut[5];
    phys_to_U(f, HW, p, m, U);
    phys_to_U(target + (int64_t)b * 5 * HW, HW, p, m, Ut);
    const float* z = zout + e * CP;
    const float* g = gout + (int64_t)b * CP;
    float* o = gy + e * CP;
    const float r = 1.f / sv[b];
    for (int c = 0; c < 5; ++c) {
      const float d = g[c] * z[c] - (Ut[c] - U[c]) * r;
      l += (double)d * d;
      o[c] = 2.f * d * inv_n;
    }
    for (int c = 5; c < CP; ++c) o[c] = 0.f;
  }
  l = wg_sum(l, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = l;
}

__global__ __launch_bounds__(RT) void k_sum_partials(const double* __restrict__ p, int n,
                                                     double* __restrict__ out) {
  __shared__ double sh[RT];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += RT) s += p[i];
  s = wg_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}

// dgamma[b][c] = sum_p g[b,p,c] z[b,p,c] (FiLM gain gradient).
// Two passes with coalesced reads: workgroup (b, s) takes
// pixel chunk s of sample b for all C channels (thread t: channel t mod C,
// every (RT / C)-th pixel), FP64 partial sums per channel added in a fixed
// order; then dgam[b][c] = sum over the S chunks in order.
__global__ __launch_bounds__(RT) void k_film_grad_part(const float* __restrict__ g,
                                                       const float* __restrict__ z, int HW, int C,
                                                       int S, double* __restrict__ part) {
  __shared__ double sh[RT];
  const int b = blockIdx.x / S, sidx = blockIdx.x - (blockIdx.x / S) * S;
  const int G = RT / C, c = threadIdx.x % C, grp = threadIdx.x / C;
  const int64_t p0 = (int64_t)HW * sidx / S, p1 = (int64_t)HW * (sidx + 1) / S;
  const float* gp = g + (int64_t)b * HW * C + c;
  const float* zp = z + (int64_t)b * HW * C + c;
  double acc = 0.0;
  if (grp < G)
    for (int64_t p = p0 + grp; p < p1; p += G) acc += (double)gp[p * C] * zp[p * C];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    double t = 0.0;
    for (int k = 0; k < G; ++k) t += sh[k * C + threadIdx.x];
    part[(int64_t)blockIdx.x * C + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(RT) void k_film_grad_sum(const double* __restrict__ part, int B,
                                                      int C, int S, float* __restrict__ dgam) {
  const int e = blockIdx.x * RT + threadIdx.x;
  if (e >= B * C) return;
  const int b = e / C, c = e - b * C;
  double t = 0.0;
  for (int k = 0; k < S; ++k) t += part[((int64_t)b * S + k) * C + c];
  dgam[e] = (float)t;
}

// da[c][m] = sum_b T[b][m] dgam[b][c]
__global__ __launch_bounds__(RT) void k_film_coef_grad(const float* __restrict__ dgam,
                                                       const float* __restrict__ T, int B, int C,
                                                       float* __restrict__ da) {
  const int e = blockIdx.x * RT + threadIdx.x;
  if (e >= C * NBASIS) return;
  const int c = e / NBASIS, m = e - c * NBASIS;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s = fmaf(T[b * NBASIS + m], dgam[b * C + c], s);
  da[e] = s;
}

__global__ __launch_bounds__(RT) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ mo, float* __restrict__ ve,
                                             int64_t n, float lr, float b1, float b2, float eps,
                                             float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float m = b1 * mo[i] + (1.f - b1) * gi;
  const float v = b2 * ve[i] + (1.f - b2) * gi * gi;
  mo[i] = m;
  ve[i] = v;
  p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---- host-side plan ----------------------------------------------------------
struct Tensor {
  float* p = nullptr;
  int H = 0, W = 0, C = 0;
};

struct Plan {
  int B, H, W, split, train;
  int64_t nparam = 0;
  int64_t woff[NL], aoff[NL];      // offsets in the parameter vector
  int64_t wq_off[NL];              // offsets in the bf16 weight arrays
  int64_t nwq = 0;
  size_t bytes = 0;
  // workspace offsets
  size_t o_param, o_grad, o_m, o_v, o_wfh, o_wfl, o_wbh, o_wbl, o_s, o_T, o_gam, o_dgam,
      o_part, o_spart, o_loss, o_x0, o_z[NL], o_pool[3], o_up[3], o_g[NL], o_gpool[3], o_gup[3],
      o_gtmp[2], o_wpart;
  int64_t wpart_floats = 0;
};

int level_h(const Plan& P, int l) { return P.H >> l; }
int level_w(const Plan& P, int l) { return P.W >> l; }

lbm_status make_plan(const sg_config* cfg, Plan* P) {
  if (!cfg) return fail(LBM_E_ARG, "null config");
  if (cfg->batch < 1 || cfg->height < 64 || cfg->width < 128)
    return fail(LBM_E_ARG, "need batch >= 1, height >= 64, width >= 128");
  if (cfg->height % 64 || cfg->width % 128)
    return fail(LBM_E_ARG, "height must be a multiple of 64 and width of 128");
  if (cfg->split != 1 && cfg->split != 3) return fail(LBM_E_ARG, "split must be 1 or 3");
  P->B = cfg->batch;
  P->H = cfg->height;
  P->W = cfg->width;
  P->split = cfg->split;
  P->train = cfg->train ? 1 : 0;
  int64_t np = 0, nq = 0;
  for (int l = 0; l < NL; ++l) {
    P->woff[l] = np;
    np += (int64_t)kLayers[l].cout * kLayers[l].cin * 9;
    P->aoff[l] = np;
    np += (int64_t)kLayers[l].cout * NBASIS;
    P->wq_off[l] = nq;
    nq += (int64_t)kLayers[l].cout * kLayers[l].cin * 9;
  }
  P->nparam = np;
  P->nwq = nq;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  const int64_t B = P->B;
  auto act = [&](int level, int C) { return (size_t)B * level_h(*P, level) * level_w(*P, level) * C * 4; };
  P->o_param = take(np * 4);
  P->o_wfh = take(nq * 2);
  P->o_wfl = take(nq * 2);
  P->o_wbh = take(nq * 2);
  P->o_wbl = take(nq * 2);
  P->o_s = take(B * 4);
  P->o_T = take(B * NBASIS * 4);
  P->o_gam = take((size_t)NL * B * 128 * 4);
  P->o_part = take(((size_t)B * P->H * P->W / RT + 1) * 8);
  P->o_spart = take((size_t)B * SB * 3 * 8);
  P->o_loss = take(8);
  P->o_x0 = take(act(0, CP));
  for (int l = 0; l < NL; ++l) P->o_z[l] = take(act(kLayers[l].level, kLayers[l].cout));
  const int pc[3] = {32, 64, 128};
  for (int k = 0; k < 3; ++k) P->o_pool[k] = take(act(k + 1, pc[k]));
  const int uc[3] = {32, 64, 128};  // u0 (level 0), u1 (level 1), u2 (level 2)
  for (int k = 0; k < 3; ++k) P->o_up[k] = take(act(k, uc[k]));
  if (P->train) {
    P->o_grad = take(np * 4);
    P->o_m = take(np * 4);
    P->o_v = take(np * 4);
    P->o_dgam = take((size_t)B * 128 * 4);
    for (int l = 0; l < NL; ++l) P->o_g[l] = take(act(kLayers[l].level, kLayers[l].cout));
    for (int k = 0; k < 3; ++k) P->o_gpool[k] = take(act(k + 1, pc[k]));
    for (int k = 0; k < 3; ++k) P->o_gup[k] = take(act(k, uc[k]));
    P->o_gtmp[0] = take(act(0, 128));  // generic scratch (largest level-0 gradient)
    P->o_gtmp[1] = take(act(0, 128));
    // weight-gradient partials: splits x 9 x Cout x Cin for the largest layer
    int64_t mx = 0;
    for (int l = 0; l < NL; ++l) {
      const int64_t v = (int64_t)9 * kLayers[l].cout * kLayers[l].cin;
      mx = v > mx ? v : mx;
    }
    P->wpart_floats = mx * 64;
    P->o_wpart = take(P->wpart_floats * 4);
  }
  P->bytes = o;
  return LBM_OK;
}

}  // namespace

struct sg_net {
  Plan P;
  char* ws;
  hipStream_t stream;
  float* param;
  float* grad;
  float *m, *v;
  unsigned short *wfh, *wfl, *wbh, *wbl;
  float* s;
  float* T;
  float* gam[NL];
  float* dgam;
  double* part;
  double* spart;  // per-sample statistics partials [B][SB][3]
  double* loss;
  float* x0;
  Tensor z[NL], pool[3], up[3], g[NL], gpool[3], gup[3], gtmp[2];
  float* wpart;
  int B;          // batch of the current forward
  int circular;   // padding of the current forward
  const float* in;
  int64_t adam_step;
  bool weights_ready;
  int conv_mode;  // 0: LDS-tiled kernel where it applies; 1: direct kernel only;
                  // 2: tiled, weights from global memory
};

namespace {

inline unsigned grid1(int64_t n) { return (unsigned)((n + RT - 1) / RT); }

template <int SPLIT, int NB, int PB, int KS>
void launch_conv(sg_net* n, const Tensor& x, const float* xscale, const unsigned short* wh,
                 const unsigned short* wl, Tensor& z, int cin, int cout, int accumulate) {
  const int64_t pixels = (int64_t)n->B * x.H * x.W;
  dim3 grid((unsigned)(pixels / (16 * PB * (4 / KS))), (unsigned)(cout / (16 * NB)));
  hipLaunchKernelGGL((k_conv<SPLIT, NB, PB, KS>), grid, dim3(256), 0, n->stream,
                     (const float*)x.p, xscale, wh, wl, z.p, x.H, x.W, cin, cout, n->circular,
                     accumulate);
}

// Tile shapes of the convolution, most work per wave first: (NB, PB, KS).
// The first one that gives at least kConvMinWG workgroups is used (else the
// one with the most workgroups), so small late layers still fill the chip.
struct ConvShape {
  int nb, pb, ks;
};
const ConvShape kConvShapes[] = {{4, 2, 1}, {4, 1, 1}, {2, 2, 1}, {2, 1, 1}, {4, 1, 2},
                                 {2, 1, 2}, {1, 1, 2}, {2, 1, 4}, {1, 1, 4}};
constexpr int64_t kConvMinWG = 1024;

int conv_shape(int64_t pixels, int cin, int cout) {
  int best = -1;
  int64_t best_wg = -1;
  for (int k = 0; k < (int)(sizeof(kConvShapes) / sizeof(kConvShapes[0])); ++k) {
    const ConvShape& c = kConvShapes[k];
    const int64_t px = 16 * c.pb * (4 / c.ks);
    if (cout % (16 * c.nb) || pixels % px || cin / 32 < c.ks) continue;
    const int64_t wg = pixels / px * (cout / (16 * c.nb));
    if (wg >= kConvMinWG) return k;
    if (wg > best_wg) best_wg = wg, best = k;
  }
  return best >= 0 ? best : 3;
}

template <int SPLIT>
void launch_conv_shape(int k, sg_net* n, const Tensor& x, const float* xscale,
                       const unsigned short* wh, const unsigned short* wl, Tensor& z, int cin,
                       int cout, int accumulate) {
  switch (k) {
    case 0: return launch_conv<SPLIT, 4, 2, 1>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 1: return launch_conv<SPLIT, 4, 1, 1>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 2: return launch_conv<SPLIT, 2, 2, 1>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 3: return launch_conv<SPLIT, 2, 1, 1>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 4: return launch_conv<SPLIT, 4, 1, 2>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 5: return launch_conv<SPLIT, 2, 1, 2>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 6: return launch_conv<SPLIT, 1, 1, 2>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    case 7: return launch_conv<SPLIT, 2, 1, 4>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    default: return launch_conv<SPLIT, 1, 1, 4>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  }
}

template <int SPLIT, int PB, int NB, bool WL, int WT, int RW = 64 / WT>
void launch_convt(sg_net* n, const Tensor& x, const float* xscale, const unsigned short* wh,
                  const unsigned short* wl, Tensor& z, int cin, int cout, int accumulate) {
  constexpr int CT = (4 / (RW * WT / (16 * PB))) * 16 * NB;
  dim3 grid((unsigned)((int64_t)n->B * x.H * x.W / (RW * WT)), (unsigned)(cout / CT));
  hipLaunchKernelGGL((k_convt<SPLIT, PB, NB, WL, WT, RW>), grid, dim3(256), 0, n->stream,
                     (const float*)x.p, xscale, wh, wl, z.p, x.H, x.W, cin, cout, n->circular,
                     accumulate);
}

// The LDS-tiled kernel where the row is a multiple of 64 pixels or 32 or 16
// pixels long and it gives at least 256 workgroups: 64 output channels per
// workgroup (2 x 2 waves of 32 x 32) when that still gives 512 workgroups,
// else 32 (4 waves of 16 pixels x 32 channels, weights staged in LDS too),
// or 16 where 32 gives fewer than 256 workgroups.
template <int SPLIT, int WT>
void conv_tiled_w(sg_net* n, const Tensor& x, const float* xscale, const unsigned short* wh,
                  const unsigned short* wl, Tensor& z, int cin, int cout, int accumulate) {
  const int64_t tiles = (int64_t)n->B * x.H * x.W / 64;
  // blocks of 4 rows x 64 pixels (one wave per row, 32 output channels)
  // where they still give 256 workgroups: the halo rows (and the weights)
  // are staged once for 4x as many pixels
  if (WT == 64 && n->conv_mode != 2 && x.H % 4 == 0 && tiles / 4 * (cout / 32) >= 256) {
    // weights read from L2 rather than staged, so that two workgroups share
    // a CU, where the grid has more than one per CU
    if (tiles / 4 * (cout / 32) >= 512)
      launch_convt<SPLIT, 4, 2, false, 64, 4>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    else
      launch_convt<SPLIT, 4, 2, true, 64, 4>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
    return;
  }
  if (cout % 64 == 0 && tiles * (cout / 64) >= 512)
    launch_convt<SPLIT, 2, 2, false, WT>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else if (tiles * (cout / 32) < 256 && n->conv_mode == 2)
    launch_convt<SPLIT, 1, 1, false, WT>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else if (tiles * (cout / 32) < 256)
    // 16 output channels per workgroup, for enough workgroups
    launch_convt<SPLIT, 1, 1, true, WT>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else if (n->conv_mode == 2)
    launch_convt<SPLIT, 1, 2, false, WT>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else
    launch_convt<SPLIT, 1, 2, true, WT>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
}

template <int SPLIT>
bool conv_tiled(sg_net* n, const Tensor& x, const float* xscale, const unsigned short* wh,
                const unsigned short* wl, Tensor& z, int cin, int cout, int accumulate) {
  if (n->conv_mode == 1 || cin % 32 || cout % 32 || ((int64_t)x.H * x.W) % 64) return false;
  // too few workgroups to fill the chip even with 16 output channels per
  // workgroup: the direct kernel splits the reduction over waves instead
  if ((int64_t)n->B * x.H * x.W / 64 * (cout / 16) < 256) return false;
  if (x.W % 64 == 0)
    conv_tiled_w<SPLIT, 64>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else if (x.W == 32)
    conv_tiled_w<SPLIT, 32>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else if (x.W == 16)
    conv_tiled_w<SPLIT, 16>(n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else
    return false;
  return true;
}

void conv(sg_net* n, const Tensor& x, const float* xscale, int l, Tensor& z, bool backward,
          int accumulate) {
  const LayerSpec& L = kLayers[l];
  const int cin = backward ? L.cout : L.cin, cout = backward ? L.cin : L.cout;
  const unsigned short* wh = (backward ? n->wbh : n->wfh) + n->P.wq_off[l];
  const unsigned short* wl = (backward ? n->wbl : n->wfl) + n->P.wq_off[l];
  const int64_t pixels = (int64_t)n->B * x.H * x.W;
  // the LDS-tiled kernel splits its input tiles itself
  if (n->P.split == 3 ? conv_tiled<3>(n, x, xscale, wh, wl, z, cin, cout, accumulate)
                      : conv_tiled<1>(n, x, xscale, wh, wl, z, cin, cout, accumulate))
    return;
  // the direct kernel splits its input (with its gain) into BF16 hi/lo parts
  // as it reads it
  const int k = conv_shape(pixels, cin, cout);
  if (n->P.split == 3)
    launch_conv_shape<3>(k, n, x, xscale, wh, wl, z, cin, cout, accumulate);
  else
    launch_conv_shape<1>(k, n, x, xscale, wh, wl, z, cin, cout, accumulate);
}

void pool(sg_net* n, const Tensor& in, const float* scale, Tensor& out) {
  const int64_t e = (int64_t)n->B * out.H * out.W * out.C / 4;  // 4 channels per thread
  hipLaunchKernelGGL(k_pool, dim3(grid1(e)), dim3(RT), 0, n->stream, in.p, scale, out.p, n->B,
                     out.H, out.W, out.C);
}

void upadd(sg_net* n, const Tensor& coarse, const float* sc, const Tensor& skip, const float* ss,
           Tensor& out) {
  const int64_t e = (int64_t)n->B * out.H * out.W * out.C / 4;  // 4 channels per thread
  hipLaunchKernelGGL(k_upadd, dim3(grid1(e)), dim3(RT), 0, n->stream, coarse.p, sc, skip.p, ss,
                     out.p, n->B, out.H, out.W, out.C);
}

void prep_weights(sg_net* n) {
  for (int l = 0; l < NL; ++l) {
    const int64_t e = (int64_t)9 * kLayers[l].cin * kLayers[l].cout;
    hipLaunchKernelGGL(k_prep_weights, dim3(grid1(e)), dim3(RT), 0, n->stream,
                       n->param + n->P.woff[l], kLayers[l].cin, kLayers[l].cout,
                       n->wfh + n->P.wq_off[l], n->wfl + n->P.wq_off[l], n->wbh + n->P.wq_off[l],
                       n->wbl + n->P.wq_off[l]);
  }
  n->weights_ready = true;
}

lbm_status forward(sg_net* n, const float* in, int B, int circular) {
  Plan& P = n->P;
  n->B = B;
  n->circular = circular;
  n->in = in;
  if (!n->weights_ready) prep_weights(n);
  const int HW = P.H * P.W;
  hipLaunchKernelGGL(k_stats_partial, dim3(SB, B), dim3(RT), 0, n->stream, in, HW, n->spart);
  hipLaunchKernelGGL(k_stats, dim3(B), dim3(RT), 0, n->stream, (const double*)n->spart, HW, n->s,
                     n->T);
  GammaArgs ga;
  ga.total = 0;
  for (int l = 0; l < NL; ++l) {
    ga.a[l] = n->param + P.aoff[l];
    ga.g[l] = n->gam[l];
    ga.cout[l] = kLayers[l].cout;
    ga.total += kLayers[l].cout;
  }
  const int64_t npre = (int64_t)B * (HW > ga.total ? HW : ga.total);
  hipLaunchKernelGGL(k_pre, dim3(grid1(npre)), dim3(RT), 0, n->stream, in, B, HW, n->s, n->x0, ga,
                     (const float*)n->T);
  Tensor x0{n->x0, P.H, P.W, CP};
  Tensor* z = n->z;
  float** gm = n->gam;
  conv(n, x0, nullptr, L_IN, z[L_IN], false, 0);
  conv(n, z[L_IN], gm[L_IN], L_E0A, z[L_E0A], false, 0);
  conv(n, z[L_E0A], gm[L_E0A], L_E0B, z[L_E0B], false, 0);
  pool(n, z[L_E0B], gm[L_E0B], n->pool[0]);
  conv(n, n->pool[0], nullptr, L_E1A, z[L_E1A], false, 0);
  conv(n, z[L_E1A], gm[L_E1A], L_E1B, z[L_E1B], false, 0);
  pool(n, z[L_E1B], gm[L_E1B], n->pool[1]);
  conv(n, n->pool[1], nullptr, L_E2A, z[L_E2A], false, 0);
  conv(n, z[L_E2A], gm[L_E2A], L_E2B, z[L_E2B], false, 0);
  pool(n, z[L_E2B], gm[L_E2B], n->pool[2]);
  conv(n, n->pool[2], nullptr, L_E3A, z[L_E3A], false, 0);
  conv(n, z[L_E3A], gm[L_E3A], L_E3B, z[L_E3B], false, 0);
  upadd(n, z[L_E3B], gm[L_E3B], z[L_E2B], gm[L_E2B], n->up[2]);
  conv(n, n->up[2], nullptr, L_D2A, z[L_D2A], false, 0);
  conv(n, z[L_D2A], gm[L_D2A], L_D2B, z[L_D2B], false, 0);
  upadd(n, z[L_D2B], gm[L_D2B], z[L_E1B], gm[L_E1B], n->up[1]);
  conv(n, n->up[1], nullptr, L_D1A, z[L_D1A], false, 0);
  conv(n, z[L_D1A], gm[L_D1A], L_D1B, z[L_D1B], false, 0);
  upadd(n, z[L_D1B], gm[L_D1B], z[L_E0B], gm[L_E0B], n->up[0]);
  conv(n, n->up[0], nullptr, L_D0A, z[L_D0A], false, 0);
  conv(n, z[L_D0A], gm[L_D0A], L_D0B, z[L_D0B], false, 0);
  conv(n, z[L_D0B], gm[L_D0B], L_OUT, z[L_OUT], false, 0);
  return launch_check("surrogate forward");
}

// backward through conv layer l: g_y (dL/dy_l) -> parameter gradients and
// dL/d(input of l) written to gin (accumulated if accumulate)
void conv_back(sg_net* n, int l, const Tensor& gy, const Tensor& xin, const float* xscale,
               Tensor& gin, int accumulate) {
  Plan& P = n->P;
  const LayerSpec& L = kLayers[l];
  const Tensor& zl = n->z[l];
  const int HW = zl.H * zl.W;
  // FiLM coefficients (the weight-gradient partials' buffer holds the
  // per-chunk sums; it is rewritten only after they have been added)
  int S = 16;
  while (S > 1 && ((int64_t)n->B * S * L.cout * 2 > n->P.wpart_floats || HW / S < 64)) S /= 2;
  hipLaunchKernelGGL(k_film_grad_part, dim3(n->B * S), dim3(RT), 0, n->stream, gy.p, zl.p, HW,
                     L.cout, S, (double*)n->wpart);
  hipLaunchKernelGGL(k_film_grad_sum, dim3(grid1((int64_t)n->B * L.cout)), dim3(RT), 0,
                     n->stream, (const double*)n->wpart, n->B, L.cout, S, n->dgam);
  hipLaunchKernelGGL(k_film_coef_grad, dim3(grid1(L.cout * NBASIS)), dim3(RT), 0, n->stream,
                     (const float*)n->dgam, (const float*)n->T, n->B, L.cout,
                     n->grad + P.aoff[l]);
  // weights: dW = sum (gamma * gy) (x) (xscale * x)
  const int64_t pixels = (int64_t)n->B * HW;
  const bool rows_fit = zl.W % 64 == 0 || (64 % zl.W == 0 && zl.H % (64 / zl.W) == 0);
  if (n->conv_mode != 1 && rows_fit && L.cin % 32 == 0 && L.cout % 32 == 0) {
    // LDS-staged kernel: ~256 workgroups (one per CU: 92 KB of LDS), as many
    // pixel-block groups as the partials' buffer holds
    const int64_t nblocks = pixels / 64;
    const int tiles = (L.cout / 32) * (L.cin / 32);
    int64_t ng = 256 / tiles;
    const int64_t cap = n->P.wpart_floats / ((int64_t)9 * L.cout * L.cin);
    ng = ng > cap ? cap : ng;
    ng = ng > nblocks ? nblocks : ng;
    ng = ng < 1 ? 1 : ng;
    if (P.split == 3)
      hipLaunchKernelGGL((k_wgradt<3>), dim3((unsigned)ng, (unsigned)tiles), dim3(256), 0,
                         n->stream, gy.p, (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B,
                         zl.H, zl.W, L.cin, L.cout, n->circular);
    else
      hipLaunchKernelGGL((k_wgradt<1>), dim3((unsigned)ng, (unsigned)tiles), dim3(256), 0,
                         n->stream, gy.p, (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B,
                         zl.H, zl.W, L.cin, L.cout, n->circular);
    const int64_t nw = (int64_t)9 * L.cout * L.cin;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nw + 63) / 64)), dim3(RT), 0, n->stream,
                       (const float*)n->wpart, (int)ng, L.cin, L.cout, n->grad + P.woff[l]);
    if (gin.p) conv(n, gy, n->gam[l], l, gin, true, accumulate);
    return;
  }
  int nsplit = 1;
  while (nsplit < 64 && pixels / (nsplit * 2) >= 2048 && (pixels % (nsplit * 2 * 128)) == 0)
    nsplit *= 2;
  const int64_t pps = pixels / nsplit;
  const int ni = L.cin >= 64 ? 4 : 2;
  dim3 grid((unsigned)(9 * (L.cout / 16) * (L.cin / (16 * ni))), (unsigned)nsplit);
  if (P.split == 3) {
    if (ni == 4)
      hipLaunchKernelGGL((k_wgrad<3, 4>), grid, dim3(256), 0, n->stream, gy.p,
                         (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B, zl.H, zl.W,
                         L.cin, L.cout, n->circular, pps);
    else
      hipLaunchKernelGGL((k_wgrad<3, 2>), grid, dim3(256), 0, n->stream, gy.p,
                         (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B, zl.H, zl.W,
                         L.cin, L.cout, n->circular, pps);
  } else {
    if (ni == 4)
      hipLaunchKernelGGL((k_wgrad<1, 4>), grid, dim3(256), 0, n->stream, gy.p,
                         (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B, zl.H, zl.W,
                         L.cin, L.cout, n->circular, pps);
    else
      hipLaunchKernelGGL((k_wgrad<1, 2>), grid, dim3(256), 0, n->stream, gy.p,
                         (const float*)n->gam[l], xin.p, xscale, n->wpart, n->B, zl.H, zl.W,
                         L.cin, L.cout, n->circular, pps);
  }
  const int64_t nw = (int64_t)9 * L.cout * L.cin;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nw + 63) / 64)), dim3(RT), 0, n->stream,
                     (const float*)n->wpart, nsplit, L.cin, L.cout, n->grad + P.woff[l]);
  // data gradient: conv with flipped, transposed weights of (gamma * gy)
  if (gin.p) conv(n, gy, n->gam[l], l, gin, true, accumulate);
}

void up_back(sg_net* n, const Tensor& g, Tensor& out) {
  const int64_t e = (int64_t)n->B * out.H * out.W * out.C / 4;  // 4 channels per thread
  hipLaunchKernelGGL(k_up_back, dim3(grid1(e)), dim3(RT), 0, n->stream, g.p, out.p, n->B, out.H,
                     out.W, out.C);
}

void pool_back(sg_net* n, const Tensor& g, const float* add, Tensor& out) {
  const int64_t e = (int64_t)n->B * out.H * out.W * out.C / 4;  // 4 channels per thread
  hipLaunchKernelGGL(k_pool_back, dim3(grid1(e)), dim3(RT), 0, n->stream, g.p, add, out.p, n->B,
                     out.H, out.W, out.C);
}

lbm_status backward(sg_net* n) {
  Tensor* z = n->z;
  Tensor* g = n->g;
  float** gm = n->gam;
  Tensor x0{n->x0, n->P.H, n->P.W, CP};
  Tensor none;
  // g[L_OUT] holds dL/dy_out from the loss kernel
  conv_back(n, L_OUT, g[L_OUT], z[L_D0B], gm[L_D0B], g[L_D0B], 0);
  conv_back(n, L_D0B, g[L_D0B], z[L_D0A], gm[L_D0A], g[L_D0A], 0);
  conv_back(n, L_D0A, g[L_D0A], n->up[0], nullptr, n->gup[0], 0);       // dL/du0
  up_back(n, n->gup[0], g[L_D1B]);                                        // dL/dy_d1b
  conv_back(n, L_D1B, g[L_D1B], z[L_D1A], gm[L_D1A], g[L_D1A], 0);
  conv_back(n, L_D1A, g[L_D1A], n->up[1], nullptr, n->gup[1], 0);       // dL/du1
  up_back(n, n->gup[1], g[L_D2B]);
  conv_back(n, L_D2B, g[L_D2B], z[L_D2A], gm[L_D2A], g[L_D2A], 0);
  conv_back(n, L_D2A, g[L_D2A], n->up[2], nullptr, n->gup[2], 0);       // dL/du2
  up_back(n, n->gup[2], g[L_E3B]);
  conv_back(n, L_E3B, g[L_E3B], z[L_E3A], gm[L_E3A], g[L_E3A], 0);
  conv_back(n, L_E3A, g[L_E3A], n->pool[2], nullptr, n->gpool[2], 0);   // dL/dp3
  pool_back(n, n->gpool[2], n->gup[2].p, g[L_E2B]);                      // + skip from u2
  conv_back(n, L_E2B, g[L_E2B], z[L_E2A], gm[L_E2A], g[L_E2A], 0);
  conv_back(n, L_E2A, g[L_E2A], n->pool[1], nullptr, n->gpool[1], 0);
  pool_back(n, n->gpool[1], n->gup[1].p, g[L_E1B]);
  conv_back(n, L_E1B, g[L_E1B], z[L_E1A], gm[L_E1A], g[L_E1A], 0);
  conv_back(n, L_E1A, g[L_E1A], n->pool[0], nullptr, n->gpool[0], 0);
  pool_back(n, n->gpool[0], n->gup[0].p, g[L_E0B]);
  conv_back(n, L_E0B, g[L_E0B], z[L_E0A], gm[L_E0A], g[L_E0A], 0);
  conv_back(n, L_E0A, g[L_E0A], z[L_IN], gm[L_IN], g[L_IN], 0);
  conv_back(n, L_IN, g[L_IN], x0, nullptr, none, 0);
  return launch_check("surrogate backward");
}

}  // namespace

extern "C" {

size_t sg_workspace_bytes(const sg_config* cfg) {
  Plan P;
  if (make_plan(cfg, &P) != LBM_OK) return 0;
  return P.bytes;
}

int64_t sg_param_count(void) {
  int64_t np = 0;
  for (int l = 0; l < NL; ++l) np += (int64_t)kLayers[l].cout * (kLayers[l].cin * 9 + NBASIS);
  return np;
}

lbm_status sg_create(const sg_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                     sg_net** out) {
  if (!out) return fail(LBM_E_ARG, "null out");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(LBM_E_ARG, "workspace null or misaligned");
  sg_net* n = new (std::nothrow) sg_net();
  if (!n) return fail(LBM_E_ARG, "out of host memory");
  lbm_status s = make_plan(cfg, &n->P);
  if (s == LBM_OK && ws_bytes < n->P.bytes) s = fail(LBM_E_SPACE, "workspace too small");
  if (s) {
    delete n;
    return s;
  }
  Plan& P = n->P;
  char* w = (char*)d_ws;
  n->ws = w;
  n->stream = (hipStream_t)hip_stream;
  n->param = (float*)(w + P.o_param);
  n->wfh = (unsigned short*)(w + P.o_wfh);
  n->wfl = (unsigned short*)(w + P.o_wfl);
  n->wbh = (unsigned short*)(w + P.o_wbh);
  n->wbl = (unsigned short*)(w + P.o_wbl);
  n->s = (float*)(w + P.o_s);
  n->T = (float*)(w + P.o_T);
  for (int l = 0; l < NL; ++l) n->gam[l] = (float*)(w + P.o_gam) + (size_t)l * P.B * 128;
  n->part = (double*)(w + P.o_part);
  n->spart = (double*)(w + P.o_spart);
  n->loss = (double*)(w + P.o_loss);
  n->x0 = (float*)(w + P.o_x0);
  for (int l = 0; l < NL; ++l) {
    const int lv = kLayers[l].level;
    n->z[l] = Tensor{(float*)(w + P.o_z[l]), level_h(P, lv), level_w(P, lv), kLayers[l].cout};
  }
  const int pc[3] = {32, 64, 128};
  for (int k = 0; k < 3; ++k) {
    n->pool[k] = Tensor{(float*)(w + P.o_pool[k]), level_h(P, k + 1), level_w(P, k + 1), pc[k]};
    n->up[k] = Tensor{(float*)(w + P.o_up[k]), level_h(P, k), level_w(P, k), pc[k]};
  }
  if (P.train) {
    n->grad = (float*)(w + P.o_grad);
    n->m = (float*)(w + P.o_m);
    n->v = (float*)(w + P.o_v);
    n->dgam = (float*)(w + P.o_dgam);
    for (int l = 0; l < NL; ++l) {
      const int lv = kLayers[l].level;
      n->g[l] = Tensor{(float*)(w + P.o_g[l]), level_h(P, lv), level_w(P, lv), kLayers[l].cout};
    }
    for (int k = 0; k < 3; ++k) {
      n->gpool[k] = Tensor{(float*)(w + P.o_gpool[k]), level_h(P, k + 1), level_w(P, k + 1), pc[k]};
      n->gup[k] = Tensor{(float*)(w + P.o_gup[k]), level_h(P, k), level_w(P, k), pc[k]};
    }
    n->wpart = (float*)(w + P.o_wpart);
  }
  n->adam_step = 0;
  n->weights_ready = false;
  *out = n;
  return LBM_OK;
}

lbm_status sg_set_conv_mode(sg_net* n, int32_t mode) {
  if (!n) return fail(LBM_E_ARG, "null net");
  if (mode < 0 || mode > 2) return fail(LBM_E_ARG, "conv mode must be 0, 1 or 2");
  n->conv_mode = mode;
  return LBM_OK;
}

lbm_status sg_destroy(sg_net* n) {
  delete n;
  return LBM_OK;
}

lbm_status sg_set_params(sg_net* n, const float* d_params) {
  if (!n || !d_params) return fail(LBM_E_ARG, "null argument");
  lbm_status s = hip_check(hipMemcpyAsync(n->param, d_params, n->P.nparam * 4,
                                          hipMemcpyDeviceToDevice, n->stream),
                           "set params");
  if (s) return s;
  n->weights_ready = false;
  if (n->P.train) {
    s = hip_check(hipMemsetAsync(n->m, 0, n->P.nparam * 4, n->stream), "reset adam");
    if (s == LBM_OK) s = hip_check(hipMemsetAsync(n->v, 0, n->P.nparam * 4, n->stream), "reset adam");
    n->adam_step = 0;
  }
  return s;
}

lbm_status sg_get_params(sg_net* n, float* d_params) {
  if (!n || !d_params) return fail(LBM_E_ARG, "null argument");
  return hip_check(hipMemcpyAsync(d_params, n->param, n->P.nparam * 4, hipMemcpyDeviceToDevice,
                                  n->stream),
                   "get params");
}

lbm_status sg_get_grads(sg_net* n, float* d_grads) {
  if (!n || !d_grads) return fail(LBM_E_ARG, "null argument");
  if (!n->P.train) return fail(LBM_E_STATE, "network created without training buffers");
  return hip_check(hipMemcpyAsync(d_grads, n->grad, n->P.nparam * 4, hipMemcpyDeviceToDevice,
                                  n->stream),
                   "get grads");
}

lbm_status sg_forward(sg_net* n, const float* d_in, int32_t batch, int32_t circular,
                      float* d_out) {
  if (!n || !d_in || !d_out) return fail(LBM_E_ARG, "null argument");
  if (batch < 1 || batch > n->P.B) return fail(LBM_E_ARG, "batch out of range");
  lbm_status s = forward(n, d_in, batch, circular ? 1 : 0);
  if (s) return s;
  const int HW = n->P.H * n->P.W;
  hipLaunchKernelGGL(k_post, dim3(grid1((int64_t)batch * HW)), dim3(RT), 0, n->stream, d_in,
                     (const float*)n->z[L_OUT].p, (const float*)n->gam[L_OUT],
                     (const float*)n->s, batch, HW, d_out);
  return launch_check("surrogate post");
}

lbm_status sg_train_step(sg_net* n, const float* d_in, const float* d_target, int32_t batch,
                         int32_t circular, float lr, double* h_loss) {
  if (!n || !d_in || !d_target) return fail(LBM_E_ARG, "null argument");
  if (!n->P.train) return fail(LBM_E_STATE, "network created without training buffers");
  if (batch < 1 || batch > n->P.B) return fail(LBM_E_ARG, "batch out of range");
  lbm_status s = forward(n, d_in, batch, circular ? 1 : 0);
  if (s) return s;
  const int HW = n->P.H * n->P.W;
  const int64_t np = (int64_t)batch * HW;
  const unsigned nb = grid1(np);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(RT), 0, n->stream, d_in, d_target,
                     (const float*)n->z[L_OUT].p, (const float*)n->gam[L_OUT],
                     (const float*)n->s, batch, HW, (float)(1.0 / (5.0 * np)), n->g[L_OUT].p,
                     n->part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RT), 0, n->stream, (const double*)n->part,
                     (int)nb, n->loss);
  s = backward(n);
  if (s) return s;
  if (lr > 0.f) {
    n->adam_step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)n->adam_step), c2 = 1.f - powf(b2, (float)n->adam_step);
    hipLaunchKernelGGL(k_adam, dim3(grid1(n->P.nparam)), dim3(RT), 0, n->stream, n->param,
                       (const float*)n->grad, n->m, n->v, n->P.nparam, lr, b1, b2, 1e-8f, c1, c2);
    n->weights_ready = false;
    prep_weights(n);
  }
  s = launch_check("surrogate train step");
  if (s) return s;
  if (h_loss) {
    double lsum;
    s = hip_check(hipMemcpyAsync(&lsum, n->loss, 8, hipMemcpyDeviceToHost, n->stream), "loss copy");
    if (s) return s;
    s = hip_check(hipStreamSynchronize(n->stream), "loss sync");
    if (s) return s;
    *h_loss = lsum / (5.0 * np);
  }
  return LBM_OK;
}

}  // extern "C"
