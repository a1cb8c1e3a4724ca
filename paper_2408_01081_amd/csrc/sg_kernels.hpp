// Kernels of the learned window surrogate: a linear U-Net on the first-order
// system's variables with FiLM gains, 3x3 convolutions as implicit GEMMs on
// gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Activations are FP32 NHWC ([batch][y][x][channel]).  A convolution operand
// is rounded to BF16 when it is fed to the matrix core; with SPLIT = 3 each
// FP32 operand x is carried as hi = bf16(x), lo = bf16(x - hi) and the product
// is hi*hi + lo*hi + hi*lo (about 16 significant bits instead of 8).
//
// Every stored conv output z is pre-FiLM; a consumer multiplies it by the
// layer's gain gamma[b][c] when it loads it ("scale on load"), which is also
// exactly what the backward pass needs (dL/dz = gamma * dL/dy).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgk {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __host__ inline unsigned short bf16_bits(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return (unsigned short)u;
}
__device__ __host__ inline float bf16_value(unsigned short b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__device__ inline bf16 as_bf16(unsigned short b) {
  bf16 r;
  __builtin_memcpy(&r, &b, 2);
  return r;
}

// BF16 hi (and, SPLIT = 3, lo) parts of 8 activations times their gains,
// rounded to nearest even (a zero activation gives zero parts)
template <int SPLIT>
__device__ __forceinline__ void split8(const float (&x)[8], const float (&s)[8], bool scaled,
                                       bf16x8& hi, bf16x8& lo) {
  uint32_t h[4], l[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float a0 = scaled ? x[2 * j] * s[2 * j] : x[2 * j];
    const float a1 = scaled ? x[2 * j + 1] * s[2 * j + 1] : x[2 * j + 1];
    const unsigned short h0 = bf16_bits(a0), h1 = bf16_bits(a1);
    h[j] = (uint32_t)h0 | ((uint32_t)h1 << 16);
    if (SPLIT == 3) {
      const unsigned short l0 = bf16_bits(a0 - bf16_value(h0));
      const unsigned short l1 = bf16_bits(a1 - bf16_value(h1));
      l[j] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
  }
  __builtin_memcpy(&hi, h, 16);
  __builtin_memcpy(&lo, l, 16);
}

// ---------------------------------------------------------------------------
// 3x3 convolution, implicit GEMM.  Z[b,y,x,o] = sum_{t,i} Wt[t][o][i] * s[b,i] * X[b,y+dy,x+dx,i]
// Operand layouts of v_mfma_f32_16x16x32_bf16 (checked on gfx950 by an
// in-bounds probe): lane l holds A[l%16][8(l/16)+j], B[8(l/16)+j][l%16] for
// j = 0..7, and D[4(l/16)+j][l%16] for j = 0..3.
// One wave computes PB blocks of 16 pixels (each one row piece, W % 16 == 0)
// x 16*NB output channels, so every weight fragment feeds PB products.  The
// 4 waves of a workgroup are 4/KS pixel groups x KS slices of the reduction
// (input-channel chunks of 32 taken round robin); the KS partial sums are
// added in LDS in slice order, so the result does not depend on timing.  A
// workgroup covers 16 * PB * 4/KS pixels.  Cin % 32 == 0.
// Used for the forward pass (Wt = [9][Cout][Cin]) and, with the flipped and
// transposed weights, for the data gradient.  The input is read in FP32 and
// split into BF16 parts (split8) with its gain as it is read.
// ---------------------------------------------------------------------------
template <int SPLIT, int NB, int PB, int KS>
__global__ __launch_bounds__(256) void k_conv(const float* __restrict__ X,
                                              const float* __restrict__ xscale,
                                              const unsigned short* __restrict__ Whi,
                                              const unsigned short* __restrict__ Wlo,
                                              float* __restrict__ Z, int H, int W, int Cin,
                                              int Cout, int circular, int accumulate) {
  static_assert(KS == 1 || KS == 2 || KS == 4, "reduction slices per workgroup");
  constexpr int PG = 4 / KS;  // pixel groups per workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pg = wave / KS, ks = wave % KS;
  const int64_t HW = (int64_t)H * W;
  const int m = lane & 15, kq = lane >> 4;
  const int co0 = blockIdx.y * 16 * NB;
  int64_t pix0[PB];
  int bb[PB], yy[PB], xx[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    pix0[pb] = ((int64_t)blockIdx.x * PG * PB + pg * PB + pb) * 16;
    bb[pb] = (int)(pix0[pb] / HW);
    const int rem = (int)(pix0[pb] - (int64_t)bb[pb] * HW);
    yy[pb] = rem / W;
    xx[pb] = rem - yy[pb] * W + m;
  }
  f32x4 acc[PB][NB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[pb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};

  for (int c0 = 32 * ks; c0 < Cin; c0 += 32 * KS) {
    // the gains of this lane's 8 input channels in each pixel block's image
    float sc[PB][8];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        sc[pb][j] = xscale ? xscale[(int64_t)bb[pb] * Cin + c0 + 8 * kq + j] : 1.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      bf16x8 ahi[PB], alo[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        int ys = yy[pb] + dy, xs = xx[pb] + dx;
        bool valid = true;
        if (circular) {
          ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
          xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
        } else {
          valid = ys >= 0 && ys < H && xs >= 0 && xs < W;
          ys = ys < 0 ? 0 : (ys >= H ? H - 1 : ys);
          xs = xs < 0 ? 0 : (xs >= W ? W - 1 : xs);
        }
        const int64_t xo = (((int64_t)bb[pb] * H + ys) * W + xs) * Cin + 8 * kq + c0;
        float4 u0 = {0.f, 0.f, 0.f, 0.f}, u1 = {0.f, 0.f, 0.f, 0.f};
        if (valid) {
          u0 = *reinterpret_cast<const float4*>(X + xo);
          u1 = *reinterpret_cast<const float4*>(X + xo + 4);
        }
        const float a[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        split8<SPLIT>(a, sc[pb], xscale != nullptr, ahi[pb], alo[pb]);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t wo = ((int64_t)t * Cout + co0 + 16 * nb + m) * Cin + 8 * kq + c0;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(Whi + wo);
        bf16x8 blo;
        if (SPLIT == 3) blo = *reinterpret_cast<const bf16x8*>(Wlo + wo);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[pb], bhi, acc[pb][nb], 0, 0, 0);
          if (SPLIT == 3) {
            acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[pb], bhi, acc[pb][nb], 0, 0, 0);
            acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[pb], blo, acc[pb][nb], 0, 0, 0);
          }
        }
      }
    }
  }
  if (KS > 1) {
    // slices 1..KS-1 hand their sums to slice 0 of the same pixel group
    __shared__ f32x4 red[KS > 1 ? 4 : 1][PB * NB][64];
    if (ks > 0) {
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) red[wave][pb * NB + nb][lane] = acc[pb][nb];
    }
    __syncthreads();
    if (ks > 0) return;
#pragma unroll
    for (int k = 1; k < KS; ++k)
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const f32x4 r = red[wave + k][pb * NB + nb][lane];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[pb][nb][j] += r[j];
        }
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float* zp = Z + (pix0[pb] + 4 * kq + j) * Cout + co0 + 16 * nb + m;
        *zp = accumulate ? *zp + acc[pb][nb][j] : acc[pb][nb][j];
      }
}

// ---------------------------------------------------------------------------
// The same convolution with the input tile staged in LDS.  A workgroup computes
// a block of RW rows x WT pixels of one image (WT = 64 with W % 64 == 0, or
// WT = W = 32 or 16; RW * WT = 64 or 256) x CT output channels; for every
// 32-channel chunk of the input the neighbourhood of those pixels (one pixel
// more on every side) is read from the FP32 activations, multiplied by the gain and
// split into BF16 hi and lo parts exactly as split8 does, and stored in
// LDS (20 dwords per pixel: 16 data + 4 padding, so the 16 lanes of an
// A-fragment read hit distinct banks), where all 9 taps and all waves read it.  Wave w owns 16 PB pixels (w mod WPX) x
// 16 NB output channels (w / WPX).  The products are accumulated in the same
// order as k_conv<SPLIT, NB, PB, 1> (chunks, taps, channel blocks, pixel
// blocks), so the two give bitwise identical results.  Cin % 32 == 0,
// Cout % CT == 0.
// ---------------------------------------------------------------------------
template <int SPLIT, int PB, int NB, bool WL = false, int WT = 64, int RW = 64 / WT>
__global__ __launch_bounds__(256) void k_convt(const float* __restrict__ X,
                                               const float* __restrict__ xscale,
                                               const unsigned short* __restrict__ Whi,
                                               const unsigned short* __restrict__ Wlo,
                                               float* __restrict__ Z, int H, int W, int Cin,
                                               int Cout, int circular, int accumulate) {
  // the workgroup's pixels: RW rows of WT pixels (WT = 64 for W >= 64, else W)
  constexpr int NPX = RW * WT;
  constexpr int WPX = NPX / (16 * PB);  // waves along the pixels
  constexpr int WCO = 4 / WPX;          // waves along the output channels
  static_assert(WPX * WCO == 4 && NPX % (16 * PB) == 0, "four waves per workgroup");
  constexpr int CT = WCO * 16 * NB;     // output channels per workgroup
  constexpr int TR = RW + 2;           // tile rows: those rows + one each side
  constexpr int TW = WT + 2;           // tile columns: WT pixels + one each side
  constexpr int PS = 20;               // dwords per tile pixel
  constexpr int NH = SPLIT == 3 ? 2 : 1;
  // WL: the chunk's weights of the workgroup's CT channels for all 9 taps
  // are staged in LDS as well ([hi/lo][tap][channel], PS dwords per channel)
  constexpr int WS = WL ? 9 * CT * PS : 0;
  __shared__ uint4 tile4[NH * (TR * TW * PS + WS) / 4];
  uint32_t* tile = reinterpret_cast<uint32_t*>(tile4);
  uint32_t* wtile = tile + NH * TR * TW * PS;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  const int wp = wave % WPX, wc = wave / WPX;
  // the workgroup's block: rows y .. y + RW - 1, columns x0 .. x0 + WT - 1
  const int tx = W / WT, tiles = (H / RW) * tx;
  const int b = (int)(blockIdx.x / (unsigned)tiles);
  const int rem = (int)(blockIdx.x - (unsigned)b * (unsigned)tiles);
  const int y = (rem / tx) * RW, x0 = (rem - (rem / tx) * tx) * WT;
  const int cw = 16 * NB * wc;  // the wave's channels within the workgroup's CT
  const int co0 = blockIdx.y * CT + cw;
  const int px0 = 16 * PB * wp;

  f32x4 acc[PB][NB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[pb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // staging: thread t handles the items t, t + 256, ... of the tile (and of
  // the weights); 256 is a multiple of 4, so its piece q of 8 channels is
  // the same in every item.  A chunk's loads (input tile, gains, weights)
  // are all issued before the first is used, so their latencies overlap, and
  // those of the next chunk are in flight during this chunk's products.
  constexpr int NTILE = TR * TW * 4, PER = (NTILE + 255) / 256;
  constexpr int NWT = WL ? 9 * CT * 4 : 1, PERW = (NWT + 255) / 256;
  const int q = threadIdx.x & 3;
  float4 u0[PER], u1[PER];
  bool valid[PER];
  float sc[8];
  // (dword arrays: arrays of uint4 were placed in scratch memory)
  uint32_t wh[WL ? PERW : 1][4], wl[WL ? PERW : 1][4];
  auto issue = [&](int c0) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      const int col = (i >> 2) % TW, row = (i >> 2) / TW;
      int ys = y + row - 1, xs = x0 + col - 1;
      bool v = i < NTILE;
      if (circular) {
        ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
        xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
      } else {
        v = v && ys >= 0 && ys < H && xs >= 0 && xs < W;
      }
      valid[k] = v;
      if (v) {
        const int64_t xo = (((int64_t)b * H + ys) * W + xs) * Cin + c0 + 8 * q;
        u0[k] = *reinterpret_cast<const float4*>(X + xo);
        u1[k] = *reinterpret_cast<const float4*>(X + xo + 4);
      }
    }
    if (xscale) {
      const float* sp = xscale + (int64_t)b * Cin + c0 + 8 * q;
#pragma unroll
      for (int j = 0; j < 8; ++j) sc[j] = sp[j];
    }
    if (WL) {
      // 9 taps x CT channels x 4 pieces of 8 input channels (from L2: every
      // workgroup reads the same weights)
#pragma unroll
      for (int k = 0; k < PERW; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NWT) {
          const int co = (i >> 2) % CT, t = (i >> 2) / CT;
          const int64_t wo = ((int64_t)t * Cout + blockIdx.y * CT + co) * Cin + c0 + 8 * q;
          const uint4 a = *reinterpret_cast<const uint4*>(Whi + wo);
          wh[k][0] = a.x; wh[k][1] = a.y; wh[k][2] = a.z; wh[k][3] = a.w;
          if (SPLIT == 3) {
            const uint4 c = *reinterpret_cast<const uint4*>(Wlo + wo);
            wl[k][0] = c.x; wl[k][1] = c.y; wl[k][2] = c.z; wl[k][3] = c.w;
          }
        }
      }
    }
  };
  issue(0);
  for (int c0 = 0; c0 < Cin; c0 += 32) {
    if (c0) __syncthreads();  // every wave is done with the previous chunk
    // TR rows x TW columns x 4 pieces of 8 channels, hi (and lo)
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (k + 1 < PER || i < NTILE) {
      const int col = (i >> 2) % TW, row = (i >> 2) / TW;
      uint4 vh = {0u, 0u, 0u, 0u}, vl = {0u, 0u, 0u, 0u};
      if (valid[k]) {
        float a[8] = {u0[k].x, u0[k].y, u0[k].z, u0[k].w, u1[k].x, u1[k].y, u1[k].z, u1[k].w};
        if (xscale) {
#pragma unroll
          for (int j = 0; j < 8; ++j) a[j] *= sc[j];
        }
        uint32_t h[4], l[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const unsigned short h0 = bf16_bits(a[2 * j]), h1 = bf16_bits(a[2 * j + 1]);
          h[j] = (uint32_t)h0 | ((uint32_t)h1 << 16);
          if (SPLIT == 3) {
            const unsigned short l0 = bf16_bits(a[2 * j] - bf16_value(h0));
            const unsigned short l1 = bf16_bits(a[2 * j + 1] - bf16_value(h1));
            l[j] = (uint32_t)l0 | ((uint32_t)l1 << 16);
          }
        }
        vh = (uint4){h[0], h[1], h[2], h[3]};
        if (SPLIT == 3) vl = (uint4){l[0], l[1], l[2], l[3]};
      }
      const int d = (row * TW + col) * PS + 4 * q;
      *reinterpret_cast<uint4*>(tile + d) = vh;
      if (SPLIT == 3) *reinterpret_cast<uint4*>(tile + TR * TW * PS + d) = vl;
      }
    }
    if (WL) {
#pragma unroll
      for (int k = 0; k < PERW; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NWT) {
          const int co = (i >> 2) % CT, t = (i >> 2) / CT;
          const int d = (t * CT + co) * PS + 4 * q;
          *reinterpret_cast<uint4*>(wtile + d) = (uint4){wh[k][0], wh[k][1], wh[k][2], wh[k][3]};
          if (SPLIT == 3)
            *reinterpret_cast<uint4*>(wtile + WS + d) = (uint4){wl[k][0], wl[k][1], wl[k][2], wl[k][3]};
        }
      }
    }
    if (c0 + 32 < Cin) issue(c0 + 32);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      bf16x8 ahi[PB], alo[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const int p = px0 + 16 * pb + m, r = p / WT, xp = p - r * WT;
        const int d = ((r + dy + 1) * TW + xp + dx + 1) * PS + 4 * kq;
        ahi[pb] = *reinterpret_cast<const bf16x8*>(tile + d);
        if (SPLIT == 3) alo[pb] = *reinterpret_cast<const bf16x8*>(tile + TR * TW * PS + d);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x8 bhi, blo;
        if (WL) {
          const int d = (t * CT + cw + 16 * nb + m) * PS + 4 * kq;
          bhi = *reinterpret_cast<const bf16x8*>(wtile + d);
          if (SPLIT == 3) blo = *reinterpret_cast<const bf16x8*>(wtile + WS + d);
        } else {
          const int64_t wo = ((int64_t)t * Cout + co0 + 16 * nb + m) * Cin + 8 * kq + c0;
          bhi = *reinterpret_cast<const bf16x8*>(Whi + wo);
          if (SPLIT == 3) blo = *reinterpret_cast<const bf16x8*>(Wlo + wo);
        }
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[pb], bhi, acc[pb][nb], 0, 0, 0);
          if (SPLIT == 3) {
            acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[pb], bhi, acc[pb][nb], 0, 0, 0);
            acc[pb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[pb], blo, acc[pb][nb], 0, 0, 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = px0 + 16 * pb + 4 * kq + j, r = p / WT, xp = p - r * WT;
        const int64_t pix = ((int64_t)b * H + y + r) * W + x0 + xp;
        float* zp = Z + pix * Cout + co0 + 16 * nb + m;
        *zp = accumulate ? *zp + acc[pb][nb][j] : acc[pb][nb][j];
      }
}

// ---------------------------------------------------------------------------
// Weight gradient.  dW[t][o][i] = sum_{b,p} G[b,p,o] * s_o[b,o] * X[b,p+off_t,i] * s_i[b,i]
// As a GEMM: D (16 o x 16 i) += A (16 o x 32 pixels) B (32 pixels x 16 i).
// grid: x = tap (9) * (Cout/16) * (Cin/(16 NI)), y = pixel split; each of the
// 4 waves takes every 4th chunk of 32 pixels of the split, the waves' sums are
// added in LDS in a fixed order and written to partial[split][t][o][i].
// ---------------------------------------------------------------------------
template <int SPLIT, int NI>
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ G,
                                               const float* __restrict__ gscale,
                                               const float* __restrict__ X,
                                               const float* __restrict__ xscale,
                                               float* __restrict__ partial, int B, int H, int W,
                                               int Cin, int Cout, int circular,
                                               int64_t pix_per_split) {
  __shared__ float red[4][16 * NI][16 + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  const int nib = Cin / (16 * NI), nob = Cout / 16;
  int id = blockIdx.x;
  const int t = id / (nob * nib);
  id -= t * nob * nib;
  const int ob = id / nib, ib = id - ob * nib;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  const int o = ob * 16 + m;  // A row for this lane
  const int64_t HW = (int64_t)H * W;
  const int64_t p_begin = (int64_t)blockIdx.y * pix_per_split;
  f32x4 acc[NI];
#pragma unroll
  for (int k = 0; k < NI; ++k) acc[k] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int64_t pc = p_begin + 32 * wave; pc < p_begin + pix_per_split; pc += 128) {
    float a[8], xv[NI][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t p = pc + 8 * kq + j;
      const int b = (int)(p / HW);
      const int r = (int)(p - (int64_t)b * HW);
      const int yy = r / W, xx = r - yy * W;
      a[j] = G[p * Cout + o] * (gscale ? gscale[(int64_t)b * Cout + o] : 1.f);
      int ys = yy + dy, xs = xx + dx;
      bool valid = true;
      if (circular) {
        ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
        xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
      } else {
        valid = ys >= 0 && ys < H && xs >= 0 && xs < W;
        ys = ys < 0 ? 0 : (ys >= H ? H - 1 : ys);
        xs = xs < 0 ? 0 : (xs >= W ? W - 1 : xs);
      }
      const float* xp = X + (((int64_t)b * H + ys) * W + xs) * Cin;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int i = (ib * NI + k) * 16 + m;
        float v = valid ? xp[i] : 0.f;
        if (xscale) v *= xscale[(int64_t)b * Cin + i];
        xv[k][j] = v;
      }
    }
    bf16x8 ahi, alo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned short h = bf16_bits(a[j]);
      ahi[j] = as_bf16(h);
      alo[j] = as_bf16(bf16_bits(a[j] - bf16_value(h)));
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      bf16x8 bhi, blo;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned short h = bf16_bits(xv[k][j]);
        bhi[j] = as_bf16(h);
        blo[j] = as_bf16(bf16_bits(xv[k][j] - bf16_value(h)));
      }
      acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[k], 0, 0, 0);
      if (SPLIT == 3) {
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[k], 0, 0, 0);
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[k], 0, 0, 0);
      }
    }
  }
  // D[row = o (4kq + j)][col = i (m)]
#pragma unroll
  for (int k = 0; k < NI; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][16 * k + m][4 * kq + j] = acc[k][j];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * 16 * NI; e += 256) {
    const int ii = e % (16 * NI), oo = e / (16 * NI);
    const float s = ((red[0][ii][oo] + red[1][ii][oo]) + red[2][ii][oo]) + red[3][ii][oo];
    const int i = ib * NI * 16 + ii, oabs = ob * 16 + oo;
    partial[(((int64_t)blockIdx.y * 9 + t) * Cout + oabs) * Cin + i] = s;
  }
}

// sum the pixel splits in a fixed order: grad[o][i][t] (master layout)
// The weight gradient with both operands staged in LDS, channel-major (the
// matrix core's reduction runs over pixels, which must be contiguous per
// channel): a workgroup owns a 32 x 32 (output, input channel) tile of all 9
// taps and sweeps blocks of 64 pixels, blocks blockIdx.x, blockIdx.x +
// gridDim.x, ...  A block is 64 pixels of one image row (W % 64 == 0) or
// RB = 64 / W whole rows (W = 16, 32; H % RB == 0), pixel p at row
// y + p / PW, column x0 + p % PW (PW = min(W, 64)).  Per block it stages
//   gT[h][o][p]       gamma-scaled gradient, split into hi/lo, 72 bf16 per row;
//   xT[h][d][i][r][p] the gain-scaled input at tap (r - 1, d - 1) of pixel p
//                     (three copies d = 0, 1, 2 so that every tap reads 8
//                     pixels at an aligned offset), 72 per row;
// (row strides of 36 and 108 dwords keep the 16 lanes of a fragment read on
// distinct banks).  Wave w computes the 16 x 16 sub-tile (w / 2, w mod 2) for
// all taps and writes partial[blockIdx.x][t][o][i] for k_wgrad_reduce.
template <int SPLIT>
__global__ __launch_bounds__(256) void k_wgradt(const float* __restrict__ G,
                                                const float* __restrict__ gscale,
                                                const float* __restrict__ X,
                                                const float* __restrict__ xscale,
                                                float* __restrict__ partial, int B, int H, int W,
                                                int Cin, int Cout, int circular) {
  constexpr int NH = SPLIT == 3 ? 2 : 1;
  constexpr int RS = 72;                      // bf16 per staged row (64 + 8 padding)
  constexpr int GT = 32 * RS;                 // gT elements per hi/lo part
  constexpr int XT = 3 * 32 * 3 * RS;         // xT elements per hi/lo part
  __shared__ uint4 lds4[NH * (GT + XT) * 2 / 16];
  unsigned short* gT = reinterpret_cast<unsigned short*>(lds4);
  unsigned short* xT = gT + NH * GT;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  const int nit = Cin / 32;
  const int o0 = (int)(blockIdx.y / (unsigned)nit) * 32, i0 = (int)(blockIdx.y % (unsigned)nit) * 32;
  const int ow = 16 * (wave >> 1), iw = 16 * (wave & 1);
  const int PW = W < 64 ? W : 64;   // pixels of a block per image row
  const int RB = 64 / PW;           // image rows per block
  const int tx = W / PW;            // blocks across a row
  const int HB = H / RB;            // block rows per image
  const int64_t nblocks = (int64_t)B * HB * tx;

  f32x4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // A block's operands pass through registers: the next block's loads are
  // issued before this block's matrix-core phase and written to LDS after
  // it, so their latency hides behind the products (one workgroup per CU).
  // Input: halo rows hr = 0 .. RB + 1 (image y - 1 + hr), halo columns
  // hc = 0 .. PW + 1 (image x0 - 1 + hc), 4 x 8 channels per element, at
  // most 4 elements per thread ((RB + 2) (PW + 2) 4 <= 1024 for 64 % W == 0
  // or W % 64 == 0); each element is tap (r - 1, d - 1) of the pixels at row
  // hr - r, column hc - d.
  const int HC = PW + 2;
  const int NIT = (RB + 2) * HC * 4;
  constexpr int MAXIT = 4;
  float gr[8], xr[MAXIT][8];
  auto fetch = [&](int64_t blk) {
    const int b = (int)(blk / ((int64_t)HB * tx));
    const int rem = (int)(blk - (int64_t)b * HB * tx);
    const int y = (rem / tx) * RB, x0 = (rem - (rem / tx) * tx) * 64;
    {
      // gradient: thread t -> pixel t mod 64, output channels 8 (t / 64) ...
      // (a wave writes one channel row at 64 consecutive pixels: no two
      // lanes on one LDS bank but the two halves of a dword)
      const int p = threadIdx.x & 63, q = threadIdx.x >> 6;
      const int64_t go = (((int64_t)b * H + y + p / PW) * W + x0 + p % PW) * Cout + o0 + 8 * q;
      const float4 u0 = *reinterpret_cast<const float4*>(G + go);
      const float4 u1 = *reinterpret_cast<const float4*>(G + go + 4);
      gr[0] = u0.x; gr[1] = u0.y; gr[2] = u0.z; gr[3] = u0.w;
      gr[4] = u1.x; gr[5] = u1.y; gr[6] = u1.z; gr[7] = u1.w;
      if (gscale) {
        const float* sc = gscale + (int64_t)b * Cout + o0 + 8 * q;
#pragma unroll
        for (int j = 0; j < 8; ++j) gr[j] *= sc[j];
      }
    }
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = threadIdx.x + 256 * k;
#pragma unroll
      for (int j = 0; j < 8; ++j) xr[k][j] = 0.f;
      if (it >= NIT) continue;
      // consecutive lanes take consecutive halo columns (see the gradient)
      const int hc = it % HC, hr = (it / HC) % (RB + 2), q = it / (HC * (RB + 2));
      int ys = y + hr - 1, xs = x0 + hc - 1;
      bool valid = true;
      if (circular) {
        ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
        xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
      } else {
        valid = ys >= 0 && ys < H && xs >= 0 && xs < W;
      }
      if (valid) {
        const int64_t xo = (((int64_t)b * H + ys) * W + xs) * Cin + i0 + 8 * q;
        const float4 u0 = *reinterpret_cast<const float4*>(X + xo);
        const float4 u1 = *reinterpret_cast<const float4*>(X + xo + 4);
        xr[k][0] = u0.x; xr[k][1] = u0.y; xr[k][2] = u0.z; xr[k][3] = u0.w;
        xr[k][4] = u1.x; xr[k][5] = u1.y; xr[k][6] = u1.z; xr[k][7] = u1.w;
        if (xscale) {
          const float* sc = xscale + (int64_t)b * Cin + i0 + 8 * q;
#pragma unroll
          for (int j = 0; j < 8; ++j) xr[k][j] *= sc[j];
        }
      }
    }
  };
  auto stage = [&]() {
    {
      const int p = threadIdx.x & 63, q = threadIdx.x >> 6;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned short h = bf16_bits(gr[j]);
        gT[(8 * q + j) * RS + p] = h;
        if (SPLIT == 3) gT[GT + (8 * q + j) * RS + p] = bf16_bits(gr[j] - bf16_value(h));
      }
    }
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = threadIdx.x + 256 * k;
      if (it >= NIT) continue;
      const int hc = it % HC, hr = (it / HC) % (RB + 2), q = it / (HC * (RB + 2));
      unsigned short hb[8], lb[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        hb[j] = bf16_bits(xr[k][j]);
        lb[j] = bf16_bits(xr[k][j] - bf16_value(hb[j]));
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int pr = hr - r;
        if (pr < 0 || pr >= RB) continue;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int c = hc - d;
          if (c < 0 || c >= PW) continue;
          const int pp = pr * PW + c;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int e = ((d * 32 + 8 * q + j) * 3 + r) * RS + pp;
            xT[e] = hb[j];
            if (SPLIT == 3) xT[XT + e] = lb[j];
          }
        }
      }
    }
  };

  if ((int64_t)blockIdx.x < nblocks) fetch(blockIdx.x);
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    __syncthreads();  // the previous block's fragments have been read
    stage();
    if (blk + gridDim.x < nblocks) fetch(blk + gridDim.x);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int pk = 32 * ks + 8 * kq;
      const int ga = (ow + m) * RS + pk;
      const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(gT + ga);
      bf16x8 alo;
      if (SPLIT == 3) alo = *reinterpret_cast<const bf16x8*>(gT + GT + ga);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int r = t / 3, d = t % 3;  // dy + 1, dx + 1
        const int xb = ((d * 32 + iw + m) * 3 + r) * RS + pk;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(xT + xb);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[t], 0, 0, 0);
        if (SPLIT == 3) {
          const bf16x8 blo = *reinterpret_cast<const bf16x8*>(xT + XT + xb);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[t], 0, 0, 0);
        }
      }
    }
  }
  // D[row = o (4 kq + j)][col = i (m)]
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      partial[(((int64_t)blockIdx.x * 9 + t) * Cout + o0 + ow + 4 * kq + j) * Cin + i0 + iw + m] =
          acc[t][j];
}

__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial,
                                                      int nsplit, int Cin, int Cout,
                                                      float* __restrict__ grad) {
  // 64 weights per workgroup, 4 groups of threads summing every 4th split,
  // the 4 group sums added in order
  __shared__ float sh[4][64];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  const int64_t n = (int64_t)9 * Cout * Cin;
  float s = 0.f;
  if (e < n)
    for (int k = g; k < nsplit; k += 4) s += partial[(int64_t)k * n + e];
  sh[g][el] = s;
  __syncthreads();
  if (g || e >= n) return;
  s = ((sh[0][el] + sh[1][el]) + sh[2][el]) + sh[3][el];
  const int t = (int)(e / ((int64_t)Cout * Cin));
  const int64_t oi = e - (int64_t)t * Cout * Cin;
  const int o = (int)(oi / Cin), i = (int)(oi - (int64_t)o * Cin);
  grad[((int64_t)o * Cin + i) * 9 + t] = s;
}

// master weights [o][i][3][3] FP32 -> BF16 hi/lo in [t][o][i] (forward) and
// flipped/transposed [t][i][o] (data gradient)
__global__ __launch_bounds__(256) void k_prep_weights(const float* __restrict__ w, int Cin,
                                                      int Cout, unsigned short* __restrict__ fhi,
                                                      unsigned short* __restrict__ flo,
                                                      unsigned short* __restrict__ bhi,
                                                      unsigned short* __restrict__ blo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)9 * Cout * Cin;
  if (e >= n) return;
  const int o = (int)(e / (9 * Cin));
  const int r = (int)(e - (int64_t)o * 9 * Cin);
  const int i = r / 9, t = r - i * 9;
  const float v = w[e];
  const unsigned short h = bf16_bits(v);
  const unsigned short l = bf16_bits(v - bf16_value(h));
  fhi[((int64_t)t * Cout + o) * Cin + i] = h;
  flo[((int64_t)t * Cout + o) * Cin + i] = l;
  const int tb = 8 - t;
  bhi[((int64_t)tb * Cin + i) * Cout + o] = h;
  blo[((int64_t)tb * Cin + i) * Cout + o] = l;
}

// ---------------------------------------------------------------------------
// pooling / up-sampling (NHWC, scale on load); thread e handles the 4
// channels 4 (e mod C/4) .. + 3 of one pixel (C % 4 == 0), each with the
// operations written for one element
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float4 scale4(const float* s, int64_t i) {
  return s ? ld4(s + i) : make_float4(1.f, 1.f, 1.f, 1.f);
}

// pixel and channel of 4-channel item e of a [B][H][W][C] tensor
__device__ __forceinline__ void item4(int64_t e, int H, int W, int C, int& b, int& y, int& x,
                                      int& c) {
  const int C4 = C >> 2;
  int64_t r = e / C4;
  c = 4 * (int)(e - r * C4);
  x = (int)(r % W);
  r /= W;
  y = (int)(r % H);
  b = (int)(r / H);
}

// out[b,Y,X,c] = 1/4 sum_{2x2} s[b,c] in[b,2Y+u,2X+v,c]
__global__ __launch_bounds__(256) void k_pool(const float* __restrict__ in,
                                              const float* __restrict__ scale,
                                              float* __restrict__ out, int B, int Ho, int Wo,
                                              int C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * Ho * Wo * C / 4) return;
  int b, Y, X, c;
  item4(e, Ho, Wo, C, b, Y, X, c);
  const int Wi = 2 * Wo;
  const float* p = in + (((int64_t)b * 2 * Ho + 2 * Y) * Wi + 2 * X) * C + c;
  const float4 s = scale4(scale, (int64_t)b * C + c);
  const float4 p0 = ld4(p), p1 = ld4(p + C), p2 = ld4(p + (int64_t)Wi * C),
               p3 = ld4(p + (int64_t)Wi * C + C);
  float4 o;
  o.x = 0.25f * s.x * ((p0.x + p1.x) + (p2.x + p3.x));
  o.y = 0.25f * s.y * ((p0.y + p1.y) + (p2.y + p3.y));
  o.z = 0.25f * s.z * ((p0.z + p1.z) + (p2.z + p3.z));
  o.w = 0.25f * s.w * ((p0.w + p1.w) + (p2.w + p3.w));
  *reinterpret_cast<float4*>(out + 4 * e) = o;
}

// out[b,y,x,c] = sc[b,c] coarse[b,y/2,x/2,c] + ss[b,c] skip[b,y,x,c]
__global__ __launch_bounds__(256) void k_upadd(const float* __restrict__ coarse,
                                               const float* __restrict__ sc,
                                               const float* __restrict__ skip,
                                               const float* __restrict__ ss,
                                               float* __restrict__ out, int B, int H, int W,
                                               int C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * H * W * C / 4) return;
  int b, y, x, c;
  item4(e, H, W, C, b, y, x, c);
  const float4 cv = ld4(coarse + (((int64_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
  const float4 a = scale4(sc, (int64_t)b * C + c), t = scale4(ss, (int64_t)b * C + c);
  const float4 k = ld4(skip + 4 * e);
  float4 o;
  o.x = a.x * cv.x + t.x * k.x;
  o.y = a.y * cv.y + t.y * k.y;
  o.z = a.z * cv.z + t.z * k.z;
  o.w = a.w * cv.w + t.w * k.w;
  *reinterpret_cast<float4*>(out + 4 * e) = o;
}

// backward of pooling, plus an optional addend:
// out[b,y,x,c] = 1/4 g[b,y/2,x/2,c] + (add ? add[b,y,x,c] : 0)
__global__ __launch_bounds__(256) void k_pool_back(const float* __restrict__ g,
                                                   const float* __restrict__ add,
                                                   float* __restrict__ out, int B, int H, int W,
                                                   int C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * H * W * C / 4) return;
  int b, y, x, c;
  item4(e, H, W, C, b, y, x, c);
  const float4 gv = ld4(g + (((int64_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
  float4 o = make_float4(0.25f * gv.x, 0.25f * gv.y, 0.25f * gv.z, 0.25f * gv.w);
  if (add) {
    const float4 d = ld4(add + 4 * e);
    o.x += d.x;
    o.y += d.y;
    o.z += d.z;
    o.w += d.w;
  }
  *reinterpret_cast<float4*>(out + 4 * e) = o;
}

// backward of nearest up-sampling: out[b,Y,X,c] = sum_{2x2} g[b,2Y+u,2X+v,c]
__global__ __launch_bounds__(256) void k_up_back(const float* __restrict__ g,
                                                 float* __restrict__ out, int B, int Ho, int Wo,
                                                 int C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * Ho * Wo * C / 4) return;
  int b, Y, X, c;
  item4(e, Ho, Wo, C, b, Y, X, c);
  const int Wi = 2 * Wo;
  const float* p = g + (((int64_t)b * 2 * Ho + 2 * Y) * Wi + 2 * X) * C + c;
  const float4 p0 = ld4(p), p1 = ld4(p + C), p2 = ld4(p + (int64_t)Wi * C),
               p3 = ld4(p + (int64_t)Wi * C + C);
  float4 o;
  o.x = (p0.x + p1.x) + (p2.x + p3.x);
  o.y = (p0.y + p1.y) + (p2.y + p3.y);
  o.z = (p0.z + p1.z) + (p2.z + p3.z);
  o.w = (p0.w + p1.w) + (p2.w + p3.w);
  *reinterpret_cast<float4*>(out + 4 * e) = o;
}

}  // namespace sgk
