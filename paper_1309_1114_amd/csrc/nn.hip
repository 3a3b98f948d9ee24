// nn.hip -- kernels of the learned x4 upscaler for gfx950.
//
// Convolutions run on the matrix cores: v_mfma_f32_16x16x32_bf16 with bf16
// operands and FP32 accumulators.  The element layout of that instruction
// (64 lanes, lane l):
//   A (16 x 32): row l % 16, columns 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16): column l % 16, rows 8 (l / 16) .. 8 (l / 16) + 7
//   D (16 x 16): column l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3
//
// Forward (and data-gradient) convolution: D[co][px] = W[co][ch] X[ch][px]
// per tap, K = 32 input channels.  The weights of the whole layer live in
// registers (A operands, read once per workgroup); the input tile with its
// one-pixel halo is staged in LDS as NHWC with a padded pixel stride, so a
// B operand (16 pixels of one row x 8 channels per lane group) is one
// conflict-free 16-byte LDS read shared by all output-channel blocks.
//
// Weight gradient: D[co][ci] = dY'[co][px] X[px + tap][ci], K = 32 pixels.
// Both operands need 8 consecutive pixels of one channel per lane, so the
// tile loader writes dY' and X transposed into LDS (X three times, shifted
// by the horizontal tap offset, which keeps every read 16-byte aligned).
// Each wave owns a subset of the nine taps and accumulates over all tiles
// of its workgroup in registers; one atomic add per weight and workgroup
// at the end.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "splotch_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// float -> bfloat16, round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// bf16 value strictly greater than zero (+inf included, NaN excluded).
__device__ __forceinline__ bool bf_pos(uint32_t m) { return m - 1u < 0x7f80u; }

__device__ __forceinline__ uint32_t mask_pair(uint32_t v, uint32_t m) {
  uint32_t lo = bf_pos(m & 0xffffu) ? (v & 0xffffu) : 0u;
  uint32_t hi = bf_pos(m >> 16) ? (v & 0xffff0000u) : 0u;
  return lo | hi;
}

__device__ __forceinline__ uint4 mask8(uint4 v, uint4 m) {
  return make_uint4(mask_pair(v.x, m.x), mask_pair(v.y, m.y), mask_pair(v.z, m.z),
                    mask_pair(v.w, m.w));
}

__device__ __forceinline__ uint32_t half_of(uint4 v, int e) {
  uint32_t w = e < 2 ? v.x : e < 4 ? v.y : e < 6 ? v.z : v.w;
  return (e & 1) ? (w >> 16) : (w & 0xffffu);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Eight consecutive channels [c0, c0 + 8) of one pixel, zero beyond cin, with
// the optional ReLU mask applied.  Vector path when cin is a multiple of 8.
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ x,
                                       const uint16_t* __restrict__ mask, size_t pix, int cin,
                                       int c0) {
  if (c0 >= cin) return make_uint4(0, 0, 0, 0);
  const size_t off = pix * (size_t)cin + c0;
  if ((cin & 7) == 0) {
    uint4 v = *reinterpret_cast<const uint4*>(x + off);
    if (mask) v = mask8(v, *reinterpret_cast<const uint4*>(mask + off));
    return v;
  }
  uint32_t e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uint32_t v = 0;
    if (c0 + k < cin) {
      v = x[off + k];
      if (mask && !bf_pos(mask[off + k])) v = 0;
    }
    e[k] = v;
  }
  return make_uint4(e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16),
                    e[6] | (e[7] << 16));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// 3x3 convolution, forward.  Output tile 16 x 16 pixels; wave w computes
// rows 4w .. 4w + 3.  KC = padded input channels / 32, CB = cout / 16.
// ---------------------------------------------------------------------------
constexpr int FT = 16;               // output tile side
constexpr int FI = FT + 2;           // input tile side (halo 1)

template <int KC, int CB>
__global__ __launch_bounds__(kThreads) void k_conv_fwd(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
    const float* __restrict__ bias, const uint16_t* __restrict__ mask, void* __restrict__ y,
    int h, int wd, int cin, int cout, int relu, int out_f32, int tiles_x, int tiles_y) {
  constexpr int CP = KC * 32;
  constexpr int PS = CP + 8;         // LDS pixel stride in bf16 (16-byte multiple, odd banks)
  constexpr int G = CP / 8;
  __shared__ __attribute__((aligned(16))) uint16_t tile[FI * FI * PS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int b = blockIdx.x;
  const int tx0 = (b % tiles_x) * FT;
  b /= tiles_x;
  const int ty0 = (b % tiles_y) * FT;
  const int img = b / tiles_y;
  const size_t img_base = (size_t)img * h * wd;

  // the layer's weights as A operands
  bf16x8 wr[9][KC][CB];
  {
    const int wl = lane & 15, wk = (lane >> 4) * 8;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int co = cb * 16 + wl;
          wr[t][kc][cb] = as_bf16x8(load8(w, nullptr, (size_t)co * 9 + t, cin, kc * 32 + wk));
        }
  }

  // the input tile: every load of a thread is issued before any LDS store,
  // so a wave waits for one memory latency, not one per 16-byte piece
  constexpr int NU = (FI * FI * G + kThreads - 1) / kThreads;
  uint4 piece[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int u = tid + k * kThreads;
    piece[k] = make_uint4(0, 0, 0, 0);
    if (u < FI * FI * G) {
      const int pix = u / G, g = u - pix * G;
      const int iy = pix / FI, ix = pix - iy * FI;
      const int gy = ty0 + iy - 1, gx = tx0 + ix - 1;
      if (gy >= 0 && gy < h && gx >= 0 && gx < wd)
        piece[k] = load8(x, mask, img_base + (size_t)gy * wd + gx, cin, g * 8);
    }
  }
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int u = tid + k * kThreads;
    if (u < FI * FI * G) {
      const int pix = u / G, g = u - pix * G;
      *reinterpret_cast<uint4*>(tile + pix * PS + g * 8) = piece[k];
    }
  }
  __syncthreads();

  f32x4 acc[4][CB];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[r][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int px = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ty = wave * 4 + r;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t % 3;
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const uint4 bv =
            *reinterpret_cast<const uint4*>(tile + ((ty + ky) * FI + px + kx) * PS + kc * 32 + kg);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[t][kc][cb], as_bf16x8(bv),
                                                               acc[r][cb], 0, 0, 0);
      }
    }
  }

  const int co_l = 4 * (lane >> 4);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gy = ty0 + wave * 4 + r, gx = tx0 + px;
    if (gy >= h || gx >= wd) continue;
    const size_t pix = img_base + (size_t)gy * wd + gx;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int co = cb * 16 + co_l;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float s = acc[r][cb][e] + (bias ? bias[co + e] : 0.f);
        if (relu && s < 0.f) s = 0.f;     // NaN passes through
        v[e] = s;
      }
      if (out_f32) {
        *reinterpret_cast<float4*>(static_cast<float*>(y) + pix * cout + co) =
            make_float4(v[0], v[1], v[2], v[3]);
      } else {
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(y) + pix * cout + co) =
            make_uint2(f2bf(v[0]) | (f2bf(v[1]) << 16), f2bf(v[2]) | (f2bf(v[3]) << 16));
      }
    }
  }
}

// wt[ci][2-ky][2-kx][co] = w[co][ky][kx][ci]
__global__ void k_flip(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int cin,
                       int cout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cout * 9 * cin) return;
  const int ci = i % cin, t = (i / cin) % 9, co = i / (9 * cin);
  wt[((size_t)ci * 9 + (8 - t)) * cout + co] = w[i];
}

// ---------------------------------------------------------------------------
// Weight and bias gradients.  Tile 8 x 16 output pixels; NB = ceil(cin / 16)
// input-channel blocks, CB = cout / 16 output-channel blocks.  Wave w owns
// taps w, w + 4, w + 8.
// ---------------------------------------------------------------------------
constexpr int WH = 8, WW = 16, WPIX = WH * WW;

template <int NB, int CB>
__global__ __launch_bounds__(kThreads) void k_conv_bwd_w(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
    const uint16_t* __restrict__ mask, float* __restrict__ dw, float* __restrict__ db, int h,
    int wd, int cin, int cout, int tiles_x, int tiles_y, int n_tiles) {
  constexpr int CI = NB * 16, CO = CB * 16;
  constexpr int DS = WPIX + 8;              // dY' channel stride (bf16)
  constexpr int XS = (WH + 2) * WW + 8;     // X channel stride (bf16)
  __shared__ __attribute__((aligned(16))) uint16_t dyT[CO * DS];
  __shared__ __attribute__((aligned(16))) uint16_t xT[3 * CI * XS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  f32x4 acc[3][CB][NB];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[j][cb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbs[CB * 8];
#pragma unroll
  for (int k = 0; k < CB * 8; ++k) dbs[k] = 0.f;

  const int p = tid & (WPIX - 1), half = tid >> 7;   // dY' loader: pixel, channel half
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    int b = tile;
    const int x0 = (b % tiles_x) * WW;
    b /= tiles_x;
    const int y0 = (b % tiles_y) * WH;
    const int img = b / tiles_y;
    const size_t img_base = (size_t)img * h * wd;
    __syncthreads();   // the previous tile's operands are consumed
    {
      const int gy = y0 + p / WW, gx = x0 + p % WW;
      const bool in = gy < h && gx < wd;
#pragma unroll
      for (int g = 0; g < CB; ++g) {
        const int c0 = (half * CB + g) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (in) v = load8(dy, mask, img_base + (size_t)gy * wd + gx, cout, c0);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t hv = half_of(v, e);
          dbs[g * 8 + e] += bf2f(hv);
          dyT[(c0 + e) * DS + p] = (uint16_t)hv;
        }
      }
    }
    for (int u = tid; u < (WH + 2) * (WW + 2) * (CI / 8); u += kThreads) {
      const int pix = u / (CI / 8), g = u - pix * (CI / 8);
      const int iy = pix / (WW + 2), ix = pix - iy * (WW + 2);
      const int gy = y0 + iy - 1, gx = x0 + ix - 1;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gy >= 0 && gy < h && gx >= 0 && gx < wd)
        v = load8(x, nullptr, img_base + (size_t)gy * wd + gx, cin, g * 8);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int c = ix - kx;
        if (c < 0 || c >= WW) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          xT[(kx * CI + g * 8 + e) * XS + iy * WW + c] = (uint16_t)half_of(v, e);
      }
    }
    __syncthreads();

#pragma unroll
    for (int s = 0; s < WPIX / 32; ++s) {
      const int P = s * 32 + (lane >> 4) * 8;
      const int r = P / WW, c = P % WW;
      uint4 a[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        a[cb] = *reinterpret_cast<const uint4*>(dyT + (cb * 16 + (lane & 15)) * DS + P);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int t = wave + 4 * j;
        if (t >= 9) continue;
        const int ky = t / 3, kx = t % 3;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const uint4 bx = *reinterpret_cast<const uint4*>(
              xT + (kx * CI + nb * 16 + (lane & 15)) * XS + (r + ky) * WW + c);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[j][cb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                as_bf16x8(a[cb]), as_bf16x8(bx), acc[j][cb][nb], 0, 0, 0);
        }
      }
    }
  }

#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int t = wave + 4 * j;
    if (t >= 9) continue;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int ci = nb * 16 + (lane & 15);
        if (ci >= cin) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int co = cb * 16 + 4 * (lane >> 4) + e;
          atomicAdd(dw + ((size_t)co * 9 + t) * cin + ci, acc[j][cb][nb][e]);
        }
      }
  }
  if (db) {
#pragma unroll
    for (int k = 0; k < CB * 8; ++k) {
      const float s = wave_sum(dbs[k]);
      if (lane == 0) atomicAdd(db + half * CB * 8 + k, s);
    }
  }
}

// ---------------------------------------------------------------------------
// Elementwise kernels.
// ---------------------------------------------------------------------------
__global__ void k_pack(const float* __restrict__ la, const int32_t* __restrict__ cc,
                       uint16_t* __restrict__ x, int64_t npix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  const float c = log1pf((float)cc[i]);
  const float r = log1pf(la[3 * i]), g = log1pf(la[3 * i + 1]), b = log1pf(la[3 * i + 2]);
  *reinterpret_cast<uint2*>(x + 4 * i) =
      make_uint2(f2bf(r) | (f2bf(g) << 16), f2bf(b) | (f2bf(c) << 16));
}

// Bilinear x4 source row/column: half-pixel centres, clamped to the image.
__device__ __forceinline__ void bl_axis(int X, int n, int& i0, int& i1, float& f) {
  float s = (float)X * 0.25f - 0.375f;       // (X + 1/2) / 4 - 1/2, exact
  s = s < 0.f ? 0.f : s;
  int i = (int)s;
  f = s - (float)i;
  i0 = i < n - 1 ? i : n - 1;
  i1 = i + 1 < n - 1 ? i + 1 : n - 1;
}

__global__ __launch_bounds__(kThreads) void k_head(
    const float* __restrict__ conv6, const float* __restrict__ L_low, float* __restrict__ rgb,
    float* __restrict__ L_full, const float* __restrict__ target, float* __restrict__ loss_sum,
    uint16_t* __restrict__ dconv6, int n, int h, int w, float grad_scale) {
  const int W = 4 * w, H = 4 * h;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n * H * W;
  float sq = 0.f;
  if (i < total) {
    const int X = (int)(i % W), Y = (int)((i / W) % H), img = (int)(i / ((int64_t)W * H));
    int y0, y1, x0, x1;
    float fy, fx;
    bl_axis(Y, h, y0, y1, fy);
    bl_axis(X, w, x0, x1, fx);
    const size_t base = (size_t)img * h * w;
    const float* p00 = L_low + 3 * (base + (size_t)y0 * w + x0);
    const float* p01 = L_low + 3 * (base + (size_t)y0 * w + x1);
    const float* p10 = L_low + 3 * (base + (size_t)y1 * w + x0);
    const float* p11 = L_low + 3 * (base + (size_t)y1 * w + x1);
    const size_t lp = base + (size_t)(Y >> 2) * w + (X >> 2);
    const int sub = 4 * (Y & 3) + (X & 3);
    for (int c = 0; c < 3; ++c) {
      const float top = p00[c] * (1.f - fx) + p01[c] * fx;
      const float bot = p10[c] * (1.f - fx) + p11[c] * fx;
      float L = conv6[lp * 48 + 16 * c + sub] + (top * (1.f - fy) + bot * fy);
      const bool pos = L > 0.f;
      if (L < 0.f) L = 0.f;          // optical depth is never negative; NaN stays NaN
      const float I = -expm1f(-L);
      rgb[3 * i + c] = I;
      if (L_full) L_full[3 * i + c] = L;
      if (target) {
        const float d = I - target[3 * i + c];
        sq += d * d;
        if (dconv6)
          dconv6[lp * 48 + 16 * c + sub] = (uint16_t)f2bf(pos ? grad_scale * d * expf(-L) : 0.f);
      }
    }
  }
  if (loss_sum) {
    __shared__ float red[kThreads / 64];
    sq = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int k = 0; k < kThreads / 64; ++k) s += red[k];
      atomicAdd(loss_sum, s);
    }
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_to_bf16(const float* __restrict__ s, uint16_t* __restrict__ d, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) d[i] = (uint16_t)f2bf(s[i]);
}

// Block partial sums of the consistency metric: added to sum_sq with one
// atomic per block, or (partials != NULL) stored per block for the
// fixed-order reduction of k_sum_partials.
__global__ __launch_bounds__(kThreads) void k_consistency(const float* __restrict__ L_full,
                                                          const float* __restrict__ L_low,
                                                          float* __restrict__ sum_sq,
                                                          float* __restrict__ partials, int n,
                                                          int h, int w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n * h * w;
  float sq = 0.f;
  if (i < total) {
    const int x = (int)(i % w), y = (int)((i / w) % h), img = (int)(i / ((int64_t)w * h));
    const int W = 4 * w;
    const size_t r1 = ((size_t)img * 4 * h + 4 * y + 1) * W, r2 = r1 + W;
    const int X1 = 4 * x + 1, X2 = X1 + 1;
    for (int c = 0; c < 3; ++c) {
      const float Lc = 0.25f * ((L_full[3 * (r1 + X1) + c] + L_full[3 * (r1 + X2) + c]) +
                                (L_full[3 * (r2 + X1) + c] + L_full[3 * (r2 + X2) + c]));
      const float d = expm1f(-L_low[3 * i + c]) - expm1f(-Lc);
      sq += d * d;
    }
  }
  __shared__ float red[kThreads / 64];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int k = 0; k < kThreads / 64; ++k) s += red[k];
    if (partials)
      partials[blockIdx.x] = s;
    else
      atomicAdd(sum_sq, s);
  }
}

// One workgroup per region of q x q low-resolution pixels (a region of 4q
// full-resolution pixels per side): the consistency terms of its pixels
// summed in a fixed order, the region's RMS compared with theta.
__global__ __launch_bounds__(kThreads) void k_region_check(const float* __restrict__ L_full,
                                                           const float* __restrict__ L_low,
                                                           int h, int w, int q, int rgx,
                                                           float theta, float* __restrict__ metric,
                                                           uint8_t* __restrict__ mask,
                                                           int32_t* __restrict__ n_marked) {
  const int rx = (int)blockIdx.x % rgx, ry = (int)blockIdx.x / rgx;
  const int x0 = rx * q, y0 = ry * q;
  const int qx = min(q, w - x0), qy = min(q, h - y0);
  const int W = 4 * w;
  float sq = 0.f;
  for (int k = threadIdx.x; k < qx * qy; k += kThreads) {
    const int x = x0 + k % qx, y = y0 + k / qx;
    const size_t r1 = (size_t)(4 * y + 1) * W, r2 = r1 + W;
    const int X1 = 4 * x + 1, X2 = X1 + 1;
    const size_t i = (size_t)y * w + x;
    for (int c = 0; c < 3; ++c) {
      const float Lc = 0.25f * ((L_full[3 * (r1 + X1) + c] + L_full[3 * (r1 + X2) + c]) +
                                (L_full[3 * (r2 + X1) + c] + L_full[3 * (r2 + X2) + c]));
      const float d = expm1f(-L_low[3 * i + c]) - expm1f(-Lc);
      sq += d * d;
    }
  }
  __shared__ float red[kThreads / 64];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int k = 0; k < kThreads / 64; ++k) s += red[k];
    const float m = sqrtf(s / (float)(3 * qx * qy));
    if (metric) metric[blockIdx.x] = m;
    const bool mark = !(m <= theta);   // NaN marks the region
    mask[blockIdx.x] = mark ? 1 : 0;
    if (mark) atomicAdd(n_marked, 1);
  }
}

// One workgroup: out[0] = sum of partials[0 .. count) in a fixed order.
__global__ __launch_bounds__(kThreads) void k_sum_partials(const float* __restrict__ partials,
                                                           int count, float* __restrict__ out) {
  __shared__ float red[kThreads];
  float s = 0.f;
  for (int i = threadIdx.x; i < count; i += kThreads) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = kThreads / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
bool dims_ok(int32_t n, int32_t h, int32_t w) {
  return n >= 1 && h >= 1 && w >= 1 && (int64_t)n * h * w < (int64_t(1) << 31);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

splotch_status launched() {
  return hipGetLastError() == hipSuccess ? SPLOTCH_OK : SPLOTCH_ERR_HIP;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

template <int KC, int CB>
void launch_fwd(const void* x, const void* w, const float* bias, const void* mask, void* y,
                int n, int h, int wd, int cin, int cout, int relu, int out_f32,
                hipStream_t st) {
  const int tx = (wd + FT - 1) / FT, ty = (h + FT - 1) / FT;
  hipLaunchKernelGGL((k_conv_fwd<KC, CB>), dim3((unsigned)((int64_t)n * tx * ty)),
                     dim3(kThreads), 0, st, static_cast<const uint16_t*>(x),
                     static_cast<const uint16_t*>(w), bias, static_cast<const uint16_t*>(mask),
                     y, h, wd, cin, cout, relu, out_f32, tx, ty);
}

template <int NB, int CB>
void launch_bwd_w(const void* x, const void* dy, const void* mask, float* dw, float* db, int n,
                  int h, int wd, int cin, int cout, hipStream_t st) {
  const int tx = (wd + WW - 1) / WW, ty = (h + WH - 1) / WH;
  const int64_t tiles = (int64_t)n * tx * ty;
  const int grid = (int)(tiles < 512 ? tiles : 512);
  hipLaunchKernelGGL((k_conv_bwd_w<NB, CB>), dim3(grid), dim3(kThreads), 0, st,
                     static_cast<const uint16_t*>(x), static_cast<const uint16_t*>(dy),
                     static_cast<const uint16_t*>(mask), dw, db, h, wd, cin, cout, tx, ty,
                     (int)tiles);
}

}  // namespace

// the C ABI is the library's only exported interface (built with
// -fvisibility=hidden)
#pragma GCC visibility push(default)
extern "C" {

splotch_status splotch_nn_conv3x3_fwd(const void* x, const void* w, const float* bias,
                                      const void* mask, void* y, int32_t n, int32_t h, int32_t w_,
                                      int32_t cin, int32_t cout, int32_t relu, int32_t out_f32,
                                      void* hip_stream) {
  if (!x || !w || !y || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if (cin < 1 || cin > 64 || (cout != 16 && cout != 32 && cout != 48) || (cin > 32 && cout > 32))
    return SPLOTCH_ERR_UNSUPPORTED;
  if (cin % 8 == 0 && (!aligned16(x) || !aligned16(w) || (mask && !aligned16(mask))))
    return SPLOTCH_ERR_INVALID_ARG;
  if (!aligned16(y)) return SPLOTCH_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int kc = cin > 32 ? 2 : 1, cb = cout / 16;
#define SPL_FWD(K, C)                                                                 \
  if (kc == K && cb == C) {                                                           \
    launch_fwd<K, C>(x, w, bias, mask, y, n, h, w_, cin, cout, relu, out_f32, st);  \
    return launched();                                                                \
  }
  SPL_FWD(1, 1) SPL_FWD(1, 2) SPL_FWD(1, 3) SPL_FWD(2, 1) SPL_FWD(2, 2)
#undef SPL_FWD
  return SPLOTCH_ERR_UNSUPPORTED;
}

splotch_status splotch_nn_flip_weights(const void* w, void* wt, int32_t cin, int32_t cout,
                                       void* hip_stream) {
  if (!w || !wt || cin < 1 || cout < 1 || cin > 4096 || cout > 4096)
    return SPLOTCH_ERR_INVALID_ARG;
  const int64_t total = (int64_t)cin * cout * 9;
  hipLaunchKernelGGL(k_flip, dim3(blocks_for(total)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), static_cast<const uint16_t*>(w),
                     static_cast<uint16_t*>(wt), cin, cout);
  return launched();
}

splotch_status splotch_nn_conv3x3_bwd_weight(const void* x, const void* dy, const void* mask,
                                             float* dw, float* db, int32_t n, int32_t h,
                                             int32_t w_, int32_t cin, int32_t cout,
                                             void* hip_stream) {
  if (!x || !dy || !dw || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if (cin < 1 || cin > 32 || (cout != 16 && cout != 32 && cout != 48))
    return SPLOTCH_ERR_UNSUPPORTED;
  if (!aligned16(dy) || (mask && !aligned16(mask)) || (cin % 8 == 0 && !aligned16(x)))
    return SPLOTCH_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nb = cin > 16 ? 2 : 1, cb = cout / 16;
#define SPL_BWD(N, C)                                                            \
  if (nb == N && cb == C) {                                                      \
    launch_bwd_w<N, C>(x, dy, mask, dw, db, n, h, w_, cin, cout, st);            \
    return launched();                                                           \
  }
  SPL_BWD(1, 1) SPL_BWD(1, 2) SPL_BWD(1, 3) SPL_BWD(2, 1) SPL_BWD(2, 2) SPL_BWD(2, 3)
#undef SPL_BWD
  return SPLOTCH_ERR_UNSUPPORTED;
}

splotch_status splotch_nn_pack_input(const float* log_accum, const int32_t* center_count,
                                     void* x, int32_t n, int32_t h, int32_t w_,
                                     void* hip_stream) {
  if (!log_accum || !center_count || !x || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(x) & 7u) != 0) return SPLOTCH_ERR_INVALID_ARG;
  const int64_t npix = (int64_t)n * h * w_;
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(npix)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), log_accum, center_count,
                     static_cast<uint16_t*>(x), npix);
  return launched();
}

splotch_status splotch_nn_head(const float* conv6, const float* L_low, float* rgb, float* L_full,
                               const float* target, float* loss_sum, void* dconv6, int32_t n,
                               int32_t h, int32_t w_, void* hip_stream) {
  if (!conv6 || !L_low || !rgb || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if ((int64_t)n * h * w_ * 16 >= (int64_t(1) << 31)) return SPLOTCH_ERR_INVALID_ARG;
  if ((loss_sum || dconv6) && !target) return SPLOTCH_ERR_INVALID_ARG;
  const int64_t total = (int64_t)n * h * w_ * 16;
  const float grad_scale = (float)(2.0 / (3.0 * (double)total));
  hipLaunchKernelGGL(k_head, dim3(blocks_for(total)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), conv6, L_low, rgb, L_full, target,
                     loss_sum, static_cast<uint16_t*>(dconv6), n, h, w_, grad_scale);
  return launched();
}

splotch_status splotch_nn_adam(float* p, const float* g, float* m, float* v, int64_t count,
                               float lr, float beta1, float beta2, float eps, int32_t step,
                               void* hip_stream) {
  if (!p || !g || !m || !v || count < 0 || step < 1) return SPLOTCH_ERR_INVALID_ARG;
  if (count == 0) return SPLOTCH_OK;
  const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(count)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), p, g, m, v, count, lr, beta1, beta2,
                     eps, c1, c2);
  return launched();
}

splotch_status splotch_nn_to_bf16(const float* src, void* dst, int64_t count, void* hip_stream) {
  if (!src || !dst || count < 0) return SPLOTCH_ERR_INVALID_ARG;
  if (count == 0) return SPLOTCH_OK;
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(count)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), src, static_cast<uint16_t*>(dst),
                     count);
  return launched();
}

splotch_status splotch_nn_consistency(const float* L_full, const float* L_low, float* sum_sq,
                                      int32_t n, int32_t h, int32_t w_, void* hip_stream) {
  if (!L_full || !L_low || !sum_sq || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if ((int64_t)n * h * w_ * 16 >= (int64_t(1) << 31)) return SPLOTCH_ERR_INVALID_ARG;
  const int64_t total = (int64_t)n * h * w_;
  hipLaunchKernelGGL(k_consistency, dim3(blocks_for(total)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), L_full, L_low, sum_sq, nullptr, n, h,
                     w_);
  return launched();
}


splotch_status splotch_nn_region_check(const float* L_full, const float* L_low, int32_t h,
                                      int32_t w_, int32_t region, float theta, float* metric,
                                      uint8_t* mask, int32_t* n_marked, void* hip_stream) {
  if (!L_full || !L_low || !mask || !n_marked || !dims_ok(1, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  if ((int64_t)h * w_ * 16 >= (int64_t(1) << 31)) return SPLOTCH_ERR_INVALID_ARG;
  if (region < 4 || region % 4 != 0 || region > 4096) return SPLOTCH_ERR_INVALID_ARG;
  const int q = region / 4;
  const int rgx = (w_ + q - 1) / q, rgy = (h + q - 1) / q;
  hipLaunchKernelGGL(k_region_check, dim3((unsigned)(rgx * rgy)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), L_full, L_low, h, w_, q, rgx, theta,
                     metric, mask, n_marked);
  return launched();
}

// Layer shapes of the upscaler network: (cin, cout, relu).
static const int kNet[6][3] = {{4, 32, 1}, {32, 32, 1}, {32, 32, 1}, {32, 32, 1}, {32, 32, 1},
                               {32, 48, 0}};

static size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

splotch_status splotch_nn_upscale_workspace_size(int32_t n, int32_t h, int32_t w_,
                                                 size_t* bytes) {
  if (!bytes || !dims_ok(n, h, w_)) return SPLOTCH_ERR_INVALID_ARG;
  const size_t px = (size_t)n * h * w_;
  *bytes = up256(px * 4 * 2) + 2 * up256(px * 32 * 2) + up256(px * 48 * 4) +
           up256(blocks_for((int64_t)px) * sizeof(float));
  return SPLOTCH_OK;
}

splotch_status splotch_nn_upscale(const splotch_nn_weights* wts, const float* log_accum,
                                  const int32_t* center_count, int32_t n, int32_t h, int32_t w_,
                                  float* rgb, float* L_full, float* check_sum_sq, void* ws,
                                  size_t ws_bytes, void* hip_stream) {
  if (!wts || !log_accum || !center_count || !rgb || !ws || !dims_ok(n, h, w_))
    return SPLOTCH_ERR_INVALID_ARG;
  if ((int64_t)n * h * w_ * 16 >= (int64_t(1) << 31)) return SPLOTCH_ERR_INVALID_ARG;
  if (check_sum_sq && !L_full) return SPLOTCH_ERR_INVALID_ARG;
  for (int k = 0; k < 6; ++k)
    if (!wts->w[k] || !wts->b[k] || !aligned16(wts->w[k])) return SPLOTCH_ERR_INVALID_ARG;
  if (!aligned16(ws)) return SPLOTCH_ERR_INVALID_ARG;
  size_t need = 0;
  splotch_nn_upscale_workspace_size(n, h, w_, &need);
  if (ws_bytes < need) return SPLOTCH_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t px = (size_t)n * h * w_;
  char* p = static_cast<char*>(ws);
  uint16_t* x = reinterpret_cast<uint16_t*>(p);
  p += up256(px * 4 * 2);
  uint16_t* a0 = reinterpret_cast<uint16_t*>(p);
  p += up256(px * 32 * 2);
  uint16_t* a1 = reinterpret_cast<uint16_t*>(p);
  p += up256(px * 32 * 2);
  float* c6 = reinterpret_cast<float*>(p);
  p += up256(px * 48 * 4);
  float* partials = reinterpret_cast<float*>(p);

  splotch_status rc = splotch_nn_pack_input(log_accum, center_count, x, n, h, w_, hip_stream);
  if (rc != SPLOTCH_OK) return rc;
  const void* in = x;
  for (int k = 0; k < 6; ++k) {
    void* out = k == 5 ? static_cast<void*>(c6) : static_cast<void*>(k % 2 ? a1 : a0);
    rc = splotch_nn_conv3x3_fwd(in, wts->w[k], wts->b[k], nullptr, out, n, h, w_, kNet[k][0],
                                kNet[k][1], kNet[k][2], k == 5, hip_stream);
    if (rc != SPLOTCH_OK) return rc;
    in = out;
  }
  rc = splotch_nn_head(c6, log_accum, rgb, L_full, nullptr, nullptr, nullptr, n, h, w_,
                       hip_stream);
  if (rc != SPLOTCH_OK || !check_sum_sq) return rc;
  // the metric decides the fallback, so it is summed in a fixed order
  const unsigned nb = blocks_for((int64_t)px);
  hipLaunchKernelGGL(k_consistency, dim3(nb), dim3(kThreads), 0, st, L_full, log_accum, nullptr,
                     partials, n, h, w_);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, st, partials, (int)nb,
                     check_sum_sq);
  return launched();
}

}  // extern "C"
#pragma GCC visibility pop
