// net_kernels.hip -- learned warm start: inference and training kernels (BF16 storage, FP32
// accumulation; the 32 -> 32 convolutions on the matrix cores).  Definitions in net.hpp.
//
// Activation layout: per sample a (G+2) x (G+2) pixel grid (the G x G coefficient grid plus a zero
// halo ring, so 3x3 taps need no bounds tests) followed by 32 slack pixels, 32 channels per pixel
// (64 bytes, channel fastest).  Pixel (y, x) of the coefficient grid, -1 <= y, x <= G, sits at
// q = (y + 1)(G + 2) + x + 1.  Kernels write interior pixels only; the halo stays zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "net.hpp"

namespace pmg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// parameter offsets in the flat layout: weights [cout][cin][3][3] then bias [cout], per layer
constexpr int kW0 = 0, kB0 = 864, kW1 = 896, kB1 = 10112, kW2 = 10144, kB2 = 19360, kW3 = 19392, kB3 = 19680;
static_assert(kB3 + 1 == kNetParams, "parameter layout");
// weight-gradient partial-sum records per workgroup
constexpr int kP0 = 9 * 3 * 32 + 32;   // [t][ci][co], then bias
constexpr int kP1 = 9 * 32 * 32 + 32;  // [t][co][ci], then bias
constexpr int kP3 = 9 * 32 + 1;        // [t][ci], then bias
constexpr int kPartBlocks = 256;       // workgroups of the weight-gradient kernels

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline float bfround(float f) { return bf2f(f2bf(f)); }
__device__ inline bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }

__host__ __device__ inline int64_t sample_stride(int G) { return (int64_t)(G + 2) * (G + 2) + 32; }

template <int NT>
__device__ double net_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------------------------

// layer 0 (3 -> 32, vector ALUs): one pixel per thread; inputs rounded to BF16 on read
__global__ void __launch_bounds__(256) net_conv_in(const float* __restrict__ x, const float* __restrict__ w0,
                                                   const float* __restrict__ b0, uint16_t* __restrict__ a0, int nb,
                                                   int G) {
  __shared__ float w[864 + 32];
  for (int i = threadIdx.x; i < 864; i += 256) w[i] = w0[i];
  if (threadIdx.x < 32) w[864 + threadIdx.x] = b0[threadIdx.x];
  __syncthreads();
  const int P = G + 2;
  const int64_t SS = sample_stride(G), tot = (int64_t)nb * G * G;
  for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < tot; pix += (int64_t)gridDim.x * 256) {
    const int n = (int)(pix / (G * G)), r = (int)(pix % (G * G)), yy = r / G, xx = r % G;
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = w[864 + c];
    for (int t = 0; t < 9; ++t) {
      const int Y = yy + t / 3 - 1, X = xx + t % 3 - 1;
      const bool ok = Y >= 0 && Y < G && X >= 0 && X < G;
      for (int ci = 0; ci < 3; ++ci) {
        const float v = ok ? bfround(x[(((int64_t)n * 3 + ci) * G + Y) * G + X]) : 0.f;
        const float* wr = w + (t * 3 + ci) * 32;
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] += v * wr[c];
      }
    }
    uint32_t pk[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
      pk[c] = (uint32_t)f2bf(fmaxf(acc[2 * c], 0.f)) | ((uint32_t)f2bf(fmaxf(acc[2 * c + 1], 0.f)) << 16);
    uint4* dst = (uint4*)(a0 + ((int64_t)n * SS + (int64_t)(yy + 1) * P + xx + 1) * 32);
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c] = make_uint4(pk[4 * c], pk[4 * c + 1], pk[4 * c + 2], pk[4 * c + 3]);
  }
}

// 32 -> 32 convolution on the matrix cores.  A wave computes a tile of 16 consecutive pixels of
// one row times 32 output channels: per tap one 16x16x32 product per 16 output channels, with
// K = the 32 input channels.  Operand layout of v_mfma_f32_16x16x32_bf16 (64 lanes): A[m][k] in
// lane m + 16 (k / 8), B[k][n] in lane n + 16 (k / 8), each lane 8 consecutive k; D[m][n] in lane
// n + 16 (m / 4), element m % 4.  wk is [tap][n][k] (k fastest) so a B fragment is 16 bytes.
// MODE 0: forward, out = bf16(relu(acc + bias)).  MODE 1: input gradient, wk holds the flipped
// transposed weights, out = bf16(acc * [layer input > 0]) with the layer input in `mask`.
template <int MODE>
__global__ void __launch_bounds__(256) net_conv32(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wk,
                                                  const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                                  uint16_t* __restrict__ out, int nb, int G) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m16 = lane & 15, kq = lane >> 4;
  const int P = G + 2;
  const int64_t SS = sample_stride(G);
  const int xt = (G + 15) / 16;
  const int64_t ntiles = (int64_t)nb * G * xt;
  bf16x8 bw[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) bw[t][h] = *(const bf16x8*)(wk + ((t * 32 + h * 16 + m16) * 32 + 8 * kq));
  float bv0 = 0.f, bv1 = 0.f;
  if (MODE == 0) {
    bv0 = bias[m16];
    bv1 = bias[16 + m16];
  }
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int n = (int)(tile / ((int64_t)G * xt));
    const int rem = (int)(tile % ((int64_t)G * xt));
    const int yy = rem / xt, x0 = (rem % xt) * 16;
    const uint16_t* base = in + (int64_t)n * SS * 32;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      // padded row yy + dy + 1 <= G + 1; column x0 + m16 + dx + 1 <= G + 16: within the sample's
      // pixels plus slack (lanes past the row end compute values that are not stored)
      const int q = (yy + t / 3) * P + x0 + m16 + t % 3;
      const bf16x8 a = *(const bf16x8*)(base + (int64_t)q * 32 + 8 * kq);
      acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t][0], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t][1], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * kq + i;
      if (xx >= G) continue;
      const int64_t o = ((int64_t)n * SS + (int64_t)(yy + 1) * P + xx + 1) * 32;
      float v0 = acc0[i], v1 = acc1[i];
      if (MODE == 0) {
        v0 = fmaxf(v0 + bv0, 0.f);
        v1 = fmaxf(v1 + bv1, 0.f);
      } else {
        v0 = bf_pos(mask[o + m16]) ? v0 : 0.f;
        v1 = bf_pos(mask[o + 16 + m16]) ? v1 : 0.f;
      }
      out[o + m16] = f2bf(v0);
      out[o + 16 + m16] = f2bf(v1);
    }
  }
}

// layer 3 (32 -> 1, vector ALUs): y = b3 + sum over taps and channels, FP32 output
__global__ void __launch_bounds__(256) net_conv_out(const uint16_t* __restrict__ a2, const float* __restrict__ w3,
                                                    const float* __restrict__ b3, float* __restrict__ y, int nb,
                                                    int G) {
  __shared__ float w[288];
  for (int i = threadIdx.x; i < 288; i += 256) w[i] = w3[i];
  __syncthreads();
  const int P = G + 2;
  const int64_t SS = sample_stride(G), tot = (int64_t)nb * G * G;
  const float bb = b3[0];
  for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < tot; pix += (int64_t)gridDim.x * 256) {
    const int n = (int)(pix / (G * G)), r = (int)(pix % (G * G)), yy = r / G, xx = r % G;
    float acc = bb;
    for (int t = 0; t < 9; ++t) {
      const uint4* src = (const uint4*)(a2 + ((int64_t)n * SS + (int64_t)(yy + t / 3) * P + xx + t % 3) * 32);
      const float* wr = w + t * 32;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint4 v = src[c];
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc += bf2f((uint16_t)(wd[e] & 0xffffu)) * wr[8 * c + 2 * e];
          acc += bf2f((uint16_t)(wd[e] >> 16)) * wr[8 * c + 2 * e + 1];
        }
      }
    }
    y[pix] = acc;
  }
}

// ---------------------------------------------------------------------------------------------
// loss and backward
// ---------------------------------------------------------------------------------------------

// dy = scale (y - t) on the interior of the grid (0 on the Dirichlet ring); per-block sums of (y - t)^2
__global__ void __launch_bounds__(256) net_loss(const float* __restrict__ y, const float* __restrict__ t,
                                                float* __restrict__ dy, double* __restrict__ lpart, int nb, int G,
                                                float scale) {
  __shared__ double red[4];
  const int64_t tot = (int64_t)nb * G * G;
  double s = 0.0;
  for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < tot; pix += (int64_t)gridDim.x * 256) {
    const int r = (int)(pix % (G * G)), yy = r / G, xx = r % G;
    const bool in = yy > 0 && yy < G - 1 && xx > 0 && xx < G - 1;
    const float e = in ? y[pix] - t[pix] : 0.f;
    dy[pix] = scale * e;
    s += (double)e * e;
  }
  s = net_block_sum<256>(s, red);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) net_sum(const double* __restrict__ p, int n, double scale,
                                               double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += p[i];
  s = net_block_sum<256>(s, red);
  if (threadIdx.x == 0) out[0] = s * scale;
}

// gradient into the last hidden layer: g2[q][ci] = bf16([a2 > 0] sum_t dy[q - o_t] w3[t][ci])
__global__ void __launch_bounds__(256) net_out_bwd_data(const float* __restrict__ dy, const float* __restrict__ w3,
                                                        const uint16_t* __restrict__ a2, uint16_t* __restrict__ g2,
                                                        int nb, int G) {
  __shared__ float w[288];
  for (int i = threadIdx.x; i < 288; i += 256) w[i] = w3[i];
  __syncthreads();
  const int P = G + 2;
  const int64_t SS = sample_stride(G), tot = (int64_t)nb * G * G;
  for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < tot; pix += (int64_t)gridDim.x * 256) {
    const int n = (int)(pix / (G * G)), r = (int)(pix % (G * G)), yy = r / G, xx = r % G;
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    for (int t = 0; t < 9; ++t) {
      const int Y = yy - (t / 3 - 1), X = xx - (t % 3 - 1);
      if (Y < 0 || Y >= G || X < 0 || X >= G) continue;
      const float g = dy[((int64_t)n * G + Y) * G + X];
#pragma unroll
      for (int c = 0; c < 32; ++c) acc[c] += g * w[t * 32 + c];
    }
    const int64_t o = ((int64_t)n * SS + (int64_t)(yy + 1) * P + xx + 1) * 32;
    const uint4* ms = (const uint4*)(a2 + o);
    uint4* dst = (uint4*)(g2 + o);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint4 mv = ms[c];
      const uint32_t md[4] = {mv.x, mv.y, mv.z, mv.w};
      uint32_t pk[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float lo = bf_pos((uint16_t)(md[e] & 0xffffu)) ? acc[8 * c + 2 * e] : 0.f;
        const float hi = bf_pos((uint16_t)(md[e] >> 16)) ? acc[8 * c + 2 * e + 1] : 0.f;
        pk[e] = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
      }
      dst[c] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    }
  }
}

// last-layer weight gradient partials: 8 pixel slots x 32 channels per workgroup; thread (slot,
// ci) accumulates dy[q] a2[q + o_t][ci] for the 9 taps (and dy for the bias) over its pixels,
// then the slots are summed in a fixed order
__global__ void __launch_bounds__(256) net_out_wgrad(const float* __restrict__ dy, const uint16_t* __restrict__ a2,
                                                     float* __restrict__ part, int nb, int G) {
  __shared__ float red[8 * kP3];
  const int ci = threadIdx.x & 31, ps = threadIdx.x >> 5;
  const int P = G + 2;
  const int64_t SS = sample_stride(G), tot = (int64_t)nb * G * G;
  float acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = 0.f;
  float bacc = 0.f;
  for (int64_t pix = (int64_t)blockIdx.x * 8 + ps; pix < tot; pix += (int64_t)gridDim.x * 8) {
    const float g = dy[pix];
    const int n = (int)(pix / (G * G)), r = (int)(pix % (G * G)), yy = r / G, xx = r % G;
    const uint16_t* base = a2 + ((int64_t)n * SS + (int64_t)yy * P + xx) * 32 + ci;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] += g * bf2f(base[((t / 3) * P + t % 3) * 32]);
    bacc += g;
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) red[ps * kP3 + t * 32 + ci] = acc[t];
  if (ci == 0) red[ps * kP3 + 288] = bacc;
  __syncthreads();
  for (int j = threadIdx.x; j < kP3; j += 256) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += red[q * kP3 + j];
    part[(int64_t)blockIdx.x * kP3 + j] = s;
  }
}

// 32 -> 32 weight gradient on the matrix cores: dW[t][co][ci] = sum_q g[q][co] a[q + o_t][ci].
// A workgroup (9 waves, wave = tap) takes segments of 32 pixels of one row: it stages g^T
// ([co][px]) and, per tap, the shifted a^T ([ci][px]) in LDS, then each wave issues the four
// 16x16x32 products of its tap with K = the 32 pixels.  Thread c < 32 also sums g[.][c] (bias).
__global__ void __launch_bounds__(576) net_conv32_wgrad(const uint16_t* __restrict__ a, const uint16_t* __restrict__ g,
                                                        float* __restrict__ part, int nb, int G) {
  __shared__ __align__(16) uint16_t gT[32 * 32];
  __shared__ __align__(16) uint16_t aT[9 * 32 * 32];
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  const int m16 = lane & 15, kq = lane >> 4;
  const int P = G + 2;
  const int64_t SS = sample_stride(G);
  const int xs = (G + 31) / 32;
  const int64_t nseg = (int64_t)nb * G * xs;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) acc[i][k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const int n = (int)(seg / ((int64_t)G * xs));
    const int rem = (int)(seg % ((int64_t)G * xs));
    const int yy = rem / xs, x0 = (rem % xs) * 32;
    const int64_t sb = (int64_t)n * SS;
    // 128 chunks of g (32 px x 4 groups of 8 channels), then 3 rows x 34 columns x 4 groups of a
    for (int c = threadIdx.x; c < 128 + 3 * 34 * 4; c += 576) {
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (c < 128) {
        const int px = c >> 2, c8 = (c & 3) * 8;
        if (x0 + px < G) v = *(const uint4*)(g + (sb + (int64_t)(yy + 1) * P + x0 + px + 1) * 32 + c8);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          gT[(c8 + 2 * e) * 32 + px] = (uint16_t)(wd[e] & 0xffffu);
          gT[(c8 + 2 * e + 1) * 32 + px] = (uint16_t)(wd[e] >> 16);
        }
      } else {
        const int c2 = c - 128, dyi = c2 / 136, r2 = c2 % 136, xi = r2 >> 2, c8 = (r2 & 3) * 8;
        const int col = x0 + xi;  // padded column of pixel x = x0 + xi - 1; padded row yy + dyi
        if (col <= P - 1) v = *(const uint4*)(a + (sb + (int64_t)(yy + dyi) * P + col) * 32 + c8);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi) {
          const int px = xi - dxi;
          if (px < 0 || px >= 32) continue;
          uint16_t* dst = aT + (dyi * 3 + dxi) * 1024 + px;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            dst[(c8 + 2 * e) * 32] = (uint16_t)(wd[e] & 0xffffu);
            dst[(c8 + 2 * e + 1) * 32] = (uint16_t)(wd[e] >> 16);
          }
        }
      }
    }
    __syncthreads();
    bf16x8 A[2], B[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      A[h] = *(const bf16x8*)(gT + (h * 16 + m16) * 32 + 8 * kq);
      B[h] = *(const bf16x8*)(aT + t * 1024 + (h * 16 + m16) * 32 + 8 * kq);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) acc[i][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], B[k], acc[i][k], 0, 0, 0);
    if (threadIdx.x < 32)
      for (int px = 0; px < 32; ++px) bacc += bf2f(gT[threadIdx.x * 32 + px]);
    __syncthreads();
  }
  float* pr = part + (int64_t)blockIdx.x * kP1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = i * 16 + 4 * kq + e, ci = k * 16 + m16;
        pr[(t * 32 + co) * 32 + ci] = acc[i][k][e];
      }
  if (threadIdx.x < 32) pr[9216 + threadIdx.x] = bacc;
}

// first-layer weight gradient partials on the matrix cores: dW0[t][ci][co] = sum_q g0[q][co]
// x[ci][q + o_t] as a 32 x 32 product per 32-pixel row segment (K = pixels, M = co, N = the 27
// (tap, ci) pairs padded to 32), the inputs rounded to BF16 as in the forward pass.  One wave per
// workgroup stages g0^T ([co][px]) and the shifted inputs ([tap ci][px]) in LDS; lane c < 32 also
// sums g0[.][c] (the bias).
constexpr int kInBlocks = 1024;
__global__ void __launch_bounds__(64) net_in_wgrad(const float* __restrict__ x, const uint16_t* __restrict__ g0,
                                                   float* __restrict__ part, int nb, int G) {
  __shared__ __align__(16) uint16_t gT[32 * 32];
  __shared__ __align__(16) uint16_t xT[32 * 32];
  const int lane = threadIdx.x, m16 = lane & 15, kq = lane >> 4;
  const int P = G + 2;
  const int64_t SS = sample_stride(G);
  const int xs = (G + 31) / 32;
  const int64_t nseg = (int64_t)nb * G * xs;
  for (int e = lane; e < 5 * 32; e += 64) xT[27 * 32 + e] = 0;  // padding rows 27..31
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) acc[i][k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const int n = (int)(seg / ((int64_t)G * xs));
    const int rem = (int)(seg % ((int64_t)G * xs));
    const int yy = rem / xs, x0 = (rem % xs) * 32;
    __syncthreads();  // the previous segment's fragments have been read
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // g0: 32 px x 4 groups of 8 channels
      const int c = lane + 64 * h, px = c >> 2, c8 = (c & 3) * 8;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (x0 + px < G) v = *(const uint4*)(g0 + ((int64_t)n * SS + (int64_t)(yy + 1) * P + x0 + px + 1) * 32 + c8);
      const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        gT[(c8 + 2 * e) * 32 + px] = (uint16_t)(wd[e] & 0xffffu);
        gT[(c8 + 2 * e + 1) * 32 + px] = (uint16_t)(wd[e] >> 16);
      }
    }
    for (int e = lane; e < 27 * 32; e += 64) {  // inputs: row tci = 3 t + ci, column px
      const int tci = e >> 5, px = e & 31, t = tci / 3, ci = tci - 3 * t;
      const int Y = yy + t / 3 - 1, X = x0 + px + t % 3 - 1;
      float v = 0.f;
      if (x0 + px < G && Y >= 0 && Y < G && X >= 0 && X < G) v = x[(((int64_t)n * 3 + ci) * G + Y) * G + X];
      xT[e] = f2bf(v);
    }
    __syncthreads();
    bf16x8 A[2], B[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      A[h] = *(const bf16x8*)(gT + (h * 16 + m16) * 32 + 8 * kq);
      B[h] = *(const bf16x8*)(xT + (h * 16 + m16) * 32 + 8 * kq);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) acc[i][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], B[k], acc[i][k], 0, 0, 0);
    if (lane < 32)
      for (int px = 0; px < 32; ++px) bacc += bf2f(gT[lane * 32 + px]);
  }
  float* pr = part + (int64_t)blockIdx.x * kP0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = i * 16 + 4 * kq + e, tci = k * 16 + m16;
        if (tci < 27) pr[tci * 32 + co] = acc[i][k][e];
      }
  if (lane < 32) pr[864 + lane] = bacc;
}

// sum the partial records of every layer into the flat gradient (fixed order: deterministic)
// (64 parameters per workgroup, 4 lanes per parameter summing every 4th record, combined in LDS)
__global__ void __launch_bounds__(256) net_reduce(const float* __restrict__ p0, const float* __restrict__ p1,
                                                  const float* __restrict__ p2, const float* __restrict__ p3,
                                                  int nblk, int nblk0, float* __restrict__ grad) {
  __shared__ float red[256];
  const int i = blockIdx.x * 64 + (threadIdx.x >> 2), q = threadIdx.x & 3;
  float s = 0.f;
  if (i < kNetParams) {
    const float* src;
    int stride, off;
    if (i < kB0) {  // W0[co][ci][t]
      const int co = i / 27, ci = (i / 9) % 3, t = i % 9;
      src = p0, stride = kP0, off = (t * 3 + ci) * 32 + co;
    } else if (i < kW1) {
      src = p0, stride = kP0, off = 864 + (i - kB0);
    } else if (i < kB1 || (i >= kW2 && i < kB2)) {  // W1, W2 [co][ci][t]
      const int l = i < kB1 ? i - kW1 : i - kW2;
      const int co = l / 288, ci = (l / 9) % 32, t = l % 9;
      src = i < kB1 ? p1 : p2, stride = kP1, off = (t * 32 + co) * 32 + ci;
    } else if (i < kW2 || (i >= kB2 && i < kW3)) {
      src = i < kW2 ? p1 : p2, stride = kP1, off = 9216 + (i < kW2 ? i - kB1 : i - kB2);
    } else if (i < kB3) {  // W3[0][ci][t]
      const int l = i - kW3, ci = l / 9, t = l % 9;
      src = p3, stride = kP3, off = t * 32 + ci;
    } else {
      src = p3, stride = kP3, off = 288;
    }
    const int nbk = src == p0 ? nblk0 : nblk;
    for (int b = q; b < nbk; b += 4) s += src[(int64_t)b * stride + off];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (q == 0 && i < kNetParams)
    grad[i] = (red[threadIdx.x] + red[threadIdx.x + 1]) + (red[threadIdx.x + 2] + red[threadIdx.x + 3]);
}

// Adam (Kingma and Ba), bias-corrected: c1 = 1 - 0.9^step, c2 = 1 - 0.999^step
__global__ void __launch_bounds__(256) net_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                                const float* __restrict__ g, float lr, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kNetParams) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// flat FP32 parameters -> kernel layouts (BF16 or BF16-rounded floats)
__global__ void __launch_bounds__(256) net_convert(const float* __restrict__ th, float* __restrict__ w0,
                                                   uint16_t* __restrict__ wf1, uint16_t* __restrict__ wb1,
                                                   uint16_t* __restrict__ wf2, uint16_t* __restrict__ wb2,
                                                   float* __restrict__ w3) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 864) {
    const int co = i / 27, ci = (i / 9) % 3, t = i % 9;
    w0[(t * 3 + ci) * 32 + co] = bfround(th[kW0 + i]);
  }
  if (i < 9216) {
    const int co = i / 288, ci = (i / 9) % 32, t = i % 9;
    const uint16_t h1 = f2bf(th[kW1 + i]), h2 = f2bf(th[kW2 + i]);
    wf1[(t * 32 + co) * 32 + ci] = h1;
    wb1[((8 - t) * 32 + ci) * 32 + co] = h1;
    wf2[(t * 32 + co) * 32 + ci] = h2;
    wb2[((8 - t) * 32 + ci) * 32 + co] = h2;
  }
  if (i < 288) {
    const int ci = i / 9, t = i % 9;
    w3[t * 32 + ci] = bfround(th[kW3 + i]);
  }
}

// zero the halo ring and slack pixels of every sample for grid size G (all other pixels are
// written before they are read): 4 (G + 1) ring pixels + 32 slack pixels, 32 channels each
__global__ void __launch_bounds__(256) net_halo_zero(uint16_t* __restrict__ a, int nb, int G) {
  const int P = G + 2, ring = 4 * (G + 1), per = ring + 32;
  const int64_t SS = sample_stride(G), tot = (int64_t)nb * per * 4;  // 4 16-byte chunks per pixel
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
    const int n = (int)(t / (per * 4)), rem = (int)(t % (per * 4)), px = rem >> 2, c = rem & 3;
    int64_t q;
    if (px < P) q = px;                                    // top row
    else if (px < 2 * P) q = (int64_t)(P - 1) * P + (px - P);  // bottom row
    else if (px < ring) {                                  // left / right columns of rows 1 .. P-2
      const int k = px - 2 * P, row = 1 + (k >> 1);
      q = (int64_t)row * P + ((k & 1) ? P - 1 : 0);
    } else q = (int64_t)P * P + (px - ring);               // slack
    ((uint4*)(a + ((int64_t)n * SS + q) * 32))[c] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// ---------------------------------------------------------------------------------------------
// samples from trajectories
// ---------------------------------------------------------------------------------------------

// explicit increment of interior dof (iy, ix): e = (w F - kappa dt K u) / m, the previous point's residual
// b - A u in the step's equation divided by the lumped mass; K u by the Kronecker bands
__device__ __forceinline__ double net_explicit(const NetSrc& S, const double* u, double w, int iy, int ix) {
  const int nin = S.nin, bw = S.bw, p = S.p;
  double ku = 0.0;
  for (int a = 0; a < bw; ++a) {
    const int jy = iy + a - p;
    if (jy < 0 || jy >= nin) continue;
    const double my = S.My[iy * bw + a], ky = S.Ky[iy * bw + a];
    const double* ur = u + (int64_t)jy * nin;
    double sk = 0.0, sm = 0.0;
    for (int c = 0; c < bw; ++c) {
      const int jx = ix + c - p;
      if (jx < 0 || jx >= nin) continue;
      sk += S.Kx[ix * bw + c] * ur[jx];
      sm += S.Mx2[ix * bw + c] * ur[jx];
    }
    ku += my * sk + ky * sm;
  }
  return (w * S.F[iy * nin + ix] - S.kdt * ku) * S.ilx[ix] * S.ily[iy];
}

// Samples are packed by two kernels over (sample, chunk) workgroups, kPackChunks per sample:
// net_pack_e forms the explicit increment e of its chunk of interior dofs into ebuf and the chunk's sums
// of u^2 and e^2; net_pack_planes adds a sample's chunk sums in a fixed order and writes the planes
// u/s_u, e/s_e, ln(kappa dt n^2)/4 and (optionally) the target (u_{k+1} - u_k)/s_e, with s_u = rms(u),
// s_e = rms(e) over the interior (1 if zero); s receives s_e, the scale of the output.
constexpr int kPackChunks = 16;

__global__ void __launch_bounds__(256) net_pack_e(const NetSrc* __restrict__ src, const NetPick* __restrict__ pick,
                                                  int kbase, int64_t estride, double* __restrict__ ebuf,
                                                  double* __restrict__ epart) {
  __shared__ double red[4];
  const int j = blockIdx.x, c = blockIdx.y;
  const NetSrc S = src[pick[j].src];
  const int k = pick[j].k + kbase, nin = S.nin, nd = nin * nin;
  const double* u = S.U + (int64_t)k * nd;
  const double w = S.scale ? S.scale[k + 1] : S.dt;
  const int per = (nd + kPackChunks - 1) / kPackChunks, i0 = c * per, i1 = min(nd, i0 + per);
  double su = 0.0, se = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const double e = net_explicit(S, u, w, i / nin, i % nin);
    ebuf[(int64_t)j * estride + i] = e;
    su += u[i] * u[i];
    se += e * e;
  }
  su = net_block_sum<256>(su, red);
  se = net_block_sum<256>(se, red);
  if (threadIdx.x == 0) {
    epart[((int64_t)j * kPackChunks + c) * 2] = su;
    epart[((int64_t)j * kPackChunks + c) * 2 + 1] = se;
  }
}

__global__ void __launch_bounds__(256) net_pack_planes(const NetSrc* __restrict__ src,
                                                       const NetPick* __restrict__ pick, int kbase, int G,
                                                       int64_t estride, const double* __restrict__ ebuf,
                                                       const double* __restrict__ epart, float* __restrict__ x,
                                                       float* __restrict__ t, double* __restrict__ s,
                                                       int with_target) {
  const int j = blockIdx.x, c = blockIdx.y;
  const NetSrc S = src[pick[j].src];
  const int k = pick[j].k + kbase, nin = S.nin, nd = nin * nin;
  const double* u = S.U + (int64_t)k * nd;
  double su = 0.0, se = 0.0;
  for (int q = 0; q < kPackChunks; ++q) {
    su += epart[((int64_t)j * kPackChunks + q) * 2];
    se += epart[((int64_t)j * kPackChunks + q) * 2 + 1];
  }
  double s_u = sqrt(su / nd), s_e = sqrt(se / nd);
  if (s_u == 0.0) s_u = 1.0;
  if (s_e == 0.0) s_e = 1.0;
  float* x0 = x + (int64_t)j * 3 * G * G;
  float* x1 = x0 + G * G;
  float* x2 = x1 + G * G;
  const float lnc = (float)S.lnc;
  const double* un = S.U + (int64_t)(k + 1) * nd;
  const double* e = ebuf + (int64_t)j * estride;
  const int per = (G * G + kPackChunks - 1) / kPackChunks, p0 = c * per, p1 = min(G * G, p0 + per);
  for (int pix = p0 + threadIdx.x; pix < p1; pix += 256) {
    const int yy = pix / G, xx = pix % G;
    const bool in = yy > 0 && yy < G - 1 && xx > 0 && xx < G - 1;
    const int i = (yy - 1) * nin + (xx - 1);
    float v0 = 0.f, v1 = 0.f, tv = 0.f;
    if (in) {
      v0 = (float)(u[i] / s_u);
      v1 = (float)(e[i] / s_e);
      if (with_target) tv = (float)((un[i] - u[i]) / s_e);
    }
    x0[pix] = v0;
    x1[pix] = v1;
    x2[pix] = lnc;
    if (with_target) t[(int64_t)j * G * G + pix] = tv;
  }
  if (c == 0 && threadIdx.x == 0) s[j] = s_e;
}

// guesses: U_out[k + 1] = U[k] + s y on the interior
__global__ void __launch_bounds__(256) net_unpack(const NetSrc* __restrict__ src, const NetPick* __restrict__ pick,
                                                  int kbase, int G, const float* __restrict__ y,
                                                  const double* __restrict__ s) {
  const int j = blockIdx.x;
  const NetSrc S = src[pick[j].src];
  const int k = pick[j].k + kbase, nin = S.nin, nd = nin * nin;
  const double* u = S.U + (int64_t)k * nd;
  double* o = S.Uout + (int64_t)(k + 1) * nd;
  const double sj = s[j];
  for (int i = threadIdx.x; i < nd; i += 256) {
    const int iy = i / nin, ix = i % nin;
    o[i] = u[i] + sj * (double)y[((int64_t)j * G + iy + 1) * G + ix + 1];
  }
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------

static int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

template <class T>
hipError_t NetState::alloc(T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, sizeof(T) * (n ? n : 1));
  if (e != hipSuccess) return e;
  allocs_.push_back(q);
  *p = (T*)q;
  return hipMemset(q, 0, sizeof(T) * (n ? n : 1));
}

NetState::~NetState() {
  if (device_ >= 0) {
    (void)hipSetDevice(device_);
    (void)hipDeviceSynchronize();
  }
  for (void* p : allocs_) (void)hipFree(p);
}

hipError_t NetState::init(int device) {
  device_ = device;
  hipError_t e;
  if ((e = alloc(&theta_, kNetParams)) || (e = alloc(&m_, kNetParams)) || (e = alloc(&v_, kNetParams)) ||
      (e = alloc(&grad_, kNetParams)) || (e = alloc(&w0_, 864)) || (e = alloc(&w3_, 288)) ||
      (e = alloc(&wf1_, 9216)) || (e = alloc(&wb1_, 9216)) || (e = alloc(&wf2_, 9216)) || (e = alloc(&wb2_, 9216)) ||
      (e = alloc(&loss_, 1)) || (e = alloc(&lpart_, 1024)))
    return e;
  part_cap_ = (int64_t)kInBlocks * kP0 + (int64_t)kPartBlocks * (2 * kP1 + kP3);
  return alloc(&part_, (size_t)part_cap_);
}

hipError_t NetState::convert(hipStream_t st) {
  hipLaunchKernelGGL(net_convert, dim3(36), dim3(256), 0, st, theta_, w0_, wf1_, wb1_, wf2_, wb2_, w3_);
  return hipGetLastError();
}

hipError_t NetState::load(const float* theta_host) {
  hipError_t e;
  if ((e = hipMemcpy(theta_, theta_host, sizeof(float) * kNetParams, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemset(m_, 0, sizeof(float) * kNetParams)) != hipSuccess) return e;
  if ((e = hipMemset(v_, 0, sizeof(float) * kNetParams)) != hipSuccess) return e;
  steps = 0;
  if ((e = convert(nullptr)) != hipSuccess) return e;
  loaded = true;
  return hipDeviceSynchronize();
}

hipError_t NetState::save(float* theta_host) const {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  return hipMemcpy(theta_host, theta_, sizeof(float) * kNetParams, hipMemcpyDeviceToHost);
}

hipError_t NetState::reserve(int nb, int G) {
  if (nb <= nb_cap_ && G <= G_cap_) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  for (void* p : sized_) {
    for (size_t i = 0; i < allocs_.size(); ++i)
      if (allocs_[i] == p) {
        allocs_.erase(allocs_.begin() + i);
        break;
      }
    (void)hipFree(p);
  }
  sized_.clear();
  nb_cap_ = nb > nb_cap_ ? nb : nb_cap_;
  G_cap_ = G > G_cap_ ? G : G_cap_;
  const size_t act = (size_t)nb_cap_ * sample_stride(G_cap_) * 32, pl = (size_t)nb_cap_ * G_cap_ * G_cap_;
  uint16_t** acts[5] = {&a0_, &a1_, &a2_, &ga_, &gb_};
  for (uint16_t** p : acts) {
    if ((e = alloc(p, act)) != hipSuccess) return e;
    sized_.push_back(*p);
  }
  if ((e = alloc(&x_, 3 * pl)) || (e = alloc(&t_, pl)) || (e = alloc(&y_, pl)) || (e = alloc(&dy_, pl)) ||
      (e = alloc(&s_, (size_t)nb_cap_)) || (e = alloc(&ebuf_, pl)) ||
      (e = alloc(&epart_, (size_t)nb_cap_ * kPackChunks * 2)))
    return e;
  for (void* p : {(void*)x_, (void*)t_, (void*)y_, (void*)dy_, (void*)s_, (void*)ebuf_, (void*)epart_})
    sized_.push_back(p);
  G_last_ = -1;
  return hipSuccess;
}

// the halo ring of the activation grids must be zero: when the grid size changes, positions that
// held interior pixels may become halo, so the new layout's halo and slack pixels are cleared (a
// kernel, so this may also sit in a captured graph)
hipError_t NetState::layout(int G, hipStream_t st) {
  if (G == G_last_) return hipSuccess;
  const int64_t work = (int64_t)nb_cap_ * (4 * (G + 1) + 32) * 4;
  const int grid = grid_for(work, 256, 4096);
  for (uint16_t* p : {a0_, a1_, a2_, ga_, gb_}) hipLaunchKernelGGL(net_halo_zero, dim3(grid), dim3(256), 0, st, p, nb_cap_, G);
  G_last_ = G;
  return hipGetLastError();
}

hipError_t NetState::run_forward(int nb, int G, const float* x, float* y, hipStream_t st) {
  hipError_t e;
  if ((e = layout(G, st)) != hipSuccess) return e;
  const int64_t pix = (int64_t)nb * G * G;
  const int gp = grid_for(pix, 256, 8192);
  const int64_t tiles = (int64_t)nb * G * ((G + 15) / 16);
  const int gt = grid_for(tiles, 4, 4096);
  hipLaunchKernelGGL(net_conv_in, dim3(gp), dim3(256), 0, st, x, w0_, theta_ + kB0, a0_, nb, G);
  hipLaunchKernelGGL(net_conv32<0>, dim3(gt), dim3(256), 0, st, a0_, wf1_, theta_ + kB1, nullptr, a1_, nb, G);
  hipLaunchKernelGGL(net_conv32<0>, dim3(gt), dim3(256), 0, st, a1_, wf2_, theta_ + kB2, nullptr, a2_, nb, G);
  hipLaunchKernelGGL(net_conv_out, dim3(gp), dim3(256), 0, st, a2_, w3_, theta_ + kB3, y, nb, G);
  return hipGetLastError();
}

hipError_t NetState::run_backward(int nb, int G, const float* x, const float* t, hipStream_t st) {
  const int64_t pix = (int64_t)nb * G * G;
  const int gp = grid_for(pix, 256, 8192);
  const int gl = grid_for(pix, 256, 1024);
  const int64_t tiles = (int64_t)nb * G * ((G + 15) / 16);
  const int gt = grid_for(tiles, 4, 4096);
  const int nseg = (int)((int64_t)nb * G * ((G + 31) / 32) < kPartBlocks ? (int64_t)nb * G * ((G + 31) / 32)
                                                                         : kPartBlocks);
  float* p0 = part_;
  float* p1 = p0 + (int64_t)kInBlocks * kP0;
  float* p2 = p1 + (int64_t)kPartBlocks * kP1;
  float* p3 = p2 + (int64_t)kPartBlocks * kP1;
  const double cnt = (double)nb * (G - 2) * (G - 2);
  hipLaunchKernelGGL(net_loss, dim3(gl), dim3(256), 0, st, y_, t, dy_, lpart_, nb, G, (float)(2.0 / cnt));
  hipLaunchKernelGGL(net_sum, dim3(1), dim3(256), 0, st, lpart_, gl, 1.0 / cnt, loss_);
  // layer 3
  hipLaunchKernelGGL(net_out_wgrad, dim3(kPartBlocks), dim3(256), 0, st, dy_, a2_, p3, nb, G);
  hipLaunchKernelGGL(net_out_bwd_data, dim3(gp), dim3(256), 0, st, dy_, w3_, a2_, ga_, nb, G);
  // layer 2: weights from (a1, ga), input gradient ga -> gb masked by a1
  if (nseg < kPartBlocks) {
    hipError_t e = hipMemsetAsync(p1, 0, sizeof(float) * (size_t)kPartBlocks * kP1 * 2, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(net_conv32_wgrad, dim3(nseg), dim3(576), 0, st, a1_, ga_, p2, nb, G);
  hipLaunchKernelGGL(net_conv32<1>, dim3(gt), dim3(256), 0, st, ga_, wb2_, nullptr, a1_, gb_, nb, G);
  // layer 1: weights from (a0, gb), input gradient gb -> ga masked by a0
  hipLaunchKernelGGL(net_conv32_wgrad, dim3(nseg), dim3(576), 0, st, a0_, gb_, p1, nb, G);
  hipLaunchKernelGGL(net_conv32<1>, dim3(gt), dim3(256), 0, st, gb_, wb1_, nullptr, a0_, ga_, nb, G);
  // layer 0
  hipLaunchKernelGGL(net_in_wgrad, dim3(kInBlocks), dim3(64), 0, st, x, ga_, p0, nb, G);
  hipLaunchKernelGGL(net_reduce, dim3((kNetParams + 63) / 64), dim3(256), 0, st, p0, p1, p2, p3, kPartBlocks,
                     kInBlocks, grad_);
  return hipGetLastError();
}

hipError_t NetState::forward(int nb, int G, const float* x, float* y, hipStream_t st) {
  hipError_t e = reserve(nb, G);
  if (e != hipSuccess) return e;
  return run_forward(nb, G, x, y, st);
}

hipError_t NetState::backward(int nb, int G, const float* x, const float* t, hipStream_t st) {
  hipError_t e = reserve(nb, G);
  if (e != hipSuccess) return e;
  if ((e = run_forward(nb, G, x, y_, st)) != hipSuccess) return e;
  return run_backward(nb, G, x, t, st);
}

hipError_t NetState::loss_and_grad(int nb, int G, const float* x, const float* t, float* grad_host,
                                   double* loss_host, hipStream_t st) {
  hipError_t e = backward(nb, G, x, t, st);
  if (e != hipSuccess) return e;
  if (grad_host &&
      (e = hipMemcpyAsync(grad_host, grad_, sizeof(float) * kNetParams, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if (loss_host && (e = hipMemcpyAsync(loss_host, loss_, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  return hipStreamSynchronize(st);
}

hipError_t NetState::adam_step(float lr, hipStream_t st) {
  ++steps;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)steps)), c2 = (float)(1.0 - std::pow(0.999, (double)steps));
  hipLaunchKernelGGL(net_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, st, theta_, m_, v_, grad_, lr, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return convert(st);
}

hipError_t NetState::pack(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G, bool with_target,
                          hipStream_t st) {
  hipError_t e = reserve(nb, G);
  if (e != hipSuccess) return e;
  const int64_t estride = (int64_t)G_cap_ * G_cap_;
  hipLaunchKernelGGL(net_pack_e, dim3(nb, kPackChunks), dim3(256), 0, st, src_dev, pick_dev, kbase, estride, ebuf_,
                     epart_);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(net_pack_planes, dim3(nb, kPackChunks), dim3(256), 0, st, src_dev, pick_dev, kbase, G, estride,
                     ebuf_, epart_, x_, t_, s_, with_target ? 1 : 0);
  return hipGetLastError();
}

hipError_t NetState::unpack(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G,
                            hipStream_t st) {
  hipLaunchKernelGGL(net_unpack, dim3(nb), dim3(256), 0, st, src_dev, pick_dev, kbase, G, y_, s_);
  return hipGetLastError();
}

hipError_t NetState::predict(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G,
                             hipStream_t st) {
  hipError_t e;
  if ((e = pack(src_dev, pick_dev, kbase, nb, G, false, st)) != hipSuccess) return e;
  if ((e = run_forward(nb, G, x_, y_, st)) != hipSuccess) return e;
  return unpack(src_dev, pick_dev, kbase, nb, G, st);
}

hipError_t NetState::train_packed(const NetSrc* src_dev, const NetPick* pick_dev, int nb, int G, float lr,
                                  hipStream_t st) {
  hipError_t e;
  if ((e = pack(src_dev, pick_dev, 0, nb, G, true, st)) != hipSuccess) return e;
  if ((e = run_forward(nb, G, x_, y_, st)) != hipSuccess) return e;
  if ((e = run_backward(nb, G, x_, t_, st)) != hipSuccess) return e;
  return adam_step(lr, st);
}

hipError_t NetState::read_loss(double* loss_host, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(loss_host, loss_, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace pmg
