// unet.hip -- the warm-start network: a 3-level 3D U-Net (16/32/64 channels,
// 3x3x3 convolutions) that maps (normalised field, signal-vertex mask) to a
// proposed change g0 - f, with its forward and backward passes and an Adam
// step.  Convolutions are implicit GEMMs on BF16 MFMA tiles with FP32
// accumulation; activations are BF16, parameters and gradients FP32.  Where
// the channel count allows it, the forward convolutions use gfx950's
// double-K BF16 MFMAs (32x32x16, 16x16x32): each lane supplies eight
// consecutive channels, half the instructions of the 8- and 16-deep forms.
//
// Layout: a volume of D x H x W voxels is stored channels-last, voxel
// v = x + W * (y + H * z), element (v, c) at v * C + c.  A convolution's
// weights are [27][Cout][Cin] with tap t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1),
// followed by Cout biases.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"
#include "unet.h"

namespace ts {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// eight BF16 values (16 bytes, aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

inline unsigned nblk(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

// FP32 -> BF16 with round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ---------------------------------------------------------------------------
// Convolution, forward form: Y[v][co] = bias[co] + sum_t sum_ci
// X[v + off_t][ci] * Wt[t][co][ci], zero outside the volume.  One wave computes
// a tile of 32 voxels x 32 output channels with the 32x32x8 BF16 MFMA: lane l
// supplies row l % 32 of A (voxel) and column l % 32 of B (output channel) at
// k = 4 * (l / 32) .. + 3; accumulator i of lane l is row
// 8 * (i / 4) + 4 * (l / 32) + i % 4, column l % 32.  Cin is a multiple of 8.
// Outputs: Yf (FP32, before the activation) and Yb (BF16, after the optional
// ReLU); either may be null.  The backward data pass uses the same kernel with
// flipped, transposed weights.  kWide (Cin a multiple of 16): the 32x32x16
// MFMA, lane l supplying channels 8 * (l / 32) .. + 7 of a 16-channel step
// (A and B take the same channels in every lane, so the sum over k is the
// convolution's sum over channels whatever order the hardware gives k).
// ---------------------------------------------------------------------------
template <bool kWide>
__global__ void __launch_bounds__(256)
k_conv_fwd(const uint16_t* __restrict__ X, int D, int H, int W, int Cin,
           const uint16_t* __restrict__ Wt, const float* __restrict__ bias, int Cout, int relu,
           float* __restrict__ Yf, uint16_t* __restrict__ Yb) {
  const int64_t V = int64_t(D) * H * W;
  const int64_t tiles_v = (V + 31) / 32;
  const int tiles_c = (Cout + 31) / 32;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (wave >= tiles_v * tiles_c) return;  // whole waves exit together
  const int lane = threadIdx.x & 63, m = lane & 31, half = lane >> 5;
  const int64_t tv = wave / tiles_c;
  const int tc = int(wave - tv * tiles_c);
  const int64_t v = tv * 32 + m;
  const int co = tc * 32 + m;
  int x = 0, y = 0, z = 0;
  if (v < V) {
    x = int(v % W);
    y = int((v / W) % H);
    z = int(v / (int64_t(W) * H));
  }
  f32x16 acc = {};
  for (int t = 0; t < 27; ++t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const bool inside = v < V && x + dx >= 0 && x + dx < W && y + dy >= 0 && y + dy < H &&
                        z + dz >= 0 && z + dz < D;
    const int64_t nb = v + dx + int64_t(W) * (dy + int64_t(H) * dz);
    const int sub = kWide ? 8 * half : 4 * half;
    const uint16_t* xa = X + nb * Cin + sub;
    const uint16_t* wb = Wt + (int64_t(t) * Cout + co) * Cin + sub;
    if constexpr (kWide) {
      for (int c0 = 0; c0 < Cin; c0 += 16) {
        bf16x8 a = {}, b = {};
        if (inside) a = load8(xa + c0);
        if (co < Cout) b = load8(wb + c0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int c0 = 0; c0 < Cin; c0 += 8) {
        bf16x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
        if (inside) a = *reinterpret_cast<const bf16x4*>(xa + c0);
        if (co < Cout) b = *reinterpret_cast<const bf16x4*>(wb + c0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
      }
    }
  }
  const int cc = tc * 32 + m;
  if (cc >= Cout) return;
  const float bc = bias ? bias[cc] : 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t vv = tv * 32 + 8 * (i / 4) + 4 * half + (i % 4);
    if (vv >= V) continue;
    float val = acc[i] + bc;
    if (Yf) Yf[vv * Cout + cc] = val;
    if (relu) val = fmaxf(val, 0.0f);
    if (Yb) Yb[vv * Cout + cc] = to_bf16(val);
  }
}

// The same convolution for Cout = 16 and Cin a multiple of 16, where a 32 x 32
// tile would leave half of every instruction idle: one wave computes 64
// voxels x 16 output channels with four 16x16x16 BF16 MFMAs per k step, which
// share the step's weights.  Lane l supplies row l % 16 of A (voxel) and column
// l % 16 of B (output channel) at k = 4 * (l / 16) .. + 3; accumulator i of
// lane l is row 4 * (l / 16) + i, column l % 16.  kWide (Cin a multiple of
// 32): the 16x16x32 MFMA, lane l supplying channels 8 * (l / 16) .. + 7 of a
// 32-channel step.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <bool kWide>
__global__ void __launch_bounds__(256)
k_conv_fwd16(const uint16_t* __restrict__ X, int D, int H, int W, int Cin,
             const uint16_t* __restrict__ Wt, const float* __restrict__ bias, int relu,
             float* __restrict__ Yf, uint16_t* __restrict__ Yb) {
  const int64_t V = int64_t(D) * H * W;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (wave >= (V + 63) / 64) return;  // whole waves exit together
  const int lane = threadIdx.x & 63, m = lane & 15, q = lane >> 4;
  int64_t v[4];
  int x[4], y[4], z[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    v[s] = wave * 64 + 16 * s + m;
    x[s] = y[s] = z[s] = 0;
    if (v[s] < V) {
      x[s] = int(v[s] % W);
      y[s] = int((v[s] / W) % H);
      z[s] = int(v[s] / (int64_t(W) * H));
    }
  }
  f32x4 acc[4] = {};
  for (int t = 0; t < 27; ++t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const uint16_t* xa[4];
    bool inside[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      inside[s] = v[s] < V && x[s] + dx >= 0 && x[s] + dx < W && y[s] + dy >= 0 &&
                  y[s] + dy < H && z[s] + dz >= 0 && z[s] + dz < D;
      xa[s] = X + (v[s] + dx + int64_t(W) * (dy + int64_t(H) * dz)) * Cin + (kWide ? 8 : 4) * q;
    }
    const uint16_t* wb = Wt + (int64_t(t) * 16 + m) * Cin + (kWide ? 8 : 4) * q;
    if constexpr (kWide) {
      for (int c0 = 0; c0 < Cin; c0 += 32) {
        const bf16x8 b = load8(wb + c0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          bf16x8 a = {};
          if (inside[s]) a = load8(xa[s] + c0);
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[s], 0, 0, 0);
        }
      }
    } else {
      for (int c0 = 0; c0 < Cin; c0 += 16) {
        const bf16x4 b = *reinterpret_cast<const bf16x4*>(wb + c0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          bf16x4 a = {0, 0, 0, 0};
          if (inside[s]) a = *reinterpret_cast<const bf16x4*>(xa[s] + c0);
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s], 0, 0, 0);
        }
      }
    }
  }
  const float bc = bias ? bias[m] : 0.0f;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t vv = wave * 64 + 16 * s + 4 * q + i;
      if (vv >= V) continue;
      float val = acc[s][i] + bc;
      if (Yf) Yf[vv * 16 + m] = val;
      if (relu) val = fmaxf(val, 0.0f);
      if (Yb) Yb[vv * 16 + m] = to_bf16(val);
    }
}

// Backward weights: dW[t][co][ci] += sum_v dY[v][co] * X[v + off_t][ci] over
// a chunk of voxels.  One wave: tap t, 32 output x 32 input channels, with the
// voxels as the MFMA's k; partial sums are added to dW atomically.
constexpr int kWgradChunk = 2048;
__global__ void __launch_bounds__(256)
k_conv_wgrad(const uint16_t* __restrict__ dY, const uint16_t* __restrict__ X, int D, int H, int W,
             int Cin, int Cout, float* __restrict__ dW) {
  const int64_t V = int64_t(D) * H * W;
  const int tco = (Cout + 31) / 32, tci = (Cin + 31) / 32;
  const int64_t chunks = (V + kWgradChunk - 1) / kWgradChunk;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (wave >= chunks * 27 * tco * tci) return;
  const int lane = threadIdx.x & 63, m = lane & 31, half = lane >> 5;
  int64_t r = wave;
  const int ti = int(r % tci);
  r /= tci;
  const int to = int(r % tco);
  r /= tco;
  const int t = int(r % 27);
  const int64_t chunk = r / 27;
  const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
  const int co = to * 32 + m, ci = ti * 32 + m;
  const int64_t v0 = chunk * kWgradChunk, v1 = v0 + kWgradChunk < V ? v0 + kWgradChunk : V;
  f32x16 acc = {};
  if (W & 3) {  // rows not a multiple of 4 voxels: coordinates per voxel
    for (int64_t k0 = v0; k0 < v1; k0 += 8) {
      bf16x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t v = k0 + 4 * half + i;
        if (v >= v1) continue;
        if (co < Cout) a[i] = short(dY[v * Cout + co]);
        const int x = int(v % W), y = int((v / W) % H), z = int(v / (int64_t(W) * H));
        const bool inside = x + dx >= 0 && x + dx < W && y + dy >= 0 && y + dy < H &&
                            z + dz >= 0 && z + dz < D;
        if (inside && ci < Cin) {
          const int64_t nb = v + dx + int64_t(W) * (dy + int64_t(H) * dz);
          b[i] = short(X[nb * Cin + ci]);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
  } else if ((W & 7) == 0) {
    // The 32x32x16 MFMA: the lane's eight voxels vb .. vb + 7 (vb = k0 + 8 *
    // half, a multiple of 8) share a row because W is a multiple of 8; their
    // coordinates advance by 16 voxels per step without divisions.
    const int64_t s0 = v0 + 8 * half;
    int xb = int(s0 % W), yb = int((s0 / W) % H), zb = int(s0 / (int64_t(W) * H));
    const int64_t shift = dx + int64_t(W) * (dy + int64_t(H) * dz);
    for (int64_t k0 = v0; k0 < v1; k0 += 16) {
      uint16_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0}, b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const int64_t vb = k0 + 8 * half;
      if (vb < v1) {
        const bool row_ok = yb + dy >= 0 && yb + dy < H && zb + dz >= 0 && zb + dz < D;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int64_t v = vb + i;
          if (v >= v1) continue;
          if (co < Cout) a[i] = dY[v * Cout + co];
          if (row_ok && ci < Cin && xb + i + dx >= 0 && xb + i + dx < W)
            b[i] = X[(v + shift) * Cin + ci];
        }
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
      xb += 16;
      while (xb >= W) {
        xb -= W;
        if (++yb == H) {
          yb = 0;
          ++zb;
        }
      }
    }
  } else {
    // The lane's four voxels vb .. vb + 3 (vb = k0 + 4 * half, a multiple of 4)
    // share a row because W is a multiple of 4; their coordinates advance by 8
    // voxels per step without divisions.
    const int64_t s0 = v0 + 4 * half;
    int xb = int(s0 % W), yb = int((s0 / W) % H), zb = int(s0 / (int64_t(W) * H));
    const int64_t shift = dx + int64_t(W) * (dy + int64_t(H) * dz);
    for (int64_t k0 = v0; k0 < v1; k0 += 8) {
      bf16x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
      const int64_t vb = k0 + 4 * half;
      if (vb < v1) {
        const bool row_ok = yb + dy >= 0 && yb + dy < H && zb + dz >= 0 && zb + dz < D;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t v = vb + i;
          if (co < Cout) a[i] = short(dY[v * Cout + co]);
          if (row_ok && ci < Cin && xb + i + dx >= 0 && xb + i + dx < W)
            b[i] = short(X[(v + shift) * Cin + ci]);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
      xb += 8;
      while (xb >= W) {
        xb -= W;
        if (++yb == H) {
          yb = 0;
          ++zb;
        }
      }
    }
  }
  if (ci >= Cin) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = to * 32 + 8 * (i / 4) + 4 * half + (i % 4);
    if (row < Cout) atomicAdd(&dW[(int64_t(t) * Cout + row) * Cin + ci], acc[i]);
  }
}

// Wf[t][ci][co] = W[26 - t][co][ci] in BF16: the backward data pass as a
// forward convolution of dY.
__global__ void k_flip_weights(const float* __restrict__ Wsrc, int Cin, int Cout,
                               uint16_t* __restrict__ Wf) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(27) * Cin * Cout) return;
  const int co = int(i % Cout);
  const int ci = int((i / Cout) % Cin);
  const int t = int(i / (int64_t(Cout) * Cin));
  Wf[i] = to_bf16(Wsrc[(int64_t(26 - t) * Cout + co) * Cin + ci]);
}

__global__ void k_to_bf16(const float* __restrict__ a, int64_t n, uint16_t* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = to_bf16(a[i]);
}

// Input [V][2] FP32 -> [V][8] BF16, channels 2..7 zero.
__global__ void k_pack_input(const float* __restrict__ in, int64_t V, uint16_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * 8) return;
  const int c = int(i & 7);
  out[i] = c < 2 ? to_bf16(in[(i >> 3) * 2 + c]) : uint16_t(0);
}

// dPre = dOut * (pre > 0) (FP32 and BF16); dOut may be the same buffer as dPre.
__global__ void k_relu_bwd(const float* dout, const float* __restrict__ pre, int64_t n,
                           float* dpre, uint16_t* __restrict__ dpre_b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = pre[i] > 0.0f ? dout[i] : 0.0f;
  dpre[i] = g;
  dpre_b[i] = to_bf16(g);
}

// db[c] += sum_v d[v][c]: one block per channel slice of voxels.
__global__ void k_bias_grad(const float* __restrict__ d, int64_t V, int C, float* __restrict__ db) {
  __shared__ float s[256];
  const int c = blockIdx.y;
  float acc = 0.0f;
  for (int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x; v < V; v += int64_t(gridDim.x) * 256)
    acc += d[v * C + c];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&db[c], s[0]);
}

// 2x2x2 average pooling (BF16) of a D x H x W volume (even sizes).
__global__ void k_pool_fwd(const uint16_t* __restrict__ X, int D, int H, int W, int C,
                           uint16_t* __restrict__ Y) {
  const int d = D / 2, h = H / 2, w = W / 2;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(d) * h * w * C) return;
  const int c = int(i % C);
  const int64_t p = i / C;
  const int x = int(p % w), y = int((p / w) % h), z = int(p / (int64_t(w) * h));
  float s = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const int64_t v = (2 * x + (k & 1)) + int64_t(W) * ((2 * y + ((k >> 1) & 1)) +
                                                        int64_t(H) * (2 * z + (k >> 2)));
    s += from_bf16(X[v * C + c]);
  }
  Y[i] = to_bf16(s * 0.125f);
}

// dX[child] += dY[parent] / 8 (FP32), over the fine volume.
__global__ void k_pool_bwd(const float* __restrict__ dY, int D, int H, int W, int C,
                           float* __restrict__ dX) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(D) * H * W * C) return;
  const int c = int(i % C);
  const int64_t v = i / C;
  const int x = int(v % W), y = int((v / W) % H), z = int(v / (int64_t(W) * H));
  const int64_t p = (x / 2) + int64_t(W / 2) * ((y / 2) + int64_t(H / 2) * (z / 2));
  dX[i] += dY[p * C + c] * 0.125f;
}

// Nearest 2x upsampling of the coarse volume (d x h x w, C channels) into
// channels [0, C) of the fine volume's concatenation (Ctot channels), and the
// skip tensor into channels [C, Ctot).
__global__ void k_up_concat(const uint16_t* __restrict__ coarse, int C, const uint16_t* __restrict__ skip,
                            int Cs, int D, int H, int W, uint16_t* __restrict__ out) {
  const int Ct = C + Cs;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(D) * H * W * Ct) return;
  const int c = int(i % Ct);
  const int64_t v = i / Ct;
  if (c < C) {
    const int x = int(v % W), y = int((v / W) % H), z = int(v / (int64_t(W) * H));
    const int64_t p = (x / 2) + int64_t(W / 2) * ((y / 2) + int64_t(H / 2) * (z / 2));
    out[i] = coarse[p * C + c];
  } else {
    out[i] = skip[v * Cs + (c - C)];
  }
}

// Backward of k_up_concat: dCoarse[p][c] = sum of the 8 children's gradient of
// channel c; dSkip[v][c] += the gradient of channel C + c.
__global__ void k_up_concat_bwd_coarse(const float* __restrict__ dcat, int C, int Cs, int D, int H,
                                       int W, float* __restrict__ dcoarse) {
  const int Ct = C + Cs, d = D / 2, h = H / 2, w = W / 2;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(d) * h * w * C) return;
  const int c = int(i % C);
  const int64_t p = i / C;
  const int x = int(p % w), y = int((p / w) % h), z = int(p / (int64_t(w) * h));
  float s = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const int64_t v = (2 * x + (k & 1)) + int64_t(W) * ((2 * y + ((k >> 1) & 1)) +
                                                        int64_t(H) * (2 * z + (k >> 2)));
    s += dcat[v * Ct + c];
  }
  dcoarse[i] = s;
}
__global__ void k_up_concat_bwd_skip(const float* __restrict__ dcat, int C, int Cs, int64_t V,
                                     float* __restrict__ dskip) {
  const int Ct = C + Cs;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * Cs) return;
  const int c = int(i % Cs);
  const int64_t v = i / Cs;
  dskip[i] += dcat[v * Ct + C + c];
}

// Head: out[v] = b + sum_c w[c] * h[v][c] (16 channels).
__global__ void k_head_fwd(const uint16_t* __restrict__ h, int64_t V, const float* __restrict__ wb,
                           float* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= V) return;
  float s = wb[16];
  for (int c = 0; c < 16; ++c) s += wb[c] * from_bf16(h[v * 16 + c]);
  out[v] = s;
}

// Mean squared error L = mean (out - target)^2 and dOut = 2 (out - target) / V;
// the sum of squares is accumulated in *sse.
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ target, int64_t V,
                      float* __restrict__ dout, float* __restrict__ sse) {
  __shared__ float s[256];
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float e = 0.0f;
  if (v < V) {
    e = out[v] - target[v];
    dout[v] = 2.0f * e / float(V);
  }
  s[threadIdx.x] = e * e;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(sse, s[0]);
}

// Head backward: dh[v][c] = dout[v] * w[c]; dw[c] += sum_v dout[v] h[v][c],
// db += sum_v dout[v].
__global__ void k_head_bwd(const uint16_t* __restrict__ h, const float* __restrict__ dout, int64_t V,
                           const float* __restrict__ wb, float* __restrict__ dh,
                           float* __restrict__ dwb) {
  __shared__ float s[17][256];
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const float g = v < V ? dout[v] : 0.0f;
  for (int c = 0; c < 16; ++c) {
    const float hv = v < V ? from_bf16(h[v * 16 + c]) : 0.0f;
    if (v < V) dh[v * 16 + c] = g * wb[c];
    s[c][threadIdx.x] = g * hv;
  }
  s[16][threadIdx.x] = g;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k)
      for (int c = 0; c < 17; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 17) atomicAdd(&dwb[threadIdx.x], s[threadIdx.x][0]);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct ConvSpec {
  int cin, cout;  // cin as stored (the first layer's 2 input channels padded to 8)
  int64_t off;    // offset of the weights in the parameter vector (biases follow)
};

// Level l works on D >> l etc.; enc1a, enc1b, enc2a, enc2b, bot_a, bot_b,
// dec2a, dec2b, dec1a, dec1b, then the head (16 weights + 1 bias).
struct Net {
  ConvSpec conv[10];
  int64_t head = 0, total = 0;
  Net() {
    const int io[10][2] = {{8, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64},
                           {64, 64}, {96, 32}, {32, 32}, {48, 16}, {16, 16}};
    int64_t o = 0;
    for (int i = 0; i < 10; ++i) {
      conv[i] = {io[i][0], io[i][1], o};
      o += int64_t(27) * io[i][0] * io[i][1] + io[i][1];
    }
    head = o;
    total = o + 17;
  }
};

struct Vol {
  int D, H, W;
  int64_t V() const { return int64_t(D) * H * W; }
};

template <class T>
T* buf(ts_ctx* ctx, const std::string& name, int64_t n) {
  return ctx->ws.get<T>("unet." + name, size_t(n > 0 ? n : 1));
}

// Everything the forward pass keeps for the backward pass.
struct Acts {
  uint16_t* in8;
  uint16_t* a[10];   // BF16 outputs of the ten convolutions (after ReLU)
  float* pre[10];    // FP32 pre-activations
  uint16_t* p1;      // pooled enc1b
  uint16_t* p2;      // pooled enc2b
  uint16_t* cat2;    // [up(bot_b), enc2b]
  uint16_t* cat1;    // [up(dec2b), enc1b]
  uint16_t* wb[10];  // BF16 weights
};

void conv_fwd(ts_ctx* ctx, const uint16_t* X, const Vol& vol, int cin, const uint16_t* Wt,
              const float* bias, int cout, bool relu, float* Yf, uint16_t* Yb) {
  if (cout == 16 && cin % 16 == 0) {
    const int64_t waves = (vol.V() + 63) / 64;
    if (cin % 32 == 0)
      k_conv_fwd16<true><<<nblk(waves * 64), 256, 0, ctx->stream>>>(X, vol.D, vol.H, vol.W, cin, Wt,
                                                                     bias, relu ? 1 : 0, Yf, Yb);
    else
      k_conv_fwd16<false><<<nblk(waves * 64), 256, 0, ctx->stream>>>(X, vol.D, vol.H, vol.W, cin, Wt,
                                                                      bias, relu ? 1 : 0, Yf, Yb);
    return;
  }
  const int64_t tiles = ((vol.V() + 31) / 32) * ((cout + 31) / 32);
  if (cin % 16 == 0)
    k_conv_fwd<true><<<nblk(tiles * 64), 256, 0, ctx->stream>>>(X, vol.D, vol.H, vol.W, cin, Wt, bias,
                                                                 cout, relu ? 1 : 0, Yf, Yb);
  else
    k_conv_fwd<false><<<nblk(tiles * 64), 256, 0, ctx->stream>>>(X, vol.D, vol.H, vol.W, cin, Wt,
                                                                  bias, cout, relu ? 1 : 0, Yf, Yb);
}

void forward(ts_ctx* ctx, const Net& N, const float* params, const float* input, const Vol& v0,
             Acts* A, float* out) {
  hipStream_t s = ctx->stream;
  const Vol v1{v0.D / 2, v0.H / 2, v0.W / 2}, v2{v0.D / 4, v0.H / 4, v0.W / 4};
  const Vol lv[10] = {v0, v0, v1, v1, v2, v2, v1, v1, v0, v0};
  for (int i = 0; i < 10; ++i) {
    const ConvSpec& c = N.conv[i];
    const int64_t nw = int64_t(27) * c.cin * c.cout;
    A->wb[i] = buf<uint16_t>(ctx, "wb" + std::to_string(i), nw);
    k_to_bf16<<<nblk(nw), 256, 0, s>>>(params + c.off, nw, A->wb[i]);
    A->a[i] = buf<uint16_t>(ctx, "a" + std::to_string(i), lv[i].V() * c.cout);
    A->pre[i] = buf<float>(ctx, "pre" + std::to_string(i), lv[i].V() * c.cout);
  }
  A->in8 = buf<uint16_t>(ctx, "in8", v0.V() * 8);
  A->p1 = buf<uint16_t>(ctx, "p1", v1.V() * 16);
  A->p2 = buf<uint16_t>(ctx, "p2", v2.V() * 32);
  A->cat2 = buf<uint16_t>(ctx, "cat2", v1.V() * 96);
  A->cat1 = buf<uint16_t>(ctx, "cat1", v0.V() * 48);
  k_pack_input<<<nblk(v0.V() * 8), 256, 0, s>>>(input, v0.V(), A->in8);
  const uint16_t* src[10] = {A->in8, A->a[0], A->p1, A->a[2], A->p2,
                             A->a[4], A->cat2, A->a[6], A->cat1, A->a[8]};
  for (int i = 0; i < 10; ++i) {
    const ConvSpec& c = N.conv[i];
    if (i == 2) k_pool_fwd<<<nblk(v1.V() * 16), 256, 0, s>>>(A->a[1], v0.D, v0.H, v0.W, 16, A->p1);
    if (i == 4) k_pool_fwd<<<nblk(v2.V() * 32), 256, 0, s>>>(A->a[3], v1.D, v1.H, v1.W, 32, A->p2);
    if (i == 6)
      k_up_concat<<<nblk(v1.V() * 96), 256, 0, s>>>(A->a[5], 64, A->a[3], 32, v1.D, v1.H, v1.W,
                                                    A->cat2);
    if (i == 8)
      k_up_concat<<<nblk(v0.V() * 48), 256, 0, s>>>(A->a[7], 32, A->a[1], 16, v0.D, v0.H, v0.W,
                                                    A->cat1);
    conv_fwd(ctx, src[i], lv[i], c.cin, A->wb[i], params + c.off + int64_t(27) * c.cin * c.cout,
             c.cout, true, A->pre[i], A->a[i]);
  }
  k_head_fwd<<<nblk(v0.V()), 256, 0, s>>>(A->a[9], v0.V(), params + N.head, out);
  TS_HIP(hipGetLastError());
}

// Backward of one convolution: dOut (FP32, gradient after the ReLU) ->
// weight and bias gradients, and dX (FP32, overwritten) unless null.
void conv_bwd(ts_ctx* ctx, const Net& N, int i, const Vol& vol, const uint16_t* X,
              const float* params, const Acts& A, float* dout, float* grad, float* dX) {
  hipStream_t s = ctx->stream;
  const ConvSpec& c = N.conv[i];
  const int64_t n = vol.V() * c.cout;
  uint16_t* db = buf<uint16_t>(ctx, "dpre_b", n);
  k_relu_bwd<<<nblk(n), 256, 0, s>>>(dout, A.pre[i], n, dout, db);
  float* gW = grad + c.off;
  float* gb = gW + int64_t(27) * c.cin * c.cout;
  k_bias_grad<<<dim3(64, c.cout), 256, 0, s>>>(dout, vol.V(), c.cout, gb);
  const int64_t chunks = (vol.V() + kWgradChunk - 1) / kWgradChunk;
  const int64_t waves = chunks * 27 * ((c.cout + 31) / 32) * ((c.cin + 31) / 32);
  k_conv_wgrad<<<nblk(waves * 64), 256, 0, s>>>(db, X, vol.D, vol.H, vol.W, c.cin, c.cout, gW);
  if (dX) {
    const int64_t nw = int64_t(27) * c.cin * c.cout;
    uint16_t* wf = buf<uint16_t>(ctx, "wflip", nw);
    k_flip_weights<<<nblk(nw), 256, 0, s>>>(params + c.off, c.cin, c.cout, wf);
    conv_fwd(ctx, db, vol, c.cout, wf, nullptr, c.cin, false, dX, nullptr);
  }
  TS_HIP(hipGetLastError());
}

}  // namespace

int64_t unet_param_count() { return Net().total; }

void unet_forward(ts_ctx* ctx, const float* params, const float* input, int D, int H, int W,
                  float* out) {
  const Net N;
  Acts A;
  forward(ctx, N, params, input, Vol{D, H, W}, &A, out);
}

double unet_backward(ts_ctx* ctx, const float* params, const float* input, const float* target,
                     int D, int H, int W, float* grad) {
  hipStream_t s = ctx->stream;
  const Net N;
  Acts A;
  const Vol v0{D, H, W}, v1{D / 2, H / 2, W / 2}, v2{D / 4, H / 4, W / 4};
  const Vol lv[10] = {v0, v0, v1, v1, v2, v2, v1, v1, v0, v0};
  float* out = buf<float>(ctx, "out", v0.V());
  forward(ctx, N, params, input, v0, &A, out);
  TS_HIP(hipMemsetAsync(grad, 0, size_t(N.total) * 4, s));
  float* dout = buf<float>(ctx, "dout", v0.V());
  float* sse = buf<float>(ctx, "sse", 1);
  TS_HIP(hipMemsetAsync(sse, 0, 4, s));
  k_mse<<<nblk(v0.V()), 256, 0, s>>>(out, target, v0.V(), dout, sse);
  // gradient buffers, one per activation (FP32)
  float* g[10];
  for (int i = 0; i < 10; ++i) g[i] = buf<float>(ctx, "g" + std::to_string(i), lv[i].V() * N.conv[i].cout);
  float* gcat2 = buf<float>(ctx, "gcat2", v1.V() * 96);
  float* gcat1 = buf<float>(ctx, "gcat1", v0.V() * 48);
  float* gp1 = buf<float>(ctx, "gp1", v1.V() * 16);
  float* gp2 = buf<float>(ctx, "gp2", v2.V() * 32);
  k_head_bwd<<<nblk(v0.V()), 256, 0, s>>>(A.a[9], dout, v0.V(), params + N.head, g[9],
                                          grad + N.head);
  // decoder level 1
  conv_bwd(ctx, N, 9, v0, A.a[8], params, A, g[9], grad, g[8]);
  conv_bwd(ctx, N, 8, v0, A.cat1, params, A, g[8], grad, gcat1);
  k_up_concat_bwd_coarse<<<nblk(v1.V() * 32), 256, 0, s>>>(gcat1, 32, 16, v0.D, v0.H, v0.W, g[7]);
  // decoder level 2
  conv_bwd(ctx, N, 7, v1, A.a[6], params, A, g[7], grad, g[6]);
  conv_bwd(ctx, N, 6, v1, A.cat2, params, A, g[6], grad, gcat2);
  k_up_concat_bwd_coarse<<<nblk(v2.V() * 64), 256, 0, s>>>(gcat2, 64, 32, v1.D, v1.H, v1.W, g[5]);
  // bottom
  conv_bwd(ctx, N, 5, v2, A.a[4], params, A, g[5], grad, g[4]);
  conv_bwd(ctx, N, 4, v2, A.p2, params, A, g[4], grad, gp2);
  // encoder level 2: enc2b's gradient = skip part of cat2 + pooled path
  TS_HIP(hipMemsetAsync(g[3], 0, size_t(v1.V()) * 32 * 4, s));
  k_up_concat_bwd_skip<<<nblk(v1.V() * 32), 256, 0, s>>>(gcat2, 64, 32, v1.V(), g[3]);
  k_pool_bwd<<<nblk(v1.V() * 32), 256, 0, s>>>(gp2, v1.D, v1.H, v1.W, 32, g[3]);
  conv_bwd(ctx, N, 3, v1, A.a[2], params, A, g[3], grad, g[2]);
  conv_bwd(ctx, N, 2, v1, A.p1, params, A, g[2], grad, gp1);
  // encoder level 1
  TS_HIP(hipMemsetAsync(g[1], 0, size_t(v0.V()) * 16 * 4, s));
  k_up_concat_bwd_skip<<<nblk(v0.V() * 16), 256, 0, s>>>(gcat1, 32, 16, v0.V(), g[1]);
  k_pool_bwd<<<nblk(v0.V() * 16), 256, 0, s>>>(gp1, v0.D, v0.H, v0.W, 16, g[1]);
  conv_bwd(ctx, N, 1, v0, A.a[0], params, A, g[1], grad, g[0]);
  conv_bwd(ctx, N, 0, v0, A.in8, params, A, g[0], grad, nullptr);
  float h = 0;
  TS_HIP(hipMemcpyAsync(&h, sse, 4, hipMemcpyDeviceToHost, s));
  TS_HIP(hipStreamSynchronize(s));
  return double(h) / double(v0.V());
}

void unet_adam(ts_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t n,
               int64_t step, float lr, float b1, float b2, float eps) {
  const float c1 = 1.0f - std::pow(b1, float(step)), c2 = 1.0f - std::pow(b2, float(step));
  k_adam<<<nblk(n), 256, 0, ctx->stream>>>(params, grad, m, v, n, lr, b1, b2, eps, c1, c2);
  TS_HIP(hipGetLastError());
}

}  // namespace ts
