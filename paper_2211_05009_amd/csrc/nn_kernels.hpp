// nn_kernels.hpp -- BF16 MFMA kernels of the warm-start surrogate (gfx950).
//
// Activations are NHWC bfloat16 (stored as uint16_t), channel counts
// multiples of 32; a tensor view is (pointer, channel stride, channel
// offset) so a layer can read or write one channel slice of a wider
// concatenation buffer.  Weights of a 3x3 convolution are [9][ci][co]
// (tap = 3 dy + dx, dy, dx in {0, 1, 2} for offsets -1, 0, +1).
//
// The three passes of a convolution are one implicit-GEMM kernel:
//   forward : Y[p, o]      = sum_{t,c} X[p + d_t, c] W[t, c, o]  (+ bias, ReLU)
//   dgrad   : GX[p, c]     = sum_{t,o} GY[p - d_t, o] W[t, c, o]
//   wgrad   : GW[t, c, o] += sum_p     X[p + d_t, c] GY[p, o]
// A block computes a 64 x 64 tile of the GEMM with four waves, each a 32 x 32
// sub-tile of 2 x 2 v_mfma_f32_16x16x32_bf16 (FP32 accumulate), staging
// 64 x 32 slices of both operands through LDS with 16-byte global loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}
// round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

enum { FWD = 0, DGRAD = 1, WGRAD = 2 };

struct ConvArgs {
  int n, h, w, ci, co;
  const uint16_t *x;   // FWD / WGRAD: input activations; DGRAD: output gradient
  int xs, xo;
  const uint16_t *g;   // WGRAD: output gradient
  int gs, go;
  const uint16_t *wt;  // FWD / DGRAD: bf16 weights [9][ci][co]
  const float *bias;   // FWD: per output channel (may be null)
  int relu;            // FWD: apply max(0, .)
  void *out;           // FWD: bf16 Y; DGRAD: bf16 GX; WGRAD: float GW [9 ci][co]
  int os, oo;
  int accumulate;      // DGRAD: add into GX
  int kchunk;          // WGRAD: pixels per block (multiple of 32)
  float *part;         // WGRAD: per-chunk partials [gridDim.z][9 ci][co], added
                       // into GW in chunk order by k_sum_parts (deterministic)
};

constexpr int kLdsK = 32 + 8;   // padded row of a staged 64 x 32 operand slice

template <int MODE>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
  __shared__ uint16_t As[64 * kLdsK];   // [row m][k]
  __shared__ uint16_t Bs[64 * kLdsK];   // [col n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int HW = a.h * a.w;
  const int M = MODE == WGRAD ? 9 * a.ci : a.n * HW;
  const int N = MODE == DGRAD ? a.ci : a.co;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  int k_begin = 0, k_end;
  if (MODE == WGRAD) {
    k_begin = blockIdx.z * a.kchunk;
    k_end = min(k_begin + a.kchunk, a.n * HW);
  } else {
    k_end = 9 * (MODE == FWD ? a.ci : a.co);
  }
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // this thread's staging slot: one 8-element vector of each operand
  const int sr = tid >> 2, sk = (tid & 3) * 8;      // rows along m / n, 8 k
  const int vk = tid >> 3, vr = (tid & 7) * 8;      // 8 rows along m / n, one k

  for (int k0 = k_begin; k0 < k_end; k0 += 32) {
    // ---- A slice [64 m][32 k] ------------------------------------------------
    uint16_t av[8];
    if (MODE != WGRAD) {
      // k = tap * C + c, contiguous in c; the 32-chunk lies in one tap
      const int C = MODE == FWD ? a.ci : a.co;
      const int tap = k0 / C, c0 = k0 - tap * C + sk;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      const int m = m0 + sr;
      const int b = m / HW, r = m - b * HW, py = r / a.w, px = r - py * a.w;
      const int qy = MODE == FWD ? py + dy : py - dy, qx = MODE == FWD ? px + dx : px - dx;
      if (m < M && qy >= 0 && qy < a.h && qx >= 0 && qx < a.w) {
        const uint16_t *src = a.x + (size_t)((b * a.h + qy) * a.w + qx) * a.xs + a.xo + c0;
        *(uint4 *)av = *(const uint4 *)src;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = 0;
      }
      *(uint4 *)&As[sr * kLdsK + sk] = *(uint4 *)av;
    } else {
      // m = tap * ci + c (8 consecutive c share a tap), k = pixel
      const int m = m0 + vr, p = k0 + vk;
      const int tap = m / a.ci, c0 = m - tap * a.ci;
      bool ok = m < M && p < k_end;
      int qy = 0, qx = 0, b = 0;
      if (ok) {
        b = p / HW;
        const int r = p - b * HW, py = r / a.w, px = r - py * a.w;
        qy = py + tap / 3 - 1;
        qx = px + tap % 3 - 1;
        ok = qy >= 0 && qy < a.h && qx >= 0 && qx < a.w;
      }
      if (ok) {
        *(uint4 *)av =
            *(const uint4 *)(a.x + (size_t)((b * a.h + qy) * a.w + qx) * a.xs + a.xo + c0);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = 0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) As[(vr + j) * kLdsK + vk] = av[j];
    }
    // ---- B slice, stored [64 n][32 k] ------------------------------------------
    uint16_t bv[8];
    if (MODE == FWD) {
      // B(k, n) = W[k][n], contiguous in n
      const int n = n0 + vr, k = k0 + vk;
      if (n < N) {
        *(uint4 *)bv = *(const uint4 *)(a.wt + (size_t)k * a.co + n);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = 0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[(vr + j) * kLdsK + vk] = bv[j];
    } else if (MODE == DGRAD) {
      // B(k = tap * co + o, n = c) = W[tap][c][o], contiguous in o (k)
      const int n = n0 + sr, k = k0 + sk;
      const int tap = k / a.co, o = k - tap * a.co;
      if (n < N) {
        *(uint4 *)bv = *(const uint4 *)(a.wt + ((size_t)tap * a.ci + n) * a.co + o);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = 0;
      }
      *(uint4 *)&Bs[sr * kLdsK + sk] = *(uint4 *)bv;
    } else {
      // B(k = pixel, n = o) = GY[p][o], contiguous in o
      const int n = n0 + vr, p = k0 + vk;
      if (n < N && p < k_end) {
        *(uint4 *)bv = *(const uint4 *)(a.g + (size_t)p * a.gs + a.go + n);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = 0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[(vr + j) * kLdsK + vk] = bv[j];
    }
    __syncthreads();
    // ---- 2 x 2 MFMA tiles per wave --------------------------------------------
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fa[i] = *(const bf16x8 *)&As[(wm * 32 + i * 16 + fr) * kLdsK + fk];
      fb[i] = *(const bf16x8 *)&Bs[(wn * 32 + i * 16 + fr) * kLdsK + fk];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  // ---- epilogue: lane holds rows 4 (lane/16) + e, column lane % 16 -------------
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][e];
        if (MODE == FWD) {
          if (a.bias) v += a.bias[n];
          if (a.relu) v = fmaxf(v, 0.f);
          ((uint16_t *)a.out)[(size_t)m * a.os + a.oo + n] = f2bf(v);
        } else if (MODE == DGRAD) {
          uint16_t *o = (uint16_t *)a.out + (size_t)m * a.os + a.oo + n;
          if (a.accumulate) v += bf2f(*o);
          *o = f2bf(v);
        } else {
          a.part[((size_t)blockIdx.z * M + m) * N + n] = v;
        }
      }
}

// out[i] += sum over k of part[k][i] for i < n: the deterministic second half
// of the split reductions (weight and bias gradients, loss).  A block takes
// 16 outputs; its 16 thread groups sum the k = g, g + 16, ... in order, and
// the group sums are added in group order, so the result is fixed while
// 16 loads per output are in flight.
constexpr int kSumOut = 16, kSumGroups = 16;
__global__ __launch_bounds__(256) void k_sum_parts(const float *part, int nparts, long long n,
                                                   float *out) {
  const int o = threadIdx.x % kSumOut, g = threadIdx.x / kSumOut;
  const long long i = blockIdx.x * (long long)kSumOut + o;
  float s = 0.f;
  if (i < n)
    for (int k = g; k < nparts; k += kSumGroups) s += part[(size_t)k * n + i];
  __shared__ float sh[kSumGroups][kSumOut];
  sh[g][o] = s;
  __syncthreads();
  if (g == 0 && i < n) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kSumGroups; ++q) t += sh[q][o];
    out[i] += t;
  }
}

// Bias gradient, first half: part[block][o] = sum of GY[p][o] over the
// block's chunk of pixels; one channel per thread (c < 256).  k_sum_parts
// adds the chunks into gb.
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *g, int gs, int go, int npix,
                                                   int co, int chunk, float *part) {
  const int o = threadIdx.x;
  if (o >= co) return;
  const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, npix);
  float s = 0.f;
  for (int p = p0; p < p1; ++p) s += bf2f(g[(size_t)p * gs + go + o]);
  part[(size_t)blockIdx.x * co + o] = s;
}

// 2 x 2 average pooling (h, w: input size, even).
__global__ void k_pool_fwd(const uint16_t *x, int xs, int xo, int n, int h, int w, int c,
                           uint16_t *y) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int ho = h / 2, wo = w / 2;
  if (i >= (long long)n * ho * wo * c) return;
  const int ch = i % c;
  const long long pix = i / c;
  const int ox = pix % wo, oy = (pix / wo) % ho, b = pix / ((long long)wo * ho);
  float s = 0.f;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx)
      s += bf2f(x[((size_t)(b * h + 2 * oy + dy) * w + 2 * ox + dx) * xs + xo + ch]);
  y[i] = f2bf(0.25f * s);
}

__global__ void k_pool_bwd(const uint16_t *gy, int n, int h, int w, int c, uint16_t *gx, int gxs,
                           int gxo, int accumulate) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)n * h * w * c) return;
  const int ch = i % c;
  const long long pix = i / c;
  const int px = pix % w, py = (pix / w) % h, b = pix / ((long long)w * h);
  const int ho = h / 2, wo = w / 2;
  float v = 0.25f * bf2f(gy[((size_t)(b * ho + py / 2) * wo + px / 2) * c + ch]);
  uint16_t *o = gx + (size_t)pix * gxs + gxo + ch;
  if (accumulate) v += bf2f(*o);
  *o = f2bf(v);
}

// Nearest 2x upsampling (h, w: input size) into a channel slice of y.
__global__ void k_up_fwd(const uint16_t *x, int n, int h, int w, int c, uint16_t *y, int ys,
                         int yo) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int H = 2 * h, W = 2 * w;
  if (i >= (long long)n * H * W * c) return;
  const int ch = i % c;
  const long long pix = i / c;
  const int px = pix % W, py = (pix / W) % H, b = pix / ((long long)W * H);
  y[(size_t)pix * ys + yo + ch] = x[((size_t)(b * h + py / 2) * w + px / 2) * c + ch];
}

__global__ void k_up_bwd(const uint16_t *gy, int gys, int gyo, int n, int h, int w, int c,
                         uint16_t *gx) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)n * h * w * c) return;
  const int ch = i % c;
  const long long pix = i / c;
  const int px = pix % w, py = (pix / w) % h, b = pix / ((long long)w * h);
  const int W = 2 * w;
  float s = 0.f;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx)
      s += bf2f(gy[((size_t)(b * 2 * h + 2 * py + dy) * W + 2 * px + dx) * gys + gyo + ch]);
  gx[i] = f2bf(s);
}

// g *= (y > 0) over a channel slice [npix][c] of both tensors.
__global__ void k_relu_bwd(const uint16_t *y, int ys, int yo, uint16_t *g, int gs, int go,
                           long long npix, int c) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= npix * c) return;
  const long long p = i / c;
  const int ch = i % c;
  if (!(bf2f(y[p * ys + yo + ch]) > 0.f)) g[p * gs + go + ch] = 0;
}

// Masked mean-squared error over the first `cu` channels of pred (stride
// ps): loss[block] = the block's sum of mask (pred - t)^2 / count (k_sum_parts
// adds the blocks); grad = 2 mask (pred - t) / count (bf16, stride gs, zero
// elsewhere).  t: FP32 [npix][cu]; mask FP32 [npix].
__global__ __launch_bounds__(256) void k_mse(const uint16_t *pred, int ps, const float *t,
                                             const float *mask, long long npix, int cu,
                                             float inv_count, uint16_t *grad, int gs,
                                             float *loss) {
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  float l = 0.f;
  if (p < npix) {
    const float mk = mask[p];
    for (int ch = 0; ch < gs; ++ch) {
      float gv = 0.f;
      if (ch < cu) {
        const float d = bf2f(pred[p * ps + ch]) - t[p * cu + ch];
        l += mk * d * d;
        gv = 2.f * mk * d * inv_count;
      }
      grad[p * gs + ch] = f2bf(gv);
    }
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  __shared__ float part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss[blockIdx.x] = (part[0] + part[1] + part[2] + part[3]) * inv_count;
}

// Adam on FP32 master weights; refreshes the bf16 copy (may be null).
__global__ void k_adam(float *w, float *m, float *v, const float *g, uint16_t *wb, long long n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

// float -> bf16 copy
__global__ void k_to_bf16(const float *a, uint16_t *b, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

}  // namespace nn
}  // namespace lbm
