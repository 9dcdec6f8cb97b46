// nn_kernels.hpp -- BF16 MFMA kernels of the warm-start surrogate (gfx950).
//
// Activations are NHWC bfloat16 (stored as uint16_t), channel counts
// multiples of 32; a tensor view is (pointer, channel stride, channel
// offset) so a layer can read or write one channel slice of a wider
// concatenation buffer.  Weights of a 3x3 convolution are [9][ci][co]
// (tap = 3 dy + dx, dy, dx in {0, 1, 2} for offsets -1, 0, +1).
//
// The three passes of a convolution:
//   forward : Y[p, o]      = sum_{t,c} X[p + d_t, c] W[t, c, o]  (+ bias, ReLU)
//   dgrad   : GX[p, c]     = sum_{t,o} GY[p - d_t, o] W[t, c, o]
//   wgrad   : GW[t, c, o] += sum_p     X[p + d_t, c] GY[p, o]
// all on v_mfma_f32_16x16x32_bf16 (FP32 accumulate): forward and dgrad as a
// direct convolution from an LDS patch of whole image rows (k_conv_patch)
// or, for widths it does not serve, a pipelined implicit GEMM (k_conv_mn);
// wgrad streamed over strips of image rows with all nine taps per block
// (k_wgrad_rows: widths 16-128) or as a pipelined GEMM over pixel chunks
// (k_wgrad: any width), the per-strip or per-chunk partials added in a
// fixed order (k_sum_parts).
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
  const uint16_t *wtt; // FWD (optional): the same weights as [9][co][ci]
  const float *bias;   // FWD: per output channel (may be null)
  int relu;            // FWD: apply max(0, .)
  void *out;           // FWD: bf16 Y; DGRAD: bf16 GX; WGRAD: float GW [9 ci][co]
  int os, oo;
  int accumulate;      // DGRAD: add into GX
  const uint16_t *mask;  // DGRAD (optional): zero GX where mask <= 0 (the
                         // ReLU of the layer that produced the input; same
                         // stride and offset as out), before the bf16 rounding
  // FWD, patch kernel (optional): the layer's output also goes, as the next
  // op would write it, to
  uint16_t *pool_out;  // its 2 x 2 average pool, dense [n][h/2][w/2][co]
  uint16_t *up_out;    // its nearest 2x upsampling, a slice (ups, upo) of
  int ups, upo;        // [n][2h][2w]
  int kchunk;          // WGRAD: pixels per block (multiple of 32)
  float *part;         // WGRAD: per-chunk partials [gridDim.z][9 ci][co], added
                       // into GW in chunk order by k_sum_parts (deterministic)
};

constexpr int kLdsK = 32 + 8;   // padded row of a staged 64 x 32 operand slice

// The hardware deals the blocks of a launch round-robin over the 8 XCDs
// (block L to XCD L % 8), each with its own L2.  xcd_block maps L to a
// block index such that each XCD runs one contiguous range of indices, so
// neighbouring tiles, which share halo rows and input strips, meet in one L2.
__device__ __forceinline__ int xcd_block(int L, int nb) {
  const int k = L & 7, q = nb >> 3, r = nb & 7;
  return k * q + (k < r ? k : r) + (L >> 3);
}

// ---------------------------------------------------------------------------
// Forward and input-gradient passes as one pipelined implicit GEMM.
//   FWD  : M = pixels, N = co, K = 9 ci;  A(p, (t,c)) = X[p + d_t][c],
//          B((t,c), o) = W[t][c][o] (16-byte vectors along n, stored into
//          LDS transposed, element by element: the weights are small).
//   DGRAD: M = pixels, N = ci, K = 9 co;  A(p, (t,o)) = GY[p - d_t][o],
//          B((t,o), c) = W[t][c][o] (contiguous along k = o).
// A block of 256 threads (WM x WN waves, each TM x TN MFMA 16 x 16 x 32
// tiles) computes a BM x BN tile, BM = 16 WM TM, BN = 16 WN TN.  K advances
// in slices of 32 (one tap, 32 channels: channel counts are multiples of 32,
// so a slice never straddles a tap); each slice is loaded from global memory
// into registers while the previous one is multiplied out of LDS, and the
// two LDS buffers alternate, so one barrier per slice suffices.
constexpr int kBK = 32;

template <int MODE, int WM, int WN, int TM, int TN>
__global__ __launch_bounds__(256) void k_conv_mn(ConvArgs a) {
  static_assert(WM * WN == 4, "four waves");
  constexpr int BM = 16 * WM * TM, BN = 16 * WN * TN;
  // 16-byte vectors per thread and operand (4 per row of 32 k)
  constexpr int AV = (BM * 4 + 255) / 256, BV = (BN * 4 + 255) / 256;
  __shared__ uint16_t As[2][BM * kLdsK];
  __shared__ uint16_t Bs[2][BN * kLdsK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int HW = a.h * a.w, M = a.n * HW;
  const int C = MODE == FWD ? a.ci : a.co;      // channels along k within a tap
  const int N = MODE == FWD ? a.co : a.ci;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int nk = 9 * C / kBK;

  // staging: vector v of this thread covers row r = (tid + 256 v) / 4, k = 8 ((tid) % 4)
  const int kq = (tid & 3) * 8;
  int apix[AV], ay[AV], ax[AV];
#pragma unroll
  for (int v = 0; v < AV; ++v) {   // rows beyond BM or M load zeros (ay out of range)
    const int m = (tid >> 2) + 64 * v < BM ? m0 + (tid >> 2) + 64 * v : M;
    const int b = m / HW, r = m - b * HW;
    ay[v] = m < M ? r / a.w : -1000000;
    ax[v] = r - (r / a.w) * a.w;
    apix[v] = b * HW;
  }
  uint4 ra[AV], rb[BV];
  auto load = [&](int ks) {
    const int k0 = ks * kBK, tap = k0 / C, c0 = k0 - tap * C + kq;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int qy = MODE == FWD ? ay[v] + dy : ay[v] - dy;
      const int qx = MODE == FWD ? ax[v] + dx : ax[v] - dx;
      if (qy >= 0 && qy < a.h && qx >= 0 && qx < a.w)
        ra[v] = *(const uint4 *)(a.x + (size_t)(apix[v] + qy * a.w + qx) * a.xs + a.xo + c0);
      else
        ra[v] = make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      if (MODE == FWD) {   // W[tap][c][o]: row k = tid % 32, 8 n from 8 (tid / 32 + 8 v)
        const int kb = tid & 31, nb = 8 * ((tid >> 5) + 8 * v);
        const int cc = k0 - tap * C + kb;
        rb[v] = (nb < BN && n0 + nb < N)
                    ? *(const uint4 *)(a.wt + ((size_t)tap * a.ci + cc) * a.co + n0 + nb)
                    : make_uint4(0, 0, 0, 0);
      } else {             // W[tap][c][o], k = o: row n = tid / 4 + 64 v, 8 k
        const int n = n0 + (tid >> 2) + 64 * v;
        rb[v] = ((tid >> 2) + 64 * v < BN && n < N)
                    ? *(const uint4 *)(a.wt + ((size_t)tap * a.ci + n) * a.co + c0)
                    : make_uint4(0, 0, 0, 0);
      }
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v)
      if ((tid >> 2) + 64 * v < BM)
        *(uint4 *)&As[buf][((tid >> 2) + 64 * v) * kLdsK + kq] = ra[v];
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      if (MODE == FWD) {
        const int kb = tid & 31, nb = 8 * ((tid >> 5) + 8 * v);
        if (nb < BN) {
          const uint16_t *e = (const uint16_t *)&rb[v];
#pragma unroll
          for (int j = 0; j < 8; ++j) Bs[buf][(nb + j) * kLdsK + kb] = e[j];
        }
      } else if ((tid >> 2) + 64 * v < BN) {
        *(uint4 *)&Bs[buf][((tid >> 2) + 64 * v) * kLdsK + kq] = rb[v];
      }
    }
  };

  floatx4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fk = (lane >> 4) * 8;
  load(0);
  stage(0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int buf = ks & 1;
    if (ks + 1 < nk) load(ks + 1);
    bf16x8 fa[TM], fb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      fa[i] = *(const bf16x8 *)&As[buf][(wm * TM * 16 + i * 16 + fr) * kLdsK + fk];
#pragma unroll
    for (int j = 0; j < TN; ++j)
      fb[j] = *(const bf16x8 *)&Bs[buf][(wn * TN * 16 + j * 16 + fr) * kLdsK + fk];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    if (ks + 1 < nk) stage(buf ^ 1);
    __syncthreads();
  }

  // epilogue: lane holds rows 4 (lane / 16) + e, column lane % 16 of each tile
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn * TN * 16 + j * 16 + (lane & 15);
      if (n >= N) continue;
      const float bn = (MODE == FWD && a.bias) ? a.bias[n] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * TM * 16 + i * 16 + (lane >> 4) * 4 + e;
        if (m >= M) continue;
        float v = acc[i][j][e];
        uint16_t *o = (uint16_t *)a.out + (size_t)m * a.os + a.oo + n;
        if (MODE == FWD) {
          v += bn;
          if (a.relu) v = fmaxf(v, 0.f);
        } else {
          if (a.accumulate) v += bf2f(*o);
          if (a.mask && !(bf2f(a.mask[o - (uint16_t *)a.out]) > 0.f)) v = 0.f;
        }
        *o = f2bf(v);
      }
    }
}

// ---------------------------------------------------------------------------
// The same two passes as direct convolutions: a tile is TPIX = R w pixels
// (R whole rows of one image; w a multiple of 16, R dividing h) by BN
// output channels; per chunk of 32 input channels the block loads the
// (R + 2) x (w + 2) patch of the input (zero halo) and the 9 taps' weights
// into LDS once, and runs the 9 taps' MFMAs out of LDS, instead of gathering
// a shifted copy of the input from global memory for every tap.  Four waves
// split the TPIX pixels (TPIX / 64 MFMA row tiles each) and share all BN
// columns.  The epilogue stages the FP32 tile in LDS (over patch and
// weights) and writes whole 16-byte vectors of 8 channels.  Patch pixels
// and FP32 rows are padded in LDS so that neither the MFMA operand reads
// nor the epilogue's writes conflict on banks.
// In the forward pass the epilogue can also write the output's 2 x 2 average
// pool or its nearest 2x upsampling (ConvArgs pool_out, up_out), the next
// op of the network, from the tile it holds.
// The blocks are persistent: block b takes tiles b, b + G, b + 2 G, ... (G
// blocks, numbered so that each XCD holds a contiguous range of tiles) and
// walks their (tile, chunk) steps in order, loading the next step's patch
// and weights into registers while the current step's MFMAs and, at a
// tile's last chunk, its epilogue run; so memory and matrix cores stay busy
// together instead of every block loading, then computing, then storing.
//   FWD  : out[p][o] = sum_{t,c} X[p + d_t][c] W[t][c][o]   (N = co, chunks of ci)
//   DGRAD: out[p][c] = sum_{t,o} GY[p - d_t][o] W[t][c][o]  (N = ci, chunks of co)
// LDS elements per patch pixel: 32 channels + 8 pad, so the 16-byte reads of
// 8 lanes at consecutive pixels (80-byte stride) cover all 32 banks once
constexpr int kPs = 40;

template <int MODE, int W, int BN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_patch(
    ConvArgs a, int ntiles) {
  // tile: R whole rows of W pixels, TPIX = R W (256 at W = 128, 128 at
  // W = 64 and 32, 64 at W = 16)
  constexpr int TPIX = W == 128 ? 256 : W == 16 ? 64 : 128;
  constexpr int R = TPIX / W, PW = W + 2, PP = (R + 2) * PW;
  constexpr int TM = TPIX / 64, TN = BN / 16;
  constexpr int OS = BN + 4;   // padded FP32 row: the 4 lane groups' writes fill 2 bank cycles
  // one LDS buffer: the patch [pixel][32 channels + pad] and the weights
  // [tap][n][k] while the taps run, the FP32 tile [pixel][OS] in the epilogue
  constexpr int PS_EL = PP * kPs, WS_EL = 9 * BN * kLdsK;
  constexpr int SM_EL = PS_EL + WS_EL > TPIX * OS * 2 ? PS_EL + WS_EL : TPIX * OS * 2;
  static_assert(TM >= 1 && SM_EL * 2 <= 80 * 1024, "two blocks per CU");
  constexpr int PV = (PP * 4 + 255) / 256;            // patch vectors per thread
  constexpr int WV = (9 * 32 * (BN / 8) + 255) / 256;  // weight vectors per thread
  __shared__ __align__(16) uint16_t Sm[SM_EL];
  uint16_t *const Ps = Sm, *const Ws = Sm + PS_EL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int HW = a.h * W;
  const int C = MODE == FWD ? a.ci : a.co;
  const int N = MODE == FWD ? a.co : a.ci;
  const int ntn = (N + BN - 1) / BN;   // column tiles per pixel tile (adjacent tile numbers)

  // Tile being loaded: its first output channel, and the image pixels of
  // this thread's patch vectors (-1: halo outside the image, or beyond the
  // patch); a thread's vectors all hold channels pkq .. pkq + 7 of a chunk.
  int ln0 = 0;
  int ppix[PV];
  const int pkq = (tid & 3) * 8;
  auto set_load_tile = [&](int tile) {
    const int lm0 = tile / ntn * TPIX;
    ln0 = tile % ntn * BN;
    const int img = lm0 / HW, y0 = (lm0 - img * HW) / W;   // first row of the tile
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int pp = (tid + 256 * u) >> 2;
      const int py = pp / PW, px = pp - py * PW;
      const int gy = y0 + py - 1, gx = px - 1;
      ppix[u] = (pp < PP && gy >= 0 && gy < a.h && gx >= 0 && gx < W) ? img * HW + gy * W + gx
                                                                        : -1;
    }
  };

  // One chunk of 32 channels: all its loads are issued into registers
  // first (unrolled, so they are in flight together), then stored to LDS.
  uint4 rp[PV], rw[WV];
  auto load = [&](int c0) {
    const int n0 = ln0;
#pragma unroll
    for (int u = 0; u < PV; ++u) {   // halo vectors read pixel 0 and are zeroed
      const uint4 x = *(const uint4 *)(a.x + (size_t)(ppix[u] >= 0 ? ppix[u] : 0) * a.xs + a.xo +
                                       pkq + c0);
      rp[u] = ppix[u] >= 0 ? x : make_uint4(0, 0, 0, 0);
    }
    // weights as [tap][n][k] rows: FWD from the transposed copy WT[t][co][ci]
    // (required), DGRAD from W[t][ci][co]; rows beyond the taps or N read row
    // 0 and are zeroed, so every load is issued without a branch
    const uint16_t *wsrc = MODE == FWD ? a.wtt : a.wt;
#pragma unroll
    for (int u = 0; u < WV; ++u) {
      const int v = tid + 256 * u;
      const int t = v / (BN * 4), r = v - t * BN * 4;
      const int n = r >> 2, kq = (r & 3) * 8;
      const bool ok = t < 9 && n0 + n < N;
      const uint4 w = *(const uint4 *)(wsrc + ((size_t)(ok ? t * N + n0 + n : 0)) * C + c0 + kq);
      rw[u] = ok ? w : make_uint4(0, 0, 0, 0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int v = tid + 256 * u;
      if ((v >> 2) < PP) *(uint4 *)&Ps[(v >> 2) * kPs + (v & 3) * 8] = rp[u];
    }
#pragma unroll
    for (int u = 0; u < WV; ++u) {
      const int v = tid + 256 * u;
      const int t = v / (BN * 4), r = v - t * BN * 4;
      if (t < 9) *(uint4 *)&Ws[(t * BN + (r >> 2)) * kLdsK + (r & 3) * 8] = rw[u];
    }
  };

  floatx4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fk = (lane >> 4) * 8;
  // LDS element offset of this lane's A fragment in each row tile at tap
  // (1, 1) (the pixel itself)
  int aoff[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int q = wave * (TPIX / 4) + i * 16 + fr;
    aoff[i] = ((q / W + 1) * PW + q % W + 1) * kPs + fk;
  }

  // epilogue of the tile at (m0, n0): lane holds rows 4 (lane / 16) + e,
  // column lane % 16 of each MFMA tile; the FP32 tile goes to LDS
  // [TPIX][OS], then each thread writes 8 consecutive channels of a pixel
  auto epilogue = [&](int m0, int n0) {
    float *Os = reinterpret_cast<float *>(Sm);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          Os[(wave * (TPIX / 4) + i * 16 + (lane >> 4) * 4 + e) * OS + j * 16 + (lane & 15)] =
              acc[i][j][e];
    // a thread always writes channels nq .. nq + 7 (256 is a multiple of
    // BN / 8): their bias values are loaded once, all in flight together
    const int nq = (tid % (BN / 8)) * 8;
    float bv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (MODE == FWD && a.bias && n0 + nq < N) {
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = a.bias[n0 + nq + j];
    }
    __syncthreads();
    if (n0 + nq >= N) return;
    for (int v = tid; v < TPIX * (BN / 8); v += 256) {
      const int pl = v / (BN / 8);
      const float *src = Os + pl * OS + nq;
      uint16_t *o = (uint16_t *)a.out + (size_t)(m0 + pl) * a.os + a.oo + n0 + nq;
      float r[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) r[j] = src[j];
      if (MODE == FWD) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          r[j] += bv[j];
          if (a.relu) r[j] = fmaxf(r[j], 0.f);
        }
      } else {
        if (a.accumulate) {
          const uint4 old = *(const uint4 *)o;
          const uint16_t *ov = (const uint16_t *)&old;
#pragma unroll
          for (int j = 0; j < 8; ++j) r[j] += bf2f(ov[j]);
        }
        if (a.mask) {
          const uint4 mv = *(const uint4 *)(a.mask + (o - (uint16_t *)a.out));
          const uint16_t *mk = (const uint16_t *)&mv;
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (!(bf2f(mk[j]) > 0.f)) r[j] = 0.f;
        }
      }
      uint4 pk;
      uint16_t *pv = (uint16_t *)&pk;
#pragma unroll
      for (int j = 0; j < 8; ++j) pv[j] = f2bf(r[j]);
      *(uint4 *)o = pk;
      if (MODE == FWD && a.up_out) {   // the 2 x 2 copies at twice the resolution
        const int p = m0 + pl, img = p / HW, y = (p - img * HW) / W, x = p % W;
        uint16_t *u = a.up_out + ((size_t)(img * 2 * a.h + 2 * y) * (2 * W) + 2 * x) * a.ups +
                      a.upo + n0 + nq;
        *(uint4 *)u = pk;
        *(uint4 *)(u + a.ups) = pk;
        *(uint4 *)(u + (size_t)2 * W * a.ups) = pk;
        *(uint4 *)(u + (size_t)(2 * W + 1) * a.ups) = pk;
      }
    }
    if (MODE == FWD && a.pool_out) {   // 2 x 2 means of the rounded outputs, in
      // k_pool_fwd's order; the tile's R rows (R even) start at an even row
      const int img = m0 / HW, y0 = (m0 - img * HW) / W;
      for (int v = tid; v < TPIX / 4 * (BN / 8); v += 256) {
        const int pp = v / (BN / 8), oy = pp / (W / 2), ox = pp % (W / 2);
        float sm[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const float *src = Os + ((2 * oy + dy) * W + 2 * ox + dx) * OS + nq;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              float r = src[j] + bv[j];
              if (a.relu) r = fmaxf(r, 0.f);
              sm[j] += bf2f(f2bf(r));
            }
          }
        uint4 pk;
        uint16_t *pv = (uint16_t *)&pk;
#pragma unroll
        for (int j = 0; j < 8; ++j) pv[j] = f2bf(0.25f * sm[j]);
        *(uint4 *)(a.pool_out +
                   ((size_t)(img * (a.h / 2) + y0 / 2 + oy) * (W / 2) + ox) * a.co + n0 + nq) = pk;
      }
    }
  };

  int tile = xcd_block(blockIdx.x, gridDim.x);   // gridDim.x <= ntiles
  int c0 = 0;
  set_load_tile(tile);
  int em0 = tile / ntn * TPIX, en0 = ln0;        // tile whose sums acc holds
  load(0);
  stage();
  __syncthreads();
  for (;;) {
    // the step after (tile, c0)
    int ntile = tile, nc0 = c0 + 32;
    if (nc0 >= C) {
      ntile = tile + gridDim.x;
      nc0 = 0;
    }
    const bool more = ntile < ntiles;
    if (more) {   // in flight during this step's taps and epilogue
      if (ntile != tile) set_load_tile(ntile);
      load(nc0);
    }
#pragma unroll 3
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      // FWD reads pixel p + d_t, DGRAD p - d_t
      const int oy = MODE == FWD ? dy - 1 : 1 - dy, ox = MODE == FWD ? dx - 1 : 1 - dx;
      bf16x8 fa[TM], fb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[i] = *(const bf16x8 *)&Ps[aoff[i] + (oy * PW + ox) * kPs];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        fb[j] = *(const bf16x8 *)&Ws[(t * BN + j * 16 + fr) * kLdsK + fk];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();   // patch and weights read by every wave
    if (nc0 == 0) {    // the tile's last chunk: write it out
      epilogue(em0, en0);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
      em0 = ntile / ntn * TPIX;
      en0 = ntile % ntn * BN;
      __syncthreads();   // the FP32 tile read by every thread
    }
    if (!more) break;
    stage();
    __syncthreads();
    tile = ntile;
    c0 = nc0;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient as a pipelined GEMM over a chunk of pixels:
//   part[z][m = (t, c)][o] = sum_{p in chunk z} X[p + d_t][c] GY[p][o]
// M = 9 ci, N = co, K = pixels.  Both operands are pixel-major in memory
// (NHWC) while the MFMA takes 8 consecutive k per lane, so each operand is
// transposed on its way into LDS: a loader thread reads 4 consecutive
// pixels x 8 channels (four 16-byte loads) and writes, per channel, the 4
// pixels as one 64-bit LDS store (As[m][k], Bs[n][k], k contiguous).  A
// block computes a 64 x BN tile with four waves (2 x 2), K advances by 64
// pixels; the next slice is loaded into registers while the current one is
// multiplied out of the other LDS buffer.
constexpr int kWBK = 64, kWLd = kWBK + 8;   // pixels per slice, padded LDS row

template <int BN>
__global__ __launch_bounds__(256) void k_wgrad(ConvArgs a) {
  constexpr int TN = BN / 32;                       // 16-wide n tiles per wave (2 x 2 waves)
  __shared__ __align__(16) uint16_t As[2][64 * kWLd];
  __shared__ __align__(16) uint16_t Bs[2][BN * kWLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int HW = a.h * a.w, M = 9 * a.ci, N = a.co;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * BN;
  const int p_begin = blockIdx.z * a.kchunk;
  const int p_end = min(p_begin + a.kchunk, a.n * HW);
  // loader roles: threads 0-127 take A (8 rows x 4 pixels each), threads
  // 128 .. 128 + 2 BN - 1 take B (8 columns x 4 pixels each)
  const bool isA = tid < 128;
  const int li = isA ? tid : tid - 128;
  const int rg = li >> 4, pq = li & 15;            // row / column group, pixel quad
  const bool active = isA || li < 2 * BN;
  // A rows 8 rg .. 8 rg + 7: tap and first channel (8 rows share a tap)
  const int am = m0 + 8 * rg;
  const int atap = am / a.ci, ac = am - atap * a.ci;
  const int ady = atap / 3 - 1, adx = atap % 3 - 1;
  const bool arow_ok = am < M;
  const int bn = n0 + 8 * rg;
  const bool bcol_ok = bn < N;

  uint4 r[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = k0 + 4 * pq + j;
      r[j] = make_uint4(0, 0, 0, 0);
      if (!active || p >= p_end) continue;
      if (isA) {
        if (!arow_ok) continue;
        const int b = p / HW, q = p - b * HW, py = q / a.w, px = q - py * a.w;
        const int qy = py + ady, qx = px + adx;
        if (qy >= 0 && qy < a.h && qx >= 0 && qx < a.w)
          r[j] = *(const uint4 *)(a.x + ((size_t)b * HW + (size_t)qy * a.w + qx) * a.xs + a.xo +
                                  ac);
      } else if (bcol_ok) {
        r[j] = *(const uint4 *)(a.g + (size_t)p * a.gs + a.go + bn);
      }
    }
  };
  auto stage = [&](int buf) {
    if (!active) return;
    uint16_t *dst = isA ? &As[buf][0] : &Bs[buf][0];
    const uint16_t *e0 = (const uint16_t *)&r[0], *e1 = (const uint16_t *)&r[1];
    const uint16_t *e2 = (const uint16_t *)&r[2], *e3 = (const uint16_t *)&r[3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      uint2 v;
      v.x = (uint32_t)e0[c] | ((uint32_t)e1[c] << 16);
      v.y = (uint32_t)e2[c] | ((uint32_t)e3[c] << 16);
      *(uint2 *)&dst[(8 * rg + c) * kWLd + 4 * pq] = v;
    }
  };

  floatx4 acc[2][TN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  load(p_begin);
  stage(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = p_begin; k0 < p_end; k0 += kWBK) {
    const bool more = k0 + kWBK < p_end;
    if (more) load(k0 + kWBK);
#pragma unroll
    for (int kk = 0; kk < kWBK; kk += 32) {
      bf16x8 fa[2], fb[TN];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        fa[i] = *(const bf16x8 *)&As[buf][(wm * 32 + i * 16 + fr) * kWLd + kk + fk];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        fb[j] = *(const bf16x8 *)&Bs[buf][(wn * TN * 16 + j * 16 + fr) * kWLd + kk + fk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
        const int n = n0 + wn * TN * 16 + j * 16 + (lane & 15);
        if (m < M && n < N) a.part[((size_t)blockIdx.z * M + m) * N + n] = acc[i][j][e];
      }
}

// Weight gradient streamed over image rows, for widths 16, 32, 64 and 128.
//   part[z][(t, c)][o] = sum over the pixels p of strip z of X[p + d_t][c] GY[p][o]
// A strip is `rows` consecutive image rows of the batch (it may run on from
// one image into the next); a block owns one strip, 32 input channels
// (c0 ..), NB = 32 NT output channels (o0 ..) and all nine taps, so each
// input and output-gradient element of the strip is loaded once per block
// (k_wgrad loads them once per 64-row tile of the 9 ci taps x channels).
// The reduction runs over pixels: a lane's 8 consecutive MFMA k are 8
// consecutive x of one row, so both operands are stored into LDS with x
// contiguous (channel rows):
//   input rows in a ring of 2U + 2 image rows, each [32 c][W + 8], the 8
//   zeros after a channel row doubling as the pad before the next one, so
//   x = -1 and x = W read zeros;
//   output-gradient rows of the current and the next iteration.
// Per tap row the three x offsets come from one aligned 16-byte read and
// two 4-byte reads by funnel shifts (v_alignbit); rows above the top or
// below the bottom of a pixel's image give zero operands.  An iteration
// covers U rows (U W pixels, a multiple of 128: U W / 32 k-steps; U <= h):
// the next iteration's rows are loaded into registers while the current
// one is multiplied out, then written into ring slots the current
// iteration does not read, so one barrier per iteration suffices.  KW groups of four waves split each
// iteration's k-steps and add their sums in LDS at the end (fixed order),
// so a block does KW times the work of one group and the strips, hence the
// partials, are KW times fewer.  With bpart set, blocks of the first
// channel tile also add up GY of their strip in FP32, the bias gradient's
// partial bpart[z][o] (fixed order: per thread, then a fixed LDS tree).
template <int W, int U, int NT, int KW>
__global__ __launch_bounds__(256 * KW) void k_wgrad_rows(ConvArgs a, int rows, float *bpart) {
  static_assert(U * W % 128 == 0 && W % 16 == 0, "an iteration is a multiple of 128 pixels");
  constexpr int NTH = 256 * KW;
  constexpr int RP = W + 8, NR = 2 * U + 2, NB = 32 * NT, KS = U * W / 32;
  static_assert(KS % KW == 0, "groups share the k-steps evenly");
  constexpr int NIN = U * W, NGO = U * W * NT;   // loader tasks: 4 pixels x 8 channels
  constexpr int IN_T = (NIN + NTH - 1) / NTH, GO_T = (NGO + NTH - 1) / NTH;
  constexpr int GCG = 4 * NT;                    // 8-channel groups of the NB outputs
  constexpr int IS_EL = NR * 32 * RP + 8, GS_EL = U * NB * RP;
  __shared__ __align__(16) uint16_t Is[IS_EL];
  __shared__ __align__(16) uint16_t Gs[2][GS_EL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = wave >> 2, gw = wave & 3;      // k-step group, wave within it
  const int wc = gw & 1, wn = gw >> 1;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  // block -> (strip, output tile, channel tile); consecutive blocks of one
  // XCD share a strip
  const int tcn = a.ci / 32, ton = a.co / NB;
  const int id = xcd_block(blockIdx.x, gridDim.x);
  const int z = id / (tcn * ton), cx = id % tcn, ox = (id / tcn) % ton;
  const int c0 = 32 * cx, o0 = NB * ox;
  const int nrow = a.n * a.h;
  const int r0 = z * rows, r1 = min(r0 + rows, nrow);
  const int nit = (r1 - r0 + U - 1) / U;
  const bool do_bias = bpart != nullptr && cx == 0;

  float bs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // 4 consecutive pixels x 8 channels of one row -> channel rows of LDS
  auto put = [&](uint16_t *dst, const uint4 (&r)[4]) {
    const uint16_t *e0 = (const uint16_t *)&r[0], *e1 = (const uint16_t *)&r[1];
    const uint16_t *e2 = (const uint16_t *)&r[2], *e3 = (const uint16_t *)&r[3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      uint2 v;
      v.x = (uint32_t)e0[c] | ((uint32_t)e1[c] << 16);
      v.y = (uint32_t)e2[c] | ((uint32_t)e3[c] << 16);
      *(uint2 *)&dst[c * RP] = v;
    }
  };
  auto bias_add = [&](const uint4 (&r)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t w4[4] = {r[e].x, r[e].y, r[e].z, r[e].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bs[2 * j] += __uint_as_float(w4[j] << 16);
        bs[2 * j + 1] += __uint_as_float(w4[j] & 0xFFFF0000u);
      }
    }
  };
  // rows outside the batch read row 0 and are zeroed (no branch around loads)
  auto fetch = [&](const uint16_t *base, int stride, int row, int quad, uint4 (&r)[4]) {
    const bool ok = row >= 0 && row < nrow;
    const uint16_t *src = base + ((size_t)(ok ? row : 0) * W + 4 * quad) * stride;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint4 v = *(const uint4 *)(src + (size_t)e * stride);
      r[e] = ok ? v : make_uint4(0, 0, 0, 0);
    }
  };
  const uint16_t *xb = a.x + a.xo + c0, *gyb = a.g + a.go + o0;
  // ring slot of image row `row`: rows r0 - 1, r0, ... take slots 0, 1, ...
  auto slot_of = [&](int row) { return (row - r0 + 1) % NR; };

  // prologue: zero pads, input rows r0 - 1 .. r0 + U, GY rows r0 .. r0 + U - 1
  for (int i = tid; i < NR * 32 + 1; i += NTH) *(uint4 *)&Is[i * RP] = make_uint4(0, 0, 0, 0);
  for (int q = tid; q < (U + 2) * W; q += NTH) {
    const int cg = q & 3, quad = (q >> 2) % (W / 4), u = (q >> 2) / (W / 4);
    uint4 r[4];
    fetch(xb + 8 * cg, a.xs, r0 - 1 + u, quad, r);
    put(&Is[(slot_of(r0 - 1 + u) * 32 + 8 * cg) * RP + 8 + 4 * quad], r);
  }
  for (int q = tid; q < NGO; q += NTH) {
    const int cg = q % GCG, quad = (q / GCG) % (W / 4), u = q / GCG / (W / 4);
    uint4 r[4];
    fetch(gyb + 8 * cg, a.gs, r0 + u, quad, r);
    put(&Gs[0][(u * NB + 8 * cg) * RP + 4 * quad], r);
    if (do_bias) bias_add(r);
  }

  floatx4 acc[9][NT];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  uint4 rin[IN_T][4], rgo[GO_T][4];
  __syncthreads();

  for (int it = 0; it < nit; ++it) {
    const int rb = r0 + it * U, buf = it & 1;
    const bool more = it + 1 < nit;
    if (more) {   // rows of the next iteration: input rb + U + 1 .., GY rb + U ..
#pragma unroll
      for (int j = 0; j < IN_T; ++j) {
        const int q = tid + NTH * j;
        if (q < NIN) {
          const int cg = q & 3, quad = (q >> 2) % (W / 4), u = (q >> 2) / (W / 4);
          fetch(xb + 8 * cg, a.xs, rb + U + 1 + u, quad, rin[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < GO_T; ++j) {
        const int q = tid + NTH * j;
        if (q < NGO) {
          const int cg = q % GCG, quad = (q / GCG) % (W / 4), u = q / GCG / (W / 4);
          fetch(gyb + 8 * cg, a.gs, rb + U + u, quad, rgo[j]);
        }
      }
    }
    const int yb = rb % a.h, sb = (it * U) % NR;
#pragma unroll
    for (int kk = 0; kk < KS / KW; ++kk) {
      const int ks = kk * KW + grp;
      const int j0 = ks * 32 + fk, u = j0 / W, x0 = j0 % W;
      int y = yb + u;
      if (y >= a.h) y -= a.h;
      bf16x8 fb[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        fb[nt] = *(const bf16x8 *)&Gs[buf][(u * NB + wn * 16 * NT + nt * 16 + fr) * RP + x0];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int yy = y + dy - 1;
        int s = sb + u + dy;
        if (s >= NR) s -= NR;
        const uint16_t *p = &Is[(s * 32 + wc * 16 + fr) * RP + 8 + x0];
        uint4 d = *(const uint4 *)p;
        uint32_t e = *(const uint32_t *)(p + 8), f = *(const uint32_t *)(p - 2);
        if (yy < 0 || yy >= a.h) {
          d = make_uint4(0, 0, 0, 0);
          e = f = 0;
        }
        const uint32_t s1 = __builtin_amdgcn_alignbit(d.y, d.x, 16);
        const uint32_t s2 = __builtin_amdgcn_alignbit(d.z, d.y, 16);
        const uint32_t s3 = __builtin_amdgcn_alignbit(d.w, d.z, 16);
        const uint4 am = make_uint4(__builtin_amdgcn_alignbit(d.x, f, 16), s1, s2, s3);
        const uint4 ap = make_uint4(s1, s2, s3, __builtin_amdgcn_alignbit(e, d.w, 16));
        const bf16x8 fm = __builtin_bit_cast(bf16x8, am), f0 = __builtin_bit_cast(bf16x8, d),
                     fp = __builtin_bit_cast(bf16x8, ap);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          acc[3 * dy][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, fb[nt], acc[3 * dy][nt], 0, 0, 0);
          acc[3 * dy + 1][nt] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, fb[nt], acc[3 * dy + 1][nt], 0, 0, 0);
          acc[3 * dy + 2][nt] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(fp, fb[nt], acc[3 * dy + 2][nt], 0, 0, 0);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < IN_T; ++j) {
        const int q = tid + NTH * j;
        if (q < NIN) {
          const int cg = q & 3, quad = (q >> 2) % (W / 4), u = (q >> 2) / (W / 4);
          put(&Is[(slot_of(rb + U + 1 + u) * 32 + 8 * cg) * RP + 8 + 4 * quad], rin[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < GO_T; ++j) {
        const int q = tid + NTH * j;
        if (q < NGO) {
          const int cg = q % GCG, quad = (q / GCG) % (W / 4), u = q / GCG / (W / 4);
          put(&Gs[buf ^ 1][(u * NB + 8 * cg) * RP + 4 * quad], rgo[j]);
          if (do_bias) bias_add(rgo[j]);
        }
      }
    }
    __syncthreads();
  }

  // groups 1 .. KW - 1 hand their sums to group 0 through LDS, three taps
  // at a time (the ring is free after the loop's last barrier)
  if (KW > 1) {
    float *xch = (float *)Is;   // [group - 1][3 taps][NT][4][256 lanes]
    static_assert((KW - 1) * 3 * NT * 4 * 256 * 4 <= IS_EL * 2, "exchange fits the ring");
#pragma unroll
    for (int t0 = 0; t0 < 9; t0 += 3) {
      if (grp > 0)
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              xch[((((grp - 1) * 3 + t) * NT + nt) * 4 + e) * 256 + (tid & 255)] =
                  acc[t0 + t][nt][e];
      __syncthreads();
      if (grp == 0)
#pragma unroll
        for (int g = 1; g < KW; ++g)
#pragma unroll
          for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int e = 0; e < 4; ++e)
                acc[t0 + t][nt][e] += xch[((((g - 1) * 3 + t) * NT + nt) * 4 + e) * 256 + tid];
      __syncthreads();
    }
  }
  const int N = a.co;
  if (grp == 0) {
    float *dst = a.part + (size_t)z * 9 * a.ci * N;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = c0 + wc * 16 + (lane >> 4) * 4 + e;
          const int o = o0 + wn * 16 * NT + nt * 16 + (lane & 15);
          dst[(size_t)(t * a.ci + c) * N + o] = acc[t][nt][e];
        }
  }
  if (do_bias) {   // threads tid = g (mod GCG) hold channel group g
    float *red = (float *)Is;   // NTH x 9 floats; the last barrier has passed
    static_assert(NTH * 9 * 4 <= IS_EL * 2, "bias tree fits the ring");
#pragma unroll
    for (int j = 0; j < 8; ++j) red[tid * 9 + j] = bs[j];
    __syncthreads();
    for (int h = NTH / GCG / 2; h > 0; h >>= 1) {
      if (tid / GCG < h)
#pragma unroll
        for (int j = 0; j < 8; ++j) red[tid * 9 + j] += red[(tid + h * GCG) * 9 + j];
      __syncthreads();
    }
    if (tid < GCG)
#pragma unroll
      for (int j = 0; j < 8; ++j) bpart[(size_t)z * N + o0 + 8 * tid + j] = red[tid * 9 + j];
  }
}

// Transposed bf16 weight copies WT[t][o][c] = W[t][c][o] of up to 16
// convolutions at once (the parameter layout of the surrogate: conv k's
// weights at element off[k]).
struct ConvTable {
  int count;
  long long off[16];
  int ci[16], co[16];
};
__global__ void k_transpose_weights(const uint16_t *w, uint16_t *wt, ConvTable tb,
                                    long long total) {
  const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (g >= total) return;
  long long i = g;
  int k = 0;
  while (k < tb.count && i >= 9LL * tb.ci[k] * tb.co[k]) {
    i -= 9LL * tb.ci[k] * tb.co[k];
    ++k;
  }
  if (k >= tb.count) return;
  const int ci = tb.ci[k], co = tb.co[k];
  const int c = i % ci;
  const long long r = i / ci;
  const int o = r % co, t = r / co;
  wt[tb.off[k] + i] = w[tb.off[k] + ((long long)t * ci + c) * co + o];
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
#pragma unroll 8
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

// out[0] += the sum of part[0 .. nparts): one block, thread t adding
// part[t], part[t + 256], ... (loads in flight together), then a fixed LDS
// tree; the loss's per-block sums.
__global__ __launch_bounds__(256) void k_sum_scalar(const float *part, int nparts, float *out) {
  float s = 0.f;
#pragma unroll 8
  for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
  __shared__ float sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += sh[0];
}

// Partial sums of a layer's weight and bias gradients in one launch:
// out[i] (+)= sum over k of part[k][i] for each of two segments (blocks below
// s1.blocks take segment 1).  A thread adds 4 consecutive outputs (16-byte
// loads); the block's `groups` thread groups (a power of two dividing 256)
// take k = g, g + groups, ... in order and the group sums are added in
// group order, so the result is fixed for a given shape.  Many groups
// serve few outputs with many partials, one group many outputs.  n, the
// pointers' element offsets: multiples of 4.
struct SumSeg {
  const float *part;
  long long n;
  float *out;
  int groups, blocks;
  int add;   // 1: out += sum, 0: out = sum
};
__global__ __launch_bounds__(256) void k_sum_parts_v4(SumSeg s1, SumSeg s2, int nparts) {
  const bool first = (int)blockIdx.x < s1.blocks;
  const float *part = first ? s1.part : s2.part;
  float *out = first ? s1.out : s2.out;
  const long long n4 = (first ? s1.n : s2.n) / 4;
  const int G = first ? s1.groups : s2.groups, V = 256 / G;
  const bool add = first ? s1.add : s2.add;
  const int b = first ? blockIdx.x : blockIdx.x - s1.blocks;
  const int g = threadIdx.x / V, vi = threadIdx.x - g * V;
  const long long i = (long long)b * V + vi;   // vector index
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < n4) {
    const float4 *p4 = (const float4 *)part + i;
#pragma unroll 4
    for (int k = g; k < nparts; k += G) {
      const float4 v = p4[(size_t)k * n4];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
  }
  __shared__ float4 sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (g == 0 && i < n4) {
    float4 t = sh[vi];
    for (int q = 1; q < G; ++q) {
      const float4 v = sh[q * V + vi];
      t.x += v.x;
      t.y += v.y;
      t.z += v.z;
      t.w += v.w;
    }
    float4 *o = (float4 *)out + i;
    if (add) {
      const float4 r = *o;
      t.x += r.x;
      t.y += r.y;
      t.z += r.z;
      t.w += r.w;
    }
    *o = t;
  }
}

// Bias gradient, first half: part[block][o] = sum of GY[p][o] over the
// block's chunk of pixels (co a multiple of 8, at most 256; gs, go multiples
// of 8).  Thread t takes channels 8 (t % (co / 8)) .. + 7 of the pixels
// p0 + t / (co / 8), + 256 / (co / 8), ... with 16-byte loads (the 256
// threads cover whole pixel rows, so a wavefront reads contiguous memory),
// then the pixel groups are added in a fixed tree order.  k_sum_parts adds
// the chunks into gb.
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *g, int gs, int go, int npix,
                                                   int co, int chunk, float *part) {
  const int cv = co / 8, groups = 256 / cv;
  const int t = threadIdx.x, q = t % cv, grp = t / cv;
  const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, npix);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (grp < groups)
    for (int p = p0 + grp; p < p1; p += groups) {
      const uint4 v = *(const uint4 *)(g + (size_t)p * gs + go + 8 * q);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s[2 * j] += __uint_as_float(w[j] << 16);
        s[2 * j + 1] += __uint_as_float(w[j] & 0xFFFF0000u);
      }
    }
  __shared__ float sh[256][9];
#pragma unroll
  for (int j = 0; j < 8; ++j) sh[t][j] = s[j];
  __syncthreads();
  int top = 1;
  while (top < groups) top <<= 1;
  for (int h = top / 2; h > 0; h >>= 1) {   // fixed tree over the pixel groups
    if (grp < h && grp + h < groups)
#pragma unroll
      for (int j = 0; j < 8; ++j) sh[t][j] += sh[t + h * cv][j];
    __syncthreads();
  }
  if (grp == 0)
#pragma unroll
    for (int j = 0; j < 8; ++j) part[(size_t)blockIdx.x * co + 8 * q + j] = sh[t][j];
}

// Elementwise kernels over groups of 8 channels (16 bytes; channel counts,
// strides and offsets are multiples of 8): thread i takes group i % (c / 8)
// of pixel i / (c / 8).
struct Bf8 {
  uint16_t v[8];
};
__device__ __forceinline__ Bf8 ld8(const uint16_t *p) {
  Bf8 r;
  *(uint4 *)r.v = *(const uint4 *)p;
  return r;
}
__device__ __forceinline__ void st8(uint16_t *p, const Bf8 &r) { *(uint4 *)p = *(const uint4 *)r.v; }

// 2 x 2 average pooling (h, w: input size, even).
__global__ void k_pool_fwd(const uint16_t *x, int xs, int xo, int n, int h, int w, int c,
                           uint16_t *y) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int cg = c / 8, ho = h / 2, wo = w / 2;
  if (i >= (long long)n * ho * wo * cg) return;
  const int g = (int)(i % cg);
  const long long pix = i / cg;
  const int ox = (int)(pix % wo), oy = (int)((pix / wo) % ho), b = (int)(pix / ((long long)wo * ho));
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const Bf8 v = ld8(x + ((size_t)(b * h + 2 * oy + dy) * w + 2 * ox + dx) * xs + xo + 8 * g);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += bf2f(v.v[j]);
    }
  Bf8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.v[j] = f2bf(0.25f * s[j]);
  st8(y + pix * c + 8 * g, r);
}

// Gradient of the pooling, written into (or added to) a slice of gx; with
// mask set, zero where mask <= 0 (mask has gx's stride and offset: the ReLU
// of the layer that produced the pooled input; k_up_bwd likewise).
__global__ void k_pool_bwd(const uint16_t *gy, int n, int h, int w, int c, uint16_t *gx, int gxs,
                           int gxo, int accumulate, const uint16_t *mask) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int cg = c / 8;
  if (i >= (long long)n * h * w * cg) return;
  const int g = (int)(i % cg);
  const long long pix = i / cg;
  const int px = (int)(pix % w), py = (int)((pix / w) % h), b = (int)(pix / ((long long)w * h));
  const int ho = h / 2, wo = w / 2;
  const Bf8 v = ld8(gy + ((size_t)(b * ho + py / 2) * wo + px / 2) * c + 8 * g);
  uint16_t *o = gx + (size_t)pix * gxs + gxo + 8 * g;
  Bf8 old{};
  if (accumulate) old = ld8(o);
  Bf8 mk{};
  if (mask) mk = ld8(mask + (o - gx));
  Bf8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float t = 0.25f * bf2f(v.v[j]);
    if (accumulate) t += bf2f(old.v[j]);
    if (mask && !(bf2f(mk.v[j]) > 0.f)) t = 0.f;
    r.v[j] = f2bf(t);
  }
  st8(o, r);
}

// Nearest 2x upsampling (h, w: input size) into a channel slice of y.
__global__ void k_up_fwd(const uint16_t *x, int n, int h, int w, int c, uint16_t *y, int ys,
                         int yo) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int H = 2 * h, W = 2 * w, cg = c / 8;
  if (i >= (long long)n * H * W * cg) return;
  const int g = (int)(i % cg);
  const long long pix = i / cg;
  const int px = (int)(pix % W), py = (int)((pix / W) % H), b = (int)(pix / ((long long)W * H));
  st8(y + (size_t)pix * ys + yo + 8 * g,
      ld8(x + ((size_t)(b * h + py / 2) * w + px / 2) * c + 8 * g));
}

__global__ void k_up_bwd(const uint16_t *gy, int gys, int gyo, int n, int h, int w, int c,
                         uint16_t *gx, const uint16_t *mask) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int cg = c / 8;
  if (i >= (long long)n * h * w * cg) return;
  const int g = (int)(i % cg);
  const long long pix = i / cg;
  const int px = (int)(pix % w), py = (int)((pix / w) % h), b = (int)(pix / ((long long)w * h));
  const int W = 2 * w;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const Bf8 v =
          ld8(gy + ((size_t)(b * 2 * h + 2 * py + dy) * W + 2 * px + dx) * gys + gyo + 8 * g);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += bf2f(v.v[j]);
    }
  if (mask) {
    const Bf8 mk = ld8(mask + pix * c + 8 * g);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (!(bf2f(mk.v[j]) > 0.f)) s[j] = 0.f;
  }
  Bf8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.v[j] = f2bf(s[j]);
  st8(gx + pix * c + 8 * g, r);
}

// g *= (y > 0) over a channel slice [npix][c] of both tensors.
__global__ void k_relu_bwd(const uint16_t *y, int ys, int yo, uint16_t *g, int gs, int go,
                           long long npix, int c) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int cg = c / 8;
  if (i >= npix * cg) return;
  const long long p = i / cg;
  const int k = (int)(i % cg);
  const Bf8 yv = ld8(y + p * ys + yo + 8 * k);
  uint16_t *gp = g + p * gs + go + 8 * k;
  Bf8 gv = ld8(gp);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (!(bf2f(yv.v[j]) > 0.f)) gv.v[j] = 0;
  st8(gp, gv);
}

// Masked mean-squared error over the first `cu` (<= 8) channels of pred
// (stride ps): loss[block] = the block's sum of mask (pred - t)^2 / count
// (k_sum_parts adds the blocks); grad = 2 mask (pred - t) / count (bf16,
// dense: gs channels, zero beyond cu).  t: FP32 [npix][cu]; mask FP32
// [npix].  One thread per 16-byte vector of grad (gs / 8 per pixel, so a
// wavefront stores contiguous memory); the first of a pixel reads its first
// 8 channels of pred (ps a multiple of 8, 16-byte aligned) and does the sums.
__global__ __launch_bounds__(256) void k_mse(const uint16_t *pred, int ps, const float *t,
                                             const float *mask, long long npix, int cu,
                                             float inv_count, uint16_t *grad, int gs,
                                             float *loss) {
  const int vp = gs / 8;   // vectors per pixel
  const long long q = blockIdx.x * 256LL + threadIdx.x;
  float l = 0.f;
  if (q < npix * vp) {
    const long long p = q / vp;
    uint4 out = make_uint4(0, 0, 0, 0);
    if (q - p * vp == 0) {
      const float mk = mask[p];
      const Bf8 pv = ld8(pred + p * ps);
      Bf8 gv;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        float g = 0.f;
        if (ch < cu) {
          const float d = bf2f(pv.v[ch]) - t[p * cu + ch];
          l += mk * d * d;
          g = 2.f * mk * d * inv_count;
        }
        gv.v[ch] = f2bf(g);
      }
      out = *(const uint4 *)gv.v;
    }
    ((uint4 *)grad)[q] = out;
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
