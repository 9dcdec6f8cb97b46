// lbm_nn.hip -- the warm-start surrogate: BF16 MFMA layer kernels behind a
// C ABI, and a native driver of the whole network (forward, backward, Adam)
// (contracts in include/lbm.h, section "Learned warm start").
//
// Network (a 4-level U-Net on a 256 x 128 canvas, NHWC bf16, channel counts
// padded to multiples of 32):
//   level 0 (256 x 128): conv 5(32)->32, conv 32->32 = skip0
//   level 1 (128 x 64):  avgpool, conv 32->64, conv 64->64 = skip1
//   level 2 (64 x 32):   avgpool, conv 64->128, conv 128->128 = skip2
//   level 3 (32 x 16):   avgpool, conv 128->256, conv 256->256
//   decoder: nearest 2x up, concat skip, conv (256+128)->128, 128->128;
//            up, concat, (128+64)->64, 64->64; up, concat, (64+32)->32,
//            32->32; head conv 32->3 (stored as 32 output channels)
// All convolutions are 3 x 3 with zero padding, bias, ReLU except the head.
// Skip tensors live directly in their concatenation buffer's channel slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"
#include "nn_kernels.hpp"

using namespace lbm::nn;

namespace {

inline unsigned blocks_for(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Pixels per weight-gradient chunk: about 2048 blocks over the layer's
// (9 ci / 64) x (co / BN) output tiles, in multiples of 64 pixels, at least
// 256 (each chunk is one chain of dependent loads; more chains hide more
// latency, at the cost of more partials for k_sum_parts to add).
inline int wgrad_kchunk(int n, int h, int w, int ci, int co) {
  const long long npix = (long long)n * h * w;
  const long long tiles = (long long)((9 * ci + 63) / 64) * (co % 64 == 0 ? co / 64 : (co + 31) / 32);
  const long long nz = std::max(1LL, 2048 / tiles);
  long long k = (npix + nz - 1) / nz;
  k = (k + 63) / 64 * 64;
  return (int)std::max(256LL, k);
}

inline int wgrad_chunks(const ConvArgs &a) {
  return (int)(((long long)a.n * a.h * a.w + a.kchunk - 1) / a.kchunk);
}

// Strips of the row-streamed weight gradient (k_wgrad_rows): widths 16,
// 32, 64 and 128, an iteration of 256 pixels = U rows (U <= h), NT = 2
// (64-channel output tiles) where co allows.  A block of kRowsKW four-wave
// groups holds 170-180 VGPRs per lane, so one block fits per CU: strips
// of whole iterations, at most kRowsBlocks (the CU count) blocks over the
// (ci / 32) x (co / 32 NT) tiles where the tiles allow, as evenly filled as
// whole iterations allow (a 257th block would run after the others).
constexpr int kRowsKW = 2;
constexpr int kRowsPix = 256;
constexpr long long kRowsBlocks = 256;
struct RowsPlan {
  bool ok;
  int nt, rows, nz;
  int nz_bound;   // bound on nz over every n up to this one (partials sizing)
};
inline RowsPlan wgrad_rows_plan(int n, int h, int w, int ci, int co) {
  RowsPlan p{false, 1, 0, 0, 0};
  if (!(w == 16 || w == 32 || w == 64 || w == 128) || ci % 32 || co % 32) return p;
  const int U = kRowsPix / w;
  if (h < U) return p;
  p.nt = co % 64 == 0 ? 2 : 1;
  const long long tiles = (long long)(ci / 32) * (co / (32 * p.nt));
  const long long nrow = (long long)n * h;
  long long nz = std::max(1LL, kRowsBlocks / tiles);
  nz = std::min(nz, (nrow + U - 1) / U);   // grows with n; p.nz <= it
  p.nz_bound = (int)nz;
  long long rows = (nrow + nz - 1) / nz;
  rows = (rows + U - 1) / U * U;
  p.rows = (int)rows;
  p.nz = (int)((nrow + rows - 1) / rows);
  p.ok = true;
  return p;
}

// One segment of k_sum_parts_v4: groups per output vector chosen so that
// about 64 k threads run (at most 16 groups, at most the number of parts).
inline SumSeg sum_seg(const float *part, long long n, float *out, int nparts, bool add) {
  const long long n4 = n / 4;
  int g = 1;
  while (g < 16 && g < nparts && n4 * g < 65536) g *= 2;
  const int V = 256 / g;
  return SumSeg{part, n, out, g, (int)((n4 + V - 1) / V), add ? 1 : 0};
}

template <int W, int U>
void wgrad_rows(const ConvArgs &a, const RowsPlan &p, float *bpart, hipStream_t st) {
  const unsigned grid = (unsigned)((a.ci / 32) * (a.co / (32 * p.nt)) * p.nz);
  if (p.nt == 2)
    hipLaunchKernelGGL((k_wgrad_rows<W, U, 2, kRowsKW>), dim3(grid), dim3(256 * kRowsKW), 0, st, a,
                       p.rows, bpart);
  else
    hipLaunchKernelGGL((k_wgrad_rows<W, U, 1, kRowsKW>), dim3(grid), dim3(256 * kRowsKW), 0, st, a,
                       p.rows, bpart);
}

hipError_t wgrad_launch(const ConvArgs &a, float *gbias, hipStream_t st, bool add = true);

// One forward or input-gradient pass with tile shape <WM, WN, TM, TN>.
template <int MODE, int WM, int WN, int TM, int TN>
void conv_mn(const ConvArgs &a, int M, int N, hipStream_t st) {
  constexpr int BM = 16 * WM * TM, BN = 16 * WN * TN;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN);
  hipLaunchKernelGGL((k_conv_mn<MODE, WM, WN, TM, TN>), grid, dim3(256), 0, st, a);
}

// Tile shape for an M x N product: N tiles as wide as the channel count
// allows (no MFMA on padding), and the larger M tile while it still gives
// at least two blocks per CU.
// Persistent patch-kernel blocks: two per CU (their LDS and registers allow
// two), each walking its share of the tiles.
constexpr int kPatchBlocks = 2 * 256;

template <int MODE, int W, int BN>
void conv_patch(const ConvArgs &a, int M, int N, hipStream_t st) {
  constexpr int TPIX = W == 128 ? 256 : W == 16 ? 64 : 128;   // as in k_conv_patch
  const int ntiles = M / TPIX * ((N + BN - 1) / BN);
  const int grid = std::min(ntiles, kPatchBlocks);
  hipLaunchKernelGGL((k_conv_patch<MODE, W, BN>), dim3(grid), dim3(256), 0, st, a, ntiles);
}

// Whether conv_fd takes the patch kernel for a w x h image: whole-row tiles
// (2 rows at widths 128 and 64, 4 at 32 and 16) and 16-byte output vectors.
inline bool patch_path(int w, int h, int os, int oo) {
  if (os % 8 || oo % 8) return false;
  return ((w == 128 || w == 64) && h % 2 == 0) || ((w == 32 || w == 16) && h % 4 == 0);
}

template <int MODE>
void conv_fd(const ConvArgs &a, hipStream_t st) {
  const int M = a.n * a.h * a.w, N = MODE == FWD ? a.co : a.ci;
  // direct convolution from an LDS patch of whole rows: 256-pixel tiles of
  // 32 channels on 128-wide images, 128-pixel tiles on 64- and 32-wide
  // ones, 64-pixel tiles on 16-wide ones (64 channels where N allows)
  // (the forward patch kernel reads the transposed weight copy a.wtt)
  const bool out_ok = patch_path(a.w, a.h, a.os, a.oo) && (MODE != FWD || a.wtt);
  const bool n64 = N % 64 == 0;
  if (out_ok && a.w == 128 && a.h % 2 == 0) {
    conv_patch<MODE, 128, 32>(a, M, N, st);
    return;
  }
  if (out_ok && a.w == 64 && a.h % 2 == 0) {
    if (n64) conv_patch<MODE, 64, 64>(a, M, N, st);
    else conv_patch<MODE, 64, 32>(a, M, N, st);
    return;
  }
  if (out_ok && a.w == 32 && a.h % 4 == 0) {
    if (n64) conv_patch<MODE, 32, 64>(a, M, N, st);
    else conv_patch<MODE, 32, 32>(a, M, N, st);
    return;
  }
  if (out_ok && a.w == 16 && a.h % 4 == 0) {
    if (n64) conv_patch<MODE, 16, 64>(a, M, N, st);
    else conv_patch<MODE, 16, 32>(a, M, N, st);
    return;
  }
  const long long big = 512;
  if (N % 128 == 0) {
    if ((long long)((M + 127) / 128) * (N / 128) >= big)
      conv_mn<MODE, 2, 2, 4, 4>(a, M, N, st);          // 128 x 128
    else if ((long long)((M + 63) / 64) * (N / 128) >= big / 2)
      conv_mn<MODE, 2, 2, 2, 4>(a, M, N, st);          // 64 x 128
    else
      conv_mn<MODE, 2, 2, 2, 2>(a, M, N, st);          // 64 x 64
  } else if (N % 64 == 0) {
    if ((long long)((M + 127) / 128) * (N / 64) >= big)
      conv_mn<MODE, 4, 1, 2, 4>(a, M, N, st);          // 128 x 64
    else
      conv_mn<MODE, 2, 2, 2, 2>(a, M, N, st);          // 64 x 64
  } else {
    if ((long long)((M + 255) / 256) * (N / 32) >= big)
      conv_mn<MODE, 4, 1, 4, 2>(a, M, N, st);          // 256 x 32
    else
      conv_mn<MODE, 4, 1, 2, 2>(a, M, N, st);          // 128 x 32
  }
}

// Weight gradient by k_wgrad: 64 x BN tiles of the [9 ci][co] result over
// pixel chunks, per-chunk partials added into GW in chunk order.
hipError_t wgrad_tiles_launch(const ConvArgs &a, hipStream_t st) {
  const int nz = wgrad_chunks(a);
  if (a.co % 64 == 0) {
    dim3 grid((9 * a.ci + 63) / 64, a.co / 64, nz);
    hipLaunchKernelGGL(k_wgrad<64>, grid, dim3(256), 0, st, a);
  } else {
    dim3 grid((9 * a.ci + 63) / 64, (a.co + 31) / 32, nz);
    hipLaunchKernelGGL(k_wgrad<32>, grid, dim3(256), 0, st, a);
  }
  const long long mn = 9LL * a.ci * a.co;
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(mn, kSumOut)), dim3(256), 0, st, a.part, nz,
                     mn, (float *)a.out);
  return hipGetLastError();
}

hipError_t conv_launch(int mode, const ConvArgs &a, hipStream_t st) {
  if (mode == FWD) {
    conv_fd<FWD>(a, st);
  } else if (mode == DGRAD) {
    conv_fd<DGRAD>(a, st);
  } else {
    return wgrad_launch(a, nullptr, st);
  }
  return hipGetLastError();
}

// Bias gradient: per-chunk sums into part [blocks][co], then added into gb in
// chunk order.
hipError_t bias_grad_launch(const uint16_t *g, int gs, int go, long long npix, int co,
                            float *part, float *gb, hipStream_t st) {
  const int chunk = 512, nb = (int)blocks_for(npix, chunk);
  hipLaunchKernelGGL(k_bias_grad, dim3(nb), dim3(256), 0, st, g, gs, go, (int)npix, co, chunk,
                     part);
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(co, kSumOut)), dim3(256), 0, st, part, nb,
                     (long long)co, gb);
  return hipGetLastError();
}

// Weight gradient of a layer into a.out (FP32 [9 ci][co]), and with gbias
// set also its bias gradient into gbias, added to what they hold (add) or
// replacing it: k_wgrad_rows where the width allows (the bias sums then
// ride along with its loads of GY), else k_wgrad and k_bias_grad.  Partials
// in a.part (wgrad_part_floats).
hipError_t wgrad_launch(const ConvArgs &a, float *gbias, hipStream_t st, bool add) {
  const RowsPlan p = wgrad_rows_plan(a.n, a.h, a.w, a.ci, a.co);
  const bool v4 = (uintptr_t)a.out % 16 == 0 && (!gbias || (uintptr_t)gbias % 16 == 0);
  if (!add && !(p.ok && v4)) {   // the paths below add: clear the targets first
    hipError_t e = hipMemsetAsync(a.out, 0, sizeof(float) * 9 * a.ci * a.co, st);
    if (e == hipSuccess && gbias) e = hipMemsetAsync(gbias, 0, sizeof(float) * a.co, st);
    if (e != hipSuccess) return e;
  }
  if (!p.ok) {
    hipError_t e = wgrad_tiles_launch(a, st);
    if (e == hipSuccess && gbias)
      e = bias_grad_launch(a.g, a.gs, a.go, (long long)a.n * a.h * a.w, a.co, a.part, gbias, st);
    return e;
  }
  const long long mn = 9LL * a.ci * a.co;
  float *bpart = gbias ? a.part + (size_t)p.nz * mn : nullptr;
  switch (a.w) {
    case 16: wgrad_rows<16, kRowsPix / 16>(a, p, bpart, st); break;
    case 32: wgrad_rows<32, kRowsPix / 32>(a, p, bpart, st); break;
    case 64: wgrad_rows<64, kRowsPix / 64>(a, p, bpart, st); break;
    default: wgrad_rows<128, kRowsPix / 128>(a, p, bpart, st); break;
  }
  if (v4) {   // mn and co are multiples of 4 (channel counts multiples of 32)
    const SumSeg s1 = sum_seg(a.part, mn, (float *)a.out, p.nz, add);
    const SumSeg s2 =
        gbias ? sum_seg(bpart, a.co, gbias, p.nz, add) : SumSeg{nullptr, 0, nullptr, 1, 0, 0};
    hipLaunchKernelGGL(k_sum_parts_v4, dim3(s1.blocks + s2.blocks), dim3(256), 0, st, s1, s2,
                       p.nz);
  } else {
    hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(mn, kSumOut)), dim3(256), 0, st, a.part, p.nz,
                       mn, (float *)a.out);
    if (gbias)
      hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(a.co, kSumOut)), dim3(256), 0, st, bpart,
                         p.nz, (long long)a.co, gbias);
  }
  return hipGetLastError();
}

// Floats of partials a weight or bias gradient needs.
size_t wgrad_part_floats(int n, int h, int w, int ci, int co) {
  const long long npix = (long long)n * h * w;
  const int kc = wgrad_kchunk(n, h, w, ci, co);
  const size_t wg = (size_t)((npix + kc - 1) / kc) * 9 * ci * co;
  const size_t bg = (size_t)blocks_for(npix, 256) * co;
  const RowsPlan p = wgrad_rows_plan(n, h, w, ci, co);
  const size_t rg = p.ok ? (size_t)p.nz_bound * (9LL * ci * co + co) : 0;
  return std::max(std::max(wg, bg), rg);
}

bool chan_ok(int c) { return c >= 32 && c <= 1024 && c % 32 == 0; }

// ------------------------------------------------------------------ network
constexpr int kH = 256, kW = 128;   // canvas rows (y) x columns (x)
constexpr int kInCh = 5, kOutCh = 3;

struct View {
  int buf;      // index into the activation arena list
  int cs, co;   // channel stride, channel offset
};

enum OpType { OP_CONV, OP_POOL, OP_UP };

struct Op {
  OpType type;
  int level;            // spatial level of the input
  int ci, co, relu;     // conv: channels in/out; pool/up: channels = ci
  View in, out;
  size_t woff, boff;    // conv parameter offsets (floats)
};

struct Buf {
  int level, ch;
};

}  // namespace

struct lbm_surrogate {
  int nmax = 0;
  std::vector<Buf> bufs;
  std::vector<Op> ops;
  size_t nparams = 0;
  std::vector<size_t> act_off;   // element offsets of each buffer (per batch of nmax)
  size_t act_elems = 0;
  uint16_t *act = nullptr, *gact = nullptr;     // activations and their gradients
  float *w = nullptr, *m = nullptr, *v = nullptr, *gw = nullptr;   // FP32 params
  uint16_t *wb = nullptr;                        // bf16 copy of the params
  uint16_t *wbt = nullptr;                       // bf16 conv weights as [9][co][ci]
  ConvTable convs{};                             // offsets and shapes of the convs
  float *target = nullptr, *mask = nullptr, *out3 = nullptr;
  float *loss_dev = nullptr, *loss_host = nullptr;
  float *part = nullptr;   // partials of the split reductions (see k_sum_parts)
  // ReLU gradients fused into the pass that writes the last contribution to
  // a ReLU conv's output gradient: mask_of[j] = that conv for op j (else -1),
  // relu_fused[p] set for such a conv p (its separate ReLU pass is skipped)
  std::vector<int> mask_of;
  std::vector<char> relu_fused;
  // forward: pool / upsample ops written by the epilogue of the conv before
  // them (fwd_into[p] = that op for conv p, else -1; fwd_fused[j] set)
  std::vector<int> fwd_into;
  std::vector<char> fwd_fused;
  double *rearr = nullptr;                       // [2 nmax] (Re, Ar)
  double *field = nullptr;                       // warm-start fields
  size_t field_doubles = 0;
  int64_t adam_t = 0;
  hipStream_t stream = nullptr, own_stream = nullptr;
  // weight gradients run on a stream of their own, forked from `stream`
  // once a layer's output gradient is complete and joined at the end of the
  // backward pass: no later kernel reads them before the join, and the
  // input-gradient chain does not wait for them
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

int level_h(int l) { return kH >> l; }
int level_w(int l) { return kW >> l; }

int add_buf(lbm_surrogate *s, int level, int ch) {
  s->bufs.push_back({level, ch});
  return (int)s->bufs.size() - 1;
}

void add_conv(lbm_surrogate *s, int level, int ci, int co, int relu, View in, View out) {
  Op o;
  o.type = OP_CONV;
  o.level = level;
  o.ci = ci;
  o.co = co;
  o.relu = relu;
  o.in = in;
  o.out = out;
  o.woff = s->nparams;
  s->nparams += (size_t)9 * ci * co;
  o.boff = s->nparams;
  s->nparams += co;
  s->ops.push_back(o);
}

void add_pool(lbm_surrogate *s, int level, int c, View in, View out) {
  Op o{};
  o.type = OP_POOL;
  o.level = level;
  o.ci = o.co = c;
  o.in = in;
  o.out = out;
  s->ops.push_back(o);
}

void add_up(lbm_surrogate *s, int level, int c, View in, View out) {
  Op o{};
  o.type = OP_UP;
  o.level = level;   // level of the (low-resolution) input
  o.ci = o.co = c;
  o.in = in;
  o.out = out;
  s->ops.push_back(o);
}

void build_net(lbm_surrogate *s) {
  const int X0 = add_buf(s, 0, 32), A0 = add_buf(s, 0, 32), C0 = add_buf(s, 0, 96);
  const int P0 = add_buf(s, 1, 32), A1 = add_buf(s, 1, 64), C1 = add_buf(s, 1, 192);
  const int P1 = add_buf(s, 2, 64), A2 = add_buf(s, 2, 128), C2 = add_buf(s, 2, 384);
  const int P2 = add_buf(s, 3, 128), B0 = add_buf(s, 3, 256), B1 = add_buf(s, 3, 256);
  const int D2a = add_buf(s, 2, 128), D2b = add_buf(s, 2, 128);
  const int D1a = add_buf(s, 1, 64), D1b = add_buf(s, 1, 64);
  const int D0a = add_buf(s, 0, 32), D0b = add_buf(s, 0, 32), Y = add_buf(s, 0, 32);
  auto full = [&](int b) { return View{b, s->bufs[b].ch, 0}; };
  add_conv(s, 0, 32, 32, 1, full(X0), full(A0));
  add_conv(s, 0, 32, 32, 1, full(A0), View{C0, 96, 64});
  add_pool(s, 0, 32, View{C0, 96, 64}, full(P0));
  add_conv(s, 1, 32, 64, 1, full(P0), full(A1));
  add_conv(s, 1, 64, 64, 1, full(A1), View{C1, 192, 128});
  add_pool(s, 1, 64, View{C1, 192, 128}, full(P1));
  add_conv(s, 2, 64, 128, 1, full(P1), full(A2));
  add_conv(s, 2, 128, 128, 1, full(A2), View{C2, 384, 256});
  add_pool(s, 2, 128, View{C2, 384, 256}, full(P2));
  add_conv(s, 3, 128, 256, 1, full(P2), full(B0));
  add_conv(s, 3, 256, 256, 1, full(B0), full(B1));
  add_up(s, 3, 256, full(B1), View{C2, 384, 0});
  add_conv(s, 2, 384, 128, 1, full(C2), full(D2a));
  add_conv(s, 2, 128, 128, 1, full(D2a), full(D2b));
  add_up(s, 2, 128, full(D2b), View{C1, 192, 0});
  add_conv(s, 1, 192, 64, 1, full(C1), full(D1a));
  add_conv(s, 1, 64, 64, 1, full(D1a), full(D1b));
  add_up(s, 1, 64, full(D1b), View{C0, 96, 0});
  add_conv(s, 0, 96, 32, 1, full(C0), full(D0a));
  add_conv(s, 0, 32, 32, 1, full(D0a), full(D0b));
  add_conv(s, 0, 32, 32, 0, full(D0b), full(Y));
}

uint16_t *bptr(lbm_surrogate *s, uint16_t *base, const View &v) {
  return base + s->act_off[v.buf];
}

// Encode (Re, Ar) pairs into the input canvas: channel 0 = cavity mask
// (rows y < round(128 Ar)), 1 = (x + 1/2)/128, 2 = (y + 1/2)/128,
// 3 = Re / 3000, 4 = Ar / 2, channels 5-31 zero.
// One thread per 16-byte vector (8 channels) of a pixel, so a wavefront
// stores 1 KB of contiguous memory: vector 0 holds channels 0-4, vectors 1-3
// are zero.
__global__ void k_encode(const double *ra, int n, uint16_t *x) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= (long long)n * kH * kW * 4) return;
  const long long i = t >> 2;   // pixel
  uint4 v = make_uint4(0, 0, 0, 0);
  if ((t & 3) == 0) {
    const int b = i / (kH * kW), r = i % (kH * kW), y = r / kW, xx = r % kW;
    const double re = ra[2 * b], ar = ra[2 * b + 1];
    const int ny = (int)rint(128.0 * ar);
    const float ch[kInCh] = {y < ny ? 1.f : 0.f, (xx + 0.5f) / 128.f, (y + 0.5f) / 128.f,
                             (float)(re / 3000.0), (float)(ar / 2.0)};
    static_assert(kInCh == 5, "channels 0-4 packed below");
    v = make_uint4(f2bf(ch[0]) | ((uint32_t)f2bf(ch[1]) << 16),
                   f2bf(ch[2]) | ((uint32_t)f2bf(ch[3]) << 16), f2bf(ch[4]), 0);
  }
  ((uint4 *)x)[t] = v;   // the canvas is dense, 32 channels
}

// Head output channels 0..2 -> FP32 [n][H][W][3].
__global__ void k_extract(const uint16_t *y, long long npix, float *out) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= npix * kOutCh) return;
  out[i] = bf2f(y[(i / kOutCh) * 32 + i % kOutCh]);
}

// Bilinear map of sample 0's prediction (rows < ny_c of the canvas) onto an
// nx x ny lattice: site (i, j) at ((i + 1/2)/nx, (j + 1/2)/nx) in units of L
// reads canvas position ((i + 1/2) 128/nx - 1/2, (j + 1/2) 128/nx - 1/2),
// clamped to the cavity's pixel centres.  Output rho = 1 + c0 / 100,
// u = u_lid c1, v = u_lid c2 (FP64 [ny][nx] each).
__global__ void k_to_lattice(const float *p3, int ny_c, int nx, int ny, double u_lid,
                             double *rho, double *ux, double *uy) {
  const long long k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= (long long)nx * ny) return;
  const int j = k / nx, i = k % nx;
  double X = (i + 0.5) * 128.0 / nx - 0.5, Y = (j + 0.5) * 128.0 / nx - 0.5;
  X = fmin(fmax(X, 0.0), 127.0);
  Y = fmin(fmax(Y, 0.0), (double)(ny_c - 1));
  int x0 = (int)floor(X), y0 = (int)floor(Y);
  if (x0 > 126) x0 = 126;
  if (y0 > ny_c - 2) y0 = max(ny_c - 2, 0);
  const int x1 = x0 + 1, y1 = min(y0 + 1, ny_c - 1);
  const double tx = X - x0, ty = Y - y0;
  double v[3];
  for (int c = 0; c < 3; ++c) {
    auto at = [&](int yy, int xx) { return (double)p3[((size_t)yy * kW + xx) * 3 + c]; };
    v[c] = (1 - tx) * (1 - ty) * at(y0, x0) + tx * (1 - ty) * at(y0, x1) +
           (1 - tx) * ty * at(y1, x0) + tx * ty * at(y1, x1);
  }
  rho[k] = 1.0 + v[0] / 100.0;
  ux[k] = u_lid * v[1];
  uy[k] = u_lid * v[2];
}

int forward(lbm_surrogate *s, int n) {
  hipStream_t st = s->stream;
  for (const Op &o : s->ops) {
    const int h = level_h(o.level), w = level_w(o.level);
    if (o.type == OP_CONV) {
      ConvArgs a{};
      a.n = n;
      a.h = h;
      a.w = w;
      a.ci = o.ci;
      a.co = o.co;
      a.x = bptr(s, s->act, o.in);
      a.xs = o.in.cs;
      a.xo = o.in.co;
      a.wt = s->wb + o.woff;
      a.wtt = s->wbt + o.woff;
      a.bias = s->w + o.boff;
      a.relu = o.relu;
      a.out = bptr(s, s->act, o.out);
      a.os = o.out.cs;
      a.oo = o.out.co;
      const int j = s->fwd_into[&o - s->ops.data()];
      if (j >= 0 && s->ops[j].type == OP_POOL) {
        a.pool_out = bptr(s, s->act, s->ops[j].out);
      } else if (j >= 0) {
        a.up_out = bptr(s, s->act, s->ops[j].out);
        a.ups = s->ops[j].out.cs;
        a.upo = s->ops[j].out.co;
      }
      HIPC(conv_launch(FWD, a, st));
    } else if (s->fwd_fused[&o - s->ops.data()]) {
      continue;   // written by the conv before it
    } else if (o.type == OP_POOL) {
      hipLaunchKernelGGL(k_pool_fwd, dim3(blocks_for((long long)n * h * w * o.ci / 32)), dim3(256),
                         0, st, bptr(s, s->act, o.in), o.in.cs, o.in.co, n, h, w, o.ci,
                         bptr(s, s->act, o.out));
      HIPC(hipGetLastError());
    } else {
      hipLaunchKernelGGL(k_up_fwd, dim3(blocks_for((long long)n * 4 * h * w * o.ci / 8)), dim3(256), 0,
                         st, bptr(s, s->act, o.in), n, h, w, o.ci, bptr(s, s->act, o.out),
                         o.out.cs, o.out.co);
      HIPC(hipGetLastError());
    }
  }
  return LBM_OK;
}

// For each ReLU conv p: its output gradient is complete once the consumer
// with the smallest op index (the last one the backward pass visits) has
// written or added its part.  If that consumer reads exactly p's output view,
// its backward pass applies p's ReLU mask while writing (same bits as a
// separate pass: the masked values are zero before rounding).
void plan_relu_masks(lbm_surrogate *s) {
  const int nop = (int)s->ops.size();
  s->mask_of.assign(nop, -1);
  s->relu_fused.assign(nop, 0);
  for (int p = 0; p < nop; ++p) {
    const Op &o = s->ops[p];
    if (o.type != OP_CONV || !o.relu) continue;
    int last = -1;
    for (int j = p + 1; j < nop && last < 0; ++j) {
      const View &v = s->ops[j].in;
      if (v.buf == o.out.buf && v.co < o.out.co + o.co && o.out.co < v.co + s->ops[j].ci) last = j;
    }
    if (last < 0) continue;
    const Op &q = s->ops[last];
    if (q.in.cs == o.out.cs && q.in.co == o.out.co && q.ci == o.co) {
      s->mask_of[last] = p;
      s->relu_fused[p] = 1;
    }
  }
}

// A pool or upsample op that reads exactly the output of the conv just
// before it is done by that conv's forward epilogue (patch kernel only).
void plan_fwd_fusion(lbm_surrogate *s) {
  const int nop = (int)s->ops.size();
  s->fwd_into.assign(nop, -1);
  s->fwd_fused.assign(nop, 0);
  for (int p = 0; p + 1 < nop; ++p) {
    const Op &o = s->ops[p], &q = s->ops[p + 1];
    if (o.type != OP_CONV || q.type == OP_CONV) continue;
    if (!patch_path(level_w(o.level), level_h(o.level), o.out.cs, o.out.co)) continue;
    if (q.in.buf != o.out.buf || q.in.cs != o.out.cs || q.in.co != o.out.co || q.ci != o.co)
      continue;
    // the pool writes a dense tensor of the conv's channels; the upsample
    // writes 16-byte vectors of a slice
    if (q.type == OP_POOL && (q.out.cs != o.co || q.out.co != 0)) continue;
    if (q.type == OP_UP && (q.out.cs % 8 || q.out.co % 8)) continue;
    s->fwd_into[p] = p + 1;
    s->fwd_fused[p + 1] = 1;
  }
}

int backward(lbm_surrogate *s, int n) {
  hipStream_t st = s->stream;
  // the main stream waits for the side stream however the pass ends
  struct Join {
    lbm_surrogate *s;
    ~Join() {
      if (hipEventRecord(s->join, s->side) == hipSuccess)
        (void)hipStreamWaitEvent(s->stream, s->join, 0);
    }
  } join{s};
  // every conv's weight and bias gradients are written once (not added)
  for (int k = (int)s->ops.size() - 1; k >= 0; --k) {
    const Op &o = s->ops[k];
    const int h = level_h(o.level), w = level_w(o.level);
    if (o.type == OP_CONV) {
      const long long npix = (long long)n * h * w;
      uint16_t *gy = bptr(s, s->gact, o.out);
      if (o.relu && !s->relu_fused[k]) {
        hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(npix * o.co / 8)), dim3(256), 0, st,
                           bptr(s, s->act, o.out), o.out.cs, o.out.co, gy, o.out.cs, o.out.co,
                           npix, o.co);
        HIPC(hipGetLastError());
      }
      ConvArgs a{};
      a.n = n;
      a.h = h;
      a.w = w;
      a.ci = o.ci;
      a.co = o.co;
      a.x = bptr(s, s->act, o.in);
      a.xs = o.in.cs;
      a.xo = o.in.co;
      a.g = gy;
      a.gs = o.out.cs;
      a.go = o.out.co;
      a.out = s->gw + o.woff;
      a.kchunk = wgrad_kchunk(n, h, w, o.ci, o.co);
      a.part = s->part;   // used by the side stream only until the join
      HIPC(hipEventRecord(s->fork, st));
      HIPC(hipStreamWaitEvent(s->side, s->fork, 0));
      HIPC(wgrad_launch(a, s->gw + o.boff, s->side, false));
      if (k > 0) {   // the network input needs no gradient
        ConvArgs d{};
        d.n = n;
        d.h = h;
        d.w = w;
        d.ci = o.ci;
        d.co = o.co;
        d.x = gy;
        d.xs = o.out.cs;
        d.xo = o.out.co;
        d.wt = s->wb + o.woff;
        d.out = bptr(s, s->gact, o.in);
        d.os = o.in.cs;
        d.oo = o.in.co;
        d.accumulate = 0;
        d.mask = s->mask_of[k] >= 0 ? bptr(s, s->act, o.in) : nullptr;
        HIPC(conv_launch(DGRAD, d, st));
      }
    } else if (o.type == OP_POOL) {
      // skip slice: add to the gradient the decoder already wrote there
      hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for((long long)n * h * w * o.ci / 8)), dim3(256), 0,
                         st, bptr(s, s->gact, o.out), n, h, w, o.ci, bptr(s, s->gact, o.in),
                         o.in.cs, o.in.co, 1,
                         s->mask_of[k] >= 0 ? bptr(s, s->act, o.in) : nullptr);
      HIPC(hipGetLastError());
    } else {
      hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for((long long)n * h * w * o.ci / 8)), dim3(256), 0, st,
                         bptr(s, s->gact, o.out), o.out.cs, o.out.co, n, h, w, o.ci,
                         bptr(s, s->gact, o.in),
                         s->mask_of[k] >= 0 ? bptr(s, s->act, o.in) : nullptr);
      HIPC(hipGetLastError());
    }
  }
  return LBM_OK;
}

const View &head_view(lbm_surrogate *s) { return s->ops.back().out; }

// Refresh the transposed bf16 weights after the bf16 copy changed.
hipError_t transpose_weights(lbm_surrogate *s) {
  long long total = 0;
  for (int k = 0; k < s->convs.count; ++k) total += 9LL * s->convs.ci[k] * s->convs.co[k];
  hipLaunchKernelGGL(k_transpose_weights, dim3(blocks_for(total)), dim3(256), 0, s->stream,
                     s->wb, s->wbt, s->convs, total);
  return hipGetLastError();
}

int encode(lbm_surrogate *s, int n, const double *re, const double *ar) {
  std::vector<double> ra(2 * n);
  for (int b = 0; b < n; ++b) {
    if (!(re[b] > 0.0) || !(ar[b] > 0.0) || !std::isfinite(re[b]) || 128.0 * ar[b] > kH + 0.5)
      return lbm_fail(LBM_EINVAL, "sample %d: Re = %g, Ar = %g outside (0, inf) x (0, 2]", b,
                      re[b], ar[b]);
    ra[2 * b] = re[b];
    ra[2 * b + 1] = ar[b];
  }
  HIPC(hipMemcpyAsync(s->rearr, ra.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice,
                      s->stream));
  const View x0{0, 32, 0};
  hipLaunchKernelGGL(k_encode, dim3(blocks_for((long long)n * kH * kW * 4)), dim3(256), 0, s->stream,
                     s->rearr, n, bptr(s, s->act, x0));
  HIPC(hipGetLastError());
  return LBM_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------ layer kernels
int lbm_nn_conv3x3(int mode, int n, int h, int w, int ci, int co, const void *x, int xs, int xo,
                   const void *g, int gs, int go, const void *wt, const float *bias, int relu,
                   void *out, int os, int oo, int accumulate, void *stream) {
  if (mode < 0 || mode > 2) return lbm_fail(LBM_EINVAL, "mode %d", mode);
  if (n < 1 || h < 1 || w < 1 || !chan_ok(ci) || !chan_ok(co))
    return lbm_fail(LBM_EINVAL, "bad shape n %d h %d w %d ci %d co %d", n, h, w, ci, co);
  if (!x || !out || (mode != WGRAD && !wt) || (mode == WGRAD && !g))
    return lbm_fail(LBM_EINVAL, "NULL tensor");
  ConvArgs a{};
  a.n = n;
  a.h = h;
  a.w = w;
  a.ci = ci;
  a.co = co;
  a.x = (const uint16_t *)x;
  a.xs = xs;
  a.xo = xo;
  a.g = (const uint16_t *)g;
  a.gs = gs;
  a.go = go;
  a.wt = (const uint16_t *)wt;
  a.bias = bias;
  a.relu = relu;
  a.out = out;
  a.os = os;
  a.oo = oo;
  a.accumulate = accumulate;
  a.kchunk = wgrad_kchunk(n, h, w, ci, co);
  const int cin = mode == DGRAD ? co : ci, cout = mode == DGRAD ? ci : co;
  if (mode != WGRAD && (xs < cin || xo < 0 || xo + cin > xs || xs % 8 || xo % 8 || os < cout ||
                        oo < 0 || oo + cout > os))
    return lbm_fail(LBM_EINVAL, "bad channel stride / offset");
  if (mode == WGRAD && (xs % 8 || xo % 8 || xo < 0 || xo + ci > xs || gs % 8 || go % 8 ||
                        go < 0 || go + co > gs))
    return lbm_fail(LBM_EINVAL, "bad channel stride / offset");
  if (mode == DGRAD) {
    HIPC(conv_launch(mode, a, (hipStream_t)stream));
    return LBM_OK;
  }
  if (mode == FWD) {   // the weights transposed in a workspace of this call
    uint16_t *wtt = nullptr;
    HIPC(hipMalloc(&wtt, sizeof(uint16_t) * 9 * (size_t)ci * co));
    ConvTable tb{};
    tb.count = 1;
    tb.ci[0] = ci;
    tb.co[0] = co;
    const long long total = 9LL * ci * co;
    hipLaunchKernelGGL(k_transpose_weights, dim3(blocks_for(total)), dim3(256), 0,
                       (hipStream_t)stream, (const uint16_t *)wt, wtt, tb, total);
    a.wtt = wtt;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = conv_launch(mode, a, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(wtt);
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "%s", hipGetErrorString(e));
    return LBM_OK;
  }
  // WGRAD: partials in a workspace of this call, freed once the work is done
  float *part = nullptr;
  HIPC(hipMalloc(&part, sizeof(float) * wgrad_part_floats(n, h, w, ci, co)));
  a.part = part;
  hipError_t e = conv_launch(mode, a, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(part);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "%s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_nn_bias_grad(int npix, int co, const void *g, int gs, int go, float *gb, void *stream) {
  if (npix < 1 || co < 8 || co > 256 || co % 8 || gs < co || gs % 8 || go < 0 || go % 8 ||
      go + co > gs || !g || !gb || (uintptr_t)g % 16)
    return lbm_fail(LBM_EINVAL,
                    "bad arguments (co a multiple of 8 in [8, 256], gs and go multiples of 8, "
                    "g 16-byte aligned)");
  float *part = nullptr;
  HIPC(hipMalloc(&part, sizeof(float) * (size_t)blocks_for(npix, 256) * co));
  hipError_t e = bias_grad_launch((const uint16_t *)g, gs, go, npix, co, part, gb,
                                  (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(part);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "%s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_nn_pool2(int backward, int n, int h, int w, int c, const void *in, int is, int io,
                 void *out, int os, int oo, int accumulate, void *stream) {
  if (n < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 8 || c % 8 || is % 8 || io % 8 ||
      os % 8 || oo % 8 || !in || !out)
    return lbm_fail(LBM_EINVAL, "bad pool arguments (c, strides and offsets multiples of 8)");
  hipStream_t st = (hipStream_t)stream;
  if (!backward) {   // in: [n][h][w] slice (is, io); out dense [n][h/2][w/2][c]
    hipLaunchKernelGGL(k_pool_fwd, dim3(blocks_for((long long)n * h * w * c / 32)), dim3(256), 0,
                       st, (const uint16_t *)in, is, io, n, h, w, c, (uint16_t *)out);
  } else {           // in: dense gradient [n][h/2][w/2][c]; out: slice (os, oo)
    hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for((long long)n * h * w * c / 8)), dim3(256), 0, st,
                       (const uint16_t *)in, n, h, w, c, (uint16_t *)out, os, oo, accumulate,
                       nullptr);
  }
  HIPC(hipGetLastError());
  return LBM_OK;
}

int lbm_nn_up2(int backward, int n, int h, int w, int c, const void *in, int is, int io,
               void *out, int os, int oo, void *stream) {
  if (n < 1 || h < 1 || w < 1 || c < 8 || c % 8 || is % 8 || io % 8 || os % 8 || oo % 8 ||
      !in || !out)
    return lbm_fail(LBM_EINVAL, "bad upsample arguments (c, strides and offsets multiples of 8)");
  hipStream_t st = (hipStream_t)stream;
  if (!backward)   // in dense [n][h][w][c] -> out slice of [n][2h][2w]
    hipLaunchKernelGGL(k_up_fwd, dim3(blocks_for((long long)n * 4 * h * w * c / 8)), dim3(256), 0, st,
                       (const uint16_t *)in, n, h, w, c, (uint16_t *)out, os, oo);
  else             // in: gradient slice of [n][2h][2w] -> out dense [n][h][w][c]
    hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for((long long)n * h * w * c / 8)), dim3(256), 0, st,
                       (const uint16_t *)in, is, io, n, h, w, c, (uint16_t *)out, nullptr);
  HIPC(hipGetLastError());
  return LBM_OK;
}

// ------------------------------------------------------------------ driver
int lbm_sur_destroy(lbm_sur_t s) {
  if (!s) return LBM_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->side) (void)hipStreamSynchronize(s->side);
  void *ptrs[] = {s->act, s->gact, s->w, s->m, s->v, s->gw, s->wb, s->wbt, s->target, s->mask,
                  s->out3, s->loss_dev, s->rearr, s->field, s->part};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (s->loss_host) (void)hipHostFree(s->loss_host);
  if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->fork) (void)hipEventDestroy(s->fork);
  if (s->join) (void)hipEventDestroy(s->join);
  delete s;
  return LBM_OK;
}

int lbm_sur_create(int max_batch, lbm_sur_t *out) {
  if (!out) return lbm_fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 256)
    return lbm_fail(LBM_EINVAL, "max_batch %d outside [1, 256]", max_batch);
  lbm_surrogate *s = new (std::nothrow) lbm_surrogate();
  if (!s) return lbm_fail(LBM_ENOMEM, "host allocation");
  s->nmax = max_batch;
  build_net(s);
  plan_relu_masks(s);
  plan_fwd_fusion(s);
  for (const Op &o : s->ops) {   // the convs are laid out one after another
    if (o.type != OP_CONV) continue;
    const int k = s->convs.count++;
    s->convs.off[k] = (long long)o.woff;
    s->convs.ci[k] = o.ci;
    s->convs.co[k] = o.co;
  }
  for (const Buf &b : s->bufs) {
    s->act_off.push_back(s->act_elems);
    s->act_elems += (size_t)max_batch * level_h(b.level) * level_w(b.level) * b.ch;
  }
  const size_t npix = (size_t)max_batch * kH * kW;
  auto bail = [&](int rc) {
    lbm_sur_destroy(s);
    return rc;
  };
  hipError_t e = hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking);
  s->stream = s->own_stream;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
  // the events only order two streams of this device: a device-scope release
  // (the default system-scope one writes back and invalidates the caches)
  const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, evf);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join, evf);
  void **allocs[] = {(void **)&s->act,    (void **)&s->gact,  (void **)&s->w,
                     (void **)&s->m,      (void **)&s->v,     (void **)&s->gw,
                     (void **)&s->wb,     (void **)&s->target, (void **)&s->mask,
                     (void **)&s->out3,   (void **)&s->loss_dev, (void **)&s->rearr};
  const size_t sizes[] = {s->act_elems * 2, s->act_elems * 2, s->nparams * 4, s->nparams * 4,
                          s->nparams * 4,   s->nparams * 4,   s->nparams * 2, npix * 3 * 4,
                          npix * 4,         npix * 3 * 4,     16,             (size_t)max_batch * 16};
  for (int i = 0; i < 12 && e == hipSuccess; ++i) e = hipMalloc(allocs[i], sizes[i]);
  // partials of the split reductions: the largest weight / bias gradient, or
  // the loss's per-block sums
  size_t part_floats = blocks_for((long long)npix * (s->ops.back().out.cs / 8));
  for (const Op &o : s->ops)
    if (o.type == OP_CONV)
      part_floats = std::max(part_floats, wgrad_part_floats(max_batch, level_h(o.level),
                                                            level_w(o.level), o.ci, o.co));
  if (e == hipSuccess) e = hipMalloc(&s->part, part_floats * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&s->wbt, s->nparams * 2);
  if (e == hipSuccess) e = hipMemsetAsync(s->wbt, 0, s->nparams * 2, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->act, 0, s->act_elems * 2, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->gact, 0, s->act_elems * 2, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->w, 0, s->nparams * 4, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, s->nparams * 4, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, s->nparams * 4, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->wb, 0, s->nparams * 2, s->stream);
  if (e == hipSuccess) e = hipHostMalloc(&s->loss_host, 16, hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess)
    return bail(lbm_fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "surrogate setup: %s",
                         hipGetErrorString(e)));
  *out = s;
  return LBM_OK;
}

int lbm_sur_num_params(lbm_sur_t s, int64_t *n) {
  if (!s || !n) return lbm_fail(LBM_EINVAL, "NULL argument");
  *n = (int64_t)s->nparams;
  return LBM_OK;
}

int lbm_sur_set_stream(lbm_sur_t s, void *hip_stream) {
  if (!s) return lbm_fail(LBM_EINVAL, "surrogate is NULL");
  HIPC(hipStreamSynchronize(s->stream));
  s->stream = hip_stream ? (hipStream_t)hip_stream : s->own_stream;
  return LBM_OK;
}

int lbm_sur_set_params(lbm_sur_t s, const float *params_host, int64_t n) {
  if (!s || !params_host) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (n != (int64_t)s->nparams)
    return lbm_fail(LBM_EINVAL, "expected %zu parameters, got %lld", s->nparams, (long long)n);
  HIPC(hipMemcpyAsync(s->w, params_host, s->nparams * 4, hipMemcpyHostToDevice, s->stream));
  HIPC(hipMemsetAsync(s->m, 0, s->nparams * 4, s->stream));
  HIPC(hipMemsetAsync(s->v, 0, s->nparams * 4, s->stream));
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((long long)s->nparams)), dim3(256), 0, s->stream,
                     s->w, s->wb, (long long)s->nparams);
  HIPC(hipGetLastError());
  HIPC(transpose_weights(s));
  s->adam_t = 0;
  HIPC(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

int lbm_sur_init_params(lbm_sur_t s, const float *normals_host, int64_t n) {
  if (!s || !normals_host) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (n != (int64_t)s->nparams)
    return lbm_fail(LBM_EINVAL, "expected %zu draws, got %lld", s->nparams, (long long)n);
  std::vector<float> p(s->nparams, 0.f);
  const size_t last = s->ops.size() - 1;
  for (size_t k = 0; k < s->ops.size(); ++k) {
    const Op &o = s->ops[k];
    if (o.type != OP_CONV) continue;
    const int ci_real = k == 0 ? kInCh : o.ci;
    const int co_real = k == last ? kOutCh : o.co;
    const float sd = std::sqrt(2.0f / (9.0f * ci_real));   // He-normal
    for (int t = 0; t < 9; ++t)
      for (int c = 0; c < ci_real; ++c)
        for (int q = 0; q < co_real; ++q) {
          const size_t i = o.woff + ((size_t)t * o.ci + c) * o.co + q;
          p[i] = sd * normals_host[i];
        }
  }
  return lbm_sur_set_params(s, p.data(), n);
}

int lbm_sur_get_params(lbm_sur_t s, float *params_host, float *grads_host) {
  if (!s) return lbm_fail(LBM_EINVAL, "NULL argument");
  HIPC(hipStreamSynchronize(s->stream));
  if (params_host) HIPC(hipMemcpy(params_host, s->w, s->nparams * 4, hipMemcpyDeviceToHost));
  if (grads_host) HIPC(hipMemcpy(grads_host, s->gw, s->nparams * 4, hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_sur_forward(lbm_sur_t s, int n, const double *re, const double *ar, float *out_dev) {
  if (!s || !re || !ar || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (n < 1 || n > s->nmax) return lbm_fail(LBM_EINVAL, "n = %d outside [1, %d]", n, s->nmax);
  int rc = encode(s, n, re, ar);
  if (rc) return rc;
  rc = forward(s, n);
  if (rc) return rc;
  const long long npix = (long long)n * kH * kW;
  hipLaunchKernelGGL(k_extract, dim3(blocks_for(npix * kOutCh)), dim3(256), 0, s->stream,
                     bptr(s, s->act, head_view(s)), npix, out_dev);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

int lbm_sur_train_step(lbm_sur_t s, int n, const double *re, const double *ar,
                       const float *target_dev, const float *mask_dev, double lr,
                       int apply_update, double *loss) {
  if (!s || !re || !ar || !target_dev || !mask_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (n < 1 || n > s->nmax) return lbm_fail(LBM_EINVAL, "n = %d outside [1, %d]", n, s->nmax);
  if (!(lr >= 0.0) || !std::isfinite(lr)) return lbm_fail(LBM_EINVAL, "lr = %g", lr);
  double count = 0.0;
  for (int b = 0; b < n; ++b) count += 128.0 * std::rint(128.0 * ar[b]);
  int rc = encode(s, n, re, ar);
  if (rc) return rc;
  rc = forward(s, n);
  if (rc) return rc;
  const long long npix = (long long)n * kH * kW;
  HIPC(hipMemsetAsync(s->loss_dev, 0, sizeof(float), s->stream));
  const View &hv = head_view(s);
  static_assert(kOutCh <= 8, "k_mse reads the head's first 8 channels");
  // the head's output is a dense buffer (channel offset 0): k_mse writes its
  // gradient as hv.cs / 8 vectors per pixel
  const unsigned mse_blocks = blocks_for(npix * (hv.cs / 8));
  hipLaunchKernelGGL(k_mse, dim3(mse_blocks), dim3(256), 0, s->stream,
                     bptr(s, s->act, hv), hv.cs, target_dev, mask_dev, npix, kOutCh,
                     (float)(1.0 / count), bptr(s, s->gact, hv), hv.cs, s->part);
  hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(256), 0, s->stream, s->part, (int)mse_blocks,
                     s->loss_dev);
  HIPC(hipGetLastError());
  rc = backward(s, n);
  if (rc) return rc;
  if (apply_update) {
    s->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 / (1.0 - std::pow(b1, (double)s->adam_t));
    const double c2 = 1.0 / (1.0 - std::pow(b2, (double)s->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for((long long)s->nparams)), dim3(256), 0, s->stream,
                       s->w, s->m, s->v, s->gw, s->wb, (long long)s->nparams, (float)lr, (float)b1,
                       (float)b2, 1e-8f, (float)c1, (float)c2);
    HIPC(hipGetLastError());
    HIPC(transpose_weights(s));
  }
  HIPC(hipMemcpyAsync(s->loss_host, s->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s->stream));
  HIPC(hipStreamSynchronize(s->stream));
  if (loss) *loss = (double)s->loss_host[0];
  if (!std::isfinite(s->loss_host[0])) return lbm_fail(LBM_EUNSTABLE, "non-finite loss");
  return LBM_OK;
}

// Predict the steady field of an nx x ny cavity at Reynolds number re and map
// it onto the lattice: s->field = (rho, ux, uy), each [ny][nx].
static int predict_lattice(lbm_sur_t s, int nx, int ny, double re, double u_lid) {
  const double ar = (double)ny / nx;
  int rc = lbm_sur_forward(s, 1, &re, &ar, s->out3);
  if (rc) return rc;
  const size_t n = (size_t)nx * ny;
  if (s->field_doubles < 3 * n) {
    if (s->field) HIPC(hipFree(s->field));
    s->field = nullptr;
    s->field_doubles = 0;
    HIPC(hipMalloc(&s->field, 3 * n * sizeof(double)));
    s->field_doubles = 3 * n;
  }
  const int ny_c = (int)std::rint(128.0 * ar);
  hipLaunchKernelGGL(k_to_lattice, dim3(blocks_for((long long)n)), dim3(256), 0, s->stream,
                     s->out3, std::max(ny_c, 2), nx, ny, u_lid, s->field, s->field + n,
                     s->field + 2 * n);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

int lbm_sur_warm_start(lbm_sur_t s, lbm_t h) {
  if (!s || !h) return lbm_fail(LBM_EINVAL, "NULL argument");
  lbm_info_t info;
  int rc = lbm_info(h, &info);
  if (rc) return rc;
  rc = predict_lattice(s, info.nx, info.ny, info.re, info.u_lid);
  if (rc) return rc;
  const size_t n = (size_t)info.nx * info.ny;
  return lbm_init_fields_device(h, s->field, s->field + n, s->field + 2 * n,
                                LBM_INIT_RENORMALISE_MASS | LBM_INIT_ZERO_STAGGERED);
}

int lbm_sur_warm_start_batch(lbm_sur_t s, lbm_batch_t b, int k) {
  if (!s || !b) return lbm_fail(LBM_EINVAL, "NULL argument");
  int nx = 0, ny = 0;
  double re = 0, u = 0;
  int rc = lbm_batch_cavity(b, k, &nx, &ny, &re, &u);
  if (rc) return rc;
  rc = predict_lattice(s, nx, ny, re, u);
  if (rc) return rc;
  const size_t n = (size_t)nx * ny;
  return lbm_batch_init_fields_device(b, k, s->field, s->field + n, s->field + 2 * n,
                                      LBM_INIT_RENORMALISE_MASS | LBM_INIT_ZERO_STAGGERED);
}

}  // extern "C"
