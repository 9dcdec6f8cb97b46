// lbm3d.hip -- C ABI of the D3Q19 lid-driven box (include/lbm.h, "3-D
// lid-driven box"): handles, 100-step chunks replayed from HIP graphs with
// the FP64 monitors, moments and populations, tile-shape autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "d3q19_step.hpp"
#include "d3q19_tb2.hpp"
#include "lbm_internal.h"

using namespace lbm;

namespace {
// tile shapes: 0-2 one step per launch (64 x BY sites of one z plane, BY
// in {1, 2, 4}); 3-7 two steps per launch: 3 a TX x TY x TZ tile in LDS
// (k_step3_tb2; FP32 32 x 8 x 4, FP64 16 x 6 x 4, 1024 threads: the window
// takes most of the LDS, one block per CU, so large blocks hide latency),
// 4-7 a TX x TY column marching through z (k_step3_zs2; FP32 64 x 8,
// 64 x 12, 32 x 16, 32 x 24; FP64 32 x 12, 32 x 8, 16 x 16, 24 x 16)
constexpr int kNum3Variants = 8;
// blocks of the monitor and mass reductions (each thread takes a few sites:
// more waves in flight than the two-dimensional handles' 1024 blocks give)
constexpr int kRed3Blocks = 8192;
}  // namespace

struct lbm_cube {
  int nx = 0, ny = 0, nz = 0, pitch = 0, plane = 0, dtype = 0;
  double re = 0, u_lid = 0, tau = 0, omega = 0;
  void *buf[2] = {nullptr, nullptr};
  size_t buf_bytes = 0;
  int cur = 0;
  double *uref = nullptr;       // [3][n] Eq. 6 reference velocity
  double *partials = nullptr;   // [kRed3Blocks][kNumSums]
  double *mon_dev = nullptr;    // chunk monitor sums
  double *aux_dev = nullptr;    // on-demand sums
  double *mon_host = nullptr;   // pinned
  double *tmp = nullptr;        // FP64 transfer scratch
  size_t tmp_doubles = 0;
  hipStream_t stream = nullptr, own_stream = nullptr, cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int variant = 1, use_graph = 1;
  int cus = 256;                       // compute units of the handle's GPU
  mutable int zs2_zc[kNum3Variants] = {};   // planes per block of a z-marching shape
  int64_t t = 0, snap_t = 0, mon_t = -1;
  bool mon_valid = false;
  double last_res = INFINITY, last_mass = NAN;
};

namespace {

long long sites(const lbm_cube *h) { return (long long)h->nx * h->ny * h->nz; }

template <typename T, bool S, int BY>
hipError_t launch3_t(const lbm_cube *h, const void *src, void *dst, hipStream_t st) {
  Step3Params<T> p{};
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.nz = h->nz;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + 63) / 64;
  p.tiles_y = (h->ny + BY - 1) / BY;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  hipLaunchKernelGGL((k_step3<T, S, BY>), dim3(p.tiles_x * p.tiles_y * h->nz), dim3(64, BY), 0,
                     st, p);
  return hipGetLastError();
}

template <typename T, bool S, int TX, int TY, int TZ, int NT>
hipError_t launch3_tb2_t(const lbm_cube *h, const void *src, void *dst, hipStream_t st) {
  Step3Params<T> p{};
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.nz = h->nz;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + TX - 1) / TX;
  p.tiles_y = (h->ny + TY - 1) / TY;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  const int tiles_z = (h->nz + TZ - 1) / TZ;
  hipLaunchKernelGGL((k_step3_tb2<T, S, TX, TY, TZ, NT>), dim3(p.tiles_x * p.tiles_y * tiles_z),
                     dim3(NT), 0, st, p);
  return hipGetLastError();
}

// Planes per block of the z-marching kernel over nz planes and cols
// columns, `slots` blocks resident on the GPU at once: the length whose
// chunk count minimises rounds x (planes + 2), a round being `slots` blocks
// and a block's time about proportional to its planes plus the two extra
// planes its step 1 computes (ties: the longer chunks, fewer blocks).
int zs2_planes(int nz, long long cols, long long slots) {
  int best = nz;
  long long best_cost = -1;
  for (int zc = nz; zc >= 1; --zc) {
    const long long chunks = (nz + zc - 1) / zc;
    const long long rounds = (cols * chunks + slots - 1) / slots;
    const long long cost = rounds * (zc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

template <typename T, bool S, int TX, int TY, int NT>
hipError_t launch3_zs2_t(const lbm_cube *h, int v, const void *src, void *dst, hipStream_t st) {
  Step3Params<T> p{};
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.nz = h->nz;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + TX - 1) / TX;
  p.tiles_y = (h->ny + TY - 1) / TY;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  // the chunk length, once per handle and shape: blocks per CU as the LDS
  // window (43 values per window site) and 2048 threads allow
  const int cols = p.tiles_x * p.tiles_y;
  if (h->zs2_zc[v] <= 0) {
    const long long lds = 43LL * (TX + 2) * (TY + 2) * (long long)sizeof(T);
    const long long per_cu = std::max(1LL, std::min(160LL * 1024 / lds, 2048LL / NT));
    h->zs2_zc[v] = zs2_planes(h->nz, cols, per_cu * std::max(1, h->cus));
  }
  p.zc = h->zs2_zc[v];
  const int chunks = (h->nz + p.zc - 1) / p.zc;
  // FP64 states below 2^31 bytes through raw buffers (+2.6 % at 192^3;
  // FP32 measured 5.5 % slower that way at 256^3)
  bool buf = false;
  if constexpr (sizeof(T) == 8) buf = 19LL * h->plane * (long long)sizeof(T) <= INT32_MAX;
  if (buf)
    hipLaunchKernelGGL((k_step3_zs2<T, S, TX, TY, NT, sizeof(T) == 8>), dim3(cols * chunks),
                       dim3(NT), 0, st, p);
  else
    hipLaunchKernelGGL((k_step3_zs2<T, S, TX, TY, NT, false>), dim3(cols * chunks), dim3(NT), 0,
                       st, p);
  return hipGetLastError();
}

// Steps of Eq. 1 one launch of shape v applies.
int steps3(int v) { return v >= 3 ? 2 : 1; }

template <typename T, bool S>
hipError_t launch3_variant(int v, const lbm_cube *h, const void *src, void *dst,
                           hipStream_t st) {
  constexpr bool f64 = sizeof(T) == 8;
  switch (v) {
    case 0: return launch3_t<T, S, 1>(h, src, dst, st);
    case 2: return launch3_t<T, S, 4>(h, src, dst, st);
    case 3:
      if constexpr (f64)
        return launch3_tb2_t<T, S, 16, 6, 4, 1024>(h, src, dst, st);
      else
        return launch3_tb2_t<T, S, 32, 8, 4, 1024>(h, src, dst, st);
    case 4:
      if constexpr (f64)
        return launch3_zs2_t<T, S, 32, 12, 512>(h, v, src, dst, st);
      else
        return launch3_zs2_t<T, S, 64, 8, 704>(h, v, src, dst, st);
    case 5:
      if constexpr (f64)
        return launch3_zs2_t<T, S, 32, 8, 384>(h, v, src, dst, st);
      else
        return launch3_zs2_t<T, S, 64, 12, 960>(h, v, src, dst, st);
    case 6:
      if constexpr (f64)
        return launch3_zs2_t<T, S, 16, 16, 384>(h, v, src, dst, st);
      else
        return launch3_zs2_t<T, S, 32, 16, 640>(h, v, src, dst, st);
    case 7:
      if constexpr (f64)
        return launch3_zs2_t<T, S, 24, 16, 512>(h, v, src, dst, st);
      else
        return launch3_zs2_t<T, S, 32, 24, 896>(h, v, src, dst, st);
    default: return launch3_t<T, S, 2>(h, src, dst, st);
  }
}

// One launch of shape v: steps3(v) steps from src into dst.
hipError_t launch3(const lbm_cube *h, int v, const void *src, void *dst, hipStream_t st) {
  if (h->dtype == LBM_F64) return launch3_variant<double, false>(v, h, src, dst, st);
  return launch3_variant<float, true>(v, h, src, dst, st);
}

// The one-step shape single steps take: the chosen one, or shape 1.
int one_step3(const lbm_cube *h) { return steps3(h->variant) == 1 ? h->variant : 1; }

int reduce_blocks(const lbm_cube *h) {
  return (int)std::min<long long>(kRed3Blocks, (sites(h) + kRedThreads - 1) / kRedThreads);
}

template <typename T, bool S>
hipError_t monitor3_t(const lbm_cube *h, const void *src, bool update, double *out,
                      hipStream_t st) {
  const int nb = reduce_blocks(h);
  if (update)
    hipLaunchKernelGGL((k_monitor3<T, S, true>), dim3(nb), dim3(kRedThreads), 0, st,
                       (const T *)src, h->nx, h->ny, h->nz, h->pitch, h->plane, h->uref,
                       h->partials);
  else
    hipLaunchKernelGGL((k_monitor3<T, S, false>), dim3(nb), dim3(kRedThreads), 0, st,
                       (const T *)src, h->nx, h->ny, h->nz, h->pitch, h->plane, h->uref,
                       h->partials);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, st, h->partials, nb, out);
  return hipGetLastError();
}

hipError_t monitor3(const lbm_cube *h, const void *src, bool update, double *out,
                    hipStream_t st) {
  if (h->dtype == LBM_F64) return monitor3_t<double, false>(h, src, update, out, st);
  return monitor3_t<float, true>(h, src, update, out, st);
}

// 100 steps from buf[c] (100 / K launches, an even number: the state ends
// in buf[c]) and the monitor.
hipError_t issue_chunk3(lbm_cube *h, int c, hipStream_t st) {
  int cur = c;
  const int K = steps3(h->variant);
  for (int k = 0; k < kChunk; k += K) {
    hipError_t e = launch3(h, h->variant, h->buf[cur], h->buf[1 - cur], st);
    if (e != hipSuccess) return e;
    cur = 1 - cur;
  }
  return monitor3(h, h->buf[cur], true, h->mon_dev, st);
}

void drop_graphs3(lbm_cube *h) {
  for (int c = 0; c < 2; ++c) {
    if (h->graph[c]) (void)hipGraphExecDestroy(h->graph[c]);
    h->graph[c] = nullptr;
  }
}

int build_graph3(lbm_cube *h, int c) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = issue_chunk3(h, c, h->cap_stream);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return lbm_fail(LBM_EDEVICE, "3-D graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&h->graph[c], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph[c] = nullptr;
    return lbm_fail(LBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

int reset3(lbm_cube *h) {
  h->t = 0;
  h->snap_t = 0;
  h->mon_t = -1;
  h->mon_valid = false;
  h->last_res = INFINITY;
  h->last_mass = NAN;
  drop_graphs3(h);
  hipError_t e = monitor3(h, h->buf[h->cur], true, h->aux_dev, h->stream);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int ensure_tmp3(lbm_cube *h, size_t doubles) {
  if (h->tmp_doubles >= doubles) return LBM_OK;
  HIPC(hipStreamSynchronize(h->stream));
  if (h->tmp) HIPC(hipFree(h->tmp));
  h->tmp = nullptr;
  h->tmp_doubles = 0;
  HIPC(hipMalloc(&h->tmp, doubles * sizeof(double)));
  h->tmp_doubles = doubles;
  return LBM_OK;
}

void note_monitor3(lbm_cube *h) {
  h->mon_valid = (h->snap_t == h->t - kChunk);
  h->snap_t = h->t;
  h->mon_t = h->t;
}

}  // namespace

int lbm3d_destroy(lbm3d_t h) {
  if (!h) return LBM_OK;
  drop_graphs3(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void *p : {h->buf[0], h->buf[1], (void *)h->uref, (void *)h->partials,
                  (void *)h->mon_dev, (void *)h->aux_dev, (void *)h->tmp})
    if (p) (void)hipFree(p);
  if (h->mon_host) (void)hipHostFree(h->mon_host);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
  return LBM_OK;
}

int lbm3d_create(int nx, int ny, int nz, double re, double u_lid, int dtype, lbm3d_t *out) {
  if (!out) return lbm_fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 2 || ny < 2 || nz < 2 || nx > 4096 || ny > 4096 || nz > 4096)
    return lbm_fail(LBM_EINVAL, "box %d x %d x %d outside [2, 4096]^3", nx, ny, nz);
  if (dtype != LBM_F64 && dtype != LBM_F32_SHIFTED)
    return lbm_fail(LBM_EINVAL, "unknown dtype %d", dtype);
  if (!std::isfinite(u_lid) || std::fabs(u_lid) >= 1.0 / std::sqrt(3.0))
    return lbm_fail(LBM_EINVAL, "|u_lid| = %g must be below c_s = 1/sqrt(3)", u_lid);
  if (!(re > 0.0) || !std::isfinite(re))
    return lbm_fail(LBM_EINVAL, "re = %g must be positive and finite", re);
  const double tau = 3.0 * u_lid * nx / re + 0.5;   // Eq. 5 with L = nx
  if (!(tau > 0.5)) return lbm_fail(LBM_EINVAL, "tau = %.17g must exceed 1/2", tau);
  const int pitch = (nx + 63) / 64 * 64;
  const long long plane = (long long)pitch * ny * nz;
  if (plane * 19 >= (1LL << 31))
    return lbm_fail(LBM_EINVAL, "box too large for 32-bit element offsets");
  if ((long long)nx * ny * nz * 3 >= (1LL << 31))
    return lbm_fail(LBM_EINVAL, "box too large for the monitor arrays");
  lbm_cube *h = new (std::nothrow) lbm_cube();
  if (!h) return lbm_fail(LBM_ENOMEM, "host allocation");
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->pitch = pitch;
  h->plane = (int)plane;
  h->dtype = dtype;
  h->re = re;
  h->u_lid = u_lid;
  h->tau = tau;
  h->omega = 1.0 / tau;
  const size_t esz = dtype == LBM_F64 ? 8 : 4;
  h->buf_bytes = (size_t)plane * 19 * esz;
  auto bail = [&](int code) {
    lbm3d_destroy(h);
    return code;
  };
  hipError_t e;
#define TRY(call)                                                                          \
  do {                                                                                     \
    e = (call);                                                                            \
    if (e != hipSuccess)                                                                   \
      return bail(lbm_fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s", \
                           #call, hipGetErrorString(e)));                                  \
  } while (0)
  TRY(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
  {
    int dev = 0;
    TRY(hipGetDevice(&dev));
    TRY(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  h->stream = h->own_stream;
  TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  for (int c = 0; c < 2; ++c) TRY(hipMalloc(&h->buf[c], h->buf_bytes));
  TRY(hipMalloc(&h->uref, sizeof(double) * 3 * (size_t)sites(h)));
  TRY(hipMalloc(&h->partials, sizeof(double) * kRed3Blocks * kNumSums));
  TRY(hipMalloc(&h->mon_dev, sizeof(double) * 4));
  TRY(hipMalloc(&h->aux_dev, sizeof(double) * 4));
  TRY(hipHostMalloc(&h->mon_host, sizeof(double) * 8, hipHostMallocDefault));
  // rest state: f = w, i.e. g = 0 in FP32 f - w storage; FP64 by populations
  if (dtype == LBM_F32_SHIFTED) {
    TRY(hipMemsetAsync(h->buf[0], 0, h->buf_bytes, h->stream));
  } else {
    std::vector<double> w(19);
    for (int i = 0; i < 19; ++i) w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    std::vector<double> row((size_t)h->plane);
    for (int i = 0; i < 19; ++i) {
      std::fill(row.begin(), row.end(), w[i]);
      TRY(hipMemcpy((double *)h->buf[0] + (size_t)i * h->plane, row.data(),
                    row.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  TRY(hipMemsetAsync(h->buf[1], 0, h->buf_bytes, h->stream));
  int rc = reset3(h);
  if (rc) return bail(rc);
  TRY(hipStreamSynchronize(h->stream));
#undef TRY
  *out = h;
  return LBM_OK;
}

int lbm3d_set_stream(lbm3d_t h, void *stream) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  HIPC(hipStreamSynchronize(h->stream));
  h->stream = stream ? (hipStream_t)stream : h->own_stream;
  return LBM_OK;
}

int lbm3d_set_option(lbm3d_t h, int option, int64_t value) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  switch (option) {
    case LBM_OPT_USE_GRAPH:
      h->use_graph = value ? 1 : 0;
      return LBM_OK;
    case LBM_OPT_STEP_VARIANT:
      if (value < 0 || value >= kNum3Variants)
        return lbm_fail(LBM_EINVAL, "variant %lld outside [0, %d)", (long long)value,
                        kNum3Variants);
      if (h->variant != (int)value) drop_graphs3(h);
      h->variant = (int)value;
      return LBM_OK;
    default:
      return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

int lbm3d_get_option(lbm3d_t h, int option, int64_t *value) {
  if (!h || !value) return lbm_fail(LBM_EINVAL, "NULL argument");
  switch (option) {
    case LBM_OPT_USE_GRAPH: *value = h->use_graph; return LBM_OK;
    case LBM_OPT_STEP_VARIANT: *value = h->variant; return LBM_OK;
    case LBM_OPT_NUM_VARIANTS: *value = kNum3Variants; return LBM_OK;
    case LBM_OPT_STEPS_PER_LAUNCH: *value = steps3(h->variant); return LBM_OK;
    default: return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

int lbm3d_step(lbm3d_t h, int64_t n) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  if (n < 0) return lbm_fail(LBM_EINVAL, "n = %lld < 0", (long long)n);
  bool monitored = false;
  hipError_t e;
  while (n > 0) {
    if (h->t % kChunk == 0 && n >= kChunk) {
      if (h->use_graph) {
        if (!h->graph[h->cur]) {
          int rc = build_graph3(h, h->cur);
          if (rc) return rc;
        }
        HIPC(hipGraphLaunch(h->graph[h->cur], h->stream));
      } else {
        e = issue_chunk3(h, h->cur, h->stream);
        if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "launch: %s", hipGetErrorString(e));
      }
      h->t += kChunk;            // an even number of launches: the state is back in buf[cur]
      n -= kChunk;
      note_monitor3(h);
      monitored = true;
      continue;
    }
    // off the 100-step grid: two-step launches of a two-step shape while t
    // is even (100 is, so none crosses a monitor point), else single steps
    const int K = steps3(h->variant) == 2 && h->t % 2 == 0 && n >= 2 ? 2 : 1;
    e = launch3(h, K == 2 ? h->variant : one_step3(h), h->buf[h->cur], h->buf[1 - h->cur],
                h->stream);
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "step launch: %s", hipGetErrorString(e));
    h->cur = 1 - h->cur;
    h->t += K;
    n -= K;
    if (h->t % kChunk == 0) {
      e = monitor3(h, h->buf[h->cur], true, h->mon_dev, h->stream);
      if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor: %s", hipGetErrorString(e));
      note_monitor3(h);
      monitored = true;
    }
  }
  if (monitored)
    HIPC(hipMemcpyAsync(h->mon_host, h->mon_dev, 3 * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  if (monitored) {
    const double *m = h->mon_host;
    h->last_mass = (double)sites(h) + m[0];
    h->last_res = (h->mon_valid && m[2] > 0.0) ? std::sqrt(m[1] / m[2]) : INFINITY;
    if (!std::isfinite(h->last_mass) || std::isnan(h->last_res))
      return lbm_fail(LBM_EUNSTABLE, "non-finite monitor at step %lld", (long long)h->t);
  }
  return LBM_OK;
}

int lbm3d_steps_done(lbm3d_t h, int64_t *steps) {
  if (!h || !steps) return lbm_fail(LBM_EINVAL, "NULL argument");
  *steps = h->t;
  return LBM_OK;
}

int lbm3d_residual(lbm3d_t h, double *residual, int64_t *at_step) {
  if (!h || !residual) return lbm_fail(LBM_EINVAL, "NULL argument");
  *residual = h->mon_t >= 0 ? h->last_res : INFINITY;
  if (at_step) *at_step = h->mon_t;
  return LBM_OK;
}

int lbm3d_mass(lbm3d_t h, double *mass) {
  if (!h || !mass) return lbm_fail(LBM_EINVAL, "NULL argument");
  hipError_t e = monitor3(h, h->buf[h->cur], false, h->aux_dev, h->stream);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor: %s", hipGetErrorString(e));
  HIPC(hipMemcpyAsync(h->mon_host + 4, h->aux_dev, sizeof(double), hipMemcpyDeviceToHost,
                      h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  *mass = (double)sites(h) + h->mon_host[4];
  return LBM_OK;
}

int lbm3d_moments(lbm3d_t h, double *rho, double *ux, double *uy, double *uz) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  const long long n = sites(h);
  int rc = ensure_tmp3(h, 4 * (size_t)n);
  if (rc) return rc;
  double *d[4] = {rho ? h->tmp : nullptr, ux ? h->tmp + n : nullptr,
                  uy ? h->tmp + 2 * n : nullptr, uz ? h->tmp + 3 * n : nullptr};
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_moments3<double, false>), dim3(blocks), dim3(256), 0, h->stream,
                       (const double *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       d[0], d[1], d[2], d[3]);
  else
    hipLaunchKernelGGL((k_moments3<float, true>), dim3(blocks), dim3(256), 0, h->stream,
                       (const float *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       d[0], d[1], d[2], d[3]);
  HIPC(hipGetLastError());
  double *outs[4] = {rho, ux, uy, uz};
  for (int k = 0; k < 4; ++k)
    if (outs[k])
      HIPC(hipMemcpyAsync(outs[k], d[k], n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm3d_set_populations(lbm3d_t h, const double *f) {
  if (!h || !f) return lbm_fail(LBM_EINVAL, "NULL argument");
  const long long n = sites(h);
  int rc = ensure_tmp3(h, 19 * (size_t)n);
  if (rc) return rc;
  HIPC(hipMemcpyAsync(h->tmp, f, 19 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_set_pop3<double, false>), dim3(blocks), dim3(256), 0, h->stream,
                       (double *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       h->tmp, h->omega);
  else
    hipLaunchKernelGGL((k_set_pop3<float, true>), dim3(blocks), dim3(256), 0, h->stream,
                       (float *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       h->tmp, h->omega);
  HIPC(hipGetLastError());
  rc = reset3(h);
  if (rc) return rc;
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm3d_get_populations(lbm3d_t h, double *fstar) {
  if (!h || !fstar) return lbm_fail(LBM_EINVAL, "NULL argument");
  const long long n = sites(h);
  int rc = ensure_tmp3(h, 19 * (size_t)n);
  if (rc) return rc;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_get_pop3<double, false>), dim3(blocks), dim3(256), 0, h->stream,
                       (const double *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       h->tmp);
  else
    hipLaunchKernelGGL((k_get_pop3<float, true>), dim3(blocks), dim3(256), 0, h->stream,
                       (const float *)h->buf[h->cur], h->nx, h->ny, h->nz, h->pitch, h->plane,
                       h->tmp);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(fstar, h->tmp, 19 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm3d_autotune(lbm3d_t h, int chunks, int *best_variant, double *ms_per_step) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  if (chunks < 1 || chunks > 1000)
    return lbm_fail(LBM_EINVAL, "chunks = %d outside [1, 1000]", chunks);
  if (h->t % kChunk != 0) return lbm_fail(LBM_EINVAL, "autotune only at a multiple of 100 steps");
  // keep the state, the Eq. 6 reference and the counters; restore them after
  void *save_f = nullptr, *save_u = nullptr;
  const size_t ubytes = sizeof(double) * 3 * (size_t)sites(h);
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMalloc(&save_f, h->buf_bytes));
  hipError_t e = hipMalloc(&save_u, ubytes);
  if (e != hipSuccess) {
    (void)hipFree(save_f);
    return lbm_fail(LBM_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  }
  const int cur0 = h->cur;
  e = hipMemcpyAsync(save_f, h->buf[cur0], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(save_u, h->uref, ubytes, hipMemcpyDeviceToDevice, h->stream);
  const int64_t t0 = h->t, snap0 = h->snap_t, mon0 = h->mon_t;
  const bool valid0 = h->mon_valid;
  const double res0 = h->last_res, mass0 = h->last_mass;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = LBM_OK, best = h->variant;
  double best_ms = INFINITY;
  for (int v = 0; v < kNum3Variants && e == hipSuccess && rc == LBM_OK; ++v) {
    rc = lbm3d_set_option(h, LBM_OPT_STEP_VARIANT, v);
    if (rc == LBM_OK) rc = lbm3d_step(h, kChunk);
    if (rc != LBM_OK) break;
    e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess) rc = lbm3d_step(h, (int64_t)chunks * kChunk);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double per = ms / ((double)chunks * kChunk);
    if (rc == LBM_OK && e == hipSuccess && per < best_ms) {
      best_ms = per;
      best = v;
    }
    h->cur = cur0;
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->buf[cur0], save_f, h->buf_bytes, hipMemcpyDeviceToDevice,
                         h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->uref, save_u, ubytes, hipMemcpyDeviceToDevice, h->stream);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(save_f);
  (void)hipFree(save_u);
  h->t = t0;
  h->snap_t = snap0;
  h->mon_t = mon0;
  h->mon_valid = valid0;
  h->last_res = res0;
  h->last_mass = mass0;
  if (rc != LBM_OK) return rc;
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "autotune: %s", hipGetErrorString(e));
  drop_graphs3(h);
  h->variant = best;
  if (best_variant) *best_variant = best;
  if (ms_per_step) *ms_per_step = best_ms;
  return LBM_OK;
}
