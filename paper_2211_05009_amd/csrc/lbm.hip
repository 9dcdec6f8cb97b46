// lbm.hip -- C ABI and host runtime of the D2Q9 lid-driven cavity library
// (declarations and contracts in include/lbm.h).
//
// Runtime structure per handle:
//   * two population buffers (A/B ping-pong); buf[cur] holds f*(t);
//   * a 100-step chunk (the monitor cadence of Sec. 2.2 (iii)) is captured
//     once per start buffer into a HIP graph: 100 step kernels, then the
//     FP64 monitor reduction (mass and Eq. 6 sums), plus probe records when
//     their cadence divides 100; lbm_step replays it; steps that do not
//     fill an aligned chunk are launched one by one;
//   * FP64 scratch for moments / probes / population transfers, allocated on
//     first use.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "d2q9_monitor.hpp"
#include "d2q9_nee.hpp"
#include "d2q9_nee_tb.hpp"
#include "d2q9_series.hpp"
#include "d2q9_step.hpp"
#include "d2q9_temporal.hpp"
#include "d2q9_vortex.hpp"
#include "lbm_internal.h"

using namespace lbm;

thread_local std::string g_lbm_err;

int lbm_fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_lbm_err = buf;
  return code;
}

// ------------------------------------------------------------ run log
// With $LBM_LOG naming a file, one JSON line is appended per lbm_step /
// lbm_batch_step call (see lbm_log_line); the file is opened once, in append
// mode, and written under a mutex.
namespace {
std::mutex g_log_mutex;
FILE *g_log = nullptr;
bool g_log_checked = false;
}  // namespace

void lbm_log_line(const char *fmt, ...) {
  std::lock_guard<std::mutex> lock(g_log_mutex);
  if (!g_log_checked) {
    g_log_checked = true;
    const char *path = std::getenv("LBM_LOG");
    if (path && *path) g_log = std::fopen(path, "a");
  }
  if (!g_log) return;
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(g_log, fmt, ap);
  va_end(ap);
  std::fputc('\n', g_log);
  std::fflush(g_log);
}

const char *lbm_json_num(double v, char *buf) {
  if (std::isfinite(v))
    std::snprintf(buf, 32, "%.17g", v);
  else
    std::snprintf(buf, 32, "null");
  return buf;
}

double lbm_wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ------------------------------------------------------------ tune cache
std::string tune_key(const char *kind, int dtype, long long a, long long b) {
  char arch[64] = "unknown";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char *c = arch; *c; ++c)
      if (*c == ' ' || *c == ':') *c = '_';
  }
  char buf[192];
  std::snprintf(buf, sizeof buf, "%s|%s|%s|%lld|%lld", arch, kind,
                dtype == LBM_F64 ? "f64" : "f32s", a, b);
  return buf;
}

int tune_cache_lookup(const std::string &key) {
  const char *path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path) return -1;
  FILE *fp = std::fopen(path, "r");
  if (!fp) return -1;
  char k[256];
  int v = -1, found = -1;
  while (std::fscanf(fp, "%255s %d", k, &v) == 2)
    if (key == k) found = v;             // the last entry wins
  std::fclose(fp);
  return found;
}

void tune_cache_store(const std::string &key, int variant) {
  const char *path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "%s %d\n", key.c_str(), variant);
  std::fclose(fp);
}

// ---------------------------------------------------------------- variants
// Step kernel variants.  Scalar (k_step): tile 64 x (BY*RY) sites, block
// 64 x BY threads.  Vector (k_step_vec): tile (64 V) x BY sites, V = 16 B /
// element, block 64 x BY.  Temporal (k_step_tb, variants 12-23): K steps per
// launch on TX x TY tiles held in LDS.  All give bit-identical results.
static const int kNumVariants = 29;
// K = 5 steps per launch on 32 x 32 tiles, 1024 threads: the fastest shape
// on the 500 x (500 Ar) lattices on gfx950 (lbm_autotune refines it).
static const int kDefaultVariant = 22;

// Steps applied by one launch of variant v.
static int steps_per_launch(int v) {
  static const int k[kNumVariants] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 4, 4, 2,
                                      5, 4, 4, 5, 5, 10, 10, 5, 5, 5, 4, 5, 5, 5};
  return (v >= 0 && v < kNumVariants) ? k[v] : 1;
}

// Core tile (sites along x, along y) of variant v: the sites one block
// updates (launch_step_variant's table; FP64 takes smaller tiles for some
// multi-step shapes).
static void tile_of(int v, int dtype, int &tx, int &ty) {
  static const int one[8] = {4, 8, 16, 8, 8, 8, 16, 16};   // k_step: 64 x (BY RY)
  static const int tb[17][2] = {{32, 32}, {32, 32}, {32, 32}, {32, 32}, {64, 16}, {16, 16},
                                {64, 16}, {16, 16}, {32, 32}, {64, 32}, {32, 32}, {64, 32},
                                {32, 32}, {32, 32}, {32, 16}, {32, 48}, {32, 64}};
  const bool f64 = dtype == LBM_F64;
  if (v < 8) {
    tx = 64;
    ty = one[v < 0 ? 0 : v];
  } else if (v < 12) {
    tx = 64 * (f64 ? 2 : 4);                                // 16-byte vectors
    ty = 1 << (v - 8);
  } else {
    tx = tb[v - 12][0];
    ty = tb[v - 12][1];
    if (f64 && v == 20) ty = 16;
    if (f64 && v == 21) tx = ty = 16;
    if (f64 && v == 23) ty = 16;
    if (f64 && (v == 24 || v == 25)) tx = ty = 16;
    if (f64 && (v == 27 || v == 28)) tx = 16;
  }
}

// Non-equilibrium extrapolation handles have their own shapes: four
// one-step ones (k_step_nee, 64 x (BY RY) nodes) and four multi-step ones
// (k_step_nee_tb): 16 x 16, K = 4; K = 5 on 32 x 16 (FP64 16 x 16); K = 4
// on 32 x 32 (FP64 16 x 32); K = 5 on 32 x 32 (FP64 K = 2 on 16 x 32).
static const int kNumNeeVariants = 8;
// default NEE shape before lbm_autotune: within 5 % of the best at 501^2
// in both precisions and the best in FP64 at 257^2 (FP32 at 257^2: 30
// against 36 GLUPS for shape 5)
static const int kDefaultNeeVariant = 6;

static int num_variants(const lbm_cavity *h) {
  return h->wall == LBM_WALL_NEE ? kNumNeeVariants : kNumVariants;
}

static int launch_steps(const lbm_cavity *h, int v) {
  if (h->wall == LBM_WALL_NEE) {
    static const int k[kNumNeeVariants] = {1, 1, 1, 1, 4, 5, 4, 5};
    if (v == 7 && h->dtype == LBM_F64) return 2;
    return (v >= 0 && v < kNumNeeVariants) ? k[v] : 1;
  }
  return steps_per_launch(v);
}

// Tile (nodes along x, along y) of NEE variant v.
static void nee_tile_of(int v, int dtype, int &tx, int &ty) {
  static const int one[4] = {4, 8, 8, 8};   // k_step_nee: 64 x (BY RY)
  const bool f64 = dtype == LBM_F64;
  if (v >= 0 && v < 4) {
    tx = 64;
    ty = one[v];
  } else if (v == 4) {
    tx = ty = 16;
  } else if (v == 5) {
    tx = f64 ? 16 : 32;
    ty = 16;
  } else {   // shapes 6 and 7
    tx = f64 ? 16 : 32;
    ty = 32;
  }
}

template <typename T, bool S, int BY, int RY>
static hipError_t launch_nee_t(const lbm_cavity *h, const void *src, void *dst,
                               hipStream_t st) {
  StepParams<T> p;
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + 63) / 64;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  p.ulid = (T)h->u_lid;
  const int tiles_y = (h->ny + BY * RY - 1) / (BY * RY);
  hipLaunchKernelGGL((k_step_nee<T, S, BY, RY>), dim3(p.tiles_x * tiles_y), dim3(64, BY), 0,
                     st, p);
  return hipGetLastError();
}

template <typename T, bool S, int K, int TX, int TY, int NT>
static hipError_t launch_nee_tb_t(const lbm_cavity *h, const void *src, void *dst,
                                  hipStream_t st) {
  StepParams<T> p;
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + TX - 1) / TX;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  p.ulid = (T)h->u_lid;
  const int tiles_y = (h->ny + TY - 1) / TY;
  hipLaunchKernelGGL((k_step_nee_tb<T, S, K, TX, TY, NT>), dim3(p.tiles_x * tiles_y), dim3(NT),
                     0, st, p);
  return hipGetLastError();
}

template <typename T, bool S>
static hipError_t launch_nee_variant(const lbm_cavity *h, int v, const void *src, void *dst,
                                     hipStream_t st) {
  constexpr bool f64 = sizeof(T) == 8;
  switch (v) {
    case 1: return launch_nee_t<T, S, 4, 2>(h, src, dst, st);
    case 2: return launch_nee_t<T, S, 8, 1>(h, src, dst, st);
    case 3: return launch_nee_t<T, S, 2, 4>(h, src, dst, st);
    case 4: return launch_nee_tb_t<T, S, 4, 16, 16, 256>(h, src, dst, st);
    case 5:
      if constexpr (f64)
        return launch_nee_tb_t<T, S, 5, 16, 16, 256>(h, src, dst, st);
      else
        return launch_nee_tb_t<T, S, 5, 32, 16, 512>(h, src, dst, st);
    case 6:
      if constexpr (f64)
        return launch_nee_tb_t<T, S, 4, 16, 32, 512>(h, src, dst, st);
      else
        return launch_nee_tb_t<T, S, 4, 32, 32, 1024>(h, src, dst, st);
    case 7:
      if constexpr (f64)
        return launch_nee_tb_t<T, S, 2, 16, 32, 512>(h, src, dst, st);
      else
        return launch_nee_tb_t<T, S, 5, 32, 32, 1024>(h, src, dst, st);
    default: return launch_nee_t<T, S, 4, 1>(h, src, dst, st);
  }
}

template <typename T, bool S, int BY, int RY>
static hipError_t launch_step_t(const lbm_cavity *h, const void *src, void *dst,
                                hipStream_t st) {
  StepParams<T> p;
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + 63) / 64;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  const int tiles_y = (h->ny + BY * RY - 1) / (BY * RY);
  hipLaunchKernelGGL((k_step<T, S, BY, RY>), dim3(p.tiles_x * tiles_y),
                     dim3(64, BY), 0, st, p);
  return hipGetLastError();
}

template <typename T, bool S, int BY>
static hipError_t launch_step_vec_t(const lbm_cavity *h, const void *src, void *dst,
                                    hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  StepParams<T> p;
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = (h->nx + 64 * V - 1) / (64 * V);
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  const int tiles_y = (h->ny + BY - 1) / BY;
  hipLaunchKernelGGL((k_step_vec<T, S, BY>), dim3(p.tiles_x * tiles_y), dim3(64, BY), 0, st,
                     p);
  return hipGetLastError();
}

// mon = 1 / 2: the first / second launch of a chunk that carries the Eq. 6
// monitor of its start state (reference field uref, result in mon_dev; see
// TbMonitor); 0: a plain launch.
template <typename T, bool S, int K, int TX, int TY, int NT, bool PP = false>
static hipError_t launch_tb_t(const lbm_cavity *h, const void *src, void *dst,
                              hipStream_t st, int mon) {
  StepParams<T> p;
  p.src = (const T *)src;
  p.dst = (T *)dst;
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.tiles_x = 0;
  p.omega = (T)h->omega;
  p.u6 = (T)(h->u_lid / 6.0);
  const int tx = (h->nx + TX - 1) / TX, ty = (h->ny + TY - 1) / TY;
  if (mon > 0 && tx * ty > h->partial_slots) return hipErrorInvalidValue;
  const TbMonitor m{h->uref, h->partials, h->mon_dev};
  if (mon == 1)
    hipLaunchKernelGGL((k_step_tb<T, S, K, TX, TY, NT, 1, PP>), dim3(tx * ty), dim3(NT), 0,
                       st, p, tx, m);
  else if (mon == 2)
    hipLaunchKernelGGL((k_step_tb<T, S, K, TX, TY, NT, 2, PP>), dim3(tx * ty), dim3(NT), 0,
                       st, p, tx, m);
  else
    hipLaunchKernelGGL((k_step_tb<T, S, K, TX, TY, NT, 0, PP>), dim3(tx * ty), dim3(NT), 0,
                       st, p, tx, m);
  return hipGetLastError();
}

// mon applies to the multi-step shapes (12-23) only.
template <typename T, bool S>
static hipError_t launch_step_variant(const lbm_cavity *h, int v, const void *src,
                                      void *dst, hipStream_t st, int mon) {
  switch (v) {
    case 12: return launch_tb_t<T, S, 4, 32, 32, 512>(h, src, dst, st, mon);
    case 13: return launch_tb_t<T, S, 4, 32, 32, 1024>(h, src, dst, st, mon);
    case 14: return launch_tb_t<T, S, 2, 32, 32, 512>(h, src, dst, st, mon);
    case 15: return launch_tb_t<T, S, 5, 32, 32, 512>(h, src, dst, st, mon);
    case 16: return launch_tb_t<T, S, 4, 64, 16, 512>(h, src, dst, st, mon);
    case 17: return launch_tb_t<T, S, 4, 16, 16, 256>(h, src, dst, st, mon);
    case 18: return launch_tb_t<T, S, 5, 64, 16, 512>(h, src, dst, st, mon);
    case 19: return launch_tb_t<T, S, 5, 16, 16, 256>(h, src, dst, st, mon);
    case 22: return launch_tb_t<T, S, 5, 32, 32, 1024>(h, src, dst, st, mon);
    // FP64 regions hold twice the bytes per site: smaller tiles keep the
    // LDS of the K = 10 and 64 x 32 shapes within 160 KiB
    case 20:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 10, 32, 16, 512>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 10, 32, 32, 512>(h, src, dst, st, mon);
    case 21:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 10, 16, 16, 256>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 10, 64, 32, 1024>(h, src, dst, st, mon);
    case 23:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 5, 64, 16, 1024>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 5, 64, 32, 1024>(h, src, dst, st, mon);
    // two LDS buffers (one barrier per in-LDS step)
    case 24:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 5, 16, 16, 256, true>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 5, 32, 32, 1024, true>(h, src, dst, st, mon);
    case 25:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 4, 16, 16, 256, true>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 4, 32, 32, 1024, true>(h, src, dst, st, mon);
    case 26:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 5, 32, 16, 512>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 5, 32, 16, 512, true>(h, src, dst, st, mon);
    // tall tiles: one tile per CU on 500 x 750 (32 x 48) and 500 x 1000 (32 x 64)
    case 27:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 5, 16, 48, 512>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 5, 32, 48, 1024>(h, src, dst, st, mon);
    case 28:
      if constexpr (sizeof(T) == 8)
        return launch_tb_t<T, S, 5, 16, 64, 512>(h, src, dst, st, mon);
      else
        return launch_tb_t<T, S, 5, 32, 64, 1024>(h, src, dst, st, mon);
    case 0: return launch_step_t<T, S, 4, 1>(h, src, dst, st);
    case 1: return launch_step_t<T, S, 4, 2>(h, src, dst, st);
    case 2: return launch_step_t<T, S, 4, 4>(h, src, dst, st);
    case 3: return launch_step_t<T, S, 8, 1>(h, src, dst, st);
    case 4: return launch_step_t<T, S, 2, 4>(h, src, dst, st);
    case 5: return launch_step_t<T, S, 1, 8>(h, src, dst, st);
    case 6: return launch_step_t<T, S, 8, 2>(h, src, dst, st);
    case 7: return launch_step_t<T, S, 16, 1>(h, src, dst, st);
    case 8: return launch_step_vec_t<T, S, 1>(h, src, dst, st);
    case 9: return launch_step_vec_t<T, S, 2>(h, src, dst, st);
    case 10: return launch_step_vec_t<T, S, 4>(h, src, dst, st);
    case 11: return launch_step_vec_t<T, S, 8>(h, src, dst, st);
    default: return hipErrorInvalidValue;   // a shape without a kernel
  }
}

// One launch of variant v (steps_per_launch(v) steps); mon (multi-step
// shapes only): see launch_tb_t.
static hipError_t launch_variant(const lbm_cavity *h, int v, const void *src, void *dst,
                                 hipStream_t st, int mon = 0) {
  if (h->wall == LBM_WALL_NEE) {
    if (h->dtype == LBM_F64) return launch_nee_variant<double, false>(h, v, src, dst, st);
    return launch_nee_variant<float, true>(h, v, src, dst, st);
  }
  if (h->dtype == LBM_F64) return launch_step_variant<double, false>(h, v, src, dst, st, mon);
  return launch_step_variant<float, true>(h, v, src, dst, st, mon);
}

// The one-step shape: the chosen shape if it is one, else shape 0.
static int one_step_variant(const lbm_cavity *h) {
  return launch_steps(h, h->variant) == 1 ? h->variant : 0;
}

// One step (a one-step variant: the chosen one, or the default).
static hipError_t launch_step(const lbm_cavity *h, const void *src, void *dst,
                              hipStream_t st) {
  return launch_variant(h, one_step_variant(h), src, dst, st);
}

// Variant used for 100-step chunks: a multi-step variant only if the probe
// cadence falls on its launch boundaries.
static int chunk_variant(const lbm_cavity *h) {
  const int k = launch_steps(h, h->variant);
  if (k > 1 && h->probe_n > 0 && h->probe_every <= kChunk && h->probe_every % k != 0) return 0;
  return h->variant;
}

// ------------------------------------------------------------ small kernels
static Geometry geom(const lbm_cavity *h) {
  Geometry g;
  g.nx = h->nx;
  g.ny = h->ny;
  g.pitch = h->pitch;
  g.plane = h->plane;
  g.on_node = h->wall == LBM_WALL_NEE;
  return g;
}

template <typename T, bool S>
static hipError_t launch_monitor_t(const lbm_cavity *h, const void *src,
                                   bool update, double *out, hipStream_t st) {
  const int n = h->nx * h->ny;
  const int blocks = std::min(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
  if (update)
    hipLaunchKernelGGL((k_monitor<T, S, true>), dim3(blocks), dim3(kRedThreads), 0,
                       st, (const T *)src, geom(h), h->uref, h->partials);
  else
    hipLaunchKernelGGL((k_monitor<T, S, false>), dim3(blocks), dim3(kRedThreads),
                       0, st, (const T *)src, geom(h), h->uref, h->partials);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, st, h->partials,
                     blocks, out);
  return hipGetLastError();
}

static hipError_t launch_monitor(const lbm_cavity *h, const void *src, bool update,
                                 double *out, hipStream_t st) {
  if (h->dtype == LBM_F64) return launch_monitor_t<double, false>(h, src, update, out, st);
  return launch_monitor_t<float, true>(h, src, update, out, st);
}

static hipError_t launch_probe_ring(const lbm_cavity *h, const void *src,
                                    hipStream_t st) {
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_probe_ring<double, false>), dim3(1), dim3(256), 0, st,
                       (const double *)src, geom(h), h->probe_xy, h->probe_n,
                       h->probe_ring, (long long)h->probe_cap, h->probe_count);
  else
    hipLaunchKernelGGL((k_probe_ring<float, true>), dim3(1), dim3(256), 0, st,
                       (const float *)src, geom(h), h->probe_xy, h->probe_n,
                       h->probe_ring, (long long)h->probe_cap, h->probe_count);
  return hipGetLastError();
}

static int ensure_tmp(lbm_cavity *h, size_t doubles) {
  if (h->tmp_doubles >= doubles) return LBM_OK;
  if (h->tmp) HIPC(hipFree(h->tmp));
  h->tmp = nullptr;
  h->tmp_doubles = 0;
  HIPC(hipMalloc(&h->tmp, doubles * sizeof(double)));
  h->tmp_doubles = doubles;
  return LBM_OK;
}

static bool probe_every_ok(int every) {
  return every > 0 && (kChunk % every == 0 || every % kChunk == 0);
}

static void drop_graphs(lbm_cavity *h) {
  for (int c = 0; c < 2; ++c) {
    if (h->graph[c]) (void)hipGraphExecDestroy(h->graph[c]);
    h->graph[c] = nullptr;
  }
}

// Buffer index holding the state after a 100-step chunk that starts in
// buf[c] (an odd number of launches per chunk swaps the buffers).
static int chunk_end(const lbm_cavity *h, int c) {
  const int launches = kChunk / launch_steps(h, chunk_variant(h));
  return (launches & 1) ? 1 - c : c;
}

// Whether chunks take the Eq. 6 monitor of their start state within their
// first two launches (multi-step shapes: at least ten launches per chunk),
// instead of a separate monitor pass at their end.  The state a fused chunk
// ends in is then monitored by the next chunk, or by a separate pass
// (step_impl's `pending`).
static bool fused_monitor(const lbm_cavity *h) {
  return h->wall != LBM_WALL_NEE && launch_steps(h, chunk_variant(h)) > 1;
}

// Issue one 100-step chunk starting from buf[c] on stream st (either
// directly or under capture): with the monitor of the start state carried
// by the first two launches, or ending with the monitor of the end state.
static hipError_t issue_chunk(lbm_cavity *h, int c, hipStream_t st) {
  const int v = chunk_variant(h);
  const int K = launch_steps(h, v);
  const bool fused = fused_monitor(h);
  int cur = c;
  for (int k = K; k <= kChunk; k += K) {
    const int mon = !fused ? 0 : k == K ? 1 : k == 2 * K ? 2 : 0;
    hipError_t e = launch_variant(h, v, h->buf[cur], h->buf[1 - cur], st, mon);
    if (e != hipSuccess) return e;
    cur = 1 - cur;
    if (h->probe_n > 0 && h->probe_every <= kChunk && k % h->probe_every == 0) {
      e = launch_probe_ring(h, h->buf[cur], st);
      if (e != hipSuccess) return e;
    }
  }
  if (fused) return hipSuccess;
  return launch_monitor(h, h->buf[cur], true, h->mon_dev, st);
}

// Add one 100-step chunk's launches (issue_chunk) to the call's record.
static void record_chunk(lbm_cavity *h) {
  lbm_launch_record_t &rec = h->last_call;
  const int v = chunk_variant(h);
  const int K = launch_steps(h, v);
  if (K > 1) {
    rec.multi_variant = v;
    rec.steps_per_launch = K;
    rec.multi_launches += kChunk / K;
  } else {
    rec.single_variant = v;
    rec.single_launches += kChunk;
  }
  if (fused_monitor(h))
    rec.multi_monitor_launches += 2;
  else
    rec.monitor_passes += 1;
  if (h->probe_n > 0 && h->probe_every <= kChunk) rec.probe_launches += kChunk / h->probe_every;
}

static int build_graph(lbm_cavity *h, int c) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = issue_chunk(h, c, h->cap_stream);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return lbm_fail(LBM_EDEVICE, "graph capture failed: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&h->graph[c], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph[c] = nullptr;
    return lbm_fail(LBM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

// Reference field of Eq. 6 := current u; restart the step counter.
static int reset_counters(lbm_cavity *h) {
  h->t = 0;
  h->snap_t = 0;
  h->mon_t = -1;
  h->last_res = INFINITY;
  h->last_mass = NAN;
  h->probe_n = 0;
  drop_graphs(h);
  hipError_t e = launch_monitor(h, h->buf[h->cur], true, h->aux_dev, h->stream);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

template <typename T, bool S>
static void launch_moments_t(lbm_cavity *h, double *r, double *u, double *v) {
  const int n = h->nx * h->ny;
  hipLaunchKernelGGL((k_moments<T, S>), dim3((n + 255) / 256), dim3(256), 0, h->stream,
                     (const T *)h->buf[h->cur], geom(h), r, u, v);
}

// ------------------------------------------------------------------- C ABI
extern "C" {

const char *lbm_last_error(void) { return g_lbm_err.c_str(); }

const char *lbm_version(void) { return "mi355x-lbm 0.1 (gfx950)"; }

static int create_impl(int nx, int ny, double tau, double re, double u_lid,
                       int dtype, int wall, lbm_t *out) {
  if (!out) return lbm_fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 2 || ny < 2 || nx > 65536 || ny > 65536)
    return lbm_fail(LBM_EINVAL, "lattice %d x %d outside [2, 65536]", nx, ny);
  if (wall != LBM_WALL_BOUNCE_BACK && wall != LBM_WALL_NEE)
    return lbm_fail(LBM_EINVAL, "unknown wall scheme %d", wall);
  if (wall == LBM_WALL_NEE && (nx < 3 || ny < 3))
    return lbm_fail(LBM_EINVAL, "on-node walls need at least 3 x 3 nodes, got %d x %d", nx,
                    ny);
  if (dtype != LBM_F64 && dtype != LBM_F32_SHIFTED)
    return lbm_fail(LBM_EINVAL, "unknown dtype %d", dtype);
  if (!std::isfinite(u_lid) || std::fabs(u_lid) >= 1.0 / std::sqrt(3.0))
    return lbm_fail(LBM_EINVAL, "|u_lid| = %g must be below c_s = 1/sqrt(3)", u_lid);
  if (!std::isfinite(tau) || !(tau > 0.5))
    return lbm_fail(LBM_EINVAL, "tau = %.17g must exceed 1/2", tau);
  const int pitch = (nx + 63) / 64 * 64;
  const long long plane = (long long)pitch * ny;
  if (plane * 9 >= (1LL << 31))
    return lbm_fail(LBM_EINVAL, "lattice too large for 32-bit element offsets");

  lbm_cavity *h = new (std::nothrow) lbm_cavity();
  if (!h) return lbm_fail(LBM_ENOMEM, "host allocation");
  h->nx = nx;
  h->ny = ny;
  h->pitch = pitch;
  h->plane = (int)plane;
  h->dtype = dtype;
  h->wall = wall;
  h->re = re;
  h->u_lid = u_lid;
  h->tau = tau;
  h->omega = 1.0 / tau;
  h->variant = wall == LBM_WALL_NEE ? kDefaultNeeVariant : kDefaultVariant;
  h->use_graph = 1;
  const size_t esz = dtype == LBM_F64 ? 8 : 4;
  h->buf_bytes = (size_t)plane * 9 * esz;
  int rc = LBM_OK;
  auto bail = [&](int code) {
    lbm_destroy(h);
    return code;
  };
  hipError_t e;
#define TRY(call)                                                              \
  do {                                                                         \
    e = (call);                                                                \
    if (e != hipSuccess)                                                       \
      return bail(lbm_fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,    \
                       "%s failed: %s", #call, hipGetErrorString(e)));         \
  } while (0)
  TRY(hipGetDevice(&h->device));
  TRY(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
  h->stream = h->own_stream;
  TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  for (int c = 0; c < 2; ++c) {
    TRY(hipMalloc(&h->buf[c], h->buf_bytes));
    TRY(hipMemsetAsync(h->buf[c], 0, h->buf_bytes, h->stream));
  }
  TRY(hipMalloc(&h->uref, sizeof(double2) * (size_t)nx * ny));
  // partial sums: the monitor's fixed grid, or one triple per tile of the
  // smallest multi-step tile (16 x 16) for the fused monitor
  h->partial_slots = std::max(kRedBlocks, ((nx + 15) / 16) * ((ny + 15) / 16));
  TRY(hipMalloc(&h->partials, sizeof(double) * kNumSums * (size_t)h->partial_slots));
  TRY(hipMalloc(&h->mon_dev, sizeof(double) * 4));
  TRY(hipMalloc(&h->aux_dev, sizeof(double) * 4));
  TRY(hipHostMalloc(&h->mon_host, sizeof(double) * 8, hipHostMallocDefault));
  h->cur = 0;
  const int total = pitch * ny;
  if (dtype == LBM_F64)
    hipLaunchKernelGGL((k_init_eq<double, false>), dim3((total + 255) / 256), dim3(256),
                       0, h->stream, (double *)h->buf[0], geom(h), nullptr, nullptr,
                       nullptr, 1.0, 0.0, 0.0);
  else
    hipLaunchKernelGGL((k_init_eq<float, true>), dim3((total + 255) / 256), dim3(256), 0,
                       h->stream, (float *)h->buf[0], geom(h), nullptr, nullptr,
                       nullptr, 1.0, 0.0, 0.0);
  TRY(hipGetLastError());
  if (wall == LBM_WALL_NEE) {   // the lid's nodes start with the lid's velocity
    if (dtype == LBM_F64)
      hipLaunchKernelGGL((k_init_lid_row<double, false>), dim3((nx + 255) / 256), dim3(256), 0,
                         h->stream, (double *)h->buf[0], geom(h), u_lid);
    else
      hipLaunchKernelGGL((k_init_lid_row<float, true>), dim3((nx + 255) / 256), dim3(256), 0,
                         h->stream, (float *)h->buf[0], geom(h), u_lid);
    TRY(hipGetLastError());
  }
  rc = reset_counters(h);
  if (rc != LBM_OK) return bail(rc);
  TRY(hipStreamSynchronize(h->stream));
#undef TRY
  *out = h;
  return LBM_OK;
}

int lbm_create(int nx, int ny, double re, double u_lid, int dtype, lbm_t *out) {
  if (!(re > 0.0) || !std::isfinite(re))
    return lbm_fail(LBM_EINVAL, "re = %g must be positive and finite", re);
  const double tau = 3.0 * u_lid * nx / re + 0.5;   // Eq. 5, nu = U L / Re
  if (!(tau > 0.5))
    return lbm_fail(LBM_EINVAL, "tau = 3 u nx / re + 1/2 = %.17g must exceed 1/2", tau);
  return create_impl(nx, ny, tau, re, u_lid, dtype, LBM_WALL_BOUNCE_BACK, out);
}

int lbm_create_tau(int nx, int ny, double tau, double u_lid, int dtype, lbm_t *out) {
  const double re = (tau > 0.5 && u_lid != 0.0) ? 3.0 * u_lid * nx / (tau - 0.5)
                                                 : INFINITY;
  return create_impl(nx, ny, tau, re, u_lid, dtype, LBM_WALL_BOUNCE_BACK, out);
}

int lbm_create_wall(int nx, int ny, double re, double u_lid, int dtype, int wall,
                    lbm_t *out) {
  if (wall != LBM_WALL_NEE) {
    if (wall != LBM_WALL_BOUNCE_BACK) {
      if (out) *out = nullptr;
      return lbm_fail(LBM_EINVAL, "unknown wall scheme %d", wall);
    }
    return lbm_create(nx, ny, re, u_lid, dtype, out);
  }
  if (!(re > 0.0) || !std::isfinite(re))
    return lbm_fail(LBM_EINVAL, "re = %g must be positive and finite", re);
  // Eq. 5 with L = nx - 1: the on-node walls are nx - 1 spacings apart
  const double tau = 3.0 * u_lid * (nx - 1) / re + 0.5;
  if (!(tau > 0.5))
    return lbm_fail(LBM_EINVAL, "tau = 3 u (nx - 1) / re + 1/2 = %.17g must exceed 1/2", tau);
  return create_impl(nx, ny, tau, re, u_lid, dtype, LBM_WALL_NEE, out);
}

int lbm_destroy(lbm_t h) {
  if (!h) return LBM_OK;
  drop_graphs(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (int c = 0; c < 2; ++c)
    if (h->buf[c]) (void)hipFree(h->buf[c]);
  if (h->uref) (void)hipFree(h->uref);
  if (h->partials) (void)hipFree(h->partials);
  if (h->mon_dev) (void)hipFree(h->mon_dev);
  if (h->aux_dev) (void)hipFree(h->aux_dev);
  if (h->mon_host) (void)hipHostFree(h->mon_host);
  if (h->tmp) (void)hipFree(h->tmp);
  if (h->probe_xy) (void)hipFree(h->probe_xy);
  if (h->probe_ring) (void)hipFree(h->probe_ring);
  if (h->probe_count) (void)hipFree(h->probe_count);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
  return LBM_OK;
}

int lbm_set_stream(lbm_t h, void *hip_stream) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  HIPC(hipStreamSynchronize(h->stream));
  h->stream = hip_stream ? (hipStream_t)hip_stream : h->own_stream;
  return LBM_OK;
}

int lbm_info(lbm_t h, lbm_info_t *info) {
  if (!h || !info) return lbm_fail(LBM_EINVAL, "NULL argument");
  info->nx = h->nx;
  info->ny = h->ny;
  info->pitch = h->pitch;
  info->dtype = h->dtype;
  info->re = h->re;
  info->u_lid = h->u_lid;
  info->tau = h->tau;
  info->omega = h->omega;
  info->steps_done = h->t;
  info->device_bytes = 2 * h->buf_bytes + sizeof(double2) * (size_t)h->nx * h->ny +
                       h->tmp_doubles * sizeof(double);
  info->wall = h->wall;
  return LBM_OK;
}

int lbm_set_option(lbm_t h, int option, int64_t value) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  switch (option) {
    case LBM_OPT_USE_GRAPH:
      h->use_graph = value ? 1 : 0;
      return LBM_OK;
    case LBM_OPT_SYNC:
      h->sync_calls = value ? 1 : 0;
      return LBM_OK;
    case LBM_OPT_STEP_VARIANT:
      if (value < 0 || value >= num_variants(h))
        return lbm_fail(LBM_EINVAL, "variant %lld outside [0, %d)", (long long)value,
                        num_variants(h));
      if (h->variant != (int)value) drop_graphs(h);
      h->variant = (int)value;
      return LBM_OK;
    default:
      return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

int lbm_get_option(lbm_t h, int option, int64_t *value) {
  if (!h || !value) return lbm_fail(LBM_EINVAL, "NULL argument");
  switch (option) {
    case LBM_OPT_USE_GRAPH: *value = h->use_graph; return LBM_OK;
    case LBM_OPT_SYNC: *value = h->sync_calls; return LBM_OK;
    case LBM_OPT_STEP_VARIANT: *value = h->variant; return LBM_OK;
    case LBM_OPT_NUM_VARIANTS: *value = num_variants(h); return LBM_OK;
    case LBM_OPT_STEPS_PER_LAUNCH: *value = launch_steps(h, h->variant); return LBM_OK;
    case LBM_OPT_TILE_X:
    case LBM_OPT_TILE_Y: {
      int tx = 64, ty = 4;
      if (h->wall == LBM_WALL_NEE) {
        nee_tile_of(h->variant, h->dtype, tx, ty);
      } else {
        tile_of(h->variant, h->dtype, tx, ty);
      }
      *value = option == LBM_OPT_TILE_X ? tx : ty;
      return LBM_OK;
    }
    default: return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

// Host bookkeeping after a monitor at step t: the Eq. 6 reference is valid
// only if it was taken exactly 100 steps earlier.
static void note_monitor(lbm_cavity *h) {
  h->mon_valid = (h->snap_t == h->t - kChunk);
  h->snap_t = h->t;
  h->mon_t = h->t;
}

static int step_impl(lbm_t h, int64_t n);

int lbm_step(lbm_t h, int64_t n) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  if (n < 0) return lbm_fail(LBM_EINVAL, "n = %lld < 0", (long long)n);
  if (n == 0) return LBM_OK;
  h->last_call = lbm_launch_record_t{};
  h->last_call.multi_variant = -1;
  h->last_call.single_variant = -1;
  const int64_t t_start = h->t;
  const double t0 = lbm_wall_seconds();
  const int rc = step_impl(h, n);
  h->last_call.steps = h->t - t_start;
  const double sec = lbm_wall_seconds() - t0;
  char mass[32], res[32];
  lbm_log_line("{\"kind\": \"cavity\", \"handle\": \"%p\", \"nx\": %d, \"ny\": %d, "
               "\"dtype\": %d, \"wall\": %d, \"steps\": %lld, \"step\": %lld, "
               "\"mass\": %s, \"residual\": %s, \"residual_step\": %lld, "
               "\"seconds\": %.6f, \"MLUPS\": %.1f, \"rc\": %d}",
               (void *)h, h->nx, h->ny, h->dtype, h->wall, (long long)n, (long long)h->t,
               lbm_json_num(h->last_mass, mass),
               lbm_json_num(h->mon_t >= 0 ? h->last_res : INFINITY, res), (long long)h->mon_t,
               sec, sec > 0 ? (double)h->nx * h->ny * n / sec / 1e6 : 0.0, rc);
  return rc;
}

static int step_impl(lbm_t h, int64_t n) {
  bool monitored = false;
  // The state at h->t is a monitor point (a multiple of 100) that no monitor
  // has seen yet: a fused chunk leaves its end state so, and so does a
  // multi-step launch off the chunk grid that ends on a multiple of 100.  The
  // next fused chunk's first launch takes it, or a separate pass before
  // further launches off the grid and at the end of the call.  (A fused
  // chunk also re-monitors a start state that was seen already: u_ref
  // receives the same values and the sums it writes are overwritten by a
  // later monitor of this call.)
  bool pending = false;
  lbm_launch_record_t &rec = h->last_call;
  hipError_t e;
  auto monitor_now = [&]() -> int {
    hipError_t me = launch_monitor(h, h->buf[h->cur], true, h->mon_dev, h->stream);
    if (me != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor: %s", hipGetErrorString(me));
    note_monitor(h);
    rec.monitor_passes += 1;
    monitored = true;
    pending = false;
    return LBM_OK;
  };
  auto probe_now = [&]() -> int {
    hipError_t pe = launch_probe_ring(h, h->buf[h->cur], h->stream);
    if (pe != hipSuccess) return lbm_fail(LBM_EDEVICE, "probe: %s", hipGetErrorString(pe));
    rec.probe_launches += 1;
    return LBM_OK;
  };
  while (n > 0) {
    const bool aligned = (h->t % kChunk) == 0;
    if (aligned && n >= kChunk) {
      const bool fused = fused_monitor(h);
      if (fused && pending) {   // the chunk's first launch monitors the state at t
        note_monitor(h);
        pending = false;
      }
      if (h->use_graph) {
        if (!h->graph[h->cur]) {
          int rc = build_graph(h, h->cur);
          if (rc != LBM_OK) return rc;
        }
        HIPC(hipGraphLaunch(h->graph[h->cur], h->stream));
        rec.graph_replays += 1;
      } else {
        e = issue_chunk(h, h->cur, h->stream);
        if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "launch: %s", hipGetErrorString(e));
      }
      record_chunk(h);
      h->cur = chunk_end(h, h->cur);
      h->t += kChunk;
      n -= kChunk;
      if (fused)
        pending = true;
      else
        note_monitor(h);
      monitored = true;
      if (h->probe_n > 0 && h->probe_every > kChunk && h->t % h->probe_every == 0) {
        const int rc = probe_now();
        if (rc != LBM_OK) return rc;
      }
      continue;
    }
    // Off the 100-step grid, up to the next chunk boundary: launches of the
    // chunk's multi-step shape while t is a multiple of its K and K steps
    // remain (K divides 100, so no launch crosses a monitor point, and the
    // chunk shape's K divides the probe cadence), one-step launches for the
    // rest.
    if (pending) {
      const int rc = monitor_now();
      if (rc != LBM_OK) return rc;
    }
    const int v = chunk_variant(h);
    const int K = launch_steps(h, v);
    const bool multi = K > 1 && h->t % K == 0 && n >= K;
    if (multi) {
      e = launch_variant(h, v, h->buf[h->cur], h->buf[1 - h->cur], h->stream, 0);
      rec.multi_variant = v;
      rec.steps_per_launch = K;
      rec.multi_launches += 1;
    } else {
      e = launch_step(h, h->buf[h->cur], h->buf[1 - h->cur], h->stream);
      rec.single_variant = one_step_variant(h);
      rec.single_launches += 1;
    }
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "step launch: %s", hipGetErrorString(e));
    const int done = multi ? K : 1;
    h->cur = 1 - h->cur;
    h->t += done;
    n -= done;
    if (h->probe_n > 0 && h->t % h->probe_every == 0) {
      const int rc = probe_now();
      if (rc != LBM_OK) return rc;
    }
    if (h->t % kChunk == 0) {
      if (fused_monitor(h)) {   // taken by the next fused chunk, or a separate pass
        pending = true;
        monitored = true;
      } else {
        const int rc = monitor_now();
        if (rc != LBM_OK) return rc;
      }
    }
  }
  if (pending) {
    const int rc = monitor_now();
    if (rc != LBM_OK) return rc;
  }
  if (!monitored && !h->sync_calls) return LBM_OK;   // issued; nothing to read back
  if (monitored) {
    HIPC(hipMemcpyAsync(h->mon_host, h->mon_dev, 3 * sizeof(double),
                        hipMemcpyDeviceToHost, h->stream));
  }
  HIPC(hipStreamSynchronize(h->stream));
  if (monitored) {
    const double *m = h->mon_host;
    h->last_mass = (double)h->nx * h->ny + m[0];
    h->last_res = (h->mon_valid && m[2] > 0.0) ? std::sqrt(m[1] / m[2]) : INFINITY;
    if (!std::isfinite(h->last_mass) || std::isnan(h->last_res))
      return lbm_fail(LBM_EUNSTABLE, "non-finite monitor at step %lld (mass %g)",
                  (long long)h->t, h->last_mass);
  }
  return LBM_OK;
}

int lbm_autotune(lbm_t h, int chunks, int use_cache, int *best_variant, double *ms_per_step) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  if (chunks < 1 || chunks > 10000)
    return lbm_fail(LBM_EINVAL, "chunks = %d outside [1, 10000]", chunks);
  if (h->t % kChunk != 0) return lbm_fail(LBM_EINVAL, "autotune only at a multiple of 100 steps");
  const std::string key =
      tune_key(h->wall == LBM_WALL_NEE ? "single-nee" : "single", h->dtype, h->nx, h->ny);
  const int cached = use_cache ? tune_cache_lookup(key) : -1;
  if (cached >= 0 && cached < num_variants(h)) {
    if (best_variant) *best_variant = cached;
    if (ms_per_step) *ms_per_step = NAN;
    return lbm_set_option(h, LBM_OPT_STEP_VARIANT, cached);
  }
  const size_t uref_bytes = sizeof(double2) * (size_t)h->nx * h->ny;
  void *save_f = nullptr, *save_u = nullptr;
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMalloc(&save_f, h->buf_bytes));
  hipError_t e = hipMalloc(&save_u, uref_bytes);
  if (e != hipSuccess) {
    (void)hipFree(save_f);
    return lbm_fail(LBM_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  }
  const int cur0 = h->cur;
  auto restore = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(h->buf[cur0], save_f, h->buf_bytes, hipMemcpyDeviceToDevice,
                                  h->stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(h->uref, save_u, uref_bytes, hipMemcpyDeviceToDevice, h->stream);
    return r;
  };
  e = hipMemcpyAsync(save_f, h->buf[cur0], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(save_u, h->uref, uref_bytes, hipMemcpyDeviceToDevice, h->stream);
  const int64_t t0 = h->t, snap0 = h->snap_t, mon0 = h->mon_t;
  const bool valid0 = h->mon_valid;
  const double res0 = h->last_res, mass0 = h->last_mass;
  const int probe_n0 = h->probe_n;
  h->probe_n = 0;                 // no probe records during the trials
  drop_graphs(h);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  double best_ms = INFINITY;
  int best = h->variant;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int v = 0; v < num_variants(h) && e == hipSuccess && rc == LBM_OK; ++v) {
    rc = lbm_set_option(h, LBM_OPT_STEP_VARIANT, v);
    if (rc == LBM_OK) rc = lbm_step(h, kChunk);           // warm-up and capture
    if (rc != LBM_OK) break;
    e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess) rc = lbm_step(h, (int64_t)chunks * kChunk);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double per_step = ms / ((double)chunks * kChunk);
    if (rc == LBM_OK && e == hipSuccess && per_step < best_ms) {
      best_ms = per_step;
      best = v;
    }
    h->cur = cur0;
    if (e == hipSuccess) e = restore();
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->cur = cur0;
  if (e == hipSuccess) e = restore();
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(save_f);
  (void)hipFree(save_u);
  h->t = t0;
  h->snap_t = snap0;
  h->mon_t = mon0;
  h->mon_valid = valid0;
  h->last_res = res0;
  h->last_mass = mass0;
  h->probe_n = probe_n0;
  drop_graphs(h);
  if (rc != LBM_OK) return rc;
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "autotune: %s", hipGetErrorString(e));
  rc = lbm_set_option(h, LBM_OPT_STEP_VARIANT, best);
  if (rc) return rc;
  tune_cache_store(key, best);
  if (best_variant) *best_variant = best;
  if (ms_per_step) *ms_per_step = best_ms;
  return LBM_OK;
}

int lbm_last_launches(lbm_t h, lbm_launch_record_t *out) {
  if (!h || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
  *out = h->last_call;
  return LBM_OK;
}

int lbm_steps_done(lbm_t h, int64_t *t) {
  if (!h || !t) return lbm_fail(LBM_EINVAL, "NULL argument");
  *t = h->t;
  return LBM_OK;
}

int lbm_moments_device(lbm_t h, double *rho, double *ux, double *uy) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  if (h->dtype == LBM_F64) launch_moments_t<double, false>(h, rho, ux, uy);
  else launch_moments_t<float, true>(h, rho, ux, uy);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_moments(lbm_t h, double *rho, double *ux, double *uy) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  const size_t n = (size_t)h->nx * h->ny;
  int rc = ensure_tmp(h, 3 * n);
  if (rc) return rc;
  double *d[3] = {rho ? h->tmp : nullptr, ux ? h->tmp + n : nullptr,
                  uy ? h->tmp + 2 * n : nullptr};
  if (h->dtype == LBM_F64) launch_moments_t<double, false>(h, d[0], d[1], d[2]);
  else launch_moments_t<float, true>(h, d[0], d[1], d[2]);
  HIPC(hipGetLastError());
  double *outs[3] = {rho, ux, uy};
  for (int k = 0; k < 3; ++k)
    if (outs[k])
      HIPC(hipMemcpyAsync(outs[k], d[k], n * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_probe(lbm_t h, int npts, const double *xy, double *out) {
  if (!h || !xy || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (npts < 1 || npts > 4096) return lbm_fail(LBM_EINVAL, "npts = %d outside [1, 4096]", npts);
  for (int i = 0; i < 2 * npts; ++i)
    if (!std::isfinite(xy[i])) return lbm_fail(LBM_EINVAL, "probe coordinate %d not finite", i);
  int rc = ensure_tmp(h, 5 * (size_t)npts);
  if (rc) return rc;
  HIPC(hipMemcpyAsync(h->tmp, xy, 2 * npts * sizeof(double), hipMemcpyHostToDevice,
                      h->stream));
  double *res = h->tmp + 2 * npts;
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_probe<double, false>), dim3((npts + 255) / 256), dim3(256), 0,
                       h->stream, (const double *)h->buf[h->cur], geom(h), h->tmp, npts, res);
  else
    hipLaunchKernelGGL((k_probe<float, true>), dim3((npts + 255) / 256), dim3(256), 0,
                       h->stream, (const float *)h->buf[h->cur], geom(h), h->tmp, npts, res);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(out, res, 3 * npts * sizeof(double), hipMemcpyDeviceToHost,
                      h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_probe_config(lbm_t h, int npts, const double *xy, int every, int64_t capacity) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  HIPC(hipStreamSynchronize(h->stream));
  drop_graphs(h);
  if (npts == 0) {
    h->probe_n = 0;
    return LBM_OK;
  }
  if (!xy || npts < 0 || npts > 4096) return lbm_fail(LBM_EINVAL, "npts = %d outside [1, 4096]", npts);
  if (!probe_every_ok(every))
    return lbm_fail(LBM_EINVAL, "every = %d must divide 100 or be a multiple of 100", every);
  if (capacity < 1 || capacity > (1LL << 26))
    return lbm_fail(LBM_EINVAL, "capacity %lld outside [1, 2^26]", (long long)capacity);
  for (int i = 0; i < 2 * npts; ++i)
    if (!std::isfinite(xy[i])) return lbm_fail(LBM_EINVAL, "probe coordinate %d not finite", i);
  if (h->probe_xy) HIPC(hipFree(h->probe_xy));
  if (h->probe_ring) HIPC(hipFree(h->probe_ring));
  if (!h->probe_count) HIPC(hipMalloc(&h->probe_count, sizeof(unsigned long long)));
  h->probe_xy = nullptr;
  h->probe_ring = nullptr;
  h->probe_n = 0;
  HIPC(hipMalloc(&h->probe_xy, 2 * npts * sizeof(double)));
  HIPC(hipMalloc(&h->probe_ring, (size_t)capacity * 3 * npts * sizeof(double)));
  HIPC(hipMemcpy(h->probe_xy, xy, 2 * npts * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemset(h->probe_count, 0, sizeof(unsigned long long)));
  h->probe_n = npts;
  h->probe_every = every;
  h->probe_cap = capacity;
  // first recorded step: next multiple of `every` after now
  h->probe_t0 = (h->t / every + 1) * every;
  return LBM_OK;
}

int lbm_probe_classify(lbm_t h, int component, int64_t window, double steady_tol,
                       double periodic_tol, int min_lag, int max_lag,
                       lbm_flow_state_t *out) {
  if (!h || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (!h->probe_ring || h->probe_n == 0) return lbm_fail(LBM_EINVAL, "no probes configured");
  if (component < 0 || component > 2)
    return lbm_fail(LBM_EINVAL, "component %d outside {0, 1, 2}", component);
  if (!(steady_tol >= 0.0) || !(periodic_tol >= 0.0))
    return lbm_fail(LBM_EINVAL, "tolerances must be >= 0 (steady %g, periodic %g)", steady_tol,
                    periodic_tol);
  int rc = check_lags(window, min_lag, max_lag);
  if (rc) return rc;
  unsigned long long count = 0;
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMemcpy(&count, h->probe_count, sizeof count, hipMemcpyDeviceToHost));
  const int64_t avail = std::min<int64_t>((int64_t)count, h->probe_cap);
  if (window > avail)
    return lbm_fail(LBM_EINVAL, "window %lld exceeds the %lld records held", (long long)window,
                    (long long)avail);
  const long long start = (long long)((count - (unsigned long long)window) %
                                      (unsigned long long)h->probe_cap);
  std::vector<SeriesDesc> d(h->probe_n);
  for (int p = 0; p < h->probe_n; ++p)
    d[p] = SeriesDesc{h->probe_ring + 3 * p + component, (long long)h->probe_cap, start,
                      (long long)window, 3LL * h->probe_n};
  return classify_series_descs(d.data(), h->probe_n, window, steady_tol, periodic_tol, min_lag,
                               max_lag, h->stream, out);
}

int lbm_probe_read(lbm_t h, double *buf, int64_t max_records, int64_t *n_records) {
  if (!h || !n_records) return lbm_fail(LBM_EINVAL, "NULL argument");
  *n_records = 0;
  if (!h->probe_ring || h->probe_n == 0) return LBM_OK;
  if (max_records > 0 && !buf) return lbm_fail(LBM_EINVAL, "buf is NULL");
  unsigned long long count = 0;
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMemcpy(&count, h->probe_count, sizeof count, hipMemcpyDeviceToHost));
  const int64_t avail = std::min<int64_t>((int64_t)count, h->probe_cap);
  const int64_t take = std::min<int64_t>(avail, max_records);
  const int rec = 3 * h->probe_n;
  std::vector<double> tmp((size_t)rec);
  for (int64_t k = 0; k < take; ++k) {
    const unsigned long long idx = count - take + k;      // record index
    const int64_t slot = (int64_t)(idx % (unsigned long long)h->probe_cap);
    HIPC(hipMemcpy(tmp.data(), h->probe_ring + slot * rec, rec * sizeof(double),
                   hipMemcpyDeviceToHost));
    double *dst = buf + k * (1 + rec);
    dst[0] = (double)(h->probe_t0 + (int64_t)idx * h->probe_every);
    std::memcpy(dst + 1, tmp.data(), rec * sizeof(double));
  }
  *n_records = take;
  return LBM_OK;
}

int lbm_mass(lbm_t h, double *mass) {
  if (!h || !mass) return lbm_fail(LBM_EINVAL, "NULL argument");
  hipError_t e = launch_monitor(h, h->buf[h->cur], false, h->aux_dev, h->stream);
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor: %s", hipGetErrorString(e));
  HIPC(hipMemcpyAsync(h->mon_host + 4, h->aux_dev, sizeof(double), hipMemcpyDeviceToHost,
                      h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  *mass = (double)h->nx * h->ny + h->mon_host[4];
  return LBM_OK;
}

int lbm_residual(lbm_t h, double *residual, int64_t *at_step) {
  if (!h || !residual) return lbm_fail(LBM_EINVAL, "NULL argument");
  *residual = h->mon_t >= 0 ? h->last_res : INFINITY;
  if (at_step) *at_step = h->mon_t;
  return LBM_OK;
}

// Psi of the current state into the device array psi ([ny][nx] FP64).
static int launch_psi(lbm_cavity *h, double *psi) {
  if (h->wall == LBM_WALL_NEE) {
    if (h->dtype == LBM_F64)
      hipLaunchKernelGGL((k_psi_nodes<double, false>), dim3((h->nx + 255) / 256), dim3(256), 0,
                         h->stream, (const double *)h->buf[h->cur], geom(h), psi);
    else
      hipLaunchKernelGGL((k_psi_nodes<float, true>), dim3((h->nx + 255) / 256), dim3(256), 0,
                         h->stream, (const float *)h->buf[h->cur], geom(h), psi);
    HIPC(hipGetLastError());
    return LBM_OK;
  }
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_psi<double, false>), dim3((h->nx + 255) / 256), dim3(256), 0,
                       h->stream, (const double *)h->buf[h->cur], geom(h), psi);
  else
    hipLaunchKernelGGL((k_psi<float, true>), dim3((h->nx + 255) / 256), dim3(256), 0,
                       h->stream, (const float *)h->buf[h->cur], geom(h), psi);
  HIPC(hipGetLastError());
  return LBM_OK;
}

int lbm_stream_function(lbm_t h, double *psi) {
  if (!h || !psi) return lbm_fail(LBM_EINVAL, "NULL argument");
  const size_t n = (size_t)h->nx * h->ny;
  int rc = ensure_tmp(h, n);
  if (rc) return rc;
  rc = launch_psi(h, h->tmp);
  if (rc) return rc;
  HIPC(hipMemcpyAsync(psi, h->tmp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

// ---------------------------------------------------------------- vortices
namespace {
// Views into h->tmp for the vortex routines: Psi, the per-block partials of
// the three regions, the three results, the centre counter and up to `cap`
// centres (value; site index and kind as an int pair).
struct VortexScratch {
  double *psi, *pv, *ov, *ev;
  int *pk, *ok, *ek;
  unsigned int *cnt;
  int nb;
};
}  // namespace

static int vortex_scratch(lbm_cavity *h, size_t cap, VortexScratch &s) {
  const size_t n = (size_t)h->nx * h->ny;
  s.nb = (int)std::min<size_t>(1024, (n + kVortexThreads - 1) / kVortexThreads);
  const size_t pk_doubles = (3 * (size_t)s.nb + 1) / 2;
  int rc = ensure_tmp(h, n + 3 * s.nb + pk_doubles + 3 + 2 + 1 + 2 * cap);
  if (rc) return rc;
  double *p = h->tmp;
  s.psi = p;
  p += n;
  s.pv = p;
  p += 3 * s.nb;
  s.pk = reinterpret_cast<int *>(p);
  p += pk_doubles;
  s.ov = p;
  p += 3;
  s.ok = reinterpret_cast<int *>(p);
  p += 2;
  s.cnt = reinterpret_cast<unsigned int *>(p);
  p += 1;
  s.ev = p;
  p += cap;
  s.ek = reinterpret_cast<int *>(p);
  return LBM_OK;
}

static lbm_vortex_t vortex_record(const lbm_cavity *h, double psi, int k, int kind) {
  lbm_vortex_t v{};
  v.psi = psi;
  v.iy = k / h->nx;
  v.ix = k - v.iy * h->nx;
  if (h->wall == LBM_WALL_NEE) {   // node positions, L = nx - 1
    v.x = (double)v.ix / (h->nx - 1);
    v.y = (double)v.iy / (h->nx - 1);
  } else {                         // site centres, L = nx
    v.x = (v.ix + 0.5) / h->nx;
    v.y = (v.iy + 0.5) / h->nx;
  }
  v.kind = kind;
  return v;
}

int lbm_vortex_extrema(lbm_t h, lbm_vortex_t *out) {
  if (!h || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (h->nx < 2) return lbm_fail(LBM_EINVAL, "nx = %d < 2", h->nx);
  VortexScratch s;
  int rc = vortex_scratch(h, 0, s);
  if (rc) return rc;
  rc = launch_psi(h, s.psi);
  if (rc) return rc;
  hipLaunchKernelGGL(k_vortex_partial, dim3(s.nb), dim3(kVortexThreads), 0, h->stream, s.psi,
                     h->nx, h->ny, s.pv, s.pk);
  HIPC(hipGetLastError());
  hipLaunchKernelGGL(k_vortex_final, dim3(1), dim3(kVortexThreads), 0, h->stream, s.pv, s.pk,
                     s.nb, s.ov, s.ok);
  HIPC(hipGetLastError());
  double v[3];
  int k[3];
  HIPC(hipMemcpyAsync(v, s.ov, sizeof(v), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipMemcpyAsync(k, s.ok, sizeof(k), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  for (int r = 0; r < 3; ++r) {
    if (k[r] < 0) return lbm_fail(LBM_EDEVICE, "vortex region %d came back empty", r);
    out[r] = vortex_record(h, v[r], k[r], r == 0 ? 1 : -1);
  }
  return LBM_OK;
}

// All vortex centres with |Psi| >= min_abs, sorted by site index.
static int find_centres(lbm_cavity *h, double min_abs, std::vector<lbm_vortex_t> &all) {
  const size_t n = (size_t)h->nx * h->ny;
  size_t cap = 4096;
  for (int pass = 0; pass < 2; ++pass) {
    VortexScratch s;
    int rc = vortex_scratch(h, cap, s);
    if (rc) return rc;
    rc = launch_psi(h, s.psi);
    if (rc) return rc;
    HIPC(hipMemsetAsync(s.cnt, 0, sizeof(unsigned int), h->stream));
    hipLaunchKernelGGL(k_vortex_centres, dim3((unsigned)((n + kVortexThreads - 1) / kVortexThreads)),
                       dim3(kVortexThreads), 0, h->stream, s.psi, h->nx, h->ny, min_abs,
                       (int)cap, s.cnt, s.ev, s.ek);
    HIPC(hipGetLastError());
    unsigned int cnt = 0;
    HIPC(hipMemcpyAsync(&cnt, s.cnt, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    if (cnt > cap) {   // more centres than slots: run again with room for all
      cap = cnt;
      continue;
    }
    std::vector<double> ev(cnt);
    std::vector<int> ek(2 * (size_t)cnt);
    if (cnt) {
      HIPC(hipMemcpyAsync(ev.data(), s.ev, cnt * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
      HIPC(hipMemcpyAsync(ek.data(), s.ek, 2 * (size_t)cnt * sizeof(int),
                          hipMemcpyDeviceToHost, h->stream));
      HIPC(hipStreamSynchronize(h->stream));
    }
    all.clear();
    for (unsigned int i = 0; i < cnt; ++i)
      all.push_back(vortex_record(h, ev[i], ek[2 * i], ek[2 * i + 1]));
    std::sort(all.begin(), all.end(), [](const lbm_vortex_t &a, const lbm_vortex_t &b) {
      return a.iy != b.iy ? a.iy < b.iy : a.ix < b.ix;
    });
    return LBM_OK;
  }
  return lbm_fail(LBM_EDEVICE, "vortex centre count changed between two scans");
}

int lbm_vortex_centres(lbm_t h, double min_abs_psi, int cap, lbm_vortex_t *out, int *count) {
  if (!h || !count) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (cap < 0 || (cap > 0 && !out))
    return lbm_fail(LBM_EINVAL, "cap = %d with out = %p", cap, (void *)out);
  if (!(min_abs_psi >= 0.0)) return lbm_fail(LBM_EINVAL, "min_abs_psi = %g", min_abs_psi);
  std::vector<lbm_vortex_t> all;
  int rc = find_centres(h, min_abs_psi, all);
  if (rc) return rc;
  *count = (int)all.size();
  for (int i = 0; i < cap && i < (int)all.size(); ++i) out[i] = all[i];
  return LBM_OK;
}

int lbm_bottom_vortex_count(lbm_t h, double min_abs_psi, int *count) {
  if (!h || !count) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (!(min_abs_psi >= 0.0)) return lbm_fail(LBM_EINVAL, "min_abs_psi = %g", min_abs_psi);
  lbm_vortex_t ext[3];
  int rc = lbm_vortex_extrema(h, ext);
  if (rc) return rc;
  std::vector<lbm_vortex_t> all;
  rc = find_centres(h, min_abs_psi, all);
  if (rc) return rc;
  int c = 0;
  for (const lbm_vortex_t &v : all) c += v.iy < ext[0].iy;
  *count = c;
  return LBM_OK;
}

int lbm_set_populations(lbm_t h, const double *f) {
  if (!h || !f) return lbm_fail(LBM_EINVAL, "NULL argument");
  const size_t n = (size_t)h->nx * h->ny;
  int rc = ensure_tmp(h, 9 * n);
  if (rc) return rc;
  HIPC(hipMemcpyAsync(h->tmp, f, 9 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_set_pop<double, false>), dim3((n + 255) / 256), dim3(256), 0,
                       h->stream, (double *)h->buf[h->cur], geom(h), h->tmp, h->omega);
  else
    hipLaunchKernelGGL((k_set_pop<float, true>), dim3((n + 255) / 256), dim3(256), 0,
                       h->stream, (float *)h->buf[h->cur], geom(h), h->tmp, h->omega);
  HIPC(hipGetLastError());
  rc = reset_counters(h);
  if (rc) return rc;
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_get_populations(lbm_t h, double *f) {
  if (!h || !f) return lbm_fail(LBM_EINVAL, "NULL argument");
  const size_t n = (size_t)h->nx * h->ny;
  int rc = ensure_tmp(h, 9 * n);
  if (rc) return rc;
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_get_pop<double, false>), dim3((n + 255) / 256), dim3(256), 0,
                       h->stream, (const double *)h->buf[h->cur], geom(h), h->tmp);
  else
    hipLaunchKernelGGL((k_get_pop<float, true>), dim3((n + 255) / 256), dim3(256), 0,
                       h->stream, (const float *)h->buf[h->cur], geom(h), h->tmp);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(f, h->tmp, 9 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

static int init_fields_impl(lbm_t h, const double *rho, const double *ux, const double *uy,
                            int flags, bool on_device) {
  if (!h) return lbm_fail(LBM_EINVAL, "handle is NULL");
  const size_t n = (size_t)h->nx * h->ny;
  const double *d[3] = {rho, ux, uy};
  if (!on_device) {
    int rc = ensure_tmp(h, 3 * n);
    if (rc) return rc;
    const double *src[3] = {rho, ux, uy};
    for (int k = 0; k < 3; ++k) {
      d[k] = nullptr;
      if (src[k]) {
        d[k] = h->tmp + k * n;
        HIPC(hipMemcpyAsync(h->tmp + k * n, src[k], n * sizeof(double), hipMemcpyHostToDevice,
                            h->stream));
      }
    }
  }
  double scale = 1.0, sx = 0.0, sy = 0.0;
  const bool renorm = (flags & LBM_INIT_RENORMALISE_MASS) && rho;
  const bool destag = (flags & LBM_INIT_ZERO_STAGGERED) && (ux || uy);
  if (renorm || destag) {
    // FP64 sums on the device (same fixed-order reduction as the monitors):
    // total mass and the two staggered momenta of the fields
    const int blocks = std::min(kRedBlocks, (int)((n + kRedThreads - 1) / kRedThreads));
    hipLaunchKernelGGL(k_init_sums, dim3(blocks), dim3(kRedThreads), 0, h->stream, d[0], d[1],
                       d[2], h->nx, (long long)n, h->partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, h->stream, h->partials,
                       blocks, h->aux_dev);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h->mon_host + 4, h->aux_dev, 3 * sizeof(double),
                        hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    const double total = h->mon_host[4];
    if (renorm) {
      if (!(total > 0.0) || !std::isfinite(total))
        return lbm_fail(LBM_EINVAL, "sum of rho = %g cannot be renormalised", total);
      scale = (double)n / total;
    }
    if (destag) {
      sx = scale * h->mon_host[5] / (double)n;
      sy = scale * h->mon_host[6] / (double)n;
    }
  }
  const int tot = h->pitch * h->ny;
  if (h->dtype == LBM_F64)
    hipLaunchKernelGGL((k_init_eq<double, false>), dim3((tot + 255) / 256), dim3(256), 0,
                       h->stream, (double *)h->buf[h->cur], geom(h), d[0], d[1], d[2], scale,
                       sx, sy);
  else
    hipLaunchKernelGGL((k_init_eq<float, true>), dim3((tot + 255) / 256), dim3(256), 0,
                       h->stream, (float *)h->buf[h->cur], geom(h), d[0], d[1], d[2], scale,
                       sx, sy);
  HIPC(hipGetLastError());
  int rc = reset_counters(h);
  if (rc) return rc;
  HIPC(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_init_fields(lbm_t h, const double *rho, const double *ux, const double *uy,
                    int flags) {
  return init_fields_impl(h, rho, ux, uy, flags, false);
}

int lbm_init_fields_device(lbm_t h, const double *rho, const double *ux, const double *uy,
                           int flags) {
  return init_fields_impl(h, rho, ux, uy, flags, true);
}

// Checkpoint file: header, stored populations of buf[cur], Eq. 6 reference.
struct CkptHeader {
  char magic[8];
  int32_t version, nx, ny, pitch, dtype, wall;
  int64_t t, snap_t, mon_t;
  double tau, u_lid, last_res, last_mass;
  uint64_t buf_bytes, uref_bytes;
};

int lbm_save(lbm_t h, const char *path) {
  if (!h || !path) return lbm_fail(LBM_EINVAL, "NULL argument");
  CkptHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, "LBMD2Q9", 8);
  hd.version = 1;
  hd.nx = h->nx;
  hd.ny = h->ny;
  hd.pitch = h->pitch;
  hd.dtype = h->dtype;
  hd.wall = h->wall;
  hd.t = h->t;
  hd.snap_t = h->snap_t;
  hd.mon_t = h->mon_t;
  hd.tau = h->tau;
  hd.u_lid = h->u_lid;
  hd.last_res = h->last_res;
  hd.last_mass = h->last_mass;
  hd.buf_bytes = h->buf_bytes;
  hd.uref_bytes = sizeof(double2) * (size_t)h->nx * h->ny;
  std::vector<char> a(hd.buf_bytes), b(hd.uref_bytes);
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMemcpy(a.data(), h->buf[h->cur], hd.buf_bytes, hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(b.data(), h->uref, hd.uref_bytes, hipMemcpyDeviceToHost));
  FILE *fp = std::fopen(path, "wb");
  if (!fp) return lbm_fail(LBM_EIO, "cannot open %s for writing", path);
  bool ok = std::fwrite(&hd, sizeof hd, 1, fp) == 1 &&
            std::fwrite(a.data(), 1, a.size(), fp) == a.size() &&
            std::fwrite(b.data(), 1, b.size(), fp) == b.size();
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return lbm_fail(LBM_EIO, "short write to %s", path);
  return LBM_OK;
}

int lbm_load(lbm_t h, const char *path) {
  if (!h || !path) return lbm_fail(LBM_EINVAL, "NULL argument");
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return lbm_fail(LBM_EIO, "cannot open %s", path);
  CkptHeader hd;
  if (std::fread(&hd, sizeof hd, 1, fp) != 1 || std::memcmp(hd.magic, "LBMD2Q9", 8) != 0 ||
      hd.version != 1) {
    std::fclose(fp);
    return lbm_fail(LBM_EIO, "%s is not a checkpoint of this library", path);
  }
  if (hd.nx != h->nx || hd.ny != h->ny || hd.pitch != h->pitch || hd.dtype != h->dtype ||
      hd.wall != h->wall || hd.buf_bytes != h->buf_bytes ||
      hd.uref_bytes != sizeof(double2) * (size_t)h->nx * h->ny) {
    std::fclose(fp);
    return lbm_fail(LBM_ESTATE,
                    "checkpoint lattice %dx%d dtype %d wall %d does not match the handle",
                    hd.nx, hd.ny, hd.dtype, hd.wall);
  }
  std::vector<char> a(hd.buf_bytes), b(hd.uref_bytes);
  const bool ok = std::fread(a.data(), 1, a.size(), fp) == a.size() &&
                  std::fread(b.data(), 1, b.size(), fp) == b.size();
  char extra;
  const bool tail = std::fread(&extra, 1, 1, fp) == 0;
  std::fclose(fp);
  if (!ok || !tail) return lbm_fail(LBM_EIO, "%s is truncated or has trailing bytes", path);
  HIPC(hipStreamSynchronize(h->stream));
  HIPC(hipMemcpy(h->buf[h->cur], a.data(), a.size(), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(h->uref, b.data(), b.size(), hipMemcpyHostToDevice));
  h->t = hd.t;
  h->snap_t = hd.snap_t;
  h->mon_t = hd.mon_t;
  h->tau = hd.tau;
  h->omega = 1.0 / hd.tau;
  h->u_lid = hd.u_lid;
  h->last_res = hd.last_res;
  h->last_mass = hd.last_mass;
  h->probe_n = 0;
  drop_graphs(h);
  return LBM_OK;
}

}  // extern "C"
