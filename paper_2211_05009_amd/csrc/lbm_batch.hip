// lbm_batch.hip -- batched sweep of uneven cavities and the tile-shape
// autotuner (contracts in include/lbm.h).
//
// A batch owns one pair of buffers holding every cavity.  One kernel launch
// advances all active cavities by one step (k_step_batch over a tile table);
// a chunk of `graph_steps` steps (default 1000, a multiple of the 100-step
// monitor cadence) with the per-cavity FP64 monitors after every 100 steps is
// captured once into a HIP graph and replayed.  Cavities whose Eq. 6
// residual falls below a threshold drop out of the tile table at a chunk
// boundary.  Chunk boundaries are reached at even step counts only, so the
// current buffer of every cavity, active or not, is buf[0] there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "d2q9_batch.hpp"
#include "d2q9_series.hpp"
#include "d2q9_monitor.hpp"
#include "d2q9_step.hpp"
#include "lbm_internal.h"

using namespace lbm;

struct lbm_batch {
  int n = 0, dtype = 0;
  double u_lid = 0;
  std::vector<int> nx, ny, pitch, plane, base, uref_off;
  std::vector<double> re, tau;
  size_t elems = 0, buf_bytes = 0;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  void *desc = nullptr;                 // CavityDesc<T>[n]
  int4 *tiles = nullptr;                // tiles of the chosen shape, active cavities
  int ntiles = 0, tiles_cap = 0;
  int4 *tiles1 = nullptr;               // 64 x 4 one-step tiles (shape 0)
  int ntiles1 = 0, tiles1_cap = 0;
  int4 *mtiles = nullptr;               // 64 x 4 monitor tiles of active cavities
  int nmtiles = 0, mtiles_cap = 0;
  int *fin = nullptr;                   // [3][n]: first, count, cavity
  int nfin = 0;
  double2 *uref = nullptr;
  double *partials = nullptr;           // partials_cap x 3
  long long partials_cap = 0;           // max(monitor tiles, 16 x 16 step tiles, kRedBlocks)
  double *mon_dev = nullptr;            // [n][3] chunk monitors
  double *aux_dev = nullptr;            // on-demand reductions
  double *mon_host = nullptr;           // pinned [n][3] + 4
  double *tmp = nullptr;
  size_t tmp_doubles = 0;
  std::vector<char> active;
  std::vector<int64_t> t, snap_t, mon_t;
  std::vector<char> mon_valid;
  std::vector<double> last_res, last_mass;
  int64_t t_global = 0;
  double threshold = 0.0;
  int variant = 12, use_graph = 1, graph_steps = 1000;   // 12: K = 5 on 32 x 32 tiles
  hipStream_t stream = nullptr, own_stream = nullptr, cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  bool tables_dirty = true;
  // probe time series, recorded at every monitor of an active cavity
  double *probe_xy = nullptr;                 // [n][probe_n][2]
  double *probe_ring = nullptr;               // [n][probe_cap][probe_n][3]
  unsigned long long *probe_count = nullptr;  // [n] records written
  int probe_n = 0;
  int64_t probe_cap = 0;
  std::vector<int64_t> probe_records, probe_last;   // host mirror: count, step of the latest
};

namespace {

// Tile shapes of the batch kernels.  kind 0: 64 x (by*ry) sites
// (k_step_batch); kind 1: (64 V) x by sites (k_step_batch_vec, V = 16 B /
// element); kind 2: tx x ty core tiles advanced k steps per launch in LDS
// (k_step_batch_tb; FP64 uses tx64 x ty64 where the FP32 region would not
// fit).  k divides 100 into an even number of launches, so every monitor
// and chunk boundary finds the state in buffer 0.
struct Shape {
  int kind, by, ry, k, tx, ty, tx64, ty64;
};
const Shape kShapes[] = {
    {0, 4, 1, 1, 0, 0, 0, 0},   {0, 4, 2, 1, 0, 0, 0, 0},   {0, 4, 4, 1, 0, 0, 0, 0},
    {0, 8, 1, 1, 0, 0, 0, 0},   {0, 2, 4, 1, 0, 0, 0, 0},   {0, 1, 8, 1, 0, 0, 0, 0},
    {0, 8, 2, 1, 0, 0, 0, 0},   {0, 16, 1, 1, 0, 0, 0, 0},  {1, 1, 1, 1, 0, 0, 0, 0},
    {1, 2, 1, 1, 0, 0, 0, 0},   {1, 4, 1, 1, 0, 0, 0, 0},   {1, 8, 1, 1, 0, 0, 0, 0},
    {2, 0, 0, 5, 32, 32, 32, 32}, {2, 0, 0, 5, 64, 16, 64, 16}, {2, 0, 0, 5, 16, 16, 16, 16},
    {2, 0, 0, 10, 32, 32, 32, 16}, {2, 0, 0, 2, 32, 32, 32, 32}, {2, 0, 0, 5, 64, 32, 64, 16}};
const int kNumShapes = 18;

int shape_steps(int v) { return kShapes[v].k; }

template <typename T, bool S, int BY, int RY>
hipError_t launch_b(const lbm_batch *b, const void *src, void *dst, hipStream_t st) {
  hipLaunchKernelGGL((k_step_batch<T, S, BY, RY>), dim3(b->ntiles), dim3(64, BY), 0, st,
                     (const T *)src, (T *)dst, (const CavityDesc<T> *)b->desc,
                     (const int4 *)b->tiles);
  return hipGetLastError();
}

template <typename T, bool S, int BY>
hipError_t launch_bv(const lbm_batch *b, const void *src, void *dst, hipStream_t st) {
  hipLaunchKernelGGL((k_step_batch_vec<T, S, BY>), dim3(b->ntiles), dim3(64, BY), 0, st,
                     (const T *)src, (T *)dst, (const CavityDesc<T> *)b->desc,
                     (const int4 *)b->tiles);
  return hipGetLastError();
}

// mon: 1 / 2 for the first / second launch of a chunk that carries the
// monitor of its start state (see k_step_batch_tb), 0 for a plain launch.
template <typename T, bool S, int K, int TX, int TY, int NT>
hipError_t launch_bt(const lbm_batch *b, const void *src, void *dst, hipStream_t st, int mon) {
  if (mon > 0 && b->ntiles > b->partials_cap) return hipErrorInvalidValue;
  const TbMonitor m{b->uref, b->partials, b->mon_dev};
  if (mon == 1)
    hipLaunchKernelGGL((k_step_batch_tb<T, S, K, TX, TY, NT, 1>), dim3(b->ntiles), dim3(NT), 0,
                       st, (const T *)src, (T *)dst, (const CavityDesc<T> *)b->desc,
                       (const int4 *)b->tiles, m);
  else if (mon == 2)
    hipLaunchKernelGGL((k_step_batch_tb<T, S, K, TX, TY, NT, 2>), dim3(b->ntiles), dim3(NT), 0,
                       st, (const T *)src, (T *)dst, (const CavityDesc<T> *)b->desc,
                       (const int4 *)b->tiles, m);
  else
    hipLaunchKernelGGL((k_step_batch_tb<T, S, K, TX, TY, NT, 0>), dim3(b->ntiles), dim3(NT), 0,
                       st, (const T *)src, (T *)dst, (const CavityDesc<T> *)b->desc,
                       (const int4 *)b->tiles, m);
  return hipGetLastError();
}

// mon applies to the multi-step shapes (12-17) only.
template <typename T, bool S>
hipError_t launch_b_variant(const lbm_batch *b, const void *src, void *dst, hipStream_t st,
                            int mon) {
  constexpr bool D = sizeof(T) == 8;
  switch (b->variant) {
    case 12: return launch_bt<T, S, 5, 32, 32, 1024>(b, src, dst, st, mon);
    case 13: return launch_bt<T, S, 5, 64, 16, 512>(b, src, dst, st, mon);
    case 14: return launch_bt<T, S, 5, 16, 16, 256>(b, src, dst, st, mon);
    case 15:
      if constexpr (D) return launch_bt<T, S, 10, 32, 16, 512>(b, src, dst, st, mon);
      else return launch_bt<T, S, 10, 32, 32, 512>(b, src, dst, st, mon);
    case 16: return launch_bt<T, S, 2, 32, 32, 512>(b, src, dst, st, mon);
    case 17:
      if constexpr (D) return launch_bt<T, S, 5, 64, 16, 1024>(b, src, dst, st, mon);
      else return launch_bt<T, S, 5, 64, 32, 1024>(b, src, dst, st, mon);
    case 8: return launch_bv<T, S, 1>(b, src, dst, st);
    case 9: return launch_bv<T, S, 2>(b, src, dst, st);
    case 10: return launch_bv<T, S, 4>(b, src, dst, st);
    case 11: return launch_bv<T, S, 8>(b, src, dst, st);
    case 0: return launch_b<T, S, 4, 1>(b, src, dst, st);
    case 1: return launch_b<T, S, 4, 2>(b, src, dst, st);
    case 2: return launch_b<T, S, 4, 4>(b, src, dst, st);
    case 3: return launch_b<T, S, 8, 1>(b, src, dst, st);
    case 4: return launch_b<T, S, 2, 4>(b, src, dst, st);
    case 5: return launch_b<T, S, 1, 8>(b, src, dst, st);
    case 6: return launch_b<T, S, 8, 2>(b, src, dst, st);
    default: return launch_b<T, S, 16, 1>(b, src, dst, st);
  }
}


// One launch of the chosen shape (shape_steps(variant) steps); mon (the
// multi-step shapes only): see launch_bt.
hipError_t batch_launch(const lbm_batch *b, int from, hipStream_t st, int mon = 0) {
  if (b->ntiles == 0) return hipSuccess;
  if (b->dtype == LBM_F64)
    return launch_b_variant<double, false>(b, b->buf[from], b->buf[1 - from], st, mon);
  return launch_b_variant<float, true>(b, b->buf[from], b->buf[1 - from], st, mon);
}

// One step with shape 0 (for steps off the 100-step grid).
hipError_t batch_step1(const lbm_batch *b, int from, hipStream_t st) {
  if (b->ntiles1 == 0) return hipSuccess;
  if (b->dtype == LBM_F64)
    hipLaunchKernelGGL((k_step_batch<double, false, 4, 1>), dim3(b->ntiles1), dim3(64, 4), 0, st,
                       (const double *)b->buf[from], (double *)b->buf[1 - from],
                       (const CavityDesc<double> *)b->desc, (const int4 *)b->tiles1);
  else
    hipLaunchKernelGGL((k_step_batch<float, true, 4, 1>), dim3(b->ntiles1), dim3(64, 4), 0, st,
                       (const float *)b->buf[from], (float *)b->buf[1 - from],
                       (const CavityDesc<float> *)b->desc, (const int4 *)b->tiles1);
  return hipGetLastError();
}

template <typename T, bool S>
hipError_t batch_monitor_t(const lbm_batch *b, int from, hipStream_t st) {
  hipLaunchKernelGGL((k_monitor_batch<T, S, true>), dim3(b->nmtiles), dim3(256), 0, st,
                     (const T *)b->buf[from], (const CavityDesc<T> *)b->desc,
                     (const int4 *)b->mtiles, b->uref, b->partials);
  hipLaunchKernelGGL(k_finalize_batch, dim3(b->nfin), dim3(kRedThreads), 0, st, b->partials,
                     b->fin, b->fin + b->n, b->fin + 2 * b->n, b->mon_dev);
  return hipGetLastError();
}

template <typename T, bool S>
hipError_t batch_probe_t(const lbm_batch *b, int from, hipStream_t st) {
  hipLaunchKernelGGL((k_probe_ring_batch<T, S>), dim3(b->nfin), dim3(256), 0, st,
                     (const T *)b->buf[from], (const CavityDesc<T> *)b->desc, b->fin + 2 * b->n,
                     b->probe_xy, b->probe_n, b->probe_ring, (long long)b->probe_cap,
                     b->probe_count);
  return hipGetLastError();
}

// The monitor pair of every active cavity, then its probe record.
hipError_t batch_monitor(const lbm_batch *b, int from, hipStream_t st) {
  if (b->nmtiles == 0) return hipSuccess;
  hipError_t e = b->dtype == LBM_F64 ? batch_monitor_t<double, false>(b, from, st)
                                     : batch_monitor_t<float, true>(b, from, st);
  if (e != hipSuccess || b->probe_n == 0 || b->nfin == 0) return e;
  return b->dtype == LBM_F64 ? batch_probe_t<double, false>(b, from, st)
                             : batch_probe_t<float, true>(b, from, st);
}

bool valid_k(const lbm_batch *b, int k) { return b && k >= 0 && k < b->n; }

// Buffer holding cavity k now: active cavities follow the global parity;
// inactive ones stopped at a chunk boundary, where the parity is 0.
int cbuf(const lbm_batch *b, int k) { return b->active[k] ? b->cur : 0; }

Geometry cav_geom(const lbm_batch *b, int k) {
  Geometry g;
  g.nx = b->nx[k];
  g.ny = b->ny[k];
  g.pitch = b->pitch[k];
  g.plane = b->plane[k];
  return g;
}

void drop_graph(lbm_batch *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
}

// Rebuild the step / monitor tile tables for the active cavities.
int rebuild_tables(lbm_batch *b) {
  const Shape sh = kShapes[b->variant];
  std::vector<int4> st, mt;
  std::vector<int> first(b->n, 0), count(b->n, 0), cav(b->n, 0);
  int nfin = 0;
  const bool d64 = b->dtype == LBM_F64;
  int tw, th;                      // tile width / height of the chosen shape
  if (sh.kind == 2) {
    tw = d64 ? sh.tx64 : sh.tx;
    th = d64 ? sh.ty64 : sh.ty;
  } else {
    tw = 64 * (sh.kind == 1 ? (d64 ? 2 : 4) : 1);
    th = sh.by * sh.ry;
  }
  std::vector<int4> s1;
  for (int c = 0; c < b->n; ++c) {
    if (!b->active[c]) continue;
    const int tx = (b->nx[c] + tw - 1) / tw;
    const int ty = (b->ny[c] + th - 1) / th;
    // .w: the cavity's tile count on its first tile (the in-chunk monitor
    // adds the cavity's partials there), 0 on the others
    for (int y = 0; y < ty; ++y)
      for (int x = 0; x < tx; ++x) st.push_back(make_int4(c, x, y, x == 0 && y == 0 ? tx * ty : 0));
    const int mx = (b->nx[c] + 63) / 64;
    const int my = (b->ny[c] + 3) / 4;
    first[nfin] = (int)mt.size();
    for (int y = 0; y < my; ++y)
      for (int x = 0; x < mx; ++x) {
        mt.push_back(make_int4(c, x, y, 0));
        s1.push_back(make_int4(c, x, y, 0));   // shape 0 uses the same 64 x 4 tiles
      }
    count[nfin] = (int)mt.size() - first[nfin];
    cav[nfin] = c;
    ++nfin;
  }
  HIPC(hipStreamSynchronize(b->stream));
  if ((int)st.size() > b->tiles_cap) {
    if (b->tiles) HIPC(hipFree(b->tiles));
    b->tiles = nullptr;
    HIPC(hipMalloc(&b->tiles, st.size() * sizeof(int4)));
    b->tiles_cap = (int)st.size();
  }
  if ((int)mt.size() > b->mtiles_cap) {
    if (b->mtiles) HIPC(hipFree(b->mtiles));
    b->mtiles = nullptr;
    HIPC(hipMalloc(&b->mtiles, mt.size() * sizeof(int4)));
    b->mtiles_cap = (int)mt.size();
  }
  if ((int)s1.size() > b->tiles1_cap) {
    if (b->tiles1) HIPC(hipFree(b->tiles1));
    b->tiles1 = nullptr;
    HIPC(hipMalloc(&b->tiles1, s1.size() * sizeof(int4)));
    b->tiles1_cap = (int)s1.size();
  }
  if (!s1.empty())
    HIPC(hipMemcpy(b->tiles1, s1.data(), s1.size() * sizeof(int4), hipMemcpyHostToDevice));
  b->ntiles1 = (int)s1.size();
  if (!st.empty())
    HIPC(hipMemcpy(b->tiles, st.data(), st.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!mt.empty())
    HIPC(hipMemcpy(b->mtiles, mt.data(), mt.size() * sizeof(int4), hipMemcpyHostToDevice));
  std::vector<int> packed(3 * b->n, 0);
  std::copy(first.begin(), first.end(), packed.begin());
  std::copy(count.begin(), count.end(), packed.begin() + b->n);
  std::copy(cav.begin(), cav.end(), packed.begin() + 2 * b->n);
  HIPC(hipMemcpy(b->fin, packed.data(), packed.size() * sizeof(int), hipMemcpyHostToDevice));
  b->ntiles = (int)st.size();
  b->nmtiles = (int)mt.size();
  b->nfin = nfin;
  b->tables_dirty = false;
  drop_graph(b);
  return LBM_OK;
}

// graph_steps steps from a monitored state at a multiple of 100, ending
// with every cavity's monitor of each later multiple of 100.  Multi-step
// shapes carry the monitor of a chunk's start state in the chunk's first
// two launches (k_step_batch_tb, MON = 1 and 2) from the second chunk on,
// and the state the graph ends in gets the separate pass, which the host
// reads.  Probe series are recorded by the separate pass, so with probes
// every chunk ends with it.
hipError_t issue_chunk(lbm_batch *b, hipStream_t st) {
  const int K = shape_steps(b->variant);
  const bool fused = kShapes[b->variant].kind == 2 && b->probe_n == 0;
  int cur = 0;
  for (int k = K; k <= b->graph_steps; k += K) {
    const int done = (k - K) % kChunk;   // steps of this chunk before the launch
    const int mon = (fused && k > kChunk) ? (done == 0 ? 1 : done == K ? 2 : 0) : 0;
    hipError_t e = batch_launch(b, cur, st, mon);
    if (e != hipSuccess) return e;
    cur = 1 - cur;
    if (k % kChunk == 0 && (!fused || k == b->graph_steps)) {
      e = batch_monitor(b, cur, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

int build_graph(lbm_batch *b) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = issue_chunk(b, b->cap_stream);
  hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return lbm_fail(LBM_EDEVICE, "batch graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return lbm_fail(LBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

void note_monitor(lbm_batch *b) {
  for (int c = 0; c < b->n; ++c) {
    if (!b->active[c]) continue;
    b->mon_valid[c] = (b->snap_t[c] == b->t[c] - kChunk);
    b->snap_t[c] = b->t[c];
    b->mon_t[c] = b->t[c];
    if (b->probe_n > 0) {      // k_probe_ring_batch recorded this cavity
      ++b->probe_records[c];
      b->probe_last[c] = b->t[c];
    }
  }
}

// Copy the chunk monitors to the host and update masses / residuals; drop
// converged cavities when a threshold is set.
int read_monitors(lbm_batch *b, bool *changed) {
  *changed = false;
  HIPC(hipMemcpyAsync(b->mon_host, b->mon_dev, 3 * b->n * sizeof(double),
                      hipMemcpyDeviceToHost, b->stream));
  HIPC(hipStreamSynchronize(b->stream));
  int bad = -1;
  for (int c = 0; c < b->n; ++c) {
    if (b->mon_t[c] < 0) continue;
    const double *m = b->mon_host + 3 * c;
    b->last_mass[c] = (double)b->nx[c] * b->ny[c] + m[0];
    b->last_res[c] = (b->mon_valid[c] && m[2] > 0.0) ? std::sqrt(m[1] / m[2]) : INFINITY;
    if ((!std::isfinite(b->last_mass[c]) || std::isnan(b->last_res[c])) && bad < 0) bad = c;
    if (b->active[c] && b->threshold > 0.0 && b->mon_valid[c] &&
        b->last_res[c] < b->threshold) {
      b->active[c] = 0;
      *changed = true;
    }
  }
  if (bad >= 0)
    return lbm_fail(LBM_EUNSTABLE, "non-finite monitor in cavity %d (%d x %d, tau %.6g) at step %lld",
                    bad, b->nx[bad], b->ny[bad], b->tau[bad], (long long)b->t[bad]);
  return LBM_OK;
}

template <typename T, bool S>
void launch_init_eq(lbm_batch *b, int k, const double *r, const double *u, const double *v,
                    double scale, double sx = 0.0, double sy = 0.0) {
  const Geometry g = cav_geom(b, k);
  const int tot = g.pitch * g.ny;
  hipLaunchKernelGGL((k_init_eq<T, S>), dim3((tot + 255) / 256), dim3(256), 0, b->stream,
                     (T *)b->buf[cbuf(b, k)] + b->base[k], g, r, u, v, scale, sx, sy);
}

template <typename T, bool S>
void launch_ref_monitor(lbm_batch *b, int k, bool update) {
  const Geometry g = cav_geom(b, k);
  const int n = g.nx * g.ny;
  const int blocks = std::min(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
  const T *src = (const T *)b->buf[cbuf(b, k)] + b->base[k];
  if (update)
    hipLaunchKernelGGL((k_monitor<T, S, true>), dim3(blocks), dim3(kRedThreads), 0, b->stream,
                       src, g, b->uref + b->uref_off[k], b->partials);
  else
    hipLaunchKernelGGL((k_monitor<T, S, false>), dim3(blocks), dim3(kRedThreads), 0,
                       b->stream, src, g, b->uref + b->uref_off[k], b->partials);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, b->stream, b->partials, blocks,
                     b->aux_dev);
}

int reset_cavity(lbm_batch *b, int k) {
  b->t[k] = 0;
  b->snap_t[k] = 0;
  b->mon_t[k] = -1;
  b->last_res[k] = INFINITY;
  if (b->dtype == LBM_F64) launch_ref_monitor<double, false>(b, k, true);
  else launch_ref_monitor<float, true>(b, k, true);
  HIPC(hipGetLastError());
  return LBM_OK;
}

int ensure_tmp(lbm_batch *b, size_t doubles) {
  if (b->tmp_doubles >= doubles) return LBM_OK;
  if (b->tmp) HIPC(hipFree(b->tmp));
  b->tmp = nullptr;
  b->tmp_doubles = 0;
  HIPC(hipMalloc(&b->tmp, doubles * sizeof(double)));
  b->tmp_doubles = doubles;
  return LBM_OK;
}

template <typename T>
int upload_desc(lbm_batch *b) {
  std::vector<CavityDesc<T>> d(b->n);
  for (int c = 0; c < b->n; ++c) {
    d[c].base = b->base[c];
    d[c].nx = b->nx[c];
    d[c].ny = b->ny[c];
    d[c].pitch = b->pitch[c];
    d[c].plane = b->plane[c];
    d[c].uref_off = b->uref_off[c];
    d[c].omega = (T)(1.0 / b->tau[c]);
    d[c].u6 = (T)(b->u_lid / 6.0);
  }
  HIPC(hipMalloc(&b->desc, b->n * sizeof(CavityDesc<T>)));
  HIPC(hipMemcpy(b->desc, d.data(), b->n * sizeof(CavityDesc<T>), hipMemcpyHostToDevice));
  return LBM_OK;
}



}  // namespace

extern "C" {

int lbm_batch_destroy(lbm_batch_t b) {
  if (!b) return LBM_OK;
  drop_graph(b);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  void *ptrs[] = {b->buf[0], b->buf[1], b->desc, b->tiles, b->tiles1, b->mtiles, b->fin,
                  b->uref, b->partials, b->mon_dev, b->aux_dev, b->tmp, b->probe_xy,
                  b->probe_ring, b->probe_count};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (b->mon_host) (void)hipHostFree(b->mon_host);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
  return LBM_OK;
}

int lbm_batch_create(int n, const int *nx, const int *ny, const double *re, double u_lid,
                     int dtype, lbm_batch_t *out) {
  if (!out) return lbm_fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096 || !nx || !ny || !re)
    return lbm_fail(LBM_EINVAL, "n = %d outside [1, 4096] or NULL arrays", n);
  if (dtype != LBM_F64 && dtype != LBM_F32_SHIFTED)
    return lbm_fail(LBM_EINVAL, "unknown dtype %d", dtype);
  if (!std::isfinite(u_lid) || std::fabs(u_lid) >= 1.0 / std::sqrt(3.0))
    return lbm_fail(LBM_EINVAL, "|u_lid| = %g must be below 1/sqrt(3)", u_lid);
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return lbm_fail(LBM_ENOMEM, "host allocation");
  auto bail = [&](int code) {
    lbm_batch_destroy(b);
    return code;
  };
  b->n = n;
  b->dtype = dtype;
  b->u_lid = u_lid;
  long long elems = 0, sites = 0, mt_total = 0, t16_total = 0;
  for (int c = 0; c < n; ++c) {
    if (nx[c] < 2 || ny[c] < 2 || nx[c] > 65536 || ny[c] > 65536)
      return bail(lbm_fail(LBM_EINVAL, "cavity %d: lattice %d x %d outside [2, 65536]", c,
                           nx[c], ny[c]));
    if (!(re[c] > 0.0) || !std::isfinite(re[c]))
      return bail(lbm_fail(LBM_EINVAL, "cavity %d: re = %g", c, re[c]));
    const double tau = 3.0 * u_lid * nx[c] / re[c] + 0.5;   // Eq. 5, nu = U L / Re
    if (!(tau > 0.5)) return bail(lbm_fail(LBM_EINVAL, "cavity %d: tau = %g <= 1/2", c, tau));
    const int p = (nx[c] + 63) / 64 * 64;
    b->nx.push_back(nx[c]);
    b->ny.push_back(ny[c]);
    b->pitch.push_back(p);
    b->plane.push_back(p * ny[c]);
    b->base.push_back((int)std::min<long long>(elems, INT32_MAX));
    b->uref_off.push_back((int)std::min<long long>(sites, INT32_MAX));
    b->re.push_back(re[c]);
    b->tau.push_back(tau);
    elems += 9LL * p * ny[c];
    sites += (long long)nx[c] * ny[c];
    mt_total += (long long)((nx[c] + 63) / 64) * ((ny[c] + 3) / 4);
    t16_total += (long long)((nx[c] + 15) / 16) * ((ny[c] + 15) / 16);
  }
  if (elems >= (1LL << 31) || sites >= (1LL << 31))
    return bail(lbm_fail(LBM_EINVAL, "batch too large for 32-bit element offsets"));
  b->elems = (size_t)elems;
  const size_t esz = dtype == LBM_F64 ? 8 : 4;
  b->buf_bytes = b->elems * esz;
  b->active.assign(n, 1);
  b->t.assign(n, 0);
  b->snap_t.assign(n, 0);
  b->mon_t.assign(n, -1);
  b->mon_valid.assign(n, 0);
  b->last_res.assign(n, INFINITY);
  b->last_mass.assign(n, NAN);
  hipError_t e;
#define TRY(call)                                                                     \
  do {                                                                                \
    e = (call);                                                                       \
    if (e != hipSuccess)                                                              \
      return bail(lbm_fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,       \
                           "%s failed: %s", #call, hipGetErrorString(e)));            \
  } while (0)
  TRY(hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking));
  b->stream = b->own_stream;
  TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  for (int c = 0; c < 2; ++c) {
    TRY(hipMalloc(&b->buf[c], b->buf_bytes));
    TRY(hipMemsetAsync(b->buf[c], 0, b->buf_bytes, b->stream));
  }
  TRY(hipMalloc(&b->uref, sizeof(double2) * (size_t)sites));
  // the step tiles of every shape are at least 16 x 16 sites
  b->partials_cap = std::max<long long>(std::max(mt_total, t16_total), kRedBlocks);
  TRY(hipMalloc(&b->partials, sizeof(double) * kNumSums * (size_t)b->partials_cap));
  TRY(hipMalloc(&b->mon_dev, sizeof(double) * kNumSums * n));
  TRY(hipMemsetAsync(b->mon_dev, 0, sizeof(double) * kNumSums * n, b->stream));
  TRY(hipMalloc(&b->aux_dev, sizeof(double) * 4));
  TRY(hipMalloc(&b->fin, sizeof(int) * 3 * n));
  TRY(hipHostMalloc(&b->mon_host, sizeof(double) * (kNumSums * n + 4), hipHostMallocDefault));
#undef TRY
  int rc = dtype == LBM_F64 ? upload_desc<double>(b) : upload_desc<float>(b);
  if (rc) return bail(rc);
  for (int c = 0; c < n; ++c) {
    if (dtype == LBM_F64) launch_init_eq<double, false>(b, c, nullptr, nullptr, nullptr, 1.0);
    else launch_init_eq<float, true>(b, c, nullptr, nullptr, nullptr, 1.0);
    rc = reset_cavity(b, c);
    if (rc) return bail(rc);
  }
  rc = rebuild_tables(b);
  if (rc) return bail(rc);
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess)
    return bail(lbm_fail(LBM_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e)));
  *out = b;
  return LBM_OK;
}

int lbm_batch_set_stream(lbm_batch_t b, void *hip_stream) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  HIPC(hipStreamSynchronize(b->stream));
  b->stream = hip_stream ? (hipStream_t)hip_stream : b->own_stream;
  return LBM_OK;
}

int lbm_batch_set_option(lbm_batch_t b, int option, int64_t value) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  switch (option) {
    case LBM_OPT_USE_GRAPH:
      b->use_graph = value ? 1 : 0;
      return LBM_OK;
    case LBM_OPT_STEP_VARIANT:
      if (value < 0 || value >= kNumShapes)
        return lbm_fail(LBM_EINVAL, "variant %lld outside [0, %d)", (long long)value, kNumShapes);
      if (b->variant != (int)value) {
        b->variant = (int)value;
        b->tables_dirty = true;
        drop_graph(b);
      }
      return LBM_OK;
    case LBM_OPT_GRAPH_STEPS:
      if (value < kChunk || value > 100000 || value % kChunk != 0)
        return lbm_fail(LBM_EINVAL, "graph steps %lld must be a multiple of 100 in [100, 1e5]",
                        (long long)value);
      if (b->graph_steps != (int)value) drop_graph(b);
      b->graph_steps = (int)value;
      return LBM_OK;
    default:
      return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

int lbm_batch_get_option(lbm_batch_t b, int option, int64_t *value) {
  if (!b || !value) return lbm_fail(LBM_EINVAL, "NULL argument");
  switch (option) {
    case LBM_OPT_USE_GRAPH: *value = b->use_graph; return LBM_OK;
    case LBM_OPT_STEP_VARIANT: *value = b->variant; return LBM_OK;
    case LBM_OPT_NUM_VARIANTS: *value = kNumShapes; return LBM_OK;
    case LBM_OPT_GRAPH_STEPS: *value = b->graph_steps; return LBM_OK;
    case LBM_OPT_STEPS_PER_LAUNCH: *value = shape_steps(b->variant); return LBM_OK;
    default: return lbm_fail(LBM_EINVAL, "unknown option %d", option);
  }
}

int lbm_batch_set_threshold(lbm_batch_t b, double residual) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  if (!(residual >= 0.0) || !std::isfinite(residual))
    return lbm_fail(LBM_EINVAL, "threshold %g must be finite and >= 0", residual);
  b->threshold = residual;
  return LBM_OK;
}

int lbm_batch_set_active(lbm_batch_t b, int k, int active) {
  if (!valid_k(b, k)) return lbm_fail(LBM_EINVAL, "cavity index %d out of range", k);
  if (b->t_global % kChunk != 0)
    return lbm_fail(LBM_EINVAL, "activity can change only at multiples of 100 steps (now %lld)",
                    (long long)b->t_global);
  if ((b->active[k] != 0) != (active != 0)) {
    b->active[k] = active ? 1 : 0;
    b->tables_dirty = true;
  }
  return LBM_OK;
}

static int batch_step_impl(lbm_batch_t b, int64_t n);

int lbm_batch_step(lbm_batch_t b, int64_t n) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  if (n < 0) return lbm_fail(LBM_EINVAL, "n = %lld < 0", (long long)n);
  int active0 = 0;
  long long sites = 0;
  for (int c = 0; c < b->n; ++c)
    if (b->active[c]) {
      ++active0;
      sites += (long long)b->nx[c] * b->ny[c];
    }
  const double t0 = lbm_wall_seconds();
  const int rc = batch_step_impl(b, n);
  const double sec = lbm_wall_seconds() - t0;
  int active = 0;
  double worst = 0.0;
  for (int c = 0; c < b->n; ++c) {
    active += b->active[c];
    if (b->active[c] && b->mon_t[c] >= 0) worst = std::max(worst, b->last_res[c]);
  }
  char wbuf[32];
  lbm_log_line("{\"kind\": \"batch\", \"handle\": \"%p\", \"cavities\": %d, "
               "\"active_before\": %d, \"active\": %d, \"steps\": %lld, \"step\": %lld, "
               "\"max_active_residual\": %s, \"seconds\": %.6f, "
               "\"MLUPS_upper\": %.1f, \"rc\": %d}",
               (void *)b, b->n, active0, active, (long long)n, (long long)b->t_global,
               lbm_json_num(worst, wbuf), sec, sec > 0 ? (double)sites * n / sec / 1e6 : 0.0, rc);
  return rc;
}

static int batch_step_impl(lbm_batch_t b, int64_t n) {
  bool monitored = false;
  while (n > 0) {
    if (b->tables_dirty) {
      int rc = rebuild_tables(b);
      if (rc) return rc;
    }
    if (b->ntiles == 0) break;       // every cavity inactive
    const bool aligned = b->t_global % kChunk == 0;
    if (aligned && n >= b->graph_steps) {
      if (b->use_graph) {
        if (!b->graph) {
          int rc = build_graph(b);
          if (rc) return rc;
        }
        HIPC(hipGraphLaunch(b->graph, b->stream));
      } else {
        hipError_t e = issue_chunk(b, b->stream);
        if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "batch chunk: %s", hipGetErrorString(e));
      }
      for (int k = 0; k < b->graph_steps / kChunk; ++k) {
        for (int c = 0; c < b->n; ++c)
          if (b->active[c]) b->t[c] += kChunk;
        b->t_global += kChunk;
        note_monitor(b);
      }
      n -= b->graph_steps;
      monitored = true;
    } else {
      hipError_t e = batch_step1(b, b->cur, b->stream);
      if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "batch step: %s", hipGetErrorString(e));
      b->cur = 1 - b->cur;
      for (int c = 0; c < b->n; ++c)
        if (b->active[c]) b->t[c] += 1;
      b->t_global += 1;
      n -= 1;
      if (b->t_global % kChunk == 0) {
        e = batch_monitor(b, b->cur, b->stream);
        if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "monitor: %s", hipGetErrorString(e));
        note_monitor(b);
        monitored = true;
      }
    }
    if (monitored && b->threshold > 0.0 && b->t_global % kChunk == 0) {
      bool changed = false;
      int rc = read_monitors(b, &changed);
      monitored = false;
      if (rc) return rc;
      if (changed) b->tables_dirty = true;
    }
  }
  if (monitored) {
    bool changed = false;
    int rc = read_monitors(b, &changed);
    if (rc) return rc;
    if (changed) b->tables_dirty = true;
  }
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_status(lbm_batch_t b, int k, int64_t *steps_done, double *residual,
                     int64_t *residual_step, int *active) {
  if (!valid_k(b, k)) return lbm_fail(LBM_EINVAL, "cavity index %d out of range", k);
  if (steps_done) *steps_done = b->t[k];
  if (residual) *residual = b->mon_t[k] >= 0 ? b->last_res[k] : INFINITY;
  if (residual_step) *residual_step = b->mon_t[k];
  if (active) *active = b->active[k];
  return LBM_OK;
}

int lbm_batch_residuals(lbm_batch_t b, double *residuals) {
  if (!b || !residuals) return lbm_fail(LBM_EINVAL, "NULL argument");
  for (int k = 0; k < b->n; ++k)
    residuals[k] = b->mon_t[k] >= 0 ? b->last_res[k] : INFINITY;
  return LBM_OK;
}

int lbm_batch_mass(lbm_batch_t b, int k, double *mass) {
  if (!valid_k(b, k) || !mass) return lbm_fail(LBM_EINVAL, "bad cavity index or NULL");
  if (b->dtype == LBM_F64) launch_ref_monitor<double, false>(b, k, false);
  else launch_ref_monitor<float, true>(b, k, false);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(b->mon_host + kNumSums * b->n, b->aux_dev, sizeof(double),
                      hipMemcpyDeviceToHost, b->stream));
  HIPC(hipStreamSynchronize(b->stream));
  *mass = (double)b->nx[k] * b->ny[k] + b->mon_host[kNumSums * b->n];
  return LBM_OK;
}

int lbm_batch_moments(lbm_batch_t b, int k, double *rho, double *ux, double *uy) {
  if (!valid_k(b, k)) return lbm_fail(LBM_EINVAL, "cavity index %d out of range", k);
  const Geometry g = cav_geom(b, k);
  const size_t n = (size_t)g.nx * g.ny;
  int rc = ensure_tmp(b, 3 * n);
  if (rc) return rc;
  double *d[3] = {rho ? b->tmp : nullptr, ux ? b->tmp + n : nullptr, uy ? b->tmp + 2 * n : nullptr};
  if (b->dtype == LBM_F64)
    hipLaunchKernelGGL((k_moments<double, false>), dim3((n + 255) / 256), dim3(256), 0,
                       b->stream, (const double *)b->buf[cbuf(b, k)] + b->base[k], g, d[0], d[1], d[2]);
  else
    hipLaunchKernelGGL((k_moments<float, true>), dim3((n + 255) / 256), dim3(256), 0, b->stream,
                       (const float *)b->buf[cbuf(b, k)] + b->base[k], g, d[0], d[1], d[2]);
  HIPC(hipGetLastError());
  double *outs[3] = {rho, ux, uy};
  for (int j = 0; j < 3; ++j)
    if (outs[j])
      HIPC(hipMemcpyAsync(outs[j], d[j], n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_get_populations(lbm_batch_t b, int k, double *f) {
  if (!valid_k(b, k) || !f) return lbm_fail(LBM_EINVAL, "bad cavity index or NULL");
  const Geometry g = cav_geom(b, k);
  const size_t n = (size_t)g.nx * g.ny;
  int rc = ensure_tmp(b, 9 * n);
  if (rc) return rc;
  if (b->dtype == LBM_F64)
    hipLaunchKernelGGL((k_get_pop<double, false>), dim3((n + 255) / 256), dim3(256), 0,
                       b->stream, (const double *)b->buf[cbuf(b, k)] + b->base[k], g, b->tmp);
  else
    hipLaunchKernelGGL((k_get_pop<float, true>), dim3((n + 255) / 256), dim3(256), 0,
                       b->stream, (const float *)b->buf[cbuf(b, k)] + b->base[k], g, b->tmp);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(f, b->tmp, 9 * n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_set_populations(lbm_batch_t b, int k, const double *f) {
  if (!valid_k(b, k) || !f) return lbm_fail(LBM_EINVAL, "bad cavity index or NULL");
  const Geometry g = cav_geom(b, k);
  const size_t n = (size_t)g.nx * g.ny;
  int rc = ensure_tmp(b, 9 * n);
  if (rc) return rc;
  HIPC(hipMemcpyAsync(b->tmp, f, 9 * n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  const double omega = 1.0 / b->tau[k];
  if (b->dtype == LBM_F64)
    hipLaunchKernelGGL((k_set_pop<double, false>), dim3((n + 255) / 256), dim3(256), 0,
                       b->stream, (double *)b->buf[cbuf(b, k)] + b->base[k], g, b->tmp, omega);
  else
    hipLaunchKernelGGL((k_set_pop<float, true>), dim3((n + 255) / 256), dim3(256), 0, b->stream,
                       (float *)b->buf[cbuf(b, k)] + b->base[k], g, b->tmp, omega);
  HIPC(hipGetLastError());
  rc = reset_cavity(b, k);
  if (rc) return rc;
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

static int batch_init_impl(lbm_batch_t b, int k, const double *rho, const double *ux,
                           const double *uy, int flags, bool on_device) {
  if (!valid_k(b, k)) return lbm_fail(LBM_EINVAL, "cavity index %d out of range", k);
  const Geometry g = cav_geom(b, k);
  const size_t n = (size_t)g.nx * g.ny;
  const double *d[3] = {rho, ux, uy};
  if (!on_device) {
    int rc = ensure_tmp(b, 3 * n);
    if (rc) return rc;
    const double *src[3] = {rho, ux, uy};
    for (int j = 0; j < 3; ++j) {
      d[j] = nullptr;
      if (src[j]) {
        d[j] = b->tmp + j * n;
        HIPC(hipMemcpyAsync(b->tmp + j * n, src[j], n * sizeof(double), hipMemcpyHostToDevice,
                            b->stream));
      }
    }
  }
  double scale = 1.0, sx = 0.0, sy = 0.0;
  const bool renorm = (flags & LBM_INIT_RENORMALISE_MASS) && rho;
  const bool destag = (flags & LBM_INIT_ZERO_STAGGERED) && (ux || uy);
  if (renorm || destag) {
    const int blocks = std::min(kRedBlocks, (int)((n + kRedThreads - 1) / kRedThreads));
    hipLaunchKernelGGL(k_init_sums, dim3(blocks), dim3(kRedThreads), 0, b->stream, d[0], d[1],
                       d[2], g.nx, (long long)n, b->partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, b->stream, b->partials, blocks,
                       b->aux_dev);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(b->mon_host + kNumSums * b->n, b->aux_dev, 3 * sizeof(double),
                        hipMemcpyDeviceToHost, b->stream));
    HIPC(hipStreamSynchronize(b->stream));
    const double *m = b->mon_host + kNumSums * b->n;
    if (renorm) {
      if (!(m[0] > 0.0) || !std::isfinite(m[0]))
        return lbm_fail(LBM_EINVAL, "sum of rho = %g cannot be renormalised", m[0]);
      scale = (double)n / m[0];
    }
    if (destag) {
      sx = scale * m[1] / (double)n;
      sy = scale * m[2] / (double)n;
    }
  }
  if (b->dtype == LBM_F64) launch_init_eq<double, false>(b, k, d[0], d[1], d[2], scale, sx, sy);
  else launch_init_eq<float, true>(b, k, d[0], d[1], d[2], scale, sx, sy);
  HIPC(hipGetLastError());
  int rc = reset_cavity(b, k);
  if (rc) return rc;
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_init_fields(lbm_batch_t b, int k, const double *rho, const double *ux,
                          const double *uy, int flags) {
  return batch_init_impl(b, k, rho, ux, uy, flags, false);
}

int lbm_batch_init_fields_device(lbm_batch_t b, int k, const double *rho, const double *ux,
                                 const double *uy, int flags) {
  return batch_init_impl(b, k, rho, ux, uy, flags, true);
}

int lbm_batch_canvas(lbm_batch_t b, int k, float *target_dev, float *mask_dev) {
  if (!valid_k(b, k) || !target_dev || !mask_dev)
    return lbm_fail(LBM_EINVAL, "bad cavity index or NULL");
  const int rows = (int)std::rint(128.0 * b->ny[k] / b->nx[k]);
  if (rows < 1 || rows > 256)
    return lbm_fail(LBM_EINVAL, "cavity %d: aspect ratio %g outside the canvas", k,
                    (double)b->ny[k] / b->nx[k]);
  const Geometry g = cav_geom(b, k);
  if (b->dtype == LBM_F64)
    hipLaunchKernelGGL((k_canvas<double, false>), dim3(128), dim3(256), 0, b->stream,
                       (const double *)b->buf[cbuf(b, k)] + b->base[k], g, b->u_lid, rows,
                       target_dev, mask_dev);
  else
    hipLaunchKernelGGL((k_canvas<float, true>), dim3(128), dim3(256), 0, b->stream,
                       (const float *)b->buf[cbuf(b, k)] + b->base[k], g, b->u_lid, rows,
                       target_dev, mask_dev);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_cavity(lbm_batch_t b, int k, int *nx, int *ny, double *re, double *u_lid) {
  if (!valid_k(b, k)) return lbm_fail(LBM_EINVAL, "cavity index %d out of range", k);
  if (nx) *nx = b->nx[k];
  if (ny) *ny = b->ny[k];
  if (re) *re = b->re[k];
  if (u_lid) *u_lid = b->u_lid;
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch_t b, int chunks, int use_cache, int *best_variant,
                       double *ms_per_step) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  if (chunks < 1 || chunks > 1000) return lbm_fail(LBM_EINVAL, "chunks = %d outside [1, 1000]", chunks);
  if (b->t_global % kChunk != 0)
    return lbm_fail(LBM_EINVAL, "autotune only at a multiple of 100 steps");
  std::string key = tune_key("batch", b->dtype, b->n, (long long)b->elems);
  int cached = use_cache ? tune_cache_lookup(key) : -1;
  if (cached >= 0 && cached < kNumShapes) {
    int rc = lbm_batch_set_option(b, LBM_OPT_STEP_VARIANT, cached);
    if (best_variant) *best_variant = cached;
    if (ms_per_step) *ms_per_step = NAN;
    return rc;
  }
  // save the state (buffer 0 holds every cavity at a chunk boundary)
  void *save_f = nullptr;
  double2 *save_u = nullptr;
  long long sites = 0;
  for (int c = 0; c < b->n; ++c) sites += (long long)b->nx[c] * b->ny[c];
  HIPC(hipStreamSynchronize(b->stream));
  HIPC(hipMalloc(&save_f, b->buf_bytes));
  hipError_t e = hipMalloc(&save_u, sizeof(double2) * sites);
  if (e != hipSuccess) {
    (void)hipFree(save_f);
    return lbm_fail(LBM_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  }
  auto restore = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(b->buf[0], save_f, b->buf_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(b->uref, save_u, sizeof(double2) * sites, hipMemcpyDeviceToDevice, b->stream);
    return r;
  };
  e = hipMemcpyAsync(save_f, b->buf[0], b->buf_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(save_u, b->uref, sizeof(double2) * sites, hipMemcpyDeviceToDevice, b->stream);
  const auto t_save = b->t, snap_save = b->snap_t, mon_t_save = b->mon_t;
  const auto valid_save = b->mon_valid;
  const auto res_save = b->last_res, mass_save = b->last_mass;
  const int64_t tg_save = b->t_global;
  const double thr_save = b->threshold;
  const int var_save = b->variant;
  b->threshold = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  double best_ms = INFINITY;
  int best = var_save;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int v = 0; v < kNumShapes && e == hipSuccess && rc == LBM_OK; ++v) {
    rc = lbm_batch_set_option(b, LBM_OPT_STEP_VARIANT, v);
    if (rc == LBM_OK) rc = lbm_batch_step(b, b->graph_steps);          // warm-up, capture
    if (rc != LBM_OK) break;
    e = hipEventRecord(e0, b->stream);
    for (int k = 0; k < chunks && rc == LBM_OK; ++k) rc = lbm_batch_step(b, b->graph_steps);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double per_step = ms / ((double)chunks * b->graph_steps);
    if (rc == LBM_OK && e == hipSuccess && per_step < best_ms) {
      best_ms = per_step;
      best = v;
    }
    if (e == hipSuccess) e = restore();
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e == hipSuccess) e = restore();
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(save_f);
  (void)hipFree(save_u);
  b->t = t_save;
  b->snap_t = snap_save;
  b->mon_t = mon_t_save;
  b->mon_valid = valid_save;
  b->last_res = res_save;
  b->last_mass = mass_save;
  b->t_global = tg_save;
  b->cur = 0;
  b->threshold = thr_save;
  if (rc != LBM_OK) return rc;
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "autotune: %s", hipGetErrorString(e));
  rc = lbm_batch_set_option(b, LBM_OPT_STEP_VARIANT, best);
  if (rc) return rc;
  tune_cache_store(key, best);
  if (best_variant) *best_variant = best;
  if (ms_per_step) *ms_per_step = best_ms;
  return LBM_OK;
}

int lbm_batch_info(lbm_batch_t b, int *n, int64_t *total_sites, int64_t *steps_done,
                   size_t *device_bytes) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  long long sites = 0;
  for (int c = 0; c < b->n; ++c) sites += (long long)b->nx[c] * b->ny[c];
  if (n) *n = b->n;
  if (total_sites) *total_sites = sites;
  if (steps_done) *steps_done = b->t_global;
  if (device_bytes) *device_bytes = 2 * b->buf_bytes + sites * sizeof(double2);
  return LBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ probes
int lbm_batch_probe_config(lbm_batch_t b, int npts, const double *xy, int64_t capacity) {
  if (!b) return lbm_fail(LBM_EINVAL, "batch is NULL");
  if (npts < 0 || npts > 4096) return lbm_fail(LBM_EINVAL, "npts = %d outside [0, 4096]", npts);
  if (npts > 0 && (!xy || capacity < 1))
    return lbm_fail(LBM_EINVAL, "npts = %d needs points and capacity >= 1", npts);
  const double bytes = (double)b->n * (double)capacity * npts * 3 * sizeof(double);
  if (npts > 0 && bytes > 64.0 * (1ull << 30))
    return lbm_fail(LBM_EINVAL, "probe rings of %.3g GB exceed 64 GB", bytes / 1e9);
  HIPC(hipStreamSynchronize(b->stream));
  drop_graph(b);
  for (void **p : {(void **)&b->probe_xy, (void **)&b->probe_ring, (void **)&b->probe_count}) {
    if (*p) HIPC(hipFree(*p));
    *p = nullptr;
  }
  b->probe_n = 0;
  b->probe_cap = 0;
  b->probe_records.assign(b->n, 0);
  b->probe_last.assign(b->n, -1);
  if (npts == 0) return LBM_OK;
  const size_t nxy = (size_t)b->n * npts * 2;
  HIPC(hipMalloc(&b->probe_xy, nxy * sizeof(double)));
  HIPC(hipMalloc(&b->probe_ring, (size_t)b->n * capacity * npts * 3 * sizeof(double)));
  HIPC(hipMalloc(&b->probe_count, (size_t)b->n * sizeof(unsigned long long)));
  HIPC(hipMemcpy(b->probe_xy, xy, nxy * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemset(b->probe_count, 0, (size_t)b->n * sizeof(unsigned long long)));
  b->probe_n = npts;
  b->probe_cap = capacity;
  return LBM_OK;
}

int lbm_batch_probe_read(lbm_batch_t b, int k, double *buf, int64_t max_records,
                         int64_t *n_records, int64_t *first_step) {
  if (!valid_k(b, k) || !n_records) return lbm_fail(LBM_EINVAL, "bad cavity index or NULL");
  *n_records = 0;
  if (first_step) *first_step = -1;
  if (b->probe_n == 0) return LBM_OK;
  if (max_records > 0 && !buf) return lbm_fail(LBM_EINVAL, "buf is NULL");
  HIPC(hipStreamSynchronize(b->stream));
  const int64_t count = b->probe_records[k];
  const int64_t take = std::min<int64_t>(std::min<int64_t>(count, b->probe_cap), max_records);
  const int rec = 3 * b->probe_n;
  for (int64_t i = 0; i < take; ++i) {
    const int64_t idx = count - take + i;
    const int64_t slot = idx % b->probe_cap;
    HIPC(hipMemcpy(buf + i * rec, b->probe_ring + ((int64_t)k * b->probe_cap + slot) * rec,
                   rec * sizeof(double), hipMemcpyDeviceToHost));
  }
  *n_records = take;
  if (first_step && take > 0) *first_step = b->probe_last[k] - (int64_t)kChunk * (take - 1);
  return LBM_OK;
}

int lbm_batch_probe_classify(lbm_batch_t b, int component, int64_t window, double steady_tol,
                             double periodic_tol, int min_lag, int max_lag,
                             lbm_flow_state_t *out) {
  if (!b || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (b->probe_n == 0) return lbm_fail(LBM_EINVAL, "no probes configured");
  if (component < 0 || component > 2)
    return lbm_fail(LBM_EINVAL, "component %d outside {0, 1, 2}", component);
  if (!(steady_tol >= 0.0) || !(periodic_tol >= 0.0))
    return lbm_fail(LBM_EINVAL, "tolerances must be >= 0");
  int rc = check_lags(window, min_lag, max_lag);
  if (rc) return rc;
  if (window > b->probe_cap)
    return lbm_fail(LBM_EINVAL, "window %lld exceeds the ring capacity %lld", (long long)window,
                    (long long)b->probe_cap);
  HIPC(hipStreamSynchronize(b->stream));
  std::vector<SeriesDesc> d;
  std::vector<int> slot_of;
  const int rec = 3 * b->probe_n;
  for (int c = 0; c < b->n; ++c)
    for (int p = 0; p < b->probe_n; ++p) {
      lbm_flow_state_t &o = out[(size_t)c * b->probe_n + p];
      std::memset(&o, 0, sizeof o);
      o.state = LBM_FLOW_TOO_SHORT;
      if (b->probe_records[c] < window) continue;
      const long long start = (long long)((b->probe_records[c] - window) % b->probe_cap);
      d.push_back(SeriesDesc{b->probe_ring + (size_t)c * b->probe_cap * rec + 3 * p + component,
                             (long long)b->probe_cap, start, (long long)window, (long long)rec});
      slot_of.push_back(c * b->probe_n + p);
    }
  if (d.empty()) return LBM_OK;
  std::vector<lbm_flow_state_t> res(d.size());
  rc = classify_series_descs(d.data(), (int)d.size(), window, steady_tol, periodic_tol, min_lag,
                             max_lag, b->stream, res.data());
  if (rc) return rc;
  for (size_t i = 0; i < d.size(); ++i) out[slot_of[i]] = res[i];
  return LBM_OK;
}
