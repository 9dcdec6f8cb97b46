// lbm_internal.h -- the handle behind lbm_t (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/lbm.h"

// Record a message for lbm_last_error() and return `code`.
int lbm_fail(int code, const char *fmt, ...);

#define HIPC(call)                                                          \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return lbm_fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, \
                      "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

// Monitor cadence: Eq. 6 compares the velocity fields of steps t and t-100.
constexpr int kChunk = 100;

// Tile-shape autotuner cache: a text file named by $LBM_TUNE_CACHE with
// lines "<key> <variant>"; the key names the device architecture, the kind
// of handle, the storage type and the lattice size.
std::string tune_key(const char *kind, int dtype, long long a, long long b);
int tune_cache_lookup(const std::string &key);      // -1 if absent
void tune_cache_store(const std::string &key, int variant);

namespace lbm {
struct SeriesDesc;
}
// Classify nseries series described on the host (d2q9_series.hpp), longest
// n_max samples, on stream st; allocates its own device scratch.
int classify_series_descs(const lbm::SeriesDesc *descs_host, int nseries, long long n_max,
                          double steady_tol, double periodic_tol, int min_lag, int max_lag,
                          hipStream_t st, lbm_flow_state_t *out_host);

// Append one line (printf format, no newline) to the JSON-lines run log
// named by $LBM_LOG; a no-op when it is unset.
void lbm_log_line(const char *fmt, ...);
// A double as JSON text: "%.17g", or "null" when it is not finite (JSON has
// no inf or nan).  buf needs 32 chars; returns buf.
const char *lbm_json_num(double v, char *buf);
// Monotonic wall clock in seconds.
double lbm_wall_seconds();

// Validate a series length and lag range (LBM_EINVAL with a message).
int check_lags(long long n, int min_lag, int max_lag);

struct lbm_cavity {
  // lattice and parameters
  int nx = 0, ny = 0, pitch = 0, plane = 0, dtype = 0;
  int wall = LBM_WALL_BOUNCE_BACK;
  double re = 0, u_lid = 0, tau = 0, omega = 0;
  int device = 0;
  // population buffers (A/B); buf[cur] holds the post-collision state
  void *buf[2] = {nullptr, nullptr};
  size_t buf_bytes = 0;
  int cur = 0;
  // Eq. 6 reference velocity field (dense [ny][nx] of (ux, uy)) and FP64
  // reduction scratch
  double2 *uref = nullptr;
  double *partials = nullptr;
  int partial_slots = 0;        // triples in partials
  double *mon_dev = nullptr;    // chunk monitor sums: sum(rho-1), num, den
  double *aux_dev = nullptr;    // on-demand reductions
  double *mon_host = nullptr;   // pinned
  double *tmp = nullptr;        // FP64 transfer scratch
  size_t tmp_doubles = 0;
  // probe time series
  double *probe_xy = nullptr;
  double *probe_ring = nullptr;
  unsigned long long *probe_count = nullptr;
  int probe_n = 0, probe_every = 0;
  int64_t probe_cap = 0, probe_t0 = 0;
  // execution
  hipStream_t stream = nullptr, own_stream = nullptr, cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int variant = 0, use_graph = 1;
  int sync_calls = 1;   // LBM_OPT_SYNC
  // counters
  int64_t t = 0, snap_t = 0, mon_t = -1;
  bool mon_valid = false;
  double last_res = 0, last_mass = 0;
  // what the last lbm_step call launched
  lbm_launch_record_t last_call{0, -1, 0, 0, 0, -1, 0, 0, 0, 0};
};
