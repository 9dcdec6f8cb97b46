// lbm_internal.h -- the handle behind lbm_t (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct lbm_cavity {
  // lattice and parameters
  int nx = 0, ny = 0, pitch = 0, plane = 0, dtype = 0;
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
  // counters
  int64_t t = 0, snap_t = 0, mon_t = -1;
  bool mon_valid = false;
  double last_res = 0, last_mass = 0;
};
