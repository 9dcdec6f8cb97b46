// d2q9_batch.hpp -- one launch advances many uneven cavities (gfx950).
//
// All cavities of a batch live in one pair of buffers; cavity c's nine
// planes start at element offset base_c and use its own pitch and plane
// size.  A tile table lists (cavity, tile x, tile y) for every 64 x (BY*RY)
// tile of every active cavity, cavity-major; the XCD-aware tile order of
// d2q9_step.hpp then gives each XCD a contiguous run of rows of one or two
// cavities.  The per-site arithmetic is exactly that of k_step (same pull,
// same collision), so a cavity advanced in a batch matches the same cavity
// advanced alone bit for bit.
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_monitor.hpp"
#include "d2q9_step.hpp"
#include "d2q9_temporal.hpp"

namespace lbm {

template <typename T>
struct CavityDesc {
  int base;       // element offset of plane 0 in each buffer
  int nx, ny, pitch, plane;
  int uref_off;   // offset of the cavity's Eq. 6 reference field
  T omega, u6;    // 1/tau, u_lid/6
};

template <typename T, bool SHIFT, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_step_batch(
    const T *__restrict__ src, T *__restrict__ dst,
    const CavityDesc<T> *__restrict__ cav, const int4 *__restrict__ tiles) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int4 te = tiles[tile];                 // (cavity, tx, ty, -)
  const CavityDesc<T> d = cav[te.x];
  const int x = te.y * 64 + threadIdx.x;
  if (x >= d.nx) return;
  const bool xl = x > 0, xr = x < d.nx - 1;
  const T *s = src + d.base;
  T *o_base = dst + d.base;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = te.z * (BY * RY) + r * BY + threadIdx.y;
    if (y >= d.ny) return;
    const int o = y * d.pitch + x;
    T f[9];
    pull<T>(s, d.plane, d.pitch, o, xl, xr, y > 0, y < d.ny - 1, d.u6, f);
    bgk_collide<T, SHIFT>(f, d.omega);
#pragma unroll
    for (int i = 0; i < 9; ++i) o_base[i * d.plane + o] = f[i];
  }
}

// Vector form (see k_step_vec): tiles of (64 V) x BY sites.
template <typename T, bool SHIFT, int BY>
__global__ __launch_bounds__(64 * BY) void k_step_batch_vec(
    const T *__restrict__ src, T *__restrict__ dst,
    const CavityDesc<T> *__restrict__ cav, const int4 *__restrict__ tiles) {
  constexpr int V = 16 / sizeof(T);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int4 te = tiles[tile];
  const CavityDesc<T> d = cav[te.x];
  const int x0 = (te.y * 64 + threadIdx.x) * V;
  const int y = te.z * BY + threadIdx.y;
  if (x0 >= d.nx || y >= d.ny) return;
  step_vec_sites<T, SHIFT, V>(src + d.base, dst + d.base, d.plane, d.pitch, d.nx, d.ny, x0, y,
                              d.omega, d.u6);
}

// Temporal form (see k_step_tb): K steps per launch on TX x TY tiles.
// MON = 1 / 2: the first / second launch of a chunk that carries the Eq. 6
// monitor of every listed cavity's start state (see TbMonitor): tile entry
// t stores partial triple t (a cavity's tiles are listed together, so its
// partials form one run), and the block of a cavity's first tile, whose
// entry holds the cavity's tile count in .w (0 elsewhere), adds that run
// in order into out[cavity].  uref is the batch's reference field, each
// cavity's at its uref_off.
template <typename T, bool SHIFT, int K, int TX, int TY, int NT, int MON = 0>
__global__ __launch_bounds__(NT) void k_step_batch_tb(
    const T *__restrict__ src, T *__restrict__ dst,
    const CavityDesc<T> *__restrict__ cav, const int4 *__restrict__ tiles, TbMonitor mon) {
  __shared__ T lds[9 * (TX + 2 * K) * (TY + 2 * K)];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int4 te = tiles[tile];
  const CavityDesc<T> d = cav[te.x];
  TbMonBlock mb{nullptr, nullptr, nullptr, 0, nullptr};
  if (MON != 0) {
    mb.uref = mon.uref + d.uref_off;
    mb.part = mon.partials + (size_t)tile * kNumSums;
    mb.fin = mb.part;
    mb.nfin = te.w;
    mb.out = mon.out + (size_t)te.x * kNumSums;
  }
  // the region through LDS in monitored launches: the sweep's state and
  // reference fields are beyond the caches (measured: 236 against 343 us
  // with the sums taken after the steps)
  tb_tile<T, SHIFT, K, TX, TY, NT, MON, false, true, true>(
      lds, src + d.base, dst + d.base, d.nx, d.ny, d.pitch, d.plane, d.omega, d.u6, te.y, te.z, mb);
}

// Monitor over a fixed 64 x 4 tiling (one site per thread): per-tile
// partials of sum(rho - 1), sum |u - u_ref|^2, sum |u_ref|^2; the
// reference field is replaced by u when UPDATE.
template <typename T, bool SHIFT, bool UPDATE>
__global__ __launch_bounds__(256) void k_monitor_batch(
    const T *__restrict__ src, const CavityDesc<T> *__restrict__ cav,
    const int4 *__restrict__ tiles, double2 *__restrict__ uref,
    double *__restrict__ partials) {
  const int4 te = tiles[blockIdx.x];
  const CavityDesc<T> d = cav[te.x];
  const int x = te.y * 64 + (threadIdx.x & 63);
  const int y = te.z * 4 + (threadIdx.x >> 6);
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  if (x < d.nx && y < d.ny) {
    double drho, jx, jy;
    site_moments<T, SHIFT>(src + d.base, d.plane, y * d.pitch + x, drho, jx, jy);
    const double rho = 1.0 + drho;
    const double ux = jx / rho, uy = jy / rho;
    acc[0] = drho;
    if (UPDATE) {
      const int k = d.uref_off + y * d.nx + x;
      const double2 r = uref[k];
      const double dx = ux - r.x, dy = uy - r.y;
      acc[1] = dx * dx + dy * dy;
      acc[2] = r.x * r.x + r.y * r.y;
      uref[k] = make_double2(ux, uy);
    }
  }
  block_reduce_store<kNumSums>(acc, partials + blockIdx.x * kNumSums);
}

// One block per listed cavity: add that cavity's tile partials
// [first[j], first[j] + count[j]) in a fixed order into out[cav[j]].
static __global__ __launch_bounds__(kRedThreads) void k_finalize_batch(
    const double *__restrict__ partials, const int *__restrict__ first,
    const int *__restrict__ count, const int *__restrict__ cav_of,
    double *__restrict__ out) {
  const int j = blockIdx.x;
  const int b0 = first[j], nb = count[j];
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) acc[k] += partials[(b0 + b) * kNumSums + k];
  block_reduce_store<kNumSums>(acc, out + cav_of[j] * kNumSums);
}

// Probe records of the batch: one block per active cavity (cav_of lists
// them), its npts points (units of L, [n][npts][2]) interpolated as
// probe_point does, written to record count[c] % cap of the cavity's ring
// ([n][cap][npts][3]); then count[c] advances.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_probe_ring_batch(
    const T *__restrict__ buf, const CavityDesc<T> *__restrict__ cav,
    const int *__restrict__ cav_of, const double *__restrict__ xy, int npts,
    double *__restrict__ ring, long long cap, unsigned long long *__restrict__ count) {
  const int c = cav_of[blockIdx.x];
  const CavityDesc<T> d = cav[c];
  Geometry g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.pitch = d.pitch;
  g.plane = d.plane;
  const unsigned long long k = count[c];
  double *rec = ring + ((long long)c * cap + (long long)(k % (unsigned long long)cap)) * 3 * npts;
  for (int p = threadIdx.x; p < npts; p += 256) {
    const long long q = ((long long)c * npts + p) * 2;
    probe_point<T, SHIFT>(buf + d.base, g, xy[q], xy[q + 1], rec + 3 * p);
  }
  __syncthreads();
  if (threadIdx.x == 0) count[c] = k + 1;
}

}  // namespace lbm
