// d2q9_vortex.hpp -- vortex extraction from the stream function (the
// stream-function values and vortex centres of Tables 1-2): arg-extrema of
// Psi over three regions and the list of all vortex centres.
//
// Psi is a dense FP64 [ny][nx] field (k_psi).  Sites are addressed by their
// linear index k = y nx + x.
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {

constexpr int kVortexThreads = 256;
constexpr int kVortexRegions = 3;

// Region r of site (x, y): 0 = whole lattice (maximum of Psi: the primary
// vortex); 1 = x < nx/2, y < hy and 2 = x >= nx/2, y < hy (minimum of Psi:
// the lower-left and lower-right vortices), hy = min(ny, nx/2).
__device__ __forceinline__ bool in_region(int r, int x, int y, int nx, int hy) {
  if (r == 0) return true;
  if (y >= hy) return false;
  return r == 1 ? x < nx / 2 : x >= nx / 2;
}

// a better than b: strictly larger (region 0) or smaller (1, 2) value, ties
// to the smaller site index; index -1 marks "no candidate".
__device__ __forceinline__ bool better(int r, double av, int ak, double bv, int bk) {
  if (ak < 0) return false;
  if (bk < 0) return true;
  if (av != bv) return r == 0 ? av > bv : av < bv;
  return ak < bk;
}

// Reduce the per-thread candidates of one block in LDS; thread 0 ends with
// the block's best.  The result does not depend on the order of reduction
// (the comparison is a total order), so it is deterministic.
__device__ __forceinline__ void block_best(int r, double &v, int &k, double *sv, int *sk) {
  const int t = threadIdx.x;
  sv[t] = v;
  sk[t] = k;
  __syncthreads();
  for (int s = kVortexThreads / 2; s > 0; s >>= 1) {
    if (t < s && better(r, sv[t + s], sk[t + s], sv[t], sk[t])) {
      sv[t] = sv[t + s];
      sk[t] = sk[t + s];
    }
    __syncthreads();
  }
  v = sv[0];
  k = sk[0];
  __syncthreads();
}

// Per-block best site of each region; partials are [region][block].
static __global__ __launch_bounds__(kVortexThreads) void k_vortex_partial(
    const double *__restrict__ psi, int nx, int ny, double *__restrict__ pv,
    int *__restrict__ pk) {
  __shared__ double sv[kVortexThreads];
  __shared__ int sk[kVortexThreads];
  const int n = nx * ny, hy = min(ny, nx / 2);
  double v[kVortexRegions];
  int k[kVortexRegions];
#pragma unroll
  for (int r = 0; r < kVortexRegions; ++r) {
    v[r] = 0.0;
    k[r] = -1;
  }
  for (int q = blockIdx.x * kVortexThreads + threadIdx.x; q < n;
       q += gridDim.x * kVortexThreads) {
    const int y = q / nx, x = q - y * nx;
    const double p = psi[q];
#pragma unroll
    for (int r = 0; r < kVortexRegions; ++r)
      if (in_region(r, x, y, nx, hy) && better(r, p, q, v[r], k[r])) {
        v[r] = p;
        k[r] = q;
      }
  }
#pragma unroll
  for (int r = 0; r < kVortexRegions; ++r) {
    block_best(r, v[r], k[r], sv, sk);
    if (threadIdx.x == 0) {
      pv[r * gridDim.x + blockIdx.x] = v[r];
      pk[r * gridDim.x + blockIdx.x] = k[r];
    }
  }
}

// One block: best of the nb partials of each region -> out_v[3], out_k[3].
static __global__ __launch_bounds__(kVortexThreads) void k_vortex_final(
    const double *__restrict__ pv, const int *__restrict__ pk, int nb,
    double *__restrict__ out_v, int *__restrict__ out_k) {
  __shared__ double sv[kVortexThreads];
  __shared__ int sk[kVortexThreads];
#pragma unroll
  for (int r = 0; r < kVortexRegions; ++r) {
    double v = 0.0;
    int k = -1;
    for (int b = threadIdx.x; b < nb; b += kVortexThreads)
      if (better(r, pv[r * nb + b], pk[r * nb + b], v, k)) {
        v = pv[r * nb + b];
        k = pk[r * nb + b];
      }
    block_best(r, v, k, sv, sk);
    if (threadIdx.x == 0) {
      out_v[r] = v;
      out_k[r] = k;
    }
  }
}

// Vortex centres: interior sites (1 <= x <= nx-2, 1 <= y <= ny-2) where Psi
// is strictly above (kind +1) or strictly below (kind -1) all eight
// neighbours and |Psi| >= min_abs.  Each centre takes a slot from *count
// (a global atomic) and, if the slot is below cap, stores (Psi, k, kind);
// the slots come in no particular order.
static __global__ __launch_bounds__(kVortexThreads) void k_vortex_centres(
    const double *__restrict__ psi, int nx, int ny, double min_abs, int cap,
    unsigned int *__restrict__ count, double *__restrict__ ev, int *__restrict__ ek) {
  const int q = blockIdx.x * kVortexThreads + threadIdx.x;
  if (q >= nx * ny) return;
  const int y = q / nx, x = q - y * nx;
  if (x < 1 || x > nx - 2 || y < 1 || y > ny - 2) return;
  const double c = psi[q];
  if (!(fabs(c) >= min_abs)) return;
  bool mx = true, mn = true;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dy == 0) continue;
      const double b = psi[q + dy * nx + dx];
      mx = mx && c > b;
      mn = mn && c < b;
    }
  if (!mx && !mn) return;
  const unsigned int slot = atomicAdd(count, 1u);
  if (slot < (unsigned int)cap) {
    ev[slot] = c;
    ek[2 * slot] = q;
    ek[2 * slot + 1] = mx ? 1 : -1;
  }
}

}  // namespace lbm
