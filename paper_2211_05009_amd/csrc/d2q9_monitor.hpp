// d2q9_monitor.hpp -- moments, FP64 reductions, probes, stream function,
// initialisation and population transfer kernels (gfx950).
//
// All reductions accumulate in FP64 whatever the storage precision: a
// 64-lane wavefront reduction by lane shuffles, then across the block's
// waves through LDS, one partial per block, and a single-block final pass
// that adds the partials in a fixed order (results do not depend on timing).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2q9_step.hpp"

namespace lbm {

constexpr int kRedThreads = 256;   // threads per reduction block
constexpr int kRedBlocks = 1024;   // fixed grid of the reduction kernels
constexpr int kNumSums = 3;        // sums carried by the monitor reduction

// on_node = 1: walls on the outermost nodes (non-equilibrium extrapolation),
// node i at i / (nx - 1) in units of L; 0: half-way walls, site i's centre
// at (i + 1/2) / nx.
struct Geometry {
  int nx, ny, pitch, plane;
  int on_node = 0;
};

// Weights of the nine directions, velocity order of d2q9_step.hpp.
__device__ __forceinline__ double wgt(int i) {
  return i == 0 ? LBM_W0 : (i < 5 ? LBM_WA : LBM_WD);
}
__device__ __forceinline__ int cxs(int i) {
  // 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
  const int t[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  return t[i];
}
__device__ __forceinline__ int cys(int i) {
  const int t[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  return t[i];
}

// rho - 1 and rho u of one site's nine stored populations, in FP64 (Eq. 3;
// a collision leaves both unchanged, so they are also the moments of the
// pre-collision f).  One order of operations wherever the values come from,
// so the monitors' sums do not depend on the path that took them.
template <typename T, bool SHIFT>
__device__ __forceinline__ void moments_of(const T (&v)[9], double &drho, double &jx,
                                           double &jy) {
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = (double)v[i];
  double sum = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  drho = SHIFT ? sum : sum - 1.0;
  jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
}

// The same at element offset o of planes `plane` apart.
template <typename T, bool SHIFT>
__device__ __forceinline__ void site_moments(const T *__restrict__ s, int plane,
                                             int o, double &drho, double &jx,
                                             double &jy) {
  T v[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = s[i * plane + o];
  moments_of<T, SHIFT>(v, drho, jx, jy);
}

template <int N>
__device__ __forceinline__ void block_reduce_store(double (&v)[N], double *out) {
  // wavefront reduction
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  __shared__ double part[kRedThreads / 64][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = 0.0;
      for (int w = 0; w < kRedThreads / 64; ++w) a += part[w][k];
      out[k] = a;
    }
  }
}

// Monitor: per-block partials of sum(rho - 1), sum |u - u_ref|^2,
// sum |u_ref|^2 (Eq. 6 numerator and denominator); if UPDATE, the reference
// field u_ref (interleaved (ux, uy) per site, dense [ny][nx]) is replaced by
// the current u.
template <typename T, bool SHIFT, bool UPDATE>
__global__ __launch_bounds__(kRedThreads) void k_monitor(
    const T *__restrict__ s, Geometry g, double2 *__restrict__ uref,
    double *__restrict__ partials) {
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  const int n = g.nx * g.ny;
  for (int k = blockIdx.x * kRedThreads + threadIdx.x; k < n;
       k += gridDim.x * kRedThreads) {
    const int y = k / g.nx, x = k - y * g.nx;
    double drho, jx, jy;
    site_moments<T, SHIFT>(s, g.plane, y * g.pitch + x, drho, jx, jy);
    const double rho = 1.0 + drho;
    const double ux = jx / rho, uy = jy / rho;
    acc[0] += drho;
    if (UPDATE) {
      const double2 r = uref[k];
      const double dx = ux - r.x, dy = uy - r.y;
      acc[1] += dx * dx + dy * dy;
      acc[2] += r.x * r.x + r.y * r.y;
      uref[k] = make_double2(ux, uy);
    }
  }
  block_reduce_store<kNumSums>(acc, partials + blockIdx.x * kNumSums);
}

// Per-block partial sums of a dense FP64 array (first slot of each triple).
static __global__ __launch_bounds__(kRedThreads) void k_sum_dense(
    const double *__restrict__ a, long long n, double *__restrict__ partials) {
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  for (long long k = blockIdx.x * (long long)kRedThreads + threadIdx.x; k < n;
       k += (long long)gridDim.x * kRedThreads)
    acc[0] += a[k];
  block_reduce_store<kNumSums>(acc, partials + blockIdx.x * kNumSums);
}

// Per-block partials for a start from fields: sum rho, sum (-1)^x rho u_x,
// sum (-1)^y rho u_y (dense [ny][nx]; null rho = 1, null velocity = 0).
static __global__ __launch_bounds__(kRedThreads) void k_init_sums(
    const double *__restrict__ rho, const double *__restrict__ ux,
    const double *__restrict__ uy, int nx, long long n, double *__restrict__ partials) {
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  for (long long k = blockIdx.x * (long long)kRedThreads + threadIdx.x; k < n;
       k += (long long)gridDim.x * kRedThreads) {
    const int x = (int)(k % nx), y = (int)(k / nx);
    const double r = rho ? rho[k] : 1.0;
    acc[0] += r;
    if (ux) acc[1] += (x & 1 ? -r : r) * ux[k];
    if (uy) acc[2] += (y & 1 ? -r : r) * uy[k];
  }
  block_reduce_store<kNumSums>(acc, partials + blockIdx.x * kNumSums);
}

// Single block: add nparts partial triples in a fixed order.
static __global__ __launch_bounds__(kRedThreads) void k_finalize(
    const double *__restrict__ partials, int nparts, double *__restrict__ out) {
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kRedThreads)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) acc[k] += partials[b * kNumSums + k];
  block_reduce_store<kNumSums>(acc, out);
}

// rho, u_x, u_y into dense [ny][nx] FP64 arrays (any may be null).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ s,
                                                 Geometry g, double *rho,
                                                 double *ux, double *uy) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= g.nx * g.ny) return;
  const int y = k / g.nx, x = k - y * g.nx;
  double drho, jx, jy;
  site_moments<T, SHIFT>(s, g.plane, y * g.pitch + x, drho, jx, jy);
  const double r = 1.0 + drho;
  if (rho) rho[k] = r;
  if (ux) ux[k] = jx / r;
  if (uy) uy[k] = jy / r;
}

// Bilinear interpolation of (rho, ux, uy) between site centres (or nodes)
// at points given in units of the width L (site i's centre is (i + 1/2)/nx;
// node i sits at i / (nx - 1)).
template <typename T, bool SHIFT>
__device__ void probe_point(const T *__restrict__ s, Geometry g, double px,
                            double py, double *out3) {
  double X, Y;
  if (g.on_node) {
    X = px * (g.nx - 1);
    Y = py * (g.nx - 1);
  } else {
    X = px * g.nx - 0.5;
    Y = py * g.nx - 0.5;
  }
  X = fmin(fmax(X, 0.0), (double)(g.nx - 1));
  Y = fmin(fmax(Y, 0.0), (double)(g.ny - 1));
  int i0 = (int)floor(X), j0 = (int)floor(Y);
  if (i0 > g.nx - 2) i0 = g.nx - 2;
  if (j0 > g.ny - 2) j0 = g.ny - 2;
  const double tx = X - i0, ty = Y - j0;
  const double wts[4] = {(1 - tx) * (1 - ty), tx * (1 - ty), (1 - tx) * ty, tx * ty};
  const int xs[4] = {i0, i0 + 1, i0, i0 + 1};
  const int ys[4] = {j0, j0, j0 + 1, j0 + 1};
  double r = 0, u = 0, v = 0;
  for (int c = 0; c < 4; ++c) {
    double drho, jx, jy;
    site_moments<T, SHIFT>(s, g.plane, ys[c] * g.pitch + xs[c], drho, jx, jy);
    const double rr = 1.0 + drho;
    r += wts[c] * rr;
    u += wts[c] * (jx / rr);
    v += wts[c] * (jy / rr);
  }
  out3[0] = r;
  out3[1] = u;
  out3[2] = v;
}

// On-demand probes: out[p*3 + {0,1,2}].
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_probe(const T *__restrict__ s, Geometry g,
                                               const double *__restrict__ xy,
                                               int npts, double *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npts) return;
  probe_point<T, SHIFT>(s, g, xy[2 * p], xy[2 * p + 1], out + 3 * p);
}

// Time-series probes into a ring of `cap` records of 3 * npts doubles.
// Single block; the record counter lives in device memory so the kernel can
// sit in a replayed graph.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_probe_ring(
    const T *__restrict__ s, Geometry g, const double *__restrict__ xy, int npts,
    double *__restrict__ ring, long long cap,
    unsigned long long *__restrict__ count) {
  const unsigned long long c = *count;
  const long long slot = (long long)(c % (unsigned long long)cap);
  double *rec = ring + slot * 3 * (long long)npts;
  for (int p = threadIdx.x; p < npts; p += 256)
    probe_point<T, SHIFT>(s, g, xy[2 * p], xy[2 * p + 1], rec + 3 * p);
  __syncthreads();
  if (threadIdx.x == 0) *count = c + 1;
}

// Resample a cavity onto the surrogate's 256 x 128 canvas: pixel (x, y) of a
// canvas row y < rows sits at ((x + 1/2)/128, (y + 1/2)/128) in units of the
// width L; its (rho, u) is the bilinear probe of the lattice there.  Outputs
// (FP32): target[y][x] = (100 (rho - 1), u_x / u_lid, u_y / u_lid), mask 1;
// rows >= rows are zero.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_canvas(const T *__restrict__ s, Geometry g, double u_lid,
                                                int rows, float *__restrict__ target,
                                                float *__restrict__ mask) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= 256 * 128) return;
  const int y = k / 128, x = k % 128;
  if (y >= rows) {
    target[3 * k] = target[3 * k + 1] = target[3 * k + 2] = 0.f;
    mask[k] = 0.f;
    return;
  }
  double v[3];
  probe_point<T, SHIFT>(s, g, (x + 0.5) / 128.0, (y + 0.5) / 128.0, v);
  target[3 * k] = (float)(100.0 * (v[0] - 1.0));
  target[3 * k + 1] = (float)(v[1] / u_lid);
  target[3 * k + 2] = (float)(v[2] / u_lid);
  mask[k] = 1.f;
}

// Stream function: one thread per column, prefix sum of -u_x upward,
// midpoint rule (Psi = 0 on the bottom wall).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_psi(const T *__restrict__ s, Geometry g,
                                             double *__restrict__ psi) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= g.nx) return;
  double acc = 0.0;
  for (int y = 0; y < g.ny; ++y) {
    double drho, jx, jy;
    site_moments<T, SHIFT>(s, g.plane, y * g.pitch + x, drho, jx, jy);
    const double ux = jx / (1.0 + drho);
    psi[(size_t)y * g.nx + x] = -(acc + 0.5 * ux);
    acc += ux;
  }
}

// Store the equilibrium of Eq. 2 for fields rho, ux, uy (dense [ny][nx];
// null rho = 1, null velocity = 0).  The equilibrium is its own collision
// result, so this is the stored post-collision state of a start at
// equilibrium (Sec. 2.2 (i)).  Padding columns are written as rest values.
// rho is scaled by rho_scale; (sx, sy) remove a staggered momentum:
// rho u_x -= sx (-1)^x and rho u_y -= sy (-1)^y.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_init_eq(T *__restrict__ d, Geometry g,
                                                 const double *__restrict__ rho,
                                                 const double *__restrict__ ux,
                                                 const double *__restrict__ uy,
                                                 double rho_scale, double sx, double sy) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= g.pitch * g.ny) return;
  const int y = k / g.pitch, x = k - y * g.pitch;
  double r = 1.0, u = 0.0, v = 0.0;
  if (x < g.nx) {
    const int q = y * g.nx + x;
    if (rho) r = rho[q] * rho_scale;
    if (ux) u = ux[q] - (x & 1 ? -sx : sx) / r;
    if (uy) v = uy[q] - (y & 1 ? -sy : sy) / r;
  }
  const double usq = 1.5 * (u * u + v * v);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double w = wgt(i);
    const double cu = cxs(i) * u + cys(i) * v;
    const double poly = 3.0 * cu + 4.5 * cu * cu - usq;
    // f^eq = w rho (1 + poly); shifted: f^eq - w = w (rho - 1 + rho poly)
    const double val = SHIFT ? w * ((r - 1.0) + r * poly) : w * r * (1.0 + poly);
    d[i * g.plane + k] = (T)val;
  }
}

// Replace the state by the collision of f (dense FP64 [9][ny][nx]): the
// stored value is f - omega (f - f^eq) computed in FP64, then rounded to the
// storage type (shifted by -w for SHIFT).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_set_pop(T *__restrict__ d, Geometry g,
                                                 const double *__restrict__ f,
                                                 double omega) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= g.nx * g.ny) return;
  const int y = k / g.nx, x = k - y * g.nx;
  const size_t n = (size_t)g.nx * g.ny;
  double v[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = f[i * n + k];
  bgk_collide<double, false>(v, omega);
  const int o = y * g.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i * g.plane + o] = (T)(SHIFT ? v[i] - wgt(i) : v[i]);
}

// Stored populations -> dense FP64 f* [9][ny][nx] (adds w back for SHIFT).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_get_pop(const T *__restrict__ s,
                                                 Geometry g, double *__restrict__ f) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= g.nx * g.ny) return;
  const int y = k / g.nx, x = k - y * g.nx;
  const size_t n = (size_t)g.nx * g.ny;
  const int o = y * g.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double v = (double)s[i * g.plane + o];
    f[i * n + k] = SHIFT ? v + wgt(i) : v;
  }
}

}  // namespace lbm
