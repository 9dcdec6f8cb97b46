// d3q19_step.hpp -- the fused D3Q19 lattice-BGK step of the lid-driven box
// (the three-dimensional extension named as future work in Sec. 4 of arXiv
// 2211.05009), and its FP64 monitors.
//
// Same method as the two-dimensional step (Eqs. 1-3, 5): pull streaming of
// the post-collision populations, half-way bounce-back on all six faces, the
// lid above the top row y = ny - 1 moving with (u_lid, 0, 0) and owning every
// link through its plane, BGK collision towards the second-order equilibrium
// with the D3Q19 weights 1/3, 1/18, 1/36.  Stored state: f*(t).
//
// Layout: 19 planes of nz x ny x pitch elements (pitch = nx rounded up to
// 64), plane i at element offset i * plane; a 64-lane wavefront covers 64
// consecutive x of one row.  SHIFT storage holds g = f - w in FP32.
//
// Velocity order (each odd index followed by its opposite):
//   0 (0,0,0); 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1) 6 (0,0,-1)
//   7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1)
//   13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1)
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_monitor.hpp"
#include "d2q9_step.hpp"

namespace lbm {

__device__ __forceinline__ int cx19(int i) {
  constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__device__ __forceinline__ int cy19(int i) {
  constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[i];
}
__device__ __forceinline__ int cz19(int i) {
  constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return v[i];
}
__device__ __forceinline__ int opp19(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__device__ __forceinline__ double w19(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

template <typename T>
struct Step3Params {
  const T *__restrict__ src;
  T *__restrict__ dst;
  int nx, ny, nz, pitch;
  int plane;        // elements per population plane
  int tiles_x, tiles_y;
  int zc;           // planes per block in the z-marching kernel (k_step3_zs2)
  T omega, u6;      // 1/tau, u_lid / 6 (the lid term of links 8 and 9)
};

// Collide one site: f[19] in (after streaming; g = f - w for SHIFT), out the
// post-collision values.  As in two dimensions, f^eq_i = w_i E_i with
// E_i = b + 3 c_i.j + (4.5 (c_i.j)^2 - 1.5 j.j) / rho (b = rho, or rho - 1 for
// the shift), and omega w_i is taken as 4, 2 or 1 times omega / 36 against
// 3 E_0 - 9 f_0, E_i - 18 f_i and E_i - 36 f_i: exact scalings, so no weight
// is rounded (FP32 weights would scale the momentum by 1 + 7.5e-9 omega at
// every collision).
template <typename T, bool SHIFT>
__device__ __forceinline__ void bgk_collide19(T (&f)[19], T omega) {
  T s = f[0];
#pragma unroll
  for (int i = 1; i < 19; ++i) s += f[i];
  // momentum from the differences of opposite links (each odd link is
  // followed by its opposite), no term with a zero velocity component
  const T d1 = f[1] - f[2], d3 = f[3] - f[4], d5 = f[5] - f[6];
  const T d7 = f[7] - f[8], d9 = f[9] - f[10], d11 = f[11] - f[12];
  const T d13 = f[13] - f[14], d15 = f[15] - f[16], d17 = f[17] - f[18];
  const T jx = d1 + d7 + d9 + d11 + d13;
  const T jy = d3 + d7 - d9 + d15 + d17;
  const T jz = d5 + d11 - d13 + d15 - d17;
  const T rho = SHIFT ? T(1) + s : s;
  const T rinv = recip<T>(rho);
  const T b = SHIFT ? s : rho;
  const T od = omega * T(1.0 / 36.0);
  const T jsq = T(1.5) * (jx * jx + jy * jy + jz * jz);
  f[0] += (T(4) * od) * (T(3) * (b - rinv * jsq) - T(9) * f[0]);
  // link a and its opposite a + 1: c_a . j = cj and -cj share E's even part
  auto pair = [&](int a, T cj, T w, T k) {
    const T q = b + rinv * (T(4.5) * cj * cj - jsq), e = T(3) * cj;
    f[a] += w * ((q + e) - k * f[a]);
    f[a + 1] += w * ((q - e) - k * f[a + 1]);
  };
  const T oa = T(2) * od;
  pair(1, jx, oa, T(18));
  pair(3, jy, oa, T(18));
  pair(5, jz, oa, T(18));
  pair(7, jx + jy, od, T(36));
  pair(9, jx - jy, od, T(36));
  pair(11, jx + jz, od, T(36));
  pair(13, jx - jz, od, T(36));
  pair(15, jy + jz, od, T(36));
  pair(17, jy - jz, od, T(36));
}

// One step: block 64 x BY threads = one tile of 64 x BY sites of one z
// plane; blocks are ordered tile-x fastest, then tile-y, then z, and handed
// to XCDs in contiguous ranges.
template <typename T, bool SHIFT, int BY>
__global__ __launch_bounds__(64 * BY) void k_step3(Step3Params<T> p) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int per_z = p.tiles_x * p.tiles_y;
  const int z = b / per_z, r = b - z * per_z;
  const int ty = r / p.tiles_x, tx = r - ty * p.tiles_x;
  const int x = tx * 64 + threadIdx.x, y = ty * BY + threadIdx.y;
  if (x >= p.nx || y >= p.ny || z >= p.nz) return;
  const int rowp = p.pitch, slab = p.pitch * p.ny;
  const int o = z * slab + y * rowp + x;
  T f[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int xs = x - cx19(i), ys = y - cy19(i), zs = z - cz19(i);
    if (xs >= 0 && xs < p.nx && ys >= 0 && ys < p.ny && zs >= 0 && zs < p.nz) {
      f[i] = p.src[i * p.plane + o - cx19(i) - cy19(i) * rowp - cz19(i) * slab];
    } else {
      // reflected at the wall the link crosses: the reverse population of
      // this site, plus the moving-wall term when the link crosses the lid
      f[i] = p.src[opp19(i) * p.plane + o];
      if (ys >= p.ny) {
        if (i == 8) f[i] -= p.u6;        // -6 w_7 (c_7 . u_w) = -u/6
        else if (i == 9) f[i] += p.u6;   // -6 w_10 (c_10 . u_w) = +u/6
      }
    }
  }
  bgk_collide19<T, SHIFT>(f, p.omega);
#pragma unroll
  for (int i = 0; i < 19; ++i) p.dst[i * p.plane + o] = f[i];
}

// FP64 moments of a stored site: drho = rho - 1, momentum j.
template <typename T, bool SHIFT>
__device__ __forceinline__ void site_moments19(const T *__restrict__ s, int plane, int o,
                                               double &drho, double &jx, double &jy,
                                               double &jz) {
  double sum = 0.0, a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {   // the zero components skipped (constants here)
    const double v = (double)s[i * plane + o];
    sum += v;
    if (cx19(i)) a += cx19(i) > 0 ? v : -v;
    if (cy19(i)) b += cy19(i) > 0 ? v : -v;
    if (cz19(i)) c += cz19(i) > 0 ? v : -v;
  }
  drho = SHIFT ? sum : sum - 1.0;
  jx = a;
  jy = b;
  jz = c;
}

// Monitor sums over the box (one site per thread, grid-stride): sum (rho - 1),
// sum |u - u_ref|^2, sum |u_ref|^2; with UPDATE the reference field (dense
// [3][n] FP64) becomes the current velocity.  Block partials [kNumSums] per
// block, added in a fixed order by k_finalize.
template <typename T, bool SHIFT, bool UPDATE>
__global__ __launch_bounds__(kRedThreads) void k_monitor3(const T *__restrict__ s, int nx,
                                                          int ny, int nz, int pitch, int plane,
                                                          double *__restrict__ uref,
                                                          double *__restrict__ partials) {
  const long long n = (long long)nx * ny * nz;
  double acc[kNumSums] = {0.0, 0.0, 0.0};
  for (long long q = blockIdx.x * (long long)kRedThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kRedThreads) {
    const int x = (int)(q % nx);
    const long long yz = q / nx;
    const int y = (int)(yz % ny), z = (int)(yz / ny);
    double drho, jx, jy, jz;
    site_moments19<T, SHIFT>(s, plane, (z * ny + y) * pitch + x, drho, jx, jy, jz);
    const double rho = 1.0 + drho;
    const double u[3] = {jx / rho, jy / rho, jz / rho};
    acc[0] += drho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double r = uref[a * n + q];
      acc[1] += (u[a] - r) * (u[a] - r);
      acc[2] += r * r;
      if (UPDATE) uref[a * n + q] = u[a];
    }
  }
  block_reduce_store<kNumSums>(acc, partials + blockIdx.x * kNumSums);
}

// Moments into dense [n] FP64 arrays (any may be null), n = nx ny nz,
// index (z ny + y) nx + x.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_moments3(const T *__restrict__ s, int nx, int ny,
                                                  int nz, int pitch, int plane,
                                                  double *__restrict__ rho,
                                                  double *__restrict__ ux,
                                                  double *__restrict__ uy,
                                                  double *__restrict__ uz) {
  const long long n = (long long)nx * ny * nz;
  const long long q = blockIdx.x * 256LL + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % nx);
  const long long yz = q / nx;
  const int y = (int)(yz % ny), z = (int)(yz / ny);
  double drho, jx, jy, jz;
  site_moments19<T, SHIFT>(s, plane, (z * ny + y) * pitch + x, drho, jx, jy, jz);
  const double r = 1.0 + drho;
  if (rho) rho[q] = r;
  if (ux) ux[q] = jx / r;
  if (uy) uy[q] = jy / r;
  if (uz) uz[q] = jz / r;
}

// Populations: set the stored state from f(t) (dense [19][n] FP64; collided
// here so the stored state is f*(t)), or read the stored f*(t) back.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_set_pop3(T *__restrict__ d, int nx, int ny, int nz,
                                                  int pitch, int plane,
                                                  const double *__restrict__ f, double omega) {
  const long long n = (long long)nx * ny * nz;
  const long long q = blockIdx.x * 256LL + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % nx);
  const long long yz = q / nx;
  const int y = (int)(yz % ny), z = (int)(yz / ny);
  double g[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) g[i] = f[i * n + q] - (SHIFT ? w19(i) : 0.0);
  bgk_collide19<double, SHIFT>(g, omega);
  const int o = (z * ny + y) * pitch + x;
#pragma unroll
  for (int i = 0; i < 19; ++i) d[i * plane + o] = (T)g[i];
}

template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_get_pop3(const T *__restrict__ s, int nx, int ny,
                                                  int nz, int pitch, int plane,
                                                  double *__restrict__ f) {
  const long long n = (long long)nx * ny * nz;
  const long long q = blockIdx.x * 256LL + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % nx);
  const long long yz = q / nx;
  const int y = (int)(yz % ny), z = (int)(yz / ny);
  const int o = (z * ny + y) * pitch + x;
#pragma unroll
  for (int i = 0; i < 19; ++i) f[i * n + q] = (double)s[i * plane + o] + (SHIFT ? w19(i) : 0.0);
}

}  // namespace lbm
