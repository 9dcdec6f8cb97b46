// d2q9_nee.hpp -- the fused step with the paper's own wall scheme:
// non-equilibrium extrapolation on on-node walls (arXiv 2211.05009,
// Sec. 2.2 (ii), after Guo, Zheng and Shi).
//
// Geometry: nx x ny nodes; the outermost rows and columns are wall nodes,
// the walls are nx - 1 spacings apart (L = nx - 1).  The top row, corners
// included, moves with (u_lid, 0); the other wall nodes are at rest.
//
// Stored state: post-collision populations f*(t) at every node, as for the
// half-way walls.  A fluid node pulls its nine populations (every source is
// a node, so no link crosses a wall) and collides (Eqs. 1-3).  A wall node b
// takes its reference node r = (clamp(x, 1, nx-2), clamp(y, 1, ny-2)) --
// the fluid neighbour along the wall normal, the diagonal one at a corner --
// pulls r's nine populations f_r, and stores
//     f*_b = f^eq(rho_r, u_w) + (1 - omega) (f_r - f^eq(rho_r, u_r)),
// the collision of the extrapolated distribution f^eq(rho_r, u_w) + f^neq_r
// (its moments are rho_r and rho_r u_w, so its own equilibrium is
// f^eq(rho_r, u_w)).  Everything comes from the state at t, so one launch
// is one step.  In the SHIFT storage every f is replaced by g = f - w; the
// differences f - f^eq are unchanged.
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_monitor.hpp"
#include "d2q9_step.hpp"

namespace lbm {

// The nine populations streaming into fluid node o (all sources are nodes).
template <typename T>
__device__ __forceinline__ void pull_fluid(const T *__restrict__ s, int P, int pitch, int o,
                                           T (&f)[9]) {
  f[0] = s[o];
  f[1] = s[P + o - 1];
  f[2] = s[2 * P + o - pitch];
  f[3] = s[3 * P + o + 1];
  f[4] = s[4 * P + o + pitch];
  f[5] = s[5 * P + o - 1 - pitch];
  f[6] = s[6 * P + o + 1 - pitch];
  f[7] = s[7 * P + o + 1 + pitch];
  f[8] = s[8 * P + o - 1 + pitch];
}

// Eq. 2 for (rho, ux, uy); base = rho (plain storage) or rho - 1 (SHIFT),
// giving f^eq or f^eq - w.  Only wall nodes use it, and a wall node is
// rebuilt from its reference node at every step, so the rounding of the
// weights (FP32: 7.5e-9 relative) scales its equilibrium part once, like a
// lid speed off by that fraction, and does not compound from step to step
// as it would inside the collision (bgk_collide avoids rounded weights).
template <typename T>
__device__ __forceinline__ void equilibrium9(T base, T rho, T ux, T uy, T (&e)[9]) {
  const T usq = T(1.5) * (ux * ux + uy * uy);
  const T w0 = T(LBM_W0), wa = T(LBM_WA), wd = T(LBM_WD);
  const T ra = wa * rho, rd = wd * rho, ba = wa * base, bd = wd * base;
  e[0] = w0 * base - (w0 * rho) * usq;
  const T sx = ra * (T(4.5) * ux * ux - usq), ax = ra * (T(3) * ux);
  const T sy = ra * (T(4.5) * uy * uy - usq), ay = ra * (T(3) * uy);
  e[1] = ba + sx + ax;
  e[3] = ba + sx - ax;
  e[2] = ba + sy + ay;
  e[4] = ba + sy - ay;
  const T p = ux + uy, m = uy - ux;
  const T sp = rd * (T(4.5) * p * p - usq), ap = rd * (T(3) * p);
  const T sm = rd * (T(4.5) * m * m - usq), am = rd * (T(3) * m);
  e[5] = bd + sp + ap;
  e[7] = bd + sp - ap;
  e[6] = bd + sm + am;
  e[8] = bd + sm - am;
}

// Node update from the populations streamed to it (a fluid node) or to its
// reference node (a wall node), in place.  A fluid node takes the BGK
// collision.  A wall node takes f^eq(rho_r, (uw, 0)) + (1 - omega)(f -
// f^eq(rho_r, u_r)) with rho_r, u_r the moments of f: since the BGK update
// of f is f^eq(rho_r, u_r) + (1 - omega)(f - f^eq(rho_r, u_r)), that is the
// BGK update plus f^eq(rho_r, (uw, 0)) - f^eq(rho_r, u_r).  So a wavefront
// holding both kinds runs the collision once, and its wall lanes add only
// the moments before it and that difference after it.
template <typename T, bool SHIFT>
__device__ __forceinline__ void nee_collide(T (&f)[9], T omega, bool wall, T uw) {
  T rho = T(1), ux = T(0), uy = T(0);
  if (wall) {
    const T s = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const T jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const T jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    rho = SHIFT ? T(1) + s : s;
    const T rinv = recip<T>(rho);
    ux = jx * rinv;
    uy = jy * rinv;
  }
  bgk_collide<T, SHIFT>(f, omega);
  if (wall) {
    // w_i rho [3 c.(uw - u) + 4.5 ((c.uw)^2 - (c.u)^2) - 1.5 (uw^2 - u^2)],
    // a link and its opposite sharing the even part
    const T du = T(1.5) * (uw * uw - (ux * ux + uy * uy));
    const T ra = T(LBM_WA) * rho, rd = T(LBM_WD) * rho;
    f[0] -= (T(LBM_W0) * rho) * du;
    auto pair = [&](int a, int b, T r, T cw, T cu) {
      const T odd = T(3) * (cw - cu), even = T(4.5) * (cw * cw - cu * cu) - du;
      f[a] += r * (even + odd);
      f[b] += r * (even - odd);
    };
    pair(1, 3, ra, uw, ux);            // (1, 0), (-1, 0)
    pair(2, 4, ra, T(0), uy);          // (0, 1), (0, -1)
    pair(5, 7, rd, uw, ux + uy);       // (1, 1), (-1, -1)
    pair(6, 8, rd, -uw, uy - ux);      // (-1, 1), (1, -1)
  }
}

// One step over a tile of 64 x (BY * RY) nodes (block 64 x BY threads,
// RY rows per thread spaced BY apart), XCD-aware tile order as in k_step.
// Needs nx, ny >= 3.
template <typename T, bool SHIFT, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_step_nee(StepParams<T> p) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int x = tx * 64 + threadIdx.x;
  if (x >= p.nx) return;
  const int xr = min(max(x, 1), p.nx - 2);
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = ty * (BY * RY) + r * BY + threadIdx.y;
    if (y >= p.ny) return;
    const int yr = min(max(y, 1), p.ny - 2);
    T f[9];
    pull_fluid<T>(p.src, p.plane, p.pitch, yr * p.pitch + xr, f);
    nee_collide<T, SHIFT>(f, p.omega, xr != x || yr != y, y == p.ny - 1 ? p.ulid : T(0));
    const int o = y * p.pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) p.dst[i * p.plane + o] = f[i];
  }
}

// Initial lid row (Sec. 2.2 (i): the top wall's nodes start with u_x = u):
// f^eq(1, (u, 0)) on row ny - 1, computed in FP64 and rounded once.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_init_lid_row(T *__restrict__ d, Geometry g, double u) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= g.nx) return;
  const int o = (g.ny - 1) * g.pitch + x;
  double e[9];
  equilibrium9<double>(SHIFT ? 0.0 : 1.0, 1.0, u, 0.0, e);
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i * g.plane + o] = (T)e[i];
}

// Stream function on nodes: Psi = 0 on the bottom row, trapezoid rule up
// each column, Psi[y] = Psi[y-1] - (u_x[y-1] + u_x[y]) / 2 (lattice units).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(256) void k_psi_nodes(const T *__restrict__ s, Geometry g,
                                                   double *__restrict__ psi) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= g.nx) return;
  double drho, jx, jy;
  site_moments<T, SHIFT>(s, g.plane, x, drho, jx, jy);
  double prev = jx / (1.0 + drho), acc = 0.0;
  psi[x] = 0.0;
  for (int y = 1; y < g.ny; ++y) {
    site_moments<T, SHIFT>(s, g.plane, y * g.pitch + x, drho, jx, jy);
    const double ux = jx / (1.0 + drho);
    acc = acc - 0.5 * (prev + ux);
    psi[(size_t)y * g.nx + x] = acc;
    prev = ux;
  }
}

}  // namespace lbm
