// d2q9_temporal.hpp -- K steps of Eq. 1 per launch with the tile in LDS.
//
// A single step moves every population once and reuses nothing, so its
// cost is the launch plus one pass over memory.  On the production lattices
// (500 x (500 Ar): 9-36 MB per buffer, resident in the Infinity Cache) the
// fixed cost of a launch is about half of the step time.  Here a block loads
// a region of (TX + 2K) x (TY + 2K) sites of the post-collision state into
// LDS, applies K complete steps in LDS (the valid window shrinks by one site
// per side and step: the halo is recomputed instead of exchanged), and
// writes the TX x TY core.  Global traffic per launch is one region read and
// one core write, launches drop K-fold, and the LDS absorbs the K-1
// intermediate states.
//
// The per-site arithmetic is that of k_step: pull with the same wall
// conditions and moving-wall term, bgk_collide, so K steps here equal K
// launches of k_step bit for bit.
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_step.hpp"

namespace lbm {

// K steps on the region in LDS; the valid window shrinks by one site per
// side and step.
template <typename T, bool SHIFT, int K, int RW, int RH, int NT, bool INTERIOR>
__device__ __forceinline__ void tb_steps(T *lds, int X0, int Y0, int nx, int ny, T omega,
                                         T u6) {
  constexpr int RS = RW * RH;
  constexpr int J = (RS + NT - 1) / NT;
  for (int s = 1; s <= K; ++s) {
    T v[J][9];
    bool act[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int q = threadIdx.x + j * NT;
      const int ry = q / RW, rx = q - ry * RW;
      const int gx = X0 + rx, gy = Y0 + ry;
      act[j] = q < RS && rx >= s && rx < RW - s && ry >= s && ry < RH - s;
      if (!INTERIOR) act[j] = act[j] && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      if (act[j]) {
        T *f = v[j];
        if (INTERIOR) {
          f[0] = lds[q];
          f[1] = lds[RS + q - 1];
          f[2] = lds[2 * RS + q - RW];
          f[3] = lds[3 * RS + q + 1];
          f[4] = lds[4 * RS + q + RW];
          f[5] = lds[5 * RS + q - 1 - RW];
          f[6] = lds[6 * RS + q + 1 - RW];
          f[7] = lds[7 * RS + q + 1 + RW];
          f[8] = lds[8 * RS + q - 1 + RW];
        } else {
          const bool xl = gx > 0, xr = gx < nx - 1, yb = gy > 0, yt = gy < ny - 1;
          f[0] = lds[q];
          f[1] = lds[xl ? (RS + q - 1) : (3 * RS + q)];
          f[2] = lds[yb ? (2 * RS + q - RW) : (4 * RS + q)];
          f[3] = lds[xr ? (3 * RS + q + 1) : (RS + q)];
          f[4] = lds[yt ? (4 * RS + q + RW) : (2 * RS + q)];
          f[5] = lds[(xl && yb) ? (5 * RS + q - 1 - RW) : (7 * RS + q)];
          f[6] = lds[(xr && yb) ? (6 * RS + q + 1 - RW) : (8 * RS + q)];
          f[7] = lds[(xr && yt) ? (7 * RS + q + 1 + RW) : (5 * RS + q)];
          f[8] = lds[(xl && yt) ? (8 * RS + q - 1 + RW) : (6 * RS + q)];
          if (!yt) {
            f[7] -= u6;
            f[8] += u6;
          }
        }
        bgk_collide<T, SHIFT>(v[j], omega);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int q = threadIdx.x + j * NT;
      if (act[j])
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[i * RS + q] = v[j][i];
    }
    __syncthreads();
  }
}

// One tile (tile_x, tile_y) of TX x TY core sites advanced K steps; src and
// dst point at plane 0 of the cavity.
template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__device__ __forceinline__ void tb_tile(T *lds, const T *__restrict__ src, T *__restrict__ dst,
                                        int nx, int ny, int pitch, int P, T omega, T u6,
                                        int tile_x, int tile_y) {
  constexpr int RW = TX + 2 * K, RH = TY + 2 * K, RS = RW * RH;
  constexpr int J = (RS + NT - 1) / NT;       // region sites per thread
  const int X0 = tile_x * TX - K;             // global x of region column 0
  const int Y0 = tile_y * TY - K;

  // load the region (sites inside the cavity)
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int q = threadIdx.x + j * NT;
    if (q < RS) {
      const int ry = q / RW, rx = q - ry * RW;
      const int gx = X0 + rx, gy = Y0 + ry;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        const int o = gy * pitch + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[i * RS + q] = src[i * P + o];
      }
    }
  }
  __syncthreads();

  // Tiles whose region lies inside the cavity (no wall within reach) take a
  // branch-free pull with constant LDS offsets; the rest test the walls.
  const bool interior = X0 >= 0 && X0 + RW <= nx && Y0 >= 0 && Y0 + RH <= ny;
  if (interior)
    tb_steps<T, SHIFT, K, RW, RH, NT, true>(lds, X0, Y0, nx, ny, omega, u6);
  else
    tb_steps<T, SHIFT, K, RW, RH, NT, false>(lds, X0, Y0, nx, ny, omega, u6);

  // store the core
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int q = threadIdx.x + j * NT;
    if (q < RS) {
      const int ry = q / RW, rx = q - ry * RW;
      const int gx = X0 + rx, gy = Y0 + ry;
      if (rx >= K && rx < K + TX && ry >= K && ry < K + TY && gx < nx && gy < ny) {
        const int o = gy * pitch + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * P + o] = lds[i * RS + q];
      }
    }
  }
}

template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step_tb(StepParams<T> p, int tiles_x) {
  __shared__ T lds[9 * (TX + 2 * K) * (TY + 2 * K)];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  tb_tile<T, SHIFT, K, TX, TY, NT>(lds, p.src, p.dst, p.nx, p.ny, p.pitch, p.plane, p.omega,
                                   p.u6, tile % tiles_x, tile / tiles_x);
}

}  // namespace lbm
