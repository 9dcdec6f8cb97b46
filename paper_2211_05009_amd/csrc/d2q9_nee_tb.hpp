// d2q9_nee_tb.hpp -- K steps per launch with the paper's on-node walls
// (non-equilibrium extrapolation, arXiv 2211.05009 Sec. 2.2 (ii)).
//
// A block owns a TX x TY tile of nodes and loads the region of the state
// f*(t) around it (clipped to the lattice) into LDS once; each
// of the K steps then updates the nodes whose inputs the previous step left
// valid, out of one LDS buffer into the other, and the last step stores the
// tile's nodes.  Per node the arithmetic is k_step_nee's, in the same order
// (pull at the node's reference node, then bgk_collide or nee_wall), so any
// number of steps per launch gives the same bits as one-step launches.
//
// Valid window: a fluid node needs its eight neighbours at the previous
// step, a wall node its reference node's (one node inward), so a node two
// nodes inside a wall is read by the wall node beside it.  Sides of the
// region that face other tiles lose one node per step; sides on the
// lattice's edge lose none (nothing lies beyond them).  The region reaches
// K + 1 nodes below and left of the tile and K above and right: a tile
// that starts at the last column (or row) holds a right (top) wall node
// whose reference's neighbour lies two nodes to its left (below), and the
// extra node keeps it in the window at step K - 1.  At step K the window
// holds the tile (and on the low sides one node more, not stored).
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_nee.hpp"
#include "d2q9_step.hpp"

namespace lbm {

template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step_nee_tb(StepParams<T> p) {
  constexpr int RW = TX + 2 * K + 1, RH = TY + 2 * K + 1, RS = RW * RH;
  static_assert(2 * 9 * RS * sizeof(T) <= 160 * 1024, "two region buffers fit the LDS");
  __shared__ T lds[2 * 9 * RS];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int nx = p.nx, ny = p.ny;
  // region origin (node coordinates of LDS site (0, 0); may be negative)
  // and the part of the region inside the lattice
  const int X0 = tx * TX - K - 1, Y0 = ty * TY - K - 1;
  const int cx0 = max(X0, 0), cx1 = min(X0 + RW, nx);
  const int cy0 = max(Y0, 0), cy1 = min(Y0 + RH, ny);
  {  // load f*(t) on the region
    const int cw = cx1 - cx0, n = cw * (cy1 - cy0);
    for (int q = threadIdx.x; q < n; q += NT) {
      const int gy = cy0 + q / cw, gx = cx0 + q % cw;
      const int o = gy * p.pitch + gx, l = (gy - Y0) * RW + (gx - X0);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * RS + l] = p.src[(size_t)i * p.plane + o];
    }
  }
  __syncthreads();
  const bool el = cx0 == 0, er = cx1 == nx, eb = cy0 == 0, et = cy1 == ny;
#pragma unroll 1
  for (int s = 1; s <= K; ++s) {
    const T *in = lds + ((s - 1) & 1) * 9 * RS;
    T *out = lds + (s & 1) * 9 * RS;
    const int wx0 = el ? 0 : cx0 + s, wx1 = er ? nx : cx1 - s;
    const int wy0 = eb ? 0 : cy0 + s, wy1 = et ? ny : cy1 - s;
    // the last step keeps only the tile's own nodes
    const int sx0 = s == K ? max(wx0, tx * TX) : wx0, sx1 = s == K ? min(wx1, tx * TX + TX) : wx1;
    const int sy0 = s == K ? max(wy0, ty * TY) : wy0, sy1 = s == K ? min(wy1, ty * TY + TY) : wy1;
    const int ww = sx1 - sx0, n = ww * (sy1 - sy0);
    for (int q = threadIdx.x; q < n; q += NT) {
      const int gy = sy0 + q / ww, gx = sx0 + q % ww;
      const int xr = min(max(gx, 1), nx - 2), yr = min(max(gy, 1), ny - 2);
      T f[9];
      pull_fluid<T>(in, RS, RW, (yr - Y0) * RW + (xr - X0), f);
      if (xr == gx && yr == gy)
        bgk_collide<T, SHIFT>(f, p.omega);
      else
        nee_wall<T, SHIFT>(f, p.omega, gy == ny - 1 ? p.ulid : T(0));
      if (s == K) {
        const int o = gy * p.pitch + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) p.dst[(size_t)i * p.plane + o] = f[i];
      } else {
        const int l = (gy - Y0) * RW + (gx - X0);
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i * RS + l] = f[i];
      }
    }
    if (s < K) __syncthreads();
  }
}

}  // namespace lbm
