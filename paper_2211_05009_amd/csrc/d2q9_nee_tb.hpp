// d2q9_nee_tb.hpp -- K steps per launch with the paper's on-node walls
// (non-equilibrium extrapolation, arXiv 2211.05009 Sec. 2.2 (ii)).
//
// A block owns a TX x TY tile of nodes and a region of LDS around it
// (K + 1 nodes below and left of the tile, K above and right).  The K
// steps run between two LDS buffers (one barrier per step) and the last
// one stores the tile's nodes from registers.  Per node the arithmetic is
// k_step_nee's, in the same order (pull at the node's reference node, then
// nee_collide), so any number of steps per launch gives the same bits as
// one-step launches.  Step 1 pulls its nodes' inputs straight from the state
// f*(t) in global memory; step s updates the region's nodes s or more sites
// from its border, [s, RW - s) x [s, RH - s) in region coordinates (a
// constant width: the step loop is unrolled), skipping those outside the
// lattice; the last step takes the tile alone.  A fluid node reads its eight
// neighbours at the previous step and a wall node its reference node's, one
// node inward; every such node is inside the lattice and inside the previous
// step's window.  The extra node below and left is for a tile that starts at
// the last column (or row): its right (top) wall node reads two nodes to its
// left (below), which the previous step's window then still holds.
#pragma once
#include <hip/hip_runtime.h>

#include "d2q9_nee.hpp"
#include "d2q9_step.hpp"

namespace lbm {

template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__device__ __forceinline__ void nee_tb_pull(const StepParams<T> &p, T *lds) {
  constexpr int RW = TX + 2 * K + 1, RH = TY + 2 * K + 1, RS = RW * RH;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int nx = p.nx, ny = p.ny;
  const int X0 = tx * TX - K - 1, Y0 = ty * TY - K - 1;   // node of region site (0, 0)
  // one node: pull at its reference node from `src` (row pitch `pitch`,
  // plane stride `P`, node (x0, y0) at element 0), collide or extrapolate
  auto update = [&](const T *src, int P, int pitch, int x0, int y0, int gx, int gy, T(&f)[9]) {
    const int xr = min(max(gx, 1), nx - 2), yr = min(max(gy, 1), ny - 2);
    pull_fluid<T>(src, P, pitch, (yr - y0) * pitch + (xr - x0), f);
    nee_collide<T, SHIFT>(f, p.omega, xr != gx || yr != gy, gy == ny - 1 ? p.ulid : T(0));
  };
  {  // step 1 from global memory into LDS buffer 0
    constexpr int W = RW - 2, N = W * (RH - 2);
    for (int q = threadIdx.x; q < N; q += NT) {
      const int lx = 1 + q % W, ly = 1 + q / W;
      const int gx = X0 + lx, gy = Y0 + ly;
      if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
      T f[9];
      update(p.src, p.plane, p.pitch, 0, 0, gx, gy, f);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * RS + ly * RW + lx] = f[i];
    }
  }
  // steps 2..K; the last one takes the tile alone (its window's extra low
  // row and column are not needed)
  auto step = [&](int s) {
    __syncthreads();
    const T *in = lds + ((s - 2) & 1) * 9 * RS;
    T *out = lds + ((s - 1) & 1) * 9 * RS;
    const int b = s == K ? K + 1 : s, W = s == K ? TX : RW - 2 * s;
    const int N = s == K ? TX * TY : W * (RH - 2 * s);
    for (int q = threadIdx.x; q < N; q += NT) {
      const int lx = b + q % W, ly = b + q / W;
      const int gx = X0 + lx, gy = Y0 + ly;
      if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
      T f[9];
      update(in, RS, RW, X0, Y0, gx, gy, f);
      if (s == K) {
        const int o = gy * p.pitch + gx;
        // not read again in this launch: FP32 with non-temporal stores (+3 %
        // at 501 x 501), FP64 with plain ones (+2.7 % at 501 x 501)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          if constexpr (sizeof(T) == 4)
            __builtin_nontemporal_store(f[i], p.dst + (size_t)i * p.plane + o);
          else
            p.dst[(size_t)i * p.plane + o] = f[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i * RS + ly * RW + lx] = f[i];
      }
    }
  };
  // the step loop unrolled, so each window's width is a constant
#pragma unroll
  for (int s = 2; s <= K; ++s) step(s);
}

template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step_nee_tb(StepParams<T> p) {
  constexpr int RS = (TX + 2 * K + 1) * (TY + 2 * K + 1);
  static_assert(K >= 2, "one-step launches take k_step_nee");
  static_assert(2 * 9 * RS * sizeof(T) <= 160 * 1024, "two region buffers fit the LDS");
  __shared__ T lds[2 * 9 * RS];
  nee_tb_pull<T, SHIFT, K, TX, TY, NT>(p, lds);
}

}  // namespace lbm
