// d3q19_tb2.hpp -- two D3Q19 steps per launch for the lid-driven box (the
// three-dimensional extension of Sec. 4 of arXiv 2211.05009).
//
// A block owns a TX x TY x TZ tile of sites.  Step 1 updates the tile and
// the one-site shell around it (the window, clipped to the box), pulling
// each site's inputs from the state f*(t) in global memory exactly as
// k_step3 does, and leaves the results in LDS; step 2 updates the tile's
// sites out of LDS (a link from outside the box reflects, with the lid's
// term, as in k_step3) and stores them.  The per-site arithmetic is
// k_step3's in the same order, so the result is bit-identical to two
// one-step launches, and each launch reads and writes the state once for
// two steps: the one-step kernel runs at the rate of a plain device copy.
#pragma once
#include <hip/hip_runtime.h>

#include "d3q19_step.hpp"

namespace lbm {

template <typename T, bool SHIFT, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_step3_tb2(Step3Params<T> p) {
  constexpr int WX = TX + 2, WY = TY + 2, WZ = TZ + 2, WS = WX * WY * WZ;
  static_assert(19 * WS * sizeof(T) <= 160 * 1024, "the window fits the LDS");
  __shared__ T lds[19 * WS];
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int per_z = p.tiles_x * p.tiles_y;
  const int tz = b / per_z, r = b - tz * per_z;
  const int ty = r / p.tiles_x, tx = r - ty * p.tiles_x;
  const int X0 = tx * TX - 1, Y0 = ty * TY - 1, Z0 = tz * TZ - 1;   // window site (0, 0, 0)
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int rowp = p.pitch, slab = p.pitch * p.ny;
  // step 1: the window's sites inside the box, from global memory
  for (int q = threadIdx.x; q < WS; q += NT) {
    const int lx = q % WX, t = q / WX, ly = t % WY, lz = t / WY;
    const int x = X0 + lx, y = Y0 + ly, z = Z0 + lz;
    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) continue;
    const int o = z * slab + y * rowp + x;
    T f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int xs = x - cx19(i), ys = y - cy19(i), zs = z - cz19(i);
      if (xs >= 0 && xs < nx && ys >= 0 && ys < ny && zs >= 0 && zs < nz) {
        f[i] = p.src[i * p.plane + o - cx19(i) - cy19(i) * rowp - cz19(i) * slab];
      } else {   // reflected, plus the lid's term where the link crosses it
        f[i] = p.src[opp19(i) * p.plane + o];
        if (ys >= ny) {
          if (i == 8) f[i] -= p.u6;
          else if (i == 9) f[i] += p.u6;
        }
      }
    }
    bgk_collide19<T, SHIFT>(f, p.omega);
#pragma unroll
    for (int i = 0; i < 19; ++i) lds[i * WS + q] = f[i];
  }
  __syncthreads();
  // step 2: the tile's sites, from the window
  constexpr int TS = TX * TY * TZ;
  for (int q = threadIdx.x; q < TS; q += NT) {
    const int lx = 1 + q % TX, t = q / TX, ly = 1 + t % TY, lz = 1 + t / TY;
    const int x = X0 + lx, y = Y0 + ly, z = Z0 + lz;
    if (x >= nx || y >= ny || z >= nz) continue;
    const int l = (lz * WY + ly) * WX + lx;
    T f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int xs = x - cx19(i), ys = y - cy19(i), zs = z - cz19(i);
      if (xs >= 0 && xs < nx && ys >= 0 && ys < ny && zs >= 0 && zs < nz) {
        f[i] = lds[i * WS + l - cx19(i) - cy19(i) * WX - cz19(i) * WX * WY];
      } else {
        f[i] = lds[opp19(i) * WS + l];
        if (ys >= ny) {
          if (i == 8) f[i] -= p.u6;
          else if (i == 9) f[i] += p.u6;
        }
      }
    }
    bgk_collide19<T, SHIFT>(f, p.omega);
    const int o = z * slab + y * rowp + x;
#pragma unroll
    for (int i = 0; i < 19; ++i)   // not read again in this launch
      __builtin_nontemporal_store(f[i], p.dst + (size_t)i * p.plane + o);
  }
}

}  // namespace lbm
