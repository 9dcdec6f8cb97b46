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

// The 19 inputs of site (x, y, z), at element o of an array with plane,
// row and slab strides ps, rs, ss: a link from outside the box reflects,
// with the lid's term where it crosses the lid, as in k_step3.  Sites whose
// every link comes from inside the box (all but the box's outer shell) take
// the unchecked pulls; the values are the same either way.
template <typename T>
__device__ __forceinline__ void pull19(const T *a, int ps, int rs, int ss, int o, int x, int y,
                                       int z, int nx, int ny, int nz, T u6, T (&f)[19]) {
  if (x >= 1 && x < nx - 1 && y >= 1 && y < ny - 1 && z >= 1 && z < nz - 1) {
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = a[i * ps + o - cx19(i) - cy19(i) * rs - cz19(i) * ss];
    return;
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int xs = x - cx19(i), ys = y - cy19(i), zs = z - cz19(i);
    if (xs >= 0 && xs < nx && ys >= 0 && ys < ny && zs >= 0 && zs < nz) {
      f[i] = a[i * ps + o - cx19(i) - cy19(i) * rs - cz19(i) * ss];
    } else {
      f[i] = a[opp19(i) * ps + o];
      if (ys >= ny) {
        if (i == 8) f[i] -= u6;
        else if (i == 9) f[i] += u6;
      }
    }
  }
}

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
    T f[19];
    pull19<T>(p.src, p.plane, rowp, slab, z * slab + y * rowp + x, x, y, z, nx, ny, nz, p.u6, f);
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
    T f[19];
    pull19<T>(lds, WS, WX, WX * WY, (lz * WY + ly) * WX + lx, x, y, z, nx, ny, nz, p.u6, f);
    bgk_collide19<T, SHIFT>(f, p.omega);
    const int o = z * slab + y * rowp + x;
#pragma unroll
    for (int i = 0; i < 19; ++i)   // not read again in this launch
      __builtin_nontemporal_store(f[i], p.dst + (size_t)i * p.plane + o);
  }
}

}  // namespace lbm
