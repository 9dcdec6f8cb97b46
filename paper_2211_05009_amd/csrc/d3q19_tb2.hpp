// d3q19_tb2.hpp -- two D3Q19 steps per launch for the lid-driven box (the
// three-dimensional extension of Sec. 4 of arXiv 2211.05009).  Two forms:
//
// k_step3_tb2: a block owns a TX x TY x TZ tile.  Step 1 updates the tile
// and the one-site shell around it (the window, clipped to the box),
// pulling each site's inputs from the state f*(t) in global memory exactly
// as k_step3 does, and leaves the results in LDS; step 2 updates the tile's
// sites out of LDS (a link from outside the box reflects, with the lid's
// term, as in k_step3) and stores them.
//
// k_step3_zs2: a block owns a TX x TY column over a range of planes and
// marches through z, keeping step-1 results of three planes in LDS, so only
// the x-y shell is computed twice.
//
// Per site both use k_step3's pulls and collision in the same order, so the
// result is bit-identical to two one-step launches, and each launch reads
// and writes the state once for two steps: the one-step kernel runs at the
// rate of a plain device copy.
#pragma once
#include <hip/hip_runtime.h>

#include "d3q19_step.hpp"

namespace lbm {

// Element reads and writes of a state array.  `at(d, o)` is element d + o,
// where d is the same for every lane (a population plane and a fixed
// neighbour offset) and o the lane's site; `elem(e)` is element e.
template <typename T>
struct PtrArray {   // any array: 64-bit addresses
  const T *a;
  __device__ __forceinline__ T at(int d, int o) const { return a[d + o]; }
  __device__ __forceinline__ T elem(int e) const { return a[e]; }
};
// Arrays below 2^31 bytes as raw buffers: the lane's byte offset in a VGPR,
// the uniform one in an SGPR, no per-access 64-bit address arithmetic.  The
// descriptor: stride 0 (raw), num_records = the array's bytes, and
// 0x00020000 as its last word (data format 32 bits) for gfx9-family GPUs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
struct BufArray {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ T at(int d, int o) const {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, o * 4, d * 4, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, o * 8, d * 8, 0));
  }
  __device__ __forceinline__ T elem(int e) const { return at(0, e); }
  // non-temporal store (cache policy NT)
  __device__ __forceinline__ void put(int d, int o, T v) const {
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, o * 4, d * 4, 2);
    else
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(unsigned __attribute__((ext_vector_type(2))), v), r, o * 8, d * 8, 2);
  }
};

// Link i of site (x, y, z) comes from a site of the box (only the nonzero
// velocity components are tested).
__device__ __forceinline__ bool from_box(int i, int x, int y, int z, int nx, int ny, int nz) {
  return (cx19(i) == 0 || (unsigned)(x - cx19(i)) < (unsigned)nx) &&
         (cy19(i) == 0 || (unsigned)(y - cy19(i)) < (unsigned)ny) &&
         (cz19(i) == 0 || (unsigned)(z - cz19(i)) < (unsigned)nz);
}

// The lid's term on a reflected link through the lid (links 8 and 9 of the
// top row y = ny - 1), as in k_step3.
template <typename T>
__device__ __forceinline__ T lid19(int i, T f, int y, int ny, T u6) {
  if (i == 8) return y == ny - 1 ? f - u6 : f;
  if (i == 9) return y == ny - 1 ? f + u6 : f;
  return f;
}

// The 19 inputs of site (x, y, z), at element o of an array with plane,
// row and slab strides ps, rs, ss: a link from outside the box reflects,
// with the lid's term where it crosses the lid, as in k_step3.  A wavefront
// whose sites all lie off the box's outer shell takes unchecked pulls; any
// other selects each link's element (the neighbour's, or the site's own
// opposite population) and loads it, without branches, so the wavefronts of
// a column at a face do not run two paths.  The values are the same.
template <typename T, typename A>
__device__ __forceinline__ void pull19(const A &a, int ps, int rs, int ss, int o, int x, int y,
                                       int z, int nx, int ny, int nz, T u6, T (&f)[19]) {
  if (__all(x >= 1 && x < nx - 1 && y >= 1 && y < ny - 1 && z >= 1 && z < nz - 1)) {
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = a.at(i * ps - cx19(i) - cy19(i) * rs - cz19(i) * ss, o);
    return;
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int e = from_box(i, x, y, z, nx, ny, nz)
                      ? o + i * ps - cx19(i) - cy19(i) * rs - cz19(i) * ss
                      : o + opp19(i) * ps;
    f[i] = lid19<T>(i, a.elem(e), y, ny, u6);
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
    pull19<T>(PtrArray<T>{p.src}, p.plane, rowp, slab, z * slab + y * rowp + x, x, y, z, nx, ny,
              nz, p.u6, f);
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
    pull19<T>(PtrArray<T>{lds}, WS, WX, WX * WY, (lz * WY + ly) * WX + lx, x, y, z, nx, ny, nz,
              p.u6, f);
    bgk_collide19<T, SHIFT>(f, p.omega);
    const int o = z * slab + y * rowp + x;
#pragma unroll
    for (int i = 0; i < 19; ++i)   // not read again in this launch
      __builtin_nontemporal_store(f[i], p.dst + (size_t)i * p.plane + o);
  }
}

// The 19 inputs of tile site l of plane z from step-1 results in LDS:
// pop(i, z') is population i's array of window sites (row stride WX) on
// plane z'.  Reflected and with the lid's term as pull19.
template <typename T, int WX, typename P>
__device__ __forceinline__ void pull19_planes(const P &pop, int l, int x, int y, int z, int nx,
                                              int ny, int nz, T u6, T (&f)[19]) {
  // a link moving +z comes from the plane below, -z from the plane above
  if (__all(x >= 1 && x < nx - 1 && y >= 1 && y < ny - 1 && z >= 1 && z < nz - 1)) {
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = pop(i, z - cz19(i))[l - cx19(i) - cy19(i) * WX];
    return;
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const T *e = from_box(i, x, y, z, nx, ny, nz) ? pop(i, z - cz19(i)) + l - cx19(i) - cy19(i) * WX
                                                  : pop(opp19(i), z) + l;
    f[i] = lid19<T>(i, *e, y, ny, u6);
  }
}

// Position of population i among those with the same c_z (c_z = -1: 6, 12,
// 13, 16, 17; 0: 0-4, 7-10; +1: 5, 11, 14, 15, 18).
__device__ __forceinline__ int kz19(int i) {
  constexpr int v[19] = {0, 1, 2, 3, 4, 0, 0, 5, 6, 7, 8, 1, 1, 2, 2, 3, 3, 4, 4};
  return v[i];
}

// Two steps per launch, marching through z.  A block owns a TX x TY column
// of the box over the planes [zb, zb + zc) and one window site (the tile
// and its one-site shell in x and y) per thread.  Walking up the planes it
// computes step 1 on the window of plane p (pulled from the state f*(t) in
// global memory, as k_step3 does) into LDS, then step 2 on the tile of
// plane p - 1 out of the step-1 results of planes p - 2, p - 1 and p, and
// stores it.  Only the x-y shell is computed twice (plus one plane below
// and above the block's range), and the next plane's step-1 inputs are
// loaded into registers while step 2 runs.  LDS keeps each population only
// as long as step 2 reads it: plane p's five -z populations serve step 2 of
// plane p - 1 (as the plane above) and of plane p (reflections), its nine
// in-plane ones step 2 of plane p, its five +z ones step 2 of planes p and
// p + 1: 2, 2 and 3 planes deep, 43 values per window site.  Per site the
// arithmetic is k_step3's in the same order: bit-identical to two one-step
// launches.  BUF: the state arrays (19 planes) are below 2^31 bytes and are
// read and written as raw buffers.
template <typename T, bool SHIFT, int TX, int TY, int NT, bool BUF>
__global__ __launch_bounds__(NT) void k_step3_zs2(Step3Params<T> p) {
  constexpr int WX = TX + 2, WY = TY + 2, WP = WX * WY, TP = TX * TY;
  constexpr int DN = 0, MID = 2 * 5 * WP, UP = MID + 2 * 9 * WP, RING = UP + 3 * 5 * WP;
  static_assert(NT >= WP, "one window site per thread");
  static_assert(RING * sizeof(T) <= 160 * 1024, "the step-1 planes fit the LDS");
  __shared__ T ring[RING];
  // population i of plane z (z >= -1)
  auto pop = [&](int i, int z) -> T * {
    if (cz19(i) < 0) return ring + DN + ((z + 2) & 1) * 5 * WP + kz19(i) * WP;
    if (cz19(i) == 0) return ring + MID + ((z + 2) & 1) * 9 * WP + kz19(i) * WP;
    return ring + UP + ((z + 3) % 3) * 5 * WP + kz19(i) * WP;
  };
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int per_c = p.tiles_x * p.tiles_y;
  const int c = b / per_c, r = b - c * per_c;
  const int ty = r / p.tiles_x, tx = r - ty * p.tiles_x;
  const int X0 = tx * TX - 1, Y0 = ty * TY - 1;   // window site (0, 0)
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int rowp = p.pitch, slab = p.pitch * p.ny;
  const int zb = c * p.zc, ze = min(zb + p.zc, nz);
  const int q = threadIdx.x;
  // this thread's window site (step 1) and tile site (step 2)
  const int wx = X0 + q % WX, wy = Y0 + q / WX;
  const bool wok = q < WP && wx >= 0 && wx < nx && wy >= 0 && wy < ny;
  const int sx = X0 + 1 + q % TX, sy = Y0 + 1 + q / TX;
  const bool sok = q < TP && sx < nx && sy < ny;
  const int sl = (1 + q / TX) * WX + 1 + q % TX;
  const long long bytes = 19LL * p.plane * (long long)sizeof(T);
  const BufArray<T> bsrc{buffer_of(p.src, bytes)}, bdst{buffer_of(p.dst, bytes)};   // BUF only
  T fin[19];
  auto load = [&](int z) {
    if (wok && z >= 0 && z < nz) {
      const int o = z * slab + wy * rowp + wx;
      if constexpr (BUF)
        pull19<T>(bsrc, p.plane, rowp, slab, o, wx, wy, z, nx, ny, nz, p.u6, fin);
      else
        pull19<T>(PtrArray<T>{p.src}, p.plane, rowp, slab, o, wx, wy, z, nx, ny, nz, p.u6, fin);
    }
  };
  load(zb - 1);
  for (int z1 = zb - 1; z1 <= ze; ++z1) {
    if (wok && z1 >= 0 && z1 < nz) {   // step 1 on plane z1
      bgk_collide19<T, SHIFT>(fin, p.omega);
#pragma unroll
      for (int i = 0; i < 19; ++i) pop(i, z1)[q] = fin[i];
    }
    __syncthreads();
    if (z1 < ze) load(z1 + 1);   // in flight during step 2
    const int z2 = z1 - 1;
    if (z2 >= zb && sok) {        // step 2 on plane z2
      T f[19];
      pull19_planes<T, WX>(pop, sl, sx, sy, z2, nx, ny, nz, p.u6, f);
      bgk_collide19<T, SHIFT>(f, p.omega);
      const int o = z2 * slab + sy * rowp + sx;
#pragma unroll
      for (int i = 0; i < 19; ++i) {   // not read again in this launch
        if constexpr (BUF)
          bdst.put(i * p.plane, o, f[i]);
        else
          __builtin_nontemporal_store(f[i], p.dst + (size_t)i * p.plane + o);
      }
    }
    __syncthreads();   // the next step 1 overwrites what step 2 read last
  }
}

}  // namespace lbm
