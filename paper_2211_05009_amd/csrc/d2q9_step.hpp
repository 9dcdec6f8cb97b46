// d2q9_step.hpp -- the fused D2Q9 lattice-BGK step for gfx950.
//
// One launch applies Eq. 1 of arXiv 2211.05009 (Sec. 2.1) once to every
// site, in pull form: each site gathers the post-collision populations of
// its neighbours (the streaming half of Eq. 1), replaces the links that
// cross a wall by the half-way bounce-back reflection (the lid adds the
// moving-wall term -6 w rho_w c.u_w, rho_w = 1), forms rho and rho u
// (Eq. 3), relaxes toward the equilibrium of Eq. 2 with omega = 1/tau
// (Eq. 5), and stores the post-collision populations into the other buffer.
// The stored state is therefore always f*(t), the right-hand side of Eq. 1.
//
// Layout: structure of arrays, nine planes of ny rows x pitch elements,
// pitch = nx rounded up to 64, plane i at element offset i * plane.  A
// 64-lane wavefront covers 64 consecutive x of one row: every load and
// store of a plane is one contiguous 256 B (FP32) or 512 B (FP64) run.
//
// Storage variants:
//   double, SHIFT = false : f itself in FP64.
//   float,  SHIFT = true  : g = f - w in FP32.  The rest state is g = 0, so
//                           the rounding error scales with the deviation
//                           from rest instead of with w.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9 weights (Sec. 2.1, below Eq. 2).
#define LBM_W0 (4.0 / 9.0)
#define LBM_WA (1.0 / 9.0)
#define LBM_WD (1.0 / 36.0)

// Map the hardware's round-robin block -> XCD assignment (block L runs on
// XCD L % 8) onto contiguous tile ranges, so each XCD's L2 serves one band
// of rows and the rows shared by neighbouring tiles are fetched once.
__device__ __forceinline__ int xcd_tile(int L, int nb) {
  const int k = L & 7, q = nb >> 3, r = nb & 7;
  return k * q + (k < r ? k : r) + (L >> 3);
}

template <typename T>
struct StepParams {
  const T *__restrict__ src;
  T *__restrict__ dst;
  int nx, ny, pitch;
  int plane;        // elements per population plane
  int tiles_x;      // tiles along x (64 sites each)
  T omega;          // 1 / tau
  T u6;             // u_lid / 6: the moving-wall term for links 7 and 8
  T ulid = T(0);    // lid speed (non-equilibrium extrapolation walls)
};

// 1 / v for the collision: IEEE division in FP64.  In FP32 the hardware
// reciprocal estimate (within 1 ulp) refined by one Newton-Raphson step,
// r <- r + r (1 - v r): the refined value is the correctly rounded
// reciprocal but for rare last-bit ties, so u = j * (1/rho) rounds as it did
// with the division, while taking two FMAs instead of the division's ten
// instructions.  The unrefined estimate is not enough: its error has a
// sign that repeats every step and shifts FP32 steady states by ~1e-5 U.
template <typename T>
__device__ __forceinline__ T recip(T v) {
  return T(1) / v;
}
template <>
__device__ __forceinline__ float recip<float>(float v) {
  const float r = __builtin_amdgcn_rcpf(v);
  return __builtin_fmaf(__builtin_fmaf(-v, r, 1.0f), r, r);
}

// Collide one site.  f[0..8] in: populations after streaming (or their
// shift g = f - w); out: post-collision values.
//
// Eq. 2 with u = j / rho multiplied out: f^eq_i = w_i E_i with
//   E_i = b + 3 c_i.j + (4.5 (c_i.j)^2 - 1.5 j.j) / rho,
// b = rho (b = rho - 1 for the shift).  The update f_i <- f_i + omega (w_i E_i
// - f_i) is taken as f_i + (36 w_i omega / 36) (E_i - f_i / w_i): 1 / w_i is
// 9 / 4, 9 or 36 and 36 w_i / 36 is 16, 4 or 1 times omega / 36, all exact
// scalings, so no weight is ever rounded.  Rounded weights would not do in
// FP32: 4/9, 1/9 and 1/36 are powers of two times FP32(1/9), 7.5e-9 too large,
// so the equilibrium's momentum would be (1 + 7.5e-9) j and each collision
// would scale the momentum by 1 + 7.5e-9 omega, a drift of 1.4e-5 after 1000
// steps at omega near 2, far above the rounding noise of the f - w storage.
// The one rounded constant left, omega / 36, moves only the viscosity.  The
// linear term needs no division (w rho 3 c.u = 3 w c.j).
template <typename T, bool SHIFT>
__device__ __forceinline__ void bgk_collide(T (&f)[9], T omega) {
  // Eq. 3
  const T s = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  const T jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const T jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  // SHIFT: s is the density deviation rho - 1 (the weights sum to 1)
  const T rho = SHIFT ? T(1) + s : s;
  const T rinv = recip<T>(rho);
  const T b = SHIFT ? s : rho;
  const T od = omega * T(1.0 / 36.0);      // omega w_i / w_d for the diagonals
  const T oa = T(4) * od, o0 = T(16) * od;  // axis links, rest population
  const T jsq = T(1.5) * (jx * jx + jy * jy);

  f[0] += o0 * ((b - rinv * jsq) - T(2.25) * f[0]);
  {  // axis pairs (1,3) and (2,4)
    const T qx = b + rinv * (T(4.5) * jx * jx - jsq), ex = T(3) * jx;
    const T qy = b + rinv * (T(4.5) * jy * jy - jsq), ey = T(3) * jy;
    f[1] += oa * ((qx + ex) - T(9) * f[1]);
    f[3] += oa * ((qx - ex) - T(9) * f[3]);
    f[2] += oa * ((qy + ey) - T(9) * f[2]);
    f[4] += oa * ((qy - ey) - T(9) * f[4]);
  }
  {  // diagonal pairs (5,7) and (6,8)
    const T p = jx + jy, m = jy - jx;
    const T qp = b + rinv * (T(4.5) * p * p - jsq), ep = T(3) * p;
    const T qm = b + rinv * (T(4.5) * m * m - jsq), em = T(3) * m;
    f[5] += od * ((qp + ep) - T(36) * f[5]);
    f[7] += od * ((qp - ep) - T(36) * f[7]);
    f[6] += od * ((qm + em) - T(36) * f[6]);
    f[8] += od * ((qm - em) - T(36) * f[8]);
  }
}

// Gather the nine populations arriving at site (x, y) at offset o = y*pitch+x
// (streaming half of Eq. 1 plus the walls).  Links whose source lies outside
// read the reverse population of the same site; the lid row (y = ny-1) adds
// -u/6 to link 7 and +u/6 to link 8 (corner links included).
template <typename T>
__device__ __forceinline__ void pull(const T *__restrict__ s, int plane,
                                     int pitch, int o, bool xl, bool xr,
                                     bool yb, bool yt, T u6, T (&f)[9]) {
  const int P = plane;
  f[0] = s[o];
  f[1] = s[xl ? (P + o - 1) : (3 * P + o)];
  f[2] = s[yb ? (2 * P + o - pitch) : (4 * P + o)];
  f[3] = s[xr ? (3 * P + o + 1) : (P + o)];
  f[4] = s[yt ? (4 * P + o + pitch) : (2 * P + o)];
  f[5] = s[(xl && yb) ? (5 * P + o - 1 - pitch) : (7 * P + o)];
  f[6] = s[(xr && yb) ? (6 * P + o + 1 - pitch) : (8 * P + o)];
  f[7] = s[(xr && yt) ? (7 * P + o + 1 + pitch) : (5 * P + o)];
  f[8] = s[(xl && yt) ? (8 * P + o - 1 + pitch) : (6 * P + o)];
  if (!yt) {       // lid: moving-wall term, u_w = (u_lid, 0)
    f[7] -= u6;
    f[8] += u6;
  }
}

// One step over a tile of 64 x (BY * RY) sites; block = 64 x BY threads,
// each thread handles RY rows spaced BY apart.
template <typename T, bool SHIFT, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_step(StepParams<T> p) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int x = tx * 64 + threadIdx.x;
  if (x >= p.nx) return;
  const bool xl = x > 0, xr = x < p.nx - 1;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = ty * (BY * RY) + r * BY + threadIdx.y;
    if (y >= p.ny) return;
    const int o = y * p.pitch + x;
    T f[9];
    pull<T>(p.src, p.plane, p.pitch, o, xl, xr, y > 0, y < p.ny - 1, p.u6, f);
    bgk_collide<T, SHIFT>(f, p.omega);
#pragma unroll
    for (int i = 0; i < 9; ++i) p.dst[i * p.plane + o] = f[i];
  }
}

// ---------------------------------------------------------------------------
// Vector form: each thread updates V = 16 / sizeof(T) consecutive sites of a
// row with 16-byte loads and stores (four FP32 or two FP64 sites), so a
// wavefront moves 1 KiB per plane and instruction.  The loads of the planes
// that move along x start one element off a 16-byte boundary; gfx950 global
// loads need only element (dword) alignment for multi-dword accesses.
// Whole-vector wall cases depend only on the row; the side walls touch only
// the first / last element and are patched from the reverse plane.  The
// per-site arithmetic is bgk_collide, as in k_step.
template <typename T, int V>
struct VecT {            // alignment of T only
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ void vload(const T *p, T (&out)[V]) {
  VecT<T, V> t;
  __builtin_memcpy(&t, p, sizeof t);
#pragma unroll
  for (int k = 0; k < V; ++k) out[k] = t.v[k];
}

template <typename T, int V>
__device__ __forceinline__ void vstore(T *p, const T (&in)[V]) {
  VecT<T, V> t;
#pragma unroll
  for (int k = 0; k < V; ++k) t.v[k] = in[k];
  __builtin_memcpy(p, &t, sizeof t);
}

// Update the V sites (x0 .. x0+V-1, y) of one thread; x0 < nx, y < ny.
template <typename T, bool SHIFT, int V>
__device__ __forceinline__ void step_vec_sites(const T *__restrict__ s, T *__restrict__ d,
                                               int P, int pitch, int nx, int ny, int x0,
                                               int y, T omega, T u6) {
  const bool yb = y > 0, yt = y < ny - 1;
  if (x0 + V > nx) {            // ragged end of the row: one site at a time
    for (int k = 0; k < V && x0 + k < nx; ++k) {
      const int x = x0 + k, o = y * pitch + x;
      T f[9];
      pull<T>(s, P, pitch, o, x > 0, x < nx - 1, yb, yt, u6, f);
      bgk_collide<T, SHIFT>(f, omega);
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i * P + o] = f[i];
    }
    return;
  }
  const int o = y * pitch + x0;
  T g[9][V];
  vload<T, V>(s + o, g[0]);
  vload<T, V>(s + P + o - 1, g[1]);
  vload<T, V>(s + 3 * P + o + 1, g[3]);
  vload<T, V>(s + (yb ? 2 * P + o - pitch : 4 * P + o), g[2]);
  vload<T, V>(s + (yt ? 4 * P + o + pitch : 2 * P + o), g[4]);
  vload<T, V>(s + (yb ? 5 * P + o - pitch - 1 : 7 * P + o), g[5]);
  vload<T, V>(s + (yb ? 6 * P + o - pitch + 1 : 8 * P + o), g[6]);
  vload<T, V>(s + (yt ? 7 * P + o + pitch + 1 : 5 * P + o), g[7]);
  vload<T, V>(s + (yt ? 8 * P + o + pitch - 1 : 6 * P + o), g[8]);
  if (!yt) {                    // lid row: moving-wall term on 7 and 8
#pragma unroll
    for (int k = 0; k < V; ++k) {
      g[7][k] -= u6;
      g[8][k] += u6;
    }
  }
  if (x0 == 0) {                // left wall: links arriving with c_x = +1
    g[1][0] = s[3 * P + o];
    if (yb) g[5][0] = s[7 * P + o];
    if (yt) g[8][0] = s[6 * P + o];
  }
  if (x0 + V == nx) {           // right wall: links arriving with c_x = -1
    const int oe = o + V - 1;
    g[3][V - 1] = s[P + oe];
    if (yb) g[6][V - 1] = s[8 * P + oe];
    if (yt) g[7][V - 1] = s[5 * P + oe];
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = g[i][k];
    bgk_collide<T, SHIFT>(f, omega);
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i][k] = f[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) vstore<T, V>(d + i * P + o, g[i]);
}

// One step over tiles of (64 V) x BY sites; block = 64 x BY threads.
template <typename T, bool SHIFT, int BY>
__global__ __launch_bounds__(64 * BY) void k_step_vec(StepParams<T> p) {
  constexpr int V = 16 / sizeof(T);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int x0 = (tx * 64 + threadIdx.x) * V;
  const int y = ty * BY + threadIdx.y;
  if (x0 >= p.nx || y >= p.ny) return;
  step_vec_sites<T, SHIFT, V>(p.src, p.dst, p.plane, p.pitch, p.nx, p.ny, x0, y, p.omega,
                              p.u6);
}

}  // namespace lbm
