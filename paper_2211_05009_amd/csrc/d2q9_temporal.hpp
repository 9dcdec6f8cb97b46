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

#include "d2q9_monitor.hpp"
#include "d2q9_step.hpp"

namespace lbm {

// The Eq. 6 monitor of the state a chunk starts from, carried by the chunk's
// first two launches instead of a separate pass.  The first launch (MON = 1)
// takes the per-site FP64 sums of k_monitor (sum (rho - 1), sum |u -
// u_ref|^2, sum |u_ref|^2, then u_ref <- u) over each block's core sites
// and stores one triple of partials per block: each thread loads its core
// sites' nine start-state values and u_ref entries together with step 1's
// pulls (from the same cache lines; after the steps where they would take
// too many registers), runs the K steps like any launch, and takes the sums
// at the end (the launch writes the other buffer, so the start state is
// intact).  The second launch (MON = 2, same grid) adds the partials in
// block order in the block of the last tile (deterministic) and writes
// out[3]; the kernel boundary between the two makes them visible, so no
// block waits on another.
struct TbMonitor {
  double2 *uref;      // dense [ny][nx] reference velocity
  double *partials;   // [gridDim.x][3]
  double *out;        // [3]
};

// One block's share of that monitor: the reference field of its cavity, the
// triple of partials it stores (MON = 1) and, on the block that completes a
// cavity's sum (MON = 2), that cavity's nfin partials in the order they are
// added and the triple they go to.  nfin is 0 on every other block.
struct TbMonBlock {
  double2 *uref;
  double *part;
  const double *fin;
  int nfin;
  double *out;
};

// Sum N values over an NT-thread block; thread 0 writes out[N].
template <int NT, int N>
__device__ __forceinline__ void block_sum_nt(double (&v)[N], double *out) {
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  __shared__ double part[NT / 64][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = 0.0;
      for (int w = 0; w < NT / 64; ++w) a += part[w][k];
      out[k] = a;
    }
  }
}

// Core-site test and dense index of region site q (the sites a block's
// monitor covers).
template <int K, int TX, int TY>
__device__ __forceinline__ bool tb_core(int q, int X0, int Y0, int nx, int ny, int &k) {
  constexpr int RW = TX + 2 * K;
  const int ry = q / RW, rx = q - ry * RW;
  const int gx = X0 + rx, gy = Y0 + ry;
  k = gy * nx + gx;
  return rx >= K && rx < K + TX && ry >= K && ry < K + TY && gx < nx && gy < ny;
}

// The monitor sums of a block's core sites from their start-state values
// fv[j] (region site q = threadIdx.x + j NT; cr[j]: a core site, dense
// index kd[j]) and u_ref entries ur[j].
template <typename T, bool SHIFT, int J, int NT>
__device__ __forceinline__ void tb_monitor_sums(const T (&fv)[J][9], const double2 (&ur)[J],
                                                const bool (&cr)[J], const int (&kd)[J],
                                                const TbMonBlock &m) {
  double acc[kNumSums] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (cr[j]) {
      double drho, jx, jy;
      moments_of<T, SHIFT>(fv[j], drho, jx, jy);
      const double rho = 1.0 + drho;
      const double ux = jx / rho, uy = jy / rho;
      const double dx = ux - ur[j].x, dy = uy - ur[j].y;
      acc[0] += drho;
      acc[1] += dx * dx + dy * dy;
      acc[2] += ur[j].x * ur[j].x + ur[j].y * ur[j].y;
      m.uref[kd[j]] = make_double2(ux, uy);
    }
  }
  block_sum_nt<NT, kNumSums>(acc, m.part);
}

// The same sums from the start state loaded into LDS (region layout), u_ref
// entries ur[j] prefetched.
template <typename T, bool SHIFT, int K, int TX, int TY, int NT>
__device__ __forceinline__ void tb_monitor_sums_lds(const T *lds, int X0, int Y0, int nx, int ny,
                                                const TbMonBlock &m,
                                                const double2 (&ur)[(
                                                    (TX + 2 * K) * (TY + 2 * K) + NT - 1) / NT]) {
  constexpr int RS = (TX + 2 * K) * (TY + 2 * K);
  constexpr int J = (RS + NT - 1) / NT;
  double acc[kNumSums] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int q = threadIdx.x + j * NT;
    int k;
    if (q < RS && tb_core<K, TX, TY>(q, X0, Y0, nx, ny, k)) {
      double drho, jx, jy;
      site_moments<T, SHIFT>(lds, RS, q, drho, jx, jy);
      const double rho = 1.0 + drho;
      const double ux = jx / rho, uy = jy / rho;
      const double dx = ux - ur[j].x, dy = uy - ur[j].y;
      acc[0] += drho;
      acc[1] += dx * dx + dy * dy;
      acc[2] += ur[j].x * ur[j].x + ur[j].y * ur[j].y;
      m.uref[k] = make_double2(ux, uy);
    }
  }
  block_sum_nt<NT, kNumSums>(acc, m.part);
}

// K steps on the region in LDS; the valid window shrinks by one site per
// side and step.  At step s the threads take the sites of that window,
// (RW - 2s) x (RH - 2s) of them, in row-major order, so a wavefront holds 64
// sites of the window rather than 64 sites of the region of which a shrinking
// share is idle; the step loop is unrolled, so the window width is a
// compile-time constant in the index arithmetic.  The last window is the
// tile's core: its sites go from registers straight to dst (pitch, plane
// stride P), with no write-back to LDS and no barrier after it.
// Steps S0 ... K (S0 = 2 after tb_first_step).
// PP: two LDS buffers (lds, lds + 9 RS) taken in turn, so a step reads one
// and writes the other and one barrier per step suffices; otherwise one
// buffer, read and then overwritten between two barriers (half the LDS, so
// more blocks fit a CU).  NTS: the last step's stores are non-temporal: the
// next launch reads them from the Infinity Cache or HBM, not from this L2,
// and streaming them leaves less dirty data in L2 at the kernel boundary
// (+4 % at 500 x 500, +8 % at 500 x 1000, +1.5 % at 4096^2 FP32, measured).
template <typename T, bool SHIFT, int K, int RW, int RH, int NT, int S0, bool INTERIOR,
          bool PP = false, bool NTS = true>
__device__ __forceinline__ void tb_steps(T *lds_in, T *__restrict__ dst, int pitch, int P,
                                         int X0, int Y0, int nx, int ny, T omega, T u6) {
  constexpr int RS = RW * RH;
  constexpr int JM = ((RW - 2) * (RH - 2) + NT - 1) / NT;   // sites per thread at s = 1
  T *lds = lds_in;
#pragma unroll
  for (int s = S0; s <= K; ++s) {
    T *out = PP ? (lds == lds_in ? lds_in + 9 * RS : lds_in) : lds;
    const int ws = RW - 2 * s, ns = ws * (RH - 2 * s);
    T v[JM][9];
    bool act[JM];
    int qs[JM], go[JM];
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      const int c = threadIdx.x + j * NT;
      const int wy = c / ws, wx = c - wy * ws;
      const int rx = s + wx, ry = s + wy;
      const int q = ry * RW + rx;
      const int gx = X0 + rx, gy = Y0 + ry;
      qs[j] = q;
      go[j] = gy * pitch + gx;
      act[j] = c < ns;
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
    if (s == K) {
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (act[j])
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            if (NTS)
              __builtin_nontemporal_store(v[j][i], dst + i * P + go[j]);
            else
              dst[i * P + go[j]] = v[j][i];
          }
    } else {
      if (!PP) __syncthreads();
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (act[j])
#pragma unroll
          for (int i = 0; i < 9; ++i) out[i * RS + qs[j]] = v[j][i];
      __syncthreads();
      lds = out;
    }
  }
}

// Step 1 without the region in LDS: each site of the first window,
// (RW - 2) x (RH - 2) in row-major order, pulls its nine populations from
// global memory exactly as k_step does (pull; the +-1 neighbours come from
// L1 / L2), collides, and leaves the result in LDS for step 2.  No load
// phase and no barrier precede the first collision: a wavefront computes as
// soon as its own loads arrive.
template <typename T, bool SHIFT, int K, int RW, int RH, int NT, bool INTERIOR>
__device__ __forceinline__ void tb_first_step(T *lds, const T *__restrict__ src, int pitch,
                                              int P, int X0, int Y0, int nx, int ny, T omega,
                                              T u6) {
  constexpr int RS = RW * RH, W1 = RW - 2, N1 = W1 * (RH - 2);
  constexpr int JM = (N1 + NT - 1) / NT;
  T v[JM][9];
  bool act[JM];
  int qs[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) {
    const int c = threadIdx.x + j * NT;
    const int wy = c / W1, wx = c - wy * W1;
    const int rx = 1 + wx, ry = 1 + wy;
    const int gx = X0 + rx, gy = Y0 + ry;
    qs[j] = ry * RW + rx;
    act[j] = c < N1;
    if (!INTERIOR) act[j] = act[j] && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    if (act[j]) {
      // an interior region keeps the first window one site away from every wall
      if (INTERIOR)
        pull<T>(src, P, pitch, gy * pitch + gx, true, true, true, true, u6, v[j]);
      else
        pull<T>(src, P, pitch, gy * pitch + gx, gx > 0, gx < nx - 1, gy > 0, gy < ny - 1, u6,
                v[j]);
      bgk_collide<T, SHIFT>(v[j], omega);
    }
  }
#pragma unroll
  for (int j = 0; j < JM; ++j)
    if (act[j])
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * RS + qs[j]] = v[j][i];
  __syncthreads();
}

// One tile (tile_x, tile_y) of TX x TY core sites advanced K steps; src and
// dst point at plane 0 of the cavity.
// MON: 0, or 1 / 2 for the first / second launch of a monitored chunk.
// MON = 1 takes the monitor sums of the start state.  Where a thread's core
// sites fit in 18 registers (PRE) it loads their nine values and u_ref
// entries with step 1's pulls (the same cache lines), runs the steps like
// any launch and takes the sums at the end (the launch writes the other
// buffer, so the start state is intact).  Otherwise (or with MON_LDS) it
// loads the whole region into LDS first, takes the sums from there and runs
// step 1 out of LDS, so that a lattice beyond the caches is still read once
// and the u_ref traffic comes before the steps rather than after them.
template <typename T, bool SHIFT, int K, int TX, int TY, int NT, int MON, bool PP = false,
          bool NTS = true, bool MON_LDS = false>
__device__ __forceinline__ void tb_tile(T *lds, const T *__restrict__ src, T *__restrict__ dst,
                                        int nx, int ny, int pitch, int P, T omega, T u6,
                                        int tile_x, int tile_y, const TbMonBlock &mon) {
  constexpr int RW = TX + 2 * K, RH = TY + 2 * K, RS = RW * RH;
  constexpr int J = (RS + NT - 1) / NT;       // region sites per thread
  static_assert(K >= 2, "the first and the last step take separate paths");
  const int X0 = tile_x * TX - K;             // global x of region column 0
  const int Y0 = tile_y * TY - K;

  constexpr bool PRE = !MON_LDS && J * 9 * (int)(sizeof(T) / 4) <= 18;
  constexpr int JM = MON == 1 ? J : 1;
  T fv[PRE ? JM : 1][9];
  double2 ur[JM];
  bool cr[JM];
  int kd[JM];
  double fin[kNumSums] = {0.0, 0.0, 0.0};
  if (MON == 1) {
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      const int q = threadIdx.x + j * NT;
      cr[j] = q < RS && tb_core<K, TX, TY>(q, X0, Y0, nx, ny, kd[j]);
      ur[j] = cr[j] ? mon.uref[kd[j]] : make_double2(0.0, 0.0);
      if constexpr (PRE) {
        if (cr[j]) {
          const int ry = q / RW, o = (Y0 + ry) * pitch + X0 + (q - ry * RW);
#pragma unroll
          for (int i = 0; i < 9; ++i) fv[j][i] = src[i * P + o];
        }
      }
    }
  }
  if (MON == 2 && threadIdx.x < mon.nfin) {
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) fin[k] = mon.fin[threadIdx.x * kNumSums + k];
  }
  if (MON == 2 && mon.nfin > 0) {
    for (int b = threadIdx.x + NT; b < mon.nfin; b += NT)
#pragma unroll
      for (int k = 0; k < kNumSums; ++k) fin[k] += mon.fin[b * kNumSums + k];
    block_sum_nt<NT, kNumSums>(fin, mon.out);
  }

  // Tiles whose region lies inside the cavity (no wall within reach) take a
  // branch-free pull with constant offsets; the rest test the walls.  The
  // last step stores the core.
  const bool interior = X0 >= 0 && X0 + RW <= nx && Y0 >= 0 && Y0 + RH <= ny;
  if constexpr (MON != 1 || PRE) {
    if (interior) {
      tb_first_step<T, SHIFT, K, RW, RH, NT, true>(lds, src, pitch, P, X0, Y0, nx, ny, omega, u6);
      tb_steps<T, SHIFT, K, RW, RH, NT, 2, true, PP, NTS>(lds, dst, pitch, P, X0, Y0, nx, ny,
                                                          omega, u6);
    } else {
      tb_first_step<T, SHIFT, K, RW, RH, NT, false>(lds, src, pitch, P, X0, Y0, nx, ny, omega,
                                                    u6);
      tb_steps<T, SHIFT, K, RW, RH, NT, 2, false, PP, NTS>(lds, dst, pitch, P, X0, Y0, nx, ny,
                                                           omega, u6);
    }
    if constexpr (MON == 1) tb_monitor_sums<T, SHIFT, JM, NT>(fv, ur, cr, kd, mon);
  } else {
    // Load the region (sites inside the cavity) straight from global memory
    // into LDS: global_load_lds_dword writes lane l's word at the wavefront's
    // LDS base + 4 l, with no round trip through registers and no LDS stores.
    // Thread c takes word c of each plane's region: site c in FP32, the low
    // (c even) or high half of site c / 2 in FP64, so the 64 lanes of a
    // wavefront fill 64 consecutive LDS words.
    constexpr int WPS = sizeof(T) / 4;             // words per site
    constexpr int JW = (WPS * RS + NT - 1) / NT;   // words per thread and plane
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      const int c = threadIdx.x + j * NT;
      const int q = c / WPS;
      if (q < RS) {
        const int ry = q / RW, rx = q - ry * RW;
        const int gx = X0 + rx, gy = Y0 + ry;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
          const float *g = reinterpret_cast<const float *>(src + gy * pitch + gx) + c % WPS;
          float *w0 = reinterpret_cast<float *>(lds) + (c - (threadIdx.x & 63));
#pragma unroll
          for (int i = 0; i < 9; ++i)
            __builtin_amdgcn_global_load_lds(g + WPS * i * P, w0 + WPS * i * RS, 4, 0, 0);
        }
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    tb_monitor_sums_lds<T, SHIFT, K, TX, TY, NT>(lds, X0, Y0, nx, ny, mon, ur);
    if (interior)
      tb_steps<T, SHIFT, K, RW, RH, NT, 1, true, PP, NTS>(lds, dst, pitch, P, X0, Y0, nx, ny, omega,
                                                         u6);
    else
      tb_steps<T, SHIFT, K, RW, RH, NT, 1, false, PP, NTS>(lds, dst, pitch, P, X0, Y0, nx, ny,
                                                          omega, u6);
  }
}

// MON: 1 / 2 for the first / second launch of a chunk that carries the
// monitor of its start state (see TbMonitor), else 0.
template <typename T, bool SHIFT, int K, int TX, int TY, int NT, int MON = 0, bool PP = false,
          bool NTS = true>
__global__ __launch_bounds__(NT) void k_step_tb(StepParams<T> p, int tiles_x, TbMonitor mon) {
  __shared__ T lds[(PP ? 18 : 9) * (TX + 2 * K) * (TY + 2 * K)];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  // block b stores partial triple b; the block of the last tile (a ragged
  // edge tile where the lattice is not a multiple of the tile: less work to
  // hide the sum behind) adds all of them, in block order
  const TbMonBlock mb{mon.uref, mon.partials + blockIdx.x * kNumSums, mon.partials,
                      tile == (int)gridDim.x - 1 ? (int)gridDim.x : 0, mon.out};
  tb_tile<T, SHIFT, K, TX, TY, NT, MON, PP, NTS>(lds, p.src, p.dst, p.nx, p.ny, p.pitch, p.plane,
                                        p.omega, p.u6, tile % tiles_x, tile / tiles_x, mb);
}

}  // namespace lbm
