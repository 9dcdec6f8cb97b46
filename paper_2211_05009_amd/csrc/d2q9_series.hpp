// d2q9_series.hpp -- flow state of probe time series (the stable / periodic /
// aperiodic states of Sec. 3.3 and the periods of Table 3).
//
// One block of kSeriesThreads threads per series.  Definition (the library
// documents it with lbm_classify_series):
//   amplitude A = max - min; steady if A <= steady_tol;
//   D(T) = mean_{k < n-T} (u[k+T] - u[k])^2 / sigma^2 for T in
//   [min_lag, max_lag]; candidates are interior local minima of D reached
//   after D exceeded 1; the parabola through D at T-1, T, T+1 refines the
//   period (vertex) and gives the mismatch sqrt(max(vertex value, 0));
//   periodic at the first candidate with mismatch <= periodic_tol; a drift
//   if there is no candidate; aperiodic otherwise.
// Every sum runs in a fixed order (per-thread sequential sums, then a fixed
// LDS tree), so the result does not depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {

constexpr int kSeriesThreads = 256;

// Sample k of a series lives at base[((start + k) % cap) * stride]: a ring
// of records (cap = n, start = 0 for a plain strided array).
struct SeriesDesc {
  const double *base;
  long long cap, start, n, stride;
};

struct SeriesOut {
  double period, amplitude, mean, std, mismatch, cycle, cycle_mismatch;
  int state, lag;
};

// Fixed-order block sum / min / max of one value per thread.
__device__ __forceinline__ void series_reduce(double &sum, double &mn, double &mx, double *s0,
                                              double *s1, double *s2) {
  const int t = threadIdx.x;
  s0[t] = sum;
  s1[t] = mn;
  s2[t] = mx;
  __syncthreads();
  for (int h = kSeriesThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      s0[t] += s0[t + h];
      s1[t] = fmin(s1[t], s1[t + h]);
      s2[t] = fmax(s2[t], s2[t + h]);
    }
    __syncthreads();
  }
  sum = s0[0];
  mn = s1[0];
  mx = s2[0];
  __syncthreads();
}

// One block classifies series d; u: n + (number of lags) doubles of scratch
// (the unwrapped series, then the D values of lags min_lag .. max_lag).
// Returns true on thread 0, which holds the result in r; the other threads
// return false.
__device__ __forceinline__ bool classify_block(const SeriesDesc &d, double steady_tol,
                                               double periodic_tol, int min_lag,
                                               int max_lag_req, double *__restrict__ u,
                                               SeriesOut &r) {
  __shared__ double s0[kSeriesThreads], s1[kSeriesThreads], s2[kSeriesThreads];
  const long long n = d.n;
  for (long long k = threadIdx.x; k < n; k += kSeriesThreads)
    u[k] = d.base[((d.start + k) % d.cap) * d.stride];
  __syncthreads();
  // mean, min, max
  double sum = 0.0, mn = INFINITY, mx = -INFINITY;
  for (long long k = threadIdx.x; k < n; k += kSeriesThreads) {
    sum += u[k];
    mn = fmin(mn, u[k]);
    mx = fmax(mx, u[k]);
  }
  series_reduce(sum, mn, mx, s0, s1, s2);
  const double mean = sum / (double)n;
  // variance about the mean (two passes, like the population std)
  double ss = 0.0, dummy0 = 0.0, dummy1 = 0.0;
  for (long long k = threadIdx.x; k < n; k += kSeriesThreads) {
    const double e = u[k] - mean;
    ss += e * e;
  }
  series_reduce(ss, dummy0, dummy1, s0, s1, s2);
  const double sd = sqrt(ss / (double)n);
  const double amp = mx - mn;
  r.period = 0.0;
  r.amplitude = amp;
  r.mean = mean;
  r.std = sd;
  r.mismatch = 0.0;
  r.cycle = 0.0;
  r.cycle_mismatch = 0.0;
  r.state = 0;
  r.lag = 0;
  if (amp <= steady_tol) return threadIdx.x == 0;
  long long max_lag = max_lag_req > 0 ? max_lag_req : n / 3;
  if (max_lag > n - 2) max_lag = n - 2;
  const long long nlags = max_lag - min_lag + 1;
  double *D = u + n;
  const double inv_var = 1.0 / (sd * sd);
  for (long long j = threadIdx.x; j < nlags; j += kSeriesThreads) {
    const long long T = min_lag + j;
    double acc = 0.0;
    for (long long k = 0; k + T < n; ++k) {
      const double e = u[k + T] - u[k];
      acc += e * e;
    }
    D[j] = acc / (double)(n - T) * inv_var;
  }
  __syncthreads();
  if (threadIdx.x != 0) return false;
  double best = INFINITY;
  bool decorrelated = false;
  r.state = 2;
  for (long long j = 1; j + 1 < nlags; ++j) {
    decorrelated = decorrelated || D[j - 1] > 1.0;
    if (!(decorrelated && D[j - 1] > D[j] && D[j] <= D[j + 1])) continue;
    const double curv = D[j - 1] - 2.0 * D[j] + D[j + 1];
    double period = (double)(min_lag + j), vertex = D[j];
    if (curv > 0.0) {
      period += 0.5 * (D[j - 1] - D[j + 1]) / curv;
      vertex = D[j] - (D[j - 1] - D[j + 1]) * (D[j - 1] - D[j + 1]) / (8.0 * curv);
    }
    const double mis = sqrt(fmax(vertex, 0.0));
    if (best == INFINITY) {   // the first return: the dominant cycle
      r.cycle = period;
      r.cycle_mismatch = mis;
    }
    best = fmin(best, mis);
    if (mis <= periodic_tol) {
      r.state = 1;
      r.lag = (int)(min_lag + j);
      r.period = period;
      r.mismatch = mis;
      return true;
    }
  }
  r.mismatch = best;
  if (best == INFINITY) {   // no return within the window: a drift
    r.state = 3;
    r.cycle_mismatch = INFINITY;
  }
  return true;
}

// Series described by desc[]; work_stride doubles of scratch per series.
static __global__ __launch_bounds__(kSeriesThreads) void k_classify_series(
    const SeriesDesc *__restrict__ desc, double steady_tol, double periodic_tol, int min_lag,
    int max_lag_req, double *__restrict__ work, long long work_stride,
    SeriesOut *__restrict__ out) {
  SeriesOut r;
  if (classify_block(desc[blockIdx.x], steady_tol, periodic_tol, min_lag, max_lag_req,
                     work + (long long)blockIdx.x * work_stride, r))
    out[blockIdx.x] = r;
}

// Plain strided series: series s at series + s * ld, n samples; the result
// of series s goes to out[s] in the ABI's record layout (OutRec: the fields
// of lbm_flow_state_t).
template <typename OutRec>
__global__ __launch_bounds__(kSeriesThreads) void k_classify_strided(
    const double *__restrict__ series, long long n, long long ld, double steady_tol,
    double periodic_tol, int min_lag, int max_lag_req, double *__restrict__ work,
    long long work_stride, OutRec *__restrict__ out) {
  const SeriesDesc d{series + (long long)blockIdx.x * ld, n, 0, n, 1};
  SeriesOut r;
  if (classify_block(d, steady_tol, periodic_tol, min_lag, max_lag_req,
                     work + (long long)blockIdx.x * work_stride, r)) {
    OutRec o;
    o.state = r.state;
    o.lag = r.lag;
    o.period = r.period;
    o.amplitude = r.amplitude;
    o.mean = r.mean;
    o.std = r.std;
    o.mismatch = r.mismatch;
    o.cycle = r.cycle;
    o.cycle_mismatch = r.cycle_mismatch;
    out[blockIdx.x] = o;
  }
}

}  // namespace lbm
