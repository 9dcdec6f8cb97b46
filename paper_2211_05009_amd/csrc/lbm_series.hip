// lbm_series.hip -- flow-state classification of time series on the device
// (d2q9_series.hpp): lbm_classify_series and the shared launcher used by
// the probe-series entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/lbm.h"
#include "d2q9_series.hpp"
#include "lbm_internal.h"

using namespace lbm;

int classify_series_descs(const SeriesDesc *descs_host, int nseries, long long n_max,
                          double steady_tol, double periodic_tol, int min_lag, int max_lag,
                          hipStream_t st, lbm_flow_state_t *out_host) {
  if (nseries <= 0) return LBM_OK;
  // lags per series are at most n_max / 3 (or max_lag) -- room for n_max
  const long long stride = 2 * n_max + 8;
  SeriesDesc *d_desc = nullptr;
  double *d_work = nullptr;
  SeriesOut *d_out = nullptr;
  int rc = LBM_OK;
  hipError_t e = hipMalloc(&d_desc, sizeof(SeriesDesc) * nseries);
  if (e == hipSuccess) e = hipMalloc(&d_work, sizeof(double) * stride * nseries);
  if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(SeriesOut) * nseries);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_desc, descs_host, sizeof(SeriesDesc) * nseries,
                       hipMemcpyHostToDevice, st);
  std::vector<SeriesOut> res(nseries);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_classify_series, dim3(nseries), dim3(kSeriesThreads), 0, st, d_desc,
                       steady_tol, periodic_tol, min_lag, max_lag, d_work, stride, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(res.data(), d_out, sizeof(SeriesOut) * nseries, hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    rc = lbm_fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "classify: %s",
                  hipGetErrorString(e));
  if (d_desc) (void)hipFree(d_desc);
  if (d_work) (void)hipFree(d_work);
  if (d_out) (void)hipFree(d_out);
  if (rc) return rc;
  for (int s = 0; s < nseries; ++s) {
    lbm_flow_state_t &o = out_host[s];
    o.state = res[s].state;
    o.lag = res[s].lag;
    o.period = res[s].period;
    o.amplitude = res[s].amplitude;
    o.mean = res[s].mean;
    o.std = res[s].std;
    o.mismatch = res[s].mismatch;
    o.cycle = res[s].cycle;
    o.cycle_mismatch = res[s].cycle_mismatch;
  }
  return LBM_OK;
}

// Lag range check shared by the entry points.
int check_lags(long long n, int min_lag, int max_lag) {
  if (n < 8) return lbm_fail(LBM_EINVAL, "n = %lld < 8 samples", n);
  if (min_lag < 1) return lbm_fail(LBM_EINVAL, "min_lag = %d < 1", min_lag);
  long long hi = max_lag > 0 ? max_lag : n / 3;
  hi = std::min(hi, n - 2);
  if (hi - min_lag + 1 < 3)
    return lbm_fail(LBM_EINVAL, "lag range [%d, %lld] holds fewer than 3 lags", min_lag, hi);
  return LBM_OK;
}

int lbm_classify_series(const double *series_dev, int nseries, int64_t n, int64_t ld,
                        double steady_tol, double periodic_tol, int min_lag, int max_lag,
                        lbm_flow_state_t *out_host, void *hip_stream) {
  if (!series_dev || !out_host) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (nseries < 1) return lbm_fail(LBM_EINVAL, "nseries = %d < 1", nseries);
  if (ld < n) return lbm_fail(LBM_EINVAL, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (!(steady_tol >= 0.0) || !(periodic_tol >= 0.0))
    return lbm_fail(LBM_EINVAL, "tolerances must be >= 0 (steady %g, periodic %g)", steady_tol,
                    periodic_tol);
  int rc = check_lags(n, min_lag, max_lag);
  if (rc) return rc;
  std::vector<SeriesDesc> d(nseries);
  for (int s = 0; s < nseries; ++s) d[s] = SeriesDesc{series_dev + (long long)s * ld, n, 0, n, 1};
  return classify_series_descs(d.data(), nseries, n, steady_tol, periodic_tol, min_lag, max_lag,
                               (hipStream_t)hip_stream, out_host);
}

// ------------------------------------------------ no-allocation classifier
// Work memory of lbm_classify_series_noalloc: one array per device, held
// from the library's load until the process ends.  Host code never uses the
// name `scratch` as an address (in host code it is a stand-in, not device
// memory): each device's address comes from hipGetSymbolAddress, taken once
// per device on that entry point's first call there.
constexpr long long kNoAllocScratchDoubles = 4LL << 20;   // 32 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr and an
// error message on failure).
static double *scratch_for_current_device(int &rc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    rc = lbm_fail(LBM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    rc = lbm_fail(LBM_EDEVICE, "device %d beyond the %d this entry point supports", dev,
                  kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      rc = lbm_fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                    hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  rc = LBM_OK;
  return g_scratch_ptr[dev];
}

int lbm_classify_series_noalloc(const double *series_dev, int nseries, int64_t n, int64_t ld,
                                double steady_tol, double periodic_tol, int min_lag,
                                int max_lag, lbm_flow_state_t *out_dev, void *hip_stream) {
  if (!series_dev || !out_dev) return lbm_fail(LBM_EINVAL, "NULL argument");
  if (nseries < 1) return lbm_fail(LBM_EINVAL, "nseries = %d < 1", nseries);
  if (ld < n) return lbm_fail(LBM_EINVAL, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (!(steady_tol >= 0.0) || !(periodic_tol >= 0.0))
    return lbm_fail(LBM_EINVAL, "tolerances must be >= 0 (steady %g, periodic %g)", steady_tol,
                    periodic_tol);
  int rc = check_lags(n, min_lag, max_lag);
  if (rc) return rc;
  // the same work layout as lbm_classify_series: the series, then its lags
  const long long stride = 2 * (long long)n + 8;
  if ((long long)nseries > kNoAllocScratchDoubles / stride)
    return lbm_fail(LBM_EINVAL,
                    "nseries * (2 n + 8) = %d * %lld doubles exceeds the %lld-double (32 MiB) "
                    "work array of the no-allocation classifier; classify fewer or shorter "
                    "series per call",
                    nseries, stride, kNoAllocScratchDoubles);
  double *work = scratch_for_current_device(rc);
  if (!work) return rc;
  hipLaunchKernelGGL(k_classify_strided<lbm_flow_state_t>, dim3(nseries), dim3(kSeriesThreads), 0,
                     (hipStream_t)hip_stream, series_dev, (long long)n, (long long)ld, steady_tol,
                     periodic_tol, min_lag, max_lag, work, stride, out_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "classify launch: %s", hipGetErrorString(e));
  return LBM_OK;
}
