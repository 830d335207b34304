// autotune.hip -- choice of the grid's cell edge by measurement.
//
// The neighbour search is the dominant kernel and its cost depends on the
// finest cell edge (in units of h): too small and the search reaches into
// coarser levels or many cells, too large and every block holds too many
// candidates. The best factor depends on k, on the surface's local dimension
// and on the density spread, so it is measured: the grid is built with each
// candidate edge and the search stage is timed over a sample of the points:
// runs of 256 consecutive points of the grid's Morton order, one run in
// every 256 x stride, so that the sampled queries meet the same block reuse
// as a search over the whole cloud (a strided sample of the caller's order
// spreads its queries stride times thinner and favours larger cells). Uses
// the public entry points plus one sampling kernel.
#include <math.h>
#include <stdlib.h>

#include <vector>

#include "grid_access.h"
#include "mls_internal.h"

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int64_t kRun = 256;  // consecutive sorted points per sample run

// Sample t of cloud c (soff[c] <= t < soff[c + 1]), i = t - soff[c]: the
// sorted point at run i / kRun (one run every kRun * stride of the cloud's
// finite points, wrapping at the end) and offset i % kRun; NaN for a cloud
// without finite points.
__global__ void k_run_sample(const float4 *__restrict__ spts, const mls::CloudDev *__restrict__ clouds,
                             const int64_t *__restrict__ soff, int32_t n_clouds, int32_t stride,
                             int64_t m, float *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  int32_t lo = 0, hi = n_clouds - 1;
  while (lo < hi) {  // last cloud whose sample range starts at or before t
    const int32_t mid = (lo + hi + 1) >> 1;
    if (soff[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const mls::CloudDev &cd = clouds[lo];
  const int64_t fin = cd.send - cd.sbegin;
  float x = __int_as_float(0x7fc00000), y = x, z = x;
  if (fin > 0) {
    const int64_t i = t - soff[lo];
    const int64_t pos = cd.sbegin + ((i / kRun) * kRun * (int64_t)stride + i % kRun) % fin;
    const float4 P = spts[pos];
    x = P.x; y = P.y; z = P.z;
  }
  out[3 * t + 0] = x;
  out[3 * t + 1] = y;
  out[3 * t + 2] = z;
}

struct TuneLayout {
  size_t grid, sample, soff, proj, total;
};

TuneLayout tune_layout(int64_t n_points, int32_t n_clouds, int32_t k, int64_t m) {
  TuneLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.grid = take(mls_grid_workspace_bytes(n_points, n_clouds));
  L.sample = take(12 * (size_t)m);
  L.soff = take(8 * ((size_t)n_clouds + 1));
  L.proj = take(mls::proj_workspace_bytes(n_clouds, k, m));
  L.total = o;
  return L;
}

int64_t sample_bound(int64_t n_points, int32_t n_clouds, int32_t stride) {
  return n_points / stride + n_clouds;
}

}  // namespace

extern "C" {

size_t mls_autotune_workspace_bytes(int64_t n_points, int32_t n_clouds, int32_t k,
                                    int32_t stride) {
  if (n_points < 1 || n_clouds < 1 || k < 1 || k > MLS_MAX_K || stride < 1) return 0;
  return tune_layout(n_points, n_clouds, k, sample_bound(n_points, n_clouds, stride)).total;
}

mls_status mls_autotune_cell(const float *points, int64_t n_points, const int64_t *cloud_offsets,
                             int32_t n_clouds, const double *h, int32_t k,
                             const double *candidates, int32_t n_candidates, int32_t stride,
                             void *workspace, size_t workspace_bytes, void *stream,
                             double *best_factor, float *ms_per_candidate) {
  if (!points || !h || !candidates || !workspace || !best_factor || n_points < 1 ||
      n_clouds < 1 || k < 1 || k > MLS_MAX_K || n_candidates < 1 || stride < 1)
    return MLS_ERR_INVALID_ARGUMENT;
  if (n_clouds > 1 && !cloud_offsets) return MLS_ERR_INVALID_ARGUMENT;
  for (int32_t i = 0; i < n_candidates; ++i)
    if (!(candidates[i] > 0.0) || !isfinite(candidates[i])) return MLS_ERR_INVALID_ARGUMENT;
  if (((uintptr_t)workspace & 255) != 0) return MLS_ERR_INVALID_ARGUMENT;
  const int64_t m_bound = sample_bound(n_points, n_clouds, stride);
  const TuneLayout L = tune_layout(n_points, n_clouds, k, m_bound);
  if (workspace_bytes < L.total) return MLS_ERR_WORKSPACE_TOO_SMALL;

  std::vector<int64_t> off(n_clouds + 1), soff(n_clouds + 1);
  if (cloud_offsets) {
    for (int32_t c = 0; c <= n_clouds; ++c) off[c] = cloud_offsets[c];
  } else {
    off[0] = 0;
    off[1] = n_points;
  }
  soff[0] = 0;
  for (int32_t c = 0; c < n_clouds; ++c) {
    const int64_t size = off[c + 1] - off[c];
    if (size < 0 || off[0] != 0 || off[n_clouds] != n_points) return MLS_ERR_INVALID_ARGUMENT;
    soff[c + 1] = soff[c] + (size + stride - 1) / stride;
  }
  const int64_t m = soff[n_clouds];
  if (m > m_bound) return MLS_ERR_INVALID_ARGUMENT;

  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  float *sample = (float *)(ws + L.sample);
  int64_t *soff_dev = (int64_t *)(ws + L.soff);
  if (hipMemcpyAsync(soff_dev, soff.data(), 8 * soff.size(), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return MLS_ERR_HIP;

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return MLS_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return MLS_ERR_HIP;
  }
  std::vector<double> cell(n_clouds);
  mls_params prm;
  prm.k = k;
  prm.precision = MLS_PREC_FP32_MOMENTS;
  prm.support_radius_h = 3.0;
  prm.min_support = 3;
  prm.stages = MLS_STAGE_SEARCH;
  prm.search_extra = 0;
  prm.plane_iters = 0;
  prm.ball = 0;
  prm.levin = 0;
  prm.slot_order = 0;
  mls_status st = MLS_OK;
  float best_ms = INFINITY;
  *best_factor = candidates[0];
  for (int32_t i = 0; i < n_candidates && st == MLS_OK; ++i) {
    for (int32_t c = 0; c < n_clouds; ++c) cell[c] = candidates[i] * h[c];
    mls_grid *grid = nullptr;
    st = mls_build_grid(points, n_points, cloud_offsets, n_clouds, h, cell.data(), ws + L.grid,
                        L.sample - L.grid, stream, &grid);
    if (st != MLS_OK) break;
    if (m > 0) {
      // the sample follows this grid's Morton order
      const mls::GridHost &gh = mls::grid_host(grid);
      hipLaunchKernelGGL(k_run_sample, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                         gh.view.pts, gh.clouds_dev, soff_dev, n_clouds, stride, m, sample);
      if (hipGetLastError() != hipSuccess) {
        mls_grid_destroy(grid);
        st = MLS_ERR_HIP;
        break;
      }
    }
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == MLS_OK; ++rep) {  // the first run warms up
      if (hipEventRecord(e0, s) != hipSuccess) st = MLS_ERR_HIP;
      if (st == MLS_OK)
        st = mls_project(grid, &prm, sample, MLS_F32, m, soff.data(), nullptr, nullptr, nullptr,
                         ws + L.proj, L.total - L.proj, stream);
      if (st == MLS_OK && (hipEventRecord(e1, s) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = MLS_ERR_HIP;
    }
    mls_grid_destroy(grid);
    if (st != MLS_OK) break;
    if (ms_per_candidate) ms_per_candidate[i] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      *best_factor = candidates[i];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return st;
}

}  // extern "C"
