// k_util.hip -- fills, the argmax of Eq. 1 over a finite pose set, and the
// non-finite point count.
#include "mi_device.h"
#include "mi_internal.h"

namespace mi {

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, uint32_t value, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  k_fill_u32<<<(unsigned)g, 256, 0, s>>>(p, value, n);
  return hipGetLastError();
}

// One workgroup per feature: the maximum, then the smallest index whose MI is
// within 1e-12 of it.
__global__ void __launch_bounds__(1024) k_argmax(const double *__restrict__ mi, int64_t K,
                                                 int64_t *out, double *out_val) {
  __shared__ double smax[16];
  __shared__ long long sidx[16];
  const double *m = mi + (int64_t)blockIdx.x * K;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, W = blockDim.x >> 6;
  double mx = -INFINITY;
  for (int64_t k = tid; k < K; k += blockDim.x) mx = fmax(mx, m[k]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) smax[wid] = mx;
  __syncthreads();
  mx = smax[0];
  for (int w = 1; w < W; ++w) mx = fmax(mx, smax[w]);
  const double thr = mx - 1e-12;
  long long best = K;
  for (int64_t k = tid; k < K; k += blockDim.x)
    if (m[k] >= thr) { best = k; break; }
  for (int o = 32; o > 0; o >>= 1) best = min(best, (long long)__shfl_xor(best, o, 64));
  if (lane == 0) sidx[wid] = best;
  __syncthreads();
  if (tid == 0) {
    long long b = sidx[0];
    for (int w = 1; w < W; ++w) b = min(b, sidx[w]);
    if (b >= K) b = 0;  // unreachable unless MI holds NaN
    out[blockIdx.x] = K > 0 ? (int64_t)b : -1;
    if (out_val) out_val[blockIdx.x] = K > 0 ? m[b] : 0.0;
  }
}

hipError_t launch_argmax(const double *mi, int64_t K, int32_t nf, int64_t *out, double *out_val,
                         hipStream_t s) {
  k_argmax<<<nf, 1024, 0, s>>>(mi, K, out, out_val);
  return hipGetLastError();
}

// Weighted search objective: out[k] = w0 * mi[k] + w1 * mi[K + k], each
// product rounded, then the sum (no fused multiply-add).
__global__ void __launch_bounds__(256) k_weighted(const double *__restrict__ mi, int64_t K,
                                                  int32_t nf, double w0, double w1,
                                                  double *__restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K;
       k += (int64_t)gridDim.x * blockDim.x) {
    double v = w0 * mi[k];
    if (nf > 1) v = v + w1 * mi[K + k];
    out[k] = v;
  }
}

hipError_t launch_weighted(const double *mi, int64_t K, int32_t nf, double w0, double w1,
                           double *out, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  int64_t g = (K + 255) / 256;
  if (g > 1024) g = 1024;
  k_weighted<<<(unsigned)g, 256, 0, s>>>(mi, K, nf, w0, w1, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_count_nonfinite(const float *__restrict__ xyz, int64_t n,
                                                         unsigned long long *out) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(xyz[i]) || !isfinite(xyz[n + i]) || !isfinite(xyz[2 * n + i])) ++c;
  c = wave_sum_u64(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

hipError_t launch_count_nonfinite(const float *xyz, int64_t n, unsigned long long *out,
                                  hipStream_t s) {
  hipError_t e = launch_fill_u32((uint32_t *)out, 0u, 2, s);
  if (e != hipSuccess || n <= 0) return e;
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  k_count_nonfinite<<<(unsigned)g, 256, 0, s>>>(xyz, n, out);
  return hipGetLastError();
}

// Writes the per-execution pointers (scan B, outputs) of the single pair of a
// reusable plan into the device tables on the stream, so that an execution
// enqueues kernels only and a captured graph picks up each execution's buffers.
__global__ void k_bind(PairDev *pair, FrameDev *frames, int32_t n_frames, const float *xyz,
                       double *mi_out, uint32_t *hist_out, mi_pose_stats *stats_out) {
  if (threadIdx.x == 0) {
    pair->mi_out = mi_out;
    pair->hist_out = hist_out;
    pair->stats_out = stats_out;
  }
  for (int i = threadIdx.x; i < n_frames; i += blockDim.x) frames[i].xyz = xyz;
}

hipError_t launch_bind(PairDev *pair, FrameDev *frames, int32_t n_frames, const float *xyz,
                       double *mi_out, uint32_t *hist_out, mi_pose_stats *stats_out,
                       hipStream_t s) {
  k_bind<<<1, 256, 0, s>>>(pair, frames, n_frames, xyz, mi_out, hist_out, stats_out);
  return hipGetLastError();
}

}  // namespace mi
