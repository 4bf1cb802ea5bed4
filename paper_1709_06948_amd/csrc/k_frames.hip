// k_frames.hip -- scan B rotated once per distinct rotation of a pose set.
//
// For every rotation R among the poses (a "frame") each finite B point is
// rotated and scaled to voxel units, v = fl(fl(R p) * s) with the rows summed
// left to right, and bucketed by its column (floor(v_x), floor(v_y)) of a
// column grid that covers every position from which some pose's translation
// can bring the point into A's grid.  A pose with that rotation and
// translation offset c then maps the point to voxel floor(fl(v + c)), the same
// doubles the per-pose transform of Alg. 1 produces.  Points that no pose can
// bring into the grid are dropped here.  Bucketing is a counting sort:
// count -> exclusive scan -> scatter.
#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

struct Rotated {
  double vx, vy, vz;
  int col;  // -1 when dropped
};

__device__ __forceinline__ Rotated rotate_point(const FrameDev &F, int64_t i) {
  Rotated r;
  r.col = -1;
  const float xf = F.xyz[i], yf = F.xyz[F.n + i], zf = F.xyz[2 * F.n + i];
  if (!isfinite(xf) || !isfinite(yf) || !isfinite(zf)) return r;
  const double x = xf, y = yf, z = zf;
  const double wx = (F.R[0] * x + F.R[1] * y) + F.R[2] * z;
  const double wy = (F.R[3] * x + F.R[4] * y) + F.R[5] * z;
  const double wz = (F.R[6] * x + F.R[7] * y) + F.R[8] * z;
  r.vx = wx * F.s;
  r.vy = wy * F.s;
  r.vz = wz * F.s;
  const double fx = floor(r.vx), fy = floor(r.vy), fz = floor(r.vz);
  const double cx = fx - (double)F.gx, cy = fy - (double)F.gy;
  if (!(cx >= 0.0 && cx < (double)F.ncx && cy >= 0.0 && cy < (double)F.ncy)) return r;
  if (!(fz >= (double)F.zlo && fz <= (double)F.zhi)) return r;
  r.col = (int)cy * F.ncx + (int)cx;
  return r;
}

__global__ void __launch_bounds__(256) k_frame_count(const FrameDev *__restrict__ frames) {
  const FrameDev &F = frames[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Rotated r = rotate_point(F, i);
    if (r.col >= 0) atomicAdd(&F.cur[r.col], 1u);
  }
}

// Exclusive scan of the column counts of one frame (one workgroup per frame);
// off[ncols] = kept points; the cursors start at the offsets.
__global__ void __launch_bounds__(1024) k_frame_scan(const FrameDev *__restrict__ frames) {
  const FrameDev &F = frames[blockIdx.x];
  const int64_t ncols = (int64_t)F.ncx * F.ncy;
  const int T = blockDim.x;
  const int64_t per = (ncols + T - 1) / T;
  const int64_t b = (int64_t)threadIdx.x * per;
  const int64_t e = b + per < ncols ? b + per : ncols;
  uint32_t sum = 0;
  for (int64_t k = b; k < e; ++k) sum += F.cur[k];
  __shared__ uint32_t part[1024];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the per-thread sums.
  for (int o = 1; o < T; o <<= 1) {
    const uint32_t add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int64_t k = b; k < e; ++k) {
    const uint32_t c = F.cur[k];
    F.off[k] = run;
    F.cur[k] = run;
    run += c;
  }
  if (threadIdx.x == T - 1) F.off[ncols] = part[T - 1];
}

__global__ void __launch_bounds__(256) k_frame_scatter(const FrameDev *__restrict__ frames) {
  const FrameDev &F = frames[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Rotated r = rotate_point(F, i);
    if (r.col < 0) continue;
    const uint32_t pos = atomicAdd(&F.cur[r.col], 1u);
    F.v[pos] = r.vx;
    F.v[F.n + pos] = r.vy;
    F.v[2 * F.n + pos] = r.vz;
  }
}

hipError_t launch_frames(const FrameDev *frames_dev, int32_t n_frames, int64_t max_points,
                         int32_t, hipStream_t s) {
  if (n_frames <= 0) return hipSuccess;
  int64_t gx = (max_points + 255) / 256;
  if (gx < 1) gx = 1;
  if (gx > 1024) gx = 1024;
  int32_t frames_left = n_frames, base = 0;
  while (frames_left > 0) {  // grid.y is limited to 65535
    const int32_t fy = frames_left > 65535 ? 65535 : frames_left;
    k_frame_count<<<dim3((unsigned)gx, (unsigned)fy), 256, 0, s>>>(frames_dev + base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_frame_scan<<<fy, 1024, 0, s>>>(frames_dev + base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_frame_scatter<<<dim3((unsigned)gx, (unsigned)fy), 256, 0, s>>>(frames_dev + base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    frames_left -= fy;
    base += fy;
  }
  return hipSuccess;
}

}  // namespace mi
