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

// Points of a scan that are neighbours in memory (consecutive samples of a
// scanner ring) usually fall in the same column: lanes with the column of the
// lane before them form runs, and only the first lane of a run touches the
// column's counter, for the whole run.
struct ColRun {
  bool head;      // first lane of a run of kept points
  int head_lane;  // first lane of this lane's run
  uint32_t len;   // run length (heads only)
};

__device__ __forceinline__ ColRun col_runs(int col) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(col, 1, 64);
  const bool kept = col >= 0;
  const bool head = kept && (lane == 0 || prev != col);
  const unsigned long long H = __ballot(head);
  const unsigned long long K = __ballot(kept);
  ColRun r;
  r.head = head;
  // the run ends at the next head or at the next dropped point
  const unsigned long long ends = H | ~K;
  const unsigned long long above = lane == 63 ? 0ull : ends >> (lane + 1);
  const int next = above ? __builtin_ctzll(above) + lane + 1 : 64;
  r.len = (uint32_t)(next - lane);
  const unsigned long long upto = lane == 63 ? H : H & ((2ull << lane) - 1ull);
  r.head_lane = upto ? 63 - __builtin_clzll(upto) : lane;
  return r;
}

__global__ void __launch_bounds__(256) k_frame_count(const FrameDev *__restrict__ frames) {
  const FrameDev &F = frames[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole waves iterate together (the run detection needs every lane)
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < F.n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const int col = i < F.n ? rotate_point(F, i).col : -1;
    const ColRun r = col_runs(col);
    if (r.head) atomicAdd(&F.cur[col], r.len);
  }
}

// Exclusive scan of the column counts of one frame (one workgroup per frame).
// A round covers 4 coalesced tiles of 4 columns per thread, all loaded before
// any is scanned, so a frame of ~10^5 columns waits on memory a handful of
// times; off[ncols] = kept points; the cursors start at the offsets.
__global__ void __launch_bounds__(1024) k_frame_scan(const FrameDev *__restrict__ frames) {
  constexpr int kTiles = 4, kPer = 4;
  const FrameDev &F = frames[blockIdx.x];
  const int64_t ncols = (int64_t)F.ncx * F.ncy;
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, W = T >> 6;
  // per-wave tile totals, in alternating buffers: one barrier per round
  // suffices, as a buffer is rewritten only two rounds later
  __shared__ uint32_t wsum[2][kTiles][16];
  uint32_t carry = 0u;  // the same in every thread
  int par = 0;
  for (int64_t t0 = 0; t0 < ncols; t0 += (int64_t)kTiles * kPer * T) {
    uint32_t c[kTiles][kPer], inc[kTiles], sum[kTiles];
#pragma unroll
    for (int r = 0; r < kTiles; ++r) {
      const int64_t b = t0 + (int64_t)r * kPer * T + kPer * (int64_t)tid;
#pragma unroll
      for (int j = 0; j < kPer; ++j) c[r][j] = b + j < ncols ? F.cur[b + j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kTiles; ++r) {
      sum[r] = 0u;
#pragma unroll
      for (int j = 0; j < kPer; ++j) sum[r] += c[r][j];
      inc[r] = sum[r];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc[r], o, 64);
        if (lane >= o) inc[r] += v;
      }
      if (lane == 63) wsum[par][r][wid] = inc[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTiles; ++r) {
      uint32_t wbase = carry, tot = 0u;
      for (int w = 0; w < W; ++w) {
        const uint32_t x = wsum[par][r][w];
        if (w < wid) wbase += x;
        tot += x;
      }
      const int64_t b = t0 + (int64_t)r * kPer * T + kPer * (int64_t)tid;
      uint32_t run = wbase + inc[r] - sum[r];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        if (b + j < ncols) {
          F.off[b + j] = run;
          F.cur[b + j] = run;
        }
        run += c[r][j];
      }
      carry += tot;
    }
    par ^= 1;
  }
  if (tid == 0) F.off[ncols] = carry;
}

__global__ void __launch_bounds__(256) k_frame_scatter(const FrameDev *__restrict__ frames) {
  const FrameDev &F = frames[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < F.n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    Rotated rp;
    rp.col = -1;
    if (i < F.n) rp = rotate_point(F, i);
    const ColRun r = col_runs(rp.col);
    uint32_t base = 0;
    if (r.head) base = atomicAdd(&F.cur[rp.col], r.len);
    base = __shfl(base, r.head_lane, 64);
    if (rp.col < 0) continue;
    const uint32_t pos = base + (uint32_t)(lane - r.head_lane);
    F.v[pos] = rp.vx;
    F.v[F.n + pos] = rp.vy;
    F.v[2 * F.n + pos] = rp.vz;
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
