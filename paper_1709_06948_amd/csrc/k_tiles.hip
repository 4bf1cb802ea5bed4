// k_tiles.hip -- scan B bucketed into tiles of its own (x, y) frame, for the
// tiled per-pose evaluator: count, exclusive scan, scatter (one launch each
// over every tiled pair of a batch).
//
// A tile keeps its own points first, then its halo: the points of its
// neighbours that lie within the halo width of it.  The evaluator keeps a
// voxel only in the tile that holds the voxel's centre mapped back into B's
// frame; every point of that voxel is within half a voxel diagonal of the
// centre, so with a halo of more than that the tile sees all of them.  The
// order of points within a tile is not fixed (atomic cursors); the voxel sums
// are integers, so the results do not depend on it.
#include <algorithm>

#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

struct TileHits {
  int own, n;
  int halo[3];
};

// The tile of a point and the tiles whose halo holds it.  The halo width is
// below half a tile, so only the tile's 8 neighbours can take the point.
__device__ __forceinline__ TileHits tiles_of(const PairDev &P, float xf, float yf) {
  const int nx = P.tile_nx, ny = P.tile_ny;
  const double fx = ((double)xf - P.tile_x0) * P.tile_ilx;
  const double fy = ((double)yf - P.tile_y0) * P.tile_ily;
  // v_cvt_i32_f64 saturates, so far-away points clamp to the edge tiles
  const int i = min(max((int)floor(fx), 0), nx - 1);
  const int j = min(max((int)floor(fy), 0), ny - 1);
  const double rx = fx - (double)i, ry = fy - (double)j;
  const int di = (i > 0 && rx < P.tile_hx) ? -1 : (i + 1 < nx && rx > 1.0 - P.tile_hx) ? 1 : 0;
  const int dj = (j > 0 && ry < P.tile_hy) ? -1 : (j + 1 < ny && ry > 1.0 - P.tile_hy) ? 1 : 0;
  TileHits r;
  r.own = j * nx + i;
  r.n = 0;
  if (di) r.halo[r.n++] = j * nx + i + di;
  if (dj) r.halo[r.n++] = (j + dj) * nx + i;
  if (di && dj) r.halo[r.n++] = (j + dj) * nx + i + di;
  return r;
}

// Tiles counted in LDS per workgroup (more fall back to global atomics only).
constexpr int kTileLds = 4096;
// Points per thread per round of the count and scatter passes.
constexpr int kTilePpt = 4;

// counts: tile_cnt[t] own points of tile t, tile_cnt[tiles + t] its halo.  A
// workgroup counts a round of kTilePpt * blockDim points in LDS, then adds its
// nonzero counts to the pair's (one global atomic per tile and round).
__global__ void __launch_bounds__(1024) k_tile_count(const PairDev *__restrict__ pairs,
                                                     const int32_t *__restrict__ tiled) {
  __shared__ uint32_t lown[kTileLds], lhalo[kTileLds];
  const PairDev &P = pairs[tiled[blockIdx.y]];
  const int64_t n = P.n_b;
  const int nt = P.tile_nx * P.tile_ny, T = blockDim.x, tid = threadIdx.x;
  uint32_t *own = P.tile_cnt, *halo = P.tile_cnt + nt;
  const float *x = P.xyz_b, *y = x + n, *z = y + n;
  const bool lds = nt <= kTileLds;
  const int64_t round = (int64_t)kTilePpt * T;
  for (int64_t base = (int64_t)blockIdx.x * round; base < n; base += (int64_t)gridDim.x * round) {
    if (lds) {
      for (int t = tid; t < nt; t += T) { lown[t] = 0u; lhalo[t] = 0u; }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kTilePpt; ++k) {
      const int64_t i = base + (int64_t)k * T + tid;
      if (i >= n) continue;
      const float xf = x[i], yf = y[i], zf = z[i];
      if (!isfinite(xf) || !isfinite(yf) || !isfinite(zf)) continue;
      const TileHits h = tiles_of(P, xf, yf);
      atomicAdd(lds ? &lown[h.own] : &own[h.own], 1u);
      for (int m = 0; m < h.n; ++m) atomicAdd(lds ? &lhalo[h.halo[m]] : &halo[h.halo[m]], 1u);
    }
    if (lds) {
      __syncthreads();
      for (int t = tid; t < nt; t += T) {
        if (lown[t]) atomicAdd(&own[t], lown[t]);
        if (lhalo[t]) atomicAdd(&halo[t], lhalo[t]);
      }
      __syncthreads();
    }
  }
}

// One workgroup per pair: tile t starts at the sum of the earlier tiles' own
// and halo counts; the counts become the own and halo cursors.
__global__ void __launch_bounds__(1024) k_tile_scan(const PairDev *__restrict__ pairs,
                                                    const int32_t *__restrict__ tiled) {
  __shared__ uint32_t wsum[16];
  const PairDev &P = pairs[tiled[blockIdx.x]];
  const int nt = P.tile_nx * P.tile_ny;
  uint32_t *own = P.tile_cnt, *halo = P.tile_cnt + nt;
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int per = (nt + T - 1) / T;
  const int t0 = min(tid * per, nt), t1 = min(t0 + per, nt);
  uint32_t sum = 0;
  for (int t = t0; t < t1; ++t) sum += own[t] + halo[t];
  uint32_t inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wid; ++w) base += wsum[w];
  uint32_t run = base + inc - sum;
  for (int t = t0; t < t1; ++t) {
    const uint32_t o = own[t], hc = halo[t];
    P.tile_off[t] = run;
    P.tile_own[t] = run + o;
    own[t] = run;
    halo[t] = run + o;
    run += o + hc;
  }
  if (tid == T - 1) P.tile_off[nt] = run;
}

// Scatter: a workgroup ranks its round's points per tile in LDS, reserves
// each tile's run of places with one global atomic on the tile's cursor, and
// writes every point to its run.
__global__ void __launch_bounds__(1024) k_tile_scatter(const PairDev *__restrict__ pairs,
                                                       const int32_t *__restrict__ tiled) {
  __shared__ uint32_t lown[kTileLds], lhalo[kTileLds];
  const PairDev &P = pairs[tiled[blockIdx.y]];
  const int64_t n = P.n_b, ts = P.tile_stride;
  const int nt = P.tile_nx * P.tile_ny, T = blockDim.x, tid = threadIdx.x;
  uint32_t *own = P.tile_cnt, *halo = P.tile_cnt + nt;
  const float *x = P.xyz_b, *y = x + n, *z = y + n;
  float *tx = P.tile_xyz, *ty = tx + ts, *tz = ty + ts;
  const bool lds = nt <= kTileLds;
  const int64_t round = (int64_t)kTilePpt * T;
  for (int64_t base = (int64_t)blockIdx.x * round; base < n; base += (int64_t)gridDim.x * round) {
    if (lds) {
      for (int t = tid; t < nt; t += T) { lown[t] = 0u; lhalo[t] = 0u; }
      __syncthreads();
    }
    float px[kTilePpt], py[kTilePpt], pz[kTilePpt];
    bool ok[kTilePpt];
    TileHits h[kTilePpt];
    uint32_t r_own[kTilePpt], r_halo[kTilePpt][3];
#pragma unroll
    for (int k = 0; k < kTilePpt; ++k) {
      const int64_t i = base + (int64_t)k * T + tid;
      ok[k] = false;
      h[k].n = 0;
      if (i >= n) continue;
      px[k] = x[i];
      py[k] = y[i];
      pz[k] = z[i];
      if (!isfinite(px[k]) || !isfinite(py[k]) || !isfinite(pz[k])) continue;
      ok[k] = true;
      h[k] = tiles_of(P, px[k], py[k]);
      // LDS: the point's rank within this round; global: its place
      r_own[k] = atomicAdd(lds ? &lown[h[k].own] : &own[h[k].own], 1u);
      for (int m = 0; m < h[k].n; ++m)
        r_halo[k][m] = atomicAdd(lds ? &lhalo[h[k].halo[m]] : &halo[h[k].halo[m]], 1u);
    }
    if (lds) {
      __syncthreads();
      // each tile's run of places for this round
      for (int t = tid; t < nt; t += T) {
        if (lown[t]) lown[t] = atomicAdd(&own[t], lown[t]);
        if (lhalo[t]) lhalo[t] = atomicAdd(&halo[t], lhalo[t]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kTilePpt; ++k) {
      if (!ok[k]) continue;
      uint32_t pos = r_own[k] + (lds ? lown[h[k].own] : 0u);
      tx[pos] = px[k];
      ty[pos] = py[k];
      tz[pos] = pz[k];
      for (int m = 0; m < h[k].n; ++m) {
        pos = r_halo[k][m] + (lds ? lhalo[h[k].halo[m]] : 0u);
        tx[pos] = px[k];
        ty[pos] = py[k];
        tz[pos] = pz[k];
      }
    }
    if (lds) __syncthreads();
  }
}

hipError_t launch_tiles(const PairDev *pairs_dev, const int32_t *tiled_dev, int32_t n_tiled,
                        int64_t max_n, uint32_t *cnt, int64_t cnt_words, hipStream_t s) {
  if (n_tiled <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(cnt, 0u, cnt_words, s);
  if (e != hipSuccess) return e;
  const int64_t round = (int64_t)kTilePpt * 1024;
  const unsigned gx = (unsigned)std::min<int64_t>(std::max<int64_t>((max_n + round - 1) / round, 1), 1024);
  // pairs along grid y, at most 65535 per launch
  for (int32_t k0 = 0; k0 < n_tiled; k0 += 65535) {
    const unsigned ny = (unsigned)std::min<int32_t>(65535, n_tiled - k0);
    k_tile_count<<<dim3(gx, ny), 1024, 0, s>>>(pairs_dev, tiled_dev + k0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  k_tile_scan<<<(unsigned)n_tiled, 1024, 0, s>>>(pairs_dev, tiled_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int32_t k0 = 0; k0 < n_tiled; k0 += 65535) {
    const unsigned ny = (unsigned)std::min<int32_t>(65535, n_tiled - k0);
    k_tile_scatter<<<dim3(gx, ny), 1024, 0, s>>>(pairs_dev, tiled_dev + k0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mi
