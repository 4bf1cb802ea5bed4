// k_ref.hip -- scan A's resident feature map (Alg. 1 initialisation).
//
// 1. scatter: voxel index of every A point (half-open voxels, FP64 in the
//    fixed order u = fl(fl(x*s) + c0)), dense per-voxel n, S1 = sum q,
//    S2 = sum q^2 with q = floor(frac(u_z) * 2^20); A's index box.
// 2. bins: bin of every voxel per feature (0 = empty, the phi value).
// 3. summed-volume table per feature and occupied bin a >= 1, so that the
//    number of A voxels of bin a inside any box is 8 lookups (used for the
//    voxels of the overlap box that B leaves empty).  Each table has the
//    fewest bytes per entry (1, 2 or 4) that hold its bin's voxel count,
//    counted in step 2; its entries are the prefix sums modulo 2^(8 width),
//    and box counts of them are exact because they lie in [0, that count].
//    On large grids the sparsest bins are a voxel list instead (step 4).
// 4. the voxel list of those bins.
#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

__global__ void k_ref_init(RefDev rd) {
  if (threadIdx.x < 3) {
    rd.abox[threadIdx.x] = threadIdx.x == 0 ? rd.nx : (threadIdx.x == 1 ? rd.ny : rd.nz);
    rd.abox[3 + threadIdx.x] = -1;
  }
  if (threadIdx.x < 4) rd.counters[threadIdx.x] = 0ull;
  for (int i = threadIdx.x; i < 128; i += blockDim.x) rd.bin_cnt[i] = 0u;
}

__global__ void __launch_bounds__(256) k_ref_scatter(RefDev rd, const float *__restrict__ xyz,
                                                     int64_t n) {
  const int nx = rd.nx, ny = rd.ny, nz = rd.nz;
  int lo0 = nx, lo1 = ny, lo2 = nz, hi0 = -1, hi1 = -1, hi2 = -1;
  unsigned long long nin = 0, nout = 0, nnf = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) { ++nnf; continue; }
    const double ux = (double)x * rd.s + rd.c0[0];
    const double uy = (double)y * rd.s + rd.c0[1];
    const double uz = (double)z * rd.s + rd.c0[2];
    const double fx = floor(ux), fy = floor(uy), fz = floor(uz);
    if (!(fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny && fz >= 0.0 &&
          fz < (double)nz)) {
      ++nout;
      continue;
    }
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const int64_t v = ((int64_t)iz * ny + iy) * nx + ix;
    const unsigned long long q = (unsigned long long)floor((uz - fz) * kQScale);
    atomicAdd(&rd.cnt[v], 1u);
    atomicAdd(&rd.s1[v], q);
    atomicAdd(&rd.s2[v], q * q);
    ++nin;
    lo0 = min(lo0, ix); lo1 = min(lo1, iy); lo2 = min(lo2, iz);
    hi0 = max(hi0, ix); hi1 = max(hi1, iy); hi2 = max(hi2, iz);
  }
  lo0 = wave_min_i32(lo0); lo1 = wave_min_i32(lo1); lo2 = wave_min_i32(lo2);
  hi0 = wave_max_i32(hi0); hi1 = wave_max_i32(hi1); hi2 = wave_max_i32(hi2);
  nin = wave_sum_u64(nin); nout = wave_sum_u64(nout); nnf = wave_sum_u64(nnf);
  if ((threadIdx.x & 63) == 0) {
    if (hi0 >= 0) {
      atomicMin(&rd.abox[0], lo0); atomicMin(&rd.abox[1], lo1); atomicMin(&rd.abox[2], lo2);
      atomicMax(&rd.abox[3], hi0); atomicMax(&rd.abox[4], hi1); atomicMax(&rd.abox[5], hi2);
    }
    if (nin) atomicAdd(&rd.counters[0], nin);
    if (nout) atomicAdd(&rd.counters[1], nout);
    if (nnf) atomicAdd(&rd.counters[2], nnf);
  }
}

// Bins per voxel and feature, and each bin's voxel count (in LDS per
// workgroup, then one global atomic per bin).
__global__ void __launch_bounds__(256) k_ref_bins(RefDev rd) {
  __shared__ uint32_t lc[128];
  for (int i = threadIdx.x; i < 128; i += blockDim.x) lc[i] = 0u;
  __syncthreads();
  const int64_t V = (int64_t)rd.nx * rd.ny * rd.nz;
  unsigned long long occ = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t n = rd.cnt[v];
    if (n) ++occ;
    for (int f = 0; f < rd.nf; ++f) {
      const int b = feature_bin_dev(rd.kind[f], n, rd.s1[v], rd.s2[v], rd.nbc, rd.count_edges,
                                    rd.nbz, rd.zvar_edges);
      rd.bins[f][v] = (uint8_t)b;
      if (b) atomicAdd(&lc[64 * f + b], 1u);
    }
  }
  occ = wave_sum_u64(occ);
  if ((threadIdx.x & 63) == 0 && occ) atomicAdd(&rd.counters[3], occ);
  __syncthreads();
  for (int i = threadIdx.x; i < 128; i += blockDim.x)
    if (lc[i]) atomicAdd(&rd.bin_cnt[i], lc[i]);
}

// Entry i of a table of w bytes per entry, written modulo 2^(8 w).
__device__ __forceinline__ void sat_store(uint8_t *S, int w, int64_t i, uint32_t v) {
  if (w == 4) ((uint32_t *)S)[i] = v;
  else if (w == 2) ((uint16_t *)S)[i] = (uint16_t)v;
  else S[i] = (uint8_t)v;
}
__device__ __forceinline__ uint32_t sat_get(const uint8_t *S, int w, int64_t i) {
  return w == 4 ? ((const uint32_t *)S)[i] : w == 2 ? (uint32_t)((const uint16_t *)S)[i] : (uint32_t)S[i];
}

// Pass 1 of the summed-volume tables: one thread per (a, yy, x) column of the
// padded table, marks voxels of bin a and sums them along z.
__global__ void __launch_bounds__(256) k_sat_z(const uint8_t *__restrict__ bins, uint8_t *S,
                                               SatLayout L, int nx, int ny, int nz, int nbm1) {
  const int64_t cols = (int64_t)(ny + 1) * (nx + 1);
  const int64_t plane = cols * (nz + 1);
  const int64_t total = cols * nbm1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / cols) + 1;
    if (!sat_has_table(L, a)) continue;
    const int64_t r = t % cols;
    const int yy = (int)(r / (nx + 1)), x = (int)(r % (nx + 1));
    uint8_t *T = S + sat_offset(L, a, plane);
    const int w = sat_width(L, a);
    sat_store(T, w, r, 0u);
    uint32_t run = 0;
    for (int zz = 1; zz <= nz; ++zz) {
      if (yy > 0 && x > 0) run += bins[((int64_t)(zz - 1) * ny + (yy - 1)) * nx + (x - 1)] == a;
      sat_store(T, w, r + (int64_t)zz * cols, run);
    }
  }
}

// Pass 2: prefix along y, one thread per (a, zz, x).
__global__ void __launch_bounds__(256) k_sat_y(uint8_t *S, SatLayout L, int nx, int ny, int nz,
                                               int nbm1) {
  const int64_t cols = (int64_t)(ny + 1) * (nx + 1);
  const int64_t plane = cols * (nz + 1);
  const int64_t per_a = (int64_t)(nz + 1) * (nx + 1);
  const int64_t total = per_a * nbm1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a1 = t / per_a;
    if (!sat_has_table(L, (int)a1 + 1)) continue;
    const int64_t r = t % per_a;
    const int64_t zz = r / (nx + 1), x = r % (nx + 1);
    uint8_t *T = S + sat_offset(L, (int)a1 + 1, plane);
    const int w = sat_width(L, (int)a1 + 1);
    const int64_t i0 = zz * cols + x;
    uint32_t run = 0;
    // eight rows' loads in flight at a time (the sums only chain the adds)
    for (int y0 = 0; y0 <= ny; y0 += 8) {
      uint32_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        v[j] = y0 + j <= ny ? sat_get(T, w, i0 + (int64_t)(y0 + j) * (nx + 1)) : 0u;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        run += v[j];
        if (y0 + j <= ny) sat_store(T, w, i0 + (int64_t)(y0 + j) * (nx + 1), run);
      }
    }
  }
}

// Pass 3: prefix along x, one wave per row (a, zz, yy) with a wave scan.
__global__ void __launch_bounds__(256) k_sat_x(uint8_t *S, SatLayout L, int nx, int ny, int nz,
                                               int nbm1) {
  const int lane = threadIdx.x & 63;
  const int64_t per_a = (int64_t)(nz + 1) * (ny + 1);
  const int64_t plane = per_a * (nx + 1);
  const int64_t rows = (int64_t)nbm1 * per_a;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = wave0; row < rows; row += nwaves) {
    const int a = (int)(row / per_a) + 1;
    if (!sat_has_table(L, a)) continue;  // uniform over the wave: one row per wave
    uint8_t *T = S + sat_offset(L, a, plane);
    const int w = sat_width(L, a);
    const int64_t i0 = (row % per_a) * (nx + 1);
    uint32_t carry = 0;
    for (int x0 = 0; x0 <= nx; x0 += 64) {
      const int x = x0 + lane;
      uint32_t v = x <= nx ? sat_get(T, w, i0 + x) : 0u;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
      }
      v += carry;
      if (x <= nx) sat_store(T, w, i0 + x, v);
      carry = __shfl(v, 63, 64);
    }
  }
}

// Starts of the voxel list's per-bin segments: bins in list_mask, in order.
__global__ void k_list_starts(uint32_t *cur, const uint32_t *cnt, uint64_t m0, uint64_t m1) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int i = 0; i < 128; ++i) {
    cur[i] = run;
    if ((((i < 64 ? m0 : m1) >> (i & 63)) & 1u)) run += cnt[i];
  }
}

// One entry per voxel of a listed bin, (f * 64 + a) << 56 | z << 40 | y << 20
// | x, at its bin's cursor (the order within a bin is not fixed; only counts
// are taken from it).
__global__ void __launch_bounds__(256) k_ref_list(RefDev rd) {
  const int64_t V = (int64_t)rd.nx * rd.ny * rd.nz;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * blockDim.x) {
    for (int f = 0; f < rd.nf; ++f) {
      const int a = rd.bins[f][v];
      if (!((rd.list_mask[f] >> a) & 1u)) continue;
      const int64_t x = v % rd.nx, y = (v / rd.nx) % rd.ny, z = v / ((int64_t)rd.nx * rd.ny);
      const uint32_t pos = atomicAdd(&rd.list_cur[64 * f + a], 1u);
      rd.alist[pos] = ((uint64_t)(64 * f + a) << 56) | ((uint64_t)z << 40) | ((uint64_t)y << 20) |
                      (uint64_t)x;
    }
  }
}

static int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

hipError_t launch_ref_bins(const RefDev &rd, const float *xyz, int64_t n, hipStream_t s) {
  const int64_t V = (int64_t)rd.nx * rd.ny * rd.nz;
  hipError_t e;
  k_ref_init<<<1, 64, 0, s>>>(rd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_u32(rd.cnt, 0u, V, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32((uint32_t *)rd.s1, 0u, 2 * V, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32((uint32_t *)rd.s2, 0u, 2 * V, s)) != hipSuccess) return e;
  if (n > 0) {
    k_ref_scatter<<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, s>>>(rd, xyz, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  k_ref_bins<<<grid_for(V, 256), 256, 0, s>>>(rd);
  return hipGetLastError();
}

hipError_t launch_ref_sat(const RefDev &rd, hipStream_t s) {
  hipError_t e;
  for (int f = 0; f < rd.nf; ++f) {
    const int nbm1 = rd.nb[f] - 1;
    const int64_t cols = (int64_t)(rd.ny + 1) * (rd.nx + 1);
    k_sat_z<<<grid_for(cols * nbm1, 256), 256, 0, s>>>(rd.bins[f], rd.sat[f], rd.sat_layout[f],
                                                       rd.nx, rd.ny, rd.nz, nbm1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_sat_y<<<grid_for((int64_t)(rd.nz + 1) * (rd.nx + 1) * nbm1, 256), 256, 0, s>>>(
        rd.sat[f], rd.sat_layout[f], rd.nx, rd.ny, rd.nz, nbm1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t rows = (int64_t)nbm1 * (rd.nz + 1) * (rd.ny + 1);
    k_sat_x<<<grid_for(rows * 64, 256), 256, 0, s>>>(rd.sat[f], rd.sat_layout[f], rd.nx, rd.ny,
                                                     rd.nz, nbm1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (rd.alist_n) {
    k_list_starts<<<1, 64, 0, s>>>(rd.list_cur, rd.bin_cnt, rd.list_mask[0], rd.list_mask[1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_ref_list<<<grid_for((int64_t)rd.nx * rd.ny * rd.nz, 256), 256, 0, s>>>(rd);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mi
