// k_plain.hip -- the per-pose launch sequence shaped like the paper's GPU
// stages (Table III: voxel mapping, find overlap, feature histograms, entropy):
//   map      : transform every B point (FP64, rows left to right), voxel index,
//              fixed-point height, B's extent (atomic min/max)
//   scatter  : per-voxel sums into a dense per-pose grid in device memory
//   hist     : dense sweep of every voxel of the overlap box, A's bin against
//              B's bin, into the joint histogram (LDS per block, then global)
//   finish   : near-face count inside the overlap and reset of the dense grid
//   entropy  : H(X), H(Y), H(X,Y), MI
// It is the simple baseline beside the batched evaluator.
#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

__global__ void k_plain_init(PlainDev pd) {
  const int t = threadIdx.x;
  const int words = pd.nb[0] * pd.nb[0] + (pd.nf > 1 ? pd.nb[1] * pd.nb[1] : 0);
  for (int i = t; i < words; i += blockDim.x) pd.hist[i] = 0u;
  if (t < 3) {
    pd.bbox[t] = t == 0 ? pd.nx : (t == 1 ? pd.ny : pd.nz);
    pd.bbox[3 + t] = -1;
  }
  if (t < 4) pd.ctr[t] = 0ull;
}

__global__ void __launch_bounds__(256) k_plain_map(PlainDev pd, const float *__restrict__ xyz,
                                                   int64_t n, const double *__restrict__ rc) {
  const double R0 = rc[0], R1 = rc[1], R2 = rc[2], R3 = rc[3], R4 = rc[4], R5 = rc[5], R6 = rc[6],
               R7 = rc[7], R8 = rc[8], c0 = rc[9], c1 = rc[10], c2 = rc[11];
  int lo0 = pd.nx, lo1 = pd.ny, lo2 = pd.nz, hi0 = -1, hi1 = -1, hi2 = -1;
  unsigned long long nin = 0, nnf = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    pd.lin[i] = -1;
    const float xf = xyz[i], yf = xyz[n + i], zf = xyz[2 * n + i];
    if (!isfinite(xf) || !isfinite(yf) || !isfinite(zf)) { ++nnf; continue; }
    const double x = xf, y = yf, z = zf;
    const double wx = (R0 * x + R1 * y) + R2 * z;
    const double wy = (R3 * x + R4 * y) + R5 * z;
    const double wz = (R6 * x + R7 * y) + R8 * z;
    const double ux = wx * pd.s + c0, uy = wy * pd.s + c1, uz = wz * pd.s + c2;
    const double fx = floor(ux), fy = floor(uy), fz = floor(uz);
    if (!(fx >= 0.0 && fx < (double)pd.nx && fy >= 0.0 && fy < (double)pd.ny && fz >= 0.0 &&
          fz < (double)pd.nz))
      continue;
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    pd.lin[i] = (iz * pd.ny + iy) * pd.nx + ix;
    pd.q[i] = (uint32_t)floor((uz - fz) * kQScale);
    double d = 1.0;
    const double fr[3] = {ux - fx, uy - fy, uz - fz};
    for (int a = 0; a < 3; ++a) {
      const double up = 1.0 - fr[a];
      const double m = fr[a] < up ? fr[a] : up;
      if (m < d) d = m;
    }
    pd.near[i] = d * pd.voxel < kNearFace ? 1 : 0;
    ++nin;
    lo0 = min(lo0, ix); lo1 = min(lo1, iy); lo2 = min(lo2, iz);
    hi0 = max(hi0, ix); hi1 = max(hi1, iy); hi2 = max(hi2, iz);
  }
  lo0 = wave_min_i32(lo0); lo1 = wave_min_i32(lo1); lo2 = wave_min_i32(lo2);
  hi0 = wave_max_i32(hi0); hi1 = wave_max_i32(hi1); hi2 = wave_max_i32(hi2);
  nin = wave_sum_u64(nin);
  nnf = wave_sum_u64(nnf);
  // one set of global atomics per block, not per wave
  __shared__ int sb[4][6];
  __shared__ unsigned long long sc[4][2];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sb[w][0] = lo0; sb[w][1] = lo1; sb[w][2] = lo2; sb[w][3] = hi0; sb[w][4] = hi1; sb[w][5] = hi2;
    sc[w][0] = nin;
    sc[w][1] = nnf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      lo0 = min(lo0, sb[k][0]); lo1 = min(lo1, sb[k][1]); lo2 = min(lo2, sb[k][2]);
      hi0 = max(hi0, sb[k][3]); hi1 = max(hi1, sb[k][4]); hi2 = max(hi2, sb[k][5]);
      nin += sc[k][0];
      nnf += sc[k][1];
    }
    if (hi0 >= 0) {
      atomicMin(&pd.bbox[0], lo0); atomicMin(&pd.bbox[1], lo1); atomicMin(&pd.bbox[2], lo2);
      atomicMax(&pd.bbox[3], hi0); atomicMax(&pd.bbox[4], hi1); atomicMax(&pd.bbox[5], hi2);
    }
    if (nin) atomicAdd(&pd.ctr[0], nin);
    if (nnf) atomicAdd(&pd.ctr[1], nnf);
  }
}

__global__ void __launch_bounds__(256) k_plain_scatter(PlainDev pd, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int v = pd.lin[i];
    if (v < 0) continue;
    const unsigned long long q = pd.q[i];
    atomicAdd(&pd.dn[v], 1u);
    atomicAdd(&pd.ds1[v], q);
    atomicAdd(&pd.ds2[v], q * q);
  }
}

struct OBox {
  int lo[3], hi[3];
  int64_t n;
};

__device__ __forceinline__ OBox overlap_box(const PlainDev &pd) {
  OBox o;
  const int dims[3] = {pd.nx, pd.ny, pd.nz};
  o.n = 1;
  for (int a = 0; a < 3; ++a) {
    o.lo[a] = max(max(pd.abox[a], pd.bbox[a]), 0);
    o.hi[a] = min(min(pd.abox[3 + a], pd.bbox[3 + a]), dims[a] - 1);
    if (o.hi[a] < o.lo[a]) o.n = 0;
    else if (o.n) o.n *= (int64_t)(o.hi[a] - o.lo[a] + 1);
  }
  return o;
}

__global__ void __launch_bounds__(256) k_plain_hist(PlainDev pd) {
  extern __shared__ uint32_t lh[];
  const int nb0 = pd.nb[0], nb1 = pd.nf > 1 ? pd.nb[1] : 0;
  const int words = nb0 * nb0 + nb1 * nb1;
  for (int i = threadIdx.x; i < words; i += blockDim.x) lh[i] = 0u;
  __syncthreads();
  const OBox o = overlap_box(pd);
  const int ex = o.hi[0] - o.lo[0] + 1, ey = o.hi[1] - o.lo[1] + 1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < o.n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int x = o.lo[0] + (int)(t % ex);
    const int y = o.lo[1] + (int)((t / ex) % ey);
    const int z = o.lo[2] + (int)(t / ((int64_t)ex * ey));
    const int64_t v = ((int64_t)z * pd.ny + y) * pd.nx + x;
    const uint32_t n = pd.dn[v];
    const unsigned long long s1 = pd.ds1[v], s2 = pd.ds2[v];
    for (int f = 0; f < pd.nf; ++f) {
      const int nb = pd.nb[f];
      const int a = pd.binA[f][v];
      const int b = feature_bin_dev(pd.kind[f], n, s1, s2, pd.nbc, pd.count_edges, pd.nbz,
                                    pd.zvar_edges);
      atomicAdd(&lh[(f ? nb0 * nb0 : 0) + a * nb + b], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < words; i += blockDim.x)
    if (lh[i]) atomicAdd(&pd.hist[i], lh[i]);
}

__global__ void __launch_bounds__(256) k_plain_finish(PlainDev pd, int64_t n, int near_face) {
  const OBox o = overlap_box(pd);
  unsigned long long nn = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int v = pd.lin[i];
    if (v < 0) continue;
    if (near_face && pd.near[i] && o.n) {
      const int x = v % pd.nx, y = (v / pd.nx) % pd.ny, z = v / (pd.nx * pd.ny);
      if (x >= o.lo[0] && x <= o.hi[0] && y >= o.lo[1] && y <= o.hi[1] && z >= o.lo[2] &&
          z <= o.hi[2])
        ++nn;
    }
    pd.dn[v] = 0u;
    pd.ds1[v] = 0ull;
    pd.ds2[v] = 0ull;
  }
  nn = wave_sum_u64(nn);
  if ((threadIdx.x & 63) == 0 && nn) atomicAdd(&pd.ctr[2], nn);
}

__global__ void __launch_bounds__(128) k_plain_entropy(PlainDev pd, int64_t n, int64_t k,
                                                       double *mi_out, int64_t K,
                                                       uint32_t *hist_out, int64_t hoff0,
                                                       int64_t hoff1, mi_pose_stats *stats_out) {
  const OBox o = overlap_box(pd);
  const int lane = threadIdx.x & 63, f = threadIdx.x >> 6;
  if (f < pd.nf) {
    const int nb = pd.nb[f];
    const uint32_t *H = pd.hist + (f ? pd.nb[0] * pd.nb[0] : 0);
    double hxy = 0.0, hx = 0.0, hy = 0.0;
    if (o.n) {
      const double N = (double)o.n;
      for (int i = lane; i < nb * nb; i += 64) hxy += plogp_term(H[i], N);
      if (lane < nb) {
        uint64_t r = 0, c = 0;
        for (int b = 0; b < nb; ++b) r += H[lane * nb + b];
        for (int a = 0; a < nb; ++a) c += H[a * nb + lane];
        hx = plogp_term(r, N);
        hy = plogp_term(c, N);
      }
    }
    hxy = wave_sum_f64(hxy);
    hx = wave_sum_f64(hx);
    hy = wave_sum_f64(hy);
    if (lane == 0) mi_out[(int64_t)f * K + k] = o.n ? (hx + hy) - hxy : 0.0;
    if (hist_out) {
      uint32_t *dst = hist_out + (f ? hoff1 : hoff0) + k * nb * nb;
      for (int i = lane; i < nb * nb; i += 64) dst[i] = H[i];
    }
  }
  if (stats_out && threadIdx.x == 0) {
    mi_pose_stats st;
    for (int a = 0; a < 3; ++a) { st.lo[a] = o.lo[a]; st.hi[a] = o.hi[a]; }
    st.n_overlap = o.n;
    st.n_in_grid = (int64_t)pd.ctr[0];
    st.n_nonfinite = (int64_t)pd.ctr[1];
    st.n_out_of_grid = n - st.n_in_grid - st.n_nonfinite;
    st.n_near_face = (int64_t)pd.ctr[2];
    stats_out[k] = st;
  }
}

static unsigned grid_pts(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (unsigned)g;
}

hipError_t launch_plain_pose(const PlainDev &pd, const PlainDev *, const float *xyz, int64_t n,
                             const double *rt_dev, int64_t k, double *mi_out, int64_t K,
                             uint32_t *hist_out, const int64_t hist_off[2],
                             mi_pose_stats *stats_out, bool near_face, hipStream_t s) {
  hipError_t e;
  k_plain_init<<<1, 256, 0, s>>>(pd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_plain_map<<<grid_pts(n), 256, 0, s>>>(pd, xyz, n, rt_dev + 12 * k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_plain_scatter<<<grid_pts(n), 256, 0, s>>>(pd, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int words = pd.nb[0] * pd.nb[0] + (pd.nf > 1 ? pd.nb[1] * pd.nb[1] : 0);
  k_plain_hist<<<1024, 256, (size_t)words * 4, s>>>(pd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_plain_finish<<<grid_pts(n), 256, 0, s>>>(pd, n, near_face ? 1 : 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_plain_entropy<<<1, 128, 0, s>>>(pd, n, k, mi_out, K, hist_out, hist_off[0], hist_off[1],
                                    stats_out);
  return hipGetLastError();
}

hipError_t launch_plain_clear_dense(const PlainDev &pd, hipStream_t s) {
  const int64_t V = (int64_t)pd.nx * pd.ny * pd.nz;
  hipError_t e = launch_fill_u32(pd.dn, 0u, V, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32((uint32_t *)pd.ds1, 0u, 2 * V, s);
  if (e != hipSuccess) return e;
  return launch_fill_u32((uint32_t *)pd.ds2, 0u, 2 * V, s);
}

}  // namespace mi
