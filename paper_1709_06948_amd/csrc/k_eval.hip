// k_eval.hip -- MI of one candidate pose per workgroup (Eqs. 1-5, Alg. 1 loop
// body), on scan B's points already rotated once per distinct rotation.
//
// A's grid is tiled into bricks of bx * by columns at full height.  Each wave
// owns one brick at a time, so every voxel's sums (n, S1, S2) are complete in
// the wave's slice of LDS without any merge across waves or workgroups:
//   1. candidate points: the columns of the rotated cloud whose points can land
//      in the brick under this pose's translation (one padded column of slack
//      per side); their row ranges come from the column offsets;
//   2. per candidate: u = fl(v + c), voxel floor(u); points inside the brick
//      add to the voxel's LDS sums (first touch appends the voxel to the
//      wave's occupied list) and to the pose's extent of B;
//   3. per occupied voxel inside A's index box (which, with B's extent, is the
//      overlap box): its B bin and A's bin add one to the joint histogram.
// After all bricks: overlap box O = A box x B extent; the cells of voxels that
// B leaves empty come from A's per-bin summed-volume tables (H[a][0] = A's
// voxels of bin a in O minus those B occupies; H[0][0] closes the mass |O|);
// then H(X), H(Y), H(X,Y) and MI.
#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

struct EvalCfgDev {
  int32_t hist_copies;
  int32_t hist_words;
  int32_t wave_bytes;
  int32_t misc_bytes;
};

static constexpr int kRowTableBytes = 512;  // 64 row starts + 64 row prefixes

// LDS layout: hist copies (rounded to 16 B) | cntA[2][64] u32 | count edges 64 u32 |
// z-variance edges 64 u64 | wave boxes [W][8] i32 | wave counts [W][2] u64 | next
// brick counter; then one slice of wave_bytes per wave.
__host__ __device__ constexpr int hist_region_bytes(int hist_copies, int hist_words) {
  return (hist_copies * hist_words * 4 + 15) & ~15;
}

__host__ __device__ constexpr int misc_bytes_for(int waves, int hist_copies, int hist_words) {
  return ((hist_region_bytes(hist_copies, hist_words) + 512 + 256 + 512 + waves * 32 +
           waves * 16 + 16) + 255) & ~255;
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool NEAR>
__global__ void __launch_bounds__(512) k_eval(const PairDev *__restrict__ pairs,
                                              const PoseDev *__restrict__ items, int64_t n_items,
                                              int64_t per_xcd, EvalCfgDev cfg) {
  extern __shared__ __align__(16) unsigned char smem[];
  // XCD-aware mapping: consecutive workgroup ids go round-robin over the XCDs,
  // so each XCD walks a contiguous run of the frame-sorted items and keeps the
  // frames it reads in its own L2.
  const int64_t item = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (item >= n_items) return;
  const PoseDev pose = items[item];
  const PairDev &P = pairs[pose.pair];

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, W = blockDim.x >> 6;
  uint32_t *hist = (uint32_t *)smem;
  uint32_t *cntA = (uint32_t *)(smem + hist_region_bytes(cfg.hist_copies, cfg.hist_words));
  uint32_t *cedge = cntA + 128;
  uint64_t *zedge = (uint64_t *)(cedge + 64);
  int *wbox = (int *)(zedge + 64);
  unsigned long long *wcnt = (unsigned long long *)(wbox + 8 * W);
  uint32_t *next = (uint32_t *)(wcnt + 2 * W);
  unsigned char *wreg = smem + cfg.misc_bytes + (size_t)wid * cfg.wave_bytes;
  uint32_t *rstart = (uint32_t *)wreg;
  uint32_t *rpre = rstart + 64;
  unsigned char *agg = wreg + kRowTableBytes;
  uint32_t *agg32 = (uint32_t *)agg;
  unsigned long long *agg64 = (unsigned long long *)agg;

  const int nx = P.nx, ny = P.ny, nz = P.nz, nf = P.nf, bx = P.bx, by = P.by, bpv = P.bpv;
  const int bvox = nz * by * bx;
  uint16_t *occ = (uint16_t *)(agg + (size_t)bvox * bpv);
  const int nb0 = P.nb[0], nb1 = nf > 1 ? P.nb[1] : 0;
  const int hoff1 = nb0 * nb0;

  for (int i = tid; i < cfg.hist_copies * cfg.hist_words; i += blockDim.x) hist[i] = 0u;
  for (int i = tid; i < 64; i += blockDim.x) {
    cedge[i] = P.count_edges[i];
    zedge[i] = P.zvar_edges[i];
  }
  for (int i = lane; i < bvox * bpv / 4; i += 64) agg32[i] = 0u;
  if (tid == 0) *next = 0u;
  __syncthreads();

  const double cx = pose.c[0], cy = pose.c[1], cz = pose.c[2];
  const double *fvx = P.fv + (int64_t)pose.frame * 3 * P.fstride;
  const double *fvy = fvx + P.fstride;
  const double *fvz = fvy + P.fstride;
  const int64_t ncols = (int64_t)P.ncx * P.ncy;
  const uint32_t *off = P.foff + (int64_t)pose.frame * (ncols + 1);
  const int alo0 = P.abox[0], alo1 = P.abox[1], alo2 = P.abox[2];
  const int ahi0 = P.abox[3], ahi1 = P.abox[4], ahi2 = P.abox[5];
  uint32_t *myhist = hist + (wid % cfg.hist_copies) * cfg.hist_words;
  const uint32_t kind0 = P.kind[0], kind1 = P.kind[1];
  const uint8_t *binA0 = P.binA[0], *binA1 = P.binA[1];

  int lo0 = nx, lo1 = ny, lo2 = nz, hi0 = -1, hi1 = -1, hi2 = -1;
  unsigned long long nin = 0, nnear = 0;
  const int nbricks = P.nbx * P.nby;

  for (;;) {
    uint32_t bi = 0;
    if (lane == 0) bi = atomicAdd(next, 1u);
    bi = __builtin_amdgcn_readfirstlane(bi);
    if ((int)bi >= nbricks) break;
    const int bxi = (int)bi % P.nbx, byi = (int)bi / P.nbx;
    const int X0 = bxi * bx, X1 = min(X0 + bx, nx), Y0 = byi * by, Y1 = min(Y0 + by, ny);
    int c0 = (int)floor((double)X0 - cx - kColEps) - P.gx;
    int c1 = (int)floor((double)X1 - cx + kColEps) - P.gx;
    int r0 = (int)floor((double)Y0 - cy - kColEps) - P.gy;
    int r1 = (int)floor((double)Y1 - cy + kColEps) - P.gy;
    c0 = max(c0, 0); c1 = min(c1, P.ncx - 1);
    r0 = max(r0, 0); r1 = min(r1, P.ncy - 1);
    if (c1 < c0 || r1 < r0) continue;
    const int nrows = r1 - r0 + 1;
    uint32_t st = 0, len = 0;
    if (lane < nrows) {
      const uint32_t *orow = off + (int64_t)(r0 + lane) * P.ncx;
      st = orow[c0];
      len = orow[c1 + 1] - st;
    }
    uint32_t inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    const uint32_t total = __shfl(inc, nrows - 1, 64);
    if (total == 0) continue;
    if (lane < nrows) {
      rstart[lane] = st;
      rpre[lane] = inc - len;
    }
    wave_fence();

    int nocc = 0;
    for (uint32_t j0 = 0; j0 < total; j0 += 64) {
      const uint32_t j = j0 + lane;
      bool first = false;
      int loc = 0;
      if (j < total) {
        int lo = 0, hi = nrows - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rpre[mid] <= j) lo = mid; else hi = mid - 1;
        }
        const uint32_t idx = rstart[lo] + (j - rpre[lo]);
        const double ux = fvx[idx] + cx, uy = fvy[idx] + cy, uz = fvz[idx] + cz;
        const double fx = floor(ux), fy = floor(uy), fz = floor(uz);
        if (fx >= (double)X0 && fx < (double)X1 && fy >= (double)Y0 && fy < (double)Y1 &&
            fz >= 0.0 && fz < (double)nz) {
          const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
          loc = (iz * by + (iy - Y0)) * bx + (ix - X0);
          if (bpv == 4) {
            first = atomicAdd(&agg32[loc], 1u) == 0u;
          } else {
            const unsigned long long q = (unsigned long long)floor((uz - fz) * kQScale);
            const unsigned long long old = atomicAdd(&agg64[2 * loc], (1ull << 44) | q);
            atomicAdd(&agg64[2 * loc + 1], q * q);
            first = (old >> 44) == 0ull;
          }
          ++nin;
          lo0 = min(lo0, ix); lo1 = min(lo1, iy); lo2 = min(lo2, iz);
          hi0 = max(hi0, ix); hi1 = max(hi1, iy); hi2 = max(hi2, iz);
          if (NEAR && ix >= alo0 && ix <= ahi0 && iy >= alo1 && iy <= ahi1 && iz >= alo2 &&
              iz <= ahi2) {
            double d = 1.0;
            const double fr[3] = {ux - fx, uy - fy, uz - fz};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double up = 1.0 - fr[a];
              const double m = fr[a] < up ? fr[a] : up;
              if (m < d) d = m;
            }
            if (d * P.voxel < kNearFace) ++nnear;
          }
        }
      }
      const unsigned long long m = __ballot(first);
      if (first) {
        const int slot = nocc + (int)__builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        occ[slot] = (uint16_t)loc;
      }
      nocc += __popcll(m);
    }
    wave_fence();

    for (int i = lane; i < nocc; i += 64) {
      const int loc = occ[i];
      const int lx = loc % bx, t2 = loc / bx, ly = t2 % by, lz = t2 / by;
      const int ix = X0 + lx, iy = Y0 + ly, iz = lz;
      uint32_t n;
      unsigned long long s1 = 0, s2 = 0;
      if (bpv == 4) {
        n = agg32[loc];
        agg32[loc] = 0u;
      } else {
        const unsigned long long a = agg64[2 * loc];
        n = (uint32_t)(a >> 44);
        s1 = a & ((1ull << 44) - 1);
        s2 = agg64[2 * loc + 1];
        agg64[2 * loc] = 0ull;
        agg64[2 * loc + 1] = 0ull;
      }
      if (ix >= alo0 && ix <= ahi0 && iy >= alo1 && iy <= ahi1 && iz >= alo2 && iz <= ahi2) {
        const int64_t lin = ((int64_t)iz * ny + iy) * nx + ix;
        {
          const int a = binA0[lin];
          const int b = kind0 == MI_FEAT_COUNT ? bin_count_dev(n, nb0, cedge)
                                               : bin_zvar_dev(n, s1, s2, nb0, zedge);
          atomicAdd(&myhist[a * nb0 + b], 1u);
        }
        if (nf > 1) {
          const int a = binA1[lin];
          const int b = kind1 == MI_FEAT_COUNT ? bin_count_dev(n, nb1, cedge)
                                               : bin_zvar_dev(n, s1, s2, nb1, zedge);
          atomicAdd(&myhist[hoff1 + a * nb1 + b], 1u);
        }
      }
    }
    wave_fence();
  }

  // ---------------------------------------------------------- pose reduction
  lo0 = wave_min_i32(lo0); lo1 = wave_min_i32(lo1); lo2 = wave_min_i32(lo2);
  hi0 = wave_max_i32(hi0); hi1 = wave_max_i32(hi1); hi2 = wave_max_i32(hi2);
  nin = wave_sum_u64(nin);
  if (NEAR) nnear = wave_sum_u64(nnear);
  if (lane == 0) {
    int *b = wbox + 8 * wid;
    b[0] = lo0; b[1] = lo1; b[2] = lo2; b[3] = hi0; b[4] = hi1; b[5] = hi2;
    wcnt[2 * wid] = nin;
    wcnt[2 * wid + 1] = nnear;
  }
  __syncthreads();
  if (cfg.hist_copies > 1) {
    for (int i = tid; i < cfg.hist_words; i += blockDim.x) {
      uint32_t s = 0;
      for (int d = 1; d < cfg.hist_copies; ++d) s += hist[d * cfg.hist_words + i];
      hist[i] += s;
    }
  }
  int blo[3] = {nx, ny, nz}, bhi[3] = {-1, -1, -1};
  unsigned long long n_in = 0, n_near = 0;
  for (int w = 0; w < W; ++w) {
    const int *b = wbox + 8 * w;
    for (int a = 0; a < 3; ++a) {
      blo[a] = min(blo[a], b[a]);
      bhi[a] = max(bhi[a], b[3 + a]);
    }
    n_in += wcnt[2 * w];
    n_near += wcnt[2 * w + 1];
  }
  const int dims[3] = {nx, ny, nz};
  const int alo[3] = {alo0, alo1, alo2}, ahi[3] = {ahi0, ahi1, ahi2};
  int olo[3], ohi[3];
  bool nonempty = true;
  int64_t nO = 1;
  for (int a = 0; a < 3; ++a) {
    olo[a] = max(max(alo[a], blo[a]), 0);
    ohi[a] = min(min(ahi[a], bhi[a]), dims[a] - 1);
    if (ohi[a] < olo[a]) nonempty = false;
    else nO *= (int64_t)(ohi[a] - olo[a] + 1);
  }
  if (!nonempty) nO = 0;
  __syncthreads();

  if (nonempty) {
    const int64_t plane = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    for (int t = tid; t < nf * 64; t += blockDim.x) {
      const int f = t >> 6, a = t & 63;
      if (a >= 1 && a < P.nb[f])
        cntA[t] = sat_box(P.sat[f] + (int64_t)(a - 1) * plane, nx, ny, olo[0], olo[1], olo[2],
                          ohi[0], ohi[1], ohi[2]);
    }
  }
  __syncthreads();
  if (nonempty) {
    for (int t = tid; t < nf * 64; t += blockDim.x) {
      const int f = t >> 6, a = t & 63, nb = P.nb[f];
      if (a >= 1 && a < nb) {
        uint32_t *row = hist + (f ? hoff1 : 0) + a * nb;
        uint32_t rs = 0;
        for (int b = 1; b < nb; ++b) rs += row[b];
        row[0] = cntA[t] - rs;
      }
    }
  }
  __syncthreads();
  if (nonempty && tid < nf) {
    const int f = tid, nb = P.nb[f];
    uint32_t *H = hist + (f ? hoff1 : 0);
    int64_t rest = nO;
    for (int a = 1; a < nb; ++a) rest -= cntA[(f << 6) + a];
    for (int b = 1; b < nb; ++b) rest -= H[b];
    H[0] = (uint32_t)rest;
  }
  __syncthreads();

  if (wid < nf) {
    const int f = wid, nb = P.nb[f];
    const uint32_t *H = hist + (f ? hoff1 : 0);
    double hxy = 0.0, hx = 0.0, hy = 0.0;
    if (nonempty) {
      const double N = (double)nO;
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
    if (lane == 0) P.mi_out[(int64_t)f * P.K + pose.out_index] = nonempty ? (hx + hy) - hxy : 0.0;
    if (P.hist_out) {
      uint32_t *dst = P.hist_out + P.hist_off[f] + (int64_t)pose.out_index * nb * nb;
      for (int i = lane; i < nb * nb; i += 64) dst[i] = nonempty ? H[i] : 0u;
    }
  }
  if (P.stats_out && tid == 0) {
    mi_pose_stats st;
    for (int a = 0; a < 3; ++a) { st.lo[a] = olo[a]; st.hi[a] = ohi[a]; }
    const unsigned long long nnf = *P.nonfinite;
    st.n_overlap = nO;
    st.n_in_grid = (int64_t)n_in;
    st.n_nonfinite = (int64_t)nnf;
    st.n_out_of_grid = P.n_b - (int64_t)nnf - (int64_t)n_in;
    st.n_near_face = NEAR ? (int64_t)n_near : 0;
    P.stats_out[pose.out_index] = st;
  }
}

size_t eval_lds_bytes(const EvalLaunch &cfg) {
  return (size_t)misc_bytes_for(cfg.waves, cfg.hist_copies, cfg.hist_words) +
         (size_t)cfg.waves * cfg.wave_bytes;
}

int32_t eval_row_table_bytes() { return kRowTableBytes; }

hipError_t launch_eval(const PairDev *pairs_dev, const PoseDev *items_dev, int64_t n_items,
                       const EvalLaunch &cfg, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  EvalCfgDev c;
  c.hist_copies = cfg.hist_copies;
  c.hist_words = cfg.hist_words;
  c.wave_bytes = cfg.wave_bytes;
  c.misc_bytes = misc_bytes_for(cfg.waves, cfg.hist_copies, cfg.hist_words);
  const size_t lds = eval_lds_bytes(cfg);
  const int64_t per_xcd = (n_items + kXcds - 1) / kXcds;
  const int64_t grid = per_xcd * kXcds;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (cfg.near_face) {
    hipError_t e = hipFuncSetAttribute((const void *)k_eval<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_eval<true><<<(unsigned)grid, cfg.waves * 64, lds, s>>>(pairs_dev, items_dev, n_items,
                                                             per_xcd, c);
  } else {
    hipError_t e = hipFuncSetAttribute((const void *)k_eval<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_eval<false><<<(unsigned)grid, cfg.waves * 64, lds, s>>>(pairs_dev, items_dev, n_items,
                                                              per_xcd, c);
  }
  return hipGetLastError();
}

}  // namespace mi
