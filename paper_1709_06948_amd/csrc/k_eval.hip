// k_eval.hip -- MI of one candidate pose per workgroup (Eqs. 1-5, Alg. 1 loop
// body), on scan B's points already rotated once per distinct rotation.
//
// Ownership: A's grid is cut into bricks (pieces of stripes of stripe_h voxel
// rows, full height).  All waves of the workgroup work on one brick at a time
// and every B point that lands in the brick is aggregated there, so each
// voxel's sums (n, S1, S2) are complete in LDS without any merge across
// workgroups.  The sums live in an LDS hash keyed by the voxel (linear probing).
// Bricks are tried optimistically: a point whose probe sequence exceeds
// kMaxProbe slots (the table is close to full) marks the brick as overflowed;
// the brick is then cleared without touching the histogram and retried in
// halves; a single x piece is retried one voxel row at a time, whose voxels
// never exceed a quarter of the slots.
//
// Per pose:
//  plan   for a group of stripes, one parallel round of loads reads the column
//         offsets of every candidate row at the stripe's piece cuts, so brick
//         boundaries and candidate ranges are known without further round trips;
//  bricks the rest of the stripe first, halved on overflow;
//  points four consecutive candidates of a column row per lane per wave step,
//         branch-free: u = fl(v+c), voxel floor(u); runs of equal voxels among a
//         lane's four are added together; each in-brick run finds or claims its
//         voxel's slot with one compare-and-swap (all four in flight together),
//         newly claimed slots are appended to the brick's occupied list, and
//         n, S1, S2 are added with LDS atomics that return nothing;
//  sweep  every slot on the brick's occupied list: B's extent and point
//         count, and, for voxels inside A's index box (with B's extent this is
//         the overlap box), one count in the joint histogram at (A's bin, B's bin);
//  finish overlap box O; the cells of voxels that B leaves empty come from A's
//         per-bin summed-volume tables; entropies and MI.
#include <algorithm>

#include "mi_device.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

namespace mi {

static constexpr uint32_t kEmpty = 0xffffffffu;
static constexpr uint32_t kNever = 0xfffffffeu;  // never a key, never empty
static constexpr int kMaxProbe = 32;
static constexpr uint32_t kNoVoxel = 0xffffffffu;  // bucket entry of a point outside the grid

struct EvalCfgDev {
  int32_t hist_copies, hist_words;
  int32_t cap;                // voxel-hash slots
  int32_t load_max;           // voxels of a brick that is known to fit (a quarter of the slots)
  int32_t off_cnta, off_edges, off_wave, off_plan, off_hash, pad;
  int64_t xcd_start[kXcds + 1];  // items of XCD x: [xcd_start[x], xcd_start[x + 1])
};

struct Layout {
  int off_cnta, off_edges, off_wave, off_plan, off_hash, total;
};

__host__ __device__ inline int al16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline Layout eval_layout(int waves, int hist_copies, int hist_words,
                                              int plan_bytes, int cap, bool zvar) {
  Layout L;
  int o = al16(hist_copies * hist_words * 4);
  L.off_cnta = o;   o += 512;                   // cntA[2][64]
  L.off_edges = o;  o += 256 + 512 + 512;       // 64 u32 + 64 u64 + 64 f64 (finish: 2 x 66 f64)
  L.off_wave = o;   o += al16(waves * 48 + 16); // box [W][8] i32, counts [W][2] u64, flags
  L.off_plan = o;   o += al16(plan_bytes);
  o = (o + 255) & ~255;
  L.off_hash = o;   o += cap * (4 + (zvar ? 16 : 4)) + 2 * cap;  // keys, sums, occupied list
  L.total = al16(o);
  return L;
}

__device__ __forceinline__ int cut_x(int q, int nx, int Q) { return (int)(((int64_t)q * nx) / Q); }

// Column rows [r0, r0 + nrows) of the rotated cloud that can reach voxel rows [y0, y1).
__device__ __forceinline__ void rows_for(int y0, int y1, double cy, int gy, int ncy, int *r0,
                                         int *nrows) {
  int a = (int)floor((double)y0 - cy - kColEps) - gy;
  int b = (int)floor((double)y1 - cy + kColEps) - gy;
  a = max(a, 0);
  b = min(b, ncy - 1);
  *r0 = a;
  *nrows = b >= a ? b - a + 1 : 0;
}

// Voxel of point i of scan B under a pose (rotation of frame F, translation
// offset c): the same doubles as the rotated frames plus the offset,
// u = fl(fl(w * s) + c) with w = ((r0 x + r1 y) + r2 z).
struct DirectVoxel {
  int ix, iy, iz;
  uint32_t q;
  bool in;     // finite and inside the grid
  bool near;   // within kNearFace of a face (when asked for)
};

// (FINITE: the point is known to be finite, as every tile entry is)
template <bool ZVAR, bool NEAR, bool FINITE = false>
__device__ __forceinline__ DirectVoxel direct_voxel(float xf, float yf, float zf,
                                                    const double (&R)[9], double s, double cx,
                                                    double cy, double cz, int nx, int ny, int nz,
                                                    double voxel) {
  DirectVoxel r;
  r.in = false;
  r.near = false;
  r.q = 0u;
  r.ix = r.iy = r.iz = -1;
  if (!FINITE && (!isfinite(xf) || !isfinite(yf) || !isfinite(zf))) return r;
  const double x = xf, y = yf, z = zf;
  const double wx = (R[0] * x + R[1] * y) + R[2] * z;
  const double wy = (R[3] * x + R[4] * y) + R[5] * z;
  const double wz = (R[6] * x + R[7] * y) + R[8] * z;
  const double vx = wx * s, vy = wy * s, vz = wz * s;
  const double ux = vx + cx, uy = vy + cy, uz = vz + cz;
  const double fx = floor(ux), fy = floor(uy), fz = floor(uz);
  r.ix = (int)fx;
  r.iy = (int)fy;
  r.iz = (int)fz;
  r.in = (uint32_t)r.ix < (uint32_t)nx && (uint32_t)r.iy < (uint32_t)ny &&
         (uint32_t)r.iz < (uint32_t)nz;
  if (ZVAR) r.q = (uint32_t)floor((uz - fz) * kQScale);
  if (NEAR && r.in) {
    double d = 1.0;
    const double fr[3] = {ux - fx, uy - fy, uz - fz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double up = 1.0 - fr[a];
      const double m = fr[a] < up ? fr[a] : up;
      if (m < d) d = m;
    }
    r.near = d * voxel < kNearFace;
  }
  return r;
}

// Bit mixer (the MurmurHash3 finalizer) for splitting an overflowed tile's
// voxels into parts independently of their hash slots.
__device__ __forceinline__ uint32_t mix32(uint32_t k) {
  k ^= k >> 16;
  k *= 0x85ebca6bu;
  k ^= k >> 13;
  k *= 0xc2b2ae35u;
  k ^= k >> 16;
  return k;
}

// MODE 0: candidates come from the pose's rotated frame (points bucketed by
// column, shared by every pose with that rotation).
// MODE 1: the workgroup buckets its pose's points itself, by stripe, into its
// own slot of `scratch` (count, scan, scatter of (key, q) pairs), for pose
// sets whose rotations are (nearly) all distinct.
// MODE 2: for such pose sets, scan B comes bucketed into tiles of its own
// (x, y) frame, each followed by its halo (the neighbours' points within
// 0.88 voxel of it).  The workgroup takes the tiles one at a time, each as
// one brick keyed by whole-grid voxels, and keeps a voxel only in the tile
// that holds the voxel's centre mapped back into B's frame: a point of the
// voxel lies within half a voxel diagonal (0.866 voxel) of that centre, so
// the tile and its halo hold every point of every voxel it keeps.
template <bool NEAR, bool ZVAR, int MODE>
__global__ void __launch_bounds__(1024) k_eval(const PairDev *__restrict__ pairs,
                                               const FrameDev *__restrict__ frames,
                                               const PoseDev *__restrict__ items, EvalCfgDev cfg,
                                               uint2 *__restrict__ scratch,
                                               int64_t scratch_stride) {
  constexpr bool DIRECT = MODE == 1, TILED = MODE == 2;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, W = T >> 6;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint32_t *hist = (uint32_t *)smem;
  uint32_t *cntA = (uint32_t *)(smem + cfg.off_cnta);
  uint32_t *cedge = (uint32_t *)(smem + cfg.off_edges);
  uint64_t *zedge = (uint64_t *)(cedge + 64);
  double *zedged = (double *)(zedge + 64);
  int *wbox = (int *)(smem + cfg.off_wave);
  unsigned long long *wcnt = (unsigned long long *)(wbox + 8 * W);
  uint32_t *ovf = (uint32_t *)(wcnt + 2 * W);   // [2] overflow flags by brick parity
  uint32_t *occn = ovf + 2;                     // [2] occupied-slot counts by brick parity
  uint2 *plan = (uint2 *)(smem + cfg.off_plan);
  const int cap = cfg.cap;
  uint32_t *hkey = (uint32_t *)(smem + cfg.off_hash);
  unsigned long long *hv1 = (unsigned long long *)(hkey + cap);   // ZVAR: n<<44 | S1
  unsigned long long *hv2 = hv1 + cap;                            // ZVAR: S2
  uint32_t *hcnt = hkey + cap;                                    // count only
  uint16_t *occ = (uint16_t *)(hkey + cap * (ZVAR ? 5 : 2));      // slots in insertion order

  // The hash starts empty and every brick's sweep empties the slots it used,
  // so it is cleared once per workgroup.
  for (int i = tid; i < cap; i += T) {
    hkey[i] = kEmpty;
    if (ZVAR) { hv1[i] = 0ull; hv2[i] = 0ull; } else { hcnt[i] = 0u; }
  }

  // XCD-aware mapping: consecutive workgroup ids go round-robin over the XCDs,
  // and each XCD walks its own run of items (whole frames, so the frames it
  // reads stay in its L2).  A workgroup takes every (grid / 8)-th item of its
  // XCD's run: one item when the grid covers the longest run, several when
  // the grid is persistent.
  const int64_t xcd = blockIdx.x % kXcds, wpx = gridDim.x / kXcds;
  const int64_t x_end = cfg.xcd_start[xcd + 1];
  for (int64_t item = cfg.xcd_start[xcd] + blockIdx.x / kXcds; item < x_end; item += wpx) {
    const PoseDev pose = items[item];
    const PairDev &P = pairs[pose.pair];
    const FrameDev &Fr = frames[pose.frame];

    const int nx = P.nx, ny = P.ny, nz = P.nz, nf = P.nf;
    const int nb0 = P.nb[0], nb1 = nf > 1 ? P.nb[1] : 0;
    const int hoff1 = nb0 * nb0;

    for (int i = tid; i < cfg.hist_copies * cfg.hist_words; i += T) hist[i] = 0u;
    for (int i = tid; i < 64; i += T) {
      cedge[i] = P.count_edges[i];
      zedge[i] = P.zvar_edges[i];
      zedged[i] = (double)P.zvar_edges[i];
    }
    if (tid < 4) ovf[tid] = 0u;
    __syncthreads();

    const double cx = pose.c[0], cy = pose.c[1], cz = pose.c[2];
    const double *fvx = Fr.v;
    const double *fvy = fvx + Fr.n;
    const double *fvz = fvy + Fr.n;
    const int ncx = Fr.ncx, ncy = Fr.ncy, gx = Fr.gx, gy = Fr.gy;
    const uint32_t *off = Fr.off;
    const int alo0 = P.abox[0], alo1 = P.abox[1], alo2 = P.abox[2];
    const int ahi0 = P.abox[3], ahi1 = P.abox[4], ahi2 = P.abox[5];
    uint32_t *myhist = hist + (wid % cfg.hist_copies) * cfg.hist_words;
    const uint32_t kind0 = P.kind[0], kind1 = P.kind[1];
    const int nbc = P.nbc, nbz = P.nbz;
    const bool count_default = P.count_default != 0;
    const int zvar_zero = P.zvar_zero_edges;
    const uint8_t *binA0 = P.binA[0], *binA1 = P.binA[1];
    const uint32_t nvox = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;  // below 2^31
    const brsrc rbin0 = buf_rsrc(binA0, nvox), rbin1 = buf_rsrc(binA1, nf > 1 ? nvox : 0u);
    const int BY = P.stripe_h, NS = P.n_stripes, Q = P.pieces, RM = BY + 2;
    const int kxb = P.kx_bits, kyb = P.ky_bits;
    const uint32_t kxm = (1u << kxb) - 1u, kym = (1u << kyb) - 1u;
    const int G = DIRECT ? NS : P.plan_stripes;
    const int PE = RM * (Q + 1);  // plan entries per stripe

    int lo0 = nx, lo1 = ny, lo2 = nz, hi0 = -1, hi1 = -1, hi2 = -1;
    unsigned long long nin = 0, nnear = 0;
    int parity = 0;
    // Pieces a stripe's first brick spans: the span that last fitted, doubled
    // after a brick that used under a third of the slots and halved after one
    // that used over half (adapts to how many voxels the points fill, so that
    // overflow retries stay rare and probe sequences short).
    int span = 1 << 30;
    int last_occ = 0;

    // DIRECT: the pose's in-grid points bucketed by stripe into this
    // workgroup's scratch slot; soff[s] .. soff[s + 1] is stripe s.
    uint32_t *soff = (uint32_t *)plan;   // [NS + 1]
    uint32_t *scur = soff + NS + 1;      // [NS]
    uint2 *mine = DIRECT ? scratch + (int64_t)blockIdx.x * scratch_stride : nullptr;
    // this workgroup's buckets: (key, q) pairs, 8 bytes each (the stride is
    // below 2^28 entries in this form)
    const brsrc rmine = buf_rsrc(mine, DIRECT ? 8u * (uint32_t)scratch_stride : 0u);
    if (DIRECT) {
      double R[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) R[a] = Fr.R[a];
      const double fs = Fr.s;
      // scan B (fewer than 2^28 points in this form) through one buffer
      // resource: the coordinate arrays at scalar offsets 0, 4n and 8n
      const uint32_t nb32 = (uint32_t)Fr.n;
      const brsrc rxyz = buf_rsrc(Fr.xyz, 12u * nb32);
      const uint32_t oy = 4u * nb32, oz = 8u * nb32;

      // stripe of a voxel row, iy / BY, by a multiply-high where that is exact:
      // with m = ceil(2^32 / BY), m * BY - 2^32 < BY, so iy * m / 2^32 has the
      // quotient's integer part while iy * BY < 2^32 (any row below 2^26)
      const uint32_t by_mag = (uint32_t)(((1ull << 32) + (uint64_t)BY - 1ull) / (uint64_t)BY);
      const bool by_mul = BY > 1 && ny <= (1 << 26);  // (for BY = 1, m = 2^32 needs 33 bits)
      auto stripe_of = [&](int iy) -> uint32_t {
        return by_mul ? __umulhi((uint32_t)iy, by_mag) : (uint32_t)iy / (uint32_t)BY;
      };
      for (int i = tid; i < NS; i += T) scur[i] = 0u;
      __syncthreads();
      // Count pass: only the y row of the transform decides the stripe.  Four
      // points per lane are loaded before any is used, so a wave waits on
      // memory once per four points.
      for (uint32_t i0 = (uint32_t)tid; i0 < nb32; i0 += 4u * (uint32_t)T) {
        float fx[4], fy[4], fz[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + (uint32_t)j * (uint32_t)T;  // past the end: reads 0
          fx[j] = buf_f32(rxyz, 4u * i, 0u);
          fy[j] = buf_f32(rxyz, 4u * i, oy);
          fz[j] = buf_f32(rxyz, 4u * i, oz);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + (uint32_t)j * (uint32_t)T;
          if (i < nb32 && isfinite(fx[j]) && isfinite(fy[j]) && isfinite(fz[j])) {
            const double x = fx[j], y = fy[j], z = fz[j];
            const double uy = ((R[3] * x + R[4] * y) + R[5] * z) * fs + cy;
            const int iy = (int)floor(uy);
            if ((uint32_t)iy < (uint32_t)ny) atomicAdd(&scur[stripe_of(iy)], 1u);
          }
        }
      }
      __syncthreads();
      if (wid == 0) {  // exclusive scan of the stripe counts
        uint32_t run = 0;
        for (int b = 0; b < NS; b += 64) {
          const uint32_t c = b + lane < NS ? scur[b + lane] : 0u;
          uint32_t inc = c;
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
          }
          if (b + lane < NS) {
            soff[b + lane] = run + inc - c;
            scur[b + lane] = run + inc - c;
          }
          run += __shfl(inc, 63, 64);
        }
        if (lane == 0) soff[NS] = run;
      }
      __syncthreads();
      // Scatter pass: the whole voxel.  Every point counted above gets an entry
      // in its stripe's bucket; one outside the grid in x or z is marked by
      // q = kNoVoxel and skipped by the bricks.
      for (uint32_t i0 = (uint32_t)tid; i0 < nb32; i0 += 4u * (uint32_t)T) {
        float fx[4], fy[4], fz[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + (uint32_t)j * (uint32_t)T;  // past the end: reads 0
          fx[j] = buf_f32(rxyz, 4u * i, 0u);
          fy[j] = buf_f32(rxyz, 4u * i, oy);
          fz[j] = buf_f32(rxyz, 4u * i, oz);
        }
        uint32_t pos[4], key[4], qv[4];
        bool put[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + (uint32_t)j * (uint32_t)T;
          const DirectVoxel dv = direct_voxel<ZVAR, NEAR>(fx[j], fy[j], fz[j], R, fs, cx, cy, cz,
                                                           nx, ny, nz, P.voxel);
          put[j] = i < nb32 && (uint32_t)dv.iy < (uint32_t)ny;
          pos[j] = 0u;
          key[j] = 0u;
          qv[j] = kNoVoxel;
          if (put[j]) {
            const uint32_t st = stripe_of(dv.iy);
            pos[j] = atomicAdd(&scur[st], 1u);
            if (dv.in) {
              key[j] = ((uint32_t)dv.iz << (kxb + kyb)) | ((uint32_t)(dv.iy - (int)st * BY) << kxb) |
                       (uint32_t)dv.ix;
              qv[j] = dv.q;
              if (NEAR && dv.near && dv.ix >= alo0 && dv.ix <= ahi0 && dv.iy >= alo1 &&
                  dv.iy <= ahi1 && dv.iz >= alo2 && dv.iz <= ahi2)
                ++nnear;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (put[j]) buf_store_u32x2((u32x2){key[j], qv[j]}, rmine, 8u * pos[j]);
      }
      __syncthreads();
    }

    // Four candidates per lane, branch-free up to the rare collisions:
    // find or claim each in-brick candidate's slot, then add its sums.
    // (p: the brick's parity, whose overflow flag and occupied count it uses;
    // max_probe: slots a probe sequence may visit before the brick overflows)
    auto insert4 = [&](bool (&inb)[4], const uint32_t (&key)[4],
                       const unsigned long long (&add1)[4],
                       const unsigned long long (&add2)[4], const int p, const int max_probe) {
      uint32_t h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = __umulhi(key[i] * 2654435761u, (uint32_t)cap);
      bool coll[4], fresh[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // one compare-and-swap finds or claims the home slot (only lanes
        // holding a run issue it)
        uint32_t old = kEmpty;
        if (inb[i]) old = atomicCAS(&hkey[h[i]], kEmpty, key[i]);
        fresh[i] = inb[i] && old == kEmpty;
        coll[i] = inb[i] && old != kEmpty && old != key[i];
      }
      if (coll[0] || coll[1] || coll[2] || coll[3]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (!coll[i]) continue;
          uint32_t hh = h[i];
          bool ok = false;
          for (int pr = 1; pr < max_probe; ++pr) {
            hh = hh + 1u == (uint32_t)cap ? 0u : hh + 1u;
            uint32_t k1 = __atomic_load_n(&hkey[hh], __ATOMIC_RELAXED);
            if (k1 == kEmpty) {
              k1 = atomicCAS(&hkey[hh], kEmpty, key[i]);
              if (k1 == kEmpty) fresh[i] = true;
            }
            if (k1 == kEmpty || k1 == key[i]) { ok = true; break; }
          }
          if (ok) h[i] = hh;
          else { ovf[p] = 1u; inb[i] = false; }
        }
      }
      // newly claimed slots go on the brick's occupied list (one LDS atomic per wave)
      {
        unsigned long long m[4];
        uint32_t tot = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          m[i] = __ballot(fresh[i]);
          tot += (uint32_t)__popcll(m[i]);
        }
        if (tot) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&occn[p], tot);
          base = __builtin_amdgcn_readfirstlane(base);  // every lane is active here
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (fresh[i]) {
              const uint32_t r = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(m[i] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[i], 0u));
              occ[base + r] = (uint16_t)h[i];
            }
            base += (uint32_t)__popcll(m[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (inb[i]) {
          if (ZVAR) {
            atomicAdd(&hv1[h[i]], add1[i]);
            atomicAdd(&hv2[h[i]], add2[i]);
          } else {
            atomicAdd(&hcnt[h[i]], (uint32_t)add1[i]);
          }
        }
      }
    };
    // One voxel of B in O: a count in each feature's joint histogram at
    // (A's bin, B's bin) from the voxel's sums n, S1, S2.
    auto hist_add = [&](const uint32_t nn, const unsigned long long s1,
                        const unsigned long long s2, const int a0, const int a1) {
      // count bins: O(1) with the default edges 1, 2, ..., nb - 1; the joint
      // feature numbers its (count, z-variance) bin pairs
      auto count_bin = [&]() -> int {
        return count_default ? (int)min(nn, (uint32_t)(nbc - 1)) : bin_count_dev(nn, nbc, cedge);
      };
      auto bin_of = [&](uint32_t kind) -> int {
        if (kind == MI_FEAT_COUNT || !ZVAR) return count_bin();
        // one point has zero variance: 1 + the number of zero edges
        const int bz = nn == 1u ? 1 + zvar_zero : bin_zvar_nodiv(nn, s1, s2, nbz, zedged, zedge);
        if (kind == MI_FEAT_ZVAR) return bz;
        return joint_value(count_bin(), bz, nbz);
      };
      atomicAdd(&myhist[a0 * nb0 + bin_of(kind0)], 1u);
      if (nf > 1) atomicAdd(&myhist[hoff1 + a1 * nb1 + bin_of(kind1)], 1u);
    };

    if (TILED) {
      double R[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) R[a] = Fr.R[a];
      const double fs = Fr.s, vox = P.voxel;
      const int tnx = P.tile_nx, tny = P.tile_ny, ntiles = tnx * tny;
      const double tx0 = P.tile_x0, ty0 = P.tile_y0, tilx = P.tile_ilx, tily = P.tile_ily;
      const int qxb = P.key_xbits, qyb = P.key_ybits;
      const uint32_t qxm = (1u << qxb) - 1u, qym = (1u << qyb) - 1u;
      // the tiles' points through one buffer resource (below 2^28 entries):
      // x, y and z arrays at scalar offsets 0, 4 * stride and 8 * stride
      const uint32_t ts = (uint32_t)P.tile_stride;
      const brsrc rt = buf_rsrc(P.tile_xyz, 12u * ts);
      const uint32_t toy = 4u * ts, toz = 8u * ts;
      for (int t = 0; t < ntiles; ++t) {
        const uint32_t tst = P.tile_off[t], ten = P.tile_off[t + 1], town = P.tile_own[t];
        if (ten == tst) continue;
        const int ti = t % tnx, tj = t / tnx;
        // A tile that overflows the hash is redone in parts: part (lvl, idx)
        // takes the voxels whose mixed key has idx in its top lvl bits, and
        // splits into (lvl + 1, 2 idx) and (lvl + 1, 2 idx + 1); parts are taken
        // depth first.  From lvl 2 on, probing is unlimited, so a part only
        // overflows if its voxels exceed the slots.
        int lvl = 0;
        uint32_t part = 0;
        for (;;) {
          const int p = parity;
          const int max_probe =
              ((int64_t)(ten - tst) <= cfg.load_max || lvl >= 2) ? cap : kMaxProbe;
          unsigned long long bnear = 0;
          // 256 consecutive entries per wave step, four per lane, 64 apart; the
          // next step's loads are issued before this step's points are hashed
          float nxf[4], nyf[4], nzf[4];
          auto load4 = [&](uint32_t b, float (&ox)[4], float (&oy)[4], float (&oz)[4]) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t idx = b + (uint32_t)j * 64u + (uint32_t)lane;
              const uint32_t e = idx < ten ? idx : tst;
              ox[j] = buf_f32(rt, 4u * e, 0u);
              oy[j] = buf_f32(rt, 4u * e, toy);
              oz[j] = buf_f32(rt, 4u * e, toz);
            }
          };
          const uint32_t bstep = 256u * (uint32_t)W;
          if (tst + (uint32_t)wid * 256u < ten) load4(tst + (uint32_t)wid * 256u, nxf, nyf, nzf);
          for (uint32_t b = tst + (uint32_t)wid * 256u; b < ten; b += bstep) {
            float fx[4], fy[4], fz[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              fx[j] = nxf[j];
              fy[j] = nyf[j];
              fz[j] = nzf[j];
            }
            if (b + bstep < ten) load4(b + bstep, nxf, nyf, nzf);
            bool inb[4];
            uint32_t key[4];
            unsigned long long add1[4], add2[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t idx = b + (uint32_t)j * 64u + (uint32_t)lane;
              const DirectVoxel dv = direct_voxel<ZVAR, NEAR, true>(fx[j], fy[j], fz[j], R, fs, cx,
                                                                     cy, cz, nx, ny, nz, vox);
              key[j] = ((uint32_t)dv.iz << (qxb + qyb)) | ((uint32_t)dv.iy << qxb) |
                       (uint32_t)dv.ix;
              inb[j] = idx < ten && dv.in &&
                       (lvl == 0 || (mix32(key[j]) >> (32 - lvl)) == part);
              add1[j] = ZVAR ? ((1ull << 44) | (unsigned long long)dv.q) : 1ull;
              add2[j] = ZVAR ? (unsigned long long)dv.q * dv.q : 0ull;
              // a point is tallied once: in its own tile, in its voxel's part
              if (NEAR && inb[j] && idx < town && dv.near && dv.ix >= alo0 && dv.ix <= ahi0 &&
                  dv.iy >= alo1 && dv.iy <= ahi1 && dv.iz >= alo2 && dv.iz <= ahi2)
                ++bnear;
            }
            insert4(inb, key, add1, add2, p, max_probe);
          }
          __syncthreads();
          const bool overflow = ovf[p] != 0u;
          const int nocc = (int)occn[p];
          if (tid == 0) { ovf[p ^ 1] = 0u; occn[p ^ 1] = 0u; }
          int blo0 = nx, blo1 = ny, blo2 = nz, bhi0 = -1, bhi1 = -1, bhi2 = -1;
          unsigned long long bnin = 0;
          for (int i = tid; i < nocc; i += 2 * T) {
            bool inO[2];
            uint32_t n[2], lin[2];
            unsigned long long s1[2], s2[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const int ii = i + j * T;
              inO[j] = false;
              n[j] = 0u;
              s1[j] = s2[j] = 0ull;
              lin[j] = 0u;
              if (ii >= nocc) continue;
              const uint32_t h = occ[ii];
              const uint32_t key = hkey[h];
              const int ix = (int)(key & qxm), iy = (int)((key >> qxb) & qym);
              const int iz = (int)(key >> (qxb + qyb));
              if (ZVAR) {
                const unsigned long long a = hv1[h];
                n[j] = (uint32_t)(a >> 44);
                s1[j] = a & ((1ull << 44) - 1);
                s2[j] = hv2[h];
                hv1[h] = 0ull;
                hv2[h] = 0ull;
              } else {
                n[j] = hcnt[h];
                hcnt[h] = 0u;
              }
              hkey[h] = kEmpty;
              // the voxel's owner: the tile holding its centre mapped back into
              // B's frame, R^T ((centre - c) voxel)
              const double dx = ((double)ix + 0.5 - cx) * vox;
              const double dy = ((double)iy + 0.5 - cy) * vox;
              const double dz = ((double)iz + 0.5 - cz) * vox;
              const double bx = (R[0] * dx + R[3] * dy) + R[6] * dz;
              const double by = (R[1] * dx + R[4] * dy) + R[7] * dz;
              const int oi = min(max((int)floor((bx - tx0) * tilx), 0), tnx - 1);
              const int oj = min(max((int)floor((by - ty0) * tily), 0), tny - 1);
              if (overflow || oi != ti || oj != tj) continue;
              bnin += n[j];
              blo0 = min(blo0, ix); blo1 = min(blo1, iy); blo2 = min(blo2, iz);
              bhi0 = max(bhi0, ix); bhi1 = max(bhi1, iy); bhi2 = max(bhi2, iz);
              inO[j] = ix >= alo0 && ix <= ahi0 && iy >= alo1 && iy <= ahi1 && iz >= alo2 &&
                       iz <= ahi2;
              lin[j] = ((uint32_t)iz * (uint32_t)ny + (uint32_t)iy) * (uint32_t)nx + (uint32_t)ix;
            }
            int a0[2], a1[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              a0[j] = inO[j] ? (int)buf_u8(rbin0, lin[j]) : 0;
              a1[j] = inO[j] && nf > 1 ? (int)buf_u8(rbin1, lin[j]) : 0;
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
              if (inO[j]) hist_add(n[j], s1[j], s2[j], a0[j], a1[j]);
          }
          __syncthreads();
          parity ^= 1;
          if (overflow) {
            ++lvl;
            part <<= 1;
            continue;
          }
          nin += bnin;
          nnear += bnear;
          lo0 = min(lo0, blo0); lo1 = min(lo1, blo1); lo2 = min(lo2, blo2);
          hi0 = max(hi0, bhi0); hi1 = max(hi1, bhi1); hi2 = max(hi2, bhi2);
          // next part, depth first
          ++part;
          while (lvl > 0 && (part & 1u) == 0u) {
            part >>= 1;
            --lvl;
          }
          if (lvl == 0) break;
        }
      }
    }

    for (int s0 = 0; !TILED && s0 < NS; s0 += G) {
      const int gn = min(G, NS - s0);
      // ---- plan: offsets of every candidate row at every piece cut
      for (int e = tid; !DIRECT && e < gn * PE; e += T) {
        const int q = e % (Q + 1);
        const int t1 = e / (Q + 1);
        const int r = t1 % RM, sl = t1 / RM;
        const int Y0 = (s0 + sl) * BY, Y1 = min(Y0 + BY, ny);
        int r0, nrows;
        rows_for(Y0, Y1, cy, gy, ncy, &r0, &nrows);
        uint2 v = make_uint2(0u, 0u);
        if (r < nrows) {
          int K = (int)floor((double)cut_x(q, nx, Q) - cx - kColEps) - gx;
          K = min(max(K, 0), ncx - 1);
          const uint32_t *orow = off + (int64_t)(r0 + r) * ncx;
          v.x = ldg(orow + K);
          v.y = ldg(orow + min(K + 2, ncx));
        }
        plan[sl * PE + r * (Q + 1) + q] = v;
      }
      if (!DIRECT) __syncthreads();

      // ---- bricks of each stripe (every thread takes the same decisions)
      for (int sl = 0; sl < gn; ++sl) {
        const int SY0 = (s0 + sl) * BY, SY1 = min(SY0 + BY, ny);
        int sr0 = 0, snrows = 0;
        uint32_t bst = 0, bend = 0;  // DIRECT: the stripe's bucket
        if (DIRECT) {
          bst = soff[s0 + sl];
          bend = soff[s0 + sl + 1];
          if (bend == bst) continue;
        } else {
          rows_for(SY0, SY1, cy, gy, ncy, &sr0, &snrows);
          if (snrows <= 0) continue;
        }
        const uint2 *ps = plan + sl * PE;
        int qa = 0;
        while (qa < Q) {
          int qe = qa + min(span, Q - qa);
          for (;;) {
            const bool whole = qe > qa;  // false: piece qa voxel row by voxel row
            const int qend = whole ? qe : qa + 1;
            const int X0 = cut_x(qa, nx, Q), X1 = cut_x(qend, nx, Q);
            const int nsub = whole ? 1 : (SY1 - SY0);
            bool all_ok = true;
            for (int sub = 0; sub < nsub; ++sub) {
              const int Y0 = whole ? SY0 : SY0 + sub, Y1 = whole ? SY1 : Y0 + 1;
              int ra = 0, nr = snrows;
              if (!whole && !DIRECT) {
                int rr0, rn;
                rows_for(Y0, Y1, cy, gy, ncy, &rr0, &rn);
                ra = rr0 - sr0;
                nr = rn;
              }
              // this brick's candidate rows, one per lane: start, length, chunk prefix
              uint32_t my_st = 0, my_len = 0;
              if (lane < nr) {
                my_st = ps[(ra + lane) * (Q + 1) + qa].x;
                my_len = ps[(ra + lane) * (Q + 1) + qend].y - my_st;
              }
              const uint32_t my_c = (my_len + 255u) >> 8;
              uint32_t inc = my_c;
  #pragma unroll
              for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
              }
              const uint32_t my_cpre = inc - my_c;
              // A brick of the whole stripe reads its rows' candidates as one
              // contiguous range (between two rows lie only columns outside the
              // grid's x range), cut into chunks of 256 without per-row padding.
              const bool contig = !DIRECT && whole && qa == 0 && qend == Q && nr > 0;
              uint32_t cs = 0, ce = 0;
              if (contig) {
                cs = ps[ra * (Q + 1)].x;
                ce = ps[(ra + nr - 1) * (Q + 1) + Q].y;
                if (ce < cs) ce = cs;
              }
              const int nch = DIRECT ? (int)((bend - bst + 63u) >> 6)
                              : contig ? (int)((ce - cs + 255u) >> 8)
                                       : (nr > 0 ? (int)__shfl(inc, nr - 1, 64) : 0);
              if (nch == 0) continue;
              const int p = parity;
              unsigned long long bnear = 0;
              // a brick with at most a quarter of the slots in voxels always has an
              // empty slot: it probes without limit and cannot overflow (single
              // voxel rows of a piece are always such bricks)
              const bool fits = (int64_t)(X1 - X0) * (Y1 - Y0) * nz <= cfg.load_max;
              const int max_probe = fits ? cap : kMaxProbe;
              // chunk k -> this lane's 4 consecutive candidates.  A row of len
              // candidates takes ceil(len/256) chunks; in chunk j of the row, lane l
              // takes candidates 256j + 4l .. 256j + 4l + 3.  Consecutive candidates
              // of a column often share a voxel (ground), and a lane adds a run of
              // equal voxels with one set of atomics.  Returns the first index
              // (the row start for lanes past the row's end, whose candidates are
              // all invalid) and how many of the 4 are in the row.
              auto chunk_base = [&](int k, int *n_valid) -> uint32_t {
                const unsigned long long mk = __ballot(lane < nr && my_cpre <= (uint32_t)k);
                const int row = __popcll(mk) - 1;
                const uint32_t st = __builtin_amdgcn_readlane(my_st, row);
                const uint32_t len = __builtin_amdgcn_readlane(my_len, row);
                const uint32_t cpre = __builtin_amdgcn_readlane(my_cpre, row);
                const uint32_t off0 = (((uint32_t)k - cpre) << 8) + 4u * (uint32_t)lane;
                const int rem = (int)len - (int)off0;
                *n_valid = rem;
                return rem > 0 ? st + off0 : st;
              };
              // Frame candidates: u = fl(v + c), voxel floor(u), in-brick test.
              auto step4 = [&](const bool (&val)[4], const double (&vx)[4], const double (&vy)[4],
                               const double (&vz)[4]) {
                bool inb[4];
                uint32_t key[4], q[4];
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const double ux = vx[i] + cx, uy = vy[i] + cy, uz = vz[i] + cz;
                  const double fx = floor(ux), fy = floor(uy), fz = floor(uz);
                  // v_cvt_i32_f64 saturates, so far-away points stay out of range
                  const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
                  inb[i] = val[i] && (uint32_t)(ix - X0) < (uint32_t)(X1 - X0) &&
                           (uint32_t)(iy - Y0) < (uint32_t)(Y1 - Y0) && (uint32_t)iz < (uint32_t)nz;
                  key[i] = ((uint32_t)iz << (kxb + kyb)) | ((uint32_t)(iy - SY0) << kxb) |
                           (uint32_t)ix;
                  // uz - fz is in [0, 1), so truncation is the floor
                  q[i] = ZVAR ? (uint32_t)((uz - fz) * kQScale) : 0u;
                  if (NEAR && inb[i] && ix >= alo0 && ix <= ahi0 && iy >= alo1 && iy <= ahi1 &&
                      iz >= alo2 && iz <= ahi2) {
                    double d = 1.0;
                    const double fr[3] = {ux - fx, uy - fy, uz - fz};
  #pragma unroll
                    for (int a = 0; a < 3; ++a) {
                      const double up = 1.0 - fr[a];
                      const double m = fr[a] < up ? fr[a] : up;
                      if (m < d) d = m;
                    }
                    if (d * P.voxel < kNearFace) ++bnear;
                  }
                }
                // runs of equal voxels among the 4 consecutive candidates: the
                // first of a run adds the whole run's n, S1, S2
                unsigned long long add1[4], add2[4];
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  add1[i] = ZVAR ? ((1ull << 44) | (unsigned long long)q[i]) : 1ull;
                  add2[i] = ZVAR ? (unsigned long long)q[i] * q[i] : 0ull;
                }
                bool same[4];
                same[0] = false;
  #pragma unroll
                for (int i = 1; i < 4; ++i) same[i] = inb[i] && inb[i - 1] && key[i] == key[i - 1];
  #pragma unroll
                for (int i = 2; i >= 0; --i) {
                  add1[i] += same[i + 1] ? add1[i + 1] : 0ull;
                  add2[i] += same[i + 1] ? add2[i + 1] : 0ull;
                }
  #pragma unroll
                for (int i = 1; i < 4; ++i) inb[i] = inb[i] && !same[i];
                insert4(inb, key, add1, add2, p, max_probe);
              };
              // Four chunks per wave step: the twelve loads are issued together, then
              // the four candidates of each lane go through step4 together.  Lanes
              // past a row's end load index 0 (always valid) and are masked off.
              for (int k = wid; DIRECT && k < nch; k += 4 * W) {
                // bucketed (key, q) pairs of the stripe, 64 consecutive per chunk
                bool inb[4];
                uint32_t key[4], q[4];
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const uint32_t idx = bst + (uint32_t)(k + i * W) * 64u + (uint32_t)lane;
                  const bool val = k + i * W < nch && idx < bend;
                  const u32x2 e = buf_u32x2(rmine, 8u * (val ? idx : bst));
                  key[i] = e.x;
                  q[i] = e.y;
                }
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const uint32_t idx = bst + (uint32_t)(k + i * W) * 64u + (uint32_t)lane;
                  const bool val = k + i * W < nch && idx < bend;
                  const int ix = (int)(key[i] & kxm);
                  const int iy = SY0 + (int)((key[i] >> kxb) & kym);
                  inb[i] = val && q[i] != kNoVoxel && (uint32_t)(ix - X0) < (uint32_t)(X1 - X0) &&
                           (uint32_t)(iy - Y0) < (uint32_t)(Y1 - Y0);
                }
                unsigned long long add1[4], add2[4];
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  add1[i] = ZVAR ? ((1ull << 44) | (unsigned long long)q[i]) : 1ull;
                  add2[i] = ZVAR ? (unsigned long long)q[i] * q[i] : 0ull;
                }
                insert4(inb, key, add1, add2, p, max_probe);
              }
              for (int k = wid; !DIRECT && k < nch; k += W) {
                int nv;
                uint32_t b;
                if (contig) {
                  const uint32_t b0 = cs + ((uint32_t)k << 8) + 4u * (uint32_t)lane;
                  nv = (int)ce - (int)b0;
                  b = nv > 0 ? b0 : cs;
                } else {
                  b = chunk_base(k, &nv);
                }
                bool v[4];
                double x[4], y[4], z[4];
                // the frame arrays are padded, so base + 3 is always readable
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  v[i] = i < nv;
                  x[i] = ldg(fvx + b + i);
                  y[i] = ldg(fvy + b + i);
                  z[i] = ldg(fvz + b + i);
                }
                step4(v, x, y, z);
              }
              __syncthreads();
              const bool overflow = ovf[p] != 0u;
              const int nocc = (int)occn[p];
              last_occ = nocc;
              if (tid == 0) { ovf[p ^ 1] = 0u; occn[p ^ 1] = 0u; }
              int blo0 = nx, blo1 = ny, blo2 = nz, bhi0 = -1, bhi1 = -1, bhi2 = -1;
              unsigned long long bnin = 0;
              // Two slots per thread per round: both slots' LDS reads, then both
              // voxels' A-bin gathers, are in flight together.
              for (int i = tid; i < nocc; i += 2 * T) {
                bool live[2], inO[2];
                uint32_t n[2];
                unsigned long long s1[2], s2[2];
                uint32_t lin[2];  // a grid has fewer than 2^31 voxels
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                  const int ii = i + j * T;
                  live[j] = ii < nocc;
                  inO[j] = false;
                  n[j] = 0u;
                  s1[j] = s2[j] = 0ull;
                  lin[j] = 0u;
                  if (!live[j]) continue;
                  const uint32_t h = occ[ii];
                  const uint32_t key = hkey[h];
                  const int ix = (int)(key & kxm);
                  const int iy = SY0 + (int)((key >> kxb) & kym);
                  const int iz = (int)(key >> (kxb + kyb));
                  if (ZVAR) {
                    const unsigned long long a = hv1[h];
                    n[j] = (uint32_t)(a >> 44);
                    s1[j] = a & ((1ull << 44) - 1);
                    s2[j] = hv2[h];
                    hv1[h] = 0ull;
                    hv2[h] = 0ull;
                  } else {
                    n[j] = hcnt[h];
                    hcnt[h] = 0u;
                  }
                  hkey[h] = kEmpty;
                  bnin += n[j];
                  blo0 = min(blo0, ix); blo1 = min(blo1, iy); blo2 = min(blo2, iz);
                  bhi0 = max(bhi0, ix); bhi1 = max(bhi1, iy); bhi2 = max(bhi2, iz);
                  inO[j] = !overflow && ix >= alo0 && ix <= ahi0 && iy >= alo1 && iy <= ahi1 &&
                           iz >= alo2 && iz <= ahi2;
                  lin[j] = ((uint32_t)iz * (uint32_t)ny + (uint32_t)iy) * (uint32_t)nx + (uint32_t)ix;
                }
                int a0[2], a1[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                  a0[j] = inO[j] ? (int)buf_u8(rbin0, lin[j]) : 0;
                  a1[j] = inO[j] && nf > 1 ? (int)buf_u8(rbin1, lin[j]) : 0;
                }
#pragma unroll
                for (int j = 0; j < 2; ++j)
                  if (inO[j]) hist_add(n[j], s1[j], s2[j], a0[j], a1[j]);
              }
              __syncthreads();
              parity ^= 1;
              if (overflow) {
                all_ok = false;
                break;
              }
              nin += bnin;
              nnear += bnear;
              lo0 = min(lo0, blo0); lo1 = min(lo1, blo1); lo2 = min(lo2, blo2);
              hi0 = max(hi0, bhi0); hi1 = max(hi1, bhi1); hi2 = max(hi2, bhi2);
            }
            if (all_ok) {
              if (whole) {
                span = qend - qa;
                if (3 * last_occ < cap) span = min(2 * span, Q);
                else if (2 * last_occ > cap) span = max(span / 2, 1);
              }
              qa = qend;
              break;
            }
            // overflow: halve the run of pieces; a single piece goes row by row
            qe = qe - qa > 1 ? qa + (qe - qa) / 2 : qa;
          }
        }
      }
      __syncthreads();
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
      for (int i = tid; i < cfg.hist_words; i += T) {
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
      for (int t = tid; t < nf * 64; t += T) {
        const int f = t >> 6, a = t & 63;
        if (a >= 1 && a < P.nb[f]) {
          const SatLayout &L = P.sat_layout[f];
          cntA[t] = sat_has_table(L, a)
                        ? sat_box(P.sat[f] + sat_offset(L, a, plane), sat_width(L, a), nx, ny,
                                  olo[0], olo[1], olo[2], ohi[0], ohi[1], ohi[2])
                        : 0u;
        }
      }
    }
    __syncthreads();
    // A's voxels of the bins kept as a list: count those inside O.  A thread
    // loads 8 entries before it tests any.  The list is grouped by bin, so a
    // wave's entries mostly share one; it then adds them with one atomic.
    if (nonempty && P.alist_n) {
      const uint32_t n = P.alist_n;
      for (uint32_t e0 = tid; e0 < n; e0 += 8u * T) {
        uint64_t q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t e = e0 + (uint32_t)k * T;
          q[k] = e < n ? ldg(P.alist + e) : ~0ull;  // ~0: past the end
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (e0 + (uint32_t)k * T >= n) break;  // the rest of this thread's entries are past it too
          const int x = (int)(q[k] & 0xFFFFFu), y = (int)((q[k] >> 20) & 0xFFFFFu);
          const int z = (int)((q[k] >> 40) & 0xFFFFu), fa = (int)(q[k] >> 56);
          const bool in = x >= olo[0] && x <= ohi[0] && y >= olo[1] && y <= ohi[1] &&
                          z >= olo[2] && z <= ohi[2];
          const int first = __ffsll((unsigned long long)__ballot(1)) - 1;  // first active lane
          const int fa0 = __shfl(fa, first, 64);
          const uint64_t inm = __ballot(in), mixed = __ballot(in && fa != fa0);
          if (mixed == 0) {
            if (inm && lane == first) atomicAdd(&cntA[fa0], (uint32_t)__popcll(inm));
          } else if (in) {
            atomicAdd(&cntA[fa], 1u);
          }
        }
      }
      __syncthreads();
    }
    // Cells of voxels empty in B (integers, exact in any order), one wave per
    // row with the lanes over the columns: H[a][0] = (A's voxels of bin a in
    // O) - sum_{b>=1} H[a][b] for a >= 1, and H[0][0] = |O| - sum_{a>=1} (A's
    // voxels of bin a in O) - sum_{b>=1} H[0][b].
    if (nonempty) {
      for (int r = wid; r < nf * 64; r += W) {
        const int f = r >> 6, a = r & 63, nb = f ? nb1 : nb0;
        if (a >= nb) continue;
        uint32_t *H = hist + (f ? hoff1 : 0);
        const bool col = lane >= 1 && lane < nb;
        if (a >= 1) {
          const unsigned long long rs =
              wave_sum_u64(col ? (unsigned long long)H[a * nb + lane] : 0ull);
          if (lane == 0) H[a * nb] = cntA[r] - (uint32_t)rs;
        } else {
          const unsigned long long s = wave_sum_u64(
              col ? (unsigned long long)cntA[(f << 6) + lane] + H[lane] : 0ull);
          if (lane == 0) H[0] = (uint32_t)(nO - (int64_t)s);
        }
      }
    }
    __syncthreads();

    // Entropies (Eqs. 2-5) in a fixed order that does not depend on the launch
    // shape: H(X,Y) as wave sums over 64-cell chunks of the histogram, then a
    // wave sum over the chunks; H(X) and H(Y) as wave sums over the rows' and
    // columns' terms.  The tasks are spread over the waves; their results go to
    // the bin-edge area of LDS, which the next item loads afresh.
    double *part = (double *)cedge;  // [feature][66]: chunks, then H(X), H(Y)
    const int ch0 = (nb0 * nb0 + 63) >> 6, ch1 = (nb1 * nb1 + 63) >> 6;
    if (nonempty) {
      const double N = (double)nO;
      const int ntask = ch0 + 2 + (nf > 1 ? ch1 + 2 : 0);
      for (int k = wid; k < ntask; k += W) {
        const int f = k < ch0 + 2 ? 0 : 1, j = f ? k - (ch0 + 2) : k;
        const int nb = f ? nb1 : nb0, ch = f ? ch1 : ch0;
        const uint32_t *H = hist + (f ? hoff1 : 0);
        double v = 0.0;
        if (j < ch) {
          const int i = (j << 6) + lane;
          if (i < nb * nb) v = plogp_term(H[i], N);
        } else if (lane < nb) {
          uint64_t m = 0;
          if (j == ch) {
            for (int b = 0; b < nb; ++b) m += H[lane * nb + b];  // row sums: H(X)
          } else {
            for (int a = 0; a < nb; ++a) m += H[a * nb + lane];  // column sums: H(Y)
          }
          v = plogp_term(m, N);
        }
        v = wave_sum_f64(v);
        if (lane == 0) part[f * 66 + (j < ch ? j : 64 + (j - ch))] = v;
      }
    }
    __syncthreads();
    if (wid < nf) {
      const int f = wid, nb = f ? nb1 : nb0, ch = f ? ch1 : ch0;
      double hxy = nonempty && lane < ch ? part[f * 66 + lane] : 0.0;
      hxy = wave_sum_f64(hxy);
      if (lane == 0)
        P.mi_out[(int64_t)f * P.K + pose.out_index] =
            nonempty ? (part[f * 66 + 64] + part[f * 66 + 65]) - hxy : 0.0;
      if (P.hist_out) {
        const uint32_t *H = hist + (f ? hoff1 : 0);
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
    __syncthreads();  // LDS (histograms, counters) is reused by the next item
  }
}

int32_t eval_hash_slot_bytes(bool zvar) { return 4 + (zvar ? 16 : 4) + 2; }

size_t eval_lds_bytes(const EvalLaunch &c) {
  return (size_t)eval_layout(c.waves, c.hist_copies, c.hist_words, c.plan_bytes, c.cap,
                             c.zvar)
      .total;
}

template <bool NEAR, bool ZVAR, int MODE>
static hipError_t launch_one(const PairDev *pairs_dev, const FrameDev *frames_dev,
                             const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                             const EvalLaunch &c, uint2 *scratch, int64_t scratch_stride,
                             int64_t max_wgs, hipStream_t s) {
  const Layout L = eval_layout(c.waves, c.hist_copies, c.hist_words, c.plan_bytes,
                               c.cap, c.zvar);
  EvalCfgDev d;
  d.hist_copies = c.hist_copies;
  d.hist_words = c.hist_words;
  d.cap = c.cap;
  d.load_max = c.cap / 4;
  d.off_cnta = L.off_cnta;
  d.off_edges = L.off_edges;
  d.off_wave = L.off_wave;
  d.off_plan = L.off_plan;
  d.off_hash = L.off_hash;
  d.pad = 0;
  // runs per XCD: the caller's split, else equal counts
  int64_t longest = 0;
  for (int x = 0; x <= kXcds; ++x)
    d.xcd_start[x] = xcd_start ? xcd_start[x] : std::min<int64_t>(n_items, x * ((n_items + kXcds - 1) / kXcds));
  for (int x = 0; x < kXcds; ++x) {
    if (d.xcd_start[x] > d.xcd_start[x + 1] || d.xcd_start[x + 1] > n_items) return hipErrorInvalidValue;
    longest = std::max(longest, d.xcd_start[x + 1] - d.xcd_start[x]);
  }
  if (d.xcd_start[0] != 0 || d.xcd_start[kXcds] != n_items) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)k_eval<NEAR, ZVAR, MODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  int64_t wpx = std::max<int64_t>(1, longest);  // workgroups per XCD
  if (max_wgs > 0) wpx = std::max<int64_t>(1, std::min<int64_t>(wpx, max_wgs / kXcds));
  const int64_t grid = wpx * kXcds;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  k_eval<NEAR, ZVAR, MODE><<<(unsigned)grid, c.waves * 64, (size_t)L.total, s>>>(
      pairs_dev, frames_dev, items_dev, d, scratch, scratch_stride);
  return hipGetLastError();
}

// Workgroups of a persistent grid for this launch shape: the compute units
// times the resident workgroups per unit (at most per_cu), a multiple of the
// XCD count.
hipError_t eval_resident_wgs(const EvalLaunch &c, int per_cu, int64_t *out, int mode) {
  const Layout L = eval_layout(c.waves, c.hist_copies, c.hist_words, c.plan_bytes,
                               c.cap, c.zvar);
  hipError_t e;
  int dev = 0, cus = 0, occ = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  const void *fn = mode == 0   ? (c.zvar ? (const void *)k_eval<false, true, 0>
                                          : (const void *)k_eval<false, false, 0>)
                   : mode == 2 ? (c.zvar ? (const void *)k_eval<false, true, 2>
                                          : (const void *)k_eval<false, false, 2>)
                               : (c.zvar ? (const void *)k_eval<false, true, 1>
                                          : (const void *)k_eval<false, false, 1>);
  if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, L.total)) !=
      hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, c.waves * 64, (size_t)L.total)) !=
      hipSuccess)
    return e;
  const int64_t per = std::max(1, std::min(occ, per_cu));
  *out = std::max<int64_t>(kXcds, ((int64_t)cus * per / kXcds) * kXcds);
  return hipSuccess;
}

hipError_t launch_eval(const PairDev *pairs_dev, const FrameDev *frames_dev,
                       const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                       const EvalLaunch &c, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  int64_t max_wgs = 0;
  if (c.wgs_per_cu > 0) {
    hipError_t e = eval_resident_wgs(c, c.wgs_per_cu, &max_wgs);
    if (e != hipSuccess) return e;
  }
  if (c.near_face)
    return c.zvar ? launch_one<true, true, 0>(pairs_dev, frames_dev, items_dev, n_items,
                                                  xcd_start, c, nullptr, 0, max_wgs, s)
                  : launch_one<true, false, 0>(pairs_dev, frames_dev, items_dev, n_items,
                                                   xcd_start, c, nullptr, 0, max_wgs, s);
  return c.zvar ? launch_one<false, true, 0>(pairs_dev, frames_dev, items_dev, n_items,
                                                 xcd_start, c, nullptr, 0, max_wgs, s)
                : launch_one<false, false, 0>(pairs_dev, frames_dev, items_dev, n_items,
                                                  xcd_start, c, nullptr, 0, max_wgs, s);
}

hipError_t launch_eval_direct(const PairDev *pairs_dev, const FrameDev *frames_dev,
                              const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                              const EvalLaunch &c, uint2 *scratch, int64_t scratch_stride,
                              int64_t slots, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (c.near_face)
    return c.zvar ? launch_one<true, true, 1>(pairs_dev, frames_dev, items_dev, n_items,
                                                 xcd_start, c, scratch, scratch_stride, slots, s)
                  : launch_one<true, false, 1>(pairs_dev, frames_dev, items_dev, n_items,
                                                  xcd_start, c, scratch, scratch_stride, slots, s);
  return c.zvar ? launch_one<false, true, 1>(pairs_dev, frames_dev, items_dev, n_items,
                                                xcd_start, c, scratch, scratch_stride, slots, s)
                : launch_one<false, false, 1>(pairs_dev, frames_dev, items_dev, n_items,
                                                 xcd_start, c, scratch, scratch_stride, slots, s);
}

hipError_t launch_eval_tiles(const PairDev *pairs_dev, const FrameDev *frames_dev,
                             const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                             const EvalLaunch &c, int64_t slots, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (c.near_face)
    return c.zvar ? launch_one<true, true, 2>(pairs_dev, frames_dev, items_dev, n_items,
                                              xcd_start, c, nullptr, 0, slots, s)
                  : launch_one<true, false, 2>(pairs_dev, frames_dev, items_dev, n_items,
                                               xcd_start, c, nullptr, 0, slots, s);
  return c.zvar ? launch_one<false, true, 2>(pairs_dev, frames_dev, items_dev, n_items,
                                             xcd_start, c, nullptr, 0, slots, s)
                : launch_one<false, false, 2>(pairs_dev, frames_dev, items_dev, n_items,
                                              xcd_start, c, nullptr, 0, slots, s);
}

}  // namespace mi
