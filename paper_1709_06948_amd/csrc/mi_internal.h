// mi_internal.h -- device-side tables and launch wrappers shared by the HIP
// sources of libmi355.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mi.h"

namespace mi {

constexpr int kMaxBins = MI_MAX_BINS;
constexpr int kXcds = 8;              // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr double kColEps = 1e-6;      // padding (voxel units) of candidate column ranges
constexpr double kQScale = 1048576.0; // 2^20: z quantum per voxel
constexpr double kNearFace = 1e-5;    // m

// Grid + feature description, host copy of the validated descriptor.
struct GridInfo {
  double origin[3];
  int32_t dims[3];
  double voxel;
  double s;       // fl(1/voxel)
  uint32_t features;
  int32_t nf;     // number of enabled features (1 or 2)
  uint32_t kind[2];
  int32_t nb[2];
  int32_t nbc, nbz;  // count and z-variance bins (also the joint feature's parts)
  int64_t V;
  uint32_t count_edges[kMaxBins];
  uint64_t zvar_edges[kMaxBins];
};

// ------------------------------------------------------------------ reference

// Layout of one feature's summed-volume tables over the (nz+1)(ny+1)(nx+1)
// padded grid: bin a's table, if it has one, has 1, 2 or 4 bytes per entry
// (bit a set in mask[0], mask[1] or mask[2]), the fewest that hold the bin's
// voxel count in scan A; its entries are kept modulo 2^(8 width), which leaves
// every box count exact, since it lies in [0, that count].  The tables follow
// each other in bin order, each rounded up to 256 bytes.  A bin without a
// table is empty in A or kept in the reference's voxel list.
struct SatLayout {
  uint64_t mask[3];
};

// Voxel lists (for sparse bins on large grids): one 64-bit entry per voxel of
// A, (f * 64 + a) << 56 | z << 40 | y << 20 | x, grouped by bin.  At most
// kListMax entries per reference, so counting them in a box is a short scan.
constexpr uint32_t kListMax = 8192;
__host__ __device__ inline bool list_fits(int nx, int ny, int nz) {
  return nx < (1 << 20) && ny < (1 << 20) && nz < (1 << 16);
}

__host__ __device__ inline bool sat_has_table(const SatLayout &L, int a) {
  return ((L.mask[0] | L.mask[1] | L.mask[2]) >> a) & 1u;
}

__host__ __device__ inline int64_t sat_table_bytes(int64_t plane, int w) {
  return (plane * w + 255) & ~(int64_t)255;
}
__host__ __device__ inline int sat_width(const SatLayout &L, int a) {
  return (L.mask[2] >> a) & 1u ? 4 : (L.mask[1] >> a) & 1u ? 2 : 1;
}
// Byte offset of bin a's table: the tables of bins 1 .. a-1 before it.
__host__ __device__ inline int64_t sat_offset(const SatLayout &L, int a, int64_t plane) {
  const uint64_t below = (a >= 64 ? ~0ull : (1ull << a) - 1ull) & ~1ull;
  return __builtin_popcountll(L.mask[0] & below) * sat_table_bytes(plane, 1) +
         __builtin_popcountll(L.mask[1] & below) * sat_table_bytes(plane, 2) +
         __builtin_popcountll(L.mask[2] & below) * sat_table_bytes(plane, 4);
}

struct RefDev {
  int32_t nx, ny, nz, nf;
  uint32_t kind[2];
  int32_t nb[2];
  int32_t nbc, nbz;
  double s;
  double c0[3];              // fl(fl(0 - origin) * s)
  uint32_t count_edges[kMaxBins];
  uint64_t zvar_edges[kMaxBins];
  // transient dense sums
  uint32_t *cnt;
  unsigned long long *s1, *s2;
  // resident
  uint8_t *bins[2];          // [V] per feature slot
  uint8_t *sat[2];           // summed-volume tables per feature slot
  SatLayout sat_layout[2];   // set by the host from bin_cnt
  uint64_t *alist;           // voxel list of the bins in list_mask
  uint32_t alist_n;
  uint64_t list_mask[2];
  uint32_t *list_cur;        // [2][64] cursors while the list is built
  uint32_t *bin_cnt;         // [2][64] voxels of A per bin
  int32_t *abox;             // lo[3], hi[3]
  unsigned long long *counters; // in, out, nonfinite, occupied
};

// The reference's voxel sums, bins and per-bin voxel counts (bin_cnt), then,
// once the host has laid out the tables from those counts (sat_layout),
// the summed-volume tables.
hipError_t launch_ref_bins(const RefDev &rd, const float *xyz, int64_t n, hipStream_t s);
hipError_t launch_ref_sat(const RefDev &rd, hipStream_t s);

// ------------------------------------------------------------------- frames

// One distinct rotation of scan B: the points rotated and scaled to voxel
// units (v = fl(fl(R p) * s)), bucketed by column of A's grid.
struct FrameDev {
  double R[9];
  double s;
  const float *xyz;
  int64_t n;                 // points of scan B
  int32_t gx, gy, ncx, ncy;  // column grid: column (cx, cy) holds floor(v) = (gx + cx, gy + cy)
  int32_t zlo, zhi;          // kept when zlo <= floor(v_z) <= zhi
  double *v;                 // sorted SoA, stride n: x, y, z
  uint32_t *off;             // [ncx*ncy + 1]
  uint32_t *cur;             // [ncx*ncy] counts, then cursors
};

hipError_t launch_frames(const FrameDev *frames_dev, int32_t n_frames, int64_t max_points,
                         int32_t max_cols, hipStream_t s);

// --------------------------------------------------------------------- eval

// One scan pair of an evaluation batch: A resident, B bucketed into frames.
struct PairDev {
  int32_t nx, ny, nz, nf;
  uint32_t kind[2];
  int32_t nb[2];
  int32_t nbc, nbz;
  double voxel;
  const uint8_t *binA[2];
  const uint8_t *sat[2];      // A's summed-volume tables
  SatLayout sat_layout[2];
  const uint64_t *alist;      // A's voxel list (sparse bins without a table)
  uint32_t alist_n;
  const int32_t *abox;
  int32_t stripe_h;          // voxel rows per stripe (bricks are pieces of stripes)
  int32_t n_stripes;
  int32_t pieces;            // x pieces per stripe in the plan
  int32_t kx_bits, ky_bits;  // hash key: iz << (kx+ky) | (iy - stripe y0) << kx | ix
  int32_t plan_stripes;      // stripes whose candidate rows are planned per round
  int32_t count_default;     // count edges are 1, 2, ..., nb - 1 (bin = min(n, nb - 1))
  int32_t zvar_zero_edges;   // z-variance edges equal to 0 (a zero variance has bin 1 + this)
  const unsigned long long *nonfinite; // device counter
  int64_t n_b;
  // Tiled per-pose form: scan B bucketed into tiles of its own (x, y) frame.
  // Tile (i, j), t = j * tile_nx + i, holds the points with
  // i = floor((x - tile_x0) * tile_ilx) (clamped to [0, tile_nx)), likewise j,
  // then its halo: the points of the neighbouring tiles that lie within
  // tile_hx (tile units) of it.  tile_nx = 0: the pair is not tiled.
  const float *xyz_b;        // scan B, [3][n_b]
  float *tile_xyz;           // [3][tile_stride]: per tile its own points, then its halo
  int64_t tile_stride;
  uint32_t *tile_off;        // [tiles + 1]: tile t is [off[t], off[t + 1])
  uint32_t *tile_own;        // [tiles]: end of tile t's own points
  uint32_t *tile_cnt;        // [2 * tiles]: own and halo counts, then cursors
  double tile_x0, tile_y0, tile_ilx, tile_ily, tile_hx, tile_hy;
  int32_t tile_nx, tile_ny;
  int32_t key_xbits, key_ybits;  // whole-grid voxel key: iz << (x + y bits) | iy << x bits | ix
  double *mi_out;
  int64_t K;                 // feature stride of mi_out
  uint32_t *hist_out;
  int64_t hist_off[2];
  mi_pose_stats *stats_out;
  uint32_t count_edges[kMaxBins];
  uint64_t zvar_edges[kMaxBins];
};

struct PoseDev {
  int32_t pair;              // index into the batch's pairs
  int32_t frame;             // index into the batch's frame table
  int32_t out_index;         // pose index in the caller's order within its pair
  int32_t pad;
  double c[3];               // fl(fl(t - origin) * s)
};

// Launch shape of the evaluator (one workgroup per pose).
struct EvalLaunch {
  int32_t waves;             // waves per workgroup (1..16)
  int32_t cap;               // LDS voxel-hash slots (a multiple of 64)
  int32_t hist_copies;       // privatized joint-histogram copies
  int32_t hist_words;        // max over pairs of sum_f nb_f^2
  int32_t plan_bytes;        // max over pairs of plan_stripes * rows * (pieces + 1) * 8
  int32_t wgs_per_cu;        // 0: one workgroup per pose; else a persistent grid
  bool zvar;                 // 16-byte voxel sums (else 4-byte counts)
  bool near_face;
};

// xcd_start (host, kXcds + 1 entries, or NULL for equal counts): the items of
// XCD x are [xcd_start[x], xcd_start[x + 1]), contiguous runs of the item array.
hipError_t launch_eval(const PairDev *pairs_dev, const FrameDev *frames_dev,
                       const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                       const EvalLaunch &cfg, hipStream_t s);
// Per-pose bucketing form (pose sets with (nearly) all rotations distinct): a
// grid of `slots` workgroups, workgroup b using scratch[b * stride ...] for
// its pose's bucketed points (stride >= the largest n_b of the launch).
hipError_t launch_eval_direct(const PairDev *pairs_dev, const FrameDev *frames_dev,
                              const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                              const EvalLaunch &cfg, uint2 *scratch, int64_t scratch_stride,
                              int64_t slots, hipStream_t s);
// Tiled per-pose form (pose sets with (nearly) all rotations distinct, scan B
// fixed when the plan is made): a grid of `slots` workgroups over the items.
hipError_t launch_eval_tiles(const PairDev *pairs_dev, const FrameDev *frames_dev,
                             const PoseDev *items_dev, int64_t n_items, const int64_t *xcd_start,
                             const EvalLaunch &cfg, int64_t slots, hipStream_t s);
// Bucketing of the tiled pairs' scans (pairs_dev[tiled_dev[k]], k < n_tiled):
// clears `cnt_words` words of counts at `cnt` (every tiled pair's tile_cnt lies
// there), counts, scans, scatters.  max_n: the most points of a tiled scan.
hipError_t launch_tiles(const PairDev *pairs_dev, const int32_t *tiled_dev, int32_t n_tiled,
                        int64_t max_n, uint32_t *cnt, int64_t cnt_words, hipStream_t s);
// Workgroups of a persistent grid of this shape (at most per_cu per compute
// unit) for the evaluator form `mode` (0 frames, 1 stripe buckets, 2 tiles).
hipError_t eval_resident_wgs(const EvalLaunch &cfg, int per_cu, int64_t *out, int mode = 1);
size_t eval_lds_bytes(const EvalLaunch &cfg);
int32_t eval_hash_slot_bytes(bool zvar);

// -------------------------------------------------------------------- plain

struct PlainDev {
  int32_t nx, ny, nz, nf;
  uint32_t kind[2];
  int32_t nb[2];
  int32_t nbc, nbz;
  double voxel, s;
  const uint8_t *binA[2];
  const int32_t *abox;
  uint32_t count_edges[kMaxBins];
  uint64_t zvar_edges[kMaxBins];
  // scratch
  uint32_t *dn;
  unsigned long long *ds1, *ds2;
  int32_t *lin;              // [n_b]
  uint32_t *q;               // [n_b]
  uint8_t *near;             // [n_b]
  int32_t *bbox;             // [6] per pose (min lo / max hi)
  unsigned long long *ctr;   // [4]: in-grid, nonfinite, near-in-overlap, pad
  uint32_t *hist;            // [nf][nb*nb]
};

hipError_t launch_plain_pose(const PlainDev &pd, const PlainDev *pd_dev, const float *xyz,
                             int64_t n, const double *rt_dev, int64_t pose_index, double *mi_out,
                             int64_t K, uint32_t *hist_out, const int64_t hist_off[2],
                             mi_pose_stats *stats_out, bool near_face, hipStream_t s);
hipError_t launch_plain_clear_dense(const PlainDev &pd, hipStream_t s);

// ------------------------------------------------------------------ utility

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_argmax(const double *mi, int64_t K, int32_t nf, int64_t *out, double *out_val,
                         hipStream_t s);
// out[k] = w0 * mi[k] + w1 * mi[K + k] (the second term when nf == 2)
hipError_t launch_weighted(const double *mi, int64_t K, int32_t nf, double w0, double w1,
                           double *out, hipStream_t s);
hipError_t launch_bind(PairDev *pair, FrameDev *frames, int32_t n_frames, const float *xyz,
                       double *mi_out, uint32_t *hist_out, mi_pose_stats *stats_out,
                       hipStream_t s);
hipError_t launch_count_nonfinite(const float *xyz, int64_t n, unsigned long long *out,
                                  hipStream_t s);

}  // namespace mi
