/*
 * mi_oracle.c -- plain FP64 CPU reference for mutual-information scan alignment
 * (Mehta, McBride, Pandey, "Robust and Fast 3D Scan Alignment using Mutual
 * Information", arXiv 1709.06948).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
 * of the benchmark call this code; the product library never links or calls it
 * and shares no source with it.
 *
 * It is slow on purpose: every pose gets dense per-voxel arrays for scan B, and
 * the joint histogram is built by a dense sweep over every voxel of the overlap
 * box, exactly as the method defines it (Sec. III-A, Eqs. 1-5, Alg. 1).  The
 * only parallelism is one pose per OpenMP thread.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math):
 * every product and sum below is rounded on its own, in the written order.
 *
 * Readings of the paper that the code fixes (the paper is silent on them):
 *  - pose eta = [tx,ty,tz,roll,pitch,yaw], R = Rz(yaw) Ry(pitch) Rx(roll),
 *    x' = R x + t maps scan B into scan A's frame (Sec. III-A, Eq. 1);
 *  - voxel coordinate per axis u = fl(fl(w*s) + c) with w the rotated point,
 *    s = fl(1/voxel) and c = fl(fl(t - origin) * s); voxel index floor(u);
 *    voxels are half-open, points outside the grid belong to no voxel;
 *  - the z-height variance feature is computed on q = floor(frac(u_z) * 2^20),
 *    the height above the voxel floor in units of voxel/2^20, with exact
 *    integer sums; bins compare n*S2 - S1^2 against E_j * n^2 exactly;
 *  - a scan's extent (Alg. 1, overlap step) is the index box of its in-grid
 *    points; the overlap box is the per-axis max of the lower and min of the
 *    upper bounds; an empty overlap gives MI = 0;
 *  - entropies use the natural log, 0 ln 0 = 0, and the marginals are the row
 *    and column sums of the joint histogram over the overlap box;
 *  - argmax picks the smallest index within 1e-12 of the maximum;
 *  - the joint feature (an extension in the direction the conclusion points,
 *    richer per-voxel features) is the pair (count bin, z-variance bin) of an
 *    occupied voxel as one value, 1 + (count bin - 1) * (nb_zvar - 1) +
 *    (z-variance bin - 1); the empty voxel keeps value 0;
 *  - a weighted search maximises w0 * MI_0 + w1 * MI_1 over the feature slots,
 *    each product rounded, then the sum.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

#define MIO_FEAT_COUNT 1u
#define MIO_FEAT_ZVAR 2u
#define MIO_FEAT_JOINT 4u

/* Grid and feature description, as the oracle's caller passes it. */
typedef struct {
  double origin[3];
  int32_t dims[3];
  double voxel;
  uint32_t features;      /* bitmask of MIO_FEAT_* */
  int32_t nb_count;       /* bins of the point-count feature */
  const uint32_t *count_edges; /* nb_count-1 ascending lower edges */
  int32_t nb_zvar;        /* bins of the z-variance feature (and the joint one's z part) */
  const uint64_t *zvar_edges;  /* nb_zvar-2 ascending edges, units (voxel/2^20)^2 */
} mio_grid;

/* Per-pose statistics, 11 int64 values:
 * lo[3], hi[3] of the overlap box, |O|, in-grid B points, out-of-grid B points,
 * non-finite B points, in-overlap B points within 1e-5 m of a voxel face. */
#define MIO_NSTATS 11

/* ---------------------------------------------------------------- pose */

/* Rotation of the 6-DOF pose (Sec. I: three translations and three rotation
 * angles; Sec. III-A: T as a 4x4 rigid transform).  R = Rz(yaw) Ry(pitch)
 * Rx(roll), row-major, each product and sum rounded separately. */
void mio_pose_matrix(const double eta[6], double R[9]) {
  const double cr = cos(eta[3]), sr = sin(eta[3]);
  const double cp = cos(eta[4]), sp = sin(eta[4]);
  const double cy = cos(eta[5]), sy = sin(eta[5]);
  R[0] = cy * cp;
  R[1] = (cy * sp) * sr - sy * cr;
  R[2] = (cy * sp) * cr + sy * sr;
  R[3] = sy * cp;
  R[4] = (sy * sp) * sr + cy * cr;
  R[5] = (sy * sp) * cr - cy * sr;
  R[6] = -sp;
  R[7] = cp * sr;
  R[8] = cp * cr;
}

/* ---------------------------------------------------------------- bins */

/* Default count edges: bin = min(n, nb-1), bin 0 = empty (phi, Sec. III-A). */
int mio_default_count_edges(int32_t nb, uint32_t *e) {
  if (nb < 2 || nb > 64) return -1;
  for (int32_t j = 0; j < nb - 1; ++j) e[j] = (uint32_t)(j + 1);
  return 0;
}

/* Default z-variance edges: nb-2 edges log-spaced from 1e-5 m^2 to voxel^2/4,
 * expressed in units of (voxel/2^20)^2 and rounded up. */
int mio_default_zvar_edges(double voxel, int32_t nb, uint64_t *E) {
  if (nb < 3 || nb > 64) return -1;
  const int32_t m = nb - 2;
  const double lo = 1e-5, hi = voxel * voxel / 4.0;
  if (!(hi > lo)) return -1;
  const double scale = (1048576.0 / voxel) * (1048576.0 / voxel);
  for (int32_t j = 0; j < m; ++j) {
    double e = (m == 1) ? lo : lo * pow(hi / lo, (double)j / (double)(m - 1));
    E[j] = (uint64_t)ceil(e * scale);
  }
  return 0;
}

/* Point-count feature (Sec. III-A, feature ii): number of edges at or below n. */
static int bin_count(uint32_t n, int32_t nb, const uint32_t *e) {
  int b = 0;
  for (int32_t j = 0; j < nb - 1; ++j)
    if (n >= e[j]) ++b;
  return b;
}

/* z-height variance feature (Sec. III-A, feature i).  Population variance of q
 * is D / n^2 with D = n*S2 - S1^2; bin 0 is the empty voxel, otherwise 1 plus
 * the number of edges E_j with D >= E_j * n^2 (exact 128-bit integers). */
static int bin_zvar(uint32_t n, uint64_t s1, uint64_t s2, int32_t nb, const uint64_t *E) {
  if (n == 0) return 0;
  const u128 D = (u128)n * (u128)s2 - (u128)s1 * (u128)s1;
  const u128 n2 = (u128)n * (u128)n;
  int b = 1;
  for (int32_t j = 0; j < nb - 2; ++j)
    if (D >= (u128)E[j] * n2) ++b;
  return b;
}

/* ------------------------------------------------------------ voxelize */

typedef struct {
  uint32_t *cnt;
  uint64_t *s1, *s2;
  int32_t *lin;     /* per point: voxel index or -1 */
  uint8_t *near;    /* per point: 1 if within 1e-5 m of a voxel face */
  int32_t lo[3], hi[3];
  int64_t n_in, n_out, n_nonfinite;
} scan_vox;

/* Voxel-point mapping and per-voxel sums of one scan under pose (R, t)
 * (Alg. 1 initialisation for scan A with R = I, t = 0; Alg. 1 loop for B).
 * The extent lo/hi is the index box of in-grid points; an empty scan gets
 * lo = dims, hi = -1. */
static void voxelize(const mio_grid *g, const float *xyz, int64_t n, const double *R,
                     const double t[3], scan_vox *sv) {
  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  memset(sv->cnt, 0, (size_t)V * sizeof(uint32_t));
  memset(sv->s1, 0, (size_t)V * sizeof(uint64_t));
  memset(sv->s2, 0, (size_t)V * sizeof(uint64_t));
  for (int a = 0; a < 3; ++a) { sv->lo[a] = g->dims[a]; sv->hi[a] = -1; }
  sv->n_in = sv->n_out = sv->n_nonfinite = 0;
  const double s = 1.0 / g->voxel;
  double c[3];
  for (int a = 0; a < 3; ++a) c[a] = (t[a] - g->origin[a]) * s;
  const float *X = xyz, *Y = xyz + n, *Z = xyz + 2 * n;
  for (int64_t i = 0; i < n; ++i) {
    const double x = X[i], y = Y[i], z = Z[i];
    if (sv->lin) sv->lin[i] = -1;
    if (sv->near) sv->near[i] = 0;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) { sv->n_nonfinite++; continue; }
    double w[3];
    if (R) {
      w[0] = (R[0] * x + R[1] * y) + R[2] * z;
      w[1] = (R[3] * x + R[4] * y) + R[5] * z;
      w[2] = (R[6] * x + R[7] * y) + R[8] * z;
    } else {
      w[0] = x; w[1] = y; w[2] = z;
    }
    double u[3], f[3];
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
      u[a] = w[a] * s + c[a];
      f[a] = floor(u[a]);
      if (!(f[a] >= 0.0 && f[a] < (double)g->dims[a])) inside = 0;
    }
    if (!inside) { sv->n_out++; continue; }
    const int32_t ix = (int32_t)f[0], iy = (int32_t)f[1], iz = (int32_t)f[2];
    const int64_t v = ((int64_t)iz * g->dims[1] + iy) * g->dims[0] + ix;
    const double fz = u[2] - f[2];
    const uint64_t q = (uint64_t)floor(fz * 1048576.0);
    sv->cnt[v] += 1;
    sv->s1[v] += q;
    sv->s2[v] += q * q;
    sv->n_in++;
    const int32_t ii[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
      if (ii[a] < sv->lo[a]) sv->lo[a] = ii[a];
      if (ii[a] > sv->hi[a]) sv->hi[a] = ii[a];
    }
    if (sv->lin) sv->lin[i] = (int32_t)v;
    if (sv->near) {
      double d = 1.0;
      for (int a = 0; a < 3; ++a) {
        const double fr = u[a] - f[a];
        const double up = 1.0 - fr;
        const double m = fr < up ? fr : up;
        if (m < d) d = m;
      }
      sv->near[i] = (d * g->voxel < 1e-5) ? 1 : 0;
    }
  }
}

static const uint32_t kFeatureOrder[3] = {MIO_FEAT_COUNT, MIO_FEAT_ZVAR, MIO_FEAT_JOINT};

static int n_features(const mio_grid *g) {
  int n = 0;
  for (int i = 0; i < 3; ++i)
    if (g->features & kFeatureOrder[i]) ++n;
  return n;
}

/* feature slot f -> kind, in the fixed order count, z-variance, joint */
static uint32_t feature_kind(const mio_grid *g, int f) {
  int k = 0;
  for (int i = 0; i < 3; ++i) {
    if (!(g->features & kFeatureOrder[i])) continue;
    if (k == f) return kFeatureOrder[i];
    ++k;
  }
  return 0;
}

/* values of the joint feature: the empty voxel, then every pair of an
 * occupied count bin (1 .. nb_count-1) and z-variance bin (1 .. nb_zvar-1) */
static int joint_nb(const mio_grid *g) { return 1 + (g->nb_count - 1) * (g->nb_zvar - 1); }

static int feature_nb(const mio_grid *g, int f) {
  const uint32_t kind = feature_kind(g, f);
  if (kind == MIO_FEAT_COUNT) return g->nb_count;
  if (kind == MIO_FEAT_ZVAR) return g->nb_zvar;
  return joint_nb(g);
}

static int voxel_bin(const mio_grid *g, uint32_t kind, uint32_t n, uint64_t s1, uint64_t s2) {
  if (kind == MIO_FEAT_COUNT) return bin_count(n, g->nb_count, g->count_edges);
  if (kind == MIO_FEAT_ZVAR) return bin_zvar(n, s1, s2, g->nb_zvar, g->zvar_edges);
  if (n == 0) return 0;
  const int bc = bin_count(n, g->nb_count, g->count_edges);
  const int bz = bin_zvar(n, s1, s2, g->nb_zvar, g->zvar_edges);
  return 1 + (bc - 1) * (g->nb_zvar - 1) + (bz - 1);
}

/* --------------------------------------------------------------- entropy */

/* Shannon entropy (natural log) of counts c[0..m) with total N (Eqs. 3-5). */
static double entropy(const uint64_t *c, int64_t m, double N) {
  double h = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    if (c[i] == 0) continue;
    const double p = (double)c[i] / N;
    h -= p * log(p);
  }
  return h;
}

/* MI(X,Y) = H(X) + H(Y) - H(X,Y) of an nb x nb joint histogram with rows = A
 * bins and columns = B bins (Eq. 2); an empty histogram gives 0. */
double mio_mi_from_hist(const uint32_t *H, int32_t nb) {
  uint64_t N = 0;
  uint64_t rows[64], cols[64], cells[64 * 64];
  for (int a = 0; a < nb; ++a) { rows[a] = 0; cols[a] = 0; }
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      const uint64_t v = H[a * nb + b];
      cells[a * nb + b] = v;
      rows[a] += v;
      cols[b] += v;
      N += v;
    }
  if (N == 0) return 0.0;
  const double Nd = (double)N;
  const double hx = entropy(rows, nb, Nd);
  const double hy = entropy(cols, nb, Nd);
  const double hxy = entropy(cells, (int64_t)nb * nb, Nd);
  return hx + hy - hxy;
}

/* Marginal entropies as well, for the tests' bound checks. */
void mio_entropies_from_hist(const uint32_t *H, int32_t nb, double out[3]) {
  uint64_t N = 0;
  uint64_t rows[64], cols[64], cells[64 * 64];
  for (int a = 0; a < nb; ++a) { rows[a] = 0; cols[a] = 0; }
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      const uint64_t v = H[a * nb + b];
      cells[a * nb + b] = v;
      rows[a] += v;
      cols[b] += v;
      N += v;
    }
  out[0] = out[1] = out[2] = 0.0;
  if (N == 0) return;
  out[0] = entropy(rows, nb, (double)N);
  out[1] = entropy(cols, nb, (double)N);
  out[2] = entropy(cells, (int64_t)nb * nb, (double)N);
}

/* ------------------------------------------------------------- validate */

static int grid_ok(const mio_grid *g) {
  for (int a = 0; a < 3; ++a)
    if (g->dims[a] < 1 || !isfinite(g->origin[a])) return 0;
  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  if (V > 2147483647LL) return 0;
  if (!(g->voxel > 0.0) || !isfinite(g->voxel)) return 0;
  const uint32_t all = MIO_FEAT_COUNT | MIO_FEAT_ZVAR | MIO_FEAT_JOINT;
  if (g->features == 0 || (g->features & ~all) || n_features(g) > 2) return 0;
  if ((g->features & (MIO_FEAT_COUNT | MIO_FEAT_JOINT)) &&
      (g->nb_count < 2 || g->nb_count > 64 || !g->count_edges))
    return 0;
  if ((g->features & MIO_FEAT_ZVAR) && (g->nb_zvar < 3 || g->nb_zvar > 64 || !g->zvar_edges))
    return 0;
  if ((g->features & MIO_FEAT_JOINT) &&
      (g->nb_zvar < 2 || g->nb_zvar > 64 || (g->nb_zvar > 2 && !g->zvar_edges) || joint_nb(g) > 64))
    return 0;
  return 1;
}

/* --------------------------------------------------------- reference A */

/* Alg. 1 initialisation: voxel ids of scan A and its feature map.  Writes the
 * per-voxel sums, the bin of every voxel per feature ([nfeat][V]), the index
 * box of A and counters (in-grid, out-of-grid, non-finite, occupied). */
int mio_scan_features(const mio_grid *g, const float *xyz, int64_t n, const double *eta,
                      uint32_t *cnt, uint64_t *s1, uint64_t *s2, uint8_t *bins,
                      int32_t box[6], int64_t counters[4]) {
  if (!grid_ok(g) || n < 0) return -1;
  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  scan_vox sv = {cnt, s1, s2, NULL, NULL, {0}, {0}, 0, 0, 0};
  double R[9], t[3] = {0, 0, 0};
  if (eta) {
    mio_pose_matrix(eta, R);
    t[0] = eta[0]; t[1] = eta[1]; t[2] = eta[2];
  }
  voxelize(g, xyz, n, eta ? R : NULL, t, &sv);
  int64_t occ = 0;
  const int nf = n_features(g);
  for (int64_t v = 0; v < V; ++v) {
    if (cnt[v]) ++occ;
    for (int f = 0; f < nf; ++f)
      if (bins) bins[f * V + v] = (uint8_t)voxel_bin(g, feature_kind(g, f), cnt[v], s1[v], s2[v]);
  }
  for (int a = 0; a < 3; ++a) { box[a] = sv.lo[a]; box[3 + a] = sv.hi[a]; }
  counters[0] = sv.n_in;
  counters[1] = sv.n_out;
  counters[2] = sv.n_nonfinite;
  counters[3] = occ;
  return 0;
}

/* ------------------------------------------------------------ per pose */

typedef struct {
  const mio_grid *g;
  const uint8_t *binA;  /* [nfeat][V] */
  int32_t Alo[3], Ahi[3];
} refA;

/* One evaluation of Eqs. 1-5 at pose eta (Alg. 1 loop body): transform B,
 * voxelize, build B's feature map, overlap box, joint histogram by a dense
 * sweep over every voxel of the overlap box, entropies, MI per feature. */
static void eval_one(const refA *ra, const float *B, int64_t nbp, const double eta[6],
                     scan_vox *sv, uint32_t *hist /* [nfeat][64*64] scratch */,
                     double *mi /* [nfeat] */, int64_t *stats /* [11] or NULL */) {
  const mio_grid *g = ra->g;
  const int nf = n_features(g);
  double R[9];
  mio_pose_matrix(eta, R);
  const double t[3] = {eta[0], eta[1], eta[2]};
  voxelize(g, B, nbp, R, t, sv);

  int32_t lo[3], hi[3];
  int64_t nO = 1;
  for (int a = 0; a < 3; ++a) {
    lo[a] = ra->Alo[a] > sv->lo[a] ? ra->Alo[a] : sv->lo[a];
    hi[a] = ra->Ahi[a] < sv->hi[a] ? ra->Ahi[a] : sv->hi[a];
    if (lo[a] < 0) lo[a] = 0;
    if (hi[a] > g->dims[a] - 1) hi[a] = g->dims[a] - 1;
    if (hi[a] < lo[a]) nO = 0;
  }
  if (nO) nO = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);

  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  for (int f = 0; f < nf; ++f) {
    const int nb = feature_nb(g, f);
    const uint32_t kind = feature_kind(g, f);
    uint32_t *H = hist + (size_t)f * 64 * 64;
    memset(H, 0, sizeof(uint32_t) * (size_t)nb * nb);
    if (nO) {
      for (int32_t z = lo[2]; z <= hi[2]; ++z)
        for (int32_t y = lo[1]; y <= hi[1]; ++y)
          for (int32_t x = lo[0]; x <= hi[0]; ++x) {
            const int64_t v = ((int64_t)z * g->dims[1] + y) * g->dims[0] + x;
            const int a = ra->binA[f * V + v];
            const int b = voxel_bin(g, kind, sv->cnt[v], sv->s1[v], sv->s2[v]);
            H[a * nb + b] += 1;
          }
    }
    mi[f] = nO ? mio_mi_from_hist(H, nb) : 0.0;
  }

  if (stats) {
    int64_t near = 0;
    if (nO)
      for (int64_t i = 0; i < nbp; ++i) {
        const int32_t v = sv->lin[i];
        if (v < 0 || !sv->near[i]) continue;
        const int32_t x = v % g->dims[0];
        const int32_t y = (v / g->dims[0]) % g->dims[1];
        const int32_t z = v / (g->dims[0] * g->dims[1]);
        if (x >= lo[0] && x <= hi[0] && y >= lo[1] && y <= hi[1] && z >= lo[2] && z <= hi[2])
          ++near;
      }
    for (int a = 0; a < 3; ++a) { stats[a] = lo[a]; stats[3 + a] = hi[a]; }
    stats[6] = nO;
    stats[7] = sv->n_in;
    stats[8] = sv->n_out;
    stats[9] = sv->n_nonfinite;
    stats[10] = near;
  }
}

static int build_ref(const mio_grid *g, const float *A, int64_t na, refA *ra, uint8_t **bins_out) {
  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  const int nf = n_features(g);
  uint32_t *cnt = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
  uint64_t *s1 = (uint64_t *)malloc((size_t)V * sizeof(uint64_t));
  uint64_t *s2 = (uint64_t *)malloc((size_t)V * sizeof(uint64_t));
  uint8_t *bins = (uint8_t *)malloc((size_t)V * nf);
  if (!cnt || !s1 || !s2 || !bins) { free(cnt); free(s1); free(s2); free(bins); return -2; }
  int32_t box[6];
  int64_t counters[4];
  mio_scan_features(g, A, na, NULL, cnt, s1, s2, bins, box, counters);
  free(cnt); free(s1); free(s2);
  ra->g = g;
  ra->binA = bins;
  for (int a = 0; a < 3; ++a) { ra->Alo[a] = box[a]; ra->Ahi[a] = box[3 + a]; }
  *bins_out = bins;
  return 0;
}

/* MI of every pose in poses[K][6] (Eq. 1 objective at each candidate).
 * mi_out[f*K + k]; hist_out (nullable) holds feature f's histograms at offset
 * sum_{f'<f} K*nb_f'^2, pose k at + k*nb_f^2; stats_out (nullable) [K][11]. */
int mio_eval_poses(const mio_grid *g, const float *A, int64_t na, const float *B, int64_t nbp,
                   const double *poses, int64_t K, double *mi_out, uint32_t *hist_out,
                   int64_t *stats_out, int32_t nthreads) {
  if (!grid_ok(g) || na < 0 || nbp < 0 || K < 0) return -1;
  refA ra;
  uint8_t *bins = NULL;
  if (build_ref(g, A, na, &ra, &bins)) return -2;
  const int64_t V = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  const int nf = n_features(g);
  int64_t hoff[2] = {0, 0};
  if (nf == 2) hoff[1] = K * (int64_t)feature_nb(g, 0) * feature_nb(g, 0);
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    scan_vox sv;
    sv.cnt = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
    sv.s1 = (uint64_t *)malloc((size_t)V * sizeof(uint64_t));
    sv.s2 = (uint64_t *)malloc((size_t)V * sizeof(uint64_t));
    sv.lin = (int32_t *)malloc((size_t)(nbp > 0 ? nbp : 1) * sizeof(int32_t));
    sv.near = (uint8_t *)malloc((size_t)(nbp > 0 ? nbp : 1));
    uint32_t *hist = (uint32_t *)malloc(sizeof(uint32_t) * 2 * 64 * 64);
    const int ok = sv.cnt && sv.s1 && sv.s2 && sv.lin && sv.near && hist;
    if (!ok) {
#pragma omp atomic write
      err = -2;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) {
      if (!ok) continue;
      double mi[2];
      eval_one(&ra, B, nbp, poses + 6 * k, &sv, hist, mi, stats_out ? stats_out + MIO_NSTATS * k : NULL);
      for (int f = 0; f < nf; ++f) {
        mi_out[f * K + k] = mi[f];
        if (hist_out) {
          const int nb = feature_nb(g, f);
          memcpy(hist_out + hoff[f] + k * (int64_t)nb * nb, hist + (size_t)f * 64 * 64,
                 sizeof(uint32_t) * (size_t)nb * nb);
        }
      }
    }
    free(sv.cnt); free(sv.s1); free(sv.s2); free(sv.lin); free(sv.near); free(hist);
  }
  free(bins);
  return err;
}

/* Argmax of Eq. 1 over a finite pose set: the smallest index whose MI is
 * within 1e-12 of the maximum. */
int64_t mio_argmax(const double *mi, int64_t K) {
  if (K <= 0) return -1;
  double mx = mi[0];
  for (int64_t k = 1; k < K; ++k)
    if (mi[k] > mx) mx = mi[k];
  for (int64_t k = 0; k < K; ++k)
    if (mi[k] >= mx - 1e-12) return k;
  return 0;
}

/* Pose grid of one coarse-to-fine level: per axis s nodes c + h*(-1 + 2j/(s-1))
 * (s = 1 gives c), row-major over (tx,ty,tz,roll,pitch,yaw) with yaw fastest. */
int64_t mio_grid_poses(const double center[6], const double half[6], const int32_t samples[6],
                       double *poses) {
  int64_t K = 1;
  for (int a = 0; a < 6; ++a) {
    if (samples[a] < 1) return -1;
    K *= samples[a];
  }
  if (!poses) return K;
  for (int64_t k = 0; k < K; ++k) {
    int64_t r = k;
    int32_t j[6];
    for (int a = 5; a >= 0; --a) { j[a] = (int32_t)(r % samples[a]); r /= samples[a]; }
    for (int a = 0; a < 6; ++a) {
      const int32_t s = samples[a];
      poses[6 * k + a] = (s == 1) ? center[a]
                                  : center[a] + half[a] * (-1.0 + (2.0 * j[a]) / (double)(s - 1));
    }
  }
  return K;
}

/* Weighted objective of every pose: w[0] * MI_0 + w[1] * MI_1 (slots present). */
void mio_weighted(const double *mi, int64_t K, int32_t nf, const double w[2], double *out) {
  for (int64_t k = 0; k < K; ++k) {
    double v = w[0] * mi[k];
    if (nf > 1) v = v + w[1] * mi[K + k];
    out[k] = v;
  }
}

/* Search for the argmax of Eq. 1 by a grid that is re-centred on the best pose
 * and shrunk at every level (the exhaustive-grid stand-in for the simplex
 * search of Sec. III-B).  feature_slot picks which feature's MI drives it; -1
 * drives it by the weighted objective of `weights`. */
int mio_align_c2f(const mio_grid *g, const float *A, int64_t na, const float *B, int64_t nbp,
                  const double init[6], const double half0[6], const int32_t samples[6],
                  int32_t levels, double shrink, int32_t feature_slot, const double *weights,
                  double pose_out[6], double *mi_best, int32_t nthreads) {
  if (!grid_ok(g) || levels < 1 || !(shrink > 0.0)) return -1;
  const int nf = n_features(g);
  if (feature_slot < -1 || feature_slot >= nf || (feature_slot == -1 && !weights)) return -1;
  double c[6], h[6];
  for (int a = 0; a < 6; ++a) { c[a] = init[a]; h[a] = half0[a]; }
  const int64_t K = mio_grid_poses(c, h, samples, NULL);
  if (K < 1) return -1;
  double *poses = (double *)malloc(sizeof(double) * 6 * (size_t)K);
  double *mi = (double *)malloc(sizeof(double) * ((size_t)nf + 1) * (size_t)K);
  if (!poses || !mi) { free(poses); free(mi); return -2; }
  double *obj = feature_slot >= 0 ? mi + (int64_t)feature_slot * K : mi + (int64_t)nf * K;
  double best = 0.0;
  for (int32_t l = 0; l < levels; ++l) {
    mio_grid_poses(c, h, samples, poses);
    int rc = mio_eval_poses(g, A, na, B, nbp, poses, K, mi, NULL, NULL, nthreads);
    if (rc) { free(poses); free(mi); return rc; }
    if (feature_slot < 0) mio_weighted(mi, K, nf, weights, obj);
    const int64_t k = mio_argmax(obj, K);
    for (int a = 0; a < 6; ++a) c[a] = poses[6 * k + a];
    best = obj[k];
    for (int a = 0; a < 6; ++a) h[a] = h[a] / shrink;
  }
  for (int a = 0; a < 6; ++a) pose_out[a] = c[a];
  if (mi_best) *mi_best = best;
  free(poses);
  free(mi);
  return 0;
}
