/*
 * mi.h -- C ABI of libmi355.so: the MI355X (gfx950) hot path of
 * mutual-information 3D scan alignment (Mehta, McBride, Pandey, "Robust and
 * Fast 3D Scan Alignment using Mutual Information", arXiv 1709.06948).
 *
 * What the library computes (Sec. III-A, Eqs. 1-5, Alg. 1):
 *   for each candidate pose eta = [tx, ty, tz, roll, pitch, yaw] it moves
 *   scan B by eta, voxelizes it on the grid of scan A, computes per-voxel
 *   features (point count, z-height variance; empty voxels keep their own
 *   bin 0, the paper's phi value), builds the joint feature histogram over the
 *   overlap box of the two scans and reduces it to
 *   MI = H(X) + H(Y) - H(X,Y) (natural log).  The argmax over the poses is the
 *   estimate of Eq. 1.
 *
 * Fixed readings where the paper is silent:
 *   - R = Rz(yaw) Ry(pitch) Rx(roll); x' = R x + t maps B into A's frame.
 *   - Voxel coordinate per axis u = fl(fl(w * s) + c) in FP64, w the rotated
 *     point (rows summed left to right, no fused multiply-add), s = fl(1/voxel),
 *     c = fl(fl(t - origin) * s); voxel index floor(u); half-open voxels.
 *   - z-variance feature on q = floor(frac(u_z) * 2^20) with exact integer
 *     sums: bin = 1 + #{j : n*S2 - S1^2 >= E_j * n^2}; count bin =
 *     #{j : n >= e_j}.  Default edges: e_j = j (bins min(n, nb-1)); E_j =
 *     ceil(e_j * (2^20/voxel)^2) for nb-2 edges e_j log-spaced from 1e-5 m^2
 *     to voxel^2/4.
 *   - A scan's extent is the index box of its in-grid points; the overlap
 *     box is max of the lower / min of the upper bounds; empty overlap gives
 *     MI = 0.
 *   - Argmax is the smallest pose index within 1e-12 of the maximum.
 *
 * Conventions for every call:
 *   - Points are float32 structure-of-arrays in device memory: x[0..n),
 *     y[0..n), z[0..n) back to back.  Non-finite points are skipped and
 *     counted; points outside the grid are counted and belong to no voxel.
 *   - The caller owns every device buffer.  Device work memory comes from a
 *     caller-provided workspace `ws` of at least the queried size (256-byte
 *     aligned); the library never allocates device memory.  Host handles
 *     (mi_grid, mi_ref, mi_plan) are malloc'd by the library and freed by the
 *     matching destroy call; a mi_ref or mi_plan points into its workspace,
 *     which must outlive it.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *     calls enqueue asynchronously on it, except where a call says it
 *     synchronizes.
 *   - Errors: argument and workspace errors are returned before anything is
 *     enqueued.  MI_E_DEVICE reports a HIP launch or runtime failure.
 *     mi_last_error() returns a thread-local message for the last failure.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.
 */
#ifndef MI355_MI_H
#define MI355_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mi_status;
#define MI_OK 0
#define MI_E_INVALID (-1)     /* bad argument */
#define MI_E_WORKSPACE (-2)   /* workspace too small or misaligned */
#define MI_E_DEVICE (-3)      /* HIP error */
#define MI_E_UNSUPPORTED (-4) /* valid but outside the supported sizes */

/* Feature bitmask (Sec. IV: MI-N and MI-VARZ), at most two set.  Feature
 * slots follow the order count, z-variance, joint. */
#define MI_FEAT_COUNT 1u /* number of points in the voxel */
#define MI_FEAT_ZVAR 2u  /* variance of z-height in the voxel */
/* Both per-voxel features as one value (an extension towards the richer
 * features the conclusion points to): an occupied voxel with count bin c
 * (1..nbins_count-1) and z-variance bin z (1..nbins_zvar-1) has value
 * 1 + (c - 1) * (nbins_zvar - 1) + (z - 1); an empty voxel has 0.  Its bins
 * number 1 + (nbins_count - 1) * (nbins_zvar - 1), at most 64. */
#define MI_FEAT_JOINT 4u

/* feature_slot value of the searches that maximises w[0] * MI_0 + w[1] * MI_1
 * over the grid's feature slots (each product rounded, then the sum). */
#define MI_SLOT_WEIGHTED (-1)

/* Evaluation flags for mi_plan_create / mi_eval_poses / batches. */
#define MI_EVAL_NEAR_FACE 1u /* count points within 1e-5 m of a voxel face (stats) */
/* How scan B reaches the evaluator (results are identical either way).  By
 * default a pose set whose rotations serve two or more poses each on average
 * shares rotated frames (B rotated once per distinct rotation and bucketed by
 * column); otherwise each pose's workgroup transforms and buckets B itself. */
#define MI_EVAL_PER_POSE 2u      /* force per-pose bucketing */
#define MI_EVAL_SHARED_FRAMES 4u /* force shared rotated frames */

/* Limits. */
#define MI_MAX_BINS 64
#define MI_MAX_POINTS ((int64_t)1 << 20) /* per scan B when MI_FEAT_ZVAR or _JOINT is on */

/* The voxel grid of resolution R_v that encompasses both scans (Sec. III-A)
 * plus the feature description.  Axis-aligned in scan A's frame. */
typedef struct mi_grid_desc {
  double origin[3];             /* m, lower corner of voxel (0,0,0) */
  int32_t dims[3];              /* voxels per axis, each >= 1, product < 2^31 */
  double voxel;                 /* edge length R_v in m, > 0 */
  uint32_t features;            /* MI_FEAT_* bitmask, one or two bits */
  int32_t nbins_count;          /* 2..64 when MI_FEAT_COUNT or MI_FEAT_JOINT */
  const uint32_t *count_edges;  /* host, nbins_count-1 ascending, first >= 1; NULL = default */
  int32_t nbins_zvar;           /* 3..64 when MI_FEAT_ZVAR; 2..64 for MI_FEAT_JOINT alone */
  const uint64_t *zvar_edges;   /* host, nbins_zvar-2 ascending; NULL = default */
} mi_grid_desc;

typedef struct mi_grid mi_grid;
typedef struct mi_ref mi_ref;
typedef struct mi_plan mi_plan;

/* Per-pose diagnostics (64 bytes). lo/hi: overlap box (lo > hi on some axis
 * when it is empty); n_overlap = |O|; B points in the grid, outside it,
 * non-finite; B points in the overlap within 1e-5 m of a voxel face (only
 * with MI_EVAL_NEAR_FACE, else 0). */
typedef struct mi_pose_stats {
  int32_t lo[3], hi[3];
  int64_t n_overlap, n_in_grid, n_out_of_grid, n_nonfinite, n_near_face;
} mi_pose_stats;

const char *mi_status_str(mi_status s);
const char *mi_last_error(void);

/* Launch shape of the batched evaluator (process-wide; read when a plan is
 * created).  waves: 1..16 waves per workgroup (a workgroup evaluates one pose
 * at a time); hash_bytes: LDS bytes for the voxel sums of one brick (the slot
 * count is the largest multiple of 64 that fits, at most 65536); hist_copies:
 * 1..8 privatized joint histograms; stripe_rows: 1..62 voxel rows per stripe
 * of bricks;
 * wgs_per_cu: 0 launches one workgroup per pose, 1..16 a persistent grid of
 * that many workgroups per compute unit, each looping over poses.  Every
 * setting gives bit-identical histograms.  hash_bytes = 0 (the default) is
 * "auto": 66 KiB, falling back to 60 KiB in launches whose histograms and plan
 * entries would otherwise leave room for only one workgroup per compute unit;
 * mi_tuning_get reports 0 while it is in force, so a get / set round trip
 * keeps it.  Other sizes are used as given. */
typedef struct mi_tuning {
  int32_t waves;
  int32_t hash_bytes;
  int32_t hist_copies;
  int32_t stripe_rows;
  int32_t wgs_per_cu;
} mi_tuning;
mi_status mi_tuning_set(const mi_tuning *t);
mi_status mi_tuning_get(mi_tuning *t);

/* Stage timing with HIP events (tracing; process-wide).  While enabled, every
 * plan execution and plain evaluation records events around its frame build,
 * evaluation and per-pose launches on the stream it runs on (so enabled
 * timing is not for graph capture).  mi_profile_read synchronizes on the
 * recorded events, returns the sums since the last read and resets them. */
typedef struct mi_profile {
  double frames_ms;        /* rotate + bucket scan B (all chunks) */
  double eval_ms;          /* batched evaluator launches */
  double plain_ms;         /* per-pose stage sequences of the plain path */
  int64_t frame_launches;  /* frame-build sequences */
  int64_t eval_launches;   /* evaluator launches */
  int64_t plain_poses;     /* poses through the plain path */
  int64_t poses;           /* poses through the evaluator */
  int64_t point_poses;     /* sum over evaluated poses of the points of scan B */
} mi_profile;
mi_status mi_profile_enable(int32_t on);
mi_status mi_profile_read(mi_profile *out);

/* ------------------------------------------------------------------ grid */

/* Validate a grid description and copy it, with its bin edges, into a host
 * handle.  MI_E_INVALID for a bad description (dims < 1, V >= 2^31, voxel
 * <= 0 or non-finite, unknown features, nbins out of range, edges not
 * ascending, default z-variance edges undefined because voxel^2/4 <= 1e-5). */
mi_status mi_grid_create(const mi_grid_desc *desc, mi_grid **out);
void mi_grid_destroy(mi_grid *g);

/* The bin edges in use (host arrays of nbins_count-1 / nbins_zvar-2; either
 * pointer may be NULL). */
mi_status mi_grid_edges(const mi_grid *g, uint32_t *count_edges, uint64_t *zvar_edges);

/* The rotation and translation of pose eta as a row-major [R | t] (3x4), the
 * exact doubles every kernel uses (Sec. III-A: T as a rigid transform). */
mi_status mi_pose_to_matrix(const double eta[6], double rt[12]);

/* ------------------------------------------------------------- reference */

/* Workspace for mi_features_ref: the resident part (bins and per-bin
 * summed-volume tables of scan A, read by every evaluation) followed by a
 * transient part that is free again once the call has completed on the
 * stream.  persistent_bytes (nullable) receives the largest resident size
 * (every table at 4 bytes per entry); mi_ref_resident_bytes gives the size a
 * built reference keeps. */
size_t mi_features_ref_workspace(const mi_grid *g, int64_t n_a, size_t *persistent_bytes);

/* Alg. 1 initialisation: voxel ids of all points of scan A and A's feature
 * map for all voxels (bin 0 = empty), A's index box and what counts A's voxels
 * of each bin inside any overlap box: per occupied bin a summed-volume table
 * with the fewest bytes per entry (1, 2 or 4) that hold the bin's voxel count,
 * entries modulo 2^(8 width) (box counts, which lie between 0 and that count,
 * stay exact); on grids of at least 2^20 table entries (fewer than 2^20
 * voxels in x and y, 2^16 in z) the sparsest bins, up to 8192 voxels in all,
 * as a list of their voxels instead.  The call reads A's per-bin voxel counts
 * back once to lay this out, so it waits for the stream's work so far.
 * xyz_a: device SoA [3][n_a], n_a >= 0.  The grid must outlive the returned
 * mi_ref. */
mi_status mi_features_ref(const mi_grid *g, const float *xyz_a, int64_t n_a, void *ws,
                          size_t ws_bytes, void *stream, mi_ref **out);
void mi_ref_destroy(mi_ref *r);

/* Bytes at the start of the reference's workspace that the reference keeps
 * (bins, box, counters, the tables and voxel list as laid out for scan A);
 * the rest of the workspace may be reused by work ordered after
 * mi_features_ref on its stream.  0 for NULL. */
size_t mi_ref_resident_bytes(const mi_ref *r);

/* Moves a built reference into another workspace (device memory of at least
 * mi_ref_resident_bytes(r) bytes, 256-byte aligned, not overlapping the old
 * one): the resident bytes are copied on the stream and the reference then
 * lives there, so that a caller can build in a workspace sized for the worst
 * case and keep only what scan A needs.  The old workspace is free once the
 * copy, and every evaluation enqueued before it that reads the reference, has
 * completed.  Plans and batches created before the move still point at the old
 * workspace: create them after it.  The copy itself does not wait. */
mi_status mi_ref_move(mi_ref *r, void *ws, size_t ws_bytes, void *stream);

/* Device pointer to A's bin of every voxel for feature slot f (slot 0 = count
 * when enabled, then z-variance), uint8 [dims z][y][x]. */
mi_status mi_ref_bins(const mi_ref *r, int32_t feature_slot, const uint8_t **dev_bins);

/* Synchronizes the stream, then reads back A's index box (lo[3], hi[3]) and
 * counters (in-grid, out-of-grid, non-finite, occupied voxels). */
mi_status mi_ref_summary(const mi_ref *r, void *stream, int32_t box[6], int64_t counters[4]);

/* --------------------------------------------------------------- evaluate */

/* Workspace for evaluating the poses (host [n_poses][6]) against a scan B of
 * n_b points: pose tables, B's points rotated once per distinct rotation and
 * bucketed by column of A's grid, and scratch.  When the rotated copies would
 * exceed frame_budget_bytes (0 = 4 GiB) they are processed in chunks. */
size_t mi_eval_poses_workspace(const mi_ref *r, int64_t n_b, const double *poses, int64_t n_poses,
                               uint32_t flags, size_t frame_budget_bytes);

/* Eqs. 1-5 for every pose: MI per feature and pose.
 *   xyz_b      device SoA [3][n_b] (n_b < 2^20 when MI_FEAT_ZVAR is on)
 *   poses      host [n_poses][6] = tx, ty, tz (m), roll, pitch, yaw (rad)
 *   mi_out     device double [n_feat][n_poses]
 *   argmax_out device int64 [n_feat] or NULL
 *   hist_out   device uint32, feature f at offset sum_{f'<f} n_poses*nb_f'^2,
 *              pose k at + k*nb_f^2, rows = A bin, cols = B bin; or NULL
 *   stats_out  device mi_pose_stats [n_poses] or NULL
 * Pose tables are staged through library-owned pinned host memory, so the
 * host `poses` array may be reused as soon as the call returns. */
mi_status mi_eval_poses(const mi_ref *r, const float *xyz_b, int64_t n_b, const double *poses,
                        int64_t n_poses, uint32_t flags, double *mi_out, int64_t *argmax_out,
                        uint32_t *hist_out, mi_pose_stats *stats_out, void *ws, size_t ws_bytes,
                        void *stream);

/* mi_eval_poses without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments (less ws / ws_bytes) and results as
 * mi_eval_poses.  Its work memory is a static device array of
 * MI_STATIC_SCRATCH_BYTES per GPU, allocated with the library's code object
 * and held until the process ends; the call makes no device or pinned-host
 * allocation (pose tables are copied from pageable host memory).  Pose sets
 * whose tables, rotated frames or per-pose buckets cannot fit it fail with
 * MI_E_UNSUPPORTED; the per-pose form runs fewer workgroups when the buckets
 * of all of them would not fit.  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialized by the caller. */
#define MI_STATIC_SCRATCH_BYTES ((int64_t)256 << 20)
mi_status mi_eval_poses_static(const mi_ref *r, const float *xyz_b, int64_t n_b,
                               const double *poses, int64_t n_poses, uint32_t flags,
                               double *mi_out, int64_t *argmax_out, uint32_t *hist_out,
                               mi_pose_stats *stats_out, void *stream);

/* The paper-shaped path: for each pose in turn, one launch sequence of
 * transform + voxel mapping + extent, scatter into a dense per-pose voxel grid
 * in device memory, dense sweep of the overlap box into the joint histogram,
 * entropy (Table III stages).  Same arguments and results as mi_eval_poses;
 * kept as the per-pose baseline. */
size_t mi_eval_poses_plain_workspace(const mi_ref *r, int64_t n_b, int64_t n_poses);
mi_status mi_eval_poses_plain(const mi_ref *r, const float *xyz_b, int64_t n_b, const double *poses,
                              int64_t n_poses, uint32_t flags, double *mi_out, int64_t *argmax_out,
                              uint32_t *hist_out, mi_pose_stats *stats_out, void *ws,
                              size_t ws_bytes, void *stream);

/* Split form of mi_eval_poses for repeated launches (e.g. capture in a HIP
 * graph): mi_plan_create uploads the pose tables (enqueued on `stream`);
 * mi_plan_execute only launches kernels that read device tables, never
 * allocates, copies from the host or synchronizes, so it can be captured and
 * replayed.  The plan lives in `ws` (size from mi_eval_poses_workspace). */
mi_status mi_plan_create(const mi_ref *r, int64_t n_b, const double *poses, int64_t n_poses,
                         uint32_t flags, void *ws, size_t ws_bytes, size_t frame_budget_bytes,
                         void *stream, mi_plan **out);
mi_status mi_plan_execute(mi_plan *p, const float *xyz_b, double *mi_out, int64_t *argmax_out,
                          uint32_t *hist_out, mi_pose_stats *stats_out, void *stream);
void mi_plan_destroy(mi_plan *p);

/* The launch shape of a plan (tests, tracing): the tuning in force when it
 * was created, with the auto hash resolved to the size used, and the LDS bytes
 * of one evaluator workgroup.  Either output may be NULL. */
mi_status mi_plan_launch(const mi_plan *p, mi_tuning *t, int32_t *lds_bytes);

/* ------------------------------------------------------------ batches */

/* One scan pair and its pose set in a batch (Eq. 1 evaluated for every pose
 * of every item).  All pointers except `poses` are device memory owned by the
 * caller and must stay valid while the batch is executed.  Items may share a
 * reference or a scan B; grids, voxel sizes, bins and point counts may differ
 * from item to item. */
typedef struct mi_work_item {
  const mi_ref *ref;          /* scan A's reference features and grid */
  const float *xyz_b;         /* scan B, SoA [3][n_b] */
  int64_t n_b;
  const double *poses;        /* host [K][6] (read during mi_batch_create only) */
  int64_t K;
  double *mi_out;             /* [nf][K] */
  int64_t *argmax_out;        /* [nf] or NULL */
  uint32_t *hist_out;         /* [nf][K][nb_f][nb_f] or NULL */
  mi_pose_stats *stats_out;   /* [K] or NULL */
} mi_work_item;

/* The poses of many scan pairs evaluated as one schedule: every pair's
 * rotated frames are built together and a single evaluator launch per frame
 * chunk covers the poses of all pairs, so pairs of uneven size share the
 * device.  Results per item are those mi_eval_poses gives for the item alone
 * (bit-identical histograms and MI).  mi_batch_workspace sizes `ws`
 * (frame_budget_bytes as for mi_eval_poses_workspace; 0 on bad items).
 * mi_batch_create validates every item (MI_E_INVALID / MI_E_UNSUPPORTED name
 * the item in mi_last_error) and uploads the tables on `stream`;
 * mi_batch_execute only enqueues kernels (capturable in a HIP graph and
 * replayable; the items' buffers are fixed at creation).  The z-variance
 * feature in any item limits every item of the batch to n_b < 2^20.
 * mi_eval_batch = create + execute + destroy. */
size_t mi_batch_workspace(const mi_work_item *items, int64_t n_items, uint32_t flags,
                          size_t frame_budget_bytes);
mi_status mi_batch_create(const mi_work_item *items, int64_t n_items, uint32_t flags, void *ws,
                          size_t ws_bytes, size_t frame_budget_bytes, void *stream,
                          mi_plan **out);
mi_status mi_batch_execute(mi_plan *p, void *stream);
mi_status mi_eval_batch(const mi_work_item *items, int64_t n_items, uint32_t flags, void *ws,
                        size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ autotune */

/* Chooses the evaluator's launch shape (mi_tuning) for a workload by timing
 * it.  A sample of the items is built (each item's poses strided down to at
 * most max_poses, keeping the mix of rotations; max_poses <= 0 keeps all),
 * and executed as a batch under candidate tunings in three stages: waves per
 * workgroup x hash capacity, then stripe height x histogram copies around
 * the best, then one workgroup per pose against persistent grids of 1, 2 and
 * 4 workgroups per compute unit.  Each candidate is run once to warm up and
 * timed over two executions with HIP events on `stream` (synchronizing).
 * Candidates that a workload cannot use are skipped.  The fastest tuning,
 * possibly the one in force, is made current (process-wide; plans created
 * meanwhile by other threads may see the candidates) and reported.  Every
 * tuning gives bit-identical results, so the choice changes speed only.  The
 * items' own outputs are not written; ws (size from mi_autotune_workspace, 0
 * on bad items) holds the sample's outputs and batch. */
typedef struct mi_autotune_report {
  mi_tuning best;
  double best_ms;   /* one execution of the sample under `best` */
  double start_ms;  /* the same under the tuning in force before the call */
  int32_t tried;    /* candidates timed */
} mi_autotune_report;

size_t mi_autotune_workspace(const mi_work_item *items, int64_t n_items, uint32_t flags,
                             int64_t max_poses);
mi_status mi_autotune(const mi_work_item *items, int64_t n_items, uint32_t flags,
                      int64_t max_poses, void *ws, size_t ws_bytes, void *stream,
                      mi_autotune_report *out);

/* Tuning cache: a JSON file of one object whose members map a workload key to
 * a tuning, [waves, hash_bytes, hist_copies, stripe_rows, wgs_per_cu].  The
 * key names what the best launch shape depends on: the GPU architecture, the
 * feature set and bin counts, and the size classes of scan B and of the grid
 * (the ceiling of log2 of the largest point count and voxel count),
 * "<arch>/f<features>/b<nb0>x<nb1>/n<bits>/v<bits>"; buf receives it (len
 * bytes at most, NUL-terminated; MI_E_INVALID when it does not fit).
 * mi_tuning_cache_get sets *found to 1 and fills *t when the file has the key
 * (a missing file is an empty cache); mi_tuning_cache_put adds or replaces
 * it, rewriting the file through a temporary in the same directory.  Host
 * only: no device is used.  Not safe against concurrent writers. */
mi_status mi_tuning_cache_key(const char *arch, uint32_t features, int32_t nb0, int32_t nb1,
                              int64_t n_b, int64_t voxels, char *buf, size_t len);
mi_status mi_tuning_cache_get(const char *path, const char *key, mi_tuning *t, int32_t *found);
mi_status mi_tuning_cache_put(const char *path, const char *key, const mi_tuning *t);

/* mi_autotune through the cache at `path`: the items' key (their largest
 * scan B and grid, the first item's features and bin counts, the current
 * device's architecture) is looked up; a cached tuning is made current without
 * timing anything (report: that tuning, tried = 0, times 0); otherwise
 * mi_autotune runs and its best tuning is stored under the key. */
mi_status mi_autotune_cached(const mi_work_item *items, int64_t n_items, uint32_t flags,
                             int64_t max_poses, void *ws, size_t ws_bytes, void *stream,
                             const char *path, mi_autotune_report *out);

/* ------------------------------------------------------------- search */

/* Coarse-to-fine grid search for Eq. 1 from the initial guess T_o = init
 * (Alg. 1 outer loop, with the simplex update of Sec. III-B replaced by
 * re-centring a shrinking pose grid on the best pose).  Level l evaluates, per
 * axis, samples[a] nodes c + h*(-1 + 2j/(samples[a]-1)) (c alone when 1),
 * row-major over (tx, ty, tz, roll, pitch, yaw), yaw fastest; the next level is
 * centred on the argmax of feature slot `feature_slot` (or, with
 * MI_SLOT_WEIGHTED, of the weighted objective) with h divided by `shrink`.
 * mi_out gets that objective at the final pose.  Synchronizes the stream once
 * per level.  ws from mi_align_workspace. */
typedef struct mi_c2f_desc {
  double half_range[6];
  int32_t samples[6];           /* each 1..1024, product < 2^31 */
  int32_t levels;               /* >= 1 */
  double shrink;                /* > 0 */
  int32_t feature_slot;         /* 0 .. slots-1, or MI_SLOT_WEIGHTED */
  double weight[2];             /* per slot, when feature_slot == MI_SLOT_WEIGHTED */
} mi_c2f_desc;

size_t mi_align_workspace(const mi_ref *r, int64_t n_b, const mi_c2f_desc *d);
mi_status mi_align_coarse_to_fine(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                  const double init[6], const mi_c2f_desc *d, double pose_out[6],
                                  double *mi_out, void *ws, size_t ws_bytes, void *stream);

/* Simplex search for Eq. 1 (Alg. 1 with the Nelder-Mead update of
 * Sec. III-B): maximises the MI of feature slot `feature_slot` (or, with
 * MI_SLOT_WEIGHTED, the weighted objective) over the pose.
 * Each start gets a simplex of N + 1 = 7 vertices (the start, and the start
 * moved by step[i] along parameter i; Sec. IV uses steps 8, 8, 1 m, 0.1, 0.1,
 * 0.8 rad), improved with the usual coefficients (reflection 1, expansion 2,
 * contraction 1/2, shrink 1/2).  An iteration evaluates the reflection,
 * expansion and both contractions of the worst vertex together (speculatively)
 * and keeps the one the method asks for; a failed contraction shrinks the
 * simplex towards its best vertex.  A simplex stops after max_iter iterations
 * or when all its vertices are within xtol (max norm) and their MI within
 * ftol of its best.  The n_starts simplexes advance together: each round is
 * one batched evaluation of every pending point, then one synchronisation.
 * pose_out / mi_out: the best final vertex over all starts (ties: earlier
 * start); iters_out (host, [n_starts], nullable): iterations per start.
 * ws from mi_align_nm_workspace. */
typedef struct mi_nm_desc {
  double step[6];
  int32_t max_iter;
  double ftol;
  double xtol;
  int32_t feature_slot;         /* 0 .. slots-1, or MI_SLOT_WEIGHTED */
  double weight[2];             /* per slot, when feature_slot == MI_SLOT_WEIGHTED */
} mi_nm_desc;

size_t mi_align_nm_workspace(const mi_ref *r, int64_t n_b, int32_t n_starts);
mi_status mi_align_nelder_mead(const mi_ref *r, const float *xyz_b, int64_t n_b,
                               const double *starts, int32_t n_starts, const mi_nm_desc *d,
                               double pose_out[6], double *mi_out, int32_t *iters_out, void *ws,
                               size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ serving */

/* A request loop for many alignments (Alg. 1 per request, with the search of
 * mi_align_coarse_to_fine): continuous batching over one device arena.
 *
 * The caller hands the server one device range (`arena`, 256-aligned; the
 * server never allocates device memory) and a slot count.  Requests are
 * queued by mi_server_submit, which copies the host scans, so the caller may
 * free them at once.  Each mi_server_step admits queued requests in arrival
 * order while a slot is free and the request's data (scan B, scan A while its
 * reference is built, the reference features) fits the arena outside the
 * step region.  It then evaluates one search level of every active request
 * in one batch (mi_batch_*) and reads back the argmaxes.  A request whose
 * last level is done gives back its memory and slot.  Requests admitted
 * later join at their first level, so levels of different requests share
 * launches.  A request's result equals mi_align_coarse_to_fine on the same
 * inputs, bit for bit, whatever else is in flight.
 *
 * step_bytes is the part of the arena kept for each step's batch (0 = a
 * quarter): pose tables, outputs and rotated frames (chunked to fit).
 * mi_server_submit fails with MI_E_UNSUPPORTED for a request whose data
 * could never fit.  mi_server_submit and mi_server_poll may be called from
 * other threads while a step runs; steps are not reentrant.  Times are
 * seconds on a monotonic clock since the server was created. */
typedef struct mi_server mi_server;

typedef struct mi_server_desc {
  void *arena;          /* device memory owned by the caller */
  size_t arena_bytes;
  size_t step_bytes;    /* 0 = arena_bytes / 4 */
  int32_t max_active;   /* slots: requests in flight at once, >= 1 */
} mi_server_desc;

typedef struct mi_request {
  mi_grid_desc grid;    /* edges, if given, are copied */
  const float *xyz_a;   /* host SoA [3][n_a] */
  int64_t n_a;
  const float *xyz_b;   /* host SoA [3][n_b] */
  int64_t n_b;
  double init[6];       /* T_o */
  mi_c2f_desc search;
} mi_request;

#define MI_REQ_QUEUED 0
#define MI_REQ_ACTIVE 1
#define MI_REQ_DONE 2
#define MI_REQ_FAILED 3

typedef struct mi_request_state {
  int32_t state;        /* MI_REQ_* */
  int32_t levels_done;
  mi_status status;     /* MI_OK, or why the request failed */
  int32_t pad;
  double pose[6];       /* best pose after the last level */
  double mi;            /* its MI (feature slot of the search) */
  double t_submit, t_admit, t_done;
} mi_request_state;

mi_status mi_server_create(const mi_server_desc *d, void *stream, mi_server **out);
mi_status mi_server_submit(mi_server *s, const mi_request *r, int64_t *id);
mi_status mi_server_step(mi_server *s, int32_t *n_active, int32_t *n_queued);
mi_status mi_server_poll(mi_server *s, int64_t id, mi_request_state *out);
mi_status mi_server_release(mi_server *s, int64_t id); /* forget a finished request */
/* Arena bookkeeping (tests, monitoring): the request heap's size and its free
 * bytes now.  Once no request is queued or active every block is back, failed
 * requests included, and heap_free equals heap_bytes. */
mi_status mi_server_info(mi_server *s, size_t *heap_bytes, size_t *heap_free);
void mi_server_destroy(mi_server *s);

/* ------------------------------------------------------------ calibration */

/* Roofline microbenchmarks (measurement support, not part of the method):
 * launches one kernel of a known operation count on `stream` and returns that
 * count in *ops; the caller times the launch.  kind: 0 = LDS 32-bit atomic
 * add, 1 = LDS 64-bit atomic add, 2 = LDS compare-and-swap (lane operations,
 * conflict-free, iters = size rounds of 8 per lane), 3 = HBM stream read of
 * the scratch buffer (bytes; needs >= 16 KiB), 4 = FP64 VALU multiply and add
 * without contraction (lane operations, size rounds of 16 per lane).
 * scratch: device memory the kernel may write (>= 8 bytes per workgroup). */
mi_status mi_calibrate_launch(int32_t kind, int64_t size, void *scratch, int64_t scratch_bytes,
                              void *stream, double *ops);

#ifdef __cplusplus
}
#endif
#endif /* MI355_MI_H */
