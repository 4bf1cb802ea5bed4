// mi_api.hip -- host side of the C ABI declared in include/mi.h.
//
// Validation, the pose -> [R | t] formula, rotation de-duplication into
// frames, column grids and brick sizes, workspace carving, pinned staging of
// the pose tables, chunked execution and the coarse-to-fine driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mi.h"
#include "mi_internal.h"

#pragma clang fp contract(off)

using namespace mi;

// ------------------------------------------------------------------ errors

static thread_local std::string t_err;

static mi_status fail(mi_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

static mi_status dev_fail(hipError_t e, const char *where) {
  return fail(MI_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Every entry point runs its body under guarded(): a host allocation that
// fails (std::bad_alloc from a container) becomes a status, and no exception
// crosses the C ABI.  A size query reports 0, as for bad arguments.
template <class F>
static mi_status guarded(const char *where, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(MI_E_INVALID, "%s: out of host memory", where);
  } catch (...) {
    return fail(MI_E_INVALID, "%s: unexpected host error", where);
  }
}

template <class F>
static size_t guarded_size(F &&body) noexcept {
  try {
    return body();
  } catch (...) {
    return 0;
  }
}

#define HIP_TRY(expr, where)                   \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return dev_fail(_e, where); \
  } while (0)

extern "C" const char *mi_status_str(mi_status s) {
  switch (s) {
    case MI_OK: return "ok";
    case MI_E_INVALID: return "invalid argument";
    case MI_E_WORKSPACE: return "workspace too small or misaligned";
    case MI_E_DEVICE: return "device error";
    case MI_E_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

extern "C" const char *mi_last_error(void) { return t_err.c_str(); }

// --------------------------------------------------------------- workspace

namespace {

struct Carver {
  uintptr_t base, cur, end;
  explicit Carver(void *p, size_t n)
      : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + n) {}
  template <class T>
  T *take(size_t count) {
    cur = (cur + 255) & ~(uintptr_t)255;
    T *p = (T *)cur;
    cur += count * sizeof(T);
    return p;
  }
  size_t used() const { return (size_t)(cur - base); }
  bool fits() const { return cur <= end; }
};

// Pinned host buffers for uploading tables; a buffer is reused once the copy
// that read it has completed on its stream.
struct Staging {
  void *p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool busy = false, inflight = false;
};

std::mutex g_staging_mu;
std::vector<Staging *> g_staging;

Staging *staging_acquire(size_t bytes, hipError_t *err) {
  std::lock_guard<std::mutex> lk(g_staging_mu);
  for (Staging *s : g_staging) {
    if (s->busy || s->cap < bytes) continue;
    if (s->inflight && hipEventQuery(s->ev) != hipSuccess) continue;
    s->busy = true;
    s->inflight = false;
    return s;
  }
  Staging *s = new Staging();
  s->cap = std::max<size_t>(bytes, 1 << 20);
  *err = hipHostMalloc(&s->p, s->cap, hipHostMallocDefault);
  if (*err != hipSuccess) { delete s; return nullptr; }
  *err = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
  if (*err != hipSuccess) {
    (void)hipHostFree(s->p);  // *err keeps the failure that matters
    delete s;
    return nullptr;
  }
  s->busy = true;
  g_staging.push_back(s);
  return s;
}

struct Upload {
  void *dst;
  size_t off, bytes;
};

// Enqueue the copies out of the pinned buffer, then record the event that
// guards the buffer's reuse and hand the buffer back to the pool.
hipError_t staging_upload(Staging *s, const Upload *ups, int n, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i)
    if (ups[i].bytes)
      e = hipMemcpyAsync(ups[i].dst, (char *)s->p + ups[i].off, ups[i].bytes,
                         hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(s->ev, st);
  std::lock_guard<std::mutex> lk(g_staging_mu);
  s->busy = false;
  s->inflight = (e == hipSuccess);
  return e;
}

}  // namespace

// ------------------------------------------------------------------ tuning

namespace {
// Default hash (hash_bytes = 0, "auto"): 66 KiB, which with the histograms
// and plan entries of a 32-bin, two-feature launch still leaves two 80 KiB
// workgroups per compute unit; a launch whose other LDS needs are larger
// falls back to kFitHashBytes.  A size set by mi_tuning_set is used as given.
constexpr int32_t kAutoHashBytes = 66 * 1024;
constexpr int32_t kFitHashBytes = 60 * 1024;
constexpr int64_t kTwoWorkgroupLds = 80 * 1024;
// The tiled per-pose form under the auto tuning: one workgroup of this many
// waves per compute unit, its voxel hash taking the LDS the rest leaves.
constexpr int32_t kTileWaves = 16;
struct Tuning {
  int32_t waves = 8;
  int32_t hash_bytes = 0;  // 0: auto
  int32_t hist_copies = 1;
  int32_t stripe_rows = 16;
  int32_t wgs_per_cu = 0;
};
Tuning g_tuning;
std::mutex g_tuning_mu;

int max_lds_per_block() {
  static int v = -1;
  if (v < 0) {
    int dev = 0, x = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        x > 0)
      v = x;
    else
      v = 160 * 1024;
  }
  return v;
}
}  // namespace

extern "C" mi_status mi_tuning_set(const mi_tuning *t) {
  return guarded("mi_tuning_set", [&]() -> mi_status {
  if (!t) return fail(MI_E_INVALID, "mi_tuning_set: NULL");
  if (t->waves < 1 || t->waves > 16) return fail(MI_E_INVALID, "waves must be 1..16");
  if (t->hash_bytes != 0 && (t->hash_bytes < 1024 || t->hash_bytes > 160 * 1024))
    return fail(MI_E_INVALID, "hash_bytes must be 0 (auto) or in [1 KiB, 160 KiB]");
  if (t->hist_copies < 1 || t->hist_copies > 8) return fail(MI_E_INVALID, "hist_copies 1..8");
  if (t->stripe_rows < 1 || t->stripe_rows > 62) return fail(MI_E_INVALID, "stripe_rows 1..62");
  if (t->wgs_per_cu < 0 || t->wgs_per_cu > 16) return fail(MI_E_INVALID, "wgs_per_cu 0..16");
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning.waves = t->waves;
  g_tuning.hash_bytes = t->hash_bytes;
  g_tuning.hist_copies = t->hist_copies;
  g_tuning.stripe_rows = t->stripe_rows;
  g_tuning.wgs_per_cu = t->wgs_per_cu;
  return MI_OK;
  });
}

extern "C" mi_status mi_tuning_get(mi_tuning *t) {
  return guarded("mi_tuning_get", [&]() -> mi_status {
  if (!t) return fail(MI_E_INVALID, "mi_tuning_get: NULL");
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  t->waves = g_tuning.waves;
  t->hash_bytes = g_tuning.hash_bytes;
  t->hist_copies = g_tuning.hist_copies;
  t->stripe_rows = g_tuning.stripe_rows;
  t->wgs_per_cu = g_tuning.wgs_per_cu;
  return MI_OK;
  });
}

static Tuning tuning_now() {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return g_tuning;
}

// ---------------------------------------------------------------- profiling

namespace {
enum Stage { kStageFrames = 0, kStageEval = 1, kStagePlain = 2 };
struct Span {
  hipEvent_t a, b;
  int stage;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Span> g_spans;
std::vector<hipEvent_t> g_event_pool;
int64_t g_prof_counts[5] = {0, 0, 0, 0, 0};  // frame, eval launches, plain poses, poses, point-poses

hipEvent_t prof_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a stage on `s`; returns false when timing is off.
bool prof_begin(hipStream_t s, hipEvent_t *a) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return false;
  *a = prof_event();
  if (!*a) return false;
  if (hipEventRecord(*a, s) != hipSuccess) {
    g_event_pool.push_back(*a);
    return false;
  }
  return true;
}

void prof_end(hipStream_t s, hipEvent_t a, int stage, int64_t poses, int64_t point_poses) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t b = prof_event();
  if (!b || hipEventRecord(b, s) != hipSuccess) return;
  g_spans.push_back({a, b, stage});
  if (stage == kStageFrames) g_prof_counts[0] += 1;
  if (stage == kStageEval) {
    g_prof_counts[1] += 1;
    g_prof_counts[3] += poses;
    g_prof_counts[4] += point_poses;
  }
  if (stage == kStagePlain) g_prof_counts[2] += poses;
}
}  // namespace

extern "C" mi_status mi_profile_enable(int32_t on) {
  return guarded("mi_profile_enable", [&]() -> mi_status {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  // the recorded spans' events go back to the pool once their work is done
  hipError_t e = hipSuccess;
  for (auto &sp : g_spans) {
    const hipError_t es = hipEventSynchronize(sp.b);
    if (e == hipSuccess) e = es;
    g_event_pool.push_back(sp.a);
    g_event_pool.push_back(sp.b);
  }
  g_spans.clear();
  for (auto &c : g_prof_counts) c = 0;
  g_prof_on = on != 0;
  if (e != hipSuccess) return dev_fail(e, "profile spans");
  return MI_OK;
  });
}

extern "C" mi_status mi_profile_read(mi_profile *out) {
  return guarded("mi_profile_read", [&]() -> mi_status {
  if (!out) return fail(MI_E_INVALID, "mi_profile_read: NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms[3] = {0, 0, 0};
  for (auto &sp : g_spans) {
    HIP_TRY(hipEventSynchronize(sp.b), "profile sync");
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, sp.a, sp.b), "profile elapsed");
    ms[sp.stage] += t;
    g_event_pool.push_back(sp.a);
    g_event_pool.push_back(sp.b);
  }
  g_spans.clear();
  out->frames_ms = ms[0];
  out->eval_ms = ms[1];
  out->plain_ms = ms[2];
  out->frame_launches = g_prof_counts[0];
  out->eval_launches = g_prof_counts[1];
  out->plain_poses = g_prof_counts[2];
  out->poses = g_prof_counts[3];
  out->point_poses = g_prof_counts[4];
  for (auto &c : g_prof_counts) c = 0;
  return MI_OK;
  });
}

// -------------------------------------------------------------------- grid

struct mi_grid {
  GridInfo gi;
};

// Default z-variance edges: nb-2 edges log-spaced from 1e-5 m^2 to voxel^2/4,
// in units of (voxel/2^20)^2, rounded up.
static int default_zvar_edges(double voxel, int nb, uint64_t *E) {
  const int m = nb - 2;
  const double lo = 1e-5, hi = voxel * voxel / 4.0;
  if (m < 1 || !(hi > lo)) return -1;
  const double scale = (1048576.0 / voxel) * (1048576.0 / voxel);
  for (int j = 0; j < m; ++j) {
    const double e = (m == 1) ? lo : lo * std::pow(hi / lo, (double)j / (double)(m - 1));
    const double v = std::ceil(e * scale);
    if (!(v < 1.8446744073709552e19)) return -1;
    E[j] = (uint64_t)v;
  }
  return 0;
}

extern "C" mi_status mi_grid_create(const mi_grid_desc *d, mi_grid **out) {
  return guarded("mi_grid_create", [&]() -> mi_status {
  if (!d || !out) return fail(MI_E_INVALID, "mi_grid_create: NULL argument");
  *out = nullptr;
  GridInfo gi;
  memset(&gi, 0, sizeof gi);
  for (int a = 0; a < 3; ++a) {
    if (d->dims[a] < 1) return fail(MI_E_INVALID, "dims[%d] = %d < 1", a, d->dims[a]);
    if (!std::isfinite(d->origin[a])) return fail(MI_E_INVALID, "origin not finite");
    gi.origin[a] = d->origin[a];
    gi.dims[a] = d->dims[a];
  }
  gi.V = (int64_t)d->dims[0] * d->dims[1] * d->dims[2];
  if (gi.V >= ((int64_t)1 << 31)) return fail(MI_E_INVALID, "grid has %lld >= 2^31 voxels",
                                              (long long)gi.V);
  if (!(d->voxel > 0.0) || !std::isfinite(d->voxel)) return fail(MI_E_INVALID, "voxel <= 0");
  gi.voxel = d->voxel;
  gi.s = 1.0 / d->voxel;
  const uint32_t all = MI_FEAT_COUNT | MI_FEAT_ZVAR | MI_FEAT_JOINT;
  if (d->features == 0 || (d->features & ~all) || d->features == all)
    return fail(MI_E_INVALID, "features bitmask %u (one or two of count, z-variance, joint)",
                d->features);
  gi.features = d->features;
  gi.nf = 0;
  if (d->features & (MI_FEAT_COUNT | MI_FEAT_JOINT)) {
    const int nb = d->nbins_count;
    if (nb < 2 || nb > kMaxBins) return fail(MI_E_INVALID, "nbins_count %d not in 2..64", nb);
    if (d->count_edges) {
      for (int j = 0; j < nb - 1; ++j) gi.count_edges[j] = d->count_edges[j];
      if (gi.count_edges[0] < 1) return fail(MI_E_INVALID, "count_edges[0] must be >= 1");
      for (int j = 1; j < nb - 1; ++j)
        if (gi.count_edges[j] < gi.count_edges[j - 1])
          return fail(MI_E_INVALID, "count_edges not ascending");
    } else {
      for (int j = 0; j < nb - 1; ++j) gi.count_edges[j] = (uint32_t)(j + 1);
    }
    gi.nbc = nb;
  }
  if (d->features & (MI_FEAT_ZVAR | MI_FEAT_JOINT)) {
    const int nb = d->nbins_zvar;
    const int lo = (d->features & MI_FEAT_ZVAR) ? 3 : 2;
    if (nb < lo || nb > kMaxBins) return fail(MI_E_INVALID, "nbins_zvar %d not in %d..64", nb, lo);
    if (nb == 2) {
      // the joint feature's z part with no edges: every occupied voxel is bin 1
    } else if (d->zvar_edges) {
      for (int j = 0; j < nb - 2; ++j) gi.zvar_edges[j] = d->zvar_edges[j];
      for (int j = 1; j < nb - 2; ++j)
        if (gi.zvar_edges[j] < gi.zvar_edges[j - 1])
          return fail(MI_E_INVALID, "zvar_edges not ascending");
    } else if (default_zvar_edges(d->voxel, nb, gi.zvar_edges)) {
      return fail(MI_E_INVALID, "default z-variance edges need voxel^2/4 > 1e-5 m^2");
    }
    gi.nbz = nb;
  }
  if (d->features & MI_FEAT_COUNT) {
    gi.kind[gi.nf] = MI_FEAT_COUNT;
    gi.nb[gi.nf++] = gi.nbc;
  }
  if (d->features & MI_FEAT_ZVAR) {
    gi.kind[gi.nf] = MI_FEAT_ZVAR;
    gi.nb[gi.nf++] = gi.nbz;
  }
  if (d->features & MI_FEAT_JOINT) {
    const int nbj = 1 + (gi.nbc - 1) * (gi.nbz - 1);
    if (nbj > kMaxBins)
      return fail(MI_E_INVALID, "joint feature has %d bins > 64 ((nbins_count-1)*(nbins_zvar-1)+1)",
                  nbj);
    gi.kind[gi.nf] = MI_FEAT_JOINT;
    gi.nb[gi.nf++] = nbj;
  }
  mi_grid *g = (mi_grid *)malloc(sizeof(mi_grid));
  if (!g) return fail(MI_E_INVALID, "out of host memory");
  g->gi = gi;
  *out = g;
  return MI_OK;
  });
}

extern "C" void mi_grid_destroy(mi_grid *g) { free(g); }

extern "C" mi_status mi_grid_edges(const mi_grid *g, uint32_t *ce, uint64_t *ze) {
  return guarded("mi_grid_edges", [&]() -> mi_status {
  if (!g) return fail(MI_E_INVALID, "mi_grid_edges: NULL grid");
  if (ce)
    for (int j = 0; j + 1 < g->gi.nbc; ++j) ce[j] = g->gi.count_edges[j];
  if (ze)
    for (int j = 0; j + 2 < g->gi.nbz; ++j) ze[j] = g->gi.zvar_edges[j];
  return MI_OK;
  });
}

// ---------------------------------------------------------------- pose

// R = Rz(yaw) Ry(pitch) Rx(roll), each product and sum rounded on its own.
static void pose_rotation(const double eta[6], double R[9]) {
  const double cr = std::cos(eta[3]), sr = std::sin(eta[3]);
  const double cp = std::cos(eta[4]), sp = std::sin(eta[4]);
  const double cy = std::cos(eta[5]), sy = std::sin(eta[5]);
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

extern "C" mi_status mi_pose_to_matrix(const double eta[6], double rt[12]) {
  return guarded("mi_pose_to_matrix", [&]() -> mi_status {
  if (!eta || !rt) return fail(MI_E_INVALID, "mi_pose_to_matrix: NULL");
  double R[9];
  pose_rotation(eta, R);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) rt[4 * r + c] = R[3 * r + c];
    rt[4 * r + 3] = eta[r];
  }
  return MI_OK;
  });
}

// -------------------------------------------------------------- reference

struct mi_ref {
  const mi_grid *g;
  RefDev rd;
  int64_t n_a;
  size_t resident;             // bytes of the workspace the reference keeps
  uint8_t *base;               // the workspace it keeps them in
};

static int64_t sat_plane(const GridInfo &gi) {
  return (int64_t)(gi.dims[0] + 1) * (gi.dims[1] + 1) * (gi.dims[2] + 1);
}

// Resident part: bins, box and counters, per-bin voxel counts and list
// cursors, then the region of the tables and the voxel list, last so that
// what they leave unused is the resident part's tail (the region is sized for
// a 4-byte table per bin; ref_finish lays it out once the bins are counted).
// Transient part: the per-voxel sums.
static size_t ref_layout(const GridInfo &gi, Carver &c, RefDev *rd, uint8_t **sat_region) {
  const int64_t V = gi.V;
  uint8_t *bins[2] = {nullptr, nullptr};
  for (int f = 0; f < gi.nf; ++f) bins[f] = c.take<uint8_t>((size_t)V);
  int32_t *abox = c.take<int32_t>(8);
  unsigned long long *ctr = c.take<unsigned long long>(4);
  uint32_t *bin_cnt = c.take<uint32_t>(128);
  uint32_t *list_cur = c.take<uint32_t>(128);
  size_t region = 0;
  for (int f = 0; f < gi.nf; ++f)
    region += (size_t)(gi.nb[f] - 1) * (size_t)sat_table_bytes(sat_plane(gi), 4);
  uint8_t *sat = c.take<uint8_t>(region);
  const size_t persistent = c.used();
  uint32_t *cnt = c.take<uint32_t>((size_t)V);
  unsigned long long *s1 = c.take<unsigned long long>((size_t)V);
  unsigned long long *s2 = c.take<unsigned long long>((size_t)V);
  if (rd) {
    for (int f = 0; f < 2; ++f) {
      rd->bins[f] = bins[f];
      rd->sat[f] = nullptr;  // placed once the bins are counted
    }
    rd->bin_cnt = bin_cnt;
    rd->list_cur = list_cur;
    rd->abox = abox;
    rd->counters = ctr;
    rd->cnt = cnt;
    rd->s1 = s1;
    rd->s2 = s2;
  }
  if (sat_region) *sat_region = sat;
  return persistent;
}

extern "C" size_t mi_features_ref_workspace(const mi_grid *g, int64_t, size_t *persistent_bytes) {
  return guarded_size([&]() -> size_t {
  if (!g) return 0;
  Carver c(nullptr, 0);
  const size_t pers = ref_layout(g->gi, c, nullptr, nullptr);
  if (persistent_bytes) *persistent_bytes = pers;
  return c.used() + 256;
  });
}

// A reference under construction: its bins and per-bin voxel counts are
// enqueued (ref_begin), the counts are copied to host memory, and once they
// have arrived the tables are laid out and built (ref_finish).  The server
// begins all of a step's new references before it waits once for their counts.
struct RefBuild {
  RefDev rd;
  uint8_t *sat_region;
  void *ws;
  int64_t n_a;
};

static mi_status ref_begin(const mi_grid *g, const float *xyz_a, int64_t n_a, void *ws,
                           size_t ws_bytes, hipStream_t hs, uint32_t *counts_host, RefBuild *b) {
  if (n_a < 0 || (n_a > 0 && !xyz_a)) return fail(MI_E_INVALID, "bad scan A");
  if (n_a >= ((int64_t)1 << 32)) return fail(MI_E_UNSUPPORTED, "n_a >= 2^32");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  const GridInfo &gi = g->gi;
  Carver c(ws, ws_bytes);
  RefDev &rd = b->rd;
  memset(&rd, 0, sizeof rd);
  ref_layout(gi, c, &rd, &b->sat_region);
  if (!c.fits()) return fail(MI_E_WORKSPACE, "features_ref workspace needs %zu bytes, got %zu",
                             c.used(), ws_bytes);
  b->ws = ws;
  b->n_a = n_a;
  rd.nx = gi.dims[0]; rd.ny = gi.dims[1]; rd.nz = gi.dims[2]; rd.nf = gi.nf;
  for (int f = 0; f < 2; ++f) { rd.kind[f] = gi.kind[f]; rd.nb[f] = gi.nb[f]; }
  rd.nbc = gi.nbc;
  rd.nbz = gi.nbz;
  rd.s = gi.s;
  for (int a = 0; a < 3; ++a) rd.c0[a] = (0.0 - gi.origin[a]) * gi.s;
  memcpy(rd.count_edges, gi.count_edges, sizeof rd.count_edges);
  memcpy(rd.zvar_edges, gi.zvar_edges, sizeof rd.zvar_edges);
  HIP_TRY(launch_ref_bins(rd, xyz_a, n_a, hs), "features_ref launch");
  HIP_TRY(hipMemcpyAsync(counts_host, rd.bin_cnt, 128 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         hs),
          "bin counts");
  return MI_OK;
}

// counts: the 128 per-bin voxel counts ref_begin copied out, already arrived.
// The layout follows them.  An empty bin has no table.  On a grid of at least
// 2^20 table entries, the sparsest bins, in ascending count up to kListMax
// voxels in all, are kept as a voxel list instead of a table (each frees at
// least 4 MiB of the region sized for 4-byte tables; the list takes at most
// 64 KiB).  Every other bin gets a table with the fewest bytes per entry that
// hold its count.
static mi_status ref_finish(const mi_grid *g, RefBuild &b, const uint32_t *counts, hipStream_t hs,
                            mi_ref **out) {
  const GridInfo &gi = g->gi;
  RefDev &rd = b.rd;
  std::unique_ptr<mi_ref, void (*)(mi_ref *)> r((mi_ref *)calloc(1, sizeof(mi_ref)),
                                                 [](mi_ref *p) { free(p); });
  if (!r) return fail(MI_E_INVALID, "out of host memory");
  const int64_t plane = sat_plane(gi);
  uint32_t listed = 0;
  if (plane >= ((int64_t)1 << 20) && list_fits(gi.dims[0], gi.dims[1], gi.dims[2])) {
    std::vector<std::pair<uint32_t, int>> sparse;
    for (int f = 0; f < gi.nf; ++f)
      for (int a = 1; a < gi.nb[f]; ++a) {
        const uint32_t n = counts[64 * f + a];
        if (n > 0 && n < 65536u) sparse.push_back({n, 64 * f + a});
      }
    std::sort(sparse.begin(), sparse.end());
    for (const auto &sb : sparse) {
      if (listed + sb.first > kListMax) break;
      listed += sb.first;
      rd.list_mask[sb.second >> 6] |= 1ull << (sb.second & 63);
    }
  }
  size_t used = 0;
  for (int f = 0; f < gi.nf; ++f) {
    rd.sat[f] = b.sat_region + used;
    SatLayout &L = rd.sat_layout[f];
    for (int a = 1; a < gi.nb[f]; ++a) {
      const uint32_t n = counts[64 * f + a];
      if (n == 0 || ((rd.list_mask[f] >> a) & 1u)) continue;
      L.mask[n < 256u ? 0 : n < 65536u ? 1 : 2] |= 1ull << a;
    }
    used += (size_t)sat_offset(L, gi.nb[f], plane);
  }
  rd.alist = listed ? (uint64_t *)(b.sat_region + used) : nullptr;
  rd.alist_n = listed;
  used += ((size_t)listed * sizeof(uint64_t) + 255) & ~(size_t)255;
  HIP_TRY(launch_ref_sat(rd, hs), "features_ref tables");
  r->g = g;
  r->rd = rd;
  r->n_a = b.n_a;
  r->resident = (size_t)(b.sat_region - (uint8_t *)b.ws) + used;
  r->base = (uint8_t *)b.ws;
  *out = r.release();
  return MI_OK;
}

extern "C" mi_status mi_features_ref(const mi_grid *g, const float *xyz_a, int64_t n_a, void *ws,
                                     size_t ws_bytes, void *stream, mi_ref **out) {
  return guarded("mi_features_ref", [&]() -> mi_status {
  if (!g || !out) return fail(MI_E_INVALID, "mi_features_ref: NULL argument");
  *out = nullptr;
  const hipStream_t hs = (hipStream_t)stream;
  RefBuild b;
  uint32_t counts[128];
  const mi_status st = ref_begin(g, xyz_a, n_a, ws, ws_bytes, hs, counts, &b);
  if (st != MI_OK) return st;
  HIP_TRY(hipStreamSynchronize(hs), "bin counts");
  return ref_finish(g, b, counts, hs, out);
  });
}

extern "C" void mi_ref_destroy(mi_ref *r) { free(r); }

extern "C" size_t mi_ref_resident_bytes(const mi_ref *r) { return r ? r->resident : 0; }

extern "C" mi_status mi_ref_move(mi_ref *r, void *ws, size_t ws_bytes, void *stream) {
  return guarded("mi_ref_move", [&]() -> mi_status {
  if (!r) return fail(MI_E_INVALID, "mi_ref_move: NULL reference");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  if (ws_bytes < r->resident)
    return fail(MI_E_WORKSPACE, "mi_ref_move needs %zu bytes, got %zu", r->resident, ws_bytes);
  uint8_t *nb = (uint8_t *)ws, *ob = r->base;
  if (nb == ob) return MI_OK;
  if (nb < ob + r->resident && ob < nb + r->resident)
    return fail(MI_E_INVALID, "mi_ref_move: the workspaces overlap");
  HIP_TRY(hipMemcpyAsync(nb, ob, r->resident, hipMemcpyDeviceToDevice, (hipStream_t)stream),
          "reference copy");
  // every resident address keeps its offset; the per-voxel sums are gone
  auto at = [&](auto *p) { return p ? (decltype(p))(nb + ((uint8_t *)p - ob)) : p; };
  RefDev &rd = r->rd;
  for (int f = 0; f < 2; ++f) {
    rd.bins[f] = at(rd.bins[f]);
    rd.sat[f] = at(rd.sat[f]);
  }
  rd.alist = at(rd.alist);
  rd.abox = at(rd.abox);
  rd.counters = at(rd.counters);
  rd.bin_cnt = at(rd.bin_cnt);
  rd.list_cur = at(rd.list_cur);
  rd.cnt = nullptr;
  rd.s1 = rd.s2 = nullptr;
  r->base = nb;
  return MI_OK;
  });
}

extern "C" mi_status mi_ref_bins(const mi_ref *r, int32_t f, const uint8_t **dev_bins) {
  return guarded("mi_ref_bins", [&]() -> mi_status {
  if (!r || !dev_bins || f < 0 || f >= r->g->gi.nf)
    return fail(MI_E_INVALID, "mi_ref_bins: bad argument");
  *dev_bins = r->rd.bins[f];
  return MI_OK;
  });
}

extern "C" mi_status mi_ref_summary(const mi_ref *r, void *stream, int32_t box[6],
                                    int64_t counters[4]) {
  return guarded("mi_ref_summary", [&]() -> mi_status {
  if (!r || !box || !counters) return fail(MI_E_INVALID, "mi_ref_summary: NULL");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "ref summary sync");
  HIP_TRY(hipMemcpy(box, r->rd.abox, 6 * sizeof(int32_t), hipMemcpyDeviceToHost), "ref box");
  unsigned long long c[4];
  HIP_TRY(hipMemcpy(c, r->rd.counters, sizeof c, hipMemcpyDeviceToHost), "ref counters");
  for (int i = 0; i < 4; ++i) counters[i] = (int64_t)c[i];
  return MI_OK;
  });
}

// ------------------------------------------------------------------ plans

namespace {

struct PoseTables {
  int64_t K = 0;
  int32_t F = 0;                     // distinct rotations
  std::vector<double> R;             // [F][9]
  std::vector<PoseDev> items;        // sorted by frame
  int32_t gx = 0, gy = 0, ncx = 1, ncy = 1, zlo = 0, zhi = 0;
};

// Open-addressing index from keys of N 64-bit words to int32 values (linear
// probing, power-of-two capacity kept at most half full).  Plan creation looks
// up every pose's rotation in it: a search level of 15,625 poses shares 125.
template <int N>
class WordIndex {
 public:
  WordIndex() { rehash(256); }
  int32_t find(const uint64_t *k) const {  // the key's value, or -1
    for (size_t i = slot_of(k);; i = (i + 1) & mask_) {
      const int32_t v = vals_[i];
      if (v < 0) return -1;
      if (memcmp(&keys_[i * N], k, N * sizeof(uint64_t)) == 0) return v;
    }
  }
  void insert(const uint64_t *k, int32_t v) {  // a key not yet present, v >= 0
    if (2 * (count_ + 1) > vals_.size()) rehash(2 * vals_.size());
    size_t i = slot_of(k);
    while (vals_[i] >= 0) i = (i + 1) & mask_;
    memcpy(&keys_[i * N], k, N * sizeof(uint64_t));
    vals_[i] = v;
    ++count_;
  }

 private:
  size_t slot_of(const uint64_t *k) const {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int j = 0; j < N; ++j) {
      h = (h ^ k[j]) * 0xff51afd7ed558ccdull;
      h ^= h >> 32;
    }
    return (size_t)h & mask_;
  }
  void rehash(size_t cap) {
    std::vector<uint64_t> old_keys;
    std::vector<int32_t> old_vals;
    old_keys.swap(keys_);
    old_vals.swap(vals_);
    keys_.assign(cap * N, 0);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    count_ = 0;
    for (size_t i = 0; i < old_vals.size(); ++i)
      if (old_vals[i] >= 0) insert(&old_keys[i * N], old_vals[i]);
  }
  std::vector<uint64_t> keys_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0, count_ = 0;
};

// Distinct rotations, per-pose translation offsets c = fl(fl(t - origin) * s),
// items sorted by frame, and the column grid covering every rotated position
// from which some pose's offset reaches A's grid.  Poses with bit-identical
// (roll, pitch, yaw) share a frame; the matrix is built once per distinct
// triple, and poses whose different triples give bit-identical matrices are
// merged too.
int build_tables(const GridInfo &gi, const double *poses, int64_t K, PoseTables &T) {
  T.K = K;
  T.R.clear();
  std::vector<PoseDev> items((size_t)K);
  WordIndex<3> by_angles;
  WordIndex<9> by_matrix;
  // Pose sets often cycle through their rotations (a pose grid varies the
  // angles fastest): once a rotation repeats, the pose one cycle back is
  // compared first, and the index is searched only when it differs.
  std::vector<int64_t> last_use;  // per frame: the latest pose with its rotation
  int64_t period = 0;
  double cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = 0; k < K; ++k) {
    const double *eta = poses + 6 * k;
    for (int a = 0; a < 6; ++a)
      if (!std::isfinite(eta[a])) return -1;
    int32_t fidx = -1;
    if (period > 0 && k >= period &&
        memcmp(poses + 6 * (k - period) + 3, eta + 3, 3 * sizeof(double)) == 0) {
      fidx = items[(size_t)(k - period)].frame;
    } else {
      uint64_t ak[3];
      memcpy(ak, eta + 3, sizeof ak);
      fidx = by_angles.find(ak);
      if (fidx >= 0) {
        period = k - last_use[(size_t)fidx];
      } else {
        double R[9];
        pose_rotation(eta, R);
        uint64_t key[9];
        memcpy(key, R, sizeof key);
        fidx = by_matrix.find(key);
        if (fidx < 0) {
          fidx = (int32_t)(T.R.size() / 9);
          by_matrix.insert(key, fidx);
          T.R.insert(T.R.end(), R, R + 9);
          last_use.push_back(k);
        }
        by_angles.insert(ak, fidx);
      }
    }
    last_use[(size_t)fidx] = k;
    PoseDev &p = items[(size_t)k];
    p.pair = 0;
    p.frame = fidx;
    p.out_index = (int32_t)k;
    p.pad = 0;
    for (int a = 0; a < 3; ++a) {
      p.c[a] = (eta[a] - gi.origin[a]) * gi.s;
      cmin[a] = std::min(cmin[a], p.c[a]);
      cmax[a] = std::max(cmax[a], p.c[a]);
    }
  }
  T.F = (int32_t)(T.R.size() / 9);
  // counting sort by frame, stable within a frame
  {
    std::vector<int64_t> start((size_t)T.F + 1, 0);
    for (const PoseDev &p : items) ++start[(size_t)p.frame + 1];
    for (int32_t f = 0; f < T.F; ++f) start[(size_t)f + 1] += start[(size_t)f];
    T.items.resize((size_t)K);
    for (const PoseDev &p : items) T.items[(size_t)start[(size_t)p.frame]++] = p;
  }
  if (K == 0) { cmin[0] = cmin[1] = cmin[2] = cmax[0] = cmax[1] = cmax[2] = 0.0; }
  // v in (-c - eps, dims - c + eps) for some pose: columns floor(v) within
  // [floor(min(-c)) - 1, floor(max(dims - c)) + 1].
  const double lo_x = std::floor(-cmax[0]) - 1.0, hi_x = std::floor(gi.dims[0] - cmin[0]) + 1.0;
  const double lo_y = std::floor(-cmax[1]) - 1.0, hi_y = std::floor(gi.dims[1] - cmin[1]) + 1.0;
  const double lo_z = std::floor(-cmax[2]) - 1.0, hi_z = std::floor(gi.dims[2] - cmin[2]) + 1.0;
  if (!(hi_x - lo_x < 1e6 && hi_y - lo_y < 1e6 && std::fabs(lo_x) < 1e9 && std::fabs(lo_y) < 1e9 &&
        std::fabs(lo_z) < 1e9 && std::fabs(hi_z) < 1e9))
    return -2;
  T.gx = (int32_t)lo_x;
  T.gy = (int32_t)lo_y;
  T.ncx = (int32_t)(hi_x - lo_x) + 1;
  T.ncy = (int32_t)(hi_y - lo_y) + 1;
  T.zlo = (int32_t)lo_z;
  T.zhi = (int32_t)hi_z;
  if ((int64_t)T.ncx * T.ncy >= ((int64_t)1 << 31)) return -2;
  return 0;
}

int bits_for(int64_t n) {  // bits to hold 0..n-1
  int b = 0;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}

// Stripes, plan pieces, hash capacity and key packing of one pair under a
// tuning (see k_eval.hip for how the evaluator uses them).
struct StripeShape {
  int stripe_h, n_stripes, pieces, kx_bits, ky_bits, cap, plan_stripes, plan_entries;
  bool zvar;
};

bool choose_stripes(const GridInfo &gi, const Tuning &tu, bool zvar, StripeShape &S,
                    const char **why) {
  S.zvar = zvar;
  const int slot = eval_hash_slot_bytes(S.zvar);
  // slots: as many as hash_bytes holds, a multiple of 64, at most 65536 (the
  // occupied list stores slot indices in 16 bits)
  const int64_t cap = std::min<int64_t>(65536, ((int64_t)tu.hash_bytes / slot) & ~(int64_t)63);
  if (cap < 64) { *why = "hash_bytes too small"; return false; }
  S.cap = (int)cap;
  // bricks of at most a quarter of the slots in voxels always fit; single voxel
  // rows of an x piece must be such bricks
  const int64_t load_max = cap / 4;
  const int nx = gi.dims[0], ny = gi.dims[1], nz = gi.dims[2];
  const int64_t wmax = load_max / nz;  // widest x piece whose single voxel row always fits
  if (wmax < 1) { *why = "grid height exceeds the voxel hash"; return false; }
  S.stripe_h = std::max(1, std::min(tu.stripe_rows, std::min(ny, 62)));
  S.n_stripes = (ny + S.stripe_h - 1) / S.stripe_h;
  int64_t Q = std::max<int64_t>(8, (nx + wmax - 1) / wmax);
  if (Q > 1024) { *why = "grid too wide for the plan"; return false; }
  S.pieces = (int)Q;
  S.kx_bits = bits_for(nx);
  S.ky_bits = bits_for(S.stripe_h);
  if (S.kx_bits + S.ky_bits + bits_for(nz) > 31) { *why = "grid dims exceed the voxel key"; return false; }
  S.plan_entries = (S.stripe_h + 2) * (S.pieces + 1);
  S.plan_stripes = (int)std::max<int64_t>(1, std::min<int64_t>(S.n_stripes,
                                                                4096 / (S.plan_entries * 8)));
  return true;
}

// ------------------------------------------------------------- scan B tiles

// Halo width of the tiled per-pose form, in voxels: above half a voxel
// diagonal (0.866), with room for the rounding of the two transforms.
constexpr double kTileHalo = 0.88;

// Most tiles of a scan of n_b points (fixes the tile tables' size before the
// scan is read).
int64_t tiles_max(int64_t n_b) { return std::max<int64_t>(1, n_b / 128); }

struct TileGeom {
  double x0 = 0.0, y0 = 0.0, ilx = 1.0, ily = 1.0, hx = 0.0, hy = 0.0;
  int32_t nx = 1, ny = 1;
  double coherence = 0.0;  // share of consecutive finite points in one voxel of B's own frame
  bool known = false;
};

// Tiles of scan B's own (x, y) frame: the box of its finite points (outliers
// aside) cut into nx x ny equal tiles, as many as keep the distinct voxels of
// a tile and its halo near half of the hash slots (counted on voxels of B's
// own frame, per cell of a grid of at most 256 x 256 cells over the box; a
// posed scan fills somewhat more, and a tile that overflows is redone in
// parts).  Tiles are at least three halo widths wide, so the halo of a tile
// only takes points of its 8 neighbours.  Also measures how often
// consecutive points share a voxel (scanner order: often; surface samples in
// random order: almost never), which decides between tiles and shared frames.
TileGeom choose_tiles(const float *xyz, int64_t n, double voxel, int32_t cap) {
  TileGeom g;
  g.known = true;
  const float *X = xyz, *Y = xyz + n, *Z = xyz + 2 * n;
  std::vector<float> xs, ys, zs;
  xs.reserve((size_t)n);
  ys.reserve((size_t)n);
  zs.reserve((size_t)n);
  int64_t same = 0, links = 0;
  double px = 0.0, py = 0.0, pz = 0.0;
  bool prev = false;
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(X[i]) || !std::isfinite(Y[i]) || !std::isfinite(Z[i])) {
      prev = false;
      continue;
    }
    const double cx = std::floor(X[i] / voxel), cy = std::floor(Y[i] / voxel),
                 cz = std::floor(Z[i] / voxel);
    if (prev) {
      ++links;
      same += cx == px && cy == py && cz == pz;
    }
    px = cx; py = cy; pz = cz;
    prev = true;
    xs.push_back(X[i]);
    ys.push_back(Y[i]);
    zs.push_back(Z[i]);
  }
  g.coherence = links ? (double)same / (double)links : 0.0;
  if (xs.empty()) return g;
  // the box of the central 99.8 % of the points (the rest clamp to the edge tiles)
  const size_t m = xs.size(), lo = m / 1000, hi = m - 1 - m / 1000;
  auto quantiles = [&](std::vector<float> v, double *a, double *b) {
    std::nth_element(v.begin(), v.begin() + lo, v.end());
    *a = v[lo];
    std::nth_element(v.begin(), v.begin() + hi, v.end());
    *b = v[hi];
  };
  double x0, x1, y0, y1, z0, z1;
  quantiles(xs, &x0, &x1);
  quantiles(ys, &y0, &y1);
  quantiles(zs, &z0, &z1);
  const double h = kTileHalo * voxel;
  const double W = std::max(x1 - x0, voxel), H = std::max(y1 - y0, voxel);
  // distinct voxels of B's own frame (a bitmap over the box, at most 2^27
  // bits; coarser voxels for a larger box), counted per cell
  double bv = voxel;
  int64_t bx = 0, by = 0, bz = 0;
  for (;;) {
    bx = (int64_t)std::ceil(W / bv) + 1;
    by = (int64_t)std::ceil(H / bv) + 1;
    bz = (int64_t)std::ceil(std::max(z1 - z0, voxel) / bv) + 1;
    if (bx * by * bz <= ((int64_t)1 << 27)) break;
    bv *= 2.0;
  }
  std::vector<uint64_t> bits((size_t)((bx * by * bz + 63) / 64), 0ull);
  const double cs = std::max(bv, std::sqrt(W * H / 65536.0));
  const int mx = (int)std::min<int64_t>(256, std::max<int64_t>(1, (int64_t)std::ceil(W / cs)));
  const int my = (int)std::min<int64_t>(256, std::max<int64_t>(1, (int64_t)std::ceil(H / cs)));
  std::vector<int32_t> cell((size_t)mx * my, 0);
  int64_t distinct = 0;
  auto clampi = [](double v, int64_t hi_) -> int64_t {
    return std::min<int64_t>(std::max<int64_t>((int64_t)std::floor(v), 0), hi_ - 1);
  };
  for (size_t i = 0; i < m; ++i) {
    const int64_t ix = clampi((xs[i] - x0) / bv, bx), iy = clampi((ys[i] - y0) / bv, by),
                  iz = clampi((zs[i] - z0) / bv, bz);
    const int64_t b = (iz * by + iy) * bx + ix;
    uint64_t &wd = bits[(size_t)(b >> 6)];
    const uint64_t bit = 1ull << (b & 63);
    if (wd & bit) continue;
    wd |= bit;
    ++distinct;
    ++cell[(size_t)(clampi((ys[i] - y0) / cs, my) * mx + clampi((xs[i] - x0) / cs, mx))];
  }
  const double target = std::max(64.0, cap / 2.0);
  const int64_t tmax = tiles_max(n);
  const int nxmax = std::max(1, (int)std::min(W / (3.0 * h), 65536.0));
  const int nymax = std::max(1, (int)std::min(H / (3.0 * h), 65536.0));
  std::vector<int64_t> cnt;
  double nt = std::ceil((double)distinct / target);
  for (int it = 0;; ++it) {
    int nx = std::max(1, (int)std::min(std::llround(std::sqrt(nt * W / H)), (long long)nxmax));
    int ny = std::max(1, std::min((int)std::ceil(nt / nx), nymax));
    while ((int64_t)nx * ny > tmax) {
      if (nx >= ny && nx > 1) --nx;
      else --ny;
    }
    g.nx = nx; g.ny = ny; g.x0 = x0; g.y0 = y0;
    g.ilx = (double)nx / W;
    g.ily = (double)ny / H;
    g.hx = nx > 1 ? h * g.ilx : 0.0;
    g.hy = ny > 1 ? h * g.ily : 0.0;
    // distinct voxels per tile with its halo, each cell's at the cell's centre
    cnt.assign((size_t)nx * ny, 0);
    int64_t worst = 0;
    for (int cy = 0; cy < my; ++cy)
      for (int cx = 0; cx < mx; ++cx) {
        const int32_t c = cell[(size_t)(cy * mx + cx)];
        if (!c) continue;
        const double fx = (cx + 0.5) * cs * g.ilx, fy = (cy + 0.5) * cs * g.ily;
        const int i = std::min(std::max((int)std::floor(fx), 0), nx - 1);
        const int j = std::min(std::max((int)std::floor(fy), 0), ny - 1);
        const double rx = fx - i, ry = fy - j;
        const int di = (i > 0 && rx < g.hx) ? -1 : (i + 1 < nx && rx > 1.0 - g.hx) ? 1 : 0;
        const int dj = (j > 0 && ry < g.hy) ? -1 : (j + 1 < ny && ry > 1.0 - g.hy) ? 1 : 0;
        worst = std::max(worst, cnt[(size_t)(j * nx + i)] += c);
        if (di) worst = std::max(worst, cnt[(size_t)(j * nx + i + di)] += c);
        if (dj) worst = std::max(worst, cnt[(size_t)((j + dj) * nx + i)] += c);
        if (di && dj) worst = std::max(worst, cnt[(size_t)((j + dj) * nx + i + di)] += c);
      }
    if (worst <= target || it >= 12 || (int64_t)nx * ny >= tmax || (nx >= nxmax && ny >= nymax))
      break;
    nt *= 1.3;
  }
  return g;
}

}  // namespace

// One scan pair of a plan as the host keeps it.
struct PairHost {
  const mi_ref *ref;
  const float *xyz;          // scan B (fixed at creation for batches, bound per execution else)
  int64_t n_b, K;
  double *mi_out;
  int64_t *argmax_out;
};

struct mi_plan {
  bool bind_per_execution;           // single-pair plan: buffers given to mi_plan_execute
  std::vector<PairHost> pairs;
  int64_t n_items;
  int32_t F;
  std::vector<int32_t> chunk_frame;  // [n_chunks + 1] over the frame table
  std::vector<int64_t> chunk_item;   // [n_chunks + 1] over the frame-sorted items
  std::vector<int64_t> chunk_cur_words;
  std::vector<int64_t> chunk_max_n;  // most points of a frame in the chunk
  std::vector<int64_t> chunk_point_poses;
  std::vector<uint32_t *> chunk_cur; // contiguous column cursors of each chunk's frames
  std::vector<std::array<int64_t, kXcds + 1>> chunk_xcd;  // runs per XCD within each chunk
  std::array<int64_t, kXcds + 1> direct_xcd;              // and within the per-pose items
  int64_t n_frame_items;             // items [n_frame_items, n_items) are per-pose:
  int64_t n_stripe_items;            // first those bucketed by stripe, then the tiled ones
  int64_t direct_point_poses, tile_point_poses;
  std::array<int64_t, kXcds + 1> tile_xcd;  // runs per XCD within the tiled items
  int32_t n_tiled;                   // tiled pairs
  int32_t *tiled_dev;                // their pair indices
  uint32_t *tile_cnt;                // every tiled pair's tile counts
  int64_t tile_cnt_words, tile_max_n;
  uint2 *scratch;                    // per-pose buckets: slots x stride
  int64_t scratch_stride, scratch_slots;
  PoseDev *items_dev;
  PairDev *pairs_dev;
  FrameDev *frames_dev;
  unsigned long long *nonfinite;     // [pairs][2]
  EvalLaunch launch;
  EvalLaunch tile_launch;            // the tiled per-pose form's
  int64_t tile_slots;
  mi_tuning tuning;                  // the tuning the plan was created under
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Items [i0, i1) regrouped by XCD.  The frame-sorted items are cut into
// pieces, a piece being a frame's items or, for a frame with many poses, at
// most a 32nd of the range of them; pieces go round-robin to the XCDs.  So
// every XCD gets an even share of every pair's frames, a frame's poses stay on
// one XCD (whose L2 then holds it) unless it has many, and a pose set with few
// distinct rotations (a translation grid) still spreads over all XCDs.  Within
// an XCD the items keep their order.  out[x] .. out[x + 1] (relative to i0) is
// XCD x's run.
void group_by_xcd(std::vector<PoseDev> &items, int64_t i0, int64_t i1,
                  std::array<int64_t, kXcds + 1> &out) {
  const int64_t cap = std::max<int64_t>(1, (i1 - i0 + 4 * kXcds - 1) / (4 * kXcds));
  std::vector<int8_t> xcd((size_t)std::max<int64_t>(i1 - i0, 0));
  std::array<int64_t, kXcds + 1> cnt;
  cnt.fill(0);
  int64_t piece = -1, in_piece = 0;
  for (int64_t k = i0; k < i1; ++k) {
    if (k == i0 || items[(size_t)k].frame != items[(size_t)k - 1].frame || in_piece == cap) {
      ++piece;
      in_piece = 0;
    }
    ++in_piece;
    const int x = (int)(piece % kXcds);
    xcd[(size_t)(k - i0)] = (int8_t)x;
    ++cnt[(size_t)x + 1];
  }
  out[0] = 0;
  for (int x = 0; x < kXcds; ++x) out[(size_t)x + 1] = out[(size_t)x] + cnt[(size_t)x + 1];
  std::array<int64_t, kXcds> pos;
  for (int x = 0; x < kXcds; ++x) pos[(size_t)x] = out[(size_t)x];
  std::vector<PoseDev> tmp(items.begin() + i0, items.begin() + i1);
  for (size_t j = 0; j < tmp.size(); ++j) items[(size_t)(i0 + pos[(size_t)xcd[j]]++)] = tmp[j];
}

// Device bytes of one frame inside a chunk's storage: rotated points, column
// offsets, and the frame's share of the chunk's contiguous cursor region.
struct FrameBytes {
  size_t v, off, cur;
};
FrameBytes frame_bytes(int64_t n_b, int64_t ncols) {
  // 4 doubles of padding: the evaluator reads 4 consecutive points from any start
  return {al256((size_t)std::max<int64_t>(n_b, 1) * 3 * sizeof(double) + 4 * sizeof(double)),
          al256((size_t)(ncols + 1) * 4), (size_t)ncols * 4};
}

// Everything a plan needs before any device memory is touched: per-pair pose
// tables and evaluator shapes, the launch, and the frame table order (pairs in
// the caller's order, each pair's frames in first-use order).
struct BatchTables {
  std::vector<PoseTables> T;
  std::vector<StripeShape> SS;
  std::vector<char> direct;          // per pair: 0 frames, 1 per-pose stripe buckets, 2 tiles
  std::vector<int64_t> n_b;          // per pair: points of scan B
  std::vector<char> maybe_tiled;     // per pair: frames until its scan's order is known
  std::vector<int32_t> frame_start;  // per pair: first entry in the frame table
  EvalLaunch L;
  EvalLaunch Lt;                     // launch of the tiled per-pose form
  int64_t tile_slots = 0;            // its workgroups
  int64_t n_items = 0;
  int64_t n_frame_items = 0;         // items of frame-mode pairs (they come first)
  int64_t n_stripe_items = 0;        // then items of stripe-bucketed pairs, then tiled ones
  int32_t n_tiled = 0;               // tiled pairs
  int32_t F = 0;                     // frame table entries
  int32_t F_built = 0;               // entries of frame-mode pairs (built; they come first)
  int64_t scratch_stride = 0;        // largest n_b of a per-pose pair
  int64_t scratch_slots = 0;         // workgroups of the per-pose launch
  mi_tuning tuning = {};             // in force, the auto hash resolved to its size
};

// The tiled form's launch under the auto tuning: one workgroup of kTileWaves
// waves per CU whose hash takes the LDS that the rest of the layout leaves.
void auto_tile_launch(EvalLaunch &Lt) {
  Lt.waves = kTileWaves;
  Lt.wgs_per_cu = 1;
  Lt.hist_copies = 1;
  Lt.plan_bytes = 8;
  const int slot = eval_hash_slot_bytes(Lt.zvar);
  Lt.cap = 64;
  const int64_t rest = (int64_t)eval_lds_bytes(Lt) - 64 * slot;
  Lt.cap = (int32_t)std::max<int64_t>(
      64, std::min<int64_t>(65536, ((int64_t)max_lds_per_block() - rest - 256) / slot) &
              ~(int64_t)63);
  while (Lt.cap > 64 && (int64_t)eval_lds_bytes(Lt) > max_lds_per_block()) Lt.cap -= 64;
}

// Hash slots of the tiled launch for one grid alone (the tile size of a scan
// evaluated on it), under the tuning in force.
int32_t tile_cap_for(const GridInfo &gi) {
  const Tuning tu = tuning_now();
  EvalLaunch L;
  L.waves = tu.waves;
  L.hist_copies = tu.hist_copies;
  L.hist_words = gi.nb[0] * gi.nb[0] + (gi.nf > 1 ? gi.nb[1] * gi.nb[1] : 0);
  L.plan_bytes = 8;
  L.wgs_per_cu = tu.wgs_per_cu;
  L.zvar = (gi.features & (MI_FEAT_ZVAR | MI_FEAT_JOINT)) != 0;
  L.near_face = false;
  if (tu.hash_bytes == 0) {
    auto_tile_launch(L);
    return L.cap;
  }
  return (int32_t)std::max<int64_t>(
      64, std::min<int64_t>(65536, ((int64_t)tu.hash_bytes / eval_hash_slot_bytes(L.zvar))) &
              ~(int64_t)63);
}

// Poses per rotation up to which a scan in random order is evaluated in tiles
// rather than in shared frames (with few poses per frame and no runs of
// neighbouring points, a frame saves little of a pose's work).
constexpr int64_t kTilePosesPerRotation = 128;
constexpr double kTileCoherenceMax = 0.25;

// tiles: pairs may be tiled (scan B is read when the plan is made): per-pose
// pairs, and pairs with shared rotations whose scan order is incoherent when
// geo (per item; known = false where not measured) says so.  Without geo such
// pairs stay in frames but get tile storage too (for workspace sizes).
mi_status prepare_batch(const mi_work_item *w, int64_t n, uint32_t flags, BatchTables &B,
                        bool tiles = false, const TileGeom *geo = nullptr) {
  if (n < 0 || (n > 0 && !w)) return fail(MI_E_INVALID, "bad work item list");
  if (n >= ((int64_t)1 << 20)) return fail(MI_E_UNSUPPORTED, "more than 2^20 work items");
  if (flags & ~(uint32_t)(MI_EVAL_NEAR_FACE | MI_EVAL_PER_POSE | MI_EVAL_SHARED_FRAMES))
    return fail(MI_E_INVALID, "unknown flags");
  if ((flags & MI_EVAL_PER_POSE) && (flags & MI_EVAL_SHARED_FRAMES))
    return fail(MI_E_INVALID, "MI_EVAL_PER_POSE and MI_EVAL_SHARED_FRAMES exclude each other");
  bool zvar = false;
  int hist_words = 1;
  for (int64_t i = 0; i < n; ++i) {
    const mi_work_item &it = w[i];
    if (!it.ref) return fail(MI_E_INVALID, "work item %lld: NULL ref", (long long)i);
    if (it.K < 0 || it.n_b < 0 || (it.K > 0 && !it.poses))
      return fail(MI_E_INVALID, "work item %lld: bad pose set or scan B", (long long)i);
    const GridInfo &gi = it.ref->g->gi;
    zvar = zvar || (gi.features & (MI_FEAT_ZVAR | MI_FEAT_JOINT)) != 0;
    hist_words = std::max(hist_words, gi.nb[0] * gi.nb[0] + (gi.nf > 1 ? gi.nb[1] * gi.nb[1] : 0));
  }
  B.T.assign((size_t)n, PoseTables());
  B.SS.assign((size_t)n, StripeShape());
  B.direct.assign((size_t)n, 0);
  B.n_b.assign((size_t)n, 0);
  B.maybe_tiled.assign((size_t)n, 0);
  B.frame_start.assign((size_t)n, 0);
  Tuning tu = tuning_now();
  const bool auto_tuned = tu.hash_bytes == 0;
  if (tu.hash_bytes == 0) {
    tu.hash_bytes = kAutoHashBytes;
    // the default hash only where the launch keeps two workgroups per CU
    // (plan entries as for shared frames, the larger of the two forms)
    int plan_max = 8;
    int32_t cap = 64;
    for (int64_t i = 0; i < n; ++i) {
      StripeShape S;
      const char *why = "";
      if (!choose_stripes(w[i].ref->g->gi, tu, zvar, S, &why)) continue;
      plan_max = std::max(plan_max, S.plan_stripes * S.plan_entries * 8);
      cap = S.cap;
    }
    EvalLaunch L0;
    L0.waves = tu.waves;
    L0.cap = cap;
    L0.hist_copies = tu.hist_copies;
    L0.hist_words = hist_words;
    L0.plan_bytes = plan_max;
    L0.wgs_per_cu = tu.wgs_per_cu;
    L0.zvar = zvar;
    L0.near_face = false;
    if ((int64_t)eval_lds_bytes(L0) > kTwoWorkgroupLds) tu.hash_bytes = kFitHashBytes;
  }
  B.tuning = mi_tuning{tu.waves, tu.hash_bytes, tu.hist_copies, tu.stripe_rows, tu.wgs_per_cu};
  int plan_bytes_max = 8;
  for (int64_t i = 0; i < n; ++i) {
    const mi_work_item &it = w[i];
    const GridInfo &gi = it.ref->g->gi;
    // the packed (n << 44 | S1) sums hold counts below 2^20
    if (zvar && it.n_b >= MI_MAX_POINTS)
      return fail(MI_E_UNSUPPORTED,
                  "work item %lld: scan B has %lld >= 2^20 points with the z-variance feature",
                  (long long)i, (long long)it.n_b);
    if (it.n_b >= ((int64_t)1 << 32))
      return fail(MI_E_UNSUPPORTED, "work item %lld: scan B has >= 2^32 points", (long long)i);
    if (it.K >= ((int64_t)1 << 31))
      return fail(MI_E_UNSUPPORTED, "work item %lld: more than 2^31 poses", (long long)i);
    const int bt = build_tables(gi, it.poses, it.K, B.T[(size_t)i]);
    if (bt == -1) return fail(MI_E_INVALID, "work item %lld: non-finite pose", (long long)i);
    if (bt) return fail(MI_E_UNSUPPORTED, "work item %lld: pose translations span too large a range",
                        (long long)i);
    const char *why = "";
    if (!choose_stripes(gi, tu, zvar, B.SS[(size_t)i], &why))
      return fail(MI_E_UNSUPPORTED, "work item %lld: evaluator: %s", (long long)i, why);
    const PoseTables &T = B.T[(size_t)i];
    // a rotation shared by fewer than two poses on average is not worth a frame;
    // the per-pose form addresses scan B with 32-bit offsets (below 2^28 points)
    const bool small = it.n_b < ((int64_t)1 << 28);
    if ((flags & MI_EVAL_PER_POSE) && !small)
      return fail(MI_E_UNSUPPORTED, "work item %lld: the per-pose form takes below 2^28 points",
                  (long long)i);
    const bool direct = (flags & MI_EVAL_PER_POSE) ||
                        (!(flags & MI_EVAL_SHARED_FRAMES) && small && it.K > 0 &&
                         2 * (int64_t)T.F > it.K);
    B.n_b[(size_t)i] = it.n_b;
    // tiled: the tile entries (at most 4 per point) are addressed with 32-bit
    // offsets, and the whole-grid voxel key fits 31 bits
    const bool tileable = tiles && it.n_b > 0 && it.n_b < ((int64_t)1 << 26) &&
                          bits_for(gi.dims[0]) + bits_for(gi.dims[1]) + bits_for(gi.dims[2]) <= 31;
    // shared rotations with few poses each, on a scan in random order
    const bool few = tileable && !direct && !(flags & MI_EVAL_SHARED_FRAMES) && it.K > 0 &&
                     it.K <= kTilePosesPerRotation * (int64_t)T.F;
    const bool tiled = tileable && (direct || (few && geo && geo[i].known &&
                                               geo[i].coherence < kTileCoherenceMax));
    B.maybe_tiled[(size_t)i] = few && !tiled && !(geo && geo[i].known);
    B.direct[(size_t)i] = tiled ? 2 : direct ? 1 : 0;
    if (direct && !tiled) {
      // A per-pose brick rescans its stripe's whole bucket, so overflow retries
      // are costly: stripes are sized for about a third of the slots, taking
      // about 0.6 occupied voxels per point spread evenly over the rows.
      const StripeShape &S0 = B.SS[(size_t)i];
      const double per_row = 0.6 * (double)std::max<int64_t>(it.n_b, 1) / (double)gi.dims[1];
      Tuning t2 = tu;
      t2.stripe_rows = (int)std::max(1.0, std::min((double)tu.stripe_rows, S0.cap / 3.0 / per_row));
      if (!choose_stripes(gi, t2, zvar, B.SS[(size_t)i], &why))
        return fail(MI_E_UNSUPPORTED, "work item %lld: evaluator: %s", (long long)i, why);
    }
    const StripeShape &S = B.SS[(size_t)i];
    if (tiled) {
      ++B.n_tiled;
    } else if (direct) {
      plan_bytes_max = std::max(plan_bytes_max, (2 * S.n_stripes + 1) * 4);
      B.scratch_stride = std::max(B.scratch_stride, std::max<int64_t>(it.n_b, 1));
      B.n_stripe_items += it.K;
    } else {
      plan_bytes_max = std::max(plan_bytes_max, S.plan_stripes * S.plan_entries * 8);
      B.n_frame_items += it.K;
    }
    B.n_items += it.K;
  }
  if (B.n_items >= ((int64_t)1 << 31)) return fail(MI_E_UNSUPPORTED, "more than 2^31 poses in all");
  // frame table: frame-mode pairs first (their frames are built), then the
  // rotations of per-pose pairs (only their matrices are read)
  int32_t f = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t i = 0; i < n; ++i)
      if ((bool)B.direct[(size_t)i] == (pass == 1)) {
        B.frame_start[(size_t)i] = f;
        f += B.T[(size_t)i].F;
        if (pass == 0) B.F_built = f;
      }
  B.F = f;
  EvalLaunch &L = B.L;
  L.waves = tu.waves;
  L.cap = n > 0 ? B.SS[0].cap : 64;
  L.hist_copies = tu.hist_copies;
  L.hist_words = hist_words;
  L.plan_bytes = plan_bytes_max;
  L.wgs_per_cu = tu.wgs_per_cu;
  L.zvar = zvar;
  L.near_face = (flags & MI_EVAL_NEAR_FACE) != 0;
  if ((int64_t)eval_lds_bytes(L) > max_lds_per_block())
    return fail(MI_E_UNSUPPORTED, "tuning needs %zu LDS bytes per workgroup, device has %d",
                eval_lds_bytes(L), max_lds_per_block());
  if (B.n_stripe_items > 0) {
    hipError_t e = eval_resident_wgs(L, L.wgs_per_cu > 0 ? L.wgs_per_cu : 2, &B.scratch_slots);
    if (e != hipSuccess) return dev_fail(e, "occupancy of the per-pose evaluator");
    // no more slots than the launch can use (a multiple of the XCD count)
    const int64_t nd = B.n_stripe_items;
    B.scratch_slots = std::min<int64_t>(B.scratch_slots, ((nd + kXcds - 1) / kXcds) * kXcds);
  }
  // The tiled form: under the auto tuning, one workgroup of kTileWaves waves
  // per CU with the largest hash the LDS holds (a tile's set-up and its two
  // barriers are then spread over more points); a set tuning is used as given.
  EvalLaunch &Lt = B.Lt;
  Lt = L;
  Lt.plan_bytes = 8;
  if (auto_tuned) auto_tile_launch(Lt);
  const int64_t n_tile_items = B.n_items - B.n_frame_items - B.n_stripe_items;
  if (n_tile_items > 0) {
    if ((int64_t)eval_lds_bytes(Lt) > max_lds_per_block())
      return fail(MI_E_UNSUPPORTED, "tiled launch needs %zu LDS bytes per workgroup, device has %d",
                  eval_lds_bytes(Lt), max_lds_per_block());
    hipError_t e = eval_resident_wgs(Lt, Lt.wgs_per_cu > 0 ? Lt.wgs_per_cu : 2, &B.tile_slots, 2);
    if (e != hipSuccess) return dev_fail(e, "occupancy of the tiled evaluator");
    B.tile_slots =
        std::min<int64_t>(B.tile_slots, ((n_tile_items + kXcds - 1) / kXcds) * kXcds);
  }
  return MI_OK;
}

// Frames go into chunks greedily in table order, as many as fit the storage
// budget (a frame larger than the budget gets a chunk of its own).
struct ChunkPlan {
  std::vector<int32_t> first;        // [chunks + 1]
  size_t max_store = 0;
};

void plan_chunks(const BatchTables &B, const mi_work_item *w, size_t budget, ChunkPlan &C) {
  C.first.assign(1, 0);
  C.max_store = 0;
  size_t v = 0, off = 0, cur = 0;
  int32_t in_chunk = 0;
  for (size_t p = 0; p < B.T.size(); ++p) {
    if (B.direct[p]) continue;
    const int64_t ncols = (int64_t)B.T[p].ncx * B.T[p].ncy;
    const FrameBytes fb = frame_bytes(w[p].n_b, ncols);
    for (int32_t f = 0; f < B.T[p].F; ++f) {
      const size_t nv = v + fb.v, noff = off + fb.off, ncur = cur + fb.cur;
      if (in_chunk > 0 && nv + noff + al256(ncur) > budget) {
        C.max_store = std::max(C.max_store, v + off + al256(cur));
        C.first.push_back(B.frame_start[p] + f);
        v = fb.v; off = fb.off; cur = fb.cur;
        in_chunk = 1;
      } else {
        v = nv; off = noff; cur = ncur;
        ++in_chunk;
      }
    }
  }
  C.max_store = std::max(C.max_store, v + off + al256(cur));
  C.first.push_back(B.F_built);
}

struct PlanLayout {
  PoseDev *items;
  PairDev *pairs;
  FrameDev *frames;
  unsigned long long *nonfinite;
  uint2 *scratch;
  int32_t *tiled;                  // [n_tiled] pair indices
  uint32_t *tile_cnt;              // [tile_cnt_words]
  int64_t tile_cnt_words;
  std::vector<float *> tile_xyz;   // per pair (tiled pairs only)
  std::vector<uint32_t *> tile_off, tile_own, tile_cnt_of;
  char *store;
};

void plan_fixed(const BatchTables &B, int64_t n_pairs, Carver &c, PlanLayout *L) {
  PoseDev *items = c.take<PoseDev>((size_t)std::max<int64_t>(B.n_items, 1));
  PairDev *pairs = c.take<PairDev>((size_t)std::max<int64_t>(n_pairs, 1));
  FrameDev *frames = c.take<FrameDev>((size_t)std::max(B.F, 1));
  unsigned long long *nf = c.take<unsigned long long>((size_t)std::max<int64_t>(2 * n_pairs, 2));
  uint2 *scratch = c.take<uint2>((size_t)(B.scratch_slots * B.scratch_stride));
  // tiled pairs: up to 4 entries per point (its tile and up to 3 halos), and
  // the tile tables at their largest
  int32_t *tiled = c.take<int32_t>((size_t)std::max(B.n_tiled, 1));
  int64_t words = 0;
  auto has_tiles = [&](size_t i) { return B.direct[i] == 2 || (!B.maybe_tiled.empty() && B.maybe_tiled[i]); };
  for (size_t i = 0; i < B.direct.size(); ++i)
    if (has_tiles(i)) words += 2 * tiles_max(B.n_b[i]);
  uint32_t *tcnt = c.take<uint32_t>((size_t)std::max<int64_t>(words, 1));
  if (L) {
    L->tile_xyz.assign(B.direct.size(), nullptr);
    L->tile_off.assign(B.direct.size(), nullptr);
    L->tile_own.assign(B.direct.size(), nullptr);
    L->tile_cnt_of.assign(B.direct.size(), nullptr);
  }
  int64_t w0 = 0;
  for (size_t i = 0; i < B.direct.size(); ++i) {
    if (!has_tiles(i)) continue;
    const int64_t tm = tiles_max(B.n_b[i]);
    float *xyz = c.take<float>((size_t)(12 * B.n_b[i]));
    uint32_t *off = c.take<uint32_t>((size_t)(tm + 1));
    uint32_t *own = c.take<uint32_t>((size_t)tm);
    if (L) {
      L->tile_xyz[i] = xyz;
      L->tile_off[i] = off;
      L->tile_own[i] = own;
      L->tile_cnt_of[i] = tcnt + w0;
    }
    w0 += 2 * tm;
  }
  char *store = c.take<char>(0);
  if (L) {
    L->items = items; L->pairs = pairs; L->frames = frames; L->nonfinite = nf;
    L->scratch = scratch; L->store = store;
    L->tiled = tiled; L->tile_cnt = tcnt; L->tile_cnt_words = words;
  }
}

constexpr size_t kDefaultFrameBudget = (size_t)4 << 30;

size_t batch_bytes(const BatchTables &B, const mi_work_item *w, int64_t n, size_t budget) {
  Carver c(nullptr, 0);
  plan_fixed(B, n, c, nullptr);
  ChunkPlan C;
  plan_chunks(B, w, budget ? budget : kDefaultFrameBudget, C);
  return c.used() + C.max_store + 512;
}

// Workspace of a single-pair plan of K poses over F rotations whose column
// grids have at most ncols columns (for callers that size before the poses
// are known, such as the coarse-to-fine search).
size_t single_plan_bytes(int64_t K, int32_t F, int64_t ncols, int64_t n_b) {
  BatchTables B;
  B.T.assign(1, PoseTables());
  B.T[0].F = F;
  B.T[0].ncx = (int32_t)std::min<int64_t>(ncols, 0x7fffffff);
  B.T[0].ncy = 1;
  B.direct.assign(1, 0);
  B.frame_start.assign(1, 0);
  B.F = F;
  B.F_built = F;
  B.n_items = K;
  B.n_frame_items = K;
  mi_work_item w;
  memset(&w, 0, sizeof w);
  w.n_b = n_b;
  return batch_bytes(B, &w, 1, 0);
}

// no_alloc: the workspace is fixed (the static scratch), so the per-pose
// buckets get as many workgroup slots as it holds, and the tables are copied
// from host memory directly instead of through pinned staging (which may
// allocate).
//
// tiles: per-pose pairs use the tiled form (batch plans, whose scans are fixed
// here: each tiled scan is copied to the host once to choose its tiles, so
// this call waits for the stream).
// geo: the tile geometry of each item's scan when the caller has it (else it
// is computed here for the pairs that may be tiled).
mi_status create_plan(const mi_work_item *w, int64_t n, uint32_t flags, void *ws, size_t ws_bytes,
                      size_t budget, void *stream, bool bind_per_execution, mi_plan **out,
                      bool no_alloc = false, bool tiles = false, const TileGeom *geo = nullptr) {
  if (!out) return fail(MI_E_INVALID, "NULL output handle");
  *out = nullptr;
  BatchTables B;
  tiles = tiles && !bind_per_execution && !no_alloc;
  // argument errors before workspace errors
  mi_status st = prepare_batch(w, n, flags, B, tiles, geo);
  if (st != MI_OK) return st;
  // tile geometry: each scan that may be tiled is read back once
  std::vector<TileGeom> geom((size_t)n);
  if (geo) {
    std::copy(geo, geo + n, geom.begin());
  } else if (tiles) {
    std::vector<int32_t> need;
    bool maybe = false;
    for (int64_t i = 0; i < n; ++i)
      if (B.direct[(size_t)i] == 2 || B.maybe_tiled[(size_t)i]) {
        need.push_back((int32_t)i);
        maybe = maybe || B.maybe_tiled[(size_t)i];
      }
    if (!need.empty()) {
      std::vector<std::vector<float>> hb(need.size());
      for (size_t k = 0; k < need.size(); ++k) {
        const int64_t nb = w[need[k]].n_b;
        hb[k].resize((size_t)(3 * nb));
        HIP_TRY(hipMemcpyAsync(hb[k].data(), w[need[k]].xyz_b, sizeof(float) * 3 * (size_t)nb,
                               hipMemcpyDeviceToHost, (hipStream_t)stream),
                "scan B to host");
      }
      HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "scan B to host");
      std::atomic<size_t> next(0);
      auto work = [&]() {
        for (size_t k; (k = next.fetch_add(1)) < need.size();) {
          const int32_t i = need[k];
          geom[(size_t)i] = choose_tiles(hb[k].data(), w[i].n_b, w[i].ref->g->gi.voxel, B.Lt.cap);
        }
      };
      const size_t nthr = std::min<size_t>(need.size(), 8);
      std::vector<std::thread> pool;
      for (size_t t = 1; t < nthr; ++t) pool.emplace_back(work);
      work();
      for (std::thread &t : pool) t.join();
      if (maybe) {  // the forms of pairs with shared rotations follow their scans' order
        B = BatchTables();
        st = prepare_batch(w, n, flags, B, tiles, geom.data());
        if (st != MI_OK) return st;
      }
    }
  }
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  if (no_alloc && B.scratch_slots > 0) {
    // the buckets take what the tables leave (half of it when frames need room too)
    const int64_t want = B.scratch_slots;
    B.scratch_slots = 0;
    Carver c0(nullptr, 0);
    plan_fixed(B, n, c0, nullptr);
    const size_t fixed = c0.used() + 4096;
    size_t room = ws_bytes > fixed ? ws_bytes - fixed : 0;
    if (B.F_built > 0) room /= 2;
    const size_t per_slot = (size_t)B.scratch_stride * sizeof(uint2);
    const int64_t fit = (int64_t)(room / per_slot) / kXcds * kXcds;
    if (fit < kXcds)
      return fail(MI_E_UNSUPPORTED,
                  "per-pose buckets of %lld points for %d workgroups need %zu bytes; %zu are left",
                  (long long)B.scratch_stride, kXcds, per_slot * kXcds, room);
    B.scratch_slots = std::min(want, fit);
  }
  Carver c(ws, ws_bytes);
  PlanLayout PL;
  plan_fixed(B, n, c, &PL);
  if (!c.fits()) return fail(MI_E_WORKSPACE, "eval workspace too small for the pose tables");
  // frame storage: the budget when given, else all that the workspace holds
  const size_t room = ws_bytes - std::min(ws_bytes, c.used() + 256);
  const size_t store_budget = budget ? std::min(budget, room) : room;
  ChunkPlan C;
  plan_chunks(B, w, store_budget, C);
  if (B.F_built > 0 && C.max_store > room)
    return fail(MI_E_WORKSPACE, "eval workspace needs %zu bytes, got %zu",
                c.used() + C.max_store + 256, ws_bytes);

  std::unique_ptr<mi_plan> p(new (std::nothrow) mi_plan());
  if (!p) return fail(MI_E_INVALID, "out of host memory");
  p->bind_per_execution = bind_per_execution;
  p->n_items = B.n_items;
  p->F = B.F;
  p->launch = B.L;
  p->tile_launch = B.Lt;
  p->tile_slots = B.tile_slots;
  p->tuning = B.tuning;
  p->items_dev = PL.items;
  p->pairs_dev = PL.pairs;
  p->frames_dev = PL.frames;
  p->nonfinite = PL.nonfinite;
  p->n_frame_items = B.n_frame_items;
  p->n_stripe_items = B.n_stripe_items;
  p->tile_point_poses = 0;
  p->n_tiled = B.n_tiled;
  p->tiled_dev = PL.tiled;
  p->tile_cnt = PL.tile_cnt;
  p->tile_cnt_words = PL.tile_cnt_words;
  p->tile_max_n = 0;
  p->scratch = PL.scratch;
  p->scratch_stride = B.scratch_stride;
  p->scratch_slots = B.scratch_slots;
  p->direct_point_poses = 0;
  p->pairs.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    p->pairs[(size_t)i] = {w[i].ref, w[i].xyz_b, w[i].n_b, w[i].K, w[i].mi_out, w[i].argmax_out};

  // pose items: frame-mode pairs in order, each pair's items sorted by frame
  // (so the items of a frame chunk are contiguous), then per-pose pairs
  std::vector<PoseDev> items;
  if (n == 1 && !B.direct[0]) {
    items.swap(B.T[0].items);  // one pair of frames: pair 0, frames from 0, already in order
  } else {
    items.resize((size_t)B.n_items);
    size_t k = 0;
    for (int pass = 0; pass < 3; ++pass)
      for (int64_t i = 0; i < n; ++i) {
        if (B.direct[(size_t)i] != pass) continue;
        for (const PoseDev &it : B.T[(size_t)i].items) {
          PoseDev d = it;
          d.pair = (int32_t)i;
          d.frame = it.frame + B.frame_start[(size_t)i];
          items[k++] = d;
          if (pass == 1) p->direct_point_poses += w[i].n_b;
          if (pass == 2) p->tile_point_poses += w[i].n_b;
        }
      }
  }
  // frame table with each frame's place in its chunk's storage
  std::vector<FrameDev> frames((size_t)B.F);
  const size_t n_chunks = C.first.size() - 1;
  p->chunk_frame = C.first;
  p->chunk_item.assign(n_chunks + 1, B.n_items);
  p->chunk_cur_words.assign(n_chunks, 0);
  p->chunk_max_n.assign(n_chunks, 0);
  p->chunk_cur.assign(n_chunks, nullptr);
  {
    std::vector<int32_t> pair_of((size_t)B.F);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t f = 0; f < B.T[(size_t)i].F; ++f)
        pair_of[(size_t)(B.frame_start[(size_t)i] + f)] = (int32_t)i;
    // rotations of per-pose pairs: matrices only, nothing is built
    for (int32_t f = B.F_built; f < B.F; ++f) {
      const size_t pi = (size_t)pair_of[(size_t)f];
      FrameDev &Fd = frames[(size_t)f];
      memset(&Fd, 0, sizeof Fd);
      memcpy(Fd.R, &B.T[pi].R[(size_t)(f - B.frame_start[pi]) * 9], sizeof Fd.R);
      Fd.s = w[pi].ref->g->gi.s;
      Fd.xyz = w[pi].xyz_b;
      Fd.n = w[pi].n_b;
    }
    for (size_t ch = 0; ch < n_chunks; ++ch) {
      const int32_t f0 = C.first[ch], f1 = C.first[ch + 1];
      size_t v = 0, off = 0, cur = 0;
      for (int32_t f = f0; f < f1; ++f) {
        const size_t pi = (size_t)pair_of[(size_t)f];
        const FrameBytes fb = frame_bytes(w[pi].n_b, (int64_t)B.T[pi].ncx * B.T[pi].ncy);
        v += fb.v; off += fb.off; cur += fb.cur;
      }
      char *vbase = PL.store, *obase = PL.store + v;
      uint32_t *cbase = (uint32_t *)(PL.store + v + off);
      p->chunk_cur[ch] = cbase;
      p->chunk_cur_words[ch] = (int64_t)(cur / 4);
      for (int32_t f = f0; f < f1; ++f) {
        const size_t pi = (size_t)pair_of[(size_t)f];
        const PoseTables &T = B.T[pi];
        const GridInfo &gi = w[pi].ref->g->gi;
        const int64_t ncols = (int64_t)T.ncx * T.ncy;
        const FrameBytes fb = frame_bytes(w[pi].n_b, ncols);
        FrameDev &Fd = frames[(size_t)f];
        memset(&Fd, 0, sizeof Fd);
        memcpy(Fd.R, &T.R[(size_t)(f - B.frame_start[pi]) * 9], sizeof Fd.R);
        Fd.s = gi.s;
        Fd.xyz = w[pi].xyz_b;
        Fd.n = w[pi].n_b;
        Fd.gx = T.gx; Fd.gy = T.gy; Fd.ncx = T.ncx; Fd.ncy = T.ncy;
        Fd.zlo = T.zlo; Fd.zhi = T.zhi;
        Fd.v = (double *)vbase;
        Fd.off = (uint32_t *)obase;
        Fd.cur = cbase;
        vbase += fb.v; obase += fb.off; cbase += ncols;
        p->chunk_max_n[ch] = std::max(p->chunk_max_n[ch], w[pi].n_b);
      }
    }
    int64_t k = 0;
    p->chunk_point_poses.assign(n_chunks, 0);
    for (size_t ch = 0; ch < n_chunks; ++ch) {
      p->chunk_item[ch] = k;
      while (k < B.n_frame_items && items[(size_t)k].frame < C.first[ch + 1]) {
        p->chunk_point_poses[ch] += w[items[(size_t)k].pair].n_b;
        ++k;
      }
    }
    p->chunk_item[n_chunks] = B.n_frame_items;
  }
  p->chunk_xcd.resize(n_chunks);
  for (size_t ch = 0; ch < n_chunks; ++ch)
    group_by_xcd(items, p->chunk_item[ch], p->chunk_item[ch + 1], p->chunk_xcd[ch]);
  group_by_xcd(items, B.n_frame_items, B.n_frame_items + B.n_stripe_items, p->direct_xcd);
  group_by_xcd(items, B.n_frame_items + B.n_stripe_items, B.n_items, p->tile_xcd);
  std::vector<int32_t> tiled;
  for (int64_t i = 0; i < n; ++i)
    if (B.direct[(size_t)i] == 2) {
      tiled.push_back((int32_t)i);
      p->tile_max_n = std::max(p->tile_max_n, w[i].n_b);
    }
  std::vector<PairDev> pairs((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const GridInfo &gi = w[i].ref->g->gi;
    const RefDev &rd = w[i].ref->rd;
    const StripeShape &S = B.SS[(size_t)i];
    PairDev &P = pairs[(size_t)i];
    memset(&P, 0, sizeof P);
    P.nx = gi.dims[0]; P.ny = gi.dims[1]; P.nz = gi.dims[2]; P.nf = gi.nf;
    for (int f = 0; f < 2; ++f) {
      P.kind[f] = gi.kind[f];
      P.nb[f] = gi.nb[f];
      P.binA[f] = rd.bins[f];
      P.sat[f] = rd.sat[f];
      P.sat_layout[f] = rd.sat_layout[f];
    }
    P.alist = rd.alist;
    P.alist_n = rd.alist_n;
    P.nbc = gi.nbc;
    P.nbz = gi.nbz;
    P.voxel = gi.voxel;
    P.abox = rd.abox;
    P.stripe_h = S.stripe_h;
    P.n_stripes = S.n_stripes;
    P.pieces = S.pieces;
    P.kx_bits = S.kx_bits;
    P.ky_bits = S.ky_bits;
    P.plan_stripes = S.plan_stripes;
    P.count_default = 1;
    for (int j = 0; j + 1 < gi.nbc; ++j)
      if (gi.count_edges[j] != (uint32_t)(j + 1)) P.count_default = 0;
    P.zvar_zero_edges = 0;
    for (int j = 0; j + 2 < gi.nbz; ++j)
      if (gi.zvar_edges[j] == 0) ++P.zvar_zero_edges;
    P.nonfinite = PL.nonfinite + 2 * i;
    P.n_b = w[i].n_b;
    P.xyz_b = w[i].xyz_b;
    if (B.direct[(size_t)i] == 2) {
      const TileGeom &g = geom[(size_t)i];
      P.tile_xyz = PL.tile_xyz[(size_t)i];
      P.tile_stride = 4 * w[i].n_b;
      P.tile_off = PL.tile_off[(size_t)i];
      P.tile_own = PL.tile_own[(size_t)i];
      P.tile_cnt = PL.tile_cnt_of[(size_t)i];
      P.tile_x0 = g.x0; P.tile_y0 = g.y0;
      P.tile_ilx = g.ilx; P.tile_ily = g.ily;
      P.tile_hx = g.hx; P.tile_hy = g.hy;
      P.tile_nx = g.nx; P.tile_ny = g.ny;
      P.key_xbits = bits_for(gi.dims[0]);
      P.key_ybits = bits_for(gi.dims[1]);
    }
    P.mi_out = w[i].mi_out;
    P.K = w[i].K;
    P.hist_out = w[i].hist_out;
    P.hist_off[0] = 0;
    P.hist_off[1] = w[i].K * (int64_t)gi.nb[0] * gi.nb[0];
    P.stats_out = w[i].stats_out;
    memcpy(P.count_edges, gi.count_edges, sizeof P.count_edges);
    memcpy(P.zvar_edges, gi.zvar_edges, sizeof P.zvar_edges);
  }
  const size_t b_items = sizeof(PoseDev) * items.size(), b_pairs = sizeof(PairDev) * pairs.size(),
               b_frames = sizeof(FrameDev) * frames.size(),
               b_tiled = sizeof(int32_t) * tiled.size();
  hipError_t e = hipSuccess;
  if (no_alloc) {
    // pageable host source: each copy has taken its data when it returns
    const hipStream_t hs = (hipStream_t)stream;
    if (b_items)
      HIP_TRY(hipMemcpyAsync(PL.items, items.data(), b_items, hipMemcpyHostToDevice, hs), "pose table");
    if (b_pairs)
      HIP_TRY(hipMemcpyAsync(PL.pairs, pairs.data(), b_pairs, hipMemcpyHostToDevice, hs), "pair table");
    if (b_frames)
      HIP_TRY(hipMemcpyAsync(PL.frames, frames.data(), b_frames, hipMemcpyHostToDevice, hs),
              "frame table");
    *out = p.release();
    return MI_OK;
  }
  Staging *sg = staging_acquire(b_items + b_pairs + b_frames + b_tiled + 64, &e);
  if (!sg) return dev_fail(e, "pinned staging");
  char *h = (char *)sg->p;
  if (b_items) memcpy(h, items.data(), b_items);
  if (b_pairs) memcpy(h + b_items, pairs.data(), b_pairs);
  if (b_frames) memcpy(h + b_items + b_pairs, frames.data(), b_frames);
  if (b_tiled) memcpy(h + b_items + b_pairs + b_frames, tiled.data(), b_tiled);
  const Upload ups[4] = {{PL.items, 0, b_items}, {PL.pairs, b_items, b_pairs},
                         {PL.frames, b_items + b_pairs, b_frames},
                         {PL.tiled, b_items + b_pairs + b_frames, b_tiled}};
  e = staging_upload(sg, ups, 4, (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "pose table upload");
  *out = p.release();
  return MI_OK;
}

// Enqueue one execution: non-finite counts, then per chunk the frames and one
// evaluator launch over the chunk's poses, then the argmax of each pair.
mi_status run_plan(mi_plan *p, hipStream_t s) {
  for (size_t i = 0; i < p->pairs.size(); ++i)
    HIP_TRY(launch_count_nonfinite(p->pairs[i].xyz, p->pairs[i].n_b, p->nonfinite + 2 * i, s),
            "count non-finite");
  if (p->n_tiled > 0) {
    hipEvent_t a = nullptr;
    const bool timed = prof_begin(s, &a);
    HIP_TRY(launch_tiles(p->pairs_dev, p->tiled_dev, p->n_tiled, p->tile_max_n, p->tile_cnt,
                         p->tile_cnt_words, s),
            "scan B tiles");
    if (timed) prof_end(s, a, kStageFrames, 0, 0);
  }
  const size_t n_chunks = p->chunk_frame.size() - 1;
  for (size_t ch = 0; ch < n_chunks; ++ch) {
    const int32_t f0 = p->chunk_frame[ch], nfr = p->chunk_frame[ch + 1] - f0;
    if (nfr > 0) {
      hipEvent_t a = nullptr;
      const bool timed = prof_begin(s, &a);
      HIP_TRY(launch_fill_u32(p->chunk_cur[ch], 0u, p->chunk_cur_words[ch], s),
              "clear column counts");
      HIP_TRY(launch_frames(p->frames_dev + f0, nfr, p->chunk_max_n[ch], 0, s), "frames");
      if (timed) prof_end(s, a, kStageFrames, 0, 0);
    }
    const int64_t i0 = p->chunk_item[ch], i1 = p->chunk_item[ch + 1];
    if (i1 > i0) {
      hipEvent_t a = nullptr;
      const bool timed = prof_begin(s, &a);
      HIP_TRY(launch_eval(p->pairs_dev, p->frames_dev, p->items_dev + i0, i1 - i0,
                          p->chunk_xcd[ch].data(), p->launch, s),
              "eval");
      if (timed) prof_end(s, a, kStageEval, i1 - i0, p->chunk_point_poses[ch]);
    }
  }
  const int64_t nd = p->n_stripe_items;
  if (nd > 0) {
    hipEvent_t a = nullptr;
    const bool timed = prof_begin(s, &a);
    HIP_TRY(launch_eval_direct(p->pairs_dev, p->frames_dev, p->items_dev + p->n_frame_items, nd,
                               p->direct_xcd.data(), p->launch, p->scratch, p->scratch_stride,
                               p->scratch_slots, s),
            "eval (per-pose buckets)");
    if (timed) prof_end(s, a, kStageEval, nd, p->direct_point_poses);
  }
  const int64_t nt = p->n_items - p->n_frame_items - p->n_stripe_items;
  if (nt > 0) {
    hipEvent_t a = nullptr;
    const bool timed = prof_begin(s, &a);
    HIP_TRY(launch_eval_tiles(p->pairs_dev, p->frames_dev,
                              p->items_dev + p->n_frame_items + p->n_stripe_items, nt,
                              p->tile_xcd.data(), p->tile_launch, p->tile_slots, s),
            "eval (tiles)");
    if (timed) prof_end(s, a, kStageEval, nt, p->tile_point_poses);
  }
  for (const PairHost &ph : p->pairs)
    if (ph.argmax_out && ph.K > 0)
      HIP_TRY(launch_argmax(ph.mi_out, ph.K, ph.ref->g->gi.nf, ph.argmax_out, nullptr, s),
              "argmax");
  return MI_OK;
}

}  // namespace

namespace {

// tiles: as for create_plan (batch plans tile their per-pose pairs; plans that
// bind scan B per execution bucket them by stripe)
size_t workspace_bytes(const mi_work_item *items, int64_t n_items, uint32_t flags, size_t budget,
                       bool tiles) {
  BatchTables B;
  if (prepare_batch(items, n_items, flags, B, tiles) != MI_OK) return 0;
  return batch_bytes(B, items, n_items, budget);
}

}  // namespace

extern "C" size_t mi_batch_workspace(const mi_work_item *items, int64_t n_items, uint32_t flags,
                                     size_t budget) {
  return guarded_size([&]() -> size_t {
  return workspace_bytes(items, n_items, flags, budget, true);
  });
}

extern "C" mi_status mi_batch_create(const mi_work_item *items, int64_t n_items, uint32_t flags,
                                     void *ws, size_t ws_bytes, size_t budget, void *stream,
                                     mi_plan **out) {
  return guarded("mi_batch_create", [&]() -> mi_status {
  for (int64_t i = 0; i < n_items && items; ++i) {
    if (items[i].K > 0 && !items[i].mi_out)
      return fail(MI_E_INVALID, "work item %lld: mi_out is NULL", (long long)i);
    if (items[i].n_b > 0 && !items[i].xyz_b)
      return fail(MI_E_INVALID, "work item %lld: xyz_b is NULL", (long long)i);
  }
  return create_plan(items, n_items, flags, ws, ws_bytes, budget, stream, false, out, false, true);
  });
}

extern "C" mi_status mi_batch_execute(mi_plan *p, void *stream) {
  return guarded("mi_batch_execute", [&]() -> mi_status {
  if (!p) return fail(MI_E_INVALID, "mi_batch_execute: NULL plan");
  if (p->bind_per_execution)
    return fail(MI_E_INVALID, "plan from mi_plan_create: execute it with mi_plan_execute");
  return run_plan(p, (hipStream_t)stream);
  });
}

extern "C" mi_status mi_eval_batch(const mi_work_item *items, int64_t n_items, uint32_t flags,
                                   void *ws, size_t ws_bytes, void *stream) {
  return guarded("mi_eval_batch", [&]() -> mi_status {
  mi_plan *p = nullptr;
  mi_status st = mi_batch_create(items, n_items, flags, ws, ws_bytes, 0, stream, &p);
  if (st != MI_OK) return st;
  st = run_plan(p, (hipStream_t)stream);
  mi_plan_destroy(p);
  return st;
  });
}

// ----------------------------------------------------------------- autotune

namespace {

// A strided sample of each item's poses (every ceil(K / max_poses)-th), so
// that the sample keeps the workload's mix of rotations and translations.
struct Sample {
  std::vector<std::vector<double>> poses;
  std::vector<mi_work_item> items;
};

void make_sample(const mi_work_item *w, int64_t n, int64_t max_poses, Sample &S) {
  S.poses.assign((size_t)n, std::vector<double>());
  S.items.assign(w, w + n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t K = w[i].K;
    const int64_t stride = max_poses > 0 && K > max_poses ? (K + max_poses - 1) / max_poses : 1;
    std::vector<double> &P = S.poses[(size_t)i];
    for (int64_t k = 0; k < K; k += stride) P.insert(P.end(), w[i].poses + 6 * k, w[i].poses + 6 * k + 6);
    mi_work_item &it = S.items[(size_t)i];
    it.poses = P.data();
    it.K = (int64_t)(P.size() / 6);
    it.argmax_out = nullptr;
    it.hist_out = nullptr;
    it.stats_out = nullptr;
  }
}

size_t sample_out_bytes(const Sample &S) {
  size_t b = 0;
  for (const mi_work_item &it : S.items)
    b += al256((size_t)it.ref->g->gi.nf * (size_t)std::max<int64_t>(it.K, 1) * sizeof(double));
  return b;
}

}  // namespace

extern "C" size_t mi_autotune_workspace(const mi_work_item *items, int64_t n_items, uint32_t flags,
                                        int64_t max_poses) {
  return guarded_size([&]() -> size_t {
  if (n_items <= 0 || !items) return 0;
  Sample S;
  make_sample(items, n_items, max_poses, S);
  BatchTables B;
  if (prepare_batch(S.items.data(), n_items, flags, B, true) != MI_OK) return 0;
  return sample_out_bytes(S) + batch_bytes(B, S.items.data(), n_items, 0) + 512;
  });
}

extern "C" mi_status mi_autotune(const mi_work_item *items, int64_t n_items, uint32_t flags,
                                 int64_t max_poses, void *ws, size_t ws_bytes, void *stream,
                                 mi_autotune_report *out) {
  return guarded("mi_autotune", [&]() -> mi_status {
  if (!items || n_items <= 0 || !out) return fail(MI_E_INVALID, "mi_autotune: bad arguments");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  hipStream_t s = (hipStream_t)stream;
  Sample S;
  make_sample(items, n_items, max_poses, S);
  Carver c(ws, ws_bytes);
  for (mi_work_item &it : S.items)
    it.mi_out = c.take<double>((size_t)it.ref->g->gi.nf * (size_t)std::max<int64_t>(it.K, 1));
  c.take<char>(0);
  if (!c.fits()) return fail(MI_E_WORKSPACE, "autotune workspace too small");
  void *bws = (void *)c.cur;
  const size_t bws_bytes = ws_bytes - c.used();
  mi_tuning start;
  mi_tuning_get(&start);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "autotune event");
  HIP_TRY(hipEventCreate(&e1), "autotune event");
  int tried = 0;
  // one warm execution, then the mean of two timed ones; <0 when the tuning
  // does not apply to this workload (LDS, key or plan limits)
  auto time_it = [&](const mi_tuning &t, double *ms) -> mi_status {
    *ms = -1.0;
    if (mi_tuning_set(&t) != MI_OK) return MI_OK;
    mi_plan *p = nullptr;
    mi_status st = create_plan(S.items.data(), n_items, flags, bws, bws_bytes, 0, stream, false, &p,
                               false, true);
    // a tuning the workload cannot use, or whose plan (per-pose scratch grows
    // with the resident workgroups) does not fit the workspace, is skipped
    if (st == MI_E_UNSUPPORTED || st == MI_E_WORKSPACE) return MI_OK;
    if (st != MI_OK) return st;
    st = run_plan(p, s);
    if (st == MI_OK) {
      if (hipEventRecord(e0, s) != hipSuccess) st = MI_E_DEVICE;
      for (int r = 0; r < 2 && st == MI_OK; ++r) st = run_plan(p, s);
      if (st == MI_OK && hipEventRecord(e1, s) != hipSuccess) st = MI_E_DEVICE;
      float f = 0.f;
      if (st == MI_OK && (hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&f, e0, e1) != hipSuccess))
        st = MI_E_DEVICE;
      if (st == MI_OK) *ms = f / 2.0;
    }
    mi_plan_destroy(p);
    ++tried;
    return st;
  };
  mi_status st = MI_OK;
  double start_ms = -1.0, best_ms = -1.0;
  mi_tuning best = start;
  auto consider = [&](const mi_tuning &t) {
    double ms = -1.0;
    if (st != MI_OK) return;
    st = time_it(t, &ms);
    if (st == MI_OK && ms >= 0.0 && (best_ms < 0.0 || ms < best_ms)) {
      best_ms = ms;
      best = t;
    }
  };
  st = time_it(start, &start_ms);
  if (st == MI_OK && start_ms >= 0.0) { best_ms = start_ms; best = start; }
  // stage 1: workgroup size and hash capacity
  const int waves[3] = {4, 8, 16};
  // 0 is the auto hash (66 KiB, or 60 KiB where 66 would leave one workgroup per CU)
  const int hashk[9] = {0, 24, 32, 48, 56, 60, 64, 66, 96};
  for (int w : waves)
    for (int hk : hashk) consider(mi_tuning{w, hk * 1024, 1, 12, 0});
  // stage 2: stripe height and histogram privatization around the best
  const mi_tuning b1 = best;
  const int rows[6] = {4, 8, 12, 16, 20, 24};
  const int copies[3] = {1, 2, 4};
  for (int r : rows)
    for (int h : copies) consider(mi_tuning{b1.waves, b1.hash_bytes, h, r, 0});
  // stage 3: one workgroup per pose, or a persistent grid
  const mi_tuning b2 = best;
  const int per_cu[3] = {1, 2, 4};
  for (int pc : per_cu) consider(mi_tuning{b2.waves, b2.hash_bytes, b2.hist_copies, b2.stripe_rows, pc});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MI_OK) {
    mi_tuning_set(&start);
    return st;
  }
  if (best_ms < 0.0) {
    mi_tuning_set(&start);
    return fail(MI_E_UNSUPPORTED, "no tuning applies to this workload");
  }
  mi_tuning_set(&best);
  out->best = best;
  out->best_ms = best_ms;
  out->start_ms = start_ms;
  out->tried = tried;
  return MI_OK;
  });
}

// ------------------------------------------------------------ tuning cache

namespace {

int ceil_log2(int64_t n) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// The cache file: {"key": [w, h, c, r, p], ...}.  Keys hold no quotes or
// backslashes (they are built by mi_tuning_cache_key).
bool cache_read(const char *path, std::map<std::string, std::array<int64_t, 5>> &m) {
  FILE *f = fopen(path, "rb");
  if (!f) return true;  // no file: an empty cache
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  fclose(f);
  size_t p = text.find('{');
  if (p == std::string::npos) return false;
  for (;;) {
    const size_t q0 = text.find('"', p);
    if (q0 == std::string::npos) break;
    const size_t q1 = text.find('"', q0 + 1);
    if (q1 == std::string::npos) return false;
    const std::string key = text.substr(q0 + 1, q1 - q0 - 1);
    const size_t b0 = text.find('[', q1), b1 = text.find(']', q1);
    if (b0 == std::string::npos || b1 == std::string::npos || b1 < b0) return false;
    std::array<int64_t, 5> v{};
    const char *c = text.c_str() + b0 + 1;
    for (int n = 0; n < 5; ++n) {
      char *end = nullptr;
      v[n] = strtoll(c, &end, 10);
      if (end == c) return false;
      c = end;
      while (*c == ' ' || *c == ',' || *c == '\n' || *c == '\t' || *c == '\r') ++c;
    }
    m[key] = v;
    p = b1 + 1;
  }
  return true;
}

bool key_ok(const char *key) {
  if (!key || !*key) return false;
  for (const char *c = key; *c; ++c)
    if (*c == '"' || *c == '\\' || (unsigned char)*c < 0x20) return false;
  return true;
}

}  // namespace

extern "C" mi_status mi_tuning_cache_key(const char *arch, uint32_t features, int32_t nb0,
                                         int32_t nb1, int64_t n_b, int64_t voxels, char *buf,
                                         size_t len) {
  return guarded("mi_tuning_cache_key", [&]() -> mi_status {
  if (!arch || !buf || len == 0) return fail(MI_E_INVALID, "mi_tuning_cache_key: bad argument");
  // the architecture up to its first ':' (feature suffixes such as :sramecc+)
  std::string a(arch);
  a = a.substr(0, a.find(':'));
  const int n = snprintf(buf, len, "%s/f%u/b%dx%d/n%d/v%d", a.c_str(), features, nb0, nb1,
                         ceil_log2(std::max<int64_t>(n_b, 1)),
                         ceil_log2(std::max<int64_t>(voxels, 1)));
  if (n < 0 || (size_t)n >= len) return fail(MI_E_INVALID, "mi_tuning_cache_key: buffer too small");
  if (!key_ok(buf)) return fail(MI_E_INVALID, "mi_tuning_cache_key: bad architecture name");
  return MI_OK;
  });
}

extern "C" mi_status mi_tuning_cache_get(const char *path, const char *key, mi_tuning *t,
                                         int32_t *found) {
  return guarded("mi_tuning_cache_get", [&]() -> mi_status {
  if (!path || !key_ok(key) || !t || !found)
    return fail(MI_E_INVALID, "mi_tuning_cache_get: bad argument");
  *found = 0;
  std::map<std::string, std::array<int64_t, 5>> m;
  if (!cache_read(path, m)) return fail(MI_E_INVALID, "tuning cache %s: not a cache file", path);
  const auto it = m.find(key);
  if (it == m.end()) return MI_OK;
  const auto &v = it->second;
  *t = mi_tuning{(int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3], (int32_t)v[4]};
  *found = 1;
  return MI_OK;
  });
}

extern "C" mi_status mi_tuning_cache_put(const char *path, const char *key, const mi_tuning *t) {
  return guarded("mi_tuning_cache_put", [&]() -> mi_status {
  if (!path || !key_ok(key) || !t) return fail(MI_E_INVALID, "mi_tuning_cache_put: bad argument");
  std::map<std::string, std::array<int64_t, 5>> m;
  if (!cache_read(path, m)) return fail(MI_E_INVALID, "tuning cache %s: not a cache file", path);
  m[key] = {t->waves, t->hash_bytes, t->hist_copies, t->stripe_rows, t->wgs_per_cu};
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) return fail(MI_E_INVALID, "tuning cache %s: cannot write", tmp.c_str());
  fputs("{\n", f);
  size_t k = 0;
  for (const auto &e : m) {
    const auto &v = e.second;
    fprintf(f, "  \"%s\": [%lld, %lld, %lld, %lld, %lld]%s\n", e.first.c_str(), (long long)v[0],
            (long long)v[1], (long long)v[2], (long long)v[3], (long long)v[4],
            ++k < m.size() ? "," : "");
  }
  fputs("}\n", f);
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return fail(MI_E_INVALID, "tuning cache %s: cannot write", path);
  }
  return MI_OK;
  });
}

extern "C" mi_status mi_autotune_cached(const mi_work_item *items, int64_t n_items,
                                        uint32_t flags, int64_t max_poses, void *ws,
                                        size_t ws_bytes, void *stream, const char *path,
                                        mi_autotune_report *out) {
  return guarded("mi_autotune_cached", [&]() -> mi_status {
  if (!items || n_items <= 0 || !out || !path)
    return fail(MI_E_INVALID, "mi_autotune_cached: bad arguments");
  int64_t nb_max = 0, v_max = 0;
  for (int64_t i = 0; i < n_items; ++i) {
    if (!items[i].ref) return fail(MI_E_INVALID, "work item %lld: NULL reference", (long long)i);
    nb_max = std::max(nb_max, items[i].n_b);
    v_max = std::max(v_max, items[i].ref->g->gi.V);
  }
  const GridInfo &gi = items[0].ref->g->gi;
  int dev = 0;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDevice(&dev), "device");
  HIP_TRY(hipGetDeviceProperties(&prop, dev), "device properties");
  char key[256];
  mi_status st = mi_tuning_cache_key(prop.gcnArchName, gi.features, gi.nb[0],
                                     gi.nf > 1 ? gi.nb[1] : 0, nb_max, v_max, key, sizeof key);
  if (st != MI_OK) return st;
  mi_tuning t;
  int32_t found = 0;
  st = mi_tuning_cache_get(path, key, &t, &found);
  if (st != MI_OK) return st;
  if (found) {
    st = mi_tuning_set(&t);
    if (st != MI_OK) return st;
    *out = mi_autotune_report{t, 0.0, 0.0, 0};
    return MI_OK;
  }
  st = mi_autotune(items, n_items, flags, max_poses, ws, ws_bytes, stream, out);
  if (st != MI_OK) return st;
  return mi_tuning_cache_put(path, key, &out->best);
  });
}

extern "C" size_t mi_eval_poses_workspace(const mi_ref *r, int64_t n_b, const double *poses,
                                          int64_t K, uint32_t flags, size_t budget) {
  return guarded_size([&]() -> size_t {
  if (!r) return 0;
  mi_work_item w;
  memset(&w, 0, sizeof w);
  w.ref = r; w.n_b = n_b; w.poses = poses; w.K = K;
  return workspace_bytes(&w, 1, flags, budget, false);
  });
}

extern "C" mi_status mi_plan_create(const mi_ref *r, int64_t n_b, const double *poses, int64_t K,
                                    uint32_t flags, void *ws, size_t ws_bytes, size_t budget,
                                    void *stream, mi_plan **out) {
  return guarded("mi_plan_create", [&]() -> mi_status {
  if (!r || !out) return fail(MI_E_INVALID, "mi_plan_create: NULL argument");
  *out = nullptr;
  mi_work_item w;
  memset(&w, 0, sizeof w);
  w.ref = r; w.n_b = n_b; w.poses = poses; w.K = K;
  return create_plan(&w, 1, flags, ws, ws_bytes, budget, stream, true, out);
  });
}

extern "C" mi_status mi_plan_execute(mi_plan *p, const float *xyz_b, double *mi_out,
                                     int64_t *argmax_out, uint32_t *hist_out,
                                     mi_pose_stats *stats_out, void *stream) {
  return guarded("mi_plan_execute", [&]() -> mi_status {
  if (!p) return fail(MI_E_INVALID, "mi_plan_execute: NULL plan");
  if (!p->bind_per_execution) return fail(MI_E_INVALID, "batch plan: execute it with mi_batch_execute");
  PairHost &ph = p->pairs[0];
  if (ph.K > 0 && !mi_out) return fail(MI_E_INVALID, "mi_out is NULL");
  if (ph.n_b > 0 && !xyz_b) return fail(MI_E_INVALID, "xyz_b is NULL");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_bind(p->pairs_dev, p->frames_dev, p->F, xyz_b, mi_out, hist_out, stats_out, s),
          "bind");
  ph.xyz = xyz_b;
  ph.mi_out = mi_out;
  ph.argmax_out = argmax_out;
  return run_plan(p, s);
  });
}

extern "C" void mi_plan_destroy(mi_plan *p) { delete p; }

extern "C" mi_status mi_plan_launch(const mi_plan *p, mi_tuning *t, int32_t *lds_bytes) {
  return guarded("mi_plan_launch", [&]() -> mi_status {
  if (!p) return fail(MI_E_INVALID, "mi_plan_launch: NULL plan");
  if (t) *t = p->tuning;
  if (lds_bytes) *lds_bytes = (int32_t)eval_lds_bytes(p->launch);
  return MI_OK;
  });
}

extern "C" mi_status mi_eval_poses(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                   const double *poses, int64_t K, uint32_t flags, double *mi_out,
                                   int64_t *argmax_out, uint32_t *hist_out,
                                   mi_pose_stats *stats_out, void *ws, size_t ws_bytes,
                                   void *stream) {
  return guarded("mi_eval_poses", [&]() -> mi_status {
  mi_plan *p = nullptr;
  mi_status st = mi_plan_create(r, n_b, poses, K, flags, ws, ws_bytes, 0, stream, &p);
  if (st != MI_OK) return st;
  st = mi_plan_execute(p, xyz_b, mi_out, argmax_out, hist_out, stats_out, stream);
  mi_plan_destroy(p);
  return st;
  });
}

// ------------------------------------------------------------ static scratch

// Device memory of mi_eval_poses_static: one array per GPU, held until the
// process ends.  In host code the array's name only stands for the symbol;
// its device address (per device) comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char static_scratch[MI_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
}  // namespace

extern "C" mi_status mi_eval_poses_static(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                          const double *poses, int64_t K, uint32_t flags,
                                          double *mi_out, int64_t *argmax_out, uint32_t *hist_out,
                                          mi_pose_stats *stats_out, void *stream) {
  return guarded("mi_eval_poses_static", [&]() -> mi_status {
  if (!r) return fail(MI_E_INVALID, "mi_eval_poses_static: NULL ref");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(MI_E_UNSUPPORTED, "device index %d", dev);
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {  // once per device, with that device current
      void *q = nullptr;
      HIP_TRY(hipGetSymbolAddress(&q, HIP_SYMBOL(static_scratch)), "static scratch address");
      g_static_ptr[dev] = q;
    }
    base = g_static_ptr[dev];
  }
  mi_work_item w;
  memset(&w, 0, sizeof w);
  w.ref = r; w.n_b = n_b; w.poses = poses; w.K = K;
  mi_plan *p = nullptr;
  mi_status st = create_plan(&w, 1, flags, base, (size_t)MI_STATIC_SCRATCH_BYTES, 0, stream, true,
                             &p, true);
  if (st == MI_E_WORKSPACE)
    return fail(MI_E_UNSUPPORTED, "mi_eval_poses_static: the %lld-byte static scratch is too small: %s",
                (long long)MI_STATIC_SCRATCH_BYTES, t_err.c_str());
  if (st != MI_OK) return st;
  st = mi_plan_execute(p, xyz_b, mi_out, argmax_out, hist_out, stats_out, stream);
  mi_plan_destroy(p);
  return st;
  });
}

// ---------------------------------------------------------------- plain

namespace {
struct PlainLayout {
  PlainDev pd;
  double *rc;
};

void plain_layout(const GridInfo &gi, int64_t n_b, int64_t K, Carver &c, PlainLayout *L) {
  const int64_t V = gi.V;
  const size_t nbp = (size_t)std::max<int64_t>(n_b, 1);
  uint32_t *dn = c.take<uint32_t>((size_t)V);
  unsigned long long *ds1 = c.take<unsigned long long>((size_t)V);
  unsigned long long *ds2 = c.take<unsigned long long>((size_t)V);
  int32_t *lin = c.take<int32_t>(nbp);
  uint32_t *q = c.take<uint32_t>(nbp);
  uint8_t *near = c.take<uint8_t>(nbp);
  int32_t *bbox = c.take<int32_t>(8);
  unsigned long long *ctr = c.take<unsigned long long>(4);
  uint32_t *hist = c.take<uint32_t>(2 * kMaxBins * kMaxBins);
  double *rc = c.take<double>((size_t)std::max<int64_t>(K, 1) * 12);
  if (L) {
    L->pd.dn = dn; L->pd.ds1 = ds1; L->pd.ds2 = ds2; L->pd.lin = lin; L->pd.q = q;
    L->pd.near = near; L->pd.bbox = bbox; L->pd.ctr = ctr; L->pd.hist = hist;
    L->rc = rc;
  }
}
}  // namespace

extern "C" size_t mi_eval_poses_plain_workspace(const mi_ref *r, int64_t n_b, int64_t K) {
  return guarded_size([&]() -> size_t {
  if (!r || n_b < 0 || K < 0) return 0;
  Carver c(nullptr, 0);
  plain_layout(r->g->gi, n_b, K, c, nullptr);
  return c.used() + 256;
  });
}

extern "C" mi_status mi_eval_poses_plain(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                         const double *poses, int64_t K, uint32_t flags,
                                         double *mi_out, int64_t *argmax_out, uint32_t *hist_out,
                                         mi_pose_stats *stats_out, void *ws, size_t ws_bytes,
                                         void *stream) {
  return guarded("mi_eval_poses_plain", [&]() -> mi_status {
  if (!r) return fail(MI_E_INVALID, "mi_eval_poses_plain: NULL ref");
  if (K < 0 || n_b < 0 || (K > 0 && (!poses || !mi_out)) || (n_b > 0 && !xyz_b))
    return fail(MI_E_INVALID, "bad arguments");
  if (flags & ~(uint32_t)MI_EVAL_NEAR_FACE) return fail(MI_E_INVALID, "unknown flags");
  if (n_b >= ((int64_t)1 << 31)) return fail(MI_E_UNSUPPORTED, "scan B too large");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  const GridInfo &gi = r->g->gi;
  Carver c(ws, ws_bytes);
  PlainLayout PL;
  memset(&PL, 0, sizeof PL);
  plain_layout(gi, n_b, K, c, &PL);
  if (!c.fits())
    return fail(MI_E_WORKSPACE, "plain workspace needs %zu bytes, got %zu", c.used() + 256,
                ws_bytes);
  for (int64_t k = 0; k < K; ++k)
    for (int a = 0; a < 6; ++a)
      if (!std::isfinite(poses[6 * k + a])) return fail(MI_E_INVALID, "non-finite pose");
  PlainDev &pd = PL.pd;
  pd.nx = gi.dims[0]; pd.ny = gi.dims[1]; pd.nz = gi.dims[2]; pd.nf = gi.nf;
  for (int f = 0; f < 2; ++f) {
    pd.kind[f] = gi.kind[f];
    pd.nb[f] = gi.nb[f];
    pd.binA[f] = r->rd.bins[f];
  }
  pd.nbc = gi.nbc;
  pd.nbz = gi.nbz;
  pd.voxel = gi.voxel;
  pd.s = gi.s;
  pd.abox = r->rd.abox;
  memcpy(pd.count_edges, gi.count_edges, sizeof pd.count_edges);
  memcpy(pd.zvar_edges, gi.zvar_edges, sizeof pd.zvar_edges);
  hipStream_t s = (hipStream_t)stream;
  if (K == 0) return MI_OK;
  hipError_t e = hipSuccess;
  const size_t bytes = sizeof(double) * 12 * (size_t)K;
  Staging *st = staging_acquire(bytes, &e);
  if (!st) return dev_fail(e, "pinned staging");
  double *h = (double *)st->p;
  for (int64_t k = 0; k < K; ++k) {
    const double *eta = poses + 6 * k;
    pose_rotation(eta, h + 12 * k);
    for (int a = 0; a < 3; ++a) h[12 * k + 9 + a] = (eta[a] - gi.origin[a]) * gi.s;
  }
  const Upload up = {PL.rc, 0, bytes};
  HIP_TRY(staging_upload(st, &up, 1, s), "plain pose upload");
  HIP_TRY(launch_plain_clear_dense(pd, s), "plain clear");
  const int64_t hoff[2] = {0, K * (int64_t)gi.nb[0] * gi.nb[0]};
  hipEvent_t a = nullptr;
  const bool timed = prof_begin(s, &a);
  for (int64_t k = 0; k < K; ++k)
    HIP_TRY(launch_plain_pose(pd, nullptr, xyz_b, n_b, PL.rc, k, mi_out, K, hist_out, hoff,
                              stats_out, (flags & MI_EVAL_NEAR_FACE) != 0, s),
            "plain pose");
  if (timed) prof_end(s, a, kStagePlain, K, K * n_b);
  if (argmax_out) HIP_TRY(launch_argmax(mi_out, K, gi.nf, argmax_out, nullptr, s), "argmax");
  return MI_OK;
  });
}

// ------------------------------------------------------------ coarse-to-fine

namespace {
// A search's objective: one feature slot, or the weighted slots (finite weights).
bool slot_ok(int32_t slot, const double w[2], int nf) {
  if (slot == MI_SLOT_WEIGHTED) return std::isfinite(w[0]) && std::isfinite(w[1]);
  return slot >= 0 && slot < nf;
}

// Row of a search's objective within mi [nf + 1][K]: the slot's row, or row nf
// after the weighted objective is written there.
hipError_t objective_row(double *mi, int64_t K, int nf, int32_t slot, const double w[2],
                         const double **row, hipStream_t s) {
  if (slot != MI_SLOT_WEIGHTED) {
    *row = mi + (int64_t)slot * K;
    return hipSuccess;
  }
  *row = mi + (int64_t)nf * K;
  return launch_weighted(mi, K, nf, w[0], w[1], mi + (int64_t)nf * K, s);
}

bool c2f_ok(const mi_c2f_desc *d, int nf) {
  if (!d || d->levels < 1 || !(d->shrink > 0.0) || !std::isfinite(d->shrink)) return false;
  if (!slot_ok(d->feature_slot, d->weight, nf)) return false;
  int64_t K = 1;
  for (int a = 0; a < 6; ++a) {
    if (d->samples[a] < 1 || d->samples[a] > 1024 || !std::isfinite(d->half_range[a]) ||
        d->half_range[a] < 0.0)
      return false;
    K *= d->samples[a];
  }
  return K < ((int64_t)1 << 31);  // a level is one plan of fewer than 2^31 poses
}

int64_t c2f_count(const mi_c2f_desc *d) {
  int64_t K = 1;
  for (int a = 0; a < 6; ++a) K *= d->samples[a];
  return K;
}

// One level's grid: per axis c + h*(-1 + 2j/(s-1)) (c when s = 1), row-major
// over (tx, ty, tz, roll, pitch, yaw) with yaw fastest.
void c2f_grid(const double c[6], const double h[6], const int32_t samples[6],
              std::vector<double> &P) {
  int64_t K = 1;
  for (int a = 0; a < 6; ++a) K *= samples[a];
  P.resize((size_t)K * 6);
  std::vector<double> node[6];
  for (int a = 0; a < 6; ++a) {
    const int32_t sa = samples[a];
    node[a].resize((size_t)sa);
    for (int32_t j = 0; j < sa; ++j)
      node[a][(size_t)j] = sa == 1 ? c[a] : c[a] + h[a] * (-1.0 + (2.0 * j) / (double)(sa - 1));
  }
  int32_t j[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = 0; k < K; ++k) {
    for (int a = 0; a < 6; ++a) P[(size_t)k * 6 + a] = node[a][(size_t)j[a]];
    for (int a = 5; a >= 0; --a) {  // yaw fastest
      if (++j[a] < samples[a]) break;
      j[a] = 0;
    }
  }
}
}  // namespace

extern "C" size_t mi_align_workspace(const mi_ref *r, int64_t n_b, const mi_c2f_desc *d) {
  return guarded_size([&]() -> size_t {
  if (!r || n_b < 0 || !c2f_ok(d, r->g->gi.nf)) return 0;
  const GridInfo &gi = r->g->gi;
  const int64_t K = c2f_count(d);
  int64_t F = (int64_t)d->samples[3] * d->samples[4] * d->samples[5];
  // column grid of the widest level (level 0), plus slack for its position
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  std::vector<double> P;
  c2f_grid(zero, d->half_range, d->samples, P);
  PoseTables T;
  if (build_tables(gi, P.data(), K, T)) return 0;
  const int64_t ncols = (int64_t)(T.ncx + 2) * (T.ncy + 2);
  Carver c(nullptr, 0);
  c.take<double>(((size_t)gi.nf + 1) * (size_t)K);
  c.take<int64_t>(2 * 8);
  return c.used() + single_plan_bytes(K, (int32_t)F, ncols, n_b) + 512;
  });
}

extern "C" mi_status mi_align_coarse_to_fine(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                             const double init[6], const mi_c2f_desc *d,
                                             double pose_out[6], double *mi_best, void *ws,
                                             size_t ws_bytes, void *stream) {
  return guarded("mi_align_coarse_to_fine", [&]() -> mi_status {
  if (!r || !init || !pose_out) return fail(MI_E_INVALID, "mi_align_coarse_to_fine: NULL");
  const GridInfo &gi = r->g->gi;
  if (!c2f_ok(d, gi.nf)) return fail(MI_E_INVALID, "bad coarse-to-fine description");
  for (int a = 0; a < 6; ++a)
    if (!std::isfinite(init[a])) return fail(MI_E_INVALID, "non-finite initial pose");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  const int64_t K = c2f_count(d);
  Carver c(ws, ws_bytes);
  double *mi_dev = c.take<double>(((size_t)gi.nf + 1) * (size_t)K);
  int64_t *am_dev = c.take<int64_t>(2);
  double *mv_dev = c.take<double>(2);
  c.take<char>(0);
  if (!c.fits()) return fail(MI_E_WORKSPACE, "align workspace too small");
  void *plan_ws = (void *)c.cur;
  const size_t plan_room = ws_bytes - c.used();
  hipStream_t s = (hipStream_t)stream;
  double ctr[6], h[6];
  for (int a = 0; a < 6; ++a) { ctr[a] = init[a]; h[a] = d->half_range[a]; }
  std::vector<double> P;
  double best = 0.0;
  for (int32_t l = 0; l < d->levels; ++l) {
    c2f_grid(ctr, h, d->samples, P);
    mi_plan *p = nullptr;
    mi_status st = mi_plan_create(r, n_b, P.data(), K, 0, plan_ws, plan_room, 0, stream, &p);
    if (st != MI_OK) return st;
    st = mi_plan_execute(p, xyz_b, mi_dev, nullptr, nullptr, nullptr, stream);
    mi_plan_destroy(p);
    if (st != MI_OK) return st;
    const double *obj = nullptr;
    HIP_TRY(objective_row(mi_dev, K, gi.nf, d->feature_slot, d->weight, &obj, s), "objective");
    HIP_TRY(launch_argmax(obj, K, 1, am_dev, mv_dev, s), "argmax");
    int64_t kbest = 0;
    double mv = 0.0;
    HIP_TRY(hipMemcpyAsync(&kbest, am_dev, sizeof kbest, hipMemcpyDeviceToHost, s), "argmax D2H");
    HIP_TRY(hipMemcpyAsync(&mv, mv_dev, sizeof mv, hipMemcpyDeviceToHost, s), "MI D2H");
    HIP_TRY(hipStreamSynchronize(s), "level sync");
    if (kbest < 0 || kbest >= K) return fail(MI_E_DEVICE, "argmax out of range");
    for (int a = 0; a < 6; ++a) ctr[a] = P[(size_t)kbest * 6 + a];
    best = mv;
    for (int a = 0; a < 6; ++a) h[a] = h[a] / d->shrink;
  }
  for (int a = 0; a < 6; ++a) pose_out[a] = ctr[a];
  if (mi_best) *mi_best = best;
  return MI_OK;
  });
}

// ---------------------------------------------------------------- serving

namespace {

// First-fit allocator over offsets of a caller-owned device range, in
// 256-byte granules; neighbours merge on release.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = al256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, o = it->first + bytes;
      free_.erase(it);
      if (rest) free_[o] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    if (!bytes) return;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;

 public:
  size_t free_bytes() const {
    size_t b = 0;
    for (const auto &kv : free_) b += kv.second;
    return b;
  }
};

struct Request {
  int64_t id = 0;
  mi_request_state st;
  mi_grid_desc gd;
  std::vector<uint32_t> ce;
  std::vector<uint64_t> ze;
  std::vector<float> a, b;
  int64_t n_a = 0, n_b = 0;
  mi_c2f_desc search;
  double ctr[6], h[6];
  mi_grid *g = nullptr;
  mi_ref *ref = nullptr;
  size_t ref_bytes = 0, ref_keep = 0;
  size_t off_b = 0, off_a = 0, off_ref = 0;
  bool holds = false;              // arena blocks of scan B and the resident reference held
  bool holds_a = false;            // scan A's block held (until its reference is built)
  bool holds_ref_tail = false;     // the reference workspace's transient tail held
  std::vector<double> P;           // poses of the current level
  size_t slot = 0;                 // place of its argmax in the pinned results
  TileGeom geo;                    // tiles of scan B (chosen when submitted)
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mi_server {
  char *arena = nullptr;
  size_t arena_bytes = 0, step_bytes = 0;
  int32_t max_active = 1;
  hipStream_t stream = nullptr;
  Arena heap;                      // offsets within [step_bytes, arena_bytes)
  std::mutex mu;                   // queue and request table
  std::deque<Request *> queue;
  std::vector<Request *> active;
  std::unordered_map<int64_t, std::unique_ptr<Request>> table;
  int64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  char *pinned = nullptr;          // [max_active] x (argmax, MI), then [max_active] x 128 counts
};

namespace {

size_t req_points_bytes(int64_t n) { return al256((size_t)std::max<int64_t>(n, 1) * 3 * sizeof(float)); }

// Device bytes a step needs for one request alone: its pose table, outputs
// and the largest of its rotated frames.
size_t req_step_bytes(const Request &r) {
  const GridInfo &gi = r.g->gi;
  const int64_t K = c2f_count(&r.search);
  const double spread_x = 2.0 * r.search.half_range[0] * gi.s + 4.0;
  const double spread_y = 2.0 * r.search.half_range[1] * gi.s + 4.0;
  const int64_t ncols = (int64_t)(gi.dims[0] + spread_x) * (int64_t)(gi.dims[1] + spread_y);
  const FrameBytes fb = frame_bytes(r.n_b, ncols);
  // tiles: up to 4 entries per point and the tile tables (a level runs in
  // frames or in tiles; both are counted)
  const int64_t tm = tiles_max(r.n_b);
  const size_t tiles = al256((size_t)(12 * std::max<int64_t>(r.n_b, 1)) * sizeof(float)) +
                       al256((size_t)(tm + 1) * 4) + al256((size_t)tm * 4) +
                       al256((size_t)(2 * tm) * 4) + 256;
  return al256((size_t)K * sizeof(PoseDev)) + al256(sizeof(PairDev)) +
         al256((size_t)K * sizeof(FrameDev)) + al256(((size_t)gi.nf + 1) * K * 8) + 4 * 256 + fb.v +
         fb.off + al256(fb.cur) + tiles + 4096;
}

// Give back every arena block the request still holds: scan B and the
// resident reference always, scan A and the reference's transient tail when a
// failure came before the reference was built.
void req_release(mi_server *s, Request *r) {
  if (r->holds_a) {
    s->heap.release(r->off_a, req_points_bytes(r->n_a));
    r->holds_a = false;
  }
  if (r->holds_ref_tail) {
    s->heap.release(r->off_ref + r->ref_keep, al256(r->ref_bytes) - r->ref_keep);
    r->holds_ref_tail = false;
  }
  if (r->holds) {
    s->heap.release(r->off_b, req_points_bytes(r->n_b));
    s->heap.release(r->off_ref, r->ref_keep);
    r->holds = false;
  }
  if (r->ref) { mi_ref_destroy(r->ref); r->ref = nullptr; }
}

void req_fail(mi_server *s, Request *r, mi_status st) {
  req_release(s, r);
  std::lock_guard<std::mutex> lk(s->mu);
  r->st.state = MI_REQ_FAILED;
  r->st.status = st;
  r->st.t_done = seconds_since(s->t0);
}

// Arena blocks for scan B, scan A and the reference workspace; all or none.
bool req_reserve(mi_server *s, Request *r) {
  size_t ob, oa, orf;
  if (!s->heap.alloc(req_points_bytes(r->n_b), &ob)) return false;
  if (!s->heap.alloc(req_points_bytes(r->n_a), &oa)) {
    s->heap.release(ob, req_points_bytes(r->n_b));
    return false;
  }
  if (!s->heap.alloc(r->ref_bytes, &orf)) {
    s->heap.release(ob, req_points_bytes(r->n_b));
    s->heap.release(oa, req_points_bytes(r->n_a));
    return false;
  }
  r->off_b = ob;
  r->off_a = oa;
  r->off_ref = orf;
  r->holds = true;
  r->holds_a = true;
  r->holds_ref_tail = true;
  return true;
}

// Upload both scans and build the reference; scan A's block and the
// reference's transient sums go back to the heap as soon as the kernels that
// use them are enqueued (later users of that memory run after them on the
// same stream).
// Upload the request's scans and begin its reference; A's per-bin voxel
// counts go to counts (pinned host memory) on the server's stream.
mi_status req_begin(mi_server *s, Request *r, RefBuild *b, uint32_t *counts) {
  char *base = s->arena + s->step_bytes;
  float *db = (float *)(base + r->off_b), *da = (float *)(base + r->off_a);
  const size_t bb = (size_t)r->n_b * 3 * sizeof(float), ba = (size_t)r->n_a * 3 * sizeof(float);
  hipError_t e = hipSuccess;
  if (bb + ba > 0) {
    Staging *sg = staging_acquire(bb + ba + 64, &e);
    if (!sg) return dev_fail(e, "pinned staging");
    if (bb) memcpy(sg->p, r->b.data(), bb);
    if (ba) memcpy((char *)sg->p + bb, r->a.data(), ba);
    const Upload ups[2] = {{db, 0, bb}, {da, bb, ba}};
    e = staging_upload(sg, ups, 2, s->stream);
    if (e != hipSuccess) return dev_fail(e, "scan upload");
  }
  return ref_begin(r->g, da, r->n_a, base + r->off_ref, r->ref_bytes, s->stream, counts, b);
}

// Once the counts have arrived: build the reference's tables, then give back
// scan A's block and everything past what the reference keeps (the transient
// sums and the part of the table region that A's bin counts left unused).
mi_status req_finish(mi_server *s, Request *r, RefBuild &b, const uint32_t *counts) {
  mi_status st = ref_finish(r->g, b, counts, s->stream, &r->ref);
  if (st != MI_OK) return st;
  s->heap.release(r->off_a, req_points_bytes(r->n_a));
  r->holds_a = false;
  const size_t keep = al256(mi_ref_resident_bytes(r->ref));
  s->heap.release(r->off_ref + keep, al256(r->ref_bytes) - keep);
  r->ref_keep = keep;
  r->holds_ref_tail = false;
  std::vector<float>().swap(r->a);
  std::vector<float>().swap(r->b);
  return MI_OK;
}

// One search level of a group of active requests as one batch, carved from
// the step region; a group that does not fit is split in halves.  The
// argmaxes land in the pinned results; nothing here waits for the device.
mi_status run_level(mi_server *s, Request *const *rs, size_t n,
                    std::vector<std::pair<Request *, mi_status>> &failed) {
  if (n == 0) return MI_OK;
  Carver c(s->arena, s->step_bytes);
  std::vector<mi_work_item> items(n);
  std::vector<double *> mis(n);
  std::vector<int64_t *> ams(n);
  std::vector<double *> mvs(n);
  std::vector<TileGeom> geo(n);
  char *base = s->arena + s->step_bytes;
  for (size_t i = 0; i < n; ++i) {
    Request *r = rs[i];
    c2f_grid(r->ctr, r->h, r->search.samples, r->P);
    const int64_t K = (int64_t)(r->P.size() / 6);
    mis[i] = c.take<double>(((size_t)r->g->gi.nf + 1) * (size_t)K);
    ams[i] = c.take<int64_t>(1);
    mvs[i] = c.take<double>(1);
    mi_work_item &w = items[i];
    memset(&w, 0, sizeof w);
    w.ref = r->ref;
    w.xyz_b = (const float *)(base + r->off_b);
    w.n_b = r->n_b;
    w.poses = r->P.data();
    w.K = K;
    w.mi_out = mis[i];
    geo[i] = r->geo;
  }
  c.take<char>(0);
  mi_status st = MI_E_WORKSPACE;
  mi_plan *p = nullptr;
  if (c.fits())
    st = create_plan(items.data(), (int64_t)n, 0, (void *)c.cur, s->step_bytes - c.used(), 0,
                     s->stream, false, &p, false, true, geo.data());
  if (st != MI_OK && st != MI_E_DEVICE && n > 1) {
    // split until every part fits, or a single request shows what is wrong with it
    const size_t h = n / 2;
    mi_status a = run_level(s, rs, h, failed);
    if (a != MI_OK) return a;
    return run_level(s, rs + h, n - h, failed);
  }
  if (st != MI_OK && st != MI_E_DEVICE) {
    failed.emplace_back(rs[0], st);
    return MI_OK;
  }
  if (st != MI_OK) return st;
  st = run_plan(p, s->stream);
  mi_plan_destroy(p);
  if (st != MI_OK) return st;
  for (size_t i = 0; i < n; ++i) {
    Request *r = rs[i];
    const int64_t K = items[i].K;
    const double *obj = nullptr;
    HIP_TRY(objective_row(mis[i], K, r->g->gi.nf, r->search.feature_slot, r->search.weight, &obj,
                          s->stream), "objective");
    HIP_TRY(launch_argmax(obj, K, 1, ams[i], mvs[i], s->stream), "argmax");
    char *dst = s->pinned + 16 * r->slot;
    HIP_TRY(hipMemcpyAsync(dst, ams[i], 8, hipMemcpyDeviceToHost, s->stream), "argmax D2H");
    HIP_TRY(hipMemcpyAsync(dst + 8, mvs[i], 8, hipMemcpyDeviceToHost, s->stream), "MI D2H");
  }
  return MI_OK;
}

}  // namespace

extern "C" mi_status mi_server_create(const mi_server_desc *d, void *stream, mi_server **out) {
  return guarded("mi_server_create", [&]() -> mi_status {
  if (!d || !out) return fail(MI_E_INVALID, "mi_server_create: NULL argument");
  *out = nullptr;
  if (!d->arena || ((uintptr_t)d->arena & 255)) return fail(MI_E_WORKSPACE, "arena NULL or not 256-aligned");
  if (d->max_active < 1 || d->max_active > 65536) return fail(MI_E_INVALID, "max_active out of range");
  size_t step = d->step_bytes ? d->step_bytes : d->arena_bytes / 4;
  step &= ~(size_t)255;
  if (step < ((size_t)1 << 20) || step >= d->arena_bytes)
    return fail(MI_E_WORKSPACE, "step region must be at least 1 MiB and leave room for requests");
  std::unique_ptr<mi_server> s(new (std::nothrow) mi_server());
  if (!s) return fail(MI_E_INVALID, "out of host memory");
  s->arena = (char *)d->arena;
  s->arena_bytes = d->arena_bytes;
  s->step_bytes = step;
  s->max_active = d->max_active;
  s->stream = (hipStream_t)stream;
  s->heap.init((d->arena_bytes - step) & ~(size_t)255);
  s->t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipHostMalloc((void **)&s->pinned, (16 + 128 * sizeof(uint32_t)) * (size_t)d->max_active,
                        hipHostMallocDefault),
          "pinned results");
  *out = s.release();
  return MI_OK;
  });
}

extern "C" mi_status mi_server_submit(mi_server *s, const mi_request *q, int64_t *id) {
  return guarded("mi_server_submit", [&]() -> mi_status {
  if (!s || !q || !id) return fail(MI_E_INVALID, "mi_server_submit: NULL argument");
  *id = 0;
  if (q->n_a < 0 || q->n_b < 0 || (q->n_a > 0 && !q->xyz_a) || (q->n_b > 0 && !q->xyz_b))
    return fail(MI_E_INVALID, "bad scans");
  for (int a = 0; a < 6; ++a)
    if (!std::isfinite(q->init[a])) return fail(MI_E_INVALID, "non-finite initial pose");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fail(MI_E_INVALID, "out of host memory");
  r->gd = q->grid;
  // the request keeps its own copy of the edges (at most as many as a valid
  // grid reads; mi_grid_create rejects larger bin counts)
  if (q->grid.count_edges && q->grid.nbins_count > 1) {
    const int ne = std::min(q->grid.nbins_count, kMaxBins) - 1;
    r->ce.assign(q->grid.count_edges, q->grid.count_edges + ne);
    r->gd.count_edges = r->ce.data();
  }
  if (q->grid.zvar_edges && q->grid.nbins_zvar > 2) {
    const int ne = std::min(q->grid.nbins_zvar, kMaxBins) - 2;
    r->ze.assign(q->grid.zvar_edges, q->grid.zvar_edges + ne);
    r->gd.zvar_edges = r->ze.data();
  }
  mi_status st = mi_grid_create(&r->gd, &r->g);
  if (st != MI_OK) return st;
  std::unique_ptr<mi_grid, void (*)(mi_grid *)> gguard(r->g, mi_grid_destroy);
  const GridInfo &gi = r->g->gi;
  if (!c2f_ok(&q->search, gi.nf)) return fail(MI_E_INVALID, "bad search description");
  if ((gi.features & (MI_FEAT_ZVAR | MI_FEAT_JOINT)) && q->n_b >= MI_MAX_POINTS)
    return fail(MI_E_UNSUPPORTED, "scan B has >= 2^20 points with the z-variance feature");
  r->search = q->search;
  r->n_a = q->n_a;
  r->n_b = q->n_b;
  r->a.assign(q->xyz_a, q->xyz_a + 3 * q->n_a);
  r->b.assign(q->xyz_b, q->xyz_b + 3 * q->n_b);
  // the tiles of scan B and its point order, from the host copy (here, in the
  // submitting thread, rather than in the step loop)
  r->geo = choose_tiles(r->b.data(), q->n_b, gi.voxel, tile_cap_for(gi));
  for (int a = 0; a < 6; ++a) { r->ctr[a] = q->init[a]; r->h[a] = q->search.half_range[a]; }
  size_t keep = 0;
  r->ref_bytes = mi_features_ref_workspace(r->g, q->n_a, &keep);
  r->ref_keep = al256(keep);
  // what an empty heap holds (its size is rounded down to 256-byte granules),
  // so that every accepted request is admitted once the others are done
  const size_t need = req_points_bytes(q->n_a) + req_points_bytes(q->n_b) + al256(r->ref_bytes);
  const size_t heap_bytes = (s->arena_bytes - s->step_bytes) & ~(size_t)255;
  if (need > heap_bytes)
    return fail(MI_E_UNSUPPORTED, "request needs %zu bytes of arena, the server has %zu", need,
                heap_bytes);
  if (req_step_bytes(*r) > s->step_bytes)
    return fail(MI_E_UNSUPPORTED, "one search level of the request needs a step region of %zu "
                "bytes, the server has %zu", req_step_bytes(*r), s->step_bytes);
  gguard.release();
  memset(&r->st, 0, sizeof r->st);
  r->st.state = MI_REQ_QUEUED;
  r->st.status = MI_OK;
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->st.t_submit = seconds_since(s->t0);
  *id = r->id;
  s->queue.push_back(r.get());
  s->table.emplace(r->id, std::move(r));
  return MI_OK;
  });
}

extern "C" mi_status mi_server_step(mi_server *s, int32_t *n_active, int32_t *n_queued) {
  return guarded("mi_server_step", [&]() -> mi_status {
  if (!s) return fail(MI_E_INVALID, "mi_server_step: NULL server");
  // admission: arrival order, while a slot is free and the data fits
  std::vector<Request *> admitted;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->queue.empty() && (int32_t)s->active.size() < s->max_active) {
      Request *r = s->queue.front();
      if (!req_reserve(s, r)) break;
      s->queue.pop_front();
      r->st.state = MI_REQ_ACTIVE;
      r->st.t_admit = seconds_since(s->t0);
      s->active.push_back(r);
      admitted.push_back(r);
    }
  }
  // new references: all begun, one wait for their bin counts, all finished
  if (!admitted.empty()) {
    uint32_t *counts = (uint32_t *)(s->pinned + 16 * (size_t)s->max_active);
    std::vector<RefBuild> builds(admitted.size());
    std::vector<mi_status> began(admitted.size());
    for (size_t i = 0; i < admitted.size(); ++i)
      began[i] = req_begin(s, admitted[i], &builds[i], counts + 128 * i);
    const hipError_t se = hipStreamSynchronize(s->stream);
    if (se != hipSuccess) {
      // none of them has a reference: they fail rather than stay active
      for (Request *r : admitted) req_fail(s, r, MI_E_DEVICE);
      return dev_fail(se, "bin counts");
    }
    for (size_t i = 0; i < admitted.size(); ++i) {
      const mi_status st =
          began[i] == MI_OK ? req_finish(s, admitted[i], builds[i], counts + 128 * i) : began[i];
      if (st != MI_OK) req_fail(s, admitted[i], st);
    }
  }
  std::vector<Request *> live;
  for (Request *r : s->active)
    if (r->st.state == MI_REQ_ACTIVE) live.push_back(r);
  for (size_t i = 0; i < live.size(); ++i) live[i]->slot = i;
  std::vector<std::pair<Request *, mi_status>> failed;
  mi_status st = run_level(s, live.data(), live.size(), failed);
  if (st != MI_OK) return st;
  HIP_TRY(hipStreamSynchronize(s->stream), "step sync");
  const double now = seconds_since(s->t0);
  for (auto &f : failed) req_fail(s, f.first, f.second);
  for (Request *r : live) {
    if (r->st.state != MI_REQ_ACTIVE) continue;
    int64_t kbest;
    double mv;
    memcpy(&kbest, s->pinned + 16 * r->slot, 8);
    memcpy(&mv, s->pinned + 16 * r->slot + 8, 8);
    const int64_t K = (int64_t)(r->P.size() / 6);
    if (kbest < 0 || kbest >= K) { req_fail(s, r, MI_E_DEVICE); continue; }
    for (int a = 0; a < 6; ++a) r->ctr[a] = r->P[(size_t)kbest * 6 + a];
    for (int a = 0; a < 6; ++a) r->h[a] = r->h[a] / r->search.shrink;
    std::lock_guard<std::mutex> lk(s->mu);
    r->st.levels_done += 1;
    for (int a = 0; a < 6; ++a) r->st.pose[a] = r->ctr[a];
    r->st.mi = mv;
    if (r->st.levels_done >= r->search.levels) {
      r->st.state = MI_REQ_DONE;
      r->st.t_done = now;
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<Request *> still;
    for (Request *r : s->active) {
      if (r->st.state == MI_REQ_ACTIVE) still.push_back(r);
      else req_release(s, r);
    }
    s->active.swap(still);
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
  }
  return MI_OK;
  });
}

extern "C" mi_status mi_server_poll(mi_server *s, int64_t id, mi_request_state *out) {
  return guarded("mi_server_poll", [&]() -> mi_status {
  if (!s || !out) return fail(MI_E_INVALID, "mi_server_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->table.find(id);
  if (it == s->table.end()) return fail(MI_E_INVALID, "unknown request %lld", (long long)id);
  *out = it->second->st;
  return MI_OK;
  });
}

extern "C" mi_status mi_server_release(mi_server *s, int64_t id) {
  return guarded("mi_server_release", [&]() -> mi_status {
  if (!s) return fail(MI_E_INVALID, "mi_server_release: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->table.find(id);
  if (it == s->table.end()) return fail(MI_E_INVALID, "unknown request %lld", (long long)id);
  const int32_t state = it->second->st.state;
  if (state != MI_REQ_DONE && state != MI_REQ_FAILED)
    return fail(MI_E_INVALID, "request %lld is still queued or active", (long long)id);
  if (it->second->g) mi_grid_destroy(it->second->g);
  s->table.erase(it);
  return MI_OK;
  });
}

extern "C" mi_status mi_server_info(mi_server *s, size_t *heap_bytes, size_t *heap_free) {
  return guarded("mi_server_info", [&]() -> mi_status {
  if (!s) return fail(MI_E_INVALID, "mi_server_info: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (heap_bytes) *heap_bytes = (s->arena_bytes - s->step_bytes) & ~(size_t)255;
  if (heap_free) *heap_free = s->heap.free_bytes();
  return MI_OK;
  });
}

extern "C" void mi_server_destroy(mi_server *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (auto &kv : s->table) {
    Request *r = kv.second.get();
    if (r->ref) mi_ref_destroy(r->ref);
    if (r->g) mi_grid_destroy(r->g);
  }
  if (s->pinned) (void)hipHostFree(s->pinned);
  delete s;
}

// ----------------------------------------------------------- simplex search

namespace {

constexpr double kNmReflect = 1.0, kNmExpand = 2.0, kNmContract = 0.5, kNmShrink = 0.5;

// One Nelder-Mead simplex over the 6 pose parameters, minimising g = -MI.
// States: kInit needs the 7 vertices, kStep the 4 speculative candidates of
// an iteration (reflection, expansion, outside and inside contraction), kShrink
// the 6 shrunk vertices.
struct Simplex {
  enum State { kInit, kStep, kShrink, kDone };
  State state = kInit;
  double x[7][6];
  double g[7];
  double cand[6][6];   // points whose values are awaited
  int n_cand = 0;
  int32_t iters = 0;

  void order() {  // by value, ties by position (stable insertion sort)
    for (int i = 1; i < 7; ++i)
      for (int j = i; j > 0 && g[j] < g[j - 1]; --j) {
        std::swap(g[j], g[j - 1]);
        for (int a = 0; a < 6; ++a) std::swap(x[j][a], x[j - 1][a]);
      }
  }
  bool converged(const mi_nm_desc &d) const {
    double sx = 0.0, sf = 0.0;
    for (int k = 1; k < 7; ++k) {
      for (int a = 0; a < 6; ++a) sx = std::max(sx, std::fabs(x[k][a] - x[0][a]));
      sf = std::max(sf, std::fabs(g[k] - g[0]));
    }
    return sx <= d.xtol && sf <= d.ftol;
  }
  // after the vertices are ordered: stop, or set up the next iteration's candidates
  void next(const mi_nm_desc &d) {
    if (iters >= d.max_iter || converged(d)) { state = kDone; n_cand = 0; return; }
    ++iters;
    double c[6];
    for (int a = 0; a < 6; ++a) {
      double s = x[0][a];
      for (int k = 1; k < 6; ++k) s = s + x[k][a];
      c[a] = s / 6.0;
    }
    for (int a = 0; a < 6; ++a) {
      const double xr = c[a] + kNmReflect * (c[a] - x[6][a]);
      cand[0][a] = xr;
      cand[1][a] = c[a] + kNmExpand * (xr - c[a]);
      cand[2][a] = c[a] + kNmContract * (xr - c[a]);
      cand[3][a] = c[a] + kNmContract * (x[6][a] - c[a]);
    }
    state = kStep;
    n_cand = 4;
  }
  // values of the awaited points are in v[0 .. n_cand)
  void take(const double *v, const mi_nm_desc &d) {
    if (state == kInit) {
      for (int k = 0; k < 7; ++k) g[k] = v[k];
      order();
      next(d);
      return;
    }
    if (state == kShrink) {
      for (int k = 1; k < 7; ++k) {
        for (int a = 0; a < 6; ++a) x[k][a] = cand[k - 1][a];
        g[k] = v[k - 1];
      }
      order();
      next(d);
      return;
    }
    const double fr = v[0], fe = v[1], foc = v[2], fic = v[3];
    const double best = g[0], second = g[5], worst = g[6];
    int accept = -1;
    if (fr < best) accept = fe < fr ? 1 : 0;
    else if (fr < second) accept = 0;
    else if (fr < worst) { if (foc <= fr) accept = 2; }
    else if (fic < worst) accept = 3;
    if (accept >= 0) {
      for (int a = 0; a < 6; ++a) x[6][a] = cand[accept][a];
      g[6] = v[accept];
      order();
      next(d);
      return;
    }
    for (int k = 1; k < 7; ++k)
      for (int a = 0; a < 6; ++a) cand[k - 1][a] = x[0][a] + kNmShrink * (x[k][a] - x[0][a]);
    state = kShrink;
    n_cand = 6;
  }
};

bool nm_ok(const mi_nm_desc *d, int nf) {
  if (!d || d->max_iter < 0 || !slot_ok(d->feature_slot, d->weight, nf)) return false;
  if (!(d->ftol >= 0.0) || !(d->xtol >= 0.0)) return false;
  for (int a = 0; a < 6; ++a)
    if (!std::isfinite(d->step[a])) return false;
  return true;
}

}  // namespace

extern "C" size_t mi_align_nm_workspace(const mi_ref *r, int64_t n_b, int32_t n_starts) {
  return guarded_size([&]() -> size_t {
  if (!r || n_b < 0 || n_starts < 1) return 0;
  const int64_t K = 7 * (int64_t)n_starts;
  std::vector<double> P((size_t)K * 6, 0.0);
  for (int64_t k = 0; k < K; ++k) P[(size_t)k * 6 + 5] = 1e-3 * (double)k;  // distinct rotations
  mi_work_item w;
  memset(&w, 0, sizeof w);
  w.ref = r; w.n_b = n_b; w.poses = P.data(); w.K = K;
  // the simplex rounds use the stripe-bucketed per-pose form (no read-back of
  // scan B per round)
  BatchTables B;
  if (prepare_batch(&w, 1, MI_EVAL_PER_POSE, B) != MI_OK) return 0;
  const size_t b = batch_bytes(B, &w, 1, 0);
  return b + al256((size_t)r->g->gi.nf * (size_t)K * sizeof(double)) + 512;
  });
}

extern "C" mi_status mi_align_nelder_mead(const mi_ref *r, const float *xyz_b, int64_t n_b,
                                          const double *starts, int32_t n_starts,
                                          const mi_nm_desc *d, double pose_out[6],
                                          double *mi_best, int32_t *iters_out, void *ws,
                                          size_t ws_bytes, void *stream) {
  return guarded("mi_align_nelder_mead", [&]() -> mi_status {
  if (!r || !starts || !pose_out || n_starts < 1)
    return fail(MI_E_INVALID, "mi_align_nelder_mead: bad arguments");
  const GridInfo &gi = r->g->gi;
  if (!nm_ok(d, gi.nf)) return fail(MI_E_INVALID, "bad simplex description");
  if (n_b > 0 && !xyz_b) return fail(MI_E_INVALID, "xyz_b is NULL");
  for (int64_t k = 0; k < 6 * (int64_t)n_starts; ++k)
    if (!std::isfinite(starts[k])) return fail(MI_E_INVALID, "non-finite start pose");
  if (!ws || ((uintptr_t)ws & 255)) return fail(MI_E_WORKSPACE, "workspace NULL or not 256-aligned");
  const int64_t Kmax = 7 * (int64_t)n_starts;
  Carver c(ws, ws_bytes);
  double *mi_dev = c.take<double>((size_t)gi.nf * (size_t)Kmax);
  c.take<char>(0);
  if (!c.fits()) return fail(MI_E_WORKSPACE, "simplex workspace too small");
  void *plan_ws = (void *)c.cur;
  const size_t plan_room = ws_bytes - c.used();
  hipStream_t s = (hipStream_t)stream;
  std::vector<Simplex> sx((size_t)n_starts);
  for (int32_t i = 0; i < n_starts; ++i) {
    Simplex &S = sx[(size_t)i];
    for (int a = 0; a < 6; ++a) S.x[0][a] = starts[6 * i + a];
    for (int k = 1; k < 7; ++k) {
      for (int a = 0; a < 6; ++a) S.x[k][a] = S.x[0][a];
      S.x[k][k - 1] = S.x[k][k - 1] + d->step[k - 1];
    }
    for (int k = 0; k < 6; ++k)
      for (int a = 0; a < 6; ++a) S.cand[k][a] = 0.0;
  }
  std::vector<double> P, vals;
  std::vector<double> host_mi;
  for (;;) {
    // every active simplex's awaited points, in start order, as one batch
    P.clear();
    for (Simplex &S : sx) {
      if (S.state == Simplex::kDone) continue;
      if (S.state == Simplex::kInit)
        for (int k = 0; k < 7; ++k) P.insert(P.end(), S.x[k], S.x[k] + 6);
      else
        for (int k = 0; k < S.n_cand; ++k) P.insert(P.end(), S.cand[k], S.cand[k] + 6);
    }
    const int64_t K = (int64_t)(P.size() / 6);
    if (K == 0) break;
    mi_work_item w;
    memset(&w, 0, sizeof w);
    w.ref = r; w.xyz_b = xyz_b; w.n_b = n_b; w.poses = P.data(); w.K = K; w.mi_out = mi_dev;
    mi_plan *p = nullptr;
    mi_status st = create_plan(&w, 1, MI_EVAL_PER_POSE, plan_ws, plan_room, 0, stream, false, &p);
    if (st != MI_OK) return st;
    st = run_plan(p, s);
    mi_plan_destroy(p);
    if (st != MI_OK) return st;
    const bool weighted = d->feature_slot == MI_SLOT_WEIGHTED;
    const int rows = weighted ? gi.nf : 1;
    host_mi.resize((size_t)rows * (size_t)K);
    HIP_TRY(hipMemcpyAsync(host_mi.data(), mi_dev + (weighted ? 0 : (int64_t)d->feature_slot * K),
                           sizeof(double) * (size_t)rows * (size_t)K, hipMemcpyDeviceToHost, s),
            "MI D2H");
    HIP_TRY(hipStreamSynchronize(s), "simplex round sync");
    vals.resize((size_t)K);
    for (int64_t k = 0; k < K; ++k) {
      double v = host_mi[(size_t)k];
      if (weighted) {
        // the weighted objective: each product rounded, then the sum
        v = d->weight[0] * host_mi[(size_t)k];
        if (gi.nf > 1) v = v + d->weight[1] * host_mi[(size_t)K + (size_t)k];
      }
      vals[(size_t)k] = -v;
    }
    size_t off = 0;
    for (Simplex &S : sx) {
      if (S.state == Simplex::kDone) continue;
      const int need = S.state == Simplex::kInit ? 7 : S.n_cand;
      S.take(vals.data() + off, *d);
      off += (size_t)need;
    }
  }
  // the best simplex result; ties go to the earlier start
  int32_t bi = 0;
  for (int32_t i = 1; i < n_starts; ++i)
    if (sx[(size_t)i].g[0] < sx[(size_t)bi].g[0]) bi = i;
  for (int a = 0; a < 6; ++a) pose_out[a] = sx[(size_t)bi].x[0][a];
  if (mi_best) *mi_best = -sx[(size_t)bi].g[0];
  if (iters_out)
    for (int32_t i = 0; i < n_starts; ++i) iters_out[i] = sx[(size_t)i].iters;
  return MI_OK;
  });
}
