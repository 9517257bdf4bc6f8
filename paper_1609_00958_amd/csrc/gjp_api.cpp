// gjp_api.cpp -- C ABI of the generalized Joseph projector (see include/gjp.h).
//
// Host responsibilities: argument validation, world -> grid conversion of the
// view vectors (double precision, no contraction), per-view detector
// projection rows for the adjoint's candidate search, stream-ordered scratch
// (zero-padded volume copies, adjoint ray tables), the forward tile
// autotuner, kernel timing for benchmarks, and the batched plan (work list,
// device queue, HIP graph).
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <set>
#include <sstream>
#include <unistd.h>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gjp.h"
#include "gjp_internal.h"

using gjp::BatchInst;
using gjp::FwdArgs;
using gjp::FwdTile;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int gjp::set_error(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

static gjp_status fail(gjp_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

static gjp_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? GJP_ENOMEM : GJP_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define GJP_HIP(call, what)                    \
  do {                                         \
    hipError_t _e = (call);                    \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

extern "C" const char* gjp_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
namespace {
struct TimingState {
  std::mutex mu;
  bool on = false;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::map<std::string, std::pair<double, int64_t>> total;
};
TimingState& timing() {
  static TimingState* t = new TimingState();
  return *t;
}
}  // namespace

gjp::TimedLaunch gjp::timing_begin(const char* name, hipStream_t s) {
  (void)name;
  TimedLaunch t;
  TimingState& T = timing();
  {
    std::lock_guard<std::mutex> lk(T.mu);
    if (!T.on) return t;
  }
  if (hipEventCreate(&t.start) != hipSuccess) return t;
  if (hipEventCreate(&t.stop) != hipSuccess) {
    (void)hipEventDestroy(t.start);
    t.start = nullptr;
    return t;
  }
  if (hipEventRecord(t.start, s) != hipSuccess) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
    t.start = t.stop = nullptr;
    return t;
  }
  t.on = true;
  return t;
}

void gjp::timing_end(const char* name, TimedLaunch& t, hipStream_t s) {
  if (!t.on) return;
  (void)hipEventRecord(t.stop, s);
  TimingState& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  T.pending[name].push_back({t.start, t.stop});
}

extern "C" gjp_status gjp_timing_enable(int32_t on) {
  TimingState& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  T.on = (on != 0);
  return GJP_OK;
}

extern "C" gjp_status gjp_timing_reset(void) {
  TimingState& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  for (auto& kv : T.pending)
    for (auto& ev : kv.second) {
      (void)hipEventSynchronize(ev.second);
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  T.pending.clear();
  T.total.clear();
  return GJP_OK;
}

extern "C" gjp_status gjp_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return fail(GJP_EINVAL, "gjp_timing_read: null pointer");
  TimingState& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  auto it = T.pending.find(kernel);
  if (it != T.pending.end()) {
    for (auto& ev : it->second) {
      GJP_HIP(hipEventSynchronize(ev.second), "timing event");
      float ms = 0.0f;
      GJP_HIP(hipEventElapsedTime(&ms, ev.first, ev.second), "timing elapsed");
      auto& tot = T.total[kernel];
      tot.first += ms;
      tot.second += 1;
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    it->second.clear();
  }
  auto jt = T.total.find(kernel);
  *total_ms = (jt == T.total.end()) ? 0.0 : jt->second.first;
  *launches = (jt == T.total.end()) ? 0 : jt->second.second;
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// trajectories
// ---------------------------------------------------------------------------
static const double kPi = 3.14159265358979323846;

extern "C" gjp_status gjp_views_circular_cone(int32_t n_views, double sod, double sdd,
                                              double pitch_u, double pitch_v, int32_t n_u,
                                              int32_t n_v, double* out) {
  if (n_views <= 0 || n_u <= 0 || n_v <= 0 || !out)
    return fail(GJP_EINVAL, "gjp_views_circular_cone: non-positive size or null output");
  if (!isfinite(sod) || !isfinite(sdd) || !isfinite(pitch_u) || !isfinite(pitch_v))
    return fail(GJP_EINVAL, "gjp_views_circular_cone: non-finite parameter");
  for (int k = 0; k < n_views; ++k) {
    const double th = 2.0 * kPi * (double)k / (double)n_views;
    const double c = cos(th), s = sin(th);
    double* o = out + 12 * (size_t)k;
    const double src[3] = {sod * c, sod * s, 0.0};
    const double dc[3] = {(sod - sdd) * c, (sod - sdd) * s, 0.0};
    const double du[3] = {-pitch_u * s, pitch_u * c, 0.0};
    const double dv[3] = {0.0, 0.0, pitch_v};
    const double hu = 0.5 * (double)(n_u - 1), hv = 0.5 * (double)(n_v - 1);
    for (int j = 0; j < 3; ++j) {
      o[0 + j] = src[j];
      o[3 + j] = dc[j] - hu * du[j] - hv * dv[j];
      o[6 + j] = du[j];
      o[9 + j] = dv[j];
    }
  }
  return GJP_OK;
}

extern "C" gjp_status gjp_views_parallel(int32_t n_views, double pitch_u, double pitch_v,
                                         int32_t n_u, int32_t n_v, double* out) {
  if (n_views <= 0 || n_u <= 0 || n_v <= 0 || !out)
    return fail(GJP_EINVAL, "gjp_views_parallel: non-positive size or null output");
  if (!isfinite(pitch_u) || !isfinite(pitch_v))
    return fail(GJP_EINVAL, "gjp_views_parallel: non-finite parameter");
  for (int k = 0; k < n_views; ++k) {
    const double th = 2.0 * kPi * (double)k / (double)n_views;
    const double c = cos(th), s = sin(th);
    double* o = out + 12 * (size_t)k;
    const double dir[3] = {-c, -s, 0.0};
    const double du[3] = {-pitch_u * s, pitch_u * c, 0.0};
    const double dv[3] = {0.0, 0.0, pitch_v};
    const double hu = 0.5 * (double)(n_u - 1), hv = 0.5 * (double)(n_v - 1);
    for (int j = 0; j < 3; ++j) {
      o[0 + j] = dir[j];
      o[3 + j] = 0.0 - hu * du[j] - hv * dv[j];
      o[6 + j] = du[j];
      o[9 + j] = dv[j];
    }
  }
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static std::atomic<uint64_t> g_next_id{1};

static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Rows (u, v, w) mapping a grid point q to homogeneous detector coordinates
// (continuous pixel indices): u = (A_u.q + b_u) / (A_w.q + b_w), w > 0 in
// front of the source. Used only to bound the adjoint's candidate rays.
static void detector_projection(const double* v, int beam, float* P) {
  const double* o = v + 3;
  const double* du = v + 6;
  const double* dv = v + 9;
  double n[3], t1[3], t2[3], eu[3], ev[3];
  cross3(du, dv, n);
  cross3(dv, n, t1);
  cross3(n, du, t2);
  const double su = dot3(du, t1), sv = dot3(dv, t2);
  for (int k = 0; k < 3; ++k) {
    eu[k] = (su != 0.0) ? t1[k] / su : 0.0;
    ev[k] = (sv != 0.0) ? t2[k] / sv : 0.0;
  }
  double R[12];
  if (beam == gjp::BEAM_CONE) {
    const double* s = v;
    double som[3] = {s[0] - o[0], s[1] - o[1], s[2] - o[2]};
    const double K = -dot3(n, som);  // n.(o - s)
    const double ns = dot3(n, s);
    const double eus = dot3(eu, som), evs = dot3(ev, som);
    for (int k = 0; k < 3; ++k) {
      R[k] = eus * n[k] + K * eu[k];
      R[4 + k] = evs * n[k] + K * ev[k];
      R[8 + k] = n[k];
    }
    R[3] = -eus * ns - K * dot3(eu, s);
    R[7] = -evs * ns - K * dot3(ev, s);
    R[11] = -ns;
    if (K < 0.0)
      for (int k = 0; k < 12; ++k) R[k] = -R[k];
  } else {
    const double* r = v;
    const double nr = dot3(n, r);
    const double au = (nr != 0.0) ? dot3(eu, r) / nr : 0.0;
    const double av = (nr != 0.0) ? dot3(ev, r) / nr : 0.0;
    const double no = dot3(n, o);
    for (int k = 0; k < 3; ++k) {
      R[k] = eu[k] - au * n[k];
      R[4 + k] = ev[k] - av * n[k];
      R[8 + k] = 0.0;
    }
    R[3] = -dot3(eu, o) + au * no;
    R[7] = -dot3(ev, o) + av * no;
    R[11] = 1.0;
  }
  for (int k = 0; k < 12; ++k) P[k] = (float)R[k];
}

// True when, in every view, dv has no component on axes 0 and 1 and no ray is
// driven by axis 2 (|r_2| stays below max(|r_0|, |r_1|) with a safety
// factor). Then d_0, d_1, r_0, r_1 and the source do not depend on iv, so the
// ray setup of all rays of a detector column yields the same driving axis and
// in-plane coefficients, bit for bit.
static bool columns_share_inplane_setup(const gjp_geometry& g) {
  for (int v = 0; v < g.n_views; ++v) {
    const double* o = g.views_grid.data() + 12 * (size_t)v;
    if (o[9] != 0.0 || o[10] != 0.0) return false;
    if (g.beam == GJP_PARALLEL) {
      if (!(fabs(o[2]) * (1.0 + 1e-9) < fmax(fabs(o[0]), fabs(o[1])))) return false;
      continue;
    }
    for (int iu = 0; iu < g.n_u; ++iu) {
      const double d0 = o[3] + (double)iu * o[6];
      const double d1 = o[4] + (double)iu * o[7];
      const double r0 = d0 - o[0], r1 = d1 - o[1];
      const double M = fmax(fabs(r0), fabs(r1));
      const double z0 = o[5] + (double)iu * o[8] - o[2];
      const double z1 = o[5] + (double)iu * o[8] + (double)(g.n_v - 1) * o[11] - o[2];
      if (!(fmax(fabs(z0), fabs(z1)) * (1.0 + 1e-9) < M)) return false;
    }
  }
  return true;
}

extern "C" gjp_status gjp_create_geometry(const gjp_geometry_desc* d, gjp_geometry** out) {
  if (!d || !out) return fail(GJP_EINVAL, "gjp_create_geometry: null pointer");
  *out = nullptr;
  for (int k = 0; k < 3; ++k) {
    if (d->vol_shape[k] <= 0 || d->vol_shape[k] > 32767)
      return fail(GJP_EINVAL, "gjp_create_geometry: vol_shape must be in [1, 32767]");
    if (!(d->voxel_size[k] > 0.0) || !isfinite(d->voxel_size[k]))
      return fail(GJP_EINVAL, "gjp_create_geometry: voxel_size must be positive and finite");
    if (!isfinite(d->vol_center[k]))
      return fail(GJP_EINVAL, "gjp_create_geometry: vol_center must be finite");
  }
  if (d->n_views <= 0 || d->n_u <= 0 || d->n_v <= 0)
    return fail(GJP_EINVAL, "gjp_create_geometry: n_views, n_u and n_v must be positive");
  if (d->beam != GJP_CONE && d->beam != GJP_PARALLEL)
    return fail(GJP_EINVAL, "gjp_create_geometry: unknown beam");
  if (d->weight != GJP_W_LINEAR && d->weight != GJP_W_SPLINE)
    return fail(GJP_EINVAL, "gjp_create_geometry: unknown weight function");
  if ((d->flags & ~GJP_CLIP_CYLINDER) != 0)
    return fail(GJP_EINVAL, "gjp_create_geometry: unknown flags");
  if (!d->views) return fail(GJP_EINVAL, "gjp_create_geometry: views is null");
  const size_t nv = (size_t)d->n_views;
  if ((unsigned long long)d->n_views * d->n_u * d->n_v > (1ull << 46))
    return fail(GJP_EINVAL, "gjp_create_geometry: sinogram too large");
  for (size_t i = 0; i < 12 * nv; ++i)
    if (!isfinite(d->views[i])) return fail(GJP_EINVAL, "gjp_create_geometry: non-finite view");
  if (d->n_views >= (1 << 20))
    return fail(GJP_EINVAL, "gjp_create_geometry: at most 2^20 - 1 views");

  std::unique_ptr<gjp_geometry> g;
  try {
    g.reset(new gjp_geometry());
    g->views_world.assign(d->views, d->views + 12 * nv);
    g->views_grid.resize(12 * nv);
    g->proj.resize(12 * nv);
  } catch (...) {
    return fail(GJP_ENOMEM, "gjp_create_geometry: host allocation failed");
  }
  g->id = g_next_id.fetch_add(1);
  for (int k = 0; k < 3; ++k) {
    g->n[k] = d->vol_shape[k];
    g->vs[k] = d->voxel_size[k];
    g->ctr[k] = d->vol_center[k];
    g->gg.n[k] = d->vol_shape[k];
    g->gg.vs[k] = d->voxel_size[k];
    uint32_t bits;
    const float fn = (float)d->vol_shape[k];
    memcpy(&bits, &fn, 4);
    bits -= 1;  // largest float below n_k (n_k >= 1)
    memcpy(&g->gg.hi[k], &bits, 4);
  }
  g->gg.beam = d->beam;
  g->gg.clip = (d->flags & GJP_CLIP_CYLINDER) ? 1 : 0;
  g->gg.cyl[0] = 0.5 * (double)(g->gg.n[0] - 1);
  g->gg.cyl[1] = 0.5 * (double)(g->gg.n[1] - 1);
  {
    const double rad = 0.5 * (double)(g->gg.n[0] < g->gg.n[1] ? g->gg.n[0] : g->gg.n[1]);
    g->gg.cyl_r2 = rad * rad;
  }
  g->n_views = d->n_views;
  g->n_u = d->n_u;
  g->n_v = d->n_v;
  g->beam = d->beam;
  g->weight = d->weight;
  for (size_t v = 0; v < nv; ++v) {
    const double* w = d->views + 12 * v;
    double* o = g->views_grid.data() + 12 * v;
    for (int k = 0; k < 3; ++k) {
      // points -> grid: (w - c) / h + (n - 1) / 2 ; directions -> grid: w / h
      if (d->beam == GJP_CONE)
        o[k] = (w[k] - g->ctr[k]) / g->vs[k] + (double)(g->n[k] - 1) * 0.5;
      else
        o[k] = w[k] / g->vs[k];
      o[3 + k] = (w[3 + k] - g->ctr[k]) / g->vs[k] + (double)(g->n[k] - 1) * 0.5;
      o[6 + k] = w[6 + k] / g->vs[k];
      o[9 + k] = w[9 + k] / g->vs[k];
    }
    detector_projection(o, d->beam, g->proj.data() + 12 * v);
  }
  g->separable = columns_share_inplane_setup(*g);
  *out = g.release();
  return GJP_OK;
}

static void invalidate_plans(uint64_t id);

extern "C" gjp_status gjp_destroy_geometry(gjp_geometry* g) {
  if (!g) return GJP_OK;
  invalidate_plans(g->id);
  bool on_device = false;
  for (int dvc = 0; dvc < gjp_geometry::kMaxDev; ++dvc) on_device |= (g->dev[dvc].views != nullptr);
  if (on_device) {  // no HIP call at all for a geometry that never reached a device
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (int dvc = 0; dvc < gjp_geometry::kMaxDev; ++dvc) {
      if (!g->dev[dvc].views) continue;
      (void)hipSetDevice(dvc);
      (void)hipFree(g->dev[dvc].views);
      (void)hipFree(g->dev[dvc].proj);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  delete g;
  return GJP_OK;
}

int gjp::geometry_device_existing(const gjp_geometry* g, const double** views,
                                  const float** proj) {
  int dvc = 0;
  hipError_t e = hipGetDevice(&dvc);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dvc < 0 || dvc >= gjp_geometry::kMaxDev) return fail(GJP_EUNSUPPORTED, "device index");
  std::lock_guard<std::mutex> lk(g->mu);
  const gjp_geometry::Dev& D = g->dev[dvc];
  if (!D.views)
    return fail(GJP_EINVAL,
                "the geometry has no copy on this device yet: any other projection call on "
                "this device makes it");
  *views = D.views;
  *proj = D.proj;
  return GJP_OK;
}

int gjp::geometry_device(const gjp_geometry* g, const double** views, const float** proj) {
  int dvc = 0;
  hipError_t e = hipGetDevice(&dvc);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dvc < 0 || dvc >= gjp_geometry::kMaxDev) return fail(GJP_EUNSUPPORTED, "device index");
  std::lock_guard<std::mutex> lk(g->mu);
  gjp_geometry::Dev& D = g->dev[dvc];
  if (!D.views) {
    const size_t nb = g->views_grid.size() * sizeof(double);
    const size_t pb = g->proj.size() * sizeof(float);
    double* dv = nullptr;
    float* dp = nullptr;
    e = hipMalloc(&dv, nb);
    if (e != hipSuccess) return hip_fail(e, "geometry upload (views)");
    e = hipMalloc(&dp, pb);
    if (e != hipSuccess) {
      (void)hipFree(dv);
      return hip_fail(e, "geometry upload (projection)");
    }
    e = hipMemcpy(dv, g->views_grid.data(), nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dp, g->proj.data(), pb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dv);
      (void)hipFree(dp);
      return hip_fail(e, "geometry upload (copy)");
    }
    D.views = dv;
    D.proj = dp;
  }
  *views = D.views;
  *proj = D.proj;
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// sample count (host, same double-precision setup as the kernels)
// ---------------------------------------------------------------------------
extern "C" gjp_status gjp_sart_residual(int64_t n, const float* d_b, const float* d_ax,
                                        const float* d_row_sum, float* d_out, void* stream) {
  if (n < 0) return fail(GJP_EINVAL, "sart_residual: negative size");
  if (n > 0 && (!d_b || !d_ax || !d_row_sum || !d_out))
    return fail(GJP_EINVAL, "sart_residual: null device pointer");
  return (gjp_status)gjp::launch_sart_residual(n, d_b, d_ax, d_row_sum, d_out,
                                               (hipStream_t)stream);
}

extern "C" gjp_status gjp_sart_update(int64_t n, float* d_x, const float* d_bp,
                                      const float* d_col_sum, float lam, int32_t nonneg,
                                      void* stream) {
  if (n < 0) return fail(GJP_EINVAL, "sart_update: negative size");
  if (n > 0 && (!d_x || !d_bp || !d_col_sum))
    return fail(GJP_EINVAL, "sart_update: null device pointer");
  if (!std::isfinite(lam)) return fail(GJP_EINVAL, "sart_update: non-finite relaxation");
  return (gjp_status)gjp::launch_sart_update(n, d_x, d_bp, d_col_sum, lam, nonneg ? 1 : 0,
                                             (hipStream_t)stream);
}

extern "C" gjp_status gjp_count_samples(const gjp_geometry* g, uint64_t* out) {
  if (!g || !out) return fail(GJP_EINVAL, "gjp_count_samples: null pointer");
  const long long n_rays = (long long)g->n_views * g->n_u * g->n_v;
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 64) nt = 64;
  if (n_rays < 65536) nt = 1;
  std::vector<uint64_t> part(nt, 0);
  auto work = [&](unsigned t) {
    uint64_t acc = 0;
    const long long per_view = (long long)g->n_u * g->n_v;
    for (long long r = t; r < n_rays; r += nt) {
      const int view = (int)(r / per_view);
      const long long rem = r - (long long)view * per_view;
      gjp::RaySetup R;
      gjp::ray_setup(g->views_grid.data() + 12 * (size_t)view, g->gg, (int)(rem / g->n_v),
                     (int)(rem % g->n_v), R);
      acc += (uint64_t)(R.i1 - R.i0);
    }
    part[t] = acc;
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  uint64_t total = 0;
  for (auto p : part) total += p;
  *out = total;
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// stream-ordered scratch
// ---------------------------------------------------------------------------
static std::once_flag g_pool_once[gjp_geometry::kMaxDev];

// The stream-ordered pool keeps up to this many freed bytes for reuse (the
// padded copies of repeated 512^3 forwards, the adjoint's ray tables); larger
// scratch, such as the padded copies of a 2048^3 volume, goes back to the
// device at the next synchronisation instead of staying cached beside the
// caller's own allocator.
static const uint64_t kPoolKeepBytes = (uint64_t)8 << 30;

static void keep_pool_memory(int dvc) {
  if (dvc < 0 || dvc >= gjp_geometry::kMaxDev) return;
  std::call_once(g_pool_once[dvc], [dvc]() {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dvc) == hipSuccess) {
      uint64_t thr = kPoolKeepBytes;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

// Blocks that came from hipMalloc because the pool refused them: freed after
// a stream synchronisation instead of in stream order.
static std::mutex g_direct_mu;
static std::set<void*> g_direct;

static hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s) {
  int dvc = 0;
  (void)hipGetDevice(&dvc);
  keep_pool_memory(dvc);
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipErrorOutOfMemory) return e;
  // The pool could not serve the block (seen for single blocks of a hundred
  // GiB and more while the device had room): return its cached memory and
  // try again, then take the block from the device directly.
  (void)hipGetLastError();
  hipMemPool_t pool;
  if (hipStreamSynchronize(s) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dvc) == hipSuccess)
    (void)hipMemPoolTrimTo(pool, 0);
  e = hipMallocAsync(p, bytes, s);
  if (e == hipSuccess) return e;
  (void)hipGetLastError();
  e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  std::lock_guard<std::mutex> lk(g_direct_mu);
  g_direct.insert(*p);
  return hipSuccess;
}

static hipError_t scratch_free(void* p, hipStream_t s) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_direct_mu);
    auto it = g_direct.find(p);
    if (it != g_direct.end()) {
      g_direct.erase(it);
      const hipError_t e = hipStreamSynchronize(s);
      const hipError_t f = hipFree(p);
      return e != hipSuccess ? e : f;
    }
  }
  return hipFreeAsync(p, s);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
namespace {
// Launch configurations of the forward by shape signature and dtype: set in
// this process (autotuner, gjp_set_forward_tile), else read from the on-disk
// cache named by GJP_TUNE_CACHE for the current device, else the default.
std::mutex g_tune_mu;
std::map<std::string, FwdTile> g_tune;                 // this process
std::map<std::string, FwdTile> g_disk;                 // device tag + key -> entry
std::set<std::string> g_disk_loaded;                   // device tags read from disk

std::string tune_key(const gjp_geometry* g, int dtype) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%d,%d,%d|%d,%d,%d|%d,%d,%d", g->n[0], g->n[1], g->n[2],
           g->n_views, g->n_u, g->n_v, g->beam, g->weight, dtype);
  return buf;
}

const char* tune_cache_path() {
  const char* p = getenv("GJP_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// Architecture name and compute-unit count of the current device ("" if there
// is none): cache entries measured on one kind of device are not used on
// another.
std::string device_tag() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return "";
  static std::mutex mu;
  static std::map<int, std::string> tags;
  std::lock_guard<std::mutex> lk(mu);
  auto it = tags.find(d);
  if (it != tags.end()) return it->second;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, d) != hipSuccess) return "";
  std::string tag = std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount) + "cu";
  for (char& c : tag)
    if (c == ' ' || c == '\t') c = '_';
  tags[d] = tag;
  return tag;
}

// Cache file: one entry per line, "<device> <key> <tile_v_log2> <view_group>
// <load_group>"; lines that do not parse are ignored.
bool parse_entry(const std::string& line, std::string& dev, std::string& key, FwdTile& t) {
  std::istringstream in(line);
  int k = 0, vg = 0, rg = 0;
  if (!(in >> dev >> key >> k >> vg >> rg)) return false;
  if (k < 4 || k > 8 || vg < 1 || vg > 64 || (rg != 2 && rg != 4)) return false;
  t = FwdTile();
  t.tile_v_log2 = k;
  t.view_group = vg;
  t.ru_group = rg;
  return true;
}

// Reads the cache's entries for `dev` once per device (caller holds g_tune_mu).
void disk_load(const std::string& dev) {
  if (dev.empty() || g_disk_loaded.count(dev)) return;
  g_disk_loaded.insert(dev);
  const char* path = tune_cache_path();
  if (!path) return;
  std::ifstream f(path);
  std::string line, d, key;
  FwdTile t;
  while (std::getline(f, line))
    if (parse_entry(line, d, key, t) && d == dev) g_disk[d + " " + key] = t;
}

// Adds or replaces one entry in the cache file (written to a temporary file
// and renamed over the old one). Failures leave the file as it was; the
// choice still applies in this process.
void disk_store(const std::string& dev, const std::string& key, const FwdTile& t) {
  const char* path = tune_cache_path();
  if (!path || dev.empty()) return;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line, d, k;
    FwdTile o;
    while (std::getline(f, line)) {
      if (parse_entry(line, d, k, o) && d == dev && k == key) continue;
      if (!line.empty()) lines.push_back(line);
    }
  }
  char buf[512];
  snprintf(buf, sizeof(buf), "%s %s %d %d %d", dev.c_str(), key.c_str(), t.tile_v_log2,
           t.view_group, t.ru_group);
  lines.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return;
    for (const auto& l : lines) f << l << "\n";
    if (!f.good()) {
      f.close();
      (void)remove(tmp.c_str());
      return;
    }
  }
  if (rename(tmp.c_str(), path) != 0) (void)remove(tmp.c_str());
  g_disk[dev + " " + key] = t;
}

FwdTile tile_for(const gjp_geometry* g, int dtype) {
  const std::string key = tune_key(g, dtype);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it != g_tune.end()) return it->second;
  if (tune_cache_path()) {
    const std::string dev = device_tag();
    disk_load(dev);
    auto jt = g_disk.find(dev + " " + key);
    if (jt != g_disk.end()) return jt->second;
  }
  return FwdTile();
}

long long padded_elems(const int* n) {
  return (long long)(n[0] + 2) * (long long)(n[1] + 2) * gjp::padded_pitch(n[2]);
}

void fill_fwd_args(const gjp_geometry* g, const double* d_views, const void* padded,
                   float* sino, const FwdTile& tile, FwdArgs& a) {
  (void)padded;
  const long long p2 = gjp::padded_pitch(g->n[2]), p1 = g->n[1] + 2;
  a.S1 = p2;
  a.S0 = p1 * p2;
  a.G = g->gg;
  a.views = d_views;
  a.sino = sino;
  a.n_u = g->n_u;
  a.n_v = g->n_v;
  a.tile_v_log2 = tile.tile_v_log2;
  a.remap = tile.remap;
  a.view_group = tile.view_group < 1 ? 1 : tile.view_group;
  a.ru_group = tile.ru_group == 2 ? 2 : 4;
  a.n_views = g->n_views;
  // k = 7: 128 pixels along v per wavefront row (two per lane), four rows;
  // k = 8: 192 pixels (three per lane), four rows
  const int tile_v = gjp::tile_v_pixels(tile.tile_v_log2);
  const int tile_u = gjp::tile_u_columns(tile.tile_v_log2);
  a.tiles_v = (g->n_v + tile_v - 1) / tile_v;
  a.tiles_u = (g->n_u + tile_u - 1) / tile_u;
  a.tiles_per_view = a.tiles_v * a.tiles_u;
}

// Bytes of one pair copy (two values per padded element), rounded up so that
// copy B starts 256-byte aligned after copy A.
unsigned long long copy_bytes(const int* n, int dtype) {
  const unsigned long long b =
      (unsigned long long)padded_elems(n) * 2ull * gjp::dtype_size(dtype);
  return (b + 255ull) & ~255ull;
}

// The per-lane sampling loop addresses both pair copies with 32-bit offsets
// and 24-bit row multiplies; larger copies take 64-bit pointer arithmetic.
bool needs_idx64(const int* n, int dtype) {
  const unsigned long long pe = 2ull * gjp::dtype_size(dtype);
  const unsigned long long s0 = (unsigned long long)(n[1] + 2) * gjp::padded_pitch(n[2]) * pe;
  return 2 * copy_bytes(n, dtype) >= (1ull << 32) || s0 >= (1ull << 23);
}

// The row-uniform loop addresses one block of 64 planes and 66 rows with
// 32-bit offsets from its base, whichever axis drives.
bool block_fits_32bit(const int* n, int dtype) {
  const unsigned long long pe = 2ull * gjp::dtype_size(dtype);
  const unsigned long long s1 = (unsigned long long)gjp::padded_pitch(n[2]) * pe;
  const unsigned long long s0 = (unsigned long long)(n[1] + 2) * s1;
  return 66ull * (s0 + s1) < (1ull << 32);
}

void set_padded(FwdArgs& a, void* copies, int dtype, const int* n) {
  a.copy_bytes = copy_bytes(n, dtype);
  a.vol_a = copies;
  a.vol_b = static_cast<const char*>(copies) + a.copy_bytes;
}

gjp_status validate_fwd(const gjp_geometry* g, const void* d_vol, int32_t dtype,
                        const float* d_sino) {
  if (!g) return fail(GJP_EINVAL, "forward: geometry is null");
  if (!d_vol || !d_sino) return fail(GJP_EINVAL, "forward: null device pointer");
  if (dtype != GJP_F32 && dtype != GJP_BF16 && dtype != GJP_F16)
    return fail(GJP_EINVAL, "forward: unknown volume dtype");
  if (((uintptr_t)d_vol) % gjp::dtype_size(dtype) != 0 || ((uintptr_t)d_sino) % 4 != 0)
    return fail(GJP_EINVAL, "forward: misaligned pointer");
  return GJP_OK;
}

// Pad into `padded` (2 * copy_bytes) and project: the forward's launches.
int forward_into(const gjp_geometry* g, const double* d_views, const void* d_vol, int dtype,
                 float* d_sino, void* padded, hipStream_t s, const FwdTile& tile) {
  FwdArgs a;
  fill_fwd_args(g, d_views, nullptr, d_sino, tile, a);
  set_padded(a, padded, dtype, g->n);
  int st = gjp::launch_pad(d_vol, const_cast<void*>(a.vol_a), const_cast<void*>(a.vol_b), dtype,
                           g->n, s);
  if (st == GJP_OK)
    st = gjp::launch_forward(a, dtype, g->weight, needs_idx64(g->n, dtype), g->n_views, s);
  return st;
}

gjp_status forward_with_tile(const gjp_geometry* g, const void* d_vol, int32_t dtype,
                             float* d_sino, hipStream_t s, const FwdTile& tile) {
  const double* d_views = nullptr;
  const float* d_proj = nullptr;
  int st = gjp::geometry_device(g, &d_views, &d_proj);
  if (st != GJP_OK) return (gjp_status)st;
  if (!block_fits_32bit(g->n, dtype))
    return fail(GJP_EUNSUPPORTED, "forward: volume planes too large for 32-bit block offsets");
  void* padded = nullptr;
  GJP_HIP(scratch_alloc(&padded, (size_t)(2 * copy_bytes(g->n, dtype)), s),
          "forward: padded pair copies");
  st = forward_into(g, d_views, d_vol, dtype, d_sino, padded, s, tile);
  const hipError_t fe = scratch_free(padded, s);
  if (st != GJP_OK) return (gjp_status)st;
  if (fe != hipSuccess) return hip_fail(fe, "forward: free padded volume");
  return GJP_OK;
}
}  // namespace

extern "C" gjp_status gjp_forward_project(const gjp_geometry* g, const void* d_vol,
                                          int32_t vol_dtype, float* d_sino, void* stream) {
  gjp_status st = validate_fwd(g, d_vol, vol_dtype, d_sino);
  if (st != GJP_OK) return st;
  return forward_with_tile(g, d_vol, vol_dtype, d_sino, (hipStream_t)stream,
                           tile_for(g, vol_dtype));
}

extern "C" gjp_status gjp_forward_project_noalloc(const gjp_geometry* g, const void* d_vol,
                                                  int32_t vol_dtype, float* d_sino, void* stream) {
  gjp_status st = validate_fwd(g, d_vol, vol_dtype, d_sino);
  if (st != GJP_OK) return st;
  const unsigned long long need = 2 * copy_bytes(g->n, vol_dtype);
  if (need > gjp::kNoAllocScratchBytes)
    return fail(GJP_EINVAL, "forward_noalloc: the padded pair copies need " +
                                std::to_string(need) + " bytes, above the fixed scratch of " +
                                std::to_string(gjp::kNoAllocScratchBytes) + " bytes");
  const double* d_views = nullptr;
  const float* d_proj = nullptr;
  int r = gjp::geometry_device_existing(g, &d_views, &d_proj);
  if (r != GJP_OK) return (gjp_status)r;
  void* padded = nullptr;
  r = gjp::noalloc_scratch(&padded);
  if (r != GJP_OK) return (gjp_status)r;
  return (gjp_status)forward_into(g, d_views, d_vol, vol_dtype, d_sino, padded,
                                  (hipStream_t)stream, tile_for(g, vol_dtype));
}

extern "C" gjp_status gjp_forward_project_naive(const gjp_geometry* g, const void* d_vol,
                                                int32_t vol_dtype, float* d_sino, void* stream) {
  gjp_status st = validate_fwd(g, d_vol, vol_dtype, d_sino);
  if (st != GJP_OK) return st;
  const double* d_views = nullptr;
  const float* d_proj = nullptr;
  int r = gjp::geometry_device(g, &d_views, &d_proj);
  if (r != GJP_OK) return (gjp_status)r;
  return (gjp_status)gjp::launch_forward_naive(g->gg, d_views, d_vol, vol_dtype, g->weight,
                                               g->n_views, g->n_u, g->n_v, d_sino,
                                               (hipStream_t)stream);
}

extern "C" gjp_status gjp_autotune_forward(const gjp_geometry* g, const void* d_vol,
                                           int32_t vol_dtype, float* d_sino, void* stream,
                                           int32_t* tile_v_out) {
  gjp_status st = validate_fwd(g, d_vol, vol_dtype, d_sino);
  if (st != GJP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  GJP_HIP(hipEventCreate(&e0), "autotune event");
  GJP_HIP(hipEventCreate(&e1), "autotune event");
  FwdTile best;
  float best_ms = 3.0e38f;
  // time one candidate: a warm-up call, then three timed calls
  auto trial = [&](const FwdTile& t) -> gjp_status {
    gjp_status r = forward_with_tile(g, d_vol, vol_dtype, d_sino, s, t);  // warm-up
    if (r != GJP_OK) return r;
    hipError_t he = hipEventRecord(e0, s);
    const int reps = 3;
    for (int i = 0; i < reps && r == GJP_OK && he == hipSuccess; ++i)
      r = forward_with_tile(g, d_vol, vol_dtype, d_sino, s, t);
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (r != GJP_OK) return r;
    if (he != hipSuccess) return hip_fail(he, "autotune timing");
    float ms = 0.0f;
    he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) return hip_fail(he, "autotune elapsed");
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
    return GJP_OK;
  };
  // tile shape and view group with four-plane load groups, then two-plane
  // groups for the best of them
  // two rays per lane (k = 7) only for 16-bit storage; three (k = 8) for all
  const bool pairs = vol_dtype != GJP_F32;
  for (int k : {8, 7, 6, 5, 4}) {
    if (k == 7 && !pairs) continue;
    for (int vg : {8, 16, 1}) {
      FwdTile t;
      t.tile_v_log2 = k;
      t.view_group = vg;
      t.ru_group = 4;
      st = trial(t);
      if (st != GJP_OK) break;
    }
    if (st != GJP_OK) break;
  }
  if (st == GJP_OK) {
    FwdTile t = best;
    t.ru_group = 2;
    st = trial(t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GJP_OK) return st;
  {
    const std::string key = tune_key(g, vol_dtype);
    const std::string dev = tune_cache_path() ? device_tag() : std::string();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    disk_load(dev);
    disk_store(dev, key, best);
  }
  if (tile_v_out) *tile_v_out = gjp::tile_v_pixels(best.tile_v_log2);
  return GJP_OK;
}

extern "C" gjp_status gjp_set_forward_tile(const gjp_geometry* g, int32_t vol_dtype,
                                           int32_t tile_v, int32_t view_group,
                                           int32_t load_group) {
  if (!g) return fail(GJP_EINVAL, "gjp_set_forward_tile: geometry is null");
  if (vol_dtype != GJP_F32 && vol_dtype != GJP_BF16 && vol_dtype != GJP_F16)
    return fail(GJP_EINVAL, "gjp_set_forward_tile: unknown dtype");
  if (tile_v == 0) {  // forget this process's choice
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.erase(tune_key(g, vol_dtype));
    return GJP_OK;
  }
  FwdTile t;
  if (tile_v == 192) t.tile_v_log2 = 8;
  else if (tile_v == 128 && vol_dtype != GJP_F32) t.tile_v_log2 = 7;
  else if (tile_v == 64) t.tile_v_log2 = 6;
  else if (tile_v == 32) t.tile_v_log2 = 5;
  else if (tile_v == 16) t.tile_v_log2 = 4;
  else
    return fail(GJP_EINVAL,
                "gjp_set_forward_tile: tile_v must be 192, 64, 32 or 16 (or 128 for 16-bit "
                "storage)");
  if (view_group < 1 || view_group > 64)
    return fail(GJP_EINVAL, "gjp_set_forward_tile: view_group must be in [1, 64]");
  if (load_group != 2 && load_group != 4)
    return fail(GJP_EINVAL, "gjp_set_forward_tile: load_group must be 2 or 4");
  t.view_group = view_group;
  t.ru_group = load_group;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[tune_key(g, vol_dtype)] = t;
  return GJP_OK;
}

extern "C" gjp_status gjp_get_forward_tile(const gjp_geometry* g, int32_t vol_dtype,
                                           int32_t* tile_v, int32_t* view_group,
                                           int32_t* load_group) {
  if (!g || !tile_v || !view_group || !load_group)
    return fail(GJP_EINVAL, "gjp_get_forward_tile: null pointer");
  if (vol_dtype != GJP_F32 && vol_dtype != GJP_BF16 && vol_dtype != GJP_F16)
    return fail(GJP_EINVAL, "gjp_get_forward_tile: unknown dtype");
  const FwdTile t = tile_for(g, vol_dtype);
  *tile_v = gjp::tile_v_pixels(t.tile_v_log2);
  *view_group = t.view_group;
  *load_group = t.ru_group;
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// Views per launch of the column-form gather (see gjp_back_project).
static const int kGatherViews = 32;

extern "C" gjp_status gjp_back_project(const gjp_geometry* g, const float* d_sino, float* d_vol,
                                       void* stream) {
  if (!g) return fail(GJP_EINVAL, "back_project: geometry is null");
  if (!d_sino || !d_vol) return fail(GJP_EINVAL, "back_project: null device pointer");
  if (((uintptr_t)d_sino) % 4 != 0 || ((uintptr_t)d_vol) % 4 != 0)
    return fail(GJP_EINVAL, "back_project: misaligned pointer");
  hipStream_t s = (hipStream_t)stream;
  const double* d_views = nullptr;
  const float* d_proj = nullptr;
  int st = gjp::geometry_device(g, &d_views, &d_proj);
  if (st != GJP_OK) return (gjp_status)st;
  // Table layouts: column geometries without clipping take the value table
  // (4 bytes per ray, positions from each column's affine map), other column
  // geometries the 16-byte ray table, the rest the 32-byte general table.
  const bool value = g->separable && !g->gg.clip;
  const size_t per_view =
      (size_t)g->n_u * (size_t)(g->separable ? g->n_v + gjp::kColumnPad : g->n_v);
  const size_t entry = value ? sizeof(float) : (g->separable ? 1 : 2) * sizeof(float4);
  const size_t col_entry =
      value ? sizeof(gjp::ResCol) : (g->separable ? sizeof(float4) : (size_t)0);
  const size_t budget = (size_t)512 << 20;
  long long chunk = (long long)(budget / (per_view * entry + (size_t)g->n_u * col_entry));
  if (chunk < 1) chunk = 1;
  if (chunk > g->n_views) chunk = g->n_views;
  void* table = nullptr;
  void* mask = nullptr;
  void* cols = nullptr;
  GJP_HIP(scratch_alloc(&table, (size_t)chunk * per_view * entry, s), "back_project: table");
  hipError_t e = scratch_alloc(&mask, (size_t)chunk * sizeof(int), s);
  if (e == hipSuccess && col_entry > 0)
    e = scratch_alloc(&cols, (size_t)chunk * g->n_u * col_entry, s);
  if (e != hipSuccess) {
    (void)scratch_free(table, s);
    (void)scratch_free(mask, s);
    return hip_fail(e, "back_project: scratch");
  }
  float4* t4 = value ? nullptr : static_cast<float4*>(table);
  float4* c4 = value ? nullptr : static_cast<float4*>(cols);
  float* tv = value ? static_cast<float*>(table) : nullptr;
  gjp::ResCol* cv = value ? static_cast<gjp::ResCol*>(cols) : nullptr;
  for (int v0 = 0; v0 < g->n_views && st == GJP_OK; v0 += (int)chunk) {
    const int nc = (int)std::min<long long>(chunk, g->n_views - v0);
    st = gjp::launch_zero_ints(static_cast<int*>(mask), nc, s);
    if (st == GJP_OK)
      st = value ? gjp::launch_adjoint_value_table(g, d_views, d_sino, v0, nc, tv, cv,
                                                   static_cast<int*>(mask), s)
                 : gjp::launch_adjoint_table(g, d_views, d_sino, v0, nc, t4, c4,
                                             static_cast<int*>(mask), s);
    // The gather runs over sub-chunks of views so that all resident
    // workgroups read the same few views' tables (L2-sized working set);
    // each sub-chunk reads and writes the volume once.
    const int sub = g->separable ? kGatherViews : nc;
    for (int c0 = 0; c0 < nc && st == GJP_OK; c0 += sub) {
      const int ns = std::min(sub, nc - c0);
      st = gjp::launch_adjoint_gather(g, d_proj, t4, c4, tv, cv, static_cast<const int*>(mask),
                                      v0, c0, ns, v0 + c0 > 0, d_vol, s);
    }
  }
  (void)scratch_free(cols, s);
  const hipError_t f1 = scratch_free(table, s);
  const hipError_t f2 = scratch_free(mask, s);
  if (st != GJP_OK) return (gjp_status)st;
  if (f1 != hipSuccess) return hip_fail(f1, "back_project: free table");
  if (f2 != hipSuccess) return hip_fail(f2, "back_project: free mask");
  return GJP_OK;
}

// ---------------------------------------------------------------------------
// batched forward: plan = instance descriptors, work list, queue, graph
// ---------------------------------------------------------------------------
namespace {
struct BatchPlan {
  std::vector<uint64_t> ids;
  std::vector<int> dtypes;
  int device = 0;
  std::vector<BatchInst> host;  // descriptors without per-call pointers
  BatchInst* d_insts = nullptr;
  uint2* d_items = nullptr;
  int* d_counter = nullptr;  // kBatchQueues per class
  int* d_qoff = nullptr;     // kBatchQueues + 1 per class
  void* padded_all = nullptr;
  int n_items = 0;
  // items are grouped by instance class; one persistent launch per class
  std::vector<int> cls, cls_begin, cls_count, cls_grid;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchInst* staging = nullptr;  // pinned
  hipEvent_t staged = nullptr;   // the descriptor upload has read `staging`
  bool staged_pending = false;
  // The last replay has finished with the plan's device buffers (descriptors,
  // padded copies, queue counters). A replay on any stream first waits for
  // the previous one on the device, so replays of one plan never overlap.
  hipEvent_t done = nullptr;
  bool done_pending = false;
  uint64_t last_use = 0;  // for least-recently-used eviction
  std::mutex mu;

  ~BatchPlan() {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    // the plan's own work only: no device-wide synchronisation
    if (done && done_pending) (void)hipEventSynchronize(done);
    if (staged && staged_pending) (void)hipEventSynchronize(staged);
    if (done) (void)hipEventDestroy(done);
    if (staged) (void)hipEventDestroy(staged);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_insts) (void)hipFree(d_insts);
    if (d_items) (void)hipFree(d_items);
    if (d_counter) (void)hipFree(d_counter);
    if (d_qoff) (void)hipFree(d_qoff);
    if (padded_all) (void)hipFree(padded_all);
    if (staging) (void)hipHostFree(staging);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
};

std::mutex g_plan_mu;
std::map<std::string, std::shared_ptr<BatchPlan>> g_plans;
uint64_t g_plan_clock = 0;  // guarded by g_plan_mu
constexpr size_t kMaxPlans = 8;

std::string plan_key(int n, const gjp_geometry* const* g, const int32_t* dtypes, int dvc) {
  std::string k = std::to_string(dvc);
  for (int i = 0; i < n; ++i) {
    k += "|" + std::to_string(g[i]->id) + ":" + std::to_string(dtypes[i]);
    const FwdTile t = tile_for(g[i], dtypes[i]);
    k += ":" + std::to_string(t.tile_v_log2);
  }
  return k;
}

// One group of work items of the batched launch and its estimated cost.
struct WorkGroup {
  int inst, v0, tile;
  double cost;    // estimated samples of the group
  double bucket;  // log-scale cost class for the ordering
};

// Estimated samples of each work group: the exact sample counts (the kernels'
// own double-precision ray setup) of five rays per tile and view -- its four
// corner pixels and its centre -- scaled to the tile's rays, plus a fixed
// per-ray setup cost.
void estimate_group_costs(const gjp_geometry* const* g, const std::vector<BatchInst>& insts,
                          std::vector<WorkGroup>& groups) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 64) nt = 64;
  if (groups.size() < 4096) nt = 1;
  auto work = [&](unsigned t) {
    for (size_t k = t; k < groups.size(); k += nt) {
      WorkGroup& w = groups[k];
      const gjp_geometry* G = g[w.inst];
      const FwdArgs& a = insts[w.inst].a;
      const int kv = a.tile_v_log2;
      const int tile_u = gjp::tile_u_columns(kv), tile_v = gjp::tile_v_pixels(kv);
      const int tv = w.tile / a.tiles_u, tu = w.tile - tv * a.tiles_u;  // the kernels' order
      const int u_lo = tu * tile_u, v_lo = tv * tile_v;
      const int u_hi = std::min(G->n_u, u_lo + tile_u) - 1;
      const int v_hi = std::min(G->n_v, v_lo + tile_v) - 1;
      const int pu[5] = {u_lo, u_lo, u_hi, u_hi, (u_lo + u_hi) / 2};
      const int pv[5] = {v_lo, v_hi, v_lo, v_hi, (v_lo + v_hi) / 2};
      const int kg = std::min(std::max(1, a.view_group), G->n_views - w.v0);
      double samples = 0.0;
      for (int v = w.v0; v < w.v0 + kg; ++v)
        for (int r = 0; r < 5; ++r) {
          gjp::RaySetup R;
          gjp::ray_setup(G->views_grid.data() + 12 * (size_t)v, G->gg, pu[r], pv[r], R);
          samples += (double)(R.i1 - R.i0);
        }
      const double rays = (double)(u_hi - u_lo + 1) * (double)(v_hi - v_lo + 1);
      w.cost = samples / 5.0 * rays + 32.0 * rays * kg;
    }
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
}

gjp_status build_plan(int n, const gjp_geometry* const* g, const int32_t* dtypes, int dvc,
                      std::shared_ptr<BatchPlan>& out) {
  auto P = std::make_shared<BatchPlan>();
  P->device = dvc;
  P->host.resize(n);
  size_t pad_bytes = 0;
  std::vector<size_t> pad_off(n);
  for (int i = 0; i < n; ++i) {
    P->ids.push_back(g[i]->id);
    P->dtypes.push_back(dtypes[i]);
    if (!block_fits_32bit(g[i]->n, dtypes[i]))
      return fail(GJP_EUNSUPPORTED, "batched: volume planes too large for 32-bit block offsets");
    pad_off[i] = pad_bytes;
    pad_bytes += (size_t)(2 * copy_bytes(g[i]->n, dtypes[i]));
  }
  GJP_HIP(hipMalloc(&P->padded_all, pad_bytes), "batched: padded volumes");
  long long total_items = 0;
  for (int i = 0; i < n; ++i) {
    const double* d_views = nullptr;
    const float* d_proj = nullptr;
    int st = gjp::geometry_device(g[i], &d_views, &d_proj);
    if (st != GJP_OK) return (gjp_status)st;
    BatchInst& I = P->host[i];
    memset(&I, 0, sizeof(I));
    const FwdTile tile = tile_for(g[i], dtypes[i]);
    FwdTile t2 = tile;
    t2.remap = 0;
    // the batched launch runs the tuned tile with one or three rays per lane;
    // a tuned two-rays-per-lane tile becomes the one-ray tile (same sums)
    if (t2.tile_v_log2 == 7) t2.tile_v_log2 = 6;
    fill_fwd_args(g[i], d_views, nullptr, nullptr, t2, I.a);
    I.padded = static_cast<char*>(P->padded_all) + pad_off[i];
    set_padded(I.a, I.padded, dtypes[i], g[i]->n);
    I.n_views = g[i]->n_views;
    I.dtype = dtypes[i];
    I.weight = g[i]->weight;
    I.padded_elems = padded_elems(g[i]->n);
    I.idx64 = needs_idx64(g[i]->n, dtypes[i]) ? 1 : 0;
    total_items += (long long)I.n_views * I.a.tiles_per_view;
  }
  if (total_items > (1ll << 31) - 1) return fail(GJP_EUNSUPPORTED, "batched: too many work items");
  // Work groups: (instance, group of view_group consecutive views, ray tile);
  // a group's items are that tile for each view of the group in turn (the
  // single launch's order: rays of nearby views share volume lines in L2).
  std::vector<WorkGroup> groups;
  try {
    for (int i = 0; i < n; ++i) {
      const BatchInst& I = P->host[i];
      const int K = std::max(1, I.a.view_group);
      for (int v0 = 0; v0 < I.n_views; v0 += K)
        for (int t = 0; t < I.a.tiles_per_view; ++t) groups.push_back({i, v0, t, 0.0});
    }
  } catch (...) {
    return fail(GJP_ENOMEM, "batched: work groups");
  }
  estimate_group_costs(g, P->host, groups);
  // Longest first within each instance class, by the host double-precision
  // sample count of a few rays per tile and view. Costs within about 20% of
  // each other share a bucket, where the natural order (instance, views,
  // tile) is kept for cache locality.
  for (auto& w : groups)
    w.bucket = w.cost > 0.0 ? std::floor(std::log(w.cost) / std::log(1.2)) : -1.0e9;
  std::stable_sort(groups.begin(), groups.end(),
                   [](const WorkGroup& x, const WorkGroup& y) { return x.bucket > y.bucket; });
  std::vector<uint2> items;
  try {
    items.reserve((size_t)total_items);
  } catch (...) {
    return fail(GJP_ENOMEM, "batched: work list");
  }
  // Per class, the groups go round robin to kBatchQueues queues (one per XCD),
  // each keeping the longest-first order; a group's items stay together.
  std::vector<int> qoff;
  for (int c = 0; c < gjp::kBatchClasses; ++c) {
    const size_t begin = items.size();
    std::vector<std::vector<uint2>> q(gjp::kBatchQueues);
    int gi = 0;
    try {
      for (const auto& w : groups) {
        const BatchInst& I = P->host[w.inst];
        if (gjp::batch_class(I.dtype, I.weight, I.idx64, I.a.tile_v_log2 == 8 ? 1 : 0) != c)
          continue;
        std::vector<uint2>& dst = q[gi++ % gjp::kBatchQueues];
        const int kg = std::min(std::max(1, I.a.view_group), I.n_views - w.v0);
        for (int v = w.v0; v < w.v0 + kg; ++v)
          dst.push_back(make_uint2((uint32_t)w.inst | ((uint32_t)v << 12), (uint32_t)w.tile));
      }
    } catch (...) {
      return fail(GJP_ENOMEM, "batched: queues");
    }
    if (gi == 0) continue;
    for (int x = 0; x < gjp::kBatchQueues; ++x) {
      qoff.push_back((int)(items.size() - begin));
      items.insert(items.end(), q[x].begin(), q[x].end());
    }
    qoff.push_back((int)(items.size() - begin));
    P->cls.push_back(c);
    P->cls_begin.push_back((int)begin);
    P->cls_count.push_back((int)(items.size() - begin));
    P->cls_grid.push_back(gjp::batched_grid_size(c));
  }
  P->n_items = (int)items.size();
  GJP_HIP(hipMalloc(&P->d_items, std::max<size_t>(1, items.size()) * sizeof(uint2)),
          "batched: items");
  GJP_HIP(hipMemcpy(P->d_items, items.data(), items.size() * sizeof(uint2),
                    hipMemcpyHostToDevice),
          "batched: items copy");
  GJP_HIP(hipMalloc(&P->d_insts, (size_t)n * sizeof(BatchInst)), "batched: descriptors");
  const size_t n_cls = std::max<size_t>(1, P->cls.size());
  GJP_HIP(hipMalloc(&P->d_counter, n_cls * gjp::kBatchQueues * sizeof(int)), "batched: queues");
  GJP_HIP(hipMalloc(&P->d_qoff, n_cls * (gjp::kBatchQueues + 1) * sizeof(int)),
          "batched: queue offsets");
  if (!qoff.empty())
    GJP_HIP(hipMemcpy(P->d_qoff, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice),
            "batched: queue offsets copy");
  GJP_HIP(hipHostMalloc(&P->staging, (size_t)n * sizeof(BatchInst), 0), "batched: staging");
  GJP_HIP(hipEventCreateWithFlags(&P->staged, hipEventDisableTiming), "batched: event");
  GJP_HIP(hipEventCreateWithFlags(&P->done, hipEventDisableTiming), "batched: event");
  // capture pad + queue reset + persistent kernel once
  hipStream_t cap;
  GJP_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "batched: capture stream");
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  int st = GJP_OK;
  if (e == hipSuccess) {
    st = gjp::launch_batched_pad(P->d_insts, n, cap);
    if (st == GJP_OK)
      st = gjp::launch_zero_ints(P->d_counter, (int)P->cls.size() * gjp::kBatchQueues, cap);
    for (size_t k = 0; k < P->cls.size() && st == GJP_OK; ++k)
      st = gjp::launch_batched_forward(P->d_insts, P->d_items + P->cls_begin[k],
                                       P->d_qoff + k * (gjp::kBatchQueues + 1),
                                       P->d_counter + k * gjp::kBatchQueues, P->cls_grid[k],
                                       P->cls[k], cap);
    const hipError_t e2 = hipStreamEndCapture(cap, &P->graph);
    if (e2 != hipSuccess && st == GJP_OK) st = hip_fail(e2, "batched: end capture");
  } else {
    st = hip_fail(e, "batched: begin capture");
  }
  (void)hipStreamDestroy(cap);
  if (st != GJP_OK) return (gjp_status)st;
  GJP_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0), "batched: instantiate");
  out = P;
  return GJP_OK;
}
}  // namespace

static void invalidate_plans(uint64_t id) {
  std::vector<std::shared_ptr<BatchPlan>> drop;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
      if (std::find(it->second->ids.begin(), it->second->ids.end(), id) !=
          it->second->ids.end()) {
        drop.push_back(it->second);
        it = g_plans.erase(it);
      } else {
        ++it;
      }
    }
  }
  drop.clear();
}

extern "C" gjp_status gjp_forward_project_batched(int32_t n, const gjp_geometry* const* g,
                                                  const void* const* d_vols,
                                                  const int32_t* dtypes, float* const* d_sinos,
                                                  void* stream) {
  if (n <= 0 || n > 4096) return fail(GJP_EINVAL, "batched: n must be in [1, 4096]");
  if (!g || !d_vols || !dtypes || !d_sinos) return fail(GJP_EINVAL, "batched: null array");
  for (int i = 0; i < n; ++i) {
    gjp_status st = validate_fwd(g[i], d_vols[i], dtypes[i], d_sinos[i]);
    if (st != GJP_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  int dvc = 0;
  GJP_HIP(hipGetDevice(&dvc), "hipGetDevice");
  const std::string key = plan_key(n, g, dtypes, dvc);
  std::shared_ptr<BatchPlan> P;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      P = it->second;
      P->last_use = ++g_plan_clock;
    }
  }
  if (!P) {
    gjp_status st = build_plan(n, g, dtypes, dvc, P);
    if (st != GJP_OK) return st;
    std::shared_ptr<BatchPlan> evicted;  // released after the lock
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= kMaxPlans) {
      auto lru = g_plans.begin();
      for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
        if (it->second->last_use < lru->second->last_use) lru = it;
      evicted = lru->second;
      g_plans.erase(lru);
    }
    P->last_use = ++g_plan_clock;
    g_plans[key] = P;
  }
  std::lock_guard<std::mutex> lk(P->mu);
  // the host staging buffer is free once the previous upload has read it
  if (P->staged_pending) GJP_HIP(hipEventSynchronize(P->staged), "batched: staging wait");
  // the device buffers are free once the previous replay (on whatever
  // stream) has finished: wait for it on this stream, without a host sync
  if (P->done_pending) GJP_HIP(hipStreamWaitEvent(s, P->done, 0), "batched: replay order");
  for (int i = 0; i < n; ++i) {
    P->staging[i] = P->host[i];
    P->staging[i].src = d_vols[i];
    P->staging[i].a.sino = d_sinos[i];
  }
  GJP_HIP(hipMemcpyAsync(P->d_insts, P->staging, (size_t)n * sizeof(BatchInst),
                         hipMemcpyHostToDevice, s),
          "batched: descriptor upload");
  GJP_HIP(hipEventRecord(P->staged, s), "batched: staging event");
  P->staged_pending = true;
  gjp::TimedLaunch t = gjp::timing_begin("batched", s);
  GJP_HIP(hipGraphLaunch(P->exec, s), "batched: graph launch");
  gjp::timing_end("batched", t, s);
  GJP_HIP(hipEventRecord(P->done, s), "batched: completion event");
  P->done_pending = true;
  return GJP_OK;
}
