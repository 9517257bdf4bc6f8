// Sanitizer driver of the library's host path (built by
// tests/test_sanitizers_cpu.py from csrc/gjp_api.cpp with host-only
// -fsanitize=address,undefined). It runs every entry point that does its work
// on the host -- argument validation, world -> grid conversion, the
// double-precision ray setup behind the sample count, trajectories, the
// launch-configuration cache on disk, timing bookkeeping -- and no entry point
// that launches a kernel; the kernel launchers are replaced by stubs that fail
// the run if they are ever reached.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "gjp.h"
#include "gjp_internal.h"

namespace gjp {
static int stub(const char* what) {
  fprintf(stderr, "kernel launcher reached on the host path: %s\n", what);
  abort();
}
int launch_pad(const void*, void*, void*, int, const int*, hipStream_t) { return stub("pad"); }
int launch_zero_ints(int*, int, hipStream_t) { return stub("zero"); }
int launch_sart_residual(long long, const float*, const float*, const float*, float*,
                         hipStream_t) { return stub("sart"); }
int launch_sart_update(long long, float*, const float*, const float*, float, int, hipStream_t) {
  return stub("sart");
}
int launch_forward(const FwdArgs&, int, int, bool, int, hipStream_t) { return stub("forward"); }
int launch_forward_naive(const GridGeom&, const double*, const void*, int, int, int, int, int,
                         float*, hipStream_t) { return stub("naive"); }
int launch_adjoint_table(const gjp_geometry*, const double*, const float*, int, int, float4*,
                         float4*, int*, hipStream_t) { return stub("table"); }
int launch_adjoint_gather(const gjp_geometry*, const float*, const float4*, const float4*,
                          const float*, const ResCol*, const int*, int, int, int, bool, float*,
                          hipStream_t) {
  return stub("gather");
}
int launch_adjoint_value_table(const gjp_geometry*, const double*, const float*, int, int, float*,
                               ResCol*, int*, hipStream_t) {
  return stub("value table");
}
int launch_batched_pad(const BatchInst*, int, hipStream_t) { return stub("batched pad"); }
int launch_batched_forward(const BatchInst*, const uint2*, const int*, int*, int, int,
                           hipStream_t) {
  return stub("batched");
}
int batched_grid_size(int) { return 1; }
size_t dtype_size(int dtype) { return dtype == 0 ? 4 : 2; }
int noalloc_scratch(void**) { return stub("noalloc scratch"); }
}  // namespace gjp

static int bad = 0;
#define CHECK(c)                                                 \
  do {                                                           \
    if (!(c)) {                                                  \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      bad = 1;                                                   \
    }                                                            \
  } while (0)

static gjp_geometry* make(int n0, int n1, int n2, int beam, int nv, int nu, int nvv,
                          const double* views, uint32_t flags, int weight) {
  gjp_geometry_desc d;
  memset(&d, 0, sizeof(d));
  d.vol_shape[0] = n0;
  d.vol_shape[1] = n1;
  d.vol_shape[2] = n2;
  for (int k = 0; k < 3; ++k) {
    d.voxel_size[k] = 1.0 + 0.125 * k;
    d.vol_center[k] = 0.25 * k;
  }
  d.n_views = nv;
  d.n_u = nu;
  d.n_v = nvv;
  d.beam = beam;
  d.views = views;
  d.weight = weight;
  d.flags = flags;
  gjp_geometry* g = nullptr;
  if (gjp_create_geometry(&d, &g) != GJP_OK) return nullptr;
  return g;
}

int main() {
  std::vector<double> views(12 * 9);
  CHECK(gjp_views_circular_cone(9, 40.0, 60.0, 1.5, 1.25, 11, 13, views.data()) == GJP_OK);
  std::vector<double> pviews(12 * 9);
  CHECK(gjp_views_parallel(9, 1.5, 1.25, 11, 13, pviews.data()) == GJP_OK);
  // every driving axis: tilt one view's detector so that axis 2 drives
  views[12 * 8 + 2] = 35.0;
  views[12 * 8 + 9] = 0.7;
  for (int beam = 0; beam < 2; ++beam)
    for (uint32_t flags = 0; flags < 2; ++flags)
      for (int weight = 0; weight < 2; ++weight) {
        const int shapes[3][3] = {{1, 1, 1}, {9, 7, 12}, {16, 3, 5}};
        for (const auto& sh : shapes) {
          gjp_geometry* g = make(sh[0], sh[1], sh[2], beam, 9, 11, 13,
                                 beam == 0 ? views.data() : pviews.data(), flags, weight);
          CHECK(g != nullptr);
          if (!g) continue;
          uint64_t n = 0;
          CHECK(gjp_count_samples(g, &n) == GJP_OK);
          CHECK(n <= (uint64_t)9 * 11 * 13 * 16);
          int32_t tv, vg, lg;
          CHECK(gjp_set_forward_tile(g, 1, 128, 16, 2) == GJP_OK);
          CHECK(gjp_get_forward_tile(g, 1, &tv, &vg, &lg) == GJP_OK && tv == 128 && vg == 16);
          CHECK(gjp_set_forward_tile(g, 1, 0, 0, 0) == GJP_OK);
          CHECK(gjp_get_forward_tile(g, 1, &tv, &vg, &lg) == GJP_OK && tv == 64 && lg == 4);
          CHECK(gjp_set_forward_tile(g, 0, 128, 8, 2) == GJP_EINVAL);
          CHECK(gjp_destroy_geometry(g) == GJP_OK);
        }
      }
  // invalid descriptors: every rejection path, with a message
  std::vector<double> nanv = views;
  nanv[5] = NAN;
  CHECK(make(0, 4, 4, 0, 9, 11, 13, views.data(), 0, 0) == nullptr);
  CHECK(make(4, 4, 40000, 0, 9, 11, 13, views.data(), 0, 0) == nullptr);
  CHECK(make(4, 4, 4, 3, 9, 11, 13, views.data(), 0, 0) == nullptr);
  CHECK(make(4, 4, 4, 0, 9, 11, 13, views.data(), 4, 0) == nullptr);
  CHECK(make(4, 4, 4, 0, 9, 11, 13, views.data(), 0, 9) == nullptr);
  CHECK(make(4, 4, 4, 0, 9, 11, 13, nanv.data(), 0, 0) == nullptr);
  CHECK(make(4, 4, 4, 0, 9, 0, 13, views.data(), 0, 0) == nullptr);
  CHECK(make(4, 4, 4, 0, 9, 11, 13, nullptr, 0, 0) == nullptr);
  CHECK(strlen(gjp_last_error()) > 0);
  CHECK(gjp_create_geometry(nullptr, nullptr) == GJP_EINVAL);
  // a degenerate ray (source on the pixel)
  double dv[12] = {0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 5.0, 0.0, 0.0, 0.0, 5.0, 0.0};
  gjp_geometry* g = make(4, 4, 4, 0, 1, 2, 2, dv, 0, 0);
  CHECK(g != nullptr);
  uint64_t n = 1;
  CHECK(gjp_count_samples(g, &n) == GJP_OK);
  // projection calls reject bad arguments before any launch
  CHECK(gjp_forward_project(g, nullptr, 0, nullptr, nullptr) == GJP_EINVAL);
  CHECK(gjp_forward_project(g, (void*)16, 7, (float*)16, nullptr) == GJP_EINVAL);
  CHECK(gjp_forward_project(g, (void*)18, 0, (float*)16, nullptr) == GJP_EINVAL);
  CHECK(gjp_back_project(g, nullptr, (float*)16, nullptr) == GJP_EINVAL);
  CHECK(gjp_forward_project_noalloc(g, nullptr, 0, nullptr, nullptr) == GJP_EINVAL);
  {
    // padded copies of a 200^3 FP32 volume exceed the fixed scratch: rejected
    // on the host, before the scratch or the geometry's device copy is looked up
    gjp_geometry* big = make(200, 200, 200, 0, 1, 2, 2, dv, 0, 0);
    CHECK(big != nullptr);
    CHECK(gjp_forward_project_noalloc(big, (void*)16, 0, (float*)16, nullptr) == GJP_EINVAL);
    CHECK(strstr(gjp_last_error(), "scratch") != nullptr);
    CHECK(gjp_destroy_geometry(big) == GJP_OK);
  }
  CHECK(gjp_forward_project_batched(0, nullptr, nullptr, nullptr, nullptr, nullptr) == GJP_EINVAL);
  CHECK(gjp_sart_residual(-1, nullptr, nullptr, nullptr, nullptr, nullptr) == GJP_EINVAL);
  CHECK(gjp_sart_update(4, nullptr, nullptr, nullptr, 1.0f, 0, nullptr) == GJP_EINVAL);
  CHECK(gjp_views_parallel(3, 1.0, 1.0, -1, 4, pviews.data()) == GJP_EINVAL);
  CHECK(gjp_destroy_geometry(g) == GJP_OK);
  CHECK(gjp_destroy_geometry(nullptr) == GJP_OK);
  double ms = 0.0;
  int64_t cnt = 0;
  CHECK(gjp_timing_reset() == GJP_OK);
  CHECK(gjp_timing_read("forward", &ms, &cnt) == GJP_OK && cnt == 0);
  printf(bad ? "host driver: FAILED\n" : "host driver: ok\n");
  return bad;
}
