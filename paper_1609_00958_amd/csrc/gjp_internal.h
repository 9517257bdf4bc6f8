// gjp_internal.h -- host-side structures shared by the C ABI and the kernel
// launchers. Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "gjp_ray.h"

struct gjp_geometry {
  uint64_t id;                     // unique per handle (never reused)
  int n[3];
  double vs[3];
  double ctr[3];
  int n_views, n_u, n_v;
  int beam, weight;
  std::vector<double> views_world;  // as given
  std::vector<double> views_grid;   // n_views x 12, grid units
  std::vector<float> proj;          // n_views x 12: detector projection rows (u, v, w)
  gjp::GridGeom gg;
  // Every view has dv without in-plane component and no ray driven by axis 2:
  // the rays of a detector column share their in-plane coefficients, and the
  // adjoint uses the column-form gather.
  bool separable = false;

  // device copies, per device (created on first use)
  struct Dev {
    double* views = nullptr;
    float* proj = nullptr;
  };
  static constexpr int kMaxDev = 64;
  mutable std::mutex mu;
  mutable Dev dev[kMaxDev];
};

namespace gjp {

// Status plumbing (defined in gjp_api.cpp).
int set_error(int status, const std::string& msg);

// Kernel timing registry (defined in gjp_api.cpp).
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
  bool on = false;
};
TimedLaunch timing_begin(const char* name, hipStream_t s);
void timing_end(const char* name, TimedLaunch& t, hipStream_t s);

// Empty entries after each detector column in the column-form ray table
// (lets the adjoint read fixed-length candidate lists past a column's end).
constexpr int kColumnPad = 8;

// Launch configuration of the forward kernel.
struct FwdTile {
  int tile_v_log2 = 6;  // 6, 5, 4: 64, 32, 16 pixels along v per wavefront row;
                        // 7, 8: 128 / 192 pixels, two / three per lane (16-bit)
  int remap = 1;        // 1: contiguous tile ranges per XCD
  int view_group = 8;   // consecutive views that share each tile's turn
  int ru_group = 4;     // planes whose wide loads a lane issues together (2 or 4)
};

// Arguments of one forward launch (one volume, a range of views).
struct FwdArgs {
  const void* vol_a;    // pair copy A (pairs along axis 1), padded element (0,0,0)
  const void* vol_b;    // pair copy B (pairs along axis 0), padded element (0,0,0)
  unsigned long long copy_bytes;  // bytes of one pair copy
  float* sino;          // sinogram of the whole geometry
  const double* views;  // device, n_views x 12 grid units
  GridGeom G;
  long long S0, S1;     // padded strides in pair elements
  int n_u, n_v;
  int tile_v_log2;
  int view_group;       // views interleaved per tile in the launch order
  int n_views;          // views of this launch
  int tiles_v, tiles_u, tiles_per_view;
  int remap;
  int ru_group;         // planes per load group of the row-uniform loop (2 or 4)
};

// Device views of a geometry on the current device (uploads on first use).
int geometry_device(const gjp_geometry* g, const double** views, const float** proj);
// The same without uploading: GJP_EINVAL if there is no copy on this device.
int geometry_device_existing(const gjp_geometry* g, const double** views, const float** proj);

// Launchers (gjp_kernels.hip). Return a gjp_status.
int launch_pad(const void* src, void* copy_a, void* copy_b, int dtype, const int n[3],
               hipStream_t s);
int launch_zero_ints(int* p, int n, hipStream_t s);
int launch_sart_residual(long long n, const float* b, const float* ax, const float* w,
                         float* out, hipStream_t s);
int launch_sart_update(long long n, float* x, const float* bp, const float* c, float lam,
                       int nonneg, hipStream_t s);
int launch_forward(const FwdArgs& a, int dtype, int weight, bool idx64, int n_views,
                   hipStream_t s);
int launch_forward_naive(const GridGeom& G, const double* views, const void* vol, int dtype,
                         int weight, int n_views, int n_u, int n_v, float* sino, hipStream_t s);
int launch_adjoint_table(const gjp_geometry* g, const double* views, const float* sino,
                         int view0, int n_chunk, float4* table, float4* cols, int* mask,
                         hipStream_t s);
// Column map of the value-table adjoint: every ray v of detector column u
// has driving axis m, in-plane coordinate fma(i, ga, ca) on plane i and
// axis-2 coordinate A + v B there, with t = (i - sm) inv_rm, A = a0 + t a1,
// B = b0 + t b1.
struct ResCol {
  int m;  // driving axis (0 or 1); -1: no samples
  float ca, ga, pad;
  double sm, inv_rm;
  double a0, a1, b0, b1;
};
int launch_adjoint_value_table(const gjp_geometry* g, const double* views, const float* sino,
                               int view0, int n_chunk, float* vals, ResCol* cols, int* mask,
                               hipStream_t s);
// Column gather from the ray table (table, cols) or, if vals is not null,
// from the value table (vals, rcols); other geometries: tile splat (table).
int launch_adjoint_gather(const gjp_geometry* g, const float* proj, const float4* table,
                          const float4* cols, const float* vals, const ResCol* rcols,
                          const int* mask, int view0, int c0, int n_chunk, bool accumulate,
                          float* vol, hipStream_t s);

// Batched forward (gjp_batched.cpp / gjp_kernels.hip).
struct BatchInst {
  FwdArgs a;
  const void* src;      // caller volume (unpadded)
  void* padded;         // plan-owned pair copies A and B (A at the start)
  int n_views;
  int dtype, weight, idx64;
  long long padded_elems;
};
int launch_batched_pad(const BatchInst* d_insts, int n_inst, hipStream_t s);
// Instance class of the batched launch: storage type, weight, 64-bit
// addressing and three rays per lane (192-wide tiles) or one.
inline int batch_class(int dtype, int weight, int idx64, int triple) {
  return ((dtype * 2 + weight) * 2 + idx64) * 2 + triple;
}
constexpr int kBatchClasses = 24;
// Queues per class of the batched launch: one per XCD.
constexpr int kBatchQueues = 8;
// One class's persistent launch: items of its kBatchQueues queues, queue q =
// d_items[d_qoff[q] .. d_qoff[q + 1]), counters d_counters[0 .. kBatchQueues).
int launch_batched_forward(const BatchInst* d_insts, const uint2* d_items, const int* d_qoff,
                           int* d_counters, int grid, int cls, hipStream_t s);
int batched_grid_size(int cls);

size_t dtype_size(int dtype);

// Detector pixels along v per wavefront row of a forward tile code, and
// detector columns per workgroup tile.
inline int tile_v_pixels(int tile_v_log2) { return tile_v_log2 == 8 ? 192 : 1 << tile_v_log2; }
inline int tile_u_columns(int tile_v_log2) { return tile_v_log2 >= 7 ? 4 : 256 >> tile_v_log2; }

// Fixed device scratch of gjp_forward_project_noalloc (gjp_kernels.hip): its
// size, and its address on the current device (looked up once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
int noalloc_scratch(void** ptr);

}  // namespace gjp
