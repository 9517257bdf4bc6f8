/*
 * gjp.h -- C ABI of the MI355X (gfx950) generalized Joseph projector.
 *
 * The projector follows Sec. III of Graetz, "High performance volume ray
 * casting: a branchless generalized Joseph projector" (arXiv 1609.00958):
 * each ray is stepped one voxel plane at a time along its driving axis
 * (Eqs. 1-6), the two transverse axes are interpolated from the four in-plane
 * neighbours (Eqs. 7-12, weight functions Eqs. 13-14) and the sum is scaled by
 * the step length (Algorithm 1).
 *
 * Conventions (all functions):
 *   - Volumes are C-order arrays vol[n0][n1][n2] (n2 fastest). Grid
 *     coordinate k is the centre of voxel k; world -> grid for a point w is
 *         g_k = (w_k - vol_center_k) / voxel_size_k + (n_k - 1) * 0.5
 *     and for a direction g_k = w_k / voxel_size_k (double precision, no
 *     fused multiply-add).
 *   - A view is 12 doubles in world units. Cone beam: src[3], det00[3],
 *     du[3], dv[3]; parallel beam: dir[3], det00[3], du[3], dv[3]. The centre
 *     of pixel (iu, iv) is det00 + iu*du + iv*dv (evaluated left to right).
 *     For a parallel beam the pixel itself is the ray's reference point.
 *   - Sinograms are C-order float arrays sino[n_views][n_u][n_v] (v fastest).
 *   - A sample (ray, plane i) exists when -1 < p_k < n_k on both transverse
 *     axes and 0 <= i < n_m (the volume is read as zero outside the grid);
 *     the driving axis is argmax |r_k| with ties to the lowest axis index. The
 *     ray setup and the sample range are evaluated in double precision;
 *     sample positions, weights and accumulation in single precision.
 *   - Device pointers must point to memory of the current HIP device; the
 *     library never frees caller memory. `stream` is a hipStream_t (NULL for
 *     the default stream); every projection call is asynchronous on it.
 *   - Every function returns a gjp_status. Arguments are validated before any
 *     GPU work is queued; on failure nothing is launched and
 *     gjp_last_error() describes the problem. No C++ exception crosses the ABI.
 */
#ifndef GJP_H
#define GJP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GJP_OK = 0,
  GJP_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad enum) */
  GJP_ENOMEM = -2,       /* host or device allocation failed */
  GJP_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  GJP_EUNSUPPORTED = -4  /* valid request that this build does not implement */
} gjp_status;

typedef enum { GJP_F32 = 0, GJP_BF16 = 1, GJP_F16 = 2 } gjp_dtype;
typedef enum { GJP_CONE = 0, GJP_PARALLEL = 1 } gjp_beam;
/* Eq. 13 (linear, classic multilinear interpolation) and Eq. 14 (cubic
   smoothstep spline, differentiable at grid points). */
typedef enum { GJP_W_LINEAR = 0, GJP_W_SPLINE = 1 } gjp_weight;

typedef struct {
  int32_t vol_shape[3];   /* n0, n1, n2 (n2 fastest); each >= 1 */
  double voxel_size[3];   /* world units per grid step; each > 0 */
  double vol_center[3];   /* world position of the grid centre */
  int32_t n_views, n_u, n_v;
  int32_t beam;           /* gjp_beam */
  const double *views;    /* host, n_views x 12 doubles (world units); copied */
  int32_t weight;         /* gjp_weight */
  uint32_t flags;         /* 0 or GJP_CLIP_CYLINDER */
} gjp_geometry_desc;

/* gjp_geometry_desc.flags: clip every ray's sample range to the cylinder
   inscribed in the grid box (Sec. IV-C: the first sample and the number of
   samples follow the ray-cylinder instead of the ray-box intersection). The
   cylinder's axis is the rotation axis (axis 2) through ((n0-1)/2, (n1-1)/2)
   in grid coordinates, its radius min(n0, n1)/2 voxels; a sample counts only
   if its axis-0/axis-1 position lies strictly inside. Forward, adjoint and
   sample count all use the clipped range. */
#define GJP_CLIP_CYLINDER 1u

typedef struct gjp_geometry gjp_geometry; /* opaque, immutable after creation */

/* Create a projection geometry (Sec. III-A: source and detector pixel
   positions in grid units). Host-only: validates `desc`, copies the view
   vectors and converts them to grid units; device copies are made on first
   use on each device. *out receives the handle (caller destroys it).
   Errors: GJP_EINVAL for a null pointer, a non-positive size, a
   non-positive voxel size, an unknown beam/weight, unknown flags, a
   non-finite view vector, or more than 32767 voxels along an axis;
   GJP_ENOMEM if the copy cannot be allocated. */
gjp_status gjp_create_geometry(const gjp_geometry_desc *desc, gjp_geometry **out);

/* Destroy a geometry and its device copies. NULL is accepted. The caller
   must make sure no queued projection still uses it. */
gjp_status gjp_destroy_geometry(gjp_geometry *g);

/* Forward projection y = A x (Algorithm 1, one ray per detector pixel).
   d_vol: device, n0*n1*n2 elements of `vol_dtype` (gjp_dtype), C order,
   aligned to its element size. d_sino: device, n_views*n_u*n_v floats,
   overwritten. BF16/FP16 volumes are widened to FP32 in registers; the
   accumulation is FP32 in every case. Two zero-padded pair copies of the
   volume (about 4x its size) are taken from the stream-ordered pool for the
   duration of the call; if the pool cannot serve them, its cached memory is
   returned to the device (after synchronising `stream`) and the request
   retried, and failing that they are allocated with hipMalloc and freed
   after synchronising `stream`. The volume must be finite.
   Errors: GJP_EINVAL (null pointer, unknown dtype), GJP_EUNSUPPORTED (a
   volume plane above about 32 MiB per pair copy, beyond 2048^2 FP32),
   GJP_ENOMEM, GJP_EHIP. */
gjp_status gjp_forward_project(const gjp_geometry *g, const void *d_vol, int32_t vol_dtype,
                               float *d_sino, void *stream);

/* gjp_forward_project without any allocation, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc). Same arguments, kernels, launch
   configuration and results as gjp_forward_project; the two padded pair
   copies are written into a fixed device scratch of 64 MiB that the library
   holds on every device it runs on until the process ends (enough for FP32
   volumes up to 158^3 voxels, 16-bit ones up to 200^3). The
   geometry must already have its device copy on the current device: any
   other projection call with it on that device makes one. Calls on one device
   share the scratch, whose contents are those of the last call: calls that
   overlap on one device (different streams, or threads) race and must be
   serialised by the caller. Calls no hipMalloc, hipFree or other allocating
   routine. Errors: GJP_EINVAL (as gjp_forward_project; padded copies larger
   than the scratch: each is (n0+2) * (n1+2) * (n2+3 rounded down to even)
   * 2 * element size bytes rounded up to 256, and both must fit; no device
   copy of the geometry yet),
   GJP_EUNSUPPORTED, GJP_EHIP. */
gjp_status gjp_forward_project_noalloc(const gjp_geometry *g, const void *d_vol,
                                       int32_t vol_dtype, float *d_sino, void *stream);

/* Plain forward projection for comparison (Algorithm 1 as written: one lane
   per ray, the four neighbours of each sample read from d_vol itself with a
   zero-padding bounds test each, Eq. 8). Arguments and layouts as for
   gjp_forward_project; the ray setup, weights and summation order are the
   same, without its padded copies, ray tiles or launch ordering. Allocates
   nothing. Errors: GJP_EINVAL (null pointer, unknown dtype),
   GJP_EUNSUPPORTED (more than 2^40 rays), GJP_EHIP. */
gjp_status gjp_forward_project_naive(const gjp_geometry *g, const void *d_vol,
                                     int32_t vol_dtype, float *d_sino, void *stream);

/* Adjoint (exact transpose) x = A^T y of gjp_forward_project for the same
   geometry: every sample's single-precision weights are recomputed exactly as
   the forward computes them. When every view's dv is parallel to axis 2 and no
   ray is driven by axis 2 (circular trajectories), each voxel gathers its
   contributions in registers; otherwise voxel tiles accumulate in LDS with
   waves owning disjoint planes. No atomics touch the volume (the only global
   atomic is an integer OR marking which driving axes each view uses); each
   voxel is written by one thread per launch. d_sino: device,
   n_views*n_u*n_v floats. d_vol: device, n0*n1*n2 floats, overwritten.
   Per-ray tables for a chunk of views are taken from the stream-ordered pool
   during the call (with the same fallback as gjp_forward_project). Errors: GJP_EINVAL, GJP_ENOMEM, GJP_EHIP. */
gjp_status gjp_back_project(const gjp_geometry *g, const float *d_sino, float *d_vol,
                            void *stream);

/* Batched forward projection of n independent instances (geometry, volume,
   dtype, sinogram) in one persistent launch: work items (instance, view, ray
   tile) are pulled from device queues (one per XCD, dealt whole groups of
   views of one tile at a time), longest first by the host double-precision
   sample count of a few rays per tile; the launch sequence is captured in a HIP graph on
   first use for a given list of geometries and replayed afterwards. Each
   instance runs its tuned tile shape (gjp_autotune_forward /
   gjp_set_forward_tile; a two-rays-per-lane choice runs as the one-ray tile,
   whose sums are the same); instances with three rays per lane form classes
   of their own, one persistent launch per class. Each sinogram is bitwise
   equal to the one gjp_forward_project produces for the same instance and
   tile shape. Arrays g, d_vols, dtypes, d_sinos are host
   arrays of length n >= 1; every d_sinos[i] holds n_views*n_u*n_v floats.
   Calls with the same geometry list share one plan (its device descriptors,
   padded copies and queue counters); a call on any stream waits on the device
   for the previous call of that plan to finish, so calls on different streams
   are safe and run one after the other. At most 8 plans are kept (least
   recently used evicted; evicting waits for that plan's last call only).
   Errors: GJP_EINVAL, GJP_ENOMEM, GJP_EHIP. */
gjp_status gjp_forward_project_batched(int32_t n, const gjp_geometry *const *g,
                                       const void *const *d_vols, const int32_t *dtypes,
                                       float *const *d_sinos, void *stream);

/* Circular cone-beam trajectory about axis 2 (the paper's benchmark setup,
   Sec. IV-C): view k at angle 2*pi*k/n_views counter-clockwise, source at
   (sod cos, sod sin, 0), flat detector centred on the central ray at
   distance sdd from the source, du = pitch_u (-sin, cos, 0), dv = (0, 0,
   pitch_v). World units, volume centred at the origin. out_views: host,
   n_views x 12 doubles. Errors: GJP_EINVAL. */
gjp_status gjp_views_circular_cone(int32_t n_views, double sod, double sdd, double pitch_u,
                                   double pitch_v, int32_t n_u, int32_t n_v, double *out_views);

/* Circular parallel-beam trajectory: dir = (-cos, -sin, 0), detector plane
   through the rotation axis, du and dv as above. Errors: GJP_EINVAL. */
gjp_status gjp_views_parallel(int32_t n_views, double pitch_u, double pitch_v, int32_t n_u,
                              int32_t n_v, double *out_views);

/* Exact number of samples (ray, plane) of the whole sinogram, from the same
   double-precision ray setup the kernels run (host, multithreaded). This is
   the ray-sample count of the throughput metric. Errors: GJP_EINVAL. */
gjp_status gjp_count_samples(const gjp_geometry *g, uint64_t *out);

/* Select the launch configuration of gjp_forward_project for this geometry
   and dtype (ray-tile shape, views interleaved per tile, planes whose loads a
   lane issues together) by timing candidates on `stream` with the caller's
   buffers (d_sino is overwritten); the sums do not depend on the
   configuration beyond rounding order (every one matches the oracle within
   the stated tolerance). The choice is kept for this process, keyed by the
   geometry's shape signature (grid, views, detector, beam, weight) and dtype,
   and used by later forward and batched calls. If the environment variable
   GJP_TUNE_CACHE names a file, the choice is also written there (one line
   per entry, tagged with the device's architecture name and compute-unit
   count; replaced atomically by rename) and later processes on the same kind
   of device read it instead of the default; an unreadable or unwritable
   file is ignored. *tile_v_out receives the chosen number of detector pixels
   along v per wavefront row (192 when three pixels per lane share their
   loads, any storage type; 128 when two do, 16-bit storage only; else 64, 32
   or 16). Synchronises `stream`.
   Errors: GJP_EINVAL, GJP_ENOMEM, GJP_EHIP. */
gjp_status gjp_autotune_forward(const gjp_geometry *g, const void *d_vol, int32_t vol_dtype,
                                float *d_sino, void *stream, int32_t *tile_v_out);

/* Fix the launch configuration that forward calls (and, for the tile shape
   and view group, batched calls) use in this process for geometries of this
   shape signature and dtype, as gjp_autotune_forward would: tile_v =
   detector pixels along v per wavefront row (64, 32 or 16; 192: three
   pixels of a detector column per lane, any storage type; 128: two, 16-bit
   storage only; the pixels of a lane share their loads where the geometry
   allows; 192 interpolates each element along the row first, equal to the
   other tiles' sums up to rounding; batched calls run 128 as 64, whose sums
   are the same); view_group =
   consecutive views that take their turn on each ray tile together (1 to
   64); load_group = planes whose volume loads a lane issues together (2 or
   4). tile_v = 0 removes this process's choice (the on-disk cache or the
   default applies again; the other arguments are ignored). Not written to
   the on-disk cache. Host-only. Errors: GJP_EINVAL. */
gjp_status gjp_set_forward_tile(const gjp_geometry *g, int32_t vol_dtype, int32_t tile_v,
                                int32_t view_group, int32_t load_group);

/* The launch configuration gjp_forward_project would use now for this
   geometry's shape signature and dtype (this process's choice, else the
   on-disk cache's entry for the current device, else the default 64 / 8 / 4).
   Errors: GJP_EINVAL (null pointer, unknown dtype). */
gjp_status gjp_get_forward_tile(const gjp_geometry *g, int32_t vol_dtype, int32_t *tile_v,
                                int32_t *view_group, int32_t *load_group);

/* SART (the reconstruction of Sec. IV-B, after Andersen and Kak): the two
   elementwise steps of one subset update
       x <- x + lam * A_S^T( (b_S - A_S x) / (A_S 1) ) / (A_S^T 1),
   the projections A_S and A_S^T being gjp_forward_project / gjp_back_project
   on a geometry holding the subset's views. A zero row sum (A_S 1) or column
   sum (A_S^T 1) makes its term zero. All pointers are device float arrays of
   n elements; queued on `stream`; no synchronisation.

   gjp_sart_residual: out[i] = row_sum[i] > 0 ? (b[i] - ax[i]) / row_sum[i] : 0.
   `out` may alias `ax`. */
gjp_status gjp_sart_residual(int64_t n, const float *d_b, const float *d_ax,
                             const float *d_row_sum, float *d_out, void *stream);

/* gjp_sart_update: x[j] += col_sum[j] > 0 ? lam * bp[j] / col_sum[j] : 0, then
   x[j] = max(x[j], 0) if nonneg != 0. bp = A_S^T of the residual. */
gjp_status gjp_sart_update(int64_t n, float *d_x, const float *d_bp, const float *d_col_sum,
                           float lam, int32_t nonneg, void *stream);

/* Per-kernel GPU timing for benchmarks. While enabled, each launch of the
   library's main kernels is bracketed by HIP events on its stream.
   gjp_timing_read waits for those events and returns the total time in
   milliseconds and the number of launches recorded for `kernel` ("forward",
   "forward_naive", "pad", "adjoint_table", "adjoint_gather", "batched",
   "sart"). */
gjp_status gjp_timing_enable(int32_t on);
gjp_status gjp_timing_reset(void);
gjp_status gjp_timing_read(const char *kernel, double *total_ms, int64_t *launches);

/* Message of the last failure on the calling thread ("" if none). */
const char *gjp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GJP_H */
