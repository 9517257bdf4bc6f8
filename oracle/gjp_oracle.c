/*
 * gjp_oracle.c -- FP64 CPU oracle of the branchless generalized Joseph
 * projector (GJP), arXiv 1609.00958.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no code, header
 * or constant with the GPU library. It is written from the method section of
 * the paper (Sec. III, Eqs. 1-14, Algorithm 1): plain loops in double
 * precision, no blocking, no fusion, no reordering beyond what the algorithm
 * states. Build with -ffp-contract=off and without -ffast-math.
 *
 * Conventions the paper leaves open (each is a documented reading):
 *   - Grid coordinate k is the centre of voxel k (memory index k), so the
 *     grid spans [-0.5, N-0.5] per axis. World -> grid for a point w:
 *         g = (w - vol_center) / voxel_size + (N - 1) * 0.5
 *     and for a direction: g = w / voxel_size.
 *   - View vectors are 12 doubles: cone = src, det00, du, dv; parallel =
 *     dir, det00, du, dv. Pixel (iu, iv) sits at det00 + iu*du + iv*dv,
 *     evaluated left to right. For a parallel beam the ray point s is the
 *     pixel itself and r = dir.
 *   - "p is in volume" (Algorithm 1) is read as the zero-padded domain:
 *     -1 < p_k < N_k on every axis, with neighbours outside [0, N_k-1]
 *     reading 0.
 *   - argmax ties (Eq. 3) go to the lowest axis index.
 *   - The driving coordinate of sample i is set to i exactly (Eq. 8 states it
 *     is an integer; in floating point s_m + (i - s_m) need not be).
 *   - The sample range is i = 0 .. N_m - 1 (Algorithm 1's loop bounds).
 *   - The step-length factor ||r~|| is applied once per ray (the algorithm
 *     applies it per term; only rounding differs). With non-unit voxels it
 *     is the world-space step || r~ * voxel_size ||.
 *   - A ray with r = 0 (source on a pixel) has no direction: its value is 0.
 *   - Cylinder clipping (Sec. IV-C: the first sample and the sample count
 *     follow the ray-cylinder instead of the ray-box intersection), when
 *     GJO_CLIP_CYLINDER is set: a sample also needs its axis-0/axis-1
 *     position strictly inside the circle of radius min(N0, N1) / 2 about
 *     ((N0 - 1) / 2, (N1 - 1) / 2), the cylinder inscribed in the grid box
 *     with its axis along the rotation axis (axis 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* the double nearest to pi */
static const double GJO_PI = 3.14159265358979323846;

#define GJO_CONE 0
#define GJO_PARALLEL 1
#define GJO_W_LINEAR 0
#define GJO_W_SPLINE 1
#define GJO_CLIP_CYLINDER 1

/* ------------------------------------------------------------------ */
/* Projection geometry: circular trajectory about the third axis.       */
/* ------------------------------------------------------------------ */

/* Circular cone-beam trajectory, view k at angle 2*pi*k/n_views
   (counter-clockwise about +axis 2). Source at distance sod from the
   rotation axis, flat detector at distance sdd from the source, centred on
   the central ray; du is tangential, dv is parallel to the rotation axis.
   World units, volume centred at the origin. out: n_views x 12 doubles. */
int gjo_views_circular_cone(int n_views, double sod, double sdd, double pitch_u,
                            double pitch_v, int n_u, int n_v, double *out) {
  if (n_views <= 0 || n_u <= 0 || n_v <= 0 || !out) return -1;
  for (int k = 0; k < n_views; ++k) {
    double th = 2.0 * GJO_PI * (double)k / (double)n_views;
    double c = cos(th), s = sin(th);
    double *o = out + 12 * (size_t)k;
    double src[3] = {sod * c, sod * s, 0.0};
    double dc[3] = {(sod - sdd) * c, (sod - sdd) * s, 0.0};
    double du[3] = {-pitch_u * s, pitch_u * c, 0.0};
    double dv[3] = {0.0, 0.0, pitch_v};
    double hu = 0.5 * (double)(n_u - 1), hv = 0.5 * (double)(n_v - 1);
    for (int j = 0; j < 3; ++j) {
      o[0 + j] = src[j];
      o[3 + j] = dc[j] - hu * du[j] - hv * dv[j];
      o[6 + j] = du[j];
      o[9 + j] = dv[j];
    }
  }
  return 0;
}

/* Circular parallel-beam trajectory: ray direction (-cos, -sin, 0), detector
   plane through the rotation axis. out: n_views x 12 doubles. */
int gjo_views_parallel(int n_views, double pitch_u, double pitch_v, int n_u, int n_v,
                       double *out) {
  if (n_views <= 0 || n_u <= 0 || n_v <= 0 || !out) return -1;
  for (int k = 0; k < n_views; ++k) {
    double th = 2.0 * GJO_PI * (double)k / (double)n_views;
    double c = cos(th), s = sin(th);
    double *o = out + 12 * (size_t)k;
    double dir[3] = {-c, -s, 0.0};
    double du[3] = {-pitch_u * s, pitch_u * c, 0.0};
    double dv[3] = {0.0, 0.0, pitch_v};
    double hu = 0.5 * (double)(n_u - 1), hv = 0.5 * (double)(n_v - 1);
    for (int j = 0; j < 3; ++j) {
      o[0 + j] = dir[j];
      o[3 + j] = 0.0 - hu * du[j] - hv * dv[j];
      o[6 + j] = du[j];
      o[9 + j] = dv[j];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Per-ray setup: Eqs. 1-5 / Algorithm 1 setup lines.                   */
/* ------------------------------------------------------------------ */

typedef struct {
  int n[3];
  double vs[3];
  double ctr[3];
  int beam;
  int n_views, n_u, n_v;
  const double *views; /* world units */
  int weight;
  int clip;            /* cylinder clipping (Sec. IV-C) */
  double cyl_c[2];     /* cylinder axis position on axes 0 and 1 */
  double cyl_r2;       /* squared radius */
} gjo_geom;

typedef struct {
  double s[3];  /* a point on the ray, grid units (the source for cone) */
  double rt[3]; /* r~ = r / r_m (Eq. 4) */
  int m;        /* driving axis (Eq. 3) */
  double len;   /* world-space step length of one plane step */
  int ok;       /* 0 for a degenerate ray (r = 0) */
} gjo_ray;

static void world_point_to_grid(const gjo_geom *g, const double *w, double *out) {
  for (int k = 0; k < 3; ++k)
    out[k] = (w[k] - g->ctr[k]) / g->vs[k] + (double)(g->n[k] - 1) * 0.5;
}

static void world_dir_to_grid(const gjo_geom *g, const double *w, double *out) {
  for (int k = 0; k < 3; ++k) out[k] = w[k] / g->vs[k];
}

static void ray_setup(const gjo_geom *g, int view, int iu, int iv, gjo_ray *ray) {
  const double *vw = g->views + 12 * (size_t)view;
  double a[3], det00[3], du[3], dv[3], d[3], r[3];
  world_point_to_grid(g, vw + 3, det00);
  world_dir_to_grid(g, vw + 6, du);
  world_dir_to_grid(g, vw + 9, dv);
  for (int k = 0; k < 3; ++k) d[k] = det00[k] + (double)iu * du[k] + (double)iv * dv[k];
  if (g->beam == GJO_CONE) {
    world_point_to_grid(g, vw + 0, a);
    for (int k = 0; k < 3; ++k) {
      ray->s[k] = a[k];
      r[k] = d[k] - a[k]; /* Eq. 2 */
    }
  } else {
    world_dir_to_grid(g, vw + 0, a);
    for (int k = 0; k < 3; ++k) {
      ray->s[k] = d[k];
      r[k] = a[k];
    }
  }
  /* Eq. 3: driving axis = largest |r_k|; ties keep the lowest index. */
  int m = 0;
  for (int k = 1; k < 3; ++k)
    if (fabs(r[k]) > fabs(r[m])) m = k;
  ray->m = m;
  ray->ok = (r[m] != 0.0);
  if (!ray->ok) {
    ray->len = 0.0;
    for (int k = 0; k < 3; ++k) ray->rt[k] = 0.0;
    return;
  }
  /* Eq. 4 */
  for (int k = 0; k < 3; ++k) ray->rt[k] = r[k] / r[m];
  ray->rt[m] = 1.0;
  double q = 0.0;
  for (int k = 0; k < 3; ++k) q += (ray->rt[k] * g->vs[k]) * (ray->rt[k] * g->vs[k]);
  ray->len = sqrt(q);
}

/* Eq. 13 / Eq. 14: the weight of the lower neighbour at fractional offset
   d in [0, 1]. */
static double weight_fn(int kind, double d) {
  if (kind == GJO_W_SPLINE) return 1.0 - 3.0 * d * d + 2.0 * d * d * d;
  return 1.0 - d;
}

/* Interpolation kernel of one transverse axis. Eqs. 10-12 give the two
   neighbours of a coordinate p the weights w(p - floor p) and
   1 - w(p - floor p); by the symmetry of Eq. 9 the second equals
   w(ceil p - p). Both are therefore h(p - j) for the voxel index j, with
   h(t) = w(|t|) for |t| < 1 and 0 elsewhere. At an integral p (Eq. 8) the
   voxel j = p receives h(0) = w(0) = 1 and j = p + 1 receives h(-1) = 0. */
static double kernel_1d(int kind, double t) {
  const double a = fabs(t);
  if (!(a < 1.0)) return 0.0;
  return weight_fn(kind, a);
}

/* Voxel (j0, j1, j2) of a volume of the geometry, with the zero padding of
   the in-volume reading: indices outside the grid read 0. dt: 0 = f64,
   1 = f32. */
static double voxel(const gjo_geom *g, const void *vol, int dt, const long long *j) {
  for (int k = 0; k < 3; ++k)
    if (j[k] < 0 || j[k] >= g->n[k]) return 0.0;
  const size_t idx = ((size_t)j[0] * (size_t)g->n[1] + (size_t)j[1]) * (size_t)g->n[2] + (size_t)j[2];
  if (dt == 1) return (double)((const float *)vol)[idx];
  return ((const double *)vol)[idx];
}

/* The point where the ray crosses plane i of its driving axis m (Eq. 6 with
   the offset o = -s_m of Eq. 5): q = s + (i - s_m) r~, with q_m taken as the
   integer i itself (Eq. 8). Returns 1 if the point is a sample of the ray:
   both transverse coordinates inside the zero-padded domain (-1, N_k) and,
   with cylinder clipping, the axis-0/axis-1 position strictly inside the
   cylinder. */
static int plane_point(const gjo_geom *g, const gjo_ray *ray, int i, double *q) {
  const int m = ray->m;
  for (int k = 0; k < 3; ++k) q[k] = ray->s[k] + (-ray->s[m] + (double)i) * ray->rt[k];
  q[m] = (double)i;
  for (int k = 0; k < 3; ++k) {
    if (k == m) continue;
    if (!(q[k] > -1.0 && q[k] < (double)g->n[k])) return 0;
  }
  if (g->clip) {
    const double dx = q[0] - g->cyl_c[0], dy = q[1] - g->cyl_c[1];
    if (!(dx * dx + dy * dy < g->cyl_r2)) return 0;
  }
  return 1;
}

/* The two transverse axes of driving axis m, in increasing order. */
static void transverse_axes(int m, int *a, int *b) {
  *a = (m == 0) ? 1 : 0;
  *b = (m == 2) ? 1 : 2;
}

/* Value of the volume interpolated at a sample point q on plane q_m: the sum
   over the 2 x 2 voxels of the plane whose indices bracket q on the two
   transverse axes (Eq. 7), each weighted by the product of the two axes'
   kernels (Eq. 12). */
static double plane_interp(const gjo_geom *g, const void *vol, int dt, int m, const double *q) {
  int a, b;
  transverse_axes(m, &a, &b);
  const long long base_a = (long long)floor(q[a]), base_b = (long long)floor(q[b]);
  double sum = 0.0;
  for (long long ja = base_a; ja <= base_a + 1; ++ja) {
    const double ha = kernel_1d(g->weight, q[a] - (double)ja);
    for (long long jb = base_b; jb <= base_b + 1; ++jb) {
      const double hb = kernel_1d(g->weight, q[b] - (double)jb);
      long long j[3];
      j[m] = (long long)q[m];
      j[a] = ja;
      j[b] = jb;
      sum += (ha * hb) * voxel(g, vol, dt, j);
    }
  }
  return sum;
}

/* One ray of the forward projection (Algorithm 1): the interpolated values
   at the ray's samples on the planes 0 .. N_m - 1 of its driving axis,
   summed and scaled by the length of one plane step. */
static double ray_forward(const gjo_geom *g, const void *vol, int dt, int view, int iu, int iv,
                          long long *count) {
  gjo_ray ray;
  ray_setup(g, view, iu, iv, &ray);
  if (count) *count = 0;
  if (!ray.ok) return 0.0;
  double sum = 0.0;
  long long n = 0;
  for (int i = 0; i < g->n[ray.m]; ++i) {
    double q[3];
    if (!plane_point(g, &ray, i, q)) continue;
    sum += plane_interp(g, vol, dt, ray.m, q);
    ++n;
  }
  if (count) *count = n;
  return ray.len * sum;
}

/* The transpose of ray_forward for one ray: each sample's 2 x 2 in-plane
   voxels receive y times the step length times their kernel weights. */
static void ray_adjoint(const gjo_geom *g, double y, int view, int iu, int iv, double *vol) {
  gjo_ray ray;
  ray_setup(g, view, iu, iv, &ray);
  if (!ray.ok || y == 0.0) return;
  const double scaled = ray.len * y;
  for (int i = 0; i < g->n[ray.m]; ++i) {
    double q[3];
    if (!plane_point(g, &ray, i, q)) continue;
    int a, b;
    transverse_axes(ray.m, &a, &b);
    const long long base_a = (long long)floor(q[a]), base_b = (long long)floor(q[b]);
    for (long long ja = base_a; ja <= base_a + 1; ++ja) {
      const double ha = kernel_1d(g->weight, q[a] - (double)ja);
      for (long long jb = base_b; jb <= base_b + 1; ++jb) {
        const double hb = kernel_1d(g->weight, q[b] - (double)jb);
        long long j[3];
        j[ray.m] = i;
        j[a] = ja;
        j[b] = jb;
        int in = 1;
        for (int k = 0; k < 3; ++k) in &= (j[k] >= 0 && j[k] < g->n[k]);
        if (!in) continue;
        const size_t idx =
            ((size_t)j[0] * (size_t)g->n[1] + (size_t)j[1]) * (size_t)g->n[2] + (size_t)j[2];
        vol[idx] += scaled * (ha * hb);
      }
    }
  }
}

static int make_geom(gjo_geom *g, const int *shape, const double *voxel_size,
                     const double *center, int beam, int n_views, const double *views, int n_u,
                     int n_v, int flags, int weight) {
  if (!shape || !voxel_size || !center || !views) return -1;
  for (int k = 0; k < 3; ++k) {
    if (shape[k] <= 0 || !(voxel_size[k] > 0.0)) return -1;
    g->n[k] = shape[k];
    g->vs[k] = voxel_size[k];
    g->ctr[k] = center[k];
  }
  if (n_views <= 0 || n_u <= 0 || n_v <= 0) return -1;
  if (beam != GJO_CONE && beam != GJO_PARALLEL) return -1;
  if (weight != GJO_W_LINEAR && weight != GJO_W_SPLINE) return -1;
  g->beam = beam;
  g->n_views = n_views;
  g->n_u = n_u;
  g->n_v = n_v;
  g->views = views;
  g->weight = weight;
  if (flags & ~GJO_CLIP_CYLINDER) return -1;
  g->clip = (flags & GJO_CLIP_CYLINDER) != 0;
  g->cyl_c[0] = 0.5 * (double)(g->n[0] - 1);
  g->cyl_c[1] = 0.5 * (double)(g->n[1] - 1);
  const double rad = 0.5 * (double)(g->n[0] < g->n[1] ? g->n[0] : g->n[1]);
  g->cyl_r2 = rad * rad;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Public entry points (plain C ABI for ctypes).                         */
/* ------------------------------------------------------------------ */

int gjo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void gjo_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Forward projection of the whole sinogram. vol: n0*n1*n2 (C order, f64 if
   vol_dt == 0, f32 if 1); sino: n_views*n_u*n_v doubles, v fastest. */
int gjo_forward(const int *shape, const double *voxel_size, const double *center, int beam,
                int n_views, const double *views, int n_u, int n_v, int flags, int weight,
                const void *vol, int vol_dt, double *sino) {
  gjo_geom g;
  if (make_geom(&g, shape, voxel_size, center, beam, n_views, views, n_u, n_v, flags, weight) != 0 ||
      !vol || !sino)
    return -1;
  const long long n_rays = (long long)n_views * n_u * n_v;
#pragma omp parallel for schedule(dynamic, 64)
  for (long long r = 0; r < n_rays; ++r) {
    int view = (int)(r / ((long long)n_u * n_v));
    int rem = (int)(r % ((long long)n_u * n_v));
    sino[r] = ray_forward(&g, vol, vol_dt, view, rem / n_v, rem % n_v, NULL);
  }
  return 0;
}

/* Forward projection of a list of rays: rays = n_rays x (view, iu, iv). */
int gjo_forward_rays(const int *shape, const double *voxel_size, const double *center, int beam,
                     int n_views, const double *views, int n_u, int n_v, int flags, int weight,
                     const void *vol, int vol_dt, long long n_rays, const int *rays,
                     double *out, long long *counts) {
  gjo_geom g;
  if (make_geom(&g, shape, voxel_size, center, beam, n_views, views, n_u, n_v, flags, weight) != 0 ||
      !vol || !rays || !out)
    return -1;
  for (long long r = 0; r < n_rays; ++r) {
    const int *q = rays + 3 * r;
    if (q[0] < 0 || q[0] >= n_views || q[1] < 0 || q[1] >= n_u || q[2] < 0 || q[2] >= n_v)
      return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (long long r = 0; r < n_rays; ++r) {
    const int *q = rays + 3 * r;
    long long c = 0;
    out[r] = ray_forward(&g, vol, vol_dt, q[0], q[1], q[2], &c);
    if (counts) counts[r] = c;
  }
  return 0;
}

/* Adjoint (transpose) of gjo_forward: vol = A^T sino, vol overwritten (f64).
   Views are split over threads, each accumulating into a private volume;
   the private volumes are summed in thread order. */
int gjo_adjoint(const int *shape, const double *voxel_size, const double *center, int beam,
                int n_views, const double *views, int n_u, int n_v, int flags, int weight,
                const double *sino, double *vol) {
  gjo_geom g;
  if (make_geom(&g, shape, voxel_size, center, beam, n_views, views, n_u, n_v, flags, weight) != 0 ||
      !vol || !sino)
    return -1;
  const size_t nvox = (size_t)g.n[0] * g.n[1] * g.n[2];
  memset(vol, 0, nvox * sizeof(double));
  int nt = gjo_num_threads();
  if ((size_t)nt * nvox * sizeof(double) > ((size_t)8 << 30)) nt = 1;
  double **priv = (double **)calloc((size_t)nt, sizeof(double *));
  if (!priv) return -2;
  for (int t = 0; t < nt; ++t) {
    priv[t] = (double *)calloc(nvox, sizeof(double));
    if (!priv[t]) {
      for (int u = 0; u < t; ++u) free(priv[u]);
      free(priv);
      return -2;
    }
  }
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
    for (int view = 0; view < n_views; ++view)
      for (int iu = 0; iu < n_u; ++iu)
        for (int iv = 0; iv < n_v; ++iv)
          ray_adjoint(&g, sino[((size_t)view * n_u + iu) * n_v + iv], view, iu, iv, priv[t]);
  }
  for (int t = 0; t < nt; ++t) {
    for (size_t i = 0; i < nvox; ++i) vol[i] += priv[t][i];
    free(priv[t]);
  }
  free(priv);
  return 0;
}

/* Number of in-volume samples (ray, plane) over the whole sinogram. */
long long gjo_count_samples(const int *shape, const double *voxel_size, const double *center,
                            int beam, int n_views, const double *views, int n_u, int n_v, int flags) {
  gjo_geom g;
  if (make_geom(&g, shape, voxel_size, center, beam, n_views, views, n_u, n_v, flags, 0) != 0)
    return -1;
  const long long n_rays = (long long)n_views * n_u * n_v;
  long long total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
  for (long long r = 0; r < n_rays; ++r) {
    int view = (int)(r / ((long long)n_u * n_v));
    int rem = (int)(r % ((long long)n_u * n_v));
    gjo_ray ray;
    ray_setup(&g, view, rem / n_v, rem % n_v, &ray);
    if (!ray.ok) continue;
    for (int i = 0; i < g.n[ray.m]; ++i) {
      double q[3];
      total += plane_point(&g, &ray, i, q);
    }
  }
  return total;
}

/* Per-ray driving axis and step length (for tests of the setup step). */
int gjo_ray_info(const int *shape, const double *voxel_size, const double *center, int beam,
                 int n_views, const double *views, int n_u, int n_v, int flags, int view, int iu, int iv,
                 int *m_out, double *len_out, double *rt_out) {
  gjo_geom g;
  if (make_geom(&g, shape, voxel_size, center, beam, n_views, views, n_u, n_v, flags, 0) != 0)
    return -1;
  gjo_ray ray;
  ray_setup(&g, view, iu, iv, &ray);
  if (m_out) *m_out = ray.ok ? ray.m : -1;
  if (len_out) *len_out = ray.len;
  if (rt_out)
    for (int k = 0; k < 3; ++k) rt_out[k] = ray.rt[k];
  return 0;
}
