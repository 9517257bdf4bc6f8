/* Sanitizer driver of the FP64 oracle (built with -fsanitize=address,undefined
   by tests/test_sanitizers_cpu.py). Runs the oracle's entry points on small
   cone, parallel, clipped and degenerate geometries, including grids of one
   voxel and rays that miss, and checks the dot-product identity
   <A x, y> = <x, A^T y>. Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int gjo_views_circular_cone(int, double, double, double, double, int, int, double *);
int gjo_views_parallel(int, double, double, int, int, double *);
int gjo_forward(const int *, const double *, const double *, int, int, const double *, int, int,
                int, int, const void *, int, double *);
int gjo_forward_rays(const int *, const double *, const double *, int, int, const double *, int,
                     int, int, int, const void *, int, long long, const int *, double *,
                     long long *);
int gjo_adjoint(const int *, const double *, const double *, int, int, const double *, int, int,
                int, int, const double *, double *);
long long gjo_count_samples(const int *, const double *, const double *, int, int, const double *,
                            int, int, int);
int gjo_ray_info(const int *, const double *, const double *, int, int, const double *, int, int,
                 int, int, int, int, int *, double *, double *);
void gjo_set_num_threads(int);

static unsigned long long rng = 88172645463325252ull;
static double urand(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(const int *shape, int beam, int n_views, int n_u, int n_v, int flags,
                    int weight, const double *views) {
  const double vs[3] = {1.0, 1.25, 0.8}, ctr[3] = {0.5, -0.25, 0.0};
  const size_t nvox = (size_t)shape[0] * shape[1] * shape[2];
  const size_t nray = (size_t)n_views * n_u * n_v;
  double *x = malloc(nvox * sizeof(double)), *y = malloc(nray * sizeof(double));
  double *ax = malloc(nray * sizeof(double)), *aty = malloc(nvox * sizeof(double));
  float *xf = malloc(nvox * sizeof(float));
  int *rays = malloc(3 * 16 * sizeof(int));
  double *out = malloc(16 * sizeof(double));
  long long *cnt = malloc(16 * sizeof(long long));
  int bad = 0;
  for (size_t i = 0; i < nvox; ++i) {
    x[i] = urand();
    xf[i] = (float)x[i];
  }
  for (size_t i = 0; i < nray; ++i) y[i] = urand() - 0.5;
  if (gjo_forward(shape, vs, ctr, beam, n_views, views, n_u, n_v, flags, weight, x, 0, ax)) bad = 1;
  if (gjo_adjoint(shape, vs, ctr, beam, n_views, views, n_u, n_v, flags, weight, y, aty)) bad = 1;
  double lhs = 0.0, rhs = 0.0, scale = 0.0;
  for (size_t i = 0; i < nray; ++i) {
    lhs += ax[i] * y[i];
    scale += fabs(ax[i] * y[i]);
  }
  for (size_t i = 0; i < nvox; ++i) rhs += x[i] * aty[i];
  if (fabs(lhs - rhs) > 1e-12 * (scale + 1e-300)) bad = 1;
  for (int r = 0; r < 16; ++r) {
    rays[3 * r] = (int)(urand() * n_views);
    rays[3 * r + 1] = (int)(urand() * n_u);
    rays[3 * r + 2] = (int)(urand() * n_v);
  }
  if (gjo_forward_rays(shape, vs, ctr, beam, n_views, views, n_u, n_v, flags, weight, xf, 1, 16,
                       rays, out, cnt))
    bad = 1;
  if (gjo_count_samples(shape, vs, ctr, beam, n_views, views, n_u, n_v, flags) < 0) bad = 1;
  int m;
  double len, rt[3];
  if (gjo_ray_info(shape, vs, ctr, beam, n_views, views, n_u, n_v, flags, 0, n_u - 1, n_v - 1,
                   &m, &len, rt))
    bad = 1;
  free(x); free(y); free(ax); free(aty); free(xf); free(rays); free(out); free(cnt);
  return bad;
}

int main(void) {
  int bad = 0;
  gjo_set_num_threads(2);
  const int shapes[4][3] = {{1, 1, 1}, {7, 5, 9}, {12, 1, 6}, {10, 11, 8}};
  for (int s = 0; s < 4; ++s)
    for (int beam = 0; beam < 2; ++beam)
      for (int flags = 0; flags < 2; ++flags)
        for (int weight = 0; weight < 2; ++weight) {
          const int n_views = 5, n_u = 6, n_v = 7;
          double views[5 * 12];
          if (beam == 0)
            gjo_views_circular_cone(n_views, 30.0, 45.0, 1.7, 1.3, n_u, n_v, views);
          else
            gjo_views_parallel(n_views, 1.9, 1.4, n_u, n_v, views);
          /* tilt the last view so that every axis can drive */
          views[12 * 4 + 9] = 0.9;
          views[12 * 4 + 2] = beam == 0 ? 25.0 : 0.7;
          bad |= run_case(shapes[s], beam, n_views, n_u, n_v, flags, weight, views);
        }
  /* a degenerate ray: the source on the pixel */
  double v[12] = {0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 5.0, 0.0, 0.0, 0.0, 5.0, 0.0};
  const int sh[3] = {4, 4, 4};
  bad |= run_case(sh, 0, 1, 2, 2, 0, 0, v);
  /* invalid arguments are rejected without touching memory */
  const double one[3] = {1, 1, 1}, zero[3] = {0, 0, 0};
  const int nil[3] = {0, 4, 4};
  double dummy[12] = {0};
  if (gjo_count_samples(nil, one, zero, 0, 1, dummy, 1, 1, 0) >= 0) bad = 1;
  if (gjo_views_circular_cone(0, 1.0, 2.0, 1.0, 1.0, 1, 1, dummy) == 0) bad = 1;
  printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
  return bad;
}
