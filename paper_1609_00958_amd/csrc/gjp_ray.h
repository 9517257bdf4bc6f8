// gjp_ray.h -- per-ray setup and per-sample weights of the generalized Joseph
// projector, shared by the host sample count and every device kernel.
//
// The ray setup (Eqs. 1-5, Algorithm 1 setup) runs in double precision and
// yields the driving axis, the exact sample range and single-precision
// coefficients of the two transverse coordinates; the sampling loop
// (Eqs. 6-13) then runs in single precision. The forward and the adjoint
// kernels evaluate a sample through the same `sample_axis` function, so the
// adjoint reproduces the forward's weights bit for bit.
//
// This file must be compiled without floating-point contraction
// (-ffp-contract=off): the driving axis and the sample range decide integer
// outcomes and have to agree between host and device, operation for
// operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GJP_HD __host__ __device__ __forceinline__

namespace gjp {

enum { W_LINEAR = 0, W_SPLINE = 1 };
enum { BEAM_CONE = 0, BEAM_PARALLEL = 1 };

// Scan geometry of one volume as the kernels see it (grid units).
struct GridGeom {
  int n[3];        // voxels per axis
  double vs[3];    // voxel size (world units per grid step)
  float hi[3];     // largest float below n[k]: upper clamp of sample coordinates
  int beam;
  // Cylinder clipping of the sample range (Sec. IV-C): a sample also needs
  // (p_0 - cyl[0])^2 + (p_1 - cyl[1])^2 < cyl_r2 (the cylinder inscribed in
  // the grid box, axis along axis 2).
  int clip;
  double cyl[2];
  double cyl_r2;
};

// Row pitch (elements) of the zero-padded volume copy: n2 + 2 rounded up to
// an even count, so that every row starts on a 4-byte boundary for 16-bit
// storage. The extra column holds zeros and is never sampled.
GJP_HD long long padded_pitch(int n2) { return (long long)((n2 + 3) & ~1); }

// Result of the per-ray setup.
struct RaySetup {
  int m;            // driving axis (Eq. 3)
  int ta, tb;       // transverse axes, ta < tb
  int i0, i1;       // sample planes [i0, i1) along m; empty if i0 >= i1
  float ca, ga;     // p_ta(i) = fma(i, ga, ca)
  float cb, gb;     // p_tb(i) = fma(i, gb, cb)
  float scale;      // world-space length of one plane step, || r~ * voxel_size ||
};

// Sample predicate on one transverse axis: the coordinate of plane i on the
// line s + (i - s_m) g (Eq. 6 with o = -s_m) lies in the zero-padded domain.
GJP_HD bool inside_axis(double s_k, double neg_sm, double g_k, double di, int n_k) {
  const double p = s_k + (neg_sm + di) * g_k;
  return p > -1.0 && p < (double)n_k;
}
GJP_HD bool inside_axis(double s_k, double neg_sm, double g_k, int i, int n_k) {
  return inside_axis(s_k, neg_sm, g_k, (double)i, n_k);
}

GJP_HD bool inside_both(const double* s, double neg_sm, const double* g, int a, int b,
                        const int* n, int i) {
  return inside_axis(s[a], neg_sm, g[a], i, n[a]) && inside_axis(s[b], neg_sm, g[b], i, n[b]);
}

// Real interval of planes where axis k stays inside (-1, n_k), widened to
// integers and clamped to [lo_i, hi_i).
GJP_HD void axis_interval(double s_k, double s_m, double g_k, int n_k, double& lo, double& hi) {
  if (g_k == 0.0) {
    const bool in = s_k > -1.0 && s_k < (double)n_k;
    lo = in ? -1.0e300 : 1.0e300;
    hi = in ? 1.0e300 : -1.0e300;
    return;
  }
  const double t0 = s_m + (-1.0 - s_k) / g_k;
  const double t1 = s_m + ((double)n_k - s_k) / g_k;
  lo = t0 < t1 ? t0 : t1;
  hi = t0 < t1 ? t1 : t0;
}

// The line of pixel (iu, iv) of a view given in grid units (v[0..2] = source
// (cone) or direction (parallel), v[3..5] = det00, v[6..8] = du,
// v[9..11] = dv): origin s (Eq. 2), driving axis m (Eq. 3, ties to the lowest
// axis), transverse axes a < b, slopes g = r / r_m (Eq. 4) and the
// world-space length of one plane step. False for a ray without direction.
GJP_HD bool ray_line(const double* __restrict__ v, const GridGeom& G, int iu, int iv, double* s,
                     double* g, int& m, int& a, int& b, float& scale) {
  double d[3], r[3];
  for (int k = 0; k < 3; ++k) d[k] = v[3 + k] + (double)iu * v[6 + k] + (double)iv * v[9 + k];
  if (G.beam == BEAM_CONE) {
    for (int k = 0; k < 3; ++k) {
      s[k] = v[k];
      r[k] = d[k] - v[k];  // Eq. 2
    }
  } else {
    for (int k = 0; k < 3; ++k) {
      s[k] = d[k];
      r[k] = v[k];
    }
  }
  m = 0;
  if (fabs(r[1]) > fabs(r[m])) m = 1;
  if (fabs(r[2]) > fabs(r[m])) m = 2;
  a = (m == 0) ? 1 : 0;
  b = (m == 2) ? 1 : 2;
  scale = 0.0f;
  if (r[m] == 0.0) return false;
  g[a] = r[a] / r[m];
  g[b] = r[b] / r[m];
  g[m] = 1.0;
  double q = 0.0;
  for (int k = 0; k < 3; ++k) q += (g[k] * G.vs[k]) * (g[k] * G.vs[k]);
  scale = (float)sqrt(q);
  return true;
}

// Per-ray setup for pixel (iu, iv): the line above, single-precision
// coefficients of the transverse coordinates and the exact sample range.
GJP_HD void ray_setup(const double* __restrict__ v, const GridGeom& G, int iu, int iv,
                      RaySetup& R) {
  double s[3], g[3];
  int m, a, b;
  float scale;
  const bool dir = ray_line(v, G, iu, iv, s, g, m, a, b, scale);
  R.m = m;
  R.ta = a;
  R.tb = b;
  R.i0 = 0;
  R.i1 = 0;
  R.ca = R.ga = R.cb = R.gb = 0.0f;
  R.scale = scale;
  if (!dir) return;  // no direction: no samples
  const double neg_sm = -s[m];  // Eq. 5
  R.ca = (float)(s[a] + neg_sm * g[a]);
  R.ga = (float)g[a];
  R.cb = (float)(s[b] + neg_sm * g[b]);
  R.gb = (float)g[b];

  // Sample range: analytic estimate, then the exact predicate at the ends.
  // Box and cylinder are convex, so the samples form one run.
  const int nm = G.n[m];
  double lo_a, hi_a, lo_b, hi_b;
  axis_interval(s[a], s[m], g[a], G.n[a], lo_a, hi_a);
  axis_interval(s[b], s[m], g[b], G.n[b], lo_b, hi_b);
  double lo = lo_a > lo_b ? lo_a : lo_b;
  double hi = hi_a < hi_b ? hi_a : hi_b;
  lo = lo < -2.0 ? -2.0 : (lo > (double)nm + 1.0 ? (double)nm + 1.0 : lo);
  hi = hi < -2.0 ? -2.0 : (hi > (double)nm + 1.0 ? (double)nm + 1.0 : hi);
  const double sa = s[a], sb = s[b], ga = g[a], gb = g[b];
  if (G.clip) {
    // the cylinder cross-section coordinates (p_0, p_1) are affine in the
    // plane index: p = u + w i; the chord is where |u + w i - c|^2 < r^2
    double u0, w0, u1, w1;
    if (m == 0) {
      u0 = 0.0; w0 = 1.0; u1 = sa + neg_sm * ga; w1 = ga;
    } else if (m == 1) {
      u0 = sa + neg_sm * ga; w0 = ga; u1 = 0.0; w1 = 1.0;
    } else {
      u0 = sa + neg_sm * ga; w0 = ga; u1 = sb + neg_sm * gb; w1 = gb;
    }
    const double e0 = u0 - G.cyl[0], e1 = u1 - G.cyl[1];
    const double qa = w0 * w0 + w1 * w1, qb = w0 * e0 + w1 * e1;
    const double qc = e0 * e0 + e1 * e1 - G.cyl_r2;
    double clo = -1.0e300, chi = 1.0e300;
    if (qa > 0.0) {
      const double disc = qb * qb - qa * qc;
      if (disc > 0.0) {
        const double sq = sqrt(disc);
        clo = (-qb - sq) / qa;
        chi = (-qb + sq) / qa;
      } else {
        clo = 1.0;  // empty (the exact predicate decides the ends below)
        chi = -1.0;
      }
    } else if (qc >= 0.0) {
      clo = 1.0;
      chi = -1.0;
    }
    // widened by a plane on each side; the exact predicate trims the ends
    lo = lo > clo - 1.0 ? lo : clo - 1.0;
    hi = hi < chi + 1.0 ? hi : chi + 1.0;
    if (hi < lo) hi = lo;
  }
  int i0 = (int)floor(lo) + 1;
  int i1 = (int)ceil(hi);
  i0 = i0 < 0 ? 0 : (i0 > nm ? nm : i0);
  i1 = i1 < 0 ? 0 : (i1 > nm ? nm : i1);
  if (i1 < i0) i1 = i0;
  // inside_both's predicate (and the cylinder test) on the plane index held
  // as an exact double next to the integer (same arithmetic; keeps the
  // device register count low)
  const int na = G.n[a], nb = G.n[b];
  const int clip = G.clip;
  const double cx = G.cyl[0], cy = G.cyl[1], cr2 = G.cyl_r2;
  auto inside = [=](double di) {
    const double pa = sa + (neg_sm + di) * ga, pb = sb + (neg_sm + di) * gb;
    if (!(pa > -1.0 && pa < (double)na && pb > -1.0 && pb < (double)nb)) return false;
    if (!clip) return true;
    const double px = (m == 0) ? di : pa;
    const double py = (m == 0) ? pa : ((m == 1) ? di : pb);
    const double dx = px - cx, dy = py - cy;
    return dx * dx + dy * dy < cr2;
  };
  double d0 = (double)i0;
  while (i0 < i1 && !inside(d0)) {
    ++i0;
    d0 += 1.0;
  }
  d0 = (double)(i0 - 1);
  while (i0 > 0 && inside(d0)) {
    --i0;
    d0 -= 1.0;
  }
  if (i1 < i0) i1 = i0;
  double d1 = (double)(i1 - 1);
  while (i1 > i0 && !inside(d1)) {
    --i1;
    d1 -= 1.0;
  }
  d1 = (double)i1;
  while (i1 < nm && inside(d1)) {
    ++i1;
    d1 += 1.0;
  }
  R.i0 = i0;
  R.i1 = i1;
}

// Eq. 13 / Eq. 14
template <int WF>
__device__ __forceinline__ float weight_fn(float d) {
  if constexpr (WF == W_SPLINE) {
    // 1 - 3 d^2 + 2 d^3 = 1 + d^2 (2 d - 3)
    return __builtin_fmaf(d * d, __builtin_fmaf(2.0f, d, -3.0f), 1.0f);
  } else {
    return 1.0f - d;
  }
}

// One transverse coordinate of the sample on plane `fi`: position, clamp to
// the padded domain [-1, n), floor, and the complementary weight pair
// (Eqs. 10-11). The clamp only acts where single-precision rounding leaves a
// coordinate outside the double-precision sample range.
template <int WF>
__device__ __forceinline__ void sample_axis_floor(float fi, float g, float c, float hi, float& f,
                                                  float& w_fl, float& w_cl) {
  float p = __builtin_fmaf(fi, g, c);
  p = __builtin_amdgcn_fmed3f(p, -1.0f, hi);
  f = __builtin_floorf(p);
  const float d = p - f;
  w_fl = weight_fn<WF>(d);
  // complementary weight (Eq. 12); for the linear weight 1 - (1 - d) is d
  if constexpr (WF == W_LINEAR)
    w_cl = d;
  else
    w_cl = 1.0f - w_fl;
}

// The same with the floor as an integer.
template <int WF>
__device__ __forceinline__ void sample_axis(float fi, float g, float c, float hi, int& i_fl,
                                            float& w_fl, float& w_cl) {
  float f;
  sample_axis_floor<WF>(fi, g, c, hi, f, w_fl, w_cl);
  i_fl = (int)f;
}

}  // namespace gjp
