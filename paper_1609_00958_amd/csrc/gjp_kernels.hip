// gjp_kernels.hip -- gfx950 kernels of the generalized Joseph projector.
//
// Forward (Algorithm 1): one lane per detector pixel. A 256-thread workgroup
// covers a tile of (64 >> k) x (4 << k) pixels; within a wavefront the fast
// lane index runs along detector v, the direction parallel to the rotation
// axis and to the fastest volume index n2. For a circular trajectory the
// driving axis is then 0 or 1 (never the fastest index, as the paper's
// Algorithm 1 caption recommends for cache efficiency), the 64 lanes of a
// wavefront share the same transverse row on every plane, and the two row
// reads of a sample are contiguous voxel pairs (z, z+1) fetched as one 8-byte
// (FP32) or 4-byte (16-bit) load. The volume is read from a zero-padded copy
// (one voxel on every side), so the sampling loop has no bounds tests.
//
// Adjoint: exact transpose of the forward. A table pass stores, per ray of a
// chunk of views, the setup the forward computes (driving axis, sample range,
// single-precision coefficients) and the sinogram value times the step length.
// A splat pass gives each workgroup a voxel tile in LDS; the rays of the view
// chunk that can touch the tile recompute their samples on the tile's planes
// with the same `sample_axis` code as the forward and add the weighted
// contributions into LDS (waves own disjoint planes, so the sum order is
// fixed). Each voxel is written to memory once per chunk; no global atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gjp_internal.h"

namespace gjp {

struct bf16_t {
  uint16_t bits;
};
struct f16_t {
  uint16_t bits;
};

typedef float f2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32a2 __attribute__((aligned(2)));

__device__ __forceinline__ void load_pair(const float* p, float& x0, float& x1) {
  const f2a4 v = *reinterpret_cast<const f2a4*>(p);
  x0 = v.x;
  x1 = v.y;
}
__device__ __forceinline__ void load_pair(const bf16_t* p, float& x0, float& x1) {
  const uint32_t u = *reinterpret_cast<const u32a2*>(p);
  x0 = __uint_as_float(u << 16);
  x1 = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void load_pair(const f16_t* p, float& x0, float& x1) {
  const uint32_t u = *reinterpret_cast<const u32a2*>(p);
  x0 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
  x1 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
}
__device__ __forceinline__ float load_one(const float* p) { return *p; }
__device__ __forceinline__ float load_one(const bf16_t* p) {
  return __uint_as_float((uint32_t)p->bits << 16);
}
__device__ __forceinline__ float load_one(const f16_t* p) {
  return (float)__builtin_bit_cast(_Float16, p->bits);
}

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs (each
// with its own L2); remap so that each XCD runs one contiguous range of tiles.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t X = 8;
  const uint32_t q = nb / X, r = nb % X;
  const uint32_t xcd = b % X, local = b / X;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

// ---------------------------------------------------------------------------
// Zero-padded copy: dst has (n0+2) x (n1+2) x (n2+2) elements.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void pad_kernel(const E* __restrict__ src, E* __restrict__ dst,
                                                  int n0, int n1, int n2) {
  const int z = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int x = blockIdx.z;
  const int p2 = n2 + 2;
  if (z >= p2) return;
  E val = 0;
  if (x >= 1 && x <= n0 && y >= 1 && y <= n1 && z >= 1 && z <= n2)
    val = src[((size_t)(x - 1) * n1 + (y - 1)) * n2 + (z - 1)];
  dst[((size_t)x * (n1 + 2) + y) * p2 + z] = val;
}

// ---------------------------------------------------------------------------
// Forward projection of one ray (Algorithm 1).
// ---------------------------------------------------------------------------
typedef float f2v __attribute__((ext_vector_type(2)));

// Row pair (z, z+1) at byte offset `off` of the padded volume, widened to FP32.
__device__ __forceinline__ void buf_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, const float*,
                                         float& x0, float& x1) {
  const f2v v = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  x0 = v.x;
  x1 = v.y;
}
__device__ __forceinline__ void buf_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, const bf16_t*,
                                         float& x0, float& x1) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  x0 = __uint_as_float(u << 16);
  x1 = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void buf_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, const f16_t*,
                                         float& x0, float& x1) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  x0 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
  x1 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
}

// Sampling loop for driving axes 0 and 1 on a padded volume below 4 GiB:
// 32-bit byte offsets into a buffer resource, two samples per iteration so
// that four row-pair loads are in flight per lane.
template <typename T, int WF>
__device__ __forceinline__ float fwd_loop_buf(const FwdArgs& a, const RaySetup& R) {
  constexpr uint32_t es = sizeof(T);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.vol_base), (short)0, (int)(uint32_t)a.vol_bytes, 0x00020000);
  const uint32_t Sm = (uint32_t)(R.m == 0 ? a.S0 : a.S1) * es;
  const int Sa = (int)((R.m == 0 ? a.S1 : a.S0) * (long long)es);
  const float h0 = a.G.hi[0], h1 = a.G.hi[1];
  const float hia = (R.m == 0) ? h1 : h0;
  const float hib = a.G.hi[2];
  // padded frame: (plane + 1, row + 1, col + 1)
  uint32_t off_m = (uint32_t)(R.i0 + 1) * Sm + (uint32_t)Sa + es;
  float acc = 0.0f;
  float fi = (float)R.i0;
  int i = R.i0;
  for (; i + 1 < R.i1; i += 2) {
    int ia0, ib0, ia1, ib1;
    float wfa0, wca0, wfb0, wcb0, wfa1, wca1, wfb1, wcb1;
    sample_axis<WF>(fi, R.ga, R.ca, hia, ia0, wfa0, wca0);
    sample_axis<WF>(fi, R.gb, R.cb, hib, ib0, wfb0, wcb0);
    sample_axis<WF>(fi + 1.0f, R.ga, R.ca, hia, ia1, wfa1, wca1);
    sample_axis<WF>(fi + 1.0f, R.gb, R.cb, hib, ib1, wfb1, wcb1);
    const uint32_t o0 = (uint32_t)__mul24(ia0, Sa) + off_m + (uint32_t)ib0 * es;
    const uint32_t o1 = (uint32_t)__mul24(ia1, Sa) + off_m + Sm + (uint32_t)ib1 * es;
    float v00, v01, v10, v11, u00, u01, u10, u11;
    buf_pair(rs, o0, (const T*)nullptr, v00, v01);
    buf_pair(rs, o0 + (uint32_t)Sa, (const T*)nullptr, v10, v11);
    buf_pair(rs, o1, (const T*)nullptr, u00, u01);
    buf_pair(rs, o1 + (uint32_t)Sa, (const T*)nullptr, u10, u11);
    acc = __builtin_fmaf(wfa0, __builtin_fmaf(wfb0, v00, wcb0 * v01), acc);
    acc = __builtin_fmaf(wca0, __builtin_fmaf(wfb0, v10, wcb0 * v11), acc);
    acc = __builtin_fmaf(wfa1, __builtin_fmaf(wfb1, u00, wcb1 * u01), acc);
    acc = __builtin_fmaf(wca1, __builtin_fmaf(wfb1, u10, wcb1 * u11), acc);
    fi += 2.0f;
    off_m += 2 * Sm;
  }
  if (i < R.i1) {
    int ia0, ib0;
    float wfa0, wca0, wfb0, wcb0;
    sample_axis<WF>(fi, R.ga, R.ca, hia, ia0, wfa0, wca0);
    sample_axis<WF>(fi, R.gb, R.cb, hib, ib0, wfb0, wcb0);
    const uint32_t o0 = (uint32_t)__mul24(ia0, Sa) + off_m + (uint32_t)ib0 * es;
    float v00, v01, v10, v11;
    buf_pair(rs, o0, (const T*)nullptr, v00, v01);
    buf_pair(rs, o0 + (uint32_t)Sa, (const T*)nullptr, v10, v11);
    acc = __builtin_fmaf(wfa0, __builtin_fmaf(wfb0, v00, wcb0 * v01), acc);
    acc = __builtin_fmaf(wca0, __builtin_fmaf(wfb0, v10, wcb0 * v11), acc);
  }
  return acc;
}

// Row pair at (scalar byte offset + lane byte offset), for the row-uniform loop.
__device__ __forceinline__ void buf_pair_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                           const float*, float& x0, float& x1) {
  const f2v v = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  x0 = v.x;
  x1 = v.y;
}
__device__ __forceinline__ void buf_pair_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                           const bf16_t*, float& x0, float& x1) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  x0 = __uint_as_float(u << 16);
  x1 = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void buf_pair_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                           const f16_t*, float& x0, float& x1) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  x0 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
  x1 = (float)__builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Sampling loop for a wavefront whose rays all share the driving axis (0 or
// 1) and the in-plane coefficients (ca, ga): the row coordinate, its weights
// and the row offset of every plane are the same for all lanes. Lane l
// evaluates them for plane base + l of each block of 64 planes, and the loop
// broadcasts plane j's values with readlane; lanes only evaluate the axis-2
// coordinate. Each lane accumulates exactly the terms, in the same order and
// with the same arithmetic, as fwd_loop_buf, so the results are identical.
//
// m, ca and ga are the shared (wave-uniform) values; every one of the 64 lanes
// must be active, since each computes the row data of one plane.
template <typename T, int WF>
__device__ __forceinline__ float fwd_loop_rowuniform(const FwdArgs& a, const RaySetup& R, int m,
                                                     float ca, float ga, int lo, int hi) {
  constexpr uint32_t es = sizeof(T);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.vol_base), (short)0, (int)(uint32_t)a.vol_bytes, 0x00020000);
  const uint32_t Sm = (uint32_t)(m == 0 ? a.S0 : a.S1) * es;
  const uint32_t Sa = (uint32_t)((m == 0 ? a.S1 : a.S0) * (long long)es);
  const float hia = (m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  const int lane = (int)(threadIdx.x & 63);
  float acc = 0.0f;
  for (int base = lo; base < hi; base += 64) {
    int ia_l;
    float wfa_l, wca_l;
    sample_axis<WF>((float)(base + lane), ga, ca, hia, ia_l, wfa_l, wca_l);
    // byte offset of (plane + 1, row + 1, 0) in the padded volume
    const uint32_t row_l = (uint32_t)(base + lane + 1) * Sm + (uint32_t)(ia_l + 1) * Sa;
    const int cnt = min(64, hi - base);
    // two planes per iteration: both planes' loads are issued before either
    // is consumed; each plane still contributes in order and only inside the
    // lane's own sample range
    for (int j = 0; j < cnt; j += 2) {
      const int i = base + j;
      const bool two = j + 1 < cnt;
      const uint32_t row0 = (uint32_t)__builtin_amdgcn_readlane((int)row_l, j);
      const float wfa0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wfa_l), j));
      const float wca0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wca_l), j));
      const uint32_t row1 = (uint32_t)__builtin_amdgcn_readlane((int)row_l, j + 1);
      const float wfa1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wfa_l), j + 1));
      const float wca1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wca_l), j + 1));
      const bool in0 = i >= R.i0 && i < R.i1;
      const bool in1 = two && i + 1 >= R.i0 && i + 1 < R.i1;
      int ib0, ib1;
      float wfb0, wcb0, wfb1, wcb1;
      sample_axis<WF>((float)i, R.gb, R.cb, hib, ib0, wfb0, wcb0);
      sample_axis<WF>((float)(i + 1), R.gb, R.cb, hib, ib1, wfb1, wcb1);
      const uint32_t vo0 = (uint32_t)(ib0 + 1) * es;
      const uint32_t vo1 = (uint32_t)(ib1 + 1) * es;
      float v00 = 0.f, v01 = 0.f, v10 = 0.f, v11 = 0.f;
      float u00 = 0.f, u01 = 0.f, u10 = 0.f, u11 = 0.f;
      if (in0) {
        buf_pair_s(rs, vo0, row0, (const T*)nullptr, v00, v01);
        buf_pair_s(rs, vo0, row0 + Sa, (const T*)nullptr, v10, v11);
      }
      if (in1) {
        buf_pair_s(rs, vo1, row1, (const T*)nullptr, u00, u01);
        buf_pair_s(rs, vo1, row1 + Sa, (const T*)nullptr, u10, u11);
      }
      if (in0) {
        acc = __builtin_fmaf(wfa0, __builtin_fmaf(wfb0, v00, wcb0 * v01), acc);
        acc = __builtin_fmaf(wca0, __builtin_fmaf(wfb0, v10, wcb0 * v11), acc);
      }
      if (in1) {
        acc = __builtin_fmaf(wfa1, __builtin_fmaf(wfb1, u00, wcb1 * u01), acc);
        acc = __builtin_fmaf(wca1, __builtin_fmaf(wfb1, u10, wcb1 * u11), acc);
      }
    }
  }
  return acc;
}

// One ray per lane. All 64 lanes of the wavefront call this together; a lane
// whose pixel lies outside the detector (valid == false) takes part in the
// wavefront-wide steps with an empty sample range and stores nothing.
template <typename T, int WF, bool IDX64>
__device__ __forceinline__ void fwd_ray(const FwdArgs& a, int view, int iu, int iv, bool valid) {
  using Index = std::conditional_t<IDX64, long long, int>;
  RaySetup R;
  ray_setup(a.views + 12 * (size_t)view, a.G, iu, iv, R);
  if (!valid) R.i1 = R.i0;
  const T* __restrict__ base = static_cast<const T*>(a.vol);
  float acc = 0.0f;
  float fi = (float)R.i0;
  if constexpr (!IDX64) {
    // row-uniform wavefront: every lane with samples shares m (0 or 1), ca
    // and ga; the shared values are the first such lane's
    const bool has = R.i1 > R.i0;
    const uint64_t hv = __ballot(has);
    bool uniform = false;
    int lm = 2;
    float lca = 0.0f, lga = 0.0f;
    if (hv != 0) {
      const int leader = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)hv) - 1);
      lm = __builtin_amdgcn_readlane(R.m, leader);
      lca = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, R.ca), leader));
      lga = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, R.ga), leader));
      uniform = lm != 2 && __ballot(has && (R.m != lm || R.ca != lca || R.ga != lga)) == 0;
    }
    if (uniform) {
      const int lo = __builtin_amdgcn_readfirstlane(wave_min(has ? R.i0 : 0x7fffffff));
      const int hi = __builtin_amdgcn_readfirstlane(wave_max(has ? R.i1 : -1));
      acc = fwd_loop_rowuniform<T, WF>(a, R, lm, lca, lga, lo, hi);
      if (valid) a.sino[((size_t)view * a.n_u + iu) * a.n_v + iv] = acc * R.scale;
      return;
    }
  }
  if (R.m != 2) {
    if constexpr (!IDX64) {
      acc = fwd_loop_buf<T, WF>(a, R);
    } else {
      // transverse axes: ta (rows, strided) and 2 (contiguous pairs)
      const Index Sm = (Index)(R.m == 0 ? a.S0 : a.S1);
      const Index Sa = (Index)(R.m == 0 ? a.S1 : a.S0);
      const float hia = (R.m == 0) ? a.G.hi[1] : a.G.hi[0];
      const float hib = a.G.hi[2];
      Index off_m = (Index)R.i0 * Sm;
      for (int i = R.i0; i < R.i1; ++i) {
        int ia, ib;
        float wfa, wca, wfb, wcb;
        sample_axis<WF>(fi, R.ga, R.ca, hia, ia, wfa, wca);
        sample_axis<WF>(fi, R.gb, R.cb, hib, ib, wfb, wcb);
        const Index off = off_m + (Index)ia * Sa + (Index)ib;
        float v00, v01, v10, v11;
        load_pair(base + off, v00, v01);
        load_pair(base + off + Sa, v10, v11);
        acc = __builtin_fmaf(wfa, __builtin_fmaf(wfb, v00, wcb * v01), acc);
        acc = __builtin_fmaf(wca, __builtin_fmaf(wfb, v10, wcb * v11), acc);
        fi += 1.0f;
        off_m += Sm;
      }
    }
  } else {
    // driving axis 2: both transverse axes strided, four single loads
    const Index S0 = (Index)a.S0, S1 = (Index)a.S1;
    const float hia = a.G.hi[0], hib = a.G.hi[1];
    for (int i = R.i0; i < R.i1; ++i) {
      int ia, ib;
      float wfa, wca, wfb, wcb;
      sample_axis<WF>(fi, R.ga, R.ca, hia, ia, wfa, wca);
      sample_axis<WF>(fi, R.gb, R.cb, hib, ib, wfb, wcb);
      const Index off = (Index)i + (Index)ia * S0 + (Index)ib * S1;
      const float v00 = load_one(base + off);
      const float v01 = load_one(base + off + S1);
      const float v10 = load_one(base + off + S0);
      const float v11 = load_one(base + off + S0 + S1);
      acc = __builtin_fmaf(wfa, __builtin_fmaf(wfb, v00, wcb * v01), acc);
      acc = __builtin_fmaf(wca, __builtin_fmaf(wfb, v10, wcb * v11), acc);
      fi += 1.0f;
    }
  }
  if (valid) a.sino[((size_t)view * a.n_u + iu) * a.n_v + iv] = acc * R.scale;
}

template <typename T, int WF, bool IDX64>
__device__ __forceinline__ void fwd_tile(const FwdArgs& a, int view, int t) {
  const int tu = t / a.tiles_v;
  const int tv = t - tu * a.tiles_v;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int k = a.tile_v_log2;
  const int rows = 64 >> k;
  const int iv = (tv << k) + (lane & ((1 << k) - 1));
  const int iu = tu * (4 * rows) + wave * rows + (lane >> k);
  const bool valid = iu < a.n_u && iv < a.n_v;
  fwd_ray<T, WF, IDX64>(a, view, valid ? iu : 0, valid ? iv : 0, valid);
}

template <typename T, int WF, bool IDX64>
__global__ __launch_bounds__(256) void fwd_kernel(const FwdArgs a) {
  uint32_t b = blockIdx.x;
  if (a.remap) b = xcd_remap(b, gridDim.x);
  const int view = (int)(b / (uint32_t)a.tiles_per_view);
  const int t = (int)(b - (uint32_t)view * (uint32_t)a.tiles_per_view);
  fwd_tile<T, WF, IDX64>(a, view, t);
}

// ---------------------------------------------------------------------------
// Adjoint pass 1: per-ray table for views [view0, view0 + n_chunk).
// General layout, two float4 per ray: {m | i0 << 2 | i1 << 17, ca, ga, cb},
// {gb, y * scale, 0, 0}. Column layout (see adj_gather_sep_kernel): one float4
// per ray {m | i0 << 2 | i1 << 17, cb, gb, y * scale} and one per detector
// column {m, ca, ga, 0}.
// mask[c] collects the driving axes that have samples in view view0 + c.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void adj_table_kernel(const double* __restrict__ views,
                                                        const GridGeom G,
                                                        const float* __restrict__ sino, int n_u,
                                                        int n_v, int view0, long long n_rays,
                                                        int separable, float4* __restrict__ table,
                                                        float4* __restrict__ cols,
                                                        int* __restrict__ mask) {
  const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long per_view = (long long)n_u * n_v;
  int bits = 0;
  int cv = 0;
  if (r < n_rays) {
    cv = (int)(r / per_view);
    const long long rem = r - (long long)cv * per_view;
    const int iu = (int)(rem / n_v);
    const int iv = (int)(rem - (long long)iu * n_v);
    RaySetup R;
    ray_setup(views + 12 * (size_t)(view0 + cv), G, iu, iv, R);
    const float y = sino[(size_t)(view0 + cv) * per_view + rem];
    const uint32_t mr = (uint32_t)R.m | ((uint32_t)R.i0 << 2) | ((uint32_t)R.i1 << 17);
    if (separable) {
      table[r] = make_float4(__uint_as_float(mr), R.cb, R.gb, y * R.scale);
      if (iv == 0)
        cols[(size_t)cv * n_u + iu] = make_float4(__uint_as_float((uint32_t)R.m), R.ca, R.ga, 0.0f);
    } else {
      table[2 * r] = make_float4(__uint_as_float(mr), R.ca, R.ga, R.cb);
      table[2 * r + 1] = make_float4(R.gb, y * R.scale, 0.0f, 0.0f);
    }
    if (R.i1 > R.i0) bits = 1 << R.m;
  }
  // driving axes per view: OR within the workgroup (LDS), then one global OR
  // per (workgroup, view); integer OR is order independent
  __shared__ int s_bits[256];
  s_bits[threadIdx.x] = 0;
  __syncthreads();
  const long long r0 = (long long)blockIdx.x * 256;
  const int cv0 = (int)(r0 / per_view);
  if (bits) atomicOr(&s_bits[cv - cv0], bits);
  __syncthreads();
  const int b = s_bits[threadIdx.x];
  if (b) atomicOr(&mask[cv0 + (int)threadIdx.x], b);
}

// ---------------------------------------------------------------------------
// Adjoint pass 2: tile splat. A workgroup owns an ATX x ATY x ATZ voxel tile
// held in LDS. For every view of the chunk and every driving axis present in
// it, the rays whose footprint can touch the tile (the detector box of the
// tile grown by one voxel) are staged in LDS in batches of 256, and their
// samples on the tile's planes are recomputed with the forward's arithmetic;
// the weighted contributions that land on tile voxels are added into LDS.
//
// Lane mapping: wave w owns planes [w T/4, (w+1) T/4) of the tile along the
// driving axis (so waves never add to the same word and the summation order
// is fixed), and within a wave lane = (plane, ray): the lanes of one LDS add
// instruction cover PW consecutive planes of 64/PW rays taken far apart in the
// batch, so they address distinct words. Odd plane strides in the padded LDS
// layout spread consecutive planes over the banks. Each voxel is written to
// memory once per chunk (no global atomics).
// proj: per view 12 floats, rows (u, v, w) of the map from a grid point q to
// homogeneous detector coordinates, u = (A_u . q + b_u) / (A_w . q + b_w).
// ---------------------------------------------------------------------------
constexpr int ATX = 32, ATY = 32, ATZ = 8;
constexpr int ASY = ATZ + 1;            // y stride (odd)
constexpr int ASX = ATY * ASY + 1;      // x stride (odd)
constexpr int ATILE = ATX * ASX;        // LDS words of the tile
constexpr int ABATCH = 256;             // rays staged per batch (one per thread)

struct StagedRay {
  float4 e0;  // {m | i0 << 2 | i1 << 17, ca, ga, cb}
  float4 e1;  // {gb, y * scale, -, -}
};

template <int WF>
__global__ __launch_bounds__(256) void adj_splat_kernel(
    const GridGeom G, int n_u, int n_v, const float* __restrict__ proj,
    const float4* __restrict__ table, const int* __restrict__ mask, int view0, int n_chunk,
    int accumulate, float* __restrict__ vol) {
  __shared__ float tile[ATILE];
  __shared__ StagedRay stage[ABATCH];
  const int x0 = blockIdx.z * ATX, y0 = blockIdx.y * ATY, z0 = blockIdx.x * ATZ;
  for (int i = threadIdx.x; i < ATILE; i += 256) tile[i] = 0.0f;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const size_t per_view = (size_t)n_u * n_v;
  for (int c = 0; c < n_chunk; ++c) {
    const int mk = mask[c];
    if (!mk) continue;
    const float* P = proj + 12 * (size_t)(view0 + c);
    // detector box of the tile grown by one voxel (convex hull of 8 corners)
    float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
    bool full = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float cx = (q & 1) ? (float)(x0 + ATX) + 0.01f : (float)x0 - 1.01f;
      const float cy = (q & 2) ? (float)(y0 + ATY) + 0.01f : (float)y0 - 1.01f;
      const float cz = (q & 4) ? (float)(z0 + ATZ) + 0.01f : (float)z0 - 1.01f;
      const float cu = __builtin_fmaf(P[0], cx, __builtin_fmaf(P[1], cy, __builtin_fmaf(P[2], cz, P[3])));
      const float cv = __builtin_fmaf(P[4], cx, __builtin_fmaf(P[5], cy, __builtin_fmaf(P[6], cz, P[7])));
      const float cw = __builtin_fmaf(P[8], cx, __builtin_fmaf(P[9], cy, __builtin_fmaf(P[10], cz, P[11])));
      if (!(cw > 1.0e-6f)) full = true;
      const float inv = 1.0f / cw;
      const float uu = cu * inv, vv = cv * inv;
      umin = fminf(umin, uu);
      umax = fmaxf(umax, uu);
      vmin = fminf(vmin, vv);
      vmax = fmaxf(vmax, vv);
    }
    int iu_lo, iu_hi, iv_lo, iv_hi;
    if (full) {
      iu_lo = 0; iu_hi = n_u - 1; iv_lo = 0; iv_hi = n_v - 1;
    } else {
      const float margin = 0.05f;
      iu_lo = max(0, (int)ceilf(fmaxf(umin - margin, -1.0f)));
      iu_hi = min(n_u - 1, (int)floorf(fminf(umax + margin, (float)n_u)));
      iv_lo = max(0, (int)ceilf(fmaxf(vmin - margin, -1.0f)));
      iv_hi = min(n_v - 1, (int)floorf(fminf(vmax + margin, (float)n_v)));
    }
    const int nbv = iv_hi - iv_lo + 1;
    const int nbox = (iu_hi >= iu_lo && nbv > 0) ? (iu_hi - iu_lo + 1) * nbv : 0;
    if (nbox == 0) continue;
    const float4* T = table + 2 * per_view * (size_t)c;
    for (int m = 0; m < 3; ++m) {
      if (!(mk & (1 << m))) continue;
      const int t0m = (m == 0) ? x0 : ((m == 1) ? y0 : z0);
      const int Tm = (m == 0) ? ATX : ((m == 1) ? ATY : ATZ);
      const int ta0 = (m == 0) ? y0 : x0;
      const int Ta = (m == 0) ? ATY : ATX;
      const int tb0 = (m == 2) ? y0 : z0;
      const int Tb = (m == 2) ? ATY : ATZ;
      const int Sm = (m == 0) ? ASX : ((m == 1) ? ASY : 1);
      const int Sa = (m == 0) ? ASY : ASX;
      const int Sb = (m == 2) ? ASY : 1;
      const float hia = (m == 0) ? G.hi[1] : G.hi[0];
      const float hib = (m == 2) ? G.hi[1] : G.hi[2];
      const int pw_log2 = (Tm == 32) ? 3 : 1;  // planes per wave: Tm / 4 (8 or 2)
      const int j = lane & ((1 << pw_log2) - 1);
      const int q = lane >> pw_log2;
      const int rq = 64 >> pw_log2;          // rays per instruction
      const int lplane = (wave << pw_log2) + j;  // plane within the tile
      const int plane = t0m + lplane;
      const float fpl = (float)plane;
      const int pidx = lplane * Sm;
      // register prefetch of the first batch
      float4 r0 = make_float4(__uint_as_float(3u), 0.0f, 0.0f, 0.0f);
      float4 r1 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      {
        const int r = threadIdx.x;
        if (r < nbox) {
          const int bu = r / nbv;
          const float4* e = T + 2 * ((size_t)(iu_lo + bu) * n_v + (iv_lo + r - bu * nbv));
          r0 = e[0];
          r1 = e[1];
        }
      }
      for (int base = 0; base < nbox; base += ABATCH) {
        __syncthreads();  // previous batch consumed (and tile zeroed on entry)
        stage[threadIdx.x].e0 = r0;
        stage[threadIdx.x].e1 = r1;
        __syncthreads();
        {
          const int r = base + ABATCH + (int)threadIdx.x;
          r0 = make_float4(__uint_as_float(3u), 0.0f, 0.0f, 0.0f);
          if (r < nbox) {
            const int bu = r / nbv;
            const float4* e = T + 2 * ((size_t)(iu_lo + bu) * n_v + (iv_lo + r - bu * nbv));
            r0 = e[0];
            r1 = e[1];
          }
        }
        const int cnt = min(ABATCH, nbox - base);
        // rays of one instruction lie K apart in the batch (distinct voxels);
        // an odd K puts their 32-byte stage entries in distinct LDS banks
        const int K = ((cnt + rq - 1) / rq) | 1;
        for (int t = 0; t < K; ++t) {
          const int k = q * K + t;
          if (k >= cnt) continue;
          const float4 e0 = stage[k].e0;
          const uint32_t mr = __float_as_uint(e0.x);
          const int em = (int)(mr & 3u);
          const int i0 = (int)((mr >> 2) & 0x7fffu);
          const int i1 = (int)(mr >> 17);
          if (em != m || plane < i0 || plane >= i1) continue;
          int ia;
          float wfa, wca;
          sample_axis<WF>(fpl, e0.z, e0.y, hia, ia, wfa, wca);
          const int la = ia - ta0;
          if (la < -1 || la >= Ta) continue;
          const float2 e1 = *reinterpret_cast<const float2*>(&stage[k].e1);
          int ib;
          float wfb, wcb;
          sample_axis<WF>(fpl, e1.x, e0.w, hib, ib, wfb, wcb);
          const int lb = ib - tb0;
          if (lb < -1 || lb >= Tb) continue;
          const int idx = pidx + la * Sa + lb * Sb;
          const float w0 = e1.y * wfa, w1 = e1.y * wca;
          if (la >= 0) {
            if (lb >= 0) atomicAdd(&tile[idx], w0 * wfb);
            if (lb + 1 < Tb) atomicAdd(&tile[idx + Sb], w0 * wcb);
          }
          if (la + 1 < Ta) {
            if (lb >= 0) atomicAdd(&tile[idx + Sa], w1 * wfb);
            if (lb + 1 < Tb) atomicAdd(&tile[idx + Sa + Sb], w1 * wcb);
          }
        }
      }
      __syncthreads();  // axis m done before another axis touches the tile
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ATX * ATY * ATZ; i += 256) {
    const int lz = i % ATZ;
    const int ly = (i / ATZ) % ATY;
    const int lx = i / (ATZ * ATY);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x < G.n[0] && y < G.n[1] && z < G.n[2]) {
      float* out = vol + ((size_t)x * G.n[1] + y) * G.n[2] + z;
      const float v = tile[lx * ASX + ly * ASY + lz];
      *out = accumulate ? (*out + v) : v;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint pass 2, column form. When dv has no in-plane component and no ray is
// driven by axis 2, all rays of a detector column share the driving axis m and
// the coefficients (c_a, g_a) of the in-plane transverse coordinate: the ray
// setup computes them from bitwise identical inputs. A lane owns two voxels
// adjacent along axis 2 (lanes along axis 2). For each view and driving axis,
// the candidate columns are those whose in-plane coordinate on the voxels'
// plane can lie within one voxel (wave-uniform); in each column the candidate
// rays are the few whose axis-2 coordinate can reach the pair, an affine range
// in the ray index (the detector's axis-2 direction keeps the projective
// denominator independent of z). Each candidate sample is evaluated once, with
// the forward's sample_axis, for both voxels; each voxel sums its
// contributions in registers and is written once per launch. No LDS, no
// barriers, no atomics.
// ---------------------------------------------------------------------------
template <int WF>
__global__ __launch_bounds__(256) void adj_gather_sep_kernel(
    const GridGeom G, int n_u, int n_v, const float* __restrict__ proj,
    const float4* __restrict__ rays, const float4* __restrict__ cols,
    const int* __restrict__ mask, int view0, int c0, int n_chunk, int accumulate,
    float* __restrict__ vol) {
  // a lane owns the voxel pair (x, y, z) and (x, y, z + 1)
  const int z = 2 * (blockIdx.x * 64 + (int)(threadIdx.x & 63));
  const int y = blockIdx.y * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int x = blockIdx.z;
  if (y >= G.n[1]) return;
  const bool zin = z < G.n[2];
  const float fx = (float)x, fy = (float)y, fz = (float)z;
  const float hx = G.hi[0], hy = G.hi[1], hz = G.hi[2];
  const float e = 0.002f;       // widened neighbourhood (voxels)
  const float margin = 0.05f;   // widened ranges (pixels)
  constexpr int NC = 6;         // candidate rays loaded together per column
  float acc0 = 0.0f, acc1 = 0.0f;
  for (int c = c0; c < c0 + n_chunk; ++c) {
    const int mk = mask[c];
    if (!mk) continue;
    const float* P = proj + 12 * (size_t)(view0 + c);
    const float4* C = cols + (size_t)c * n_u;
    const float4* RY = rays + (size_t)c * n_u * n_v;
    for (int m = 0; m < 2; ++m) {
      if (!(mk & (1 << m))) continue;
      const int plane = (m == 0) ? x : y;
      const float fplane = (m == 0) ? fx : fy;
      const int va = (m == 0) ? y : x;
      const float ha = (m == 0) ? hy : hx;
      // candidate columns: u of (plane, va -+ (1 + e)); u does not depend on z here
      const float ea = 1.0f + e;
      const float qx0 = (m == 0) ? fx : fx - ea, qy0 = (m == 0) ? fy - ea : fy;
      const float qx1 = (m == 0) ? fx : fx + ea, qy1 = (m == 0) ? fy + ea : fy;
      const float un0 = __builtin_fmaf(P[0], qx0, __builtin_fmaf(P[1], qy0, P[3]));
      const float w0 = __builtin_fmaf(P[8], qx0, __builtin_fmaf(P[9], qy0, P[11]));
      const float un1 = __builtin_fmaf(P[0], qx1, __builtin_fmaf(P[1], qy1, P[3]));
      const float w1 = __builtin_fmaf(P[8], qx1, __builtin_fmaf(P[9], qy1, P[11]));
      int iu_lo = 0, iu_hi = n_u - 1;
      if (w0 > 1.0e-6f && w1 > 1.0e-6f) {
        const float u0 = un0 / w0, u1 = un1 / w1;
        iu_lo = max(0, (int)ceilf(fmaxf(fminf(u0, u1) - margin, -1.0f)));
        iu_hi = min(n_u - 1, (int)floorf(fminf(fmaxf(u0, u1) + margin, (float)n_u)));
      }
      for (int iu = iu_lo; iu <= iu_hi; ++iu) {
        const float4 col = C[iu];
        if ((int)__float_as_uint(col.x) != m) continue;
        int ia;
        float wfa, wca;
        sample_axis<WF>(fplane, col.z, col.y, ha, ia, wfa, wca);
        const float wA = (ia == va) ? wfa : ((ia + 1 == va) ? wca : 0.0f);
        if (wA == 0.0f) continue;
        // v of the column's rays on this plane: (A + B z) / W
        const float pa = __builtin_fmaf(fplane, col.z, col.y);
        const float qx = (m == 0) ? fx : pa, qy = (m == 0) ? pa : fy;
        const float A = __builtin_fmaf(P[4], qx, __builtin_fmaf(P[5], qy, P[7]));
        const float W = __builtin_fmaf(P[8], qx, __builtin_fmaf(P[9], qy, P[11]));
        int iv_lo = 0, iv_hi = n_v - 1;
        if (W > 1.0e-6f) {
          // rays whose axis-2 coordinate lies in [z - 1, z + 2) reach the pair
          const float inv = 1.0f / W;
          const float v0 = (A + P[6] * (fz - 1.0f - e)) * inv;
          const float v1 = (A + P[6] * (fz + 2.0f + e)) * inv;
          iv_lo = max(0, (int)ceilf(fmaxf(fminf(v0, v1) - margin, -1.0f)));
          iv_hi = min(n_v - 1, (int)floorf(fminf(fmaxf(v0, v1) + margin, (float)n_v)));
        }
        if (!zin) iv_hi = iv_lo - 1;
        const float4* R = RY + (size_t)iu * n_v;
        // the first NC candidates are loaded together (indices clamped into
        // the column), then consumed; wider ranges fall through to a loop
        float4 rr[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) rr[k] = R[min(iv_lo + k, n_v - 1)];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const float4 r = rr[k];
          const uint32_t mr = __float_as_uint(r.x);
          const int i0 = (int)((mr >> 2) & 0x7fffu);
          const int i1 = (int)(mr >> 17);
          int ib;
          float wfb, wcb;
          sample_axis<WF>(fplane, r.z, r.y, hz, ib, wfb, wcb);
          const int d = ib - z;  // the sample's floor relative to the pair
          float b0 = (d == 0) ? wfb : ((d == -1) ? wcb : 0.0f);
          float b1 = (d == 1) ? wfb : ((d == 0) ? wcb : 0.0f);
          const bool ok = (iv_lo + k <= iv_hi) && plane >= i0 && plane < i1;
          const float wa = ok ? r.w * wA : 0.0f;
          acc0 = __builtin_fmaf(wa, b0, acc0);
          acc1 = __builtin_fmaf(wa, b1, acc1);
        }
        for (int iv = iv_lo + NC; iv <= iv_hi; ++iv) {
          const float4 r = R[iv];
          const uint32_t mr = __float_as_uint(r.x);
          const int i0 = (int)((mr >> 2) & 0x7fffu);
          const int i1 = (int)(mr >> 17);
          if (plane < i0 || plane >= i1) continue;
          int ib;
          float wfb, wcb;
          sample_axis<WF>(fplane, r.z, r.y, hz, ib, wfb, wcb);
          const int d = ib - z;
          const float b0 = (d == 0) ? wfb : ((d == -1) ? wcb : 0.0f);
          const float b1 = (d == 1) ? wfb : ((d == 0) ? wcb : 0.0f);
          const float wa = r.w * wA;
          acc0 = __builtin_fmaf(wa, b0, acc0);
          acc1 = __builtin_fmaf(wa, b1, acc1);
        }
      }
    }
  }
  if (zin) {
    float* out = vol + ((size_t)x * G.n[1] + y) * G.n[2] + z;
    out[0] = accumulate ? (out[0] + acc0) : acc0;
    if (z + 1 < G.n[2]) out[1] = accumulate ? (out[1] + acc1) : acc1;
  }
}

// ---------------------------------------------------------------------------
// Batched forward: zero-padded copies of every instance, queue reset, and a
// persistent kernel pulling (instance, view, tile) items from a device queue.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void batched_pad_kernel(const BatchInst* __restrict__ insts) {
  const BatchInst& I = insts[blockIdx.y];
  const int n0 = I.a.G.n[0], n1 = I.a.G.n[1], n2 = I.a.G.n[2];
  const long long p2 = n2 + 2, p1 = n1 + 2;
  const long long total = I.padded_elems;
  const bool two = (I.dtype != 0);
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (long long)gridDim.x * 256) {
    const long long z = e % p2;
    const long long t = e / p2;
    const long long y = t % p1;
    const long long x = t / p1;
    const bool in = x >= 1 && x <= n0 && y >= 1 && y <= n1 && z >= 1 && z <= n2;
    const long long src = ((x - 1) * n1 + (y - 1)) * (long long)n2 + (z - 1);
    if (two) {
      const uint16_t* s = static_cast<const uint16_t*>(I.src);
      static_cast<uint16_t*>(I.padded)[e] = in ? s[src] : (uint16_t)0;
    } else {
      const uint32_t* s = static_cast<const uint32_t*>(I.src);
      static_cast<uint32_t*>(I.padded)[e] = in ? s[src] : 0u;
    }
  }
}

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

template <typename T, int WF>
__device__ __forceinline__ void batched_item_t(const FwdArgs& a, int idx64, int view, int t) {
  if (idx64)
    fwd_tile<T, WF, true>(a, view, t);
  else
    fwd_tile<T, WF, false>(a, view, t);
}

__global__ __launch_bounds__(256) void batched_fwd_kernel(const BatchInst* __restrict__ insts,
                                                          const uint2* __restrict__ items,
                                                          int n_items, int* __restrict__ counter) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= n_items) break;
    const uint2 it = items[item];
    const int inst = (int)(it.x & 0xfffu);
    const int view = (int)(it.x >> 12);
    const int t = (int)it.y;
    const BatchInst& I = insts[inst];
    const FwdArgs a = I.a;
    const int sel = I.dtype * 2 + I.weight;
    switch (sel) {
      case 0: batched_item_t<float, W_LINEAR>(a, I.idx64, view, t); break;
      case 1: batched_item_t<float, W_SPLINE>(a, I.idx64, view, t); break;
      case 2: batched_item_t<bf16_t, W_LINEAR>(a, I.idx64, view, t); break;
      case 3: batched_item_t<bf16_t, W_SPLINE>(a, I.idx64, view, t); break;
      case 4: batched_item_t<f16_t, W_LINEAR>(a, I.idx64, view, t); break;
      default: batched_item_t<f16_t, W_SPLINE>(a, I.idx64, view, t); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(-3, std::string(what) + ": " + hipGetErrorString(e));
  return 0;
}

size_t dtype_size(int dtype) { return dtype == 0 ? 4 : 2; }

int launch_pad(const void* src, void* dst, int dtype, const int n[3], hipStream_t s) {
  dim3 grid((unsigned)((n[2] + 2 + 255) / 256), (unsigned)(n[1] + 2), (unsigned)(n[0] + 2));
  TimedLaunch t = timing_begin("pad", s);
  if (dtype == 0)
    pad_kernel<uint32_t><<<grid, 256, 0, s>>>(static_cast<const uint32_t*>(src),
                                               static_cast<uint32_t*>(dst), n[0], n[1], n[2]);
  else
    pad_kernel<uint16_t><<<grid, 256, 0, s>>>(static_cast<const uint16_t*>(src),
                                               static_cast<uint16_t*>(dst), n[0], n[1], n[2]);
  timing_end("pad", t, s);
  return check_launch("pad kernel");
}

template <typename T, int WF>
static void launch_fwd_t(const FwdArgs& a, bool idx64, unsigned grid, hipStream_t s) {
  if (idx64)
    fwd_kernel<T, WF, true><<<grid, 256, 0, s>>>(a);
  else
    fwd_kernel<T, WF, false><<<grid, 256, 0, s>>>(a);
}

int launch_forward(const FwdArgs& a, int dtype, int weight, bool idx64, int n_views,
                   hipStream_t s) {
  const unsigned long long nb = (unsigned long long)n_views * (unsigned long long)a.tiles_per_view;
  if (nb == 0) return 0;
  if (nb > 0xffffffffull) return set_error(-4, "forward: too many workgroups for one launch");
  const unsigned grid = (unsigned)nb;
  TimedLaunch t = timing_begin("forward", s);
  const int sel = dtype * 2 + weight;
  switch (sel) {
    case 0: launch_fwd_t<float, W_LINEAR>(a, idx64, grid, s); break;
    case 1: launch_fwd_t<float, W_SPLINE>(a, idx64, grid, s); break;
    case 2: launch_fwd_t<bf16_t, W_LINEAR>(a, idx64, grid, s); break;
    case 3: launch_fwd_t<bf16_t, W_SPLINE>(a, idx64, grid, s); break;
    case 4: launch_fwd_t<f16_t, W_LINEAR>(a, idx64, grid, s); break;
    default: launch_fwd_t<f16_t, W_SPLINE>(a, idx64, grid, s); break;
  }
  timing_end("forward", t, s);
  return check_launch("forward kernel");
}

int launch_adjoint_table(const gjp_geometry* g, const double* views, const float* sino,
                         int view0, int n_chunk, float4* table, float4* cols, int* mask,
                         hipStream_t s) {
  const long long n_rays = (long long)n_chunk * g->n_u * g->n_v;
  const long long nb = (n_rays + 255) / 256;
  if (nb > 0xffffffffll) return set_error(-4, "adjoint: view chunk too large");
  TimedLaunch t = timing_begin("adjoint_table", s);
  adj_table_kernel<<<(unsigned)nb, 256, 0, s>>>(views, g->gg, sino, g->n_u, g->n_v, view0,
                                                 n_rays, g->separable ? 1 : 0, table, cols, mask);
  timing_end("adjoint_table", t, s);
  return check_launch("adjoint table kernel");
}

int launch_adjoint_gather(const gjp_geometry* g, const float* proj, const float4* table,
                          const float4* cols, const int* mask, int view0, int c0, int n_chunk,
                          bool accumulate, float* vol, hipStream_t s) {
  TimedLaunch t = timing_begin("adjoint_gather", s);
  const int acc = accumulate ? 1 : 0;
  if (g->separable) {
    dim3 grid((unsigned)((g->n[2] + 127) / 128), (unsigned)((g->n[1] + 3) / 4),
              (unsigned)g->n[0]);
    if (g->weight == W_SPLINE)
      adj_gather_sep_kernel<W_SPLINE><<<grid, 256, 0, s>>>(g->gg, g->n_u, g->n_v, proj, table,
                                                           cols, mask, view0, c0, n_chunk, acc,
                                                           vol);
    else
      adj_gather_sep_kernel<W_LINEAR><<<grid, 256, 0, s>>>(g->gg, g->n_u, g->n_v, proj, table,
                                                           cols, mask, view0, c0, n_chunk, acc,
                                                           vol);
  } else {
    if (c0 != 0) return set_error(-4, "adjoint: the tile splat takes whole chunks");
    dim3 grid((unsigned)((g->n[2] + ATZ - 1) / ATZ), (unsigned)((g->n[1] + ATY - 1) / ATY),
              (unsigned)((g->n[0] + ATX - 1) / ATX));
    if (g->weight == W_SPLINE)
      adj_splat_kernel<W_SPLINE><<<grid, 256, 0, s>>>(g->gg, g->n_u, g->n_v, proj, table, mask,
                                                      view0, n_chunk, acc, vol);
    else
      adj_splat_kernel<W_LINEAR><<<grid, 256, 0, s>>>(g->gg, g->n_u, g->n_v, proj, table, mask,
                                                      view0, n_chunk, acc, vol);
  }
  timing_end("adjoint_gather", t, s);
  return check_launch("adjoint kernel");
}

int launch_batched_pad(const BatchInst* d_insts, int n_inst, hipStream_t s) {
  dim3 grid(512, (unsigned)n_inst);
  batched_pad_kernel<<<grid, 256, 0, s>>>(d_insts);
  return check_launch("batched pad kernel");
}

int launch_zero_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return 0;
  zero_ints_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return check_launch("zero kernel");
}

int launch_reset_counter(int* counter, hipStream_t s) {
  reset_counter_kernel<<<1, 64, 0, s>>>(counter);
  return check_launch("queue reset kernel");
}

int batched_grid_size() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_fwd_kernel, 256, 0) !=
          hipSuccess ||
      per <= 0)
    per = 4;
  return cus * per;
}

int launch_batched_forward(const BatchInst* d_insts, const uint2* d_items, int n_items,
                           int* counter, int grid, hipStream_t s) {
  batched_fwd_kernel<<<grid, 256, 0, s>>>(d_insts, d_items, n_items, counter);
  return check_launch("batched forward kernel");
}

}  // namespace gjp
