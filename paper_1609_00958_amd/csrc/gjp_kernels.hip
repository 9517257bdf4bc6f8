// gjp_kernels.hip -- gfx950 kernels of the generalized Joseph projector.
//
// Forward (Algorithm 1): one lane per detector pixel. A 256-thread workgroup
// covers a tile of (64 >> k) x (4 << k) pixels; within a wavefront the fast
// lane index runs along detector v, the direction parallel to the rotation
// axis and to the fastest volume index n2. For a circular trajectory the
// driving axis is then 0 or 1 (never the fastest index, as the paper's
// Algorithm 1 caption recommends for cache efficiency) and the 64 lanes of a
// wavefront share the same transverse row on every plane. The volume is read
// from zero-padded pair copies (one voxel of border on every side; each
// element also holds its neighbour along one transverse axis), so the four
// in-plane neighbours of a sample arrive in one wide load and the sampling
// loop has no bounds tests. The address path of the vector memory unit, not
// bytes, bounds this loop (one tag lookup per quad of lanes per clock for
// each load instruction, whatever its width), so for 16-bit storage a lane
// may take two pixels of one detector column and serve both with one load of
// three consecutive pair elements.
//
// Adjoint: exact transpose of the forward. A table pass stores, per ray of a
// chunk of views, the setup the forward computes (driving axis, sample range,
// single-precision coefficients) and the sinogram value times the step length.
// For circular trajectories a voxel-driven gather evaluates, for each voxel
// block, the few rays of each nearby detector column that reach it; otherwise
// a splat pass accumulates ray samples into a voxel tile held in LDS. Both
// recompute the forward's weights and write each voxel once per launch; no
// atomics touch the volume in memory (the table pass ORs a per-view mask of
// driving axes).
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

// ---------------------------------------------------------------------------
// Pair layout of the zero-padded volume. The padded grid has P0 x P1 x P2
// elements (P0 = n0 + 2, P1 = n1 + 2, P2 = padded_pitch(n2)); padded index k
// holds voxel k - 1 and the border holds zeros. Copy A stores at (x, y, z) the
// pair (v(x, y, z), v(x, y + 1, z)), copy B the pair (v(x, y, z), v(x + 1, y,
// z)), zero past the padded grid. A sample driven by axis 0 finds its four
// in-plane neighbours (rows y, y + 1 at z, z + 1) in copy A as two adjacent
// pairs: one 16-byte (FP32) or 8-byte (16-bit) load. A sample driven by axis 1
// reads copy B the same way; one driven by axis 2 reads two pairs of copy A.
// The address unit handles an irregular 16-byte load per lane at the rate of
// an irregular 4-byte one, so one wide load per sample halves its work
// against two row-pair loads.
// ---------------------------------------------------------------------------

// Neighbours of one sample: rows a, a + 1 of the in-plane transverse axis at
// the axis-2 positions z, z + 1.
struct Quad {
  float a0z0, a1z0, a0z1, a1z1;
};

typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef float f2a8 __attribute__((ext_vector_type(2), aligned(8)));
typedef uint32_t u1a4 __attribute__((aligned(4)));

__device__ __forceinline__ Quad widen4(u2v d, const bf16_t*) {
  return {__uint_as_float(d.x << 16), __uint_as_float(d.x & 0xffff0000u),
          __uint_as_float(d.y << 16), __uint_as_float(d.y & 0xffff0000u)};
}
__device__ __forceinline__ Quad widen4(u2v d, const f16_t*) {
  typedef _Float16 h4v __attribute__((ext_vector_type(4)));
  const h4v h = __builtin_bit_cast(h4v, d);
  return {(float)h.x, (float)h.y, (float)h.z, (float)h.w};
}
__device__ __forceinline__ void widen2(uint32_t u, const bf16_t*, float& x0, float& x1) {
  x0 = __uint_as_float(u << 16);
  x1 = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void widen2(uint32_t u, const f16_t*, float& x0, float& x1) {
  typedef _Float16 h2v __attribute__((ext_vector_type(2)));
  const h2v h = __builtin_bit_cast(h2v, u);
  x0 = (float)h.x;
  x1 = (float)h.y;
}

// Two adjacent pair elements at byte offset voff + soff of a buffer resource.
__device__ __forceinline__ Quad buf_quad(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                         const float*) {
  const f4v v = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  return {v.x, v.y, v.z, v.w};
}
template <typename T>
__device__ __forceinline__ Quad buf_quad(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                         const T* t) {
  return widen4(__builtin_bit_cast(u2v, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0)), t);
}
// The same through a plain pointer to the first pair (64-bit addressing).
__device__ __forceinline__ Quad ptr_quad(const float* p) {
  const f4a8 v = *reinterpret_cast<const f4a8*>(p);
  return {v.x, v.y, v.z, v.w};
}
template <typename T>
__device__ __forceinline__ Quad ptr_quad(const T* p) {
  return widen4(__builtin_bit_cast(u2v, *reinterpret_cast<const u2a4*>(p)), p);
}
// One pair element through a plain pointer.
__device__ __forceinline__ void ptr_pair(const float* p, float& x0, float& x1) {
  const f2a8 v = *reinterpret_cast<const f2a8*>(p);
  x0 = v.x;
  x1 = v.y;
}
template <typename T>
__device__ __forceinline__ void ptr_pair(const T* p, float& x0, float& x1) {
  widen2(*reinterpret_cast<const u1a4*>(p), p, x0, x1);
}

// -0.0f in a scalar register, opaque to the compiler: w * v is issued as the
// fused w * v + (-0), which gives the identical result for every w and v, and
// for 16-bit storage takes the half-precision value directly (mixed-precision
// FMA) instead of a separate conversion.
__device__ __forceinline__ float opaque_neg_zero() {
  float z;
  asm("s_mov_b32 %0, 0x80000000" : "=s"(z));
  return z;
}

// acc += wfa (wfb v(a, z) + wcb v(a, z+1)) + wca (wfb v(a+1, z) + wcb v(a+1, z+1)),
// as two fused steps in this order (Eq. 13 with the weights of Eqs. 10-12).
__device__ __forceinline__ float accumulate4(float acc, float wfa, float wca, float wfb,
                                             float wcb, const Quad& q) {
  const float nz = opaque_neg_zero();
  const float r0 = __builtin_fmaf(wfb, q.a0z0, __builtin_fmaf(wcb, q.a0z1, nz));
  const float r1 = __builtin_fmaf(wfb, q.a1z0, __builtin_fmaf(wcb, q.a1z1, nz));
  acc = __builtin_fmaf(wfa, r0, acc);
  acc = __builtin_fmaf(wca, r1, acc);
  return acc;
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
// Zero-padded pair copies A and B (layout above) of an n0 x n1 x n2 volume of
// E-sized elements. One thread per padded element (x, y, z).
// ---------------------------------------------------------------------------
template <typename E>
__device__ __forceinline__ E padded_value(const E* __restrict__ src, int n0, int n1, int n2,
                                          int x, int y, int z) {
  if (x >= 1 && x <= n0 && y >= 1 && y <= n1 && z >= 1 && z <= n2)
    return src[((size_t)(x - 1) * n1 + (y - 1)) * n2 + (z - 1)];
  return (E)0;
}

// One pair element of each copy, written as one 2-element store.
template <typename E>
__device__ __forceinline__ void pad_pair_element(const E* __restrict__ src, E* __restrict__ A,
                                                 E* __restrict__ B, int n0, int n1, int n2,
                                                 long long e, int x, int y, int z) {
  typedef E E2 __attribute__((ext_vector_type(2)));
  const E v = padded_value(src, n0, n1, n2, x, y, z);
  E2 pa, pb;
  pa.x = v;
  pa.y = padded_value(src, n0, n1, n2, x, y + 1, z);
  pb.x = v;
  pb.y = padded_value(src, n0, n1, n2, x + 1, y, z);
  reinterpret_cast<E2*>(A)[e] = pa;
  reinterpret_cast<E2*>(B)[e] = pb;
}

template <typename E>
__global__ __launch_bounds__(256) void pad_kernel(const E* __restrict__ src, E* __restrict__ A,
                                                  E* __restrict__ B, int n0, int n1, int n2) {
  const int z = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int x = blockIdx.z;
  const int p2 = (int)padded_pitch(n2);
  if (z >= p2) return;
  const long long e = ((long long)x * (n1 + 2) + y) * p2 + z;
  pad_pair_element(src, A, B, n0, n1, n2, e, x, y, z);
}

// ---------------------------------------------------------------------------
// Forward projection of one ray (Algorithm 1).
// ---------------------------------------------------------------------------

// Sampling loop for driving axes 0 and 1 with 32-bit offsets from copy A
// (copy B follows it; both below 4 GiB together), two samples per iteration so
// that two wide loads are in flight per lane. The lanes of a wavefront may
// differ in m, so the copy is chosen by offset, not by resource.
template <typename T, int WF>
__device__ __forceinline__ float fwd_loop_buf(const FwdArgs& a, const RaySetup& R) {
  constexpr uint32_t pe = 2 * sizeof(T);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.vol_a), (short)0, (int)(uint32_t)(2 * a.copy_bytes), 0x00020000);
  const uint32_t Sm = (uint32_t)(R.m == 0 ? a.S0 : a.S1) * pe;
  const int Sa = (int)((R.m == 0 ? a.S1 : a.S0) * (long long)pe);
  const float hia = (R.m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  // padded frame: (plane + 1, row + 1, col + 1) of the ray's copy
  uint32_t off_m = (R.m == 0 ? 0u : (uint32_t)a.copy_bytes) + (uint32_t)(R.i0 + 1) * Sm +
                   (uint32_t)Sa + pe;
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
    const uint32_t o0 = (uint32_t)__mul24(ia0, Sa) + off_m + (uint32_t)ib0 * pe;
    const uint32_t o1 = (uint32_t)__mul24(ia1, Sa) + off_m + Sm + (uint32_t)ib1 * pe;
    const Quad q0 = buf_quad(rs, o0, 0, (const T*)nullptr);
    const Quad q1 = buf_quad(rs, o1, 0, (const T*)nullptr);
    acc = accumulate4(acc, wfa0, wca0, wfb0, wcb0, q0);
    acc = accumulate4(acc, wfa1, wca1, wfb1, wcb1, q1);
    fi += 2.0f;
    off_m += 2 * Sm;
  }
  if (i < R.i1) {
    int ia0, ib0;
    float wfa0, wca0, wfb0, wcb0;
    sample_axis<WF>(fi, R.ga, R.ca, hia, ia0, wfa0, wca0);
    sample_axis<WF>(fi, R.gb, R.cb, hib, ib0, wfb0, wcb0);
    const uint32_t o0 = (uint32_t)__mul24(ia0, Sa) + off_m + (uint32_t)ib0 * pe;
    acc = accumulate4(acc, wfa0, wca0, wfb0, wcb0, buf_quad(rs, o0, 0, (const T*)nullptr));
  }
  return acc;
}

// The same with 64-bit element indices (pair copies of 4 GiB or more).
template <typename T, int WF>
__device__ __forceinline__ float fwd_loop_ptr(const FwdArgs& a, const RaySetup& R) {
  const T* base = static_cast<const T*>(R.m == 0 ? a.vol_a : a.vol_b);
  const long long Sm = (R.m == 0 ? a.S0 : a.S1), Sa = (R.m == 0 ? a.S1 : a.S0);
  const float hia = (R.m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  long long off_m = (long long)(R.i0 + 1) * Sm + Sa + 1;
  float acc = 0.0f;
  float fi = (float)R.i0;
  for (int i = R.i0; i < R.i1; ++i) {
    int ia, ib;
    float wfa, wca, wfb, wcb;
    sample_axis<WF>(fi, R.ga, R.ca, hia, ia, wfa, wca);
    sample_axis<WF>(fi, R.gb, R.cb, hib, ib, wfb, wcb);
    const long long e = off_m + (long long)ia * Sa + ib;
    acc = accumulate4(acc, wfa, wca, wfb, wcb, ptr_quad(base + 2 * e));
    fi += 1.0f;
    off_m += Sm;
  }
  return acc;
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

// NP consecutive planes i .. i + NP - 1 of the row-uniform loop, slots[k] =
// {row byte offset, wfa, wca, plane index as a float} of plane i + k
// (wave-uniform). All NP wide loads are issued before the first is consumed,
// so each lane keeps NP loads in flight. CHECK zeroes the row weights of
// lanes whose sample range excludes a plane (the load stays in bounds: the row
// is inside the copy and the axis-2 coordinate is clamped); a zeroed plane
// adds +-0, so the lane's sum is unchanged.
template <typename T, int WF, bool CHECK, int NP>
__device__ __forceinline__ void ru_planes(__amdgpu_buffer_rsrc_t rs, const float4* slots, int i,
                                          const RaySetup& R, float hib, float& acc) {
  constexpr uint32_t pe = 2 * sizeof(T);
  float4 q[NP];
  Quad u[NP];
  float wfb[NP], wcb[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) q[k] = slots[k];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    int ib;
    sample_axis<WF>(q[k].w, R.gb, R.cb, hib, ib, wfb[k], wcb[k]);
    const uint32_t vo = (uint32_t)(ib + 1) * pe + __float_as_uint(q[k].x);
    u[k] = buf_quad(rs, vo, 0, (const T*)nullptr);
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    float wfa = q[k].y, wca = q[k].z;
    if (CHECK) {
      const bool in = i + k >= R.i0 && i + k < R.i1;
      wfa = in ? wfa : 0.0f;
      wca = in ? wca : 0.0f;
    }
    acc = accumulate4(acc, wfa, wca, wfb[k], wcb[k], u[k]);
  }
}

// Planes per load group of the row-uniform loop in the batched launch (the
// single launch takes it from its arguments; the sums do not depend on it).
constexpr int kBatchRuGroup = 4;

// Sampling loop for a wavefront whose rays all share the driving axis m (0 or
// 1) and the in-plane coefficients (ca, ga): the row coordinate, its weights
// and the row offset of every plane are the same for all lanes. Lane l
// evaluates them for plane base + l of each block of 64 planes and stores
// them in the wavefront's LDS slots; each plane reads its slot back as a
// broadcast, so lanes only evaluate the axis-2 coordinate. Each block reads
// through a buffer resource based at its first plane and lowest row, so the
// offsets stay 32-bit for any volume size. Planes in [mid_lo, mid_hi) lie
// inside every sampling lane's range and skip the range test. Each lane
// accumulates exactly the terms, in the same order and with the same
// arithmetic, as fwd_loop_buf, so the sums are identical (up to the sign of a
// zero). Every one of the 64 lanes must take part; the sums of lanes without
// samples are meaningless and must be discarded by the caller.
template <typename T, int WF, int GRP>
__device__ __forceinline__ float fwd_loop_rowuniform(const FwdArgs& a, const RaySetup& R, int m,
                                                     float ca, float ga, int lo, int hi,
                                                     int mid_lo, int mid_hi) {
  constexpr uint32_t pe = 2 * sizeof(T);
  __shared__ float4 s_planes[4][64];
  float4* slots = s_planes[threadIdx.x >> 6];
  const char* copy = static_cast<const char*>(m == 0 ? a.vol_a : a.vol_b);
  const unsigned long long Sm = (unsigned long long)(m == 0 ? a.S0 : a.S1) * pe;
  const unsigned long long Sa = (unsigned long long)(m == 0 ? a.S1 : a.S0) * pe;
  const float hia = (m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  const int lane = (int)(threadIdx.x & 63);
  float acc = 0.0f;
  for (int base = lo; base < hi; base += 64) {
    int ia_l;
    float wfa_l, wca_l;
    sample_axis<WF>((float)(base + lane), ga, ca, hia, ia_l, wfa_l, wca_l);
    // block origin: padded plane base + 1, padded row ia_min + 1, column 0
    const int ia_min = __builtin_amdgcn_readfirstlane(wave_min(ia_l));
    const unsigned long long org = (unsigned long long)(base + 1) * Sm +
                                   (unsigned long long)(ia_min + 1) * Sa;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(copy + org), (short)0,
        (int)(uint32_t)min(a.copy_bytes - org, 0xffffffffull), 0x00020000);
    const uint32_t row_l = (uint32_t)((unsigned long long)lane * Sm +
                                      (unsigned long long)(ia_l - ia_min) * Sa);
    slots[lane] = make_float4(__uint_as_float(row_l), wfa_l, wca_l, (float)(base + lane));
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(64, hi - base);
    const int j0 = min(max(mid_lo - base, 0), cnt);
    const int j1 = min(max(mid_hi - base, j0), cnt);
    int j = 0;
    for (; j + GRP <= j0; j += GRP)
      ru_planes<T, WF, true, GRP>(rs, slots + j, base + j, R, hib, acc);
    for (; j < j0; ++j) ru_planes<T, WF, true, 1>(rs, slots + j, base + j, R, hib, acc);
    for (; j + GRP <= j1; j += GRP)
      ru_planes<T, WF, false, GRP>(rs, slots + j, base + j, R, hib, acc);
    for (; j < j1; ++j) ru_planes<T, WF, false, 1>(rs, slots + j, base + j, R, hib, acc);
    for (; j + GRP <= cnt; j += GRP)
      ru_planes<T, WF, true, GRP>(rs, slots + j, base + j, R, hib, acc);
    for (; j < cnt; ++j) ru_planes<T, WF, true, 1>(rs, slots + j, base + j, R, hib, acc);
    // every lane has read the slots before the next block rewrites them
    __builtin_amdgcn_wave_barrier();
  }
  return acc;
}

// Sum of one ray per lane (before the step length). All 64 lanes of the
// wavefront call this together; a lane without samples (R.i0 == R.i1, e.g. a
// pixel outside the detector) takes part in the wavefront-wide steps and its
// sum is meaningless.
template <typename T, int WF, bool IDX64, int GRP>
__device__ __forceinline__ float fwd_sum(const FwdArgs& a, const RaySetup& R) {
  float acc = 0.0f;
  // row-uniform wavefront: every lane with samples shares m (0 or 1), ca and
  // ga; the shared values are the first such lane's
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
    const int mid_lo = __builtin_amdgcn_readfirstlane(wave_max(has ? R.i0 : -1));
    const int mid_hi = __builtin_amdgcn_readfirstlane(wave_min(has ? R.i1 : 0x7fffffff));
    acc = fwd_loop_rowuniform<T, WF, GRP>(a, R, lm, lca, lga, lo, hi, mid_lo, mid_hi);
    if (!has) acc = 0.0f;
  } else if (R.m != 2) {
    if constexpr (!IDX64)
      acc = fwd_loop_buf<T, WF>(a, R);
    else
      acc = fwd_loop_ptr<T, WF>(a, R);
  } else {
    // driving axis 2: transverse axes 0 (rows of copy A, stride S0) and 1
    // (pairs of copy A); two pair loads per sample
    const T* base = static_cast<const T*>(a.vol_a);
    const long long S0 = a.S0, S1 = a.S1;
    const float hia = a.G.hi[0], hib = a.G.hi[1];
    float fi = (float)R.i0;
    for (int i = R.i0; i < R.i1; ++i) {
      int ia, ib;
      float wfa, wca, wfb, wcb;
      sample_axis<WF>(fi, R.ga, R.ca, hia, ia, wfa, wca);
      sample_axis<WF>(fi, R.gb, R.cb, hib, ib, wfb, wcb);
      const long long e = (long long)(ia + 1) * S0 + (long long)(ib + 1) * S1 + (i + 1);
      Quad q;
      ptr_pair(base + 2 * e, q.a0z0, q.a0z1);
      ptr_pair(base + 2 * (e + S0), q.a1z0, q.a1z1);
      acc = accumulate4(acc, wfa, wca, wfb, wcb, q);
      fi += 1.0f;
    }
  }
  return acc;
}

template <typename T, int WF, bool IDX64, int GRP>
__device__ __forceinline__ void fwd_ray(const FwdArgs& a, int view, int iu, int iv, bool valid) {
  RaySetup R;
  ray_setup(a.views + 12 * (size_t)view, a.G, iu, iv, R);
  if (!valid) R.i1 = R.i0;
  const float acc = fwd_sum<T, WF, IDX64, GRP>(a, R);
  if (valid) a.sino[((size_t)view * a.n_u + iu) * a.n_v + iv] = acc * R.scale;
}

// Three consecutive pair elements at byte offset voff of a 16-bit copy: the
// samples at axis-2 floors z (elements 0, 1) and z + 1 (elements 1, 2).
struct Triple {
  uint32_t e0, e1, e2;
};
__device__ __forceinline__ Triple buf_triple(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  typedef uint32_t u3v __attribute__((ext_vector_type(3)));
  const u3v v = __builtin_bit_cast(u3v, __builtin_amdgcn_raw_buffer_load_b96(r, voff, 0, 0));
  return {v.x, v.y, v.z};
}

// The two rays' neighbour quads from three consecutive pair elements: the
// first ray's at elements 0, 1; the second's at 0, 1 or, one floor up, 1, 2.
// FP16 selects whole elements (the mixed-precision FMAs widen them); BF16
// widens the three elements once and selects the values.
__device__ __forceinline__ void pair_quads(const Triple& t, bool up, const f16_t* tag, Quad& q1,
                                           Quad& q2) {
  q1 = widen4(u2v{t.e0, t.e1}, tag);
  q2 = widen4(u2v{up ? t.e1 : t.e0, up ? t.e2 : t.e1}, tag);
}
__device__ __forceinline__ void pair_quads(const Triple& t, bool up, const bf16_t*, Quad& q1,
                                           Quad& q2) {
  const float l0 = __uint_as_float(t.e0 << 16), h0 = __uint_as_float(t.e0 & 0xffff0000u);
  const float l1 = __uint_as_float(t.e1 << 16), h1 = __uint_as_float(t.e1 & 0xffff0000u);
  const float l2 = __uint_as_float(t.e2 << 16), h2 = __uint_as_float(t.e2 & 0xffff0000u);
  q1 = {l0, h0, l1, h1};
  q2 = {up ? l1 : l0, up ? h1 : h0, up ? l2 : l1, up ? h2 : h1};
}

// Row-uniform loop over two rays per lane for 16-bit storage. The two rays of
// a lane share the driving axis and the in-plane coefficients with every
// other ray of the wavefront (one detector column), so on each plane they
// share the row, its weights and its offset, and the caller has checked that
// on every plane of [lo, hi) the second ray's axis-2 coordinate exceeds the
// first's by less than one voxel (so its floor is the first's or one more).
// One 12-byte load of the pair elements at floors z, z + 1, z + 2 of the first
// ray then serves both. Each ray accumulates exactly the terms, in the same
// order and with the same arithmetic, as the one-ray loop.
constexpr int kPairGroup = 2;  // planes per load group (two samples each)

template <typename T, int WF, int GRP>
__device__ __forceinline__ void fwd_loop_rowuniform_pair(const FwdArgs& a, const RaySetup& R1,
                                                         const RaySetup& R2, int m, float ca,
                                                         float ga, int lo, int hi, int mid_lo,
                                                         int mid_hi, float& acc1, float& acc2) {
  constexpr uint32_t pe = 2 * sizeof(T);
  __shared__ float4 s_planes[4][64];
  float4* slots = s_planes[threadIdx.x >> 6];
  const char* copy = static_cast<const char*>(m == 0 ? a.vol_a : a.vol_b);
  const unsigned long long Sm = (unsigned long long)(m == 0 ? a.S0 : a.S1) * pe;
  const unsigned long long Sa = (unsigned long long)(m == 0 ? a.S1 : a.S0) * pe;
  const float hia = (m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  const int lane = (int)(threadIdx.x & 63);
  acc1 = 0.0f;
  acc2 = 0.0f;
  for (int base = lo; base < hi; base += 64) {
    int ia_l;
    float wfa_l, wca_l;
    sample_axis<WF>((float)(base + lane), ga, ca, hia, ia_l, wfa_l, wca_l);
    const int ia_min = __builtin_amdgcn_readfirstlane(wave_min(ia_l));
    const unsigned long long org = (unsigned long long)(base + 1) * Sm +
                                   (unsigned long long)(ia_min + 1) * Sa;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(copy + org), (short)0,
        (int)(uint32_t)min(a.copy_bytes - org, 0xffffffffull), 0x00020000);
    const uint32_t row_l = (uint32_t)((unsigned long long)lane * Sm +
                                      (unsigned long long)(ia_l - ia_min) * Sa);
    slots[lane] = make_float4(__uint_as_float(row_l), wfa_l, wca_l, (float)(base + lane));
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(64, hi - base);
    const int j0 = min(max(mid_lo - base, 0), cnt);
    const int j1 = min(max(mid_hi - base, j0), cnt);
    // planes [j0, j1) lie inside both rays' ranges on every lane
    auto group = [&](int j, auto check_tag, auto np_tag) {
      constexpr bool CHECK = decltype(check_tag)::value;
      constexpr int NP = decltype(np_tag)::value;
      float4 q[NP];
      Triple u[NP];
      float wfb1[NP], wcb1[NP], wfb2[NP], wcb2[NP];
      bool up[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) q[k] = slots[j + k];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        // floors compared as floats: only the first ray's becomes an address
        float f1, f2;
        sample_axis_floor<WF>(q[k].w, R1.gb, R1.cb, hib, f1, wfb1[k], wcb1[k]);
        sample_axis_floor<WF>(q[k].w, R2.gb, R2.cb, hib, f2, wfb2[k], wcb2[k]);
        up[k] = f2 != f1;
        const uint32_t vo = (uint32_t)((int)f1 + 1) * pe + __float_as_uint(q[k].x);
        u[k] = buf_triple(rs, vo);
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        float wfa1 = q[k].y, wca1 = q[k].z, wfa2 = q[k].y, wca2 = q[k].z;
        if (CHECK) {
          const int i = base + j + k;
          const bool in1 = i >= R1.i0 && i < R1.i1, in2 = i >= R2.i0 && i < R2.i1;
          wfa1 = in1 ? wfa1 : 0.0f;
          wca1 = in1 ? wca1 : 0.0f;
          wfa2 = in2 ? wfa2 : 0.0f;
          wca2 = in2 ? wca2 : 0.0f;
        }
        Quad q1, q2;
        pair_quads(u[k], up[k], (const T*)nullptr, q1, q2);
        acc1 = accumulate4(acc1, wfa1, wca1, wfb1[k], wcb1[k], q1);
        acc2 = accumulate4(acc2, wfa2, wca2, wfb2[k], wcb2[k], q2);
      }
    };
    using yes = std::true_type;
    using no = std::false_type;
    using two = std::integral_constant<int, kPairGroup>;
    using one = std::integral_constant<int, 1>;
    int j = 0;
    for (; j + kPairGroup <= j0; j += kPairGroup) group(j, yes(), two());
    for (; j < j0; ++j) group(j, yes(), one());
    for (; j + kPairGroup <= j1; j += kPairGroup) group(j, no(), two());
    for (; j < j1; ++j) group(j, no(), one());
    for (; j + kPairGroup <= cnt; j += kPairGroup) group(j, yes(), two());
    for (; j < cnt; ++j) group(j, yes(), one());
    __builtin_amdgcn_wave_barrier();
  }
}

// Two rays per lane, pixels (iu, iv) and (iu, iv + 1) of one detector column
// (16-bit storage). When the wavefront is row-uniform and the two rays' axis-2
// coordinates stay less than a voxel apart on every plane (checked here, with
// a margin for single-precision rounding), one load serves both rays' samples;
// otherwise each ray set runs the one-ray path. The sums are the one-ray
// path's in every case.
template <typename T, int WF, bool IDX64, int GRP>
__device__ __forceinline__ void fwd_ray_pair(const FwdArgs& a, int view, int iu, int iv,
                                             bool valid1, bool valid2) {
  RaySetup R1, R2;
  const double* vv = a.views + 12 * (size_t)view;
  {
    // the first ray's setup waits in LDS while the second one's double
    // precision setup runs, so that the two are never live in registers
    // together (the register peak of this kernel)
    __shared__ float4 s_stash[2][256];
    RaySetup T1;
    ray_setup(vv, a.G, iu, iv, T1);
    s_stash[0][threadIdx.x] = make_float4(T1.ca, T1.ga, T1.cb, T1.gb);
    s_stash[1][threadIdx.x] = make_float4(__int_as_float(T1.m), __int_as_float(T1.i0),
                                          __int_as_float(T1.i1), T1.scale);
    // compiler barriers: the second setup starts after the stash is written
    // (its pixel index passes through the barrier) and the stash is read
    // back after the second setup has finished
    int iv2 = iv + 1;
    asm volatile("" : "+v"(iv2) : : "memory");
    ray_setup(vv, a.G, iu, iv2, R2);
    asm volatile("" : : "v"(R2.i0), "v"(R2.i1), "v"(R2.cb), "v"(R2.gb), "v"(R2.scale) : "memory");
    const float4 c0 = s_stash[0][threadIdx.x], c1 = s_stash[1][threadIdx.x];
    R1.ca = c0.x;
    R1.ga = c0.y;
    R1.cb = c0.z;
    R1.gb = c0.w;
    R1.m = __float_as_int(c1.x);
    R1.i0 = __float_as_int(c1.y);
    R1.i1 = __float_as_int(c1.z);
    R1.scale = c1.w;
    R1.ta = R1.m == 0 ? 1 : 0;
    R1.tb = R1.m == 2 ? 1 : 2;
  }
  if (!valid1) R1.i1 = R1.i0;
  if (!valid2) R2.i1 = R2.i0;
  const bool has1 = R1.i1 > R1.i0, has2 = R2.i1 > R2.i0;
  float acc1 = 0.0f, acc2 = 0.0f;
  // a lane with one empty ray runs the other ray's coefficients in its place
  // (same floors, so the shared load is that ray's own) and drops that sum
  RaySetup P1 = R1, P2 = R2;
  if (!has1) {
    P1.cb = R2.cb;
    P1.gb = R2.gb;
  }
  if (!has2) {
    P2.cb = P1.cb;
    P2.gb = P1.gb;
  }
  const bool any = has1 || has2;
  const uint64_t hv = __ballot(any);
  bool paired = false, swap = false;
  int lm = 2, lo = 0, hi = 0, mid_lo = 0, mid_hi = 0;
  float lca = 0.0f, lga = 0.0f;
  if (hv != 0) {
    const int leader = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)hv) - 1);
    const RaySetup& L = has1 ? R1 : R2;
    lm = __builtin_amdgcn_readlane(L.m, leader);
    lca = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, L.ca), leader));
    lga = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, L.ga), leader));
    const bool off1 = has1 && (R1.m != lm || R1.ca != lca || R1.ga != lga);
    const bool off2 = has2 && (R2.m != lm || R2.ca != lca || R2.ga != lga);
    if (lm != 2 && __ballot(off1 || off2) == 0) {
      const int i0 = min(has1 ? R1.i0 : 0x7fffffff, has2 ? R2.i0 : 0x7fffffff);
      const int i1 = max(has1 ? R1.i1 : -1, has2 ? R2.i1 : -1);
      const int j0 = max(has1 ? R1.i0 : -1, has2 ? R2.i0 : -1);
      const int j1 = min(has1 ? R1.i1 : 0x7fffffff, has2 ? R2.i1 : 0x7fffffff);
      lo = __builtin_amdgcn_readfirstlane(wave_min(any ? i0 : 0x7fffffff));
      hi = __builtin_amdgcn_readfirstlane(wave_max(any ? i1 : -1));
      mid_lo = __builtin_amdgcn_readfirstlane(wave_max(any ? j0 : -1));
      mid_hi = __builtin_amdgcn_readfirstlane(wave_min(any ? j1 : 0x7fffffff));
      // the difference of the two axis-2 coordinates is affine in the plane
      // index, so its extremes over [lo, hi) are at the ends
      const float fl = (float)lo, fh = (float)(hi - 1);
      const float p1l = __builtin_fmaf(fl, P1.gb, P1.cb), p2l = __builtin_fmaf(fl, P2.gb, P2.cb);
      const float p1h = __builtin_fmaf(fh, P1.gb, P1.cb), p2h = __builtin_fmaf(fh, P2.gb, P2.cb);
      const float M = fmaxf(fmaxf(fmaxf(fabsf(p1l), fabsf(p2l)), fmaxf(fabsf(p1h), fabsf(p2h))),
                            1.0f);
      const float eps = M * 0x1p-20f;
      const float dl = p2l - p1l, dh = p2h - p1h;
      const bool same = P1.cb == P2.cb && P1.gb == P2.gb;
      const bool pos = same || (dl >= eps && dl <= 1.0f - eps && dh >= eps && dh <= 1.0f - eps);
      const bool neg = same || (-dl >= eps && -dl <= 1.0f - eps && -dh >= eps && -dh <= 1.0f - eps);
      if (__ballot(!pos) == 0) {
        paired = true;
      } else if (__ballot(!neg) == 0) {
        paired = true;
        swap = true;
      }
    }
  }
  if (paired) {
    // the ray with the lower axis-2 coordinate addresses the shared load
    const RaySetup& A = swap ? P2 : P1;
    const RaySetup& B = swap ? P1 : P2;
    RaySetup Ac = A, Bc = B;
    Ac.i0 = swap ? R2.i0 : R1.i0;
    Ac.i1 = swap ? R2.i1 : R1.i1;
    Bc.i0 = swap ? R1.i0 : R2.i0;
    Bc.i1 = swap ? R1.i1 : R2.i1;
    float sa, sb;
    fwd_loop_rowuniform_pair<T, WF, GRP>(a, Ac, Bc, lm, lca, lga, lo, hi, mid_lo, mid_hi, sa, sb);
    acc1 = has1 ? (swap ? sb : sa) : 0.0f;
    acc2 = has2 ? (swap ? sa : sb) : 0.0f;
    float* out = a.sino + ((size_t)view * a.n_u + iu) * a.n_v + iv;
    if (valid1) out[0] = acc1 * R1.scale;
    if (valid2) out[1] = acc2 * R2.scale;
  } else {
    // one ray set after the other; the second ray's setup is recomputed so
    // that it does not stay live through the first one's loop
    fwd_ray<T, WF, IDX64, GRP>(a, view, iu, iv, valid1);
    fwd_ray<T, WF, IDX64, GRP>(a, view, iu, iv + 1, valid2);
  }
}

// Four consecutive pair elements at byte offset voff of a 16-bit copy (one
// 16-byte load): the samples of three rays whose axis-2 floors are z, z or
// z + 1, and z .. z + 2.
struct Quadruple {
  uint32_t e0, e1, e2, e3;
};
__device__ __forceinline__ Quadruple buf_quadruple(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  typedef uint32_t u4v __attribute__((ext_vector_type(4)));
  const u4v v = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
  return {v.x, v.y, v.z, v.w};
}

// Row interpolation of one pair element: wfa v(a, z) + wca v(a + 1, z), the
// product issued as a fused w v + (-0) so that FP16 values enter the
// mixed-precision FMA directly; BF16 values are widened first.
__device__ __forceinline__ float row_mix(uint32_t e, float wfa, float wca, float nz,
                                         const f16_t*) {
  typedef _Float16 h2v __attribute__((ext_vector_type(2)));
  const h2v h = __builtin_bit_cast(h2v, e);
  return __builtin_fmaf(wca, (float)h.y, __builtin_fmaf(wfa, (float)h.x, nz));
}
__device__ __forceinline__ float row_mix(uint32_t e, float wfa, float wca, float nz,
                                         const bf16_t*) {
  return __builtin_fmaf(wca, __uint_as_float(e & 0xffff0000u),
                        __builtin_fmaf(wfa, __uint_as_float(e << 16), nz));
}

// Row-uniform loop over three rays per lane: pixels v, v + 1 and v + 2 of one
// detector column, ordered so that the first has the lowest axis-2
// coordinate; the caller has checked that on every plane of [lo, hi) each
// ray's coordinate exceeds the previous one's by less than one voxel, so the
// floors are z, z or z + 1, and that or one more. The pair elements at
// z .. z + 3 (one 16-byte load for 16-bit storage, two for FP32) then serve
// all three. Each element is first
// interpolated along the in-plane row (the row and its weights are the same
// for every ray of the wavefront), then each ray combines the two elements at
// its floor with its axis-2 weights: the bilinear weights of Eqs. 10-12 in
// the other order of the two axes, so the sums equal the one-ray loop's up to
// rounding (not bit for bit).
constexpr int kTripleGroup = 2;  // planes per load group (three samples each)

template <typename T, int WF, int GRP>
__device__ __forceinline__ void fwd_loop_rowuniform_triple(const FwdArgs& a, const RaySetup& R1,
                                                           const RaySetup& R2, const RaySetup& R3,
                                                           int m, float ca, float ga, int lo, int hi,
                                                           int mid_lo, int mid_hi, float& acc1,
                                                           float& acc2, float& acc3) {
  constexpr uint32_t pe = 2 * sizeof(T);
  __shared__ float4 s_planes[4][64];
  float4* slots = s_planes[threadIdx.x >> 6];
  const char* copy = static_cast<const char*>(m == 0 ? a.vol_a : a.vol_b);
  const unsigned long long Sm = (unsigned long long)(m == 0 ? a.S0 : a.S1) * pe;
  const unsigned long long Sa = (unsigned long long)(m == 0 ? a.S1 : a.S0) * pe;
  const float hia = (m == 0) ? a.G.hi[1] : a.G.hi[0];
  const float hib = a.G.hi[2];
  const int lane = (int)(threadIdx.x & 63);
  const float nz = opaque_neg_zero();
  acc1 = 0.0f;
  acc2 = 0.0f;
  acc3 = 0.0f;
  for (int base = lo; base < hi; base += 64) {
    int ia_l;
    float wfa_l, wca_l;
    sample_axis<WF>((float)(base + lane), ga, ca, hia, ia_l, wfa_l, wca_l);
    const int ia_min = __builtin_amdgcn_readfirstlane(wave_min(ia_l));
    const unsigned long long org = (unsigned long long)(base + 1) * Sm +
                                   (unsigned long long)(ia_min + 1) * Sa;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(copy + org), (short)0,
        (int)(uint32_t)min(a.copy_bytes - org, 0xffffffffull), 0x00020000);
    const uint32_t row_l = (uint32_t)((unsigned long long)lane * Sm +
                                      (unsigned long long)(ia_l - ia_min) * Sa);
    slots[lane] = make_float4(__uint_as_float(row_l), wfa_l, wca_l, (float)(base + lane));
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(64, hi - base);
    const int j0 = min(max(mid_lo - base, 0), cnt);
    const int j1 = min(max(mid_hi - base, j0), cnt);
    // planes [j0, j1) lie inside all three rays' ranges on every lane
    auto group = [&](int j, auto check_tag, auto np_tag) {
      constexpr bool CHECK = decltype(check_tag)::value;
      constexpr int NP = decltype(np_tag)::value;
      float4 q[NP];
      Quadruple u[NP];   // 16-bit: four pair elements
      f4v u0[NP], u1[NP];  // FP32: the same four elements in two loads
      float wfb1[NP], wcb1[NP], wfb2[NP], wcb2[NP], wfb3[NP], wcb3[NP];
      bool up2[NP], up3[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) q[k] = slots[j + k];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        // floors compared as floats: only the first ray's becomes an address
        float f1, f2, f3;
        sample_axis_floor<WF>(q[k].w, R1.gb, R1.cb, hib, f1, wfb1[k], wcb1[k]);
        sample_axis_floor<WF>(q[k].w, R2.gb, R2.cb, hib, f2, wfb2[k], wcb2[k]);
        sample_axis_floor<WF>(q[k].w, R3.gb, R3.cb, hib, f3, wfb3[k], wcb3[k]);
        up2[k] = f2 != f1;
        up3[k] = f3 != f2;
        const uint32_t vo = (uint32_t)((int)f1 + 1) * pe + __float_as_uint(q[k].x);
        if constexpr (sizeof(T) == 4) {
          u0[k] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, 0, 0));
          u1[k] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 16u, 0, 0));
        } else {
          u[k] = buf_quadruple(rs, vo);
        }
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const float wfa = q[k].y, wca = q[k].z;
        float t0, t1, t2, t3;
        if constexpr (sizeof(T) == 4) {
          t0 = __builtin_fmaf(wca, u0[k].y, __builtin_fmaf(wfa, u0[k].x, nz));
          t1 = __builtin_fmaf(wca, u0[k].w, __builtin_fmaf(wfa, u0[k].z, nz));
          t2 = __builtin_fmaf(wca, u1[k].y, __builtin_fmaf(wfa, u1[k].x, nz));
          t3 = __builtin_fmaf(wca, u1[k].w, __builtin_fmaf(wfa, u1[k].z, nz));
        } else {
          t0 = row_mix(u[k].e0, wfa, wca, nz, (const T*)nullptr);
          t1 = row_mix(u[k].e1, wfa, wca, nz, (const T*)nullptr);
          t2 = row_mix(u[k].e2, wfa, wca, nz, (const T*)nullptr);
          t3 = row_mix(u[k].e3, wfa, wca, nz, (const T*)nullptr);
        }
        // the second ray's two elements start at its floor: z or z + 1; the
        // third's one further or not
        const float p0 = up2[k] ? t1 : t0, p1 = up2[k] ? t2 : t1, p2 = up2[k] ? t3 : t2;
        const float r0 = up3[k] ? p1 : p0, r1 = up3[k] ? p2 : p1;
        const float n1 = __builtin_fmaf(wcb1[k], t1, __builtin_fmaf(wfb1[k], t0, acc1));
        const float n2 = __builtin_fmaf(wcb2[k], p1, __builtin_fmaf(wfb2[k], p0, acc2));
        const float n3 = __builtin_fmaf(wcb3[k], r1, __builtin_fmaf(wfb3[k], r0, acc3));
        if (CHECK) {
          // a ray whose sample range excludes the plane keeps its sum
          const int i = base + j + k;
          acc1 = (i >= R1.i0 && i < R1.i1) ? n1 : acc1;
          acc2 = (i >= R2.i0 && i < R2.i1) ? n2 : acc2;
          acc3 = (i >= R3.i0 && i < R3.i1) ? n3 : acc3;
        } else {
          acc1 = n1;
          acc2 = n2;
          acc3 = n3;
        }
      }
    };
    using yes = std::true_type;
    using no = std::false_type;
    using two = std::integral_constant<int, kTripleGroup>;
    using one = std::integral_constant<int, 1>;
    int j = 0;
    for (; j + kTripleGroup <= j0; j += kTripleGroup) group(j, yes(), two());
    for (; j < j0; ++j) group(j, yes(), one());
    for (; j + kTripleGroup <= j1; j += kTripleGroup) group(j, no(), two());
    for (; j < j1; ++j) group(j, no(), one());
    for (; j + kTripleGroup <= cnt; j += kTripleGroup) group(j, yes(), two());
    for (; j < cnt; ++j) group(j, yes(), one());
    __builtin_amdgcn_wave_barrier();
  }
}

// Is b's axis-2 coordinate above a's by at least eps and at most 1 - eps at
// the two ends of the plane range (the difference is affine in the plane),
// or are the two coefficient sets the same?
__device__ __forceinline__ bool step_ok(float cb_a, float gb_a, float cb_b, float gb_b, float fl,
                                        float fh, float sign) {
  if (cb_a == cb_b && gb_a == gb_b) return true;
  const float al = __builtin_fmaf(fl, gb_a, cb_a), bl = __builtin_fmaf(fl, gb_b, cb_b);
  const float ah = __builtin_fmaf(fh, gb_a, cb_a), bh = __builtin_fmaf(fh, gb_b, cb_b);
  const float M = fmaxf(fmaxf(fmaxf(fabsf(al), fabsf(bl)), fmaxf(fabsf(ah), fabsf(bh))), 1.0f);
  const float eps = M * 0x1p-20f;
  const float dl = sign * (bl - al), dh = sign * (bh - ah);
  return dl >= eps && dl <= 1.0f - eps && dh >= eps && dh <= 1.0f - eps;
}

// Three rays per lane, pixels (iu, iv), (iu, iv + 1) and (iu, iv + 2) of one
// detector column. When the wavefront is row-uniform and on
// every plane each ray's axis-2 coordinate exceeds the previous one's by less
// than a voxel (checked here, with a margin for single-precision rounding; in
// either direction along v), one load serves the three rays' samples;
// otherwise each ray runs the one-ray path.
template <typename T, int WF, bool IDX64, int GRP>
__device__ __forceinline__ void fwd_ray_triple(const FwdArgs& a, int view, int iu, int iv,
                                               bool valid1, bool valid2, bool valid3) {
  RaySetup R1, R2, R3;
  const double* vv = a.views + 12 * (size_t)view;
  {
    // the first two rays' setups wait in LDS while the next one's double
    // precision setup runs, so that they are never live in registers
    // together (the register peak of this kernel)
    __shared__ float4 s_stash[4][256];
    RaySetup T1;
    ray_setup(vv, a.G, iu, iv, T1);
    s_stash[0][threadIdx.x] = make_float4(T1.ca, T1.ga, T1.cb, T1.gb);
    s_stash[1][threadIdx.x] = make_float4(__int_as_float(T1.m), __int_as_float(T1.i0),
                                          __int_as_float(T1.i1), T1.scale);
    int iv2 = iv + 1;
    asm volatile("" : "+v"(iv2) : : "memory");
    RaySetup T2;
    ray_setup(vv, a.G, iu, iv2, T2);
    s_stash[2][threadIdx.x] = make_float4(T2.ca, T2.ga, T2.cb, T2.gb);
    s_stash[3][threadIdx.x] = make_float4(__int_as_float(T2.m), __int_as_float(T2.i0),
                                          __int_as_float(T2.i1), T2.scale);
    int iv3 = iv + 2;
    asm volatile("" : "+v"(iv3) : : "memory");
    ray_setup(vv, a.G, iu, iv3, R3);
    asm volatile("" : : "v"(R3.i0), "v"(R3.i1), "v"(R3.cb), "v"(R3.gb), "v"(R3.scale) : "memory");
    auto unstash = [&](int k, RaySetup& R) {
      const float4 c0 = s_stash[2 * k][threadIdx.x], c1 = s_stash[2 * k + 1][threadIdx.x];
      R.ca = c0.x;
      R.ga = c0.y;
      R.cb = c0.z;
      R.gb = c0.w;
      R.m = __float_as_int(c1.x);
      R.i0 = __float_as_int(c1.y);
      R.i1 = __float_as_int(c1.z);
      R.scale = c1.w;
      R.ta = R.m == 0 ? 1 : 0;
      R.tb = R.m == 2 ? 1 : 2;
    };
    unstash(0, R1);
    unstash(1, R2);
  }
  if (!valid1) R1.i1 = R1.i0;
  if (!valid2) R2.i1 = R2.i0;
  if (!valid3) R3.i1 = R3.i0;
  const bool has1 = R1.i1 > R1.i0, has2 = R2.i1 > R2.i0, has3 = R3.i1 > R3.i0;
  // a ray without samples runs a neighbour's coefficients in its place (same
  // floors, so the shared load is that ray's own) and drops its sum
  RaySetup P1 = R1, P2 = R2, P3 = R3;
  if (!has1) {
    const RaySetup& N = has2 ? R2 : R3;
    P1.cb = N.cb;
    P1.gb = N.gb;
  }
  if (!has2) {
    P2.cb = P1.cb;
    P2.gb = P1.gb;
  }
  if (!has3) {
    P3.cb = P2.cb;
    P3.gb = P2.gb;
  }
  const bool any = has1 || has2 || has3;
  const uint64_t hv = __ballot(any);
  bool tripled = false, swap = false;
  int lm = 2, lo = 0, hi = 0, mid_lo = 0, mid_hi = 0;
  float lca = 0.0f, lga = 0.0f;
  if (hv != 0) {
    const int leader = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)hv) - 1);
    const RaySetup& L = has1 ? R1 : (has2 ? R2 : R3);
    lm = __builtin_amdgcn_readlane(L.m, leader);
    lca = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, L.ca), leader));
    lga = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, L.ga), leader));
    const bool off1 = has1 && (R1.m != lm || R1.ca != lca || R1.ga != lga);
    const bool off2 = has2 && (R2.m != lm || R2.ca != lca || R2.ga != lga);
    const bool off3 = has3 && (R3.m != lm || R3.ca != lca || R3.ga != lga);
    if (lm != 2 && __ballot(off1 || off2 || off3) == 0) {
      const int big = 0x7fffffff;
      const int i0 = min(min(has1 ? R1.i0 : big, has2 ? R2.i0 : big), has3 ? R3.i0 : big);
      const int i1 = max(max(has1 ? R1.i1 : -1, has2 ? R2.i1 : -1), has3 ? R3.i1 : -1);
      const int j0 = max(max(has1 ? R1.i0 : -1, has2 ? R2.i0 : -1), has3 ? R3.i0 : -1);
      const int j1 = min(min(has1 ? R1.i1 : big, has2 ? R2.i1 : big), has3 ? R3.i1 : big);
      lo = __builtin_amdgcn_readfirstlane(wave_min(any ? i0 : big));
      hi = __builtin_amdgcn_readfirstlane(wave_max(any ? i1 : -1));
      mid_lo = __builtin_amdgcn_readfirstlane(wave_max(any ? j0 : -1));
      mid_hi = __builtin_amdgcn_readfirstlane(wave_min(any ? j1 : big));
      const float fl = (float)lo, fh = (float)(hi - 1);
      const bool pos = step_ok(P1.cb, P1.gb, P2.cb, P2.gb, fl, fh, 1.0f) &&
                       step_ok(P2.cb, P2.gb, P3.cb, P3.gb, fl, fh, 1.0f);
      const bool neg = step_ok(P1.cb, P1.gb, P2.cb, P2.gb, fl, fh, -1.0f) &&
                       step_ok(P2.cb, P2.gb, P3.cb, P3.gb, fl, fh, -1.0f);
      if (__ballot(!pos) == 0) {
        tripled = true;
      } else if (__ballot(!neg) == 0) {
        tripled = true;
        swap = true;
      }
    }
  }
  if (tripled) {
    // the ray with the lowest axis-2 coordinate addresses the shared load
    RaySetup A = swap ? P3 : P1, B = P2, C = swap ? P1 : P3;
    A.i0 = swap ? R3.i0 : R1.i0;
    A.i1 = swap ? R3.i1 : R1.i1;
    B.i0 = R2.i0;
    B.i1 = R2.i1;
    C.i0 = swap ? R1.i0 : R3.i0;
    C.i1 = swap ? R1.i1 : R3.i1;
    float sa, sb, sc;
    fwd_loop_rowuniform_triple<T, WF, GRP>(a, A, B, C, lm, lca, lga, lo, hi, mid_lo, mid_hi, sa,
                                           sb, sc);
    const float acc1 = has1 ? (swap ? sc : sa) : 0.0f;
    const float acc2 = has2 ? sb : 0.0f;
    const float acc3 = has3 ? (swap ? sa : sc) : 0.0f;
    float* out = a.sino + ((size_t)view * a.n_u + iu) * a.n_v + iv;
    if (valid1) out[0] = acc1 * R1.scale;
    if (valid2) out[1] = acc2 * R2.scale;
    if (valid3) out[2] = acc3 * R3.scale;
  } else {
    // one ray set after another; the setups are recomputed so that they do
    // not stay live through the other rays' loops
    fwd_ray<T, WF, IDX64, GRP>(a, view, iu, iv, valid1);
    fwd_ray<T, WF, IDX64, GRP>(a, view, iu, iv + 1, valid2);
    fwd_ray<T, WF, IDX64, GRP>(a, view, iu, iv + 2, valid3);
  }
}

// RPL: rays per lane (1; 2 in 128-wide tiles or 3 in 192-wide tiles, 16-bit
// storage).
// Tile t of a view: consecutive tiles are neighbouring column groups of one
// band of detector rows (v), so the workgroups that run together on an XCD
// read neighbouring voxel rows of the same axis-2 range and share them in L2
// (c3 FP32 forward 83.5 -> 69.3 ms against row bands taken one after another
// within a column group; bitwise the same sums).
template <typename T, int WF, bool IDX64, int GRP, int RPL>
__device__ __forceinline__ void fwd_tile(const FwdArgs& a, int view, int t) {
  const int tv = t / a.tiles_u;
  const int tu = t - tv * a.tiles_u;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int k = a.tile_v_log2;
  if constexpr (RPL == 3) {
    if (k == 8) {
      // 192 pixels along v per wavefront, three per lane; four columns
      const int iv = tv * 192 + 3 * lane;
      const int iu = tu * 4 + wave;
      const bool col = iu < a.n_u;
      const bool v1 = col && iv < a.n_v, v2 = v1 && iv + 1 < a.n_v, v3 = v1 && iv + 2 < a.n_v;
      fwd_ray_triple<T, WF, IDX64, GRP>(a, view, col ? iu : 0, v1 ? iv : 0, v1, v2, v3);
      return;
    }
  }
  if constexpr (RPL == 2 && sizeof(T) == 2) {
    if (k == 7) {
      // 128 pixels along v per wavefront, two per lane; four columns
      const int iv = (tv << 7) + 2 * lane;
      const int iu = tu * 4 + wave;
      const bool col = iu < a.n_u;
      const bool v1 = col && iv < a.n_v, v2 = col && iv + 1 < a.n_v;
      fwd_ray_pair<T, WF, IDX64, GRP>(a, view, col ? iu : 0, v1 ? iv : 0, v1, v2 && v1);
      return;
    }
  }
  const int rows = 64 >> k;
  const int iv = (tv << k) + (lane & ((1 << k) - 1));
  const int iu = tu * (4 * rows) + wave * rows + (lane >> k);
  const bool valid = iu < a.n_u && iv < a.n_v;
  fwd_ray<T, WF, IDX64, GRP>(a, view, valid ? iu : 0, valid ? iv : 0, valid);
}

// Launch order: groups of view_group consecutive views; within a group each
// tile comes up for all the group's views in turn. Rays of nearby views cross
// nearly the same voxels, so the workgroups resident on an XCD share their
// volume reads in L2 instead of each view streaming the volume again.
template <typename T, int WF, bool IDX64, int GRP, int RPL>
__device__ __forceinline__ void fwd_block(const FwdArgs& a) {
  uint32_t b = blockIdx.x;
  if (a.remap) b = xcd_remap(b, gridDim.x);
  const uint32_t K = (uint32_t)a.view_group, tpv = (uint32_t)a.tiles_per_view;
  const uint32_t grp = b / (K * tpv);
  const uint32_t r = b - grp * K * tpv;
  const uint32_t v0 = grp * K;
  const uint32_t kg = min(K, (uint32_t)a.n_views - v0);  // views in this group
  const uint32_t t = r / kg;
  fwd_tile<T, WF, IDX64, GRP, RPL>(a, (int)(v0 + (r - t * kg)), (int)t);
}

template <typename T, int WF, bool IDX64, int GRP>
__global__ __launch_bounds__(256) void fwd_kernel(const FwdArgs a) {
  fwd_block<T, WF, IDX64, GRP, 1>(a);
}

// Two rays per lane (16-bit storage, 128-wide tiles).
template <typename T, int WF, bool IDX64, int GRP>
__global__ __launch_bounds__(256) void fwd_pair_kernel(const FwdArgs a) {
  fwd_block<T, WF, IDX64, GRP, 2>(a);
}

// Three rays per lane (192-wide tiles).
template <typename T, int WF, bool IDX64, int GRP>
__global__ __launch_bounds__(256) void fwd_triple_kernel(const FwdArgs a) {
  fwd_block<T, WF, IDX64, GRP, 3>(a);
}

// ---------------------------------------------------------------------------
// Plain forward for comparison: one lane per ray in sinogram order (v
// fastest), the four neighbours of a sample read one by one from the
// unpadded volume with a bounds test each (zero outside, Eq. 8), no padded
// copies, tiling, view grouping or shared row setup. Same ray setup, weights
// and summation order as the tuned kernel.
__device__ __forceinline__ float widen1(float x) { return x; }
__device__ __forceinline__ float widen1(bf16_t x) { return __uint_as_float((uint32_t)x.bits << 16); }
__device__ __forceinline__ float widen1(f16_t x) {
  return (float)__builtin_bit_cast(_Float16, x.bits);
}

// Voxel (i, a, b) on the (driving, first, second transverse) axes, zero
// outside the grid; i is always inside.
template <typename T>
__device__ __forceinline__ float voxel_or_zero(const T* __restrict__ vol, long long off, int a,
                                               int b, int na, int nb, long long sa, long long sb) {
  if (a < 0 || a >= na || b < 0 || b >= nb) return 0.0f;
  return widen1(vol[off + a * sa + b * sb]);
}

template <typename T, int WF>
__global__ __launch_bounds__(256) void naive_fwd_kernel(const GridGeom G,
                                                        const double* __restrict__ views,
                                                        const T* __restrict__ vol, int n_u,
                                                        int n_v, long long n_rays,
                                                        float* __restrict__ sino) {
  const long long ray = (long long)blockIdx.x * 256 + threadIdx.x;
  if (ray >= n_rays) return;
  const long long per_view = (long long)n_u * n_v;
  const int view = (int)(ray / per_view);
  const int rem = (int)(ray - (long long)view * per_view);
  const int iu = rem / n_v, iv = rem - (rem / n_v) * n_v;
  RaySetup R;
  ray_setup(views + 12 * (size_t)view, G, iu, iv, R);
  // strides of the C-order volume: axis 0 n1*n2, axis 1 n2, axis 2 1
  const long long st0 = (long long)G.n[1] * G.n[2], st1 = G.n[2];
  const long long sm = R.m == 0 ? st0 : (R.m == 1 ? st1 : 1);
  const long long sa = R.ta == 0 ? st0 : st1;  // ta < tb, so ta is 0 or 1
  const long long sb = R.tb == 1 ? st1 : 1;    // and tb is 1 or 2
  const int na = G.n[R.ta == 0 ? 0 : 1], nb = G.n[R.tb == 1 ? 1 : 2];
  const float hia = G.hi[R.ta == 0 ? 0 : 1], hib = G.hi[R.tb == 1 ? 1 : 2];
  float acc = 0.0f;
  float fi = (float)R.i0;
  for (int i = R.i0; i < R.i1; ++i) {
    int ia, ib;
    float wfa, wca, wfb, wcb;
    sample_axis<WF>(fi, R.ga, R.ca, hia, ia, wfa, wca);
    sample_axis<WF>(fi, R.gb, R.cb, hib, ib, wfb, wcb);
    const long long off = (long long)i * sm;
    Quad q;
    q.a0z0 = voxel_or_zero(vol, off, ia, ib, na, nb, sa, sb);
    q.a0z1 = voxel_or_zero(vol, off, ia, ib + 1, na, nb, sa, sb);
    q.a1z0 = voxel_or_zero(vol, off, ia + 1, ib, na, nb, sa, sb);
    q.a1z1 = voxel_or_zero(vol, off, ia + 1, ib + 1, na, nb, sa, sb);
    acc = accumulate4(acc, wfa, wca, wfb, wcb, q);
    fi += 1.0f;
  }
  sino[ray] = acc * R.scale;
}

// ---------------------------------------------------------------------------
// Adjoint pass 1: per-ray table for views [view0, view0 + n_chunk).
// General layout, two float4 per ray: {m | i0 << 2 | i1 << 17, ca, ga, cb},
// {gb, y * scale, 0, 0}. Column layout (see adj_gather_sep_kernel): one float4
// per ray {m | i0 << 2 | i1 << 17, cb, gb, y * scale}, each detector column's
// rays followed by kColumnPad zero entries, and one float4 per detector column
// {m, ca, ga, 0}.
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
      float4* col = table + ((size_t)cv * n_u + iu) * (size_t)(n_v + kColumnPad);
      col[iv] = make_float4(__uint_as_float(mr), R.cb, R.gb, y * R.scale);
      if (iv == 0) {
        cols[(size_t)cv * n_u + iu] = make_float4(__uint_as_float((uint32_t)R.m), R.ca, R.ga, 0.0f);
        for (int k = 0; k < kColumnPad; ++k) col[n_v + k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
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

// Value table of the column layout for unclipped column geometries: per ray
// only y * step length, each detector column's rays followed by kColumnPad
// zeros, and per column the double-precision affine map of its rays
// (ResCol). Only the ray's line is set up (no sample range: without clipping
// a ray with no samples has no position within a voxel of the grid, so the
// gather never weights its value). mask: driving axes per view.
__global__ __launch_bounds__(256) void adj_value_table_kernel(const double* __restrict__ views,
                                                              const GridGeom G,
                                                              const float* __restrict__ sino,
                                                              int n_u, int n_v, int view0,
                                                              long long n_rays,
                                                              float* __restrict__ vals,
                                                              ResCol* __restrict__ cols,
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
    const double* v = views + 12 * (size_t)(view0 + cv);
    double s[3], g[3];
    int m, a, b;
    float scale;
    const bool dir = ray_line(v, G, iu, iv, s, g, m, a, b, scale);
    const float y = sino[(size_t)(view0 + cv) * per_view + rem];
    float* col = vals + ((size_t)cv * n_u + iu) * (size_t)(n_v + kColumnPad);
    col[iv] = y * scale;
    if (iv == 0) {
      for (int k = 0; k < kColumnPad; ++k) col[n_v + k] = 0.0f;
      // every ray v of the column: driving axis m, in-plane coordinate
      // fma(i, ga, ca) (the forward's coefficients), axis-2 coordinate
      // A + v B on plane i with t = (i - sm) inv_rm, A = a0 + t a1,
      // B = b0 + t b1 (dv_m = 0)
      ResCol c;
      c.m = (dir && m < 2) ? m : -1;
      const double neg_sm = -s[m];
      c.ca = dir ? (float)(s[a] + neg_sm * g[a]) : 0.0f;
      c.ga = dir ? (float)g[a] : 0.0f;
      c.pad = 0.0f;
      const int mm = c.m < 0 ? 0 : c.m;
      const double dm = v[3 + mm] + (double)iu * v[6 + mm];
      const double d2 = v[5] + (double)iu * v[8];
      double rm;
      if (G.beam == BEAM_CONE) {  // s + t (d(v) - s)
        rm = dm - v[mm];
        c.sm = v[mm];
        c.a0 = v[2];
        c.a1 = d2 - v[2];
        c.b0 = 0.0;
        c.b1 = v[11];
      } else {  // d(v) + t r
        rm = v[mm];
        c.sm = dm;
        c.a0 = d2;
        c.a1 = v[2];
        c.b0 = v[11];
        c.b1 = 0.0;
      }
      if (rm == 0.0) c.m = -1;
      c.inv_rm = rm != 0.0 ? 1.0 / rm : 0.0;
      cols[(size_t)cv * n_u + iu] = c;
      if (c.m >= 0) bits = 1 << c.m;
    }
  }
  __shared__ int s_bits[256];
  s_bits[threadIdx.x] = 0;
  __syncthreads();
  const long long r0 = (long long)blockIdx.x * 256;
  const int cv0 = (int)(r0 / per_view);
  if (bits) atomicOr(&s_bits[cv - cv0], bits);
  __syncthreads();
  const int bo = s_bits[threadIdx.x];
  if (bo) atomicOr(&mask[cv0 + (int)threadIdx.x], bo);
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
// memory once per chunk (no atomics on the volume in memory).
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
// denominator independent of z) whose length is bounded by a wave-uniform
// count. Each candidate sample is evaluated once for both voxels; each voxel
// sums its contributions in registers and is written once per launch. No LDS,
// no barriers, no atomics.
//
// The table holds each detector column's rays followed by kColumnPad empty
// entries (no samples, value 0), so a candidate list may run past the
// column's end.
// ---------------------------------------------------------------------------

// Weights of one sample for the voxels z and z + 1 (zero unless the sample's
// floor or floor + 1 is one of them). Linear, on the clamped coordinate p with
// s = p - z: voxel z takes the tent 1 - |s|, voxel z + 1 the tent
// min(s, 2 - s) cut at 0. These reproduce the forward's 1 - d and d bit for
// bit: p - z, p - floor(p) and 2 - s are exact differences of nearby floats,
// and 1 - (z - p) equals p - (z - 1) exactly. Other weights: the forward's
// floor and complementary weights, selected by the floor's position.
template <int WF>
__device__ __forceinline__ void pair_weights(float fplane, float g, float c, float hz, float fz,
                                             int z, float& b0, float& b1) {
  if constexpr (WF == W_LINEAR) {
    float p = __builtin_fmaf(fplane, g, c);
    p = __builtin_amdgcn_fmed3f(p, -1.0f, hz);
    const float s0 = p - fz;
    // clamp to [0, 1] (one instruction with the clamp modifier); 1 - |s| <= 1
    b0 = __builtin_amdgcn_fmed3f(1.0f - __builtin_fabsf(s0), 0.0f, 1.0f);
    // min(s, 2 - s) <= 1, so only the cut at 0 remains: the median of the three
    b1 = __builtin_amdgcn_fmed3f(s0, 2.0f - s0, 0.0f);
  } else {
    int ib;
    float wfb, wcb;
    sample_axis<WF>(fplane, g, c, hz, ib, wfb, wcb);
    const int d = ib - z;  // the sample's floor relative to the pair
    b0 = (d == 0) ? wfb : ((d == -1) ? wcb : 0.0f);
    b1 = (d == 1) ? wfb : ((d == 0) ? wcb : 0.0f);
  }
}

// NC candidate rays R[iv_lo .. iv_lo + NC), each loaded once and evaluated on
// the two planes p0 and p0 + 1 for the voxel pair (z, z + 1): sums s<plane><z>.
template <int WF, int NC>
__device__ __forceinline__ void block_candidates(const float4* __restrict__ R, int iv_lo, int p0,
                                                 float fp0, float hz, float fz, int z,
                                                 float& s00, float& s01, float& s10,
                                                 float& s11) {
  float4 rr[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) rr[k] = R[iv_lo + k];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const float4 r = rr[k];
    const uint32_t mr = __float_as_uint(r.x);
    const int i0 = (int)((mr >> 2) & 0x7fffu);
    const int i1 = (int)(mr >> 17);
    float b0, b1;
    pair_weights<WF>(fp0, r.z, r.y, hz, fz, z, b0, b1);
    const float wy0 = (p0 >= i0 && p0 < i1) ? r.w : 0.0f;
    s00 = __builtin_fmaf(wy0, b0, s00);
    s01 = __builtin_fmaf(wy0, b1, s01);
    pair_weights<WF>(fp0 + 1.0f, r.z, r.y, hz, fz, z, b0, b1);
    const float wy1 = (p0 + 1 >= i0 && p0 + 1 < i1) ? r.w : 0.0f;
    s10 = __builtin_fmaf(wy1, b0, s10);
    s11 = __builtin_fmaf(wy1, b1, s11);
  }
}

// Weights of a sample at signed distance s = p - z from voxel z for the voxels
// z and z + 1 (the tents of pair_weights on the unclamped coordinate; the
// spline of Eq. 14 at |s| and |s - 1|).
template <int WF>
__device__ __forceinline__ void pair_weights_rel(float s, float& b0, float& b1) {
  if constexpr (WF == W_LINEAR) {
    b0 = __builtin_amdgcn_fmed3f(1.0f - __builtin_fabsf(s), 0.0f, 1.0f);
    b1 = __builtin_amdgcn_fmed3f(s, 2.0f - s, 0.0f);
  } else {
    const float t0 = fminf(__builtin_fabsf(s), 1.0f), t1 = fminf(__builtin_fabsf(s - 1.0f), 1.0f);
    b0 = __builtin_fmaf(t0 * t0, __builtin_fmaf(2.0f, t0, -3.0f), 1.0f);
    b1 = __builtin_fmaf(t1 * t1, __builtin_fmaf(2.0f, t1, -3.0f), 1.0f);
  }
}

// Value-table form of block_candidates (unclipped column geometries): NC
// candidate values R[iv_lo ...]; candidate k lies at signed distance
// base_p + k B_p from voxel z on plane p0 + p (base_p formed in double
// precision per lane, so positions keep single-precision accuracy relative to
// the voxel).
template <int WF, int NC>
__device__ __forceinline__ void block_candidates_val(const float* __restrict__ R, int iv_lo,
                                                     float base0, float B0, float base1,
                                                     float B1, float& s00, float& s01,
                                                     float& s10, float& s11) {
  float g[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) g[k] = R[iv_lo + k];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    float b0, b1;
    pair_weights_rel<WF>(__builtin_fmaf((float)k, B0, base0), b0, b1);
    s00 = __builtin_fmaf(g[k], b0, s00);
    s01 = __builtin_fmaf(g[k], b1, s01);
    pair_weights_rel<WF>(__builtin_fmaf((float)k, B1, base1), b0, b1);
    s10 = __builtin_fmaf(g[k], b0, s10);
    s11 = __builtin_fmaf(g[k], b1, s11);
  }
}

// Workgroup placement of the gather: a lane owns a 2 x 2 x 2 voxel block
// (x, x+1) x (y, y+1) x (z, z+1); a wavefront covers 128 voxels along axis 2
// and a workgroup four such wavefronts along y (8 rows). Logical workgroup
// indices are ordered in tiles of GTX x-pairs by GTY row blocks (axis-2 blocks
// fastest), and each XCD walks one contiguous range of them, so the
// workgroups resident on an XCD cover a compact (x, y) region whose rays come
// from a few detector columns per view: the ray table they read stays in that
// XCD's L2.
constexpr int GTX = 8, GTY = 4;

__host__ __device__ inline void gather_grid(const int* n, int& nzb, int& nyb, int& ntx, int& nty) {
  nzb = (n[2] + 127) / 128;
  nyb = (n[1] + 7) / 8;
  ntx = ((n[0] + 1) / 2 + GTX - 1) / GTX;
  nty = (nyb + GTY - 1) / GTY;
}

// The two planes of a lane's block along the driving axis m, each with the
// two in-plane rows: one candidate list per column serves both rows (the
// column's in-plane weight differs per row, the axis-2 weights do not).
// VAL: value table (adj_value_table_kernel) with positions from each
// column's affine map and no per-ray range test (unclipped geometries only);
// otherwise the ray table of adj_table_kernel.
template <int WF, bool VAL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void adj_gather_sep_kernel(
    const GridGeom G, int n_u, int n_v, const float* __restrict__ proj,
    const float4* __restrict__ rays, const float4* __restrict__ cols,
    const float* __restrict__ vals, const ResCol* __restrict__ rcols,
    const int* __restrict__ mask, int view0, int c0, int n_chunk, int accumulate,
    float* __restrict__ vol) {
  int nzb, nyb, ntx, nty;
  gather_grid(G.n, nzb, nyb, ntx, nty);
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t per_tile = (uint32_t)(GTX * GTY * nzb);
  const int tile = (int)(L / per_tile);
  const int w = (int)(L - (uint32_t)tile * per_tile);
  const int zb = w % nzb;
  const int iyb = (w / nzb) % GTY;
  const int ixp = w / (nzb * GTY);
  const int x = 2 * ((tile / nty) * GTX + ixp);
  const int yb = (tile % nty) * GTY + iyb;
  if (x >= G.n[0] || yb >= nyb) return;
  const int y = yb * 8 + 2 * __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (y >= G.n[1]) return;
  const int z = 2 * (zb * 64 + (int)(threadIdx.x & 63));
  const bool zin = z < G.n[2];
  const float fz = (float)z;
  const double dz = (double)z;
  const float hz = G.hi[2];
  const float e = 0.002f;       // widened neighbourhood (voxels)
  const float margin = 0.05f;   // widened ranges (pixels)
  const int pitch = n_v + kColumnPad;  // table entries per detector column
  // acc_XYZ: voxel (x + X, y + Y, z + Z)
  float acc000 = 0.0f, acc001 = 0.0f, acc010 = 0.0f, acc011 = 0.0f;
  float acc100 = 0.0f, acc101 = 0.0f, acc110 = 0.0f, acc111 = 0.0f;
  // The block's planes are x for driving axis 0 and y for axis 1: around the
  // columns of axis 1 the accumulators of voxels (x + 1, y, .) and
  // (x, y + 1, .) trade places, so that one plane/row mapping serves both axes
  // (no per-column select).
  auto swap_planes_rows = [&]() {
    const float t0 = acc010, t1 = acc011;
    acc010 = acc100;
    acc011 = acc101;
    acc100 = t0;
    acc101 = t1;
  };
  for (int c = c0; c < c0 + n_chunk; ++c) {
    const int mk = mask[c];
    if (!mk) continue;
    const float* P = proj + 12 * (size_t)(view0 + c);
    const float4* C = VAL ? nullptr : cols + (size_t)c * n_u;
    const float4* RY = VAL ? nullptr : rays + (size_t)c * n_u * pitch;
    const ResCol* RC = VAL ? rcols + (size_t)c * n_u : nullptr;
    const float* RV = VAL ? vals + (size_t)c * n_u * pitch : nullptr;
    for (int m = 0; m < 2; ++m) {
      if (!(mk & (1 << m))) continue;
      if (m == 1) swap_planes_rows();
      const int va = (m == 0) ? y : x;  // first of the two in-plane rows
      const float fva = (float)va;
      const float ha = (m == 0) ? G.hi[1] : G.hi[0];
      const int p0 = (m == 0) ? x : y;  // first of the two planes
      const float fp0 = (float)p0, fp1 = fp0 + 1.0f;
      const bool two = p0 + 1 < G.n[m];
      // candidate columns: u of (plane, va - (1 + e)) and (plane, va + 1 + (1 + e))
      // on both planes
      const float qa0 = fva - 1.0f - e, qa1 = fva + 2.0f + e;
      int iu_lo = n_u, iu_hi = -1;
      bool iu_all = false;
      for (int dp = 0; dp < 2; ++dp) {
        const float fpl = dp ? fp1 : fp0;
        const float qx0 = (m == 0) ? fpl : qa0, qy0 = (m == 0) ? qa0 : fpl;
        const float qx1 = (m == 0) ? fpl : qa1, qy1 = (m == 0) ? qa1 : fpl;
        const float un0 = __builtin_fmaf(P[0], qx0, __builtin_fmaf(P[1], qy0, P[3]));
        const float w0 = __builtin_fmaf(P[8], qx0, __builtin_fmaf(P[9], qy0, P[11]));
        const float un1 = __builtin_fmaf(P[0], qx1, __builtin_fmaf(P[1], qy1, P[3]));
        const float w1 = __builtin_fmaf(P[8], qx1, __builtin_fmaf(P[9], qy1, P[11]));
        if (w0 > 1.0e-6f && w1 > 1.0e-6f) {
          const float u0 = un0 * __builtin_amdgcn_rcpf(w0), u1 = un1 * __builtin_amdgcn_rcpf(w1);
          iu_lo = min(iu_lo, max(0, (int)ceilf(fmaxf(fminf(u0, u1) - margin, -1.0f))));
          iu_hi = max(iu_hi, min(n_u - 1, (int)floorf(fminf(fmaxf(u0, u1) + margin, (float)n_u))));
        } else {
          iu_all = true;
        }
      }
      if (iu_all) {
        iu_lo = 0;
        iu_hi = n_u - 1;
      }
      // the projective rows' terms in the driving coordinate (fixed per plane)
      // and their coefficients of the in-plane coordinate (the window below
      // is a bound with margins, so this order of rounding is free)
      const float PfA = (m == 0) ? P[4] : P[5], PaA = (m == 0) ? P[5] : P[4];
      const float PfW = (m == 0) ? P[8] : P[9], PaW = (m == 0) ? P[9] : P[8];
      const float KA0 = __builtin_fmaf(PfA, fp0, P[7]), KA1 = __builtin_fmaf(PfA, fp1, P[7]);
      const float KW0 = __builtin_fmaf(PfW, fp0, P[11]), KW1 = __builtin_fmaf(PfW, fp1, P[11]);
      for (int iu = iu_lo; iu <= iu_hi; ++iu) {
        float4 col;
        if constexpr (VAL) {
          const ResCol& rc = RC[iu];
          col = make_float4(__int_as_float(rc.m), rc.ca, rc.ga, 0.0f);
        } else {
          col = C[iu];
        }
        if ((int)__float_as_uint(col.x) != m) continue;
        // in-plane weights wA<plane><row> (rows va, va + 1; va is even, as z
        // is, so the tents reproduce the forward's weights exactly)
        float wA00, wA01, wA10, wA11;
        pair_weights<WF>(fp0, col.z, col.y, ha, fva, va, wA00, wA01);
        pair_weights<WF>(fp1, col.z, col.y, ha, fva, va, wA10, wA11);
        if (!two) {
          wA10 = 0.0f;
          wA11 = 0.0f;
        }
        if (wA00 == 0.0f && wA01 == 0.0f && wA10 == 0.0f && wA11 == 0.0f) continue;
        const float4* R = VAL ? nullptr : RY + (size_t)iu * pitch;
        const float* RVc = VAL ? RV + (size_t)iu * pitch : nullptr;
        float s00 = 0.0f, s01 = 0.0f, s10 = 0.0f, s11 = 0.0f;
        int nc = 0;  // wave-uniform bound on the candidates per lane
        float win_hi = 3.0e38f;  // upper end of the lane's window (none: every ray)
        int iv_lo = 0, iv_hi = n_v - 1;
        double Ad0 = 0.0, Bd0 = 0.0, Ad1 = 0.0, Bd1 = 0.0;
        if constexpr (VAL) {
          // the column's rays on the two planes: A + v B (double precision);
          // ray v reaches axis-2 position zz at v = (zz - A) / B
          const ResCol& rc = RC[iu];
          const double t0 = ((double)p0 - rc.sm) * rc.inv_rm;
          Ad0 = fma(t0, rc.a1, rc.a0);
          Bd0 = fma(t0, rc.b1, rc.b0);
          Ad1 = fma(rc.inv_rm, rc.a1, Ad0);
          Bd1 = fma(rc.inv_rm, rc.b1, Bd0);
          const float Bf0 = (float)Bd0, Bf1 = (float)Bd1;
          const float ib0 = __builtin_amdgcn_rcpf(Bf0), ib1 = __builtin_amdgcn_rcpf(Bf1);
          if (Bf0 * Bf1 > 0.0f && __builtin_fabsf(ib0) < 1.0e4f && __builtin_fabsf(ib1) < 1.0e4f) {
            // rays whose axis-2 coordinate lies in [z - 1, z + 2) on either plane
            const float Af0 = (float)Ad0, Af1 = (float)Ad1;
            const float za = fz - 1.0f - e, zc = fz + 2.0f + e;
            const float a0 = (za - Af0) * ib0, a1 = (zc - Af0) * ib0;
            const float c0 = (za - Af1) * ib1, c1 = (zc - Af1) * ib1;
            const float lo = fminf(fminf(a0, a1), fminf(c0, c1)) - 0.01f;
            win_hi = fmaxf(fmaxf(a0, a1), fmaxf(c0, c1)) + 0.01f;
            iv_lo = min(max((int)ceilf(fmaxf(lo, -1.0f)), 0), n_v);
            // longest window of the wavefront: lanes 0 and 63, as below
            const float len = win_hi - lo;
            const int len_a = __builtin_amdgcn_readlane(__builtin_bit_cast(int, len), 0);
            const int len_b = __builtin_amdgcn_readlane(__builtin_bit_cast(int, len), 63);
            nc = (int)(__builtin_bit_cast(float, max(len_a, len_b)) + 1.0e-3f) + 1;
            if (!zin) iv_lo = n_v;  // reads the column's zero padding only
          }
        } else {
          // v of the column's rays on each plane: (A + P6 z) / W, affine in z;
          // A and W are the plane terms (per axis) plus the column's in-plane term
          const float pa0 = __builtin_fmaf(fp0, col.z, col.y), pa1 = __builtin_fmaf(fp1, col.z, col.y);
          const float A0 = __builtin_fmaf(PaA, pa0, KA0), W0 = __builtin_fmaf(PaW, pa0, KW0);
          const float A1 = __builtin_fmaf(PaA, pa1, KA1), W1 = __builtin_fmaf(PaW, pa1, KW1);
          if (W0 > 1.0e-6f && W1 > 1.0e-6f) {
            // rays whose axis-2 coordinate lies in [z - 1, z + 2) on either plane
            const float inv0 = __builtin_amdgcn_rcpf(W0), inv1 = __builtin_amdgcn_rcpf(W1);
            const float sl0 = P[6] * inv0, sl1 = P[6] * inv1;  // pixels per voxel along z
            const float b0 = A0 * inv0, b1 = A1 * inv1;
            // span of the union window at axis-2 position zz (convex in zz)
            auto window = [&](float zz, float& lo, float& hi) {
              const float a0 = __builtin_fmaf(sl0, zz - 1.0f - e, b0);
              const float a1 = __builtin_fmaf(sl0, zz + 2.0f + e, b0);
              const float c0 = __builtin_fmaf(sl1, zz - 1.0f - e, b1);
              const float c1 = __builtin_fmaf(sl1, zz + 2.0f + e, b1);
              lo = fminf(fminf(a0, a1), fminf(c0, c1)) - margin;
              hi = fmaxf(fmaxf(a0, a1), fmaxf(c0, c1)) + margin;
            };
            float lo;
            window(fz, lo, win_hi);
            iv_lo = min(max((int)ceilf(fmaxf(lo, -1.0f)), 0), n_v);
            // an interval of length L holds at most floor(L) + 1 integers; the
            // longest window of the wavefront is at one of its ends, which are
            // lanes 0 and 63 (axis-2 positions 128 zb and 128 zb + 126; every
            // branch of the column loop is wave-uniform, so all 64 lanes are
            // active here). The lengths are positive floats, whose bit patterns
            // order as they do.
            const float len = win_hi - lo;
            const int len_a = __builtin_amdgcn_readlane(__builtin_bit_cast(int, len), 0);
            const int len_b = __builtin_amdgcn_readlane(__builtin_bit_cast(int, len), 63);
            nc = (int)(__builtin_bit_cast(float, max(len_a, len_b)) + 1.0e-3f) + 1;
            if (!zin) iv_lo = n_v;  // reads the column's empty entries only
          }
        }
        if constexpr (VAL) {
          // candidate positions relative to the voxel, from iv_lo on
          const double dlo = (double)iv_lo;
          const float base0 = (float)fma(dlo, Bd0, Ad0 - dz);
          const float base1 = (float)fma(dlo, Bd1, Ad1 - dz);
          const float B0 = (float)Bd0, B1 = (float)Bd1;
          switch (nc) {
            case 1:
            case 2: block_candidates_val<WF, 2>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 3: block_candidates_val<WF, 3>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 4: block_candidates_val<WF, 4>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 5: block_candidates_val<WF, 5>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 6: block_candidates_val<WF, 6>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 7: block_candidates_val<WF, 7>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            case 8: block_candidates_val<WF, 8>(RVc, iv_lo, base0, B0, base1, B1, s00, s01, s10, s11); break;
            default:
              // long or unbounded candidate ranges: explicit per-lane loop
              iv_hi = min(n_v - 1, (int)floorf(fminf(win_hi, (float)n_v)));
              if (!zin) iv_hi = iv_lo - 1;
              for (int iv = iv_lo; iv <= iv_hi; ++iv) {
                const float gv = RVc[iv];
                const float fk = (float)(iv - iv_lo);
                float c0, c1;
                pair_weights_rel<WF>(__builtin_fmaf(fk, B0, base0), c0, c1);
                s00 = __builtin_fmaf(gv, c0, s00);
                s01 = __builtin_fmaf(gv, c1, s01);
                pair_weights_rel<WF>(__builtin_fmaf(fk, B1, base1), c0, c1);
                s10 = __builtin_fmaf(gv, c0, s10);
                s11 = __builtin_fmaf(gv, c1, s11);
              }
              break;
          }
        } else {
          switch (nc) {
            case 1:
            case 2: block_candidates<WF, 2>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 3: block_candidates<WF, 3>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 4: block_candidates<WF, 4>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 5: block_candidates<WF, 5>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 6: block_candidates<WF, 6>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 7: block_candidates<WF, 7>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            case 8: block_candidates<WF, 8>(R, iv_lo, p0, fp0, hz, fz, z, s00, s01, s10, s11); break;
            default:
              // long or unbounded candidate ranges: explicit per-lane loop
              iv_hi = min(n_v - 1, (int)floorf(fminf(win_hi, (float)n_v)));
              if (!zin) iv_hi = iv_lo - 1;
              for (int iv = iv_lo; iv <= iv_hi; ++iv) {
                const float4 r = R[iv];
                const uint32_t mr = __float_as_uint(r.x);
                const int i0 = (int)((mr >> 2) & 0x7fffu);
                const int i1 = (int)(mr >> 17);
                float c0, c1;
                if (p0 >= i0 && p0 < i1) {
                  pair_weights<WF>(fp0, r.z, r.y, hz, fz, z, c0, c1);
                  s00 = __builtin_fmaf(r.w, c0, s00);
                  s01 = __builtin_fmaf(r.w, c1, s01);
                }
                if (p0 + 1 >= i0 && p0 + 1 < i1) {
                  pair_weights<WF>(fp1, r.z, r.y, hz, fz, z, c0, c1);
                  s10 = __builtin_fmaf(r.w, c0, s10);
                  s11 = __builtin_fmaf(r.w, c1, s11);
                }
              }
              break;
          }
        }
        // block voxel (plane p0 + d, row va + r, z + k) gets wA<d><r> s<d><k>
        acc000 = __builtin_fmaf(wA00, s00, acc000); acc001 = __builtin_fmaf(wA00, s01, acc001);
        acc010 = __builtin_fmaf(wA01, s00, acc010); acc011 = __builtin_fmaf(wA01, s01, acc011);
        acc100 = __builtin_fmaf(wA10, s10, acc100); acc101 = __builtin_fmaf(wA10, s11, acc101);
        acc110 = __builtin_fmaf(wA11, s10, acc110); acc111 = __builtin_fmaf(wA11, s11, acc111);
      }
      if (m == 1) swap_planes_rows();
    }
  }
  if (!zin) return;
  const bool z1 = z + 1 < G.n[2];
  const bool y1 = y + 1 < G.n[1];
  const bool x1 = x + 1 < G.n[0];
  const size_t sx = (size_t)G.n[1] * G.n[2], sy = (size_t)G.n[2];
  float* o = vol + (size_t)x * sx + (size_t)y * sy + z;
  auto put = [&](float* q, float v) { *q = accumulate ? (*q + v) : v; };
  put(o, acc000);
  if (z1) put(o + 1, acc001);
  if (y1) {
    put(o + sy, acc010);
    if (z1) put(o + sy + 1, acc011);
  }
  if (x1) {
    put(o + sx, acc100);
    if (z1) put(o + sx + 1, acc101);
    if (y1) {
      put(o + sx + sy, acc110);
      if (z1) put(o + sx + sy + 1, acc111);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched forward: zero-padded copies of every instance, queue reset, and a
// persistent kernel pulling (instance, view, tile) items from a device queue.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void batched_pad_kernel(const BatchInst* __restrict__ insts) {
  const BatchInst& I = insts[blockIdx.y];
  const int n0 = I.a.G.n[0], n1 = I.a.G.n[1], n2 = I.a.G.n[2];
  const long long p2 = padded_pitch(n2), p1 = n1 + 2;
  const long long total = I.padded_elems;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (long long)gridDim.x * 256) {
    const int z = (int)(e % p2);
    const long long t = e / p2;
    const int y = (int)(t % p1);
    const int x = (int)(t / p1);
    if (I.dtype != 0)
      pad_pair_element(static_cast<const uint16_t*>(I.src),
                       static_cast<uint16_t*>(const_cast<void*>(I.a.vol_a)),
                       static_cast<uint16_t*>(const_cast<void*>(I.a.vol_b)), n0, n1, n2, e, x,
                       y, z);
    else
      pad_pair_element(static_cast<const uint32_t*>(I.src),
                       static_cast<uint32_t*>(const_cast<void*>(I.a.vol_a)),
                       static_cast<uint32_t*>(const_cast<void*>(I.a.vol_b)), n0, n1, n2, e, x,
                       y, z);
  }
}

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Persistent batched forward for one instance class (storage type T, weight
// WF, addressing IDX64, rays per lane RPL). The class's items come in
// kBatchQueues queues, one per XCD, each holding whole view groups (a tile's
// items for the group's views in turn) so that the views sharing volume lines
// run on one XCD's L2: queue q is items [qoff[q], qoff[q + 1]) with counter
// counters[q]. A workgroup drains the queue of the XCD it runs on (workgroups
// are dispatched to the XCDs round robin), then helps with the others; every
// counter only grows, so each workgroup leaves after at most one failed pull
// per queue.
template <typename T, int WF, bool IDX64, int RPL>
__device__ __forceinline__ void batched_loop(const BatchInst* __restrict__ insts,
                                             const uint2* __restrict__ items,
                                             const int* __restrict__ qoff,
                                             int* __restrict__ counters) {
  __shared__ int s_item;
  const int home = (int)(blockIdx.x % kBatchQueues);
  for (int d = 0; d < kBatchQueues; ++d) {
    const int q = (home + d) % kBatchQueues;
    const int begin = qoff[q], n = qoff[q + 1] - begin;
    for (;;) {
      if (threadIdx.x == 0) s_item = atomicAdd(&counters[q], 1);
      __syncthreads();
      const int item = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
      if (item >= n) break;
      const uint2 it = items[begin + item];
      const int inst = (int)(it.x & 0xfffu);
      const int view = (int)(it.x >> 12);
      fwd_tile<T, WF, IDX64, kBatchRuGroup, RPL>(insts[inst].a, view, (int)it.y);
    }
  }
}

// One ray per lane (tiles of 64, 32 or 16 pixels along v).
template <typename T, int WF, bool IDX64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void batched_fwd_kernel(
    const BatchInst* __restrict__ insts, const uint2* __restrict__ items,
    const int* __restrict__ qoff, int* __restrict__ counters) {
  batched_loop<T, WF, IDX64, 1>(insts, items, qoff, counters);
}

// Three rays per lane (192-wide tiles): the instances whose tuned tile is the
// three-rays-per-lane one; a kernel of its own, as in the single launch, so
// that the one-ray class keeps its occupancy.
template <typename T, int WF, bool IDX64>
__global__ __launch_bounds__(256) void batched_fwd_triple_kernel(
    const BatchInst* __restrict__ insts, const uint2* __restrict__ items,
    const int* __restrict__ qoff, int* __restrict__ counters) {
  batched_loop<T, WF, IDX64, 3>(insts, items, qoff, counters);
}

// ---------------------------------------------------------------------------
// SART elementwise steps (subset update of the Sec. IV-B reconstruction).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sart_residual_kernel(long long n,
                                                            const float* __restrict__ b,
                                                            const float* ax,
                                                            const float* __restrict__ w,
                                                            float* out) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    const float wi = w[i];
    out[i] = wi > 0.0f ? (b[i] - ax[i]) / wi : 0.0f;
  }
}

__global__ __launch_bounds__(256) void sart_update_kernel(long long n, float* __restrict__ x,
                                                          const float* __restrict__ bp,
                                                          const float* __restrict__ c,
                                                          float lam, int nonneg) {
  for (long long j = (long long)blockIdx.x * 256 + threadIdx.x; j < n;
       j += (long long)gridDim.x * 256) {
    const float cj = c[j];
    float v = x[j];
    if (cj > 0.0f) v += lam * bp[j] / cj;
    if (nonneg) v = fmaxf(v, 0.0f);
    x[j] = v;
  }
}

static int check_launch(const char* what);

static unsigned elementwise_grid(long long n) {
  const long long blocks = (n + 255) / 256;
  return (unsigned)(blocks < 8192 ? (blocks < 1 ? 1 : blocks) : 8192);
}

int launch_sart_residual(long long n, const float* b, const float* ax, const float* w,
                         float* out, hipStream_t s) {
  if (n <= 0) return 0;
  TimedLaunch t = timing_begin("sart", s);
  sart_residual_kernel<<<elementwise_grid(n), 256, 0, s>>>(n, b, ax, w, out);
  timing_end("sart", t, s);
  return check_launch("sart residual kernel");
}

int launch_sart_update(long long n, float* x, const float* bp, const float* c, float lam,
                       int nonneg, hipStream_t s) {
  if (n <= 0) return 0;
  TimedLaunch t = timing_begin("sart", s);
  sart_update_kernel<<<elementwise_grid(n), 256, 0, s>>>(n, x, bp, c, lam, nonneg);
  timing_end("sart", t, s);
  return check_launch("sart update kernel");
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

// ---------------------------------------------------------------------------
// Fixed device scratch of the forward that allocates nothing
// (gjp_forward_project_noalloc): the two padded pair copies live in this
// file-scope array instead of the stream-ordered pool. Every device the
// library runs on holds its own copy until the process ends. In host code the
// array's name is only a stand-in for the symbol: its device address on the
// current device comes from hipGetSymbolAddress, once per device, and only
// that address is passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[gjp_geometry::kMaxDev] = {};
}  // namespace

int noalloc_scratch(void** ptr) {
  int dvc = 0;
  hipError_t e = hipGetDevice(&dvc);
  if (e != hipSuccess) return set_error(-3, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dvc < 0 || dvc >= gjp_geometry::kMaxDev) return set_error(-4, "device index");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dvc]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(-3, std::string("noalloc scratch: hipGetSymbolAddress: ") +
                               hipGetErrorString(e));
    g_scratch_ptr[dvc] = p;
  }
  *ptr = g_scratch_ptr[dvc];
  return 0;
}

int launch_pad(const void* src, void* copy_a, void* copy_b, int dtype, const int n[3],
               hipStream_t s) {
  dim3 grid((unsigned)((padded_pitch(n[2]) + 255) / 256), (unsigned)(n[1] + 2), (unsigned)(n[0] + 2));
  TimedLaunch t = timing_begin("pad", s);
  if (dtype == 0)
    pad_kernel<uint32_t><<<grid, 256, 0, s>>>(static_cast<const uint32_t*>(src),
                                               static_cast<uint32_t*>(copy_a),
                                               static_cast<uint32_t*>(copy_b), n[0], n[1], n[2]);
  else
    pad_kernel<uint16_t><<<grid, 256, 0, s>>>(static_cast<const uint16_t*>(src),
                                               static_cast<uint16_t*>(copy_a),
                                               static_cast<uint16_t*>(copy_b), n[0], n[1], n[2]);
  timing_end("pad", t, s);
  return check_launch("pad kernel");
}

#define GJP_FWD_LAUNCH(KERNEL)                                   \
  do {                                                           \
    if (a.ru_group == 2) {                                       \
      if (idx64)                                                 \
        KERNEL<T, WF, true, 2><<<grid, 256, 0, s>>>(a);          \
      else                                                       \
        KERNEL<T, WF, false, 2><<<grid, 256, 0, s>>>(a);         \
    } else {                                                     \
      if (idx64)                                                 \
        KERNEL<T, WF, true, 4><<<grid, 256, 0, s>>>(a);          \
      else                                                       \
        KERNEL<T, WF, false, 4><<<grid, 256, 0, s>>>(a);         \
    }                                                            \
  } while (0)

// Two rays per lane (tile_v_log2 7, 16-bit storage only) and three (8) are
// kernels of their own: their extra ray setups raise the register count,
// which the one-ray tiles should not pay in occupancy.
template <typename T, int WF>
static void launch_fwd_t(const FwdArgs& a, bool idx64, unsigned grid, hipStream_t s) {
  if (a.tile_v_log2 == 8) {
    GJP_FWD_LAUNCH(fwd_triple_kernel);
    return;
  }
  if constexpr (sizeof(T) == 2) {
    if (a.tile_v_log2 == 7) {
      GJP_FWD_LAUNCH(fwd_pair_kernel);
      return;
    }
  }
  GJP_FWD_LAUNCH(fwd_kernel);
}
#undef GJP_FWD_LAUNCH

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

template <typename T, int WF>
static void launch_naive_t(const GridGeom& G, const double* views, const void* vol, int n_u,
                           int n_v, long long n_rays, float* sino, unsigned grid, hipStream_t s) {
  naive_fwd_kernel<T, WF><<<grid, 256, 0, s>>>(G, views, static_cast<const T*>(vol), n_u, n_v,
                                                n_rays, sino);
}

int launch_forward_naive(const GridGeom& G, const double* views, const void* vol, int dtype,
                         int weight, int n_views, int n_u, int n_v, float* sino, hipStream_t s) {
  const long long n_rays = (long long)n_views * n_u * n_v;
  if (n_rays == 0) return 0;
  const long long nb = (n_rays + 255) / 256;
  if (nb > 0xffffffffll) return set_error(-4, "naive forward: too many rays for one launch");
  const unsigned grid = (unsigned)nb;
  TimedLaunch t = timing_begin("forward_naive", s);
  switch (dtype * 2 + weight) {
    case 0: launch_naive_t<float, W_LINEAR>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
    case 1: launch_naive_t<float, W_SPLINE>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
    case 2: launch_naive_t<bf16_t, W_LINEAR>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
    case 3: launch_naive_t<bf16_t, W_SPLINE>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
    case 4: launch_naive_t<f16_t, W_LINEAR>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
    default: launch_naive_t<f16_t, W_SPLINE>(G, views, vol, n_u, n_v, n_rays, sino, grid, s); break;
  }
  timing_end("forward_naive", t, s);
  return check_launch("naive forward kernel");
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

int launch_adjoint_value_table(const gjp_geometry* g, const double* views, const float* sino,
                               int view0, int n_chunk, float* vals, ResCol* cols, int* mask,
                               hipStream_t s) {
  const long long n_rays = (long long)n_chunk * g->n_u * g->n_v;
  const long long nb = (n_rays + 255) / 256;
  if (nb > 0xffffffffll) return set_error(-4, "adjoint: view chunk too large");
  TimedLaunch t = timing_begin("adjoint_table", s);
  adj_value_table_kernel<<<(unsigned)nb, 256, 0, s>>>(views, g->gg, sino, g->n_u, g->n_v, view0,
                                                       n_rays, vals, cols, mask);
  timing_end("adjoint_table", t, s);
  return check_launch("adjoint table kernel");
}

int launch_adjoint_gather(const gjp_geometry* g, const float* proj, const float4* table,
                          const float4* cols, const float* vals, const ResCol* rcols,
                          const int* mask, int view0, int c0, int n_chunk, bool accumulate,
                          float* vol, hipStream_t s) {
  TimedLaunch t = timing_begin("adjoint_gather", s);
  const int acc = accumulate ? 1 : 0;
  if (g->separable) {
    int nzb, nyb, ntx, nty;
    gather_grid(g->gg.n, nzb, nyb, ntx, nty);
    const unsigned long long nwg = (unsigned long long)ntx * GTX * nty * GTY * nzb;
    if (nwg > 0x7fffffffull) return set_error(-4, "adjoint: volume too large for one launch");
    const unsigned grid = (unsigned)nwg;
#define GJP_GATHER(W, V)                                                                      \
  adj_gather_sep_kernel<W, V><<<grid, 256, 0, s>>>(g->gg, g->n_u, g->n_v, proj, table, cols, \
                                                   vals, rcols, mask, view0, c0, n_chunk, acc, \
                                                   vol)
    if (vals) {
      if (g->weight == W_SPLINE)
        GJP_GATHER(W_SPLINE, true);
      else
        GJP_GATHER(W_LINEAR, true);
    } else {
      if (g->weight == W_SPLINE)
        GJP_GATHER(W_SPLINE, false);
      else
        GJP_GATHER(W_LINEAR, false);
    }
#undef GJP_GATHER
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

// Resident workgroups of a persistent kernel on the whole device.
static int persistent_grid(const void* kernel) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess ||
      per <= 0)
    per = 4;
  return cus * per;
}

template <typename T, int WF, bool IDX64, bool TRIPLE>
static int batched_grid_t() {
  if constexpr (TRIPLE)
    return persistent_grid(reinterpret_cast<const void*>(batched_fwd_triple_kernel<T, WF, IDX64>));
  else
    return persistent_grid(reinterpret_cast<const void*>(batched_fwd_kernel<T, WF, IDX64>));
}

template <typename T, int WF, bool IDX64, bool TRIPLE>
static void launch_batched_t(const BatchInst* d_insts, const uint2* d_items, const int* qoff,
                             int* counters, int grid, hipStream_t s) {
  if constexpr (TRIPLE)
    batched_fwd_triple_kernel<T, WF, IDX64><<<grid, 256, 0, s>>>(d_insts, d_items, qoff,
                                                                 counters);
  else
    batched_fwd_kernel<T, WF, IDX64><<<grid, 256, 0, s>>>(d_insts, d_items, qoff, counters);
}

// class = ((dtype * 2 + weight) * 2 + idx64) * 2 + triple (batch_class)
#define GJP_BATCH_CLASSES_RPL(X, R, o)                                                      \
  X(o + 0, float, W_LINEAR, false, R) X(o + 2, float, W_LINEAR, true, R)                    \
  X(o + 4, float, W_SPLINE, false, R) X(o + 6, float, W_SPLINE, true, R)                    \
  X(o + 8, bf16_t, W_LINEAR, false, R) X(o + 10, bf16_t, W_LINEAR, true, R)                 \
  X(o + 12, bf16_t, W_SPLINE, false, R) X(o + 14, bf16_t, W_SPLINE, true, R)                \
  X(o + 16, f16_t, W_LINEAR, false, R) X(o + 18, f16_t, W_LINEAR, true, R)                  \
  X(o + 20, f16_t, W_SPLINE, false, R) X(o + 22, f16_t, W_SPLINE, true, R)
#define GJP_BATCH_CLASSES(X) GJP_BATCH_CLASSES_RPL(X, false, 0) GJP_BATCH_CLASSES_RPL(X, true, 1)

int batched_grid_size(int cls) {
  switch (cls) {
#define GJP_CASE(k, T, W, I, R) \
  case k:                       \
    return batched_grid_t<T, W, I, R>();
    GJP_BATCH_CLASSES(GJP_CASE)
#undef GJP_CASE
    default:
      return 1024;
  }
}

int launch_batched_forward(const BatchInst* d_insts, const uint2* d_items, const int* d_qoff,
                           int* d_counters, int grid, int cls, hipStream_t s) {
  switch (cls) {
#define GJP_CASE(k, T, W, I, R)                                                 \
  case k:                                                                       \
    launch_batched_t<T, W, I, R>(d_insts, d_items, d_qoff, d_counters, grid, s); \
    break;
    GJP_BATCH_CLASSES(GJP_CASE)
#undef GJP_CASE
    default:
      return set_error(-4, "batched: unknown instance class");
  }
  return check_launch("batched forward kernel");
}

}  // namespace gjp
