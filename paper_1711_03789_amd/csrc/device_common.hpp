// Device-side helpers shared by the gfx950 kernels: complex arithmetic, matrix-core tile
// products, wavefront reductions, publication of block results and bounded waits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mx {

constexpr int kTile = 64;          // block-skyline tile edge
constexpr int kTileElems = kTile * kTile;
constexpr long kSpinLimit = 1L << 21;  // bounded waits: ~1-2 s before reporting MX_ESTALL

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a += b * c
template <typename T>
__device__ __forceinline__ void cfma(cx<T> &a, cx<T> b, cx<T> c) {
  a.re += b.re * c.re - b.im * c.im;
  a.im += b.re * c.im + b.im * c.re;
}
template <typename T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
template <typename T>
__device__ __forceinline__ cx<T> cinv(cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return {b.re / d, -b.im / d};
}
template <typename To, typename Ti>
__device__ __forceinline__ cx<To> ccast(cx<Ti> a) { return {(To)a.re, (To)a.im}; }

template <typename T>
__device__ __forceinline__ cx<T> shfl_xor_c(cx<T> v, int m) {
  return {__shfl_xor(v.re, m), __shfl_xor(v.im, m)};
}

// ---- matrix cores --------------------------------------------------------------------------------
// 16x16x4 products: lane l supplies A[l%16][l/16] and B[l/16][l%16].  Accumulator value r of lane
// l holds D[row][l%16] with row = 4*(l/16) + r for the FP32 instruction and row = 4*r + l/16 for
// the FP64 one (checked at run time by mx_selftest).
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Complex tile product on one wavefront: a 32x32 quadrant (rows r0.., cols c0..) of
//     P[i][j] = sum_k A[i][k] * s[k] * B[j][k]        (A, B row-major 64x64 tiles)
// with complex products split into four real matrix-core products.  Each lane loads four
// consecutive k of a row at once; the k order inside a 16-wide slab is permuted identically for
// A and B, which leaves the sum unchanged.
//   SCALE:   multiply B's column k by s[k] (the LDL^T diagonal D)
//   UNITDIAG: B is a unit-lower tile stored with something else on its diagonal: read 1 there
//             and 0 above it.
template <typename T, bool SCALE, bool UNITDIAG>
__device__ __forceinline__ void tile_nt_quadrant(const cx<T> *__restrict__ A,
                                                 const cx<T> *__restrict__ B,
                                                 const cx<T> *__restrict__ s, int r0, int c0,
                                                 typename Mfma<T>::acc_t acc[2][2][2]) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][b][c] = acc_t{0, 0, 0, 0};
  for (int kk = 0; kk < kTile; kk += 16) {
    const int kb = kk + 4 * lk;  // this lane's 4 consecutive k
    cx<T> av[2][4], bv[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const cx<T> *p = A + (r0 + rb * 16 + li) * kTile + kb;
#pragma unroll
      for (int e = 0; e < 4; ++e) av[rb][e] = p[e];
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int j = c0 + cb * 16 + li;
      const cx<T> *p = B + j * kTile + kb;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cx<T> v = p[e];
        if (UNITDIAG) {
          // v m + d with m = [k < j], d = [k == j], in arithmetic rather than a branch: a branch
          // lets the compiler skip the load per lane and wait for every load on its own (the
          // entries are finite: D on the diagonal, zeros above it)
          const int k = kb + e;
          const T m = k < j ? (T)1 : (T)0, d = k == j ? (T)1 : (T)0;
          v = {v.re * m + d, v.im * m};
        }
        if (SCALE) v = cmul(v, s[kb + e]);
        bv[cb][e] = v;
      }
    }
    // two passes over the eight accumulators per k group, so that consecutive matrix-core
    // instructions never depend on each other (a dependent one waits for the previous result)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc[rb][cb][0] = Mfma<T>::op(av[rb][e].re, bv[cb][e].re, acc[rb][cb][0]);
          acc[rb][cb][1] = Mfma<T>::op(av[rb][e].re, bv[cb][e].im, acc[rb][cb][1]);
        }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc[rb][cb][0] = Mfma<T>::op(-av[rb][e].im, bv[cb][e].im, acc[rb][cb][0]);
          acc[rb][cb][1] = Mfma<T>::op(av[rb][e].im, bv[cb][e].re, acc[rb][cb][1]);
        }
    }
  }
}

// Row/column of accumulator element (rb, cb, r) of this lane inside the 64x64 tile.
template <typename T>
__device__ __forceinline__ int acc_row(int r0, int rb, int r);
template <>
__device__ __forceinline__ int acc_row<float>(int r0, int rb, int r) {
  return r0 + rb * 16 + 4 * ((threadIdx.x & 63) >> 4) + r;
}
template <>
__device__ __forceinline__ int acc_row<double>(int r0, int rb, int r) {
  return r0 + rb * 16 + 4 * r + ((threadIdx.x & 63) >> 4);
}
__device__ __forceinline__ int acc_col(int c0, int cb) { return c0 + cb * 16 + (threadIdx.x & 15); }

// ---- agent-scope flags, publication and bounded waits ---------------------------------------------
__device__ __forceinline__ int load_flag(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_flag(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Cross-workgroup publication of small results (one 64-entry block) without cache-wide fences:
// the producer writes with device-coherent atomic stores; the consumer reads with device-coherent
// atomic loads, which cannot hit a stale line in a non-coherent cache, and knows a value is
// published when it no longer holds the sentinel (below).  Whole-cache writeback / invalidate
// fences at agent scope would cost more than the data moved (measured: they halve the streaming
// bandwidth of the sweeps).
template <typename T>
__device__ __forceinline__ void pub_store(cx<T> *p, cx<T> v) {
  __hip_atomic_store(&p->re, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->im, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ cx<T> pub_load(const cx<T> *p) {
  return {__hip_atomic_load(&p->re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
          __hip_atomic_load(&p->im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}
// Sentinel marking a not-yet-written result value: a NaN bit pattern that no computed value has
// (it is a signalling NaN, and arithmetic only ever produces quiet ones).  A result vector is
// filled with it before each sweep, and a consumer polls the values it needs until none is the
// sentinel: the data is its own completion flag, so the producer neither waits for its stores to
// be acknowledged nor stores a flag after them, and no ordering between a flag and the data has to
// hold.  Each half of a complex value is written by one 4- or 8-byte store, so a value is complete
// when neither half is the sentinel.
__device__ __forceinline__ bool is_sentinel(double v) {
  return __double_as_longlong(v) == (long long)0x7FF75EA700000001ull;
}
__device__ __forceinline__ bool is_sentinel(float v) { return __float_as_uint(v) == 0x7FB5EA71u; }
template <typename T>
__device__ __forceinline__ cx<T> sentinel();
template <>
__device__ __forceinline__ cx<double> sentinel<double>() {
  const double s = __longlong_as_double((long long)0x7FF75EA700000001ull);
  return {s, s};
}
template <>
__device__ __forceinline__ cx<float> sentinel<float>() {
  const float s = __uint_as_float(0x7FB5EA71u);
  return {s, s};
}

// Loads this wave's values at p, waiting (bounded) until no lane sees the sentinel in either half;
// returns false (and raises *abort) after kSpinLimit polls or when another workgroup has raised it.
// While waiting only lane 0 polls (its own value), so a waiting wave costs one 16-byte load per
// poll instead of a whole block: a block is written by one store instruction of one wave, so the
// rest of it lands right after lane 0's value.
template <typename T>
__device__ inline bool wait_values(const cx<T> *p, cx<T> &v, int *abort) {
  v = pub_load(p);
  if (__all(!is_sentinel(v.re) && !is_sentinel(v.im))) return true;
  const bool lead = (threadIdx.x & 63) == 0;
  for (long it = 0; it < kSpinLimit; ++it) {
    __builtin_amdgcn_s_sleep(1);
    int seen = 0;
    if (lead) {
      const cx<T> u = pub_load(p);
      seen = !is_sentinel(u.re) && !is_sentinel(u.im);
    }
    if (__builtin_amdgcn_readfirstlane(seen)) {
      v = pub_load(p);
      if (__all(!is_sentinel(v.re) && !is_sentinel(v.im))) return true;
    }
    if ((it & 63) == 0 && load_flag(abort)) return false;
  }
  store_flag(abort, 1);
  return false;
}

}  // namespace mx
