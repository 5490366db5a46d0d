// One-level Schwarz preconditioner on gfx950: batched block-skyline LDL^T factorisation of all
// local problems (matrix-core trailing updates) and the application
//     z = sum_l R_l^T D_l (A^l)^-1 R_l v            (eq:defAS without the coarse term; RAS_1 and
//                                                     ImpRAS_1 of Sec. 6.3 with Boolean D_l)
// as restrict-gather -> persistent forward/backward block sweeps -> owner gather (or sum).
//
// Storage: each local matrix is reordered by reverse Cuthill-McKee and stored as 64x64 tiles of
// its lower triangle, block row I holding tiles J = bfirst(I)..I (bfirst monotone, so the fill of
// a pivot-free factorisation stays inside).  After factorisation a tile (I,J), J < I, holds L_IJ;
// the diagonal tile holds inv(L_II) strictly below its diagonal and D_I on it.
//
// The local matrices are complex symmetric (A = A^T, Sec. 2.2), so A^l = L D L^T with no
// conjugation; no pivoting is needed for xi != 0 because every principal submatrix of
// Theta A^l has positive definite imaginary part (coercivity lemma of Sec. 2.3).
#include <type_traits>
#include <utility>
#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "device_common.hpp"
#include "objects.hpp"

namespace mx {

// ---- tile addressing ---------------------------------------------------------------------------
// After the factorisation a tile keeps only its rows that meet the envelope (row i of block row I
// is kept in tile (I, J) iff first_i < 64 (J + 1); diagonal tiles keep all rows), packed as
// consecutive 64-entry rows from pack[base]; the kept row with index r inside the tile is the
// popcount(mask & (2^r - 1))-th one.
struct TileMeta {
  int64_t base;
  uint64_t mask;
};

__device__ __forceinline__ int rank_below(uint64_t mask, int r) {
  return __popcll(mask & ((1ull << r) - 1));
}

struct SubView {
  const int32_t *nb, *brow_base;
  const int64_t *tile_base, *vec_base;
  const int64_t *brow_off;
  const int32_t *bfirst, *blast;
  // trimmed tiles read by the sweeps (see TileMeta): rmeta in tile order, cmeta by block column
  // (tile (I, B) of a subdomain at cmeta[cptr[brow_base + B] + I - B] for B <= I <= blast(B))
  const TileMeta *rmeta, *cmeta;
  const int64_t *cptr;
  int64_t tile_shift;  // factorisation: first tile of the group held in the tile pool
};

template <typename T>
__device__ __forceinline__ cx<T> *tile_ptr(cx<T> *pool, const SubView &v, int l, int I, int J) {
  const int bb = v.brow_base[l];
  const int64_t t = v.tile_base[l] - v.tile_shift + v.brow_off[bb + I] + (J - v.bfirst[bb + I]);
  return pool + t * (int64_t)kTileElems;
}

__device__ __forceinline__ int find_sub(const int32_t *pref, int nsub, int g) {
  int lo = 0, hi = nsub;  // pref[lo] <= g < pref[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pref[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- setup kernels ------------------------------------------------------------------------------
template <typename T>
__global__ void k_scatter(int64_t n, const int64_t *__restrict__ off,
                          const cx<double> *__restrict__ val, int64_t shift, cx<T> *__restrict__ pool) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pool[off[i] - shift] = ccast<T>(val[i]);
}

__global__ void k_zero(int64_t n16, uint4 *__restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

// ---- factorisation: diagonal tile ----------------------------------------------------------------
// One workgroup of four waves per subdomain.  Thread (w, c) keeps column c of rows i = 4q + w
// (q = 0..15) of two 64x64 matrices in registers: S, the symmetric tile being reduced, and X,
// which starts as the identity.  Pivot j is eliminated right-looking: the wave holding row j
// publishes, through LDS, row j of S, the same row divided by the pivot d_j (column j of L, by
// symmetry) and row j of X; after one barrier every thread updates its rows i > j,
//   S_i -= L_ij S_j,   X_i -= L_ij X_j,
// i.e. Gauss elimination applied to [A | I], which ends with X = inv(L).  The published rows are
// double-buffered, so a step costs one barrier.  Written back as X below the diagonal, D on it,
// 0 above.
// Pivots 4Q .. 4Q+3 (held in register Q of waves 0..3).  Q is a template argument so that every
// register index is static and the arrays stay in registers.
template <typename T, int Q>
__device__ __forceinline__ void diag_pivots(cx<T> (&s)[16], cx<T> (&x)[16], cx<T> (*R)[3][kTile], int w,
                                            int c, bool &bad) {
#pragma unroll 1
  for (int p = 0; p < 4; ++p) {
    const int j = 4 * Q + p;
    cx<T>(*B)[kTile] = R[j & 1];
    if (w == p) {
      cx<T> d = {__shfl(s[Q].re, j), __shfl(s[Q].im, j)};
      const T mag = d.re * d.re + d.im * d.im;
      if (!(mag > (T)0) || !isfinite(mag)) {
        bad = true;
        d = {(T)1, (T)0};
      }
      B[0][c] = s[Q];
      B[1][c] = cmul(s[Q], cinv(d));
      B[2][c] = x[Q];
    }
    __syncthreads();
    const cx<T> sj = B[0][c], xj = B[2][c];
#pragma unroll
    for (int r = Q; r < 16; ++r) {
      if (r == Q && w <= p) continue;  // only rows 4r + w > j
      const cx<T> lij = B[1][4 * r + w];
      s[r] = csub(s[r], cmul(lij, sj));
      x[r] = csub(x[r], cmul(lij, xj));
    }
  }
}
template <typename T, int... Q>
__device__ __forceinline__ void diag_all_pivots(cx<T> (&s)[16], cx<T> (&x)[16], cx<T> (*R)[3][kTile], int w,
                                                int c, bool &bad, std::integer_sequence<int, Q...>) {
  (diag_pivots<T, Q>(s, x, R, w, c, bad), ...);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fac_diag(int K, int l0, SubView v, cx<T> *pool, int *ctrl) {
  const int l = l0 + blockIdx.x;
  if (K >= v.nb[l]) return;
  __shared__ cx<T> S[kTile][kTile + 1];  // the symmetric input, staged once
  __shared__ cx<T> R[2][3][kTile];       // published row j: S_j, S_j / d_j, X_j
  cx<T> *tile = tile_ptr(pool, v, l, K, K);
  const int tid = threadIdx.x, c = tid & 63, w = tid >> 6;
  for (int i = w; i < kTile; i += 4)
    if (c <= i) {
      const cx<T> a = tile[i * kTile + c];
      S[i][c] = a;
      S[c][i] = a;
    }
  __syncthreads();
  cx<T> s[16], x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    s[q] = S[4 * q + w][c];
    x[q] = {(T)(4 * q + w == c ? 1 : 0), (T)0};
  }
  bool bad = false;
  diag_all_pivots<T>(s, x, R, w, c, bad, std::make_integer_sequence<int, 16>());
  if (bad) atomicOr(&ctrl[3], 1);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = 4 * q + w;
    tile[i * kTile + c] = c < i ? x[q] : c == i ? s[q] : cx<T>{(T)0, (T)0};
  }
}

// ---- factorisation: panel L_IK = A_IK inv(L_KK)^T D_K^-1 -------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fac_panel(int K, int g0, SubView v, const int32_t *pref, int nsub,
                                                   cx<T> *pool) {
  const int g = g0 + blockIdx.x;
  const int l = find_sub(pref, nsub, g);
  const int I = K + 1 + (g - pref[l]);
  cx<T> *A = tile_ptr(pool, v, l, I, K);
  const cx<T> *X = tile_ptr(pool, v, l, K, K);
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  typename Mfma<T>::acc_t acc[2][2][2];
  tile_nt_quadrant<T, false, true>(A, X, nullptr, r0, c0, acc);
  __syncthreads();  // every wave has read all of A before any writes
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int col = acc_col(c0, cb);
    const cx<T> dinv = cinv(X[col * kTile + col]);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = acc_row<T>(r0, rb, r);
        A[row * kTile + col] = cmul(cx<T>{acc[rb][cb][0][r], acc[rb][cb][1][r]}, dinv);
      }
  }
}

// ---- factorisation: trailing update A_IJ -= L_IK D_K L_JK^T ---------------------------------------
// Split in two launches so that the next diagonal tile and panel can start early (look-ahead):
//   NEXT = true:  the tiles of block column K+1, (I, K+1) for K+1 <= I <= blast(K)  (pref: m per
//                 subdomain, m = blast(K) - K);
//   NEXT = false: all other tiles, (I, J) with K+2 <= J <= I <= blast(K)  (pref: m(m-1)/2).
// Staged complex tile product for the trailing update, one 32x32 quadrant per wave:
//     acc[i][j] = sum_k A[i][k] * d[k] * B[j][k]      (A, B row-major 64x64 tiles)
// The workgroup copies 16-wide k slabs of A and of d-scaled B into LDS (double-buffered, rows
// padded by one entry so the 16 rows read by one instruction fall in different banks) while the
// waves run the matrix-core products of the previous slab, so every tile entry is read from L2
// once per workgroup instead of once per wave.
template <typename T>
struct UpdateStage {
  cx<T> a[2][kTile][17];
  cx<T> b[2][kTile][17];
};

// Waves per trailing-update workgroup: each wave owns 32 rows x (128 / kUpdWaves) columns of the
// 64x64 tile, so two 70 KB workgroups per CU keep 16 waves resident to hide LDS and L2 latency.
constexpr int kUpdWaves = 8;
constexpr int kUpdCB = 8 / kUpdWaves;  // 16-column blocks per wave

// Operands of one trailing-update tile: up to kMaxWidth source block columns q, each a pair of
// tiles (A[q] = L_IK, B[q] = L_JK) and the pivots d[q] = D_K in LDS; 4 16-wide k slabs per source.
// The slab loop is unrolled, so every index into these arrays is a constant.
constexpr int kMaxWidth = 4;
// block columns per look-ahead trailing update unless asked (measured best at 64^3: 4 for
// complex128, 3 for complex64, whose cheaper matrix-core products leave less to hide the main
// stream's longer critical path behind)
constexpr int kDefaultWidthC128 = 4, kDefaultWidthC64 = 3;
template <typename T>
struct UpdSources {
  const cx<T> *A[kMaxWidth], *B[kMaxWidth], *d[kMaxWidth];
  int n;  // sources in use
};

// acc = sum over the sources of A diag(d) B^T for this wave's 32 x (16 kUpdCB) part of the tile.
// The 16-wide k slabs of A and B (B already scaled by d) are staged through LDS, double-buffered:
// slab s+1 is loaded into registers while slab s feeds the matrix cores, across the boundaries
// between sources too.  SLABS = 4 per source column.
template <typename T, int SLABS>
__device__ __forceinline__ void update_product(const UpdSources<T> src, UpdateStage<T> &st, int r0, int c0,
                                               typename Mfma<T>::acc_t acc[2][kUpdCB][2]) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int kPer = 1024 / (64 * kUpdWaves);  // staged entries per thread and operand
  const int tid = threadIdx.x, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int lrow = tid / (16 / kPer), lq = (tid % (16 / kPer)) * kPer;  // staging: row, first k
  static_assert(SLABS % 4 == 0 && SLABS / 4 <= kMaxWidth, "whole source columns");
  constexpr int ns = SLABS;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < kUpdCB; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][b][c] = acc_t{0, 0, 0, 0};
  cx<T> ra[kPer], rb[kPer];
  auto fetch = [&](int slab) {
    const int q = slab >> 2, kk = (slab & 3) * 16;
    const cx<T> *A = src.A[q], *B = src.B[q], *d = src.d[q];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      ra[e] = A[lrow * kTile + kk + lq + e];
      rb[e] = cmul(B[lrow * kTile + kk + lq + e], d[kk + lq + e]);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      st.a[buf][lrow][lq + e] = ra[e];
      st.b[buf][lrow][lq + e] = rb[e];
    }
  };
  // one slab: feed buffer BUF to the matrix cores while slab s+1 is loaded into the other buffer
  auto step = [&](int s, auto bufc) {
    constexpr int buf = decltype(bufc)::value;
    if (s + 1 < ns) fetch(s + 1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cx<T> av[2], bv[kUpdCB];
#pragma unroll
      for (int q = 0; q < 2; ++q) av[q] = st.a[buf][r0 + q * 16 + li][4 * lk + e];
#pragma unroll
      for (int p = 0; p < kUpdCB; ++p) bv[p] = st.b[buf][c0 + p * 16 + li][4 * lk + e];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < kUpdCB; ++p) {
          acc[q][p][0] = Mfma<T>::op(av[q].re, bv[p].re, acc[q][p][0]);
          acc[q][p][1] = Mfma<T>::op(av[q].re, bv[p].im, acc[q][p][1]);
        }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < kUpdCB; ++p) {
          acc[q][p][0] = Mfma<T>::op(-av[q].im, bv[p].im, acc[q][p][0]);
          acc[q][p][1] = Mfma<T>::op(av[q].im, bv[p].re, acc[q][p][1]);
        }
    }
    if (s + 1 < ns) stash(buf ^ 1);
    __syncthreads();
  };
  fetch(0);
  stash(0);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < ns; s += 2) {
    step(s, std::integral_constant<int, 0>());
    step(s + 1, std::integral_constant<int, 1>());
  }
}

// C -= the sources' product for one 64x64 tile (one workgroup).
template <typename T, int SLABS>
__device__ __forceinline__ void update_tile(const UpdSources<T> src, UpdateStage<T> &stage, cx<T> *C) {
  const int w = threadIdx.x >> 6;
  constexpr int kColWaves = kUpdWaves / 2;
  const int r0 = (w / kColWaves) * 32, c0 = (w % kColWaves) * (16 * kUpdCB);
  typename Mfma<T>::acc_t acc[2][kUpdCB][2];
  if constexpr (SLABS > 0) update_product<T, SLABS>(src, stage, r0, c0, acc);
  else if (src.n == 4) update_product<T, 16>(src, stage, r0, c0, acc);
  else if (src.n == 3) update_product<T, 12>(src, stage, r0, c0, acc);
  else if (src.n == 2) update_product<T, 8>(src, stage, r0, c0, acc);
  else update_product<T, 4>(src, stage, r0, c0, acc);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < kUpdCB; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = acc_row<T>(r0, rb, q), col = acc_col(c0, cb);
        cx<T> cur = C[row * kTile + col];
        C[row * kTile + col] = {cur.re - acc[rb][cb][0][q], cur.im - acc[rb][cb][1][q]};
      }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Remapping the
// block index gives every XCD a contiguous range of tiles, so consecutive tiles (same block row I,
// hence the same L_IK, and neighbouring L_JK) meet in one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  constexpr int kXcd = 8;
  const int per = n / kXcd, rem = n % kXcd, x = b % kXcd, q = b / kXcd;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + q;
}

template <typename T, bool NEXT>
__global__ __launch_bounds__(64 * kUpdWaves) void k_fac_update(int K, int g0, SubView v, const int32_t *pref,
                                                    int nsub, cx<T> *pool) {
  const int g = g0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int l = find_sub(pref, nsub, g);
  const int t = g - pref[l];
  int I, J;
  if (NEXT) {
    I = K + 1 + t;
    J = K + 1;
  } else {
    int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    I = K + 2 + r;
    J = K + 2 + (t - r * (r + 1) / 2);
  }
  __shared__ cx<T> dk[kTile];
  __shared__ UpdateStage<T> stage;
  const cx<T> *Xk = tile_ptr(pool, v, l, K, K);
  if (threadIdx.x < kTile) dk[threadIdx.x] = Xk[threadIdx.x * kTile + threadIdx.x];
  __syncthreads();
  UpdSources<T> src;
  src.A[0] = tile_ptr(pool, v, l, I, K);
  src.B[0] = tile_ptr(pool, v, l, J, K);
  src.d[0] = dk;
  src.n = 1;
  update_tile<T, 4>(src, stage, tile_ptr(pool, v, l, I, J));
}

// Trailing updates from a group of W <= kMaxWidth factored block columns G .. G+W-1 at once:
//   A_IJ -= sum over the group's columns S with I <= blast(S) of L_IS D_S L_JS^T
// in one pass over A_IJ, so each tile is read and written once per group instead of once per
// column (blast is nondecreasing, so the columns present for row I are the group's last ones).
//   UpdIntra: block column Kc of the group (G < Kc < G+W) from the group's columns before it.
//   UpdNext:  the next group's columns G+W .. G+2W-1, rows up to b = blast(G+W-1).
//   UpdRest:  tiles G+2W <= J <= I <= b.
enum UpdMode { UpdIntra, UpdNext, UpdRest };
template <typename T, int MODE>
__global__ __launch_bounds__(64 * kUpdWaves) void k_fac_update_group(int G, int W, int Kc, int g0, SubView v,
                                                          const int32_t *pref, int nsub, cx<T> *pool) {
  const int g = g0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int l = find_sub(pref, nsub, g);
  int t = g - pref[l];
  const int bb = v.brow_base[l];
  const int send = MODE == UpdIntra ? Kc : min(G + W, v.nb[l]);  // sources G .. send-1
  const int b = v.blast[bb + send - 1];
  int I, J;
  if (MODE == UpdIntra) {
    I = Kc + t;
    J = Kc;
  } else if (MODE == UpdNext) {
    J = G + W;
    while (t >= b - J + 1) {  // column J holds rows J .. b
      t -= b - J + 1;
      ++J;
    }
    I = J + t;
  } else {
    int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    I = G + 2 * W + r;
    J = G + 2 * W + (t - r * (r + 1) / 2);
  }
  int s0 = G;  // first source column that reaches row I
  while (v.blast[bb + s0] < I) ++s0;
  const int n = send - s0;
  __shared__ cx<T> dk[kMaxWidth][kTile];
  __shared__ UpdateStage<T> stage;
  for (int x = threadIdx.x; x < n * kTile; x += blockDim.x) {
    const int q = x >> 6, i = x & 63;
    dk[q][i] = tile_ptr(pool, v, l, s0 + q, s0 + q)[i * kTile + i];
  }
  __syncthreads();
  UpdSources<T> src;
#pragma unroll
  for (int q = 0; q < kMaxWidth; ++q) {
    const int S = s0 + min(q, n - 1);
    src.A[q] = tile_ptr(pool, v, l, I, S);
    src.B[q] = tile_ptr(pool, v, l, J, S);
    src.d[q] = dk[min(q, n - 1)];
  }
  src.n = n;
  update_tile<T, 0>(src, stage, tile_ptr(pool, v, l, I, J));
}

// ---- application: restrict, persistent sweeps, prolong ---------------------------------------------
template <typename T>
__global__ void k_restrict(int64_t n, const int32_t *__restrict__ glob,
                           const cx<double> *__restrict__ vin, cx<T> *__restrict__ r,
                           cx<T> *__restrict__ y, cx<T> *__restrict__ z, int *ctrl) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    ctrl[1] = 0;  // ticket counters of the forward and backward sweeps
    ctrl[4] = 0;
  }
  if (p < n) {
    int32_t g = glob[p];
    r[p] = g >= 0 ? ccast<T>(vin[g]) : cx<T>{0, 0};
    y[p] = sentinel<T>();  // results of the two sweeps: not yet written
    z[p] = sentinel<T>();
  }
}

template <typename T>
__global__ void k_prolong_owner(int64_t E, const int64_t *__restrict__ src,
                                const cx<T> *__restrict__ z, cx<double> *__restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) {
    const int64_t q = src[e];
    out[e] = q >= 0 ? ccast<double>(z[q]) : cx<double>{0, 0};
  }
}

template <typename T>
__global__ void k_prolong_sum(int64_t E, const int64_t *__restrict__ ptr,
                              const int64_t *__restrict__ idx, const cx<T> *__restrict__ z,
                              cx<double> *__restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  cx<double> s = {0, 0};
  for (int64_t q = ptr[e]; q < ptr[e + 1]; ++q) s = cadd(s, ccast<double>(z[idx[q]]));
  out[e] = s;
}

// Reduce 8 per-lane complex partial sums (one per row r of this wave's 8 rows) across the 64
// lanes; afterwards lanes with (lane & 7) == 0 hold the total of row (lane >> 3).  Each halving
// step exchanges the half of the rows the partner keeps (compile-time indices throughout, so the
// partial sums stay in registers).
template <typename T, int O, int CNT>
__device__ __forceinline__ void butterfly_step(cx<T> acc[8]) {
  constexpr int half = CNT / 2;
  const bool upper = ((threadIdx.x & 63) & O) != 0;
#pragma unroll
  for (int q = 0; q < half; ++q) {
    cx<T> send = upper ? acc[q] : acc[q + half];
    cx<T> keep = upper ? acc[q + half] : acc[q];
    acc[q] = cadd(keep, shfl_xor_c(send, O));
  }
}
template <typename T>
__device__ __forceinline__ cx<T> butterfly8(cx<T> acc[8]) {
  butterfly_step<T, 32, 8>(acc);
  butterfly_step<T, 16, 4>(acc);
  butterfly_step<T, 8, 2>(acc);
  acc[0] = cadd(acc[0], shfl_xor_c(acc[0], 4));
  acc[0] = cadd(acc[0], shfl_xor_c(acc[0], 2));
  acc[0] = cadd(acc[0], shfl_xor_c(acc[0], 1));
  return acc[0];
}

constexpr int kSweepWaves = 8;              // 512-thread workgroups, 8 tile rows per wave
constexpr int kSweepThreads = 64 * kSweepWaves;
constexpr int kRows = kTile / kSweepWaves;  // = 8
// The sweeps run one workgroup per CU (a second co-resident workgroup delays the dependency
// chain of the first more than it adds bandwidth), so both precisions get the full register
// budget of two waves per SIMD.
template <typename T>
struct SweepMinWaves {
  static constexpr int value = 2;
};

// Block sweeps of all subdomains in one persistent launch per direction.  Work items
// (subdomain, block row) are handed out by an atomic ticket in an order in which every item
// comes after all items it depends on (a subdomain's rows ascending for the forward sweep,
// descending for the backward one), so a workgroup only ever waits for tickets already taken by
// running workgroups.  A block row is complete when its results no longer hold the sentinel the
// result vectors are filled with before the sweep; all waits are bounded.
//   forward  (FWD): y_I = inv(L_II) (r_I - sum_{J<I} L_IJ y_J)
//   backward      : z_J = inv(L_JJ)^T (y_J / D_J - sum_{I>J} L_IJ^T z_I)
// Tiles are read row by row with the lanes along a tile row (coalesced) in both directions, up to
// four tiles per wave in flight.  The two tiles needed right after the last dependency (the
// neighbour tile and the diagonal tile) are staged in LDS when the item starts, so the dependency
// chain itself carries no tile loads.  Results of a block are written by wave 0 only, with
// device-coherent stores; readers load them with device-coherent loads and check them.
// Streaming helpers over the trimmed tiles.  A wave owns 8 consecutive rows of a tile; a row
// missing from a tile contributes zero and is not read.
// The factor is read once per sweep: nontemporal loads keep it from displacing reusable lines
// (measured: 7.0 TB/s instead of 6.3 TB/s for this access pattern).
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T> *p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void wave_rows(const cx<T> *__restrict__ pack, TileMeta m, int row0,
                                          cx<T> a[kRows]) {
  const int lane = threadIdx.x & 63;
  const uint32_t mb = (uint32_t)(m.mask >> row0) & 0xFFu;
  const int k0 = rank_below(m.mask, row0);
  const cx<T> *tp = pack + m.base + lane;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int k = k0 + __popc(mb & ((1u << r) - 1u));
    a[r] = (mb >> r) & 1u ? load_stream(tp + (int64_t)k * kTile) : cx<T>{0, 0};
  }
}

// A batch of NT tiles per wave in flight.  The block results it multiplies are validated by their
// values: a result still holding the sentinel is not published yet, and the wave waits (bounded)
// for it.  Returns false after an expired wait or an abort.
template <typename T>
__device__ __forceinline__ bool published(cx<T> v) {
  return !is_sentinel(v.re) && !is_sentinel(v.im);
}

template <typename T, int NT>
__device__ __forceinline__ bool stream_fwd(const cx<T> *__restrict__ pack, const TileMeta *rm, int J,
                                           int row0, const cx<T> *yp, cx<T> acc[kRows], int *abort) {
  // tiles (B, J..J+NT-1) of this wave's rows; rm[J] = meta of tile (B, J); yp = y of block J
  cx<T> a[NT][kRows], y[NT];
  bool ready = true;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    y[t] = pub_load(yp + t * kTile);
    ready = ready && published(y[t]);
    wave_rows(pack, rm[J + t], row0, a[t]);
  }
  if (!__all(ready)) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (!__all(published(y[t])) && !wait_values(yp + t * kTile, y[t], abort)) return false;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < kRows; ++r) cfma(acc[r], a[t][r], y[t]);
  return true;
}

template <typename T>
__device__ __forceinline__ cx<T> bcast(cx<T> v, int src) {
  return {__shfl(v.re, src), __shfl(v.im, src)};
}

template <typename T, int NT>
__device__ __forceinline__ bool stream_bwd(const cx<T> *__restrict__ pack, const TileMeta *cm,
                                           int64_t vb, int I, int row0, const cx<T> *zvec,
                                           cx<T> &acc, int *abort) {
  // tiles (I, B), (I-1, B), ...; cm[I] = meta of tile (I, B); the wave needs z of its 8 rows
  const int lane = threadIdx.x & 63;
  cx<T> a[NT][kRows], z[NT];
  bool ready = true;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    z[t] = pub_load(zvec + vb + (int64_t)(I - t) * kTile + row0 + (lane & (kRows - 1)));
    ready = ready && published(z[t]);
    wave_rows(pack, cm[I - t], row0, a[t]);
  }
  if (!__all(ready)) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (!__all(published(z[t])) &&
          !wait_values(zvec + vb + (int64_t)(I - t) * kTile + row0 + (lane & (kRows - 1)), z[t], abort))
        return false;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < kRows; ++r) cfma(acc, a[t][r], bcast(z[t], r));
  return true;
}

// complex64 streaming with 16-byte lanes: lane (h, c) = (lane / 32, lane % 32) loads entries 2c
// and 2c+1 of one tile row, so one load instruction covers two rows (1 KiB, like complex128)
// instead of one (512 bytes).  Instruction i of a wave reads rows row0 + 2i + h.
typedef float f4 __attribute__((ext_vector_type(4)));  // (re, im) of entries 2c and 2c+1

__device__ __forceinline__ f4 load_stream4(const cx<float> *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
}

__device__ __forceinline__ void wave_rows_wide(const cx<float> *__restrict__ pack, TileMeta m, int row0,
                                               f4 a[kRows / 2]) {
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const uint32_t mb = (uint32_t)(m.mask >> row0) & 0xFFu;
  const int k0 = rank_below(m.mask, row0);
  const cx<float> *tp = pack + m.base + 2 * c;
#pragma unroll
  for (int i = 0; i < kRows / 2; ++i) {
    const int r = 2 * i + h;
    const int k = k0 + __popc(mb & ((1u << r) - 1u));
    a[i] = (mb >> r) & 1u ? load_stream4(tp + (int64_t)k * kTile) : f4{0.f, 0.f, 0.f, 0.f};
  }
}

// acc[i] += row (row0 + 2i + h) of tiles (B, J..J+NT-1), restricted to entries 2c, 2c+1, times y;
// yb = y of block J.
template <int NT>
__device__ __forceinline__ bool stream_fwd_wide(const cx<float> *__restrict__ pack, const TileMeta *rm, int J,
                                                int row0, const cx<float> *yb, cx<float> acc[kRows / 2],
                                                int *abort) {
  const int c = threadIdx.x & 31;
  f4 a[NT][kRows / 2];
  cx<float> y0[NT], y1[NT];
  bool ready = true;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    y0[t] = pub_load(yb + t * kTile + 2 * c);
    y1[t] = pub_load(yb + t * kTile + 2 * c + 1);
    ready = ready && published(y0[t]) && published(y1[t]);
    wave_rows_wide(pack, rm[J + t], row0, a[t]);
  }
  if (!__all(ready)) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (!__all(published(y0[t])) && !wait_values(yb + t * kTile + 2 * c, y0[t], abort)) return false;
      if (!__all(published(y1[t])) && !wait_values(yb + t * kTile + 2 * c + 1, y1[t], abort)) return false;
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < kRows / 2; ++i) {
      cfma(acc[i], cx<float>{a[t][i].x, a[t][i].y}, y0[t]);
      cfma(acc[i], cx<float>{a[t][i].z, a[t][i].w}, y1[t]);
    }
  return true;
}

// acc0/acc1 (entries 2c, 2c+1 of block B) += sum over this wave's rows r of tiles (I-t, B) of
// L[r][.] z_I[r]; the wave's 8 values of z_I are loaded once and broadcast.
template <int NT>
__device__ __forceinline__ bool stream_bwd_wide(const cx<float> *__restrict__ pack, const TileMeta *cm,
                                                int64_t vb, int I, int row0, const cx<float> *zvec,
                                                cx<float> &acc0, cx<float> &acc1, int *abort) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
  f4 a[NT][kRows / 2];
  cx<float> z[NT];
  bool ready = true;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    z[t] = pub_load(zvec + vb + (int64_t)(I - t) * kTile + row0 + (lane & (kRows - 1)));
    ready = ready && published(z[t]);
    wave_rows_wide(pack, cm[I - t], row0, a[t]);
  }
  if (!__all(ready)) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (!__all(published(z[t])) &&
          !wait_values(zvec + vb + (int64_t)(I - t) * kTile + row0 + (lane & (kRows - 1)), z[t], abort))
        return false;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < kRows / 2; ++i) {
      const cx<float> zr = bcast(z[t], 2 * i + h);
      cfma(acc0, cx<float>{a[t][i].x, a[t][i].y}, zr);
      cfma(acc1, cx<float>{a[t][i].z, a[t][i].w}, zr);
    }
  return true;
}

// One sweep of several preconditioners in one launch (serving several requests at once): each
// preconditioner's items keep their own order, and the jobs follow one another in the ticket
// order, so an item still comes after every item it depends on.  A job is a preconditioner's
// view of its factors, ticket orders and local vectors; batch launches find an item's job from
// the prefix of item counts (slot[j] = the job's entry in the device array of jobs).
template <typename T>
struct SweepJob {
  SubView v;
  const cx<T> *pack;
  const int32_t *sub_f, *blk_f, *sub_b, *blk_b;  // forward and backward ticket orders
  int n_half;                                      // items per direction
  cx<T> *r, *y, *z;
  int *ctrl;                                       // the preconditioner's control block
};
constexpr int kMaxBatch = 16;
struct BatchIndex {
  int njobs;
  int slot[kMaxBatch];
  int prefix[kMaxBatch + 1];
};

template <typename T, bool FWD, bool BATCH>
__global__ __launch_bounds__(kSweepThreads, SweepMinWaves<T>::value) void k_sweep(
    SubView v0, const cx<T> *__restrict__ pack0, const int32_t *__restrict__ sched_sub0,
    const int32_t *__restrict__ sched_blk0, int n_items, const cx<T> *__restrict__ rvec0,
    cx<T> *yvec0, cx<T> *zvec0, int *ctrl, const SweepJob<T> *__restrict__ jobs, BatchIndex bidx) {
  __shared__ int s_item;
  __shared__ int s_dead;
  __shared__ cx<T> sL[kTile][kTile];  // neighbour tile of the last dependency
  __shared__ cx<T> sX[kTile][kTile];  // diagonal tile (inverse unit-lower factor, D on the diagonal)
  __shared__ cx<T> s_vec[kTile];
  __shared__ cx<T> s_out[kTile];
  __shared__ cx<T> s_red[kSweepWaves][kTile];
  // the wave index is uniform: keeping it scalar keeps the tile metadata in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = w * kRows;  // this wave's first row inside a block
  // tiles per wave in flight (eight for complex float measured slower than four)
  constexpr int kBatch = 4;
  int *abort = &ctrl[2];
  int *ticket = &ctrl[FWD ? 1 : 4];
  while (true) {
    if (tid == 0) {
      int t = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_item = load_flag(abort) ? n_items : t;
      s_dead = 0;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= n_items) break;
    SubView v = v0;
    const cx<T> *__restrict__ pack = pack0;
    const int32_t *sched_sub = sched_sub0, *sched_blk = sched_blk0;
    const cx<T> *__restrict__ rvec = rvec0;
    cx<T> *yvec = yvec0, *zvec = zvec0;
    int li = item;
    if constexpr (BATCH) {  // the job holding this item (uniform across the workgroup)
      int j = 0;
      while (j + 1 < bidx.njobs && bidx.prefix[j + 1] <= item) ++j;
      const SweepJob<T> &jb = jobs[bidx.slot[j]];
      v = jb.v;
      pack = jb.pack;
      sched_sub = FWD ? jb.sub_f : jb.sub_b;
      sched_blk = FWD ? jb.blk_f : jb.blk_b;
      rvec = jb.r;
      yvec = jb.y;
      zvec = jb.z;
      li = item - bidx.prefix[j];
    }
    const int l = sched_sub[li], B = sched_blk[li];
    const int bb = v.brow_base[l];
    const int64_t vb = v.vec_base[l];
    // Every wave streams its own 8 rows and checks the block results it multiplies by itself, so
    // waves only meet at the final reductions.
    bool dead = false;
    if (FWD) {
      const int f = v.bfirst[bb + B];
      const bool has_prev = B - 1 >= f;
      const TileMeta *rm = v.rmeta + (v.tile_base[l] + v.brow_off[bb + B] - f);  // rm[J]: (B, J)
      {  // stage this wave's rows of the diagonal tile and of tile (B, B-1)
        cx<T> x[kRows], p[kRows];
        wave_rows(pack, rm[B], row0, x);
        if (has_prev) wave_rows(pack, rm[B - 1], row0, p);
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          sX[row0 + r][lane] = lane <= row0 + r ? x[r] : cx<T>{0, 0};
          sL[row0 + r][lane] = has_prev ? p[r] : cx<T>{0, 0};
        }
      }
      cx<T> acc[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) acc[r] = {0, 0};
      const cx<T> rB = rvec[vb + (int64_t)B * kTile + lane];
      int J = f;
      if constexpr (sizeof(T) == 4) {
        cx<float> accw[kRows / 2];
#pragma unroll
        for (int i = 0; i < kRows / 2; ++i) accw[i] = {0, 0};
        for (; !dead && J + kBatch - 1 < B - 1; J += kBatch)
          dead = !stream_fwd_wide<kBatch>(pack, rm, J, row0, yvec + vb + (int64_t)J * kTile, accw, abort);
        for (; !dead && J < B - 1; ++J)
          dead = !stream_fwd_wide<1>(pack, rm, J, row0, yvec + vb + (int64_t)J * kTile, accw, abort);
        // fold into the one-entry-per-lane layout: row row0 + 2i + h lives in half h
        const bool upper = lane >= 32;
#pragma unroll
        for (int i = 0; i < kRows / 2; ++i) {
          acc[2 * i] = upper ? acc[2 * i] : cadd(acc[2 * i], accw[i]);
          acc[2 * i + 1] = upper ? cadd(acc[2 * i + 1], accw[i]) : acc[2 * i + 1];
        }
      } else {
        for (; !dead && J + kBatch - 1 < B - 1; J += kBatch)
          dead = !stream_fwd<T, kBatch>(pack, rm, J, row0, yvec + vb + (int64_t)J * kTile + lane, acc, abort);
        for (; !dead && J < B - 1; ++J)
          dead = !stream_fwd<T, 1>(pack, rm, J, row0, yvec + vb + (int64_t)J * kTile + lane, acc, abort);
      }
      if (has_prev && !dead) {
        // the last dependency: its tile is staged in LDS already
        cx<T> y0;
        if (!wait_values(yvec + vb + (int64_t)(B - 1) * kTile + lane, y0, abort)) {
          dead = true;
        } else {
#pragma unroll
          for (int r = 0; r < kRows; ++r) cfma(acc[r], sL[row0 + r][lane], y0);
        }
      }
      if (dead && lane == 0) s_dead = 1;
      cx<T> s = butterfly8(acc);
      if ((lane & 7) == 0) s_vec[row0 + (lane >> 3)] = s;
      __syncthreads();
      // t = r_B - s;  y_B = inv(L_BB) t  (unit lower: y_i = t_i + sum_{m<i} X[i][m] t_m)
      const cx<T> tm = csub(rB, s_vec[lane]);
#pragma unroll
      for (int r = 0; r < kRows; ++r)
        acc[r] = lane < row0 + r ? cmul(sX[row0 + r][lane], tm) : cx<T>{0, 0};
      s = butterfly8(acc);
      if ((lane & 7) == 0) s_out[row0 + (lane >> 3)] = s;
      __syncthreads();
      if (w == 0 && !s_dead) {
        pub_store(yvec + vb + (int64_t)B * kTile + lane, cadd(tm, s_out[lane]));
      }
    } else {
      const int last = v.blast[bb + B];
      const bool has_next = B + 1 <= last;
      const TileMeta *cm = v.cmeta + (v.cptr[bb + B] - B);  // cm[I]: tile (I, B)
      const TileMeta md = cm[B];
      {  // stage this wave's rows of the diagonal tile and of tile (B+1, B)
        cx<T> x[kRows], p[kRows];
        wave_rows(pack, md, row0, x);
        if (has_next) wave_rows(pack, cm[B + 1], row0, p);
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          sX[row0 + r][lane] = lane <= row0 + r ? x[r] : cx<T>{0, 0};
          sL[row0 + r][lane] = has_next ? p[r] : cx<T>{0, 0};
        }
      }
      const int64_t pd = vb + (int64_t)B * kTile + lane;
      const cx<T> dB = pack[md.base + (int64_t)lane * kTile + lane];  // diagonal tiles keep all rows
      const cx<T> yB = yvec[pd];
      cx<T> acc = {0, 0};
      // rows far below B finish first: consume I = last, last-1, ..., B+2 as they become ready
      int I = last;
      if constexpr (sizeof(T) == 4) {
        cx<float> a0 = {0, 0}, a1 = {0, 0};
        for (; !dead && I - (kBatch - 1) > B + 1; I -= kBatch)
          dead = !stream_bwd_wide<kBatch>(pack, cm, vb, I, row0, zvec, a0, a1, abort);
        for (; !dead && I > B + 1; --I) dead = !stream_bwd_wide<1>(pack, cm, vb, I, row0, zvec, a0, a1, abort);
        // both halves hold partial sums for entries 2c, 2c+1: add them, then move entry j to lane j
        a0 = cadd(a0, shfl_xor_c(a0, 32));
        a1 = cadd(a1, shfl_xor_c(a1, 32));
        const cx<float> e0 = bcast(a0, lane >> 1), e1 = bcast(a1, lane >> 1);
        acc = cadd(acc, (lane & 1) ? e1 : e0);
      } else {
        for (; !dead && I - (kBatch - 1) > B + 1; I -= kBatch)
          dead = !stream_bwd<T, kBatch>(pack, cm, vb, I, row0, zvec, acc, abort);
        for (; !dead && I > B + 1; --I) dead = !stream_bwd<T, 1>(pack, cm, vb, I, row0, zvec, acc, abort);
      }
      if (has_next && !dead) {
        cx<T> zv;  // the last dependency, read directly (sentinel polling)
        if (!wait_values(zvec + vb + (int64_t)(B + 1) * kTile + row0 + (lane & (kRows - 1)), zv, abort)) {
          dead = true;
        } else {
#pragma unroll
          for (int r = 0; r < kRows; ++r) cfma(acc, sL[row0 + r][lane], bcast(zv, r));
        }
      }
      if (dead && lane == 0) s_dead = 1;
      s_red[w][lane] = acc;
      __syncthreads();
      if (w == 0) {
        cx<T> t = s_red[0][lane];
#pragma unroll
        for (int q = 1; q < kSweepWaves; ++q) t = cadd(t, s_red[q][lane]);
        s_vec[lane] = csub(cdiv(yB, dB), t);
      }
      __syncthreads();
      // z_B = inv(L_BB)^T s:  z_j = s_j + sum_{i>j} X[i][j] s_i
      acc = {0, 0};
#pragma unroll
      for (int r = 0; r < kRows; ++r)
        if (row0 + r > lane) cfma(acc, sX[row0 + r][lane], s_vec[row0 + r]);
      s_red[w][lane] = acc;
      __syncthreads();
      if (w == 0 && !s_dead) {
        cx<T> t = s_red[0][lane];
#pragma unroll
        for (int q = 1; q < kSweepWaves; ++q) t = cadd(t, s_red[q][lane]);
        pub_store(zvec + vb + (int64_t)B * kTile + lane, cadd(s_vec[lane], t));
      }
    }
  }
}

// Copies the kept rows of every factored tile into the trimmed layout: one workgroup per tile,
// each wave 16 rows, lanes along the row.
template <typename T>
__global__ __launch_bounds__(256) void k_pack(int64_t ntiles, const TileMeta *__restrict__ rmeta,
                                              const cx<T> *__restrict__ pool, cx<T> *__restrict__ pack) {
  const int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  const TileMeta m = rmeta[t];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const cx<T> *src = pool + t * (int64_t)kTileElems + lane;
  cx<T> *dst = pack + m.base + lane;
  for (int r = w * 16; r < w * 16 + 16; ++r)
    if ((m.mask >> r) & 1ull) dst[(int64_t)rank_below(m.mask, r) * kTile] = src[r * kTile];
}

// ---- host side ------------------------------------------------------------------------------------
static SubView view_of(const mx_precond *P) {
  SubView v;
  v.nb = P->d_sub_nb.as<int32_t>();
  v.brow_base = P->d_sub_brow_base.as<int32_t>();
  v.tile_base = P->d_sub_tile_base.as<int64_t>();
  v.vec_base = P->d_sub_vec_base.as<int64_t>();
  v.brow_off = P->d_brow_off.as<int64_t>();
  v.bfirst = P->d_bfirst.as<int32_t>();
  v.blast = P->d_blast.as<int32_t>();
  v.rmeta = P->d_rmeta.as<TileMeta>();
  v.cmeta = P->d_cmeta.as<TileMeta>();
  v.cptr = P->d_cptr.as<int64_t>();
  v.tile_shift = 0;
  return v;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Right-looking blocked LDL^T over the subdomains [l0, l1) at once (their tiles are in `pool`,
// starting with tile v.tile_shift), block column after block column.  Either on one stream, or
// with look-ahead on two: the main stream carries the chain that gates the next block columns
// (their updates, diagonal tiles and panels) while the aux stream applies the bulk of each
// trailing update, from groups of P->width block columns at a time.
template <typename T>
static void factor_group(mx_precond *P, hipStream_t st, int l0, int l1, SubView v, cx<T> *pool) {
  const int N = P->nsub;
  int nb = 0;
  for (int l = l0; l < l1; ++l) nb = std::max(nb, P->sub_nb[l]);
  auto range = [&](const std::vector<int32_t> &pref, int K, int &g0) {
    g0 = pref[(int64_t)K * (N + 1) + l0];
    return pref[(int64_t)K * (N + 1) + l1] - g0;
  };
  const int32_t *dpp = P->d_panel_pref.as<int32_t>(), *dup = P->d_update_pref.as<int32_t>();
  int64_t total_updates = 0;
  for (int K = 0; K < nb; ++K) {
    int g;
    total_updates += range(P->update_pref, K, g) + range(P->panel_pref, K, g);
  }
  int sched = P->schedule;
  if (sched == MX_FACTOR_AUTO) sched = total_updates < 2048LL * std::max(1, nb) ? MX_FACTOR_ONE_STREAM : MX_FACTOR_LOOKAHEAD;
  if (sched == MX_FACTOR_ONE_STREAM) {
    // small steps (a few tiles per CU): launch latency dominates and the second stream's event
    // traffic costs more than the overlap gains; one stream, four launches per step
    for (int K = 0; K < nb; ++K) {
      int gp, gu;
      const int np = range(P->panel_pref, K, gp), nu = range(P->update_pref, K, gu);
      const int32_t *pp = dpp + (int64_t)K * (N + 1), *up = dup + (int64_t)K * (N + 1);
      k_fac_diag<T><<<l1 - l0, 256, 0, st>>>(K, l0, v, pool, P->d_ctrl.as<int>());
      if (np > 0) k_fac_panel<T><<<np, 256, 0, st>>>(K, gp, v, pp, N, pool);
      if (np > 0) k_fac_update<T, true><<<np, 64 * kUpdWaves, 0, st>>>(K, gp, v, pp, N, pool);
      if (nu > 0) k_fac_update<T, false><<<nu, 64 * kUpdWaves, 0, st>>>(K, gu, v, up, N, pool);
    }
    MX_HIP(hipGetLastError());
    return;
  }
  // Look-ahead on two streams.  The main stream carries the critical path (the next block
  // columns' updates, diagonal tiles and panels); the aux stream applies the rest of each trailing
  // update as soon as the panels it reads are done.  An aux update must finish before the main
  // stream updates the columns it also touches (event ev_rest, waited on before it is recorded
  // again).
  hipStream_t sx;
  hipEvent_t ev_panel, ev_rest;
  MX_HIP(hipStreamCreateWithFlags(&sx, hipStreamNonBlocking));
  MX_HIP(hipEventCreateWithFlags(&ev_panel, hipEventDisableTiming));
  MX_HIP(hipEventCreateWithFlags(&ev_rest, hipEventDisableTiming));
  auto diag_panel = [&](int K) {
    k_fac_diag<T><<<l1 - l0, 256, 0, st>>>(K, l0, v, pool, P->d_ctrl.as<int>());
    int gp;
    const int np = range(P->panel_pref, K, gp);
    if (np > 0) k_fac_panel<T><<<np, 256, 0, st>>>(K, gp, v, dpp + (int64_t)K * (N + 1), N, pool);
  };
  auto next_column = [&](int K) {  // block column K+1 from column K (main stream)
    int gp;
    const int np = range(P->panel_pref, K, gp);
    if (np > 0) k_fac_update<T, true><<<np, 64 * kUpdWaves, 0, st>>>(K, gp, v, dpp + (int64_t)K * (N + 1), N, pool);
  };
  auto aux_after_panels = [&]() {
    MX_HIP(hipEventRecord(ev_panel, st));
    MX_HIP(hipStreamWaitEvent(sx, ev_panel, 0));
  };
  MX_HIP(hipEventRecord(ev_rest, sx));  // nothing pending on the aux stream yet
  diag_panel(0);
  if (P->width == 1) {
    for (int K = 0; K < nb; ++K) {
      int gu;
      const int nu = range(P->update_pref, K, gu);
      // aux: tiles (I, J), J >= K+2, once panel K is done (and, in stream order, step K-1's rest)
      aux_after_panels();
      if (nu > 0) k_fac_update<T, false><<<nu, 64 * kUpdWaves, 0, sx>>>(K, gu, v, dup + (int64_t)K * (N + 1), N, pool);
      // main: block column K+1 needs step K-1's rest (recorded before this step's rest is queued)
      MX_HIP(hipStreamWaitEvent(st, ev_rest, 0));
      next_column(K);
      MX_HIP(hipEventRecord(ev_rest, sx));
      if (K + 1 < nb) diag_panel(K + 1);
    }
  } else {
    // W block columns per trailing update: each pass over a tile applies a whole group of W
    // columns, so the bulk update reads and writes every tile W times less often.  At the start
    // of group G the columns G .. G+W-1 hold every update from the columns before G, and column
    // G is factored.
    const int W = P->width;
    const int32_t *dip = P->d_intra_pref.as<int32_t>(), *dnp = P->d_next_pref.as<int32_t>();
    const int32_t *drp = P->d_rest_pref.as<int32_t>();
    for (int G = 0; G < nb; G += W) {
      for (int Kc = G + 1; Kc < std::min(G + W, nb); ++Kc) {  // the group's own columns, in turn
        int gi;
        const int ni = range(P->intra_pref, Kc, gi);
        if (ni > 0)
          k_fac_update_group<T, UpdIntra><<<ni, 64 * kUpdWaves, 0, st>>>(G, W, Kc, gi, v, dip + (int64_t)Kc * (N + 1), N, pool);
        diag_panel(Kc);
      }
      int gn, gr;
      const int nn = range(P->next_pref, G, gn), nr = range(P->rest_pref, G, gr);
      // aux: tiles G+2W <= J <= I from the whole group, after its panels (and the previous rest)
      aux_after_panels();
      // main: the next group's columns overlap the previous group's rest, so wait for it first
      MX_HIP(hipStreamWaitEvent(st, ev_rest, 0));
      if (nr > 0)
        k_fac_update_group<T, UpdRest><<<nr, 64 * kUpdWaves, 0, sx>>>(G, W, 0, gr, v, drp + (int64_t)G * (N + 1), N, pool);
      MX_HIP(hipEventRecord(ev_rest, sx));
      if (nn > 0)
        k_fac_update_group<T, UpdNext><<<nn, 64 * kUpdWaves, 0, st>>>(G, W, 0, gn, v, dnp + (int64_t)G * (N + 1), N, pool);
      if (G + W < nb) diag_panel(G + W);
    }
  }
  MX_HIP(hipStreamWaitEvent(st, ev_rest, 0));
  MX_HIP(hipGetLastError());
  (void)hipEventDestroy(ev_panel);
  (void)hipEventDestroy(ev_rest);
  (void)hipStreamDestroy(sx);
}

template <typename T>
static void apply_t(mx_precond *P, const void *vin, void *zout, hipStream_t st) {
  SubView v = view_of(P);
  const int64_t n = P->vec_total;
  k_restrict<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      n, P->d_glob.as<int32_t>(), (const cx<double> *)vin, P->d_r.as<cx<T>>(), P->d_y.as<cx<T>>(),
      P->d_z.as<cx<T>>(), P->d_ctrl.as<int>());
  if (P->timing) {
    if (P->n_timed == P->ev_start.size()) {
      hipEvent_t a, b, c;
      MX_HIP(hipEventCreate(&a));
      MX_HIP(hipEventCreate(&b));
      MX_HIP(hipEventCreate(&c));
      P->ev_start.push_back(a);
      P->ev_mid.push_back(b);
      P->ev_stop.push_back(c);
    }
    MX_HIP(hipEventRecord(P->ev_start[P->n_timed], st));
  }
  const int half = P->n_items / 2;
  k_sweep<T, true, false><<<P->trsv_grid, kSweepThreads, 0, st>>>(
      v, P->pack.as<cx<T>>(), P->d_sched_sub.as<int32_t>(), P->d_sched_blk.as<int32_t>(), half,
      P->d_r.as<cx<T>>(), P->d_y.as<cx<T>>(), P->d_z.as<cx<T>>(), P->d_ctrl.as<int>(), nullptr,
      BatchIndex{});
  if (P->timing) MX_HIP(hipEventRecord(P->ev_mid[P->n_timed], st));
  k_sweep<T, false, false><<<P->trsv_grid, kSweepThreads, 0, st>>>(
      v, P->pack.as<cx<T>>(), P->d_sched_sub.as<int32_t>() + half,
      P->d_sched_blk.as<int32_t>() + half, half, P->d_r.as<cx<T>>(), P->d_y.as<cx<T>>(),
      P->d_z.as<cx<T>>(), P->d_ctrl.as<int>(), nullptr, BatchIndex{});
  if (P->timing) MX_HIP(hipEventRecord(P->ev_stop[P->n_timed++], st));
  const int64_t E = P->E;
  if (P->kind == MX_AS)
    k_prolong_sum<T><<<(unsigned)((E + 255) / 256), 256, 0, st>>>(
        E, P->d_sum_ptr.as<int64_t>(), P->d_sum_idx.as<int64_t>(), P->d_z.as<cx<T>>(),
        (cx<double> *)zout);
  else
    k_prolong_owner<T><<<(unsigned)((E + 255) / 256), 256, 0, st>>>(
        E, P->d_src.as<int64_t>(), P->d_z.as<cx<T>>(), (cx<double> *)zout);
  MX_HIP(hipGetLastError());
}

// ---- batched applications of several preconditioners (serving) ------------------------------------
template <typename T>
static SweepJob<T> job_of(mx_precond *P) {
  SweepJob<T> j{};
  j.v = view_of(P);
  j.pack = P->pack.as<cx<T>>();
  const int half = P->n_items / 2;
  j.sub_f = P->d_sched_sub.as<int32_t>();
  j.blk_f = P->d_sched_blk.as<int32_t>();
  j.sub_b = j.sub_f + half;
  j.blk_b = j.blk_f + half;
  j.n_half = half;
  j.r = P->d_r.as<cx<T>>();
  j.y = P->d_y.as<cx<T>>();
  j.z = P->d_z.as<cx<T>>();
  j.ctrl = P->d_ctrl.as<int>();
  return j;
}

static_assert(sizeof(SweepJob<double>) == sizeof(SweepJob<float>), "one job layout for both precisions");
size_t batch_job_bytes() { return sizeof(SweepJob<double>); }

void batch_job_write(mx_precond *P, void *jobs, int slot) {
  if (P->plan) fail(MX_EINVAL, "preconditioner is planned but not materialised");
  const size_t b = batch_job_bytes();
  if (P->prec == MX_C128) {
    SweepJob<double> j = job_of<double>(P);
    MX_HIP(hipMemcpy((char *)jobs + (size_t)slot * b, &j, sizeof(j), hipMemcpyHostToDevice));
  } else {
    SweepJob<float> j = job_of<float>(P);
    MX_HIP(hipMemcpy((char *)jobs + (size_t)slot * b, &j, sizeof(j), hipMemcpyHostToDevice));
  }
}

// ticket counters and abort word of a batch launch to zero
__global__ void k_batch_reset(int *ctrl) {
  if (threadIdx.x < 8) ctrl[threadIdx.x] = 0;
}
// an expired wait in a batch is reported by every preconditioner of the batch
template <typename T>
__global__ void k_batch_finish(const int *ctrl, const SweepJob<T> *jobs, BatchIndex bi) {
  const int j = threadIdx.x;
  if (j < bi.njobs && ctrl[2]) jobs[bi.slot[j]].ctrl[2] = 1;
}

template <typename T>
static void batch_apply_t(int njobs, const int *slots, mx_precond *const *Ps, const void *const *vin,
                          void *const *zout, const void *jobs_dev, int *bctrl, int grid_cap,
                          hipStream_t st) {
  BatchIndex bi{};
  bi.njobs = njobs;
  bi.prefix[0] = 0;
  for (int j = 0; j < njobs; ++j) {
    bi.slot[j] = slots[j];
    bi.prefix[j + 1] = bi.prefix[j] + Ps[j]->n_items / 2;
  }
  const int total = bi.prefix[njobs];
  const SweepJob<T> *jobs = (const SweepJob<T> *)jobs_dev;
  for (int j = 0; j < njobs; ++j) {
    mx_precond *P = Ps[j];
    const int64_t n = P->vec_total;
    k_restrict<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        n, P->d_glob.as<int32_t>(), (const cx<double> *)vin[j], P->d_r.as<cx<T>>(),
        P->d_y.as<cx<T>>(), P->d_z.as<cx<T>>(), P->d_ctrl.as<int>());
  }
  k_batch_reset<<<1, 64, 0, st>>>(bctrl);
  const int grid = std::max(1, std::min(total, grid_cap));
  k_sweep<T, true, true><<<grid, kSweepThreads, 0, st>>>(SubView{}, nullptr, nullptr, nullptr, total, nullptr,
                                                         nullptr, nullptr, bctrl, jobs, bi);
  k_sweep<T, false, true><<<grid, kSweepThreads, 0, st>>>(SubView{}, nullptr, nullptr, nullptr, total, nullptr,
                                                          nullptr, nullptr, bctrl, jobs, bi);
  k_batch_finish<T><<<1, 64, 0, st>>>(bctrl, jobs, bi);
  for (int j = 0; j < njobs; ++j) {
    mx_precond *P = Ps[j];
    const int64_t E = P->E;
    if (P->kind == MX_AS)
      k_prolong_sum<T><<<(unsigned)((E + 255) / 256), 256, 0, st>>>(
          E, P->d_sum_ptr.as<int64_t>(), P->d_sum_idx.as<int64_t>(), P->d_z.as<cx<T>>(),
          (cx<double> *)zout[j]);
    else
      k_prolong_owner<T><<<(unsigned)((E + 255) / 256), 256, 0, st>>>(
          E, P->d_src.as<int64_t>(), P->d_z.as<cx<T>>(), (cx<double> *)zout[j]);
  }
  MX_HIP(hipGetLastError());
}

// z_j = B_j^-1 v_j for up to kMaxBatch one-level preconditioners of one precision: their
// restrictions, one forward and one backward sweep launch over all of them, their prolongations.
// Their sweep jobs must have been written to jobs_dev[slots[j]] (batch_job_write); bctrl is a
// control block of 8 ints owned by the caller.  Each result equals that of precond_apply_level1.
void batch_apply(int njobs, const int *slots, mx_precond *const *Ps, const void *const *vin,
                 void *const *zout, const void *jobs_dev, int *bctrl, int grid_cap, hipStream_t st) {
  if (njobs < 1 || njobs > kMaxBatch) fail(MX_EINVAL, "batch of 1 .. 16 applications");
  const int prec = Ps[0]->prec;
  for (int j = 0; j < njobs; ++j)
    if (Ps[j]->prec != prec || Ps[j]->coarse) fail(MX_EINVAL, "batched applications need one-level preconditioners of one precision");
  if (prec == MX_C128) batch_apply_t<double>(njobs, slots, Ps, vin, zout, jobs_dev, bctrl, grid_cap, st);
  else batch_apply_t<float>(njobs, slots, Ps, vin, zout, jobs_dev, bctrl, grid_cap, st);
}

void precond_apply_level1(mx_precond *P, const void *vin, void *zout, hipStream_t st) {
  if (P->apply_hook) {  // applications routed elsewhere (a server's batcher)
    P->apply_hook(P->apply_hook_arg, P, vin, zout, st);
    return;
  }
  precond_apply_direct(P, vin, zout, st);
}

void precond_apply_direct(mx_precond *P, const void *vin, void *zout, hipStream_t st) {
  if (P->prec == MX_C128) apply_t<double>(P, vin, zout, st);
  else apply_t<float>(P, vin, zout, st);
}

template <typename T>
__global__ void k_gather_diag(SubView v, int l, int64_t n, const cx<T> *__restrict__ pack,
                              cx<double> *__restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int I = (int)(i / kTile), r = (int)(i % kTile), bb = v.brow_base[l];
  const int64_t t = v.tile_base[l] + v.brow_off[bb + I] + (I - v.bfirst[bb + I]);
  d[i] = ccast<double>(pack[v.rmeta[t].base + (int64_t)r * kTile + r]);  // diagonal tiles keep all rows
}

void precond_export_diag(const mx_precond *P, int l, double *d) {
  const int64_t n = P->sky[l].n;
  if (n == 0) return;
  DevBuf out;
  out.alloc((size_t)n * 16);
  const unsigned g = (unsigned)((n + 255) / 256);
  if (P->prec == MX_C128)
    k_gather_diag<double><<<g, 256>>>(view_of(P), l, n, P->pack.as<cx<double>>(), out.as<cx<double>>());
  else
    k_gather_diag<float><<<g, 256>>>(view_of(P), l, n, P->pack.as<cx<float>>(), out.as<cx<double>>());
  MX_HIP(hipGetLastError());
  MX_HIP(hipMemcpy(d, out.p, (size_t)n * 16, hipMemcpyDeviceToHost));
}

void precond_timing(mx_precond *P, int enable, int64_t *launches, double *ms_fwd, double *ms_bwd) {
  if (enable) {
    P->timing = true;
    P->n_timed = 0;
    return;
  }
  double tf = 0, tb = 0;
  for (size_t i = 0; i < P->n_timed; ++i) {
    MX_HIP(hipEventSynchronize(P->ev_stop[i]));
    float a = 0, b = 0;
    MX_HIP(hipEventElapsedTime(&a, P->ev_start[i], P->ev_mid[i]));
    MX_HIP(hipEventElapsedTime(&b, P->ev_mid[i], P->ev_stop[i]));
    tf += a;
    tb += b;
  }
  if (launches) *launches = (int64_t)P->n_timed;
  if (ms_fwd) *ms_fwd = tf;
  if (ms_bwd) *ms_bwd = tb;
  P->timing = false;
  P->n_timed = 0;
}

void precond_autotune(mx_ctx *ctx, mx_precond *P, hipStream_t st, int32_t *best_grid, double *best_ms) {
  DevBuf vin, zout;
  vin.alloc((size_t)P->E * 16);
  zout.alloc((size_t)P->E * 16);
  MX_HIP(hipMemsetAsync(vin.p, 0, (size_t)P->E * 16, st));
  const int cus = ctx->cus;
  std::vector<int> cand = {cus / 4, cus / 2, (3 * cus) / 4, cus};
  const int saved = P->trsv_grid;
  hipEvent_t a, b;
  MX_HIP(hipEventCreate(&a));
  MX_HIP(hipEventCreate(&b));
  int best = saved;
  double best_t = 1e300;
  for (int g : cand) {
    if (g < 1) continue;
    P->trsv_grid = std::min(g, std::max(1, P->n_items / 2));
    precond_apply_level1(P, vin.p, zout.p, st);  // warm-up
    MX_HIP(hipEventRecord(a, st));
    for (int r = 0; r < 3; ++r) precond_apply_level1(P, vin.p, zout.p, st);
    MX_HIP(hipEventRecord(b, st));
    MX_HIP(hipEventSynchronize(b));
    float ms = 0;
    MX_HIP(hipEventElapsedTime(&ms, a, b));
    if (ms / 3 < best_t) best_t = ms / 3, best = P->trsv_grid;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  P->trsv_grid = best;
  precond_check(P);
  if (best_grid) *best_grid = best;
  if (best_ms) *best_ms = best_t;
}

// Factorisation tuner: sets up the preconditioner described by opts once per candidate
// schedule (one stream; look-ahead with 1 .. 4 block columns per trailing-update pass) and keeps
// the one whose factorisation took least time.  Every candidate computes the same factors up to
// rounding; only the launch shapes differ.
void precond_tune_factor(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *mh, const mx_partition *ph,
                         const mx_precond_opts *opts, hipStream_t st, int32_t *best_schedule,
                         int32_t *best_width, double *best_ms, double *ms_each) {
  struct Cand {
    int sched, width;
  };
  const Cand cand[5] = {{MX_FACTOR_ONE_STREAM, 1}, {MX_FACTOR_LOOKAHEAD, 1}, {MX_FACTOR_LOOKAHEAD, 2},
                        {MX_FACTOR_LOOKAHEAD, 3}, {MX_FACTOR_LOOKAHEAD, 4}};
  double best = 1e300;
  int bs = cand[0].sched, bw = cand[0].width;
  for (int c = 0; c < 5; ++c) {
    mx_precond_opts o = *opts;
    o.factor_schedule = cand[c].sched;
    o.factor_width = cand[c].width;
    double ms;
    {
      mx_precond T;
      PrecondPlan plan;
      precond_plan(ctx, A, mh, ph, &o, &T, plan);
      set_sweep_grid(&T, ctx->cus);
      precond_materialize(&T, plan, st);
      ms = T.info.t_factor * 1e3;
    }  // its device memory goes back to the block cache before the next candidate
    if (ms_each) ms_each[c] = ms;
    if (ms < best) best = ms, bs = cand[c].sched, bw = cand[c].width;
  }
  if (best_schedule) *best_schedule = bs;
  if (best_width) *best_width = bw;
  if (best_ms) *best_ms = best;
}

int precond_check(mx_precond *P, hipStream_t st) {
  int h[4];
  MX_HIP(hipMemcpyAsync(h, P->d_ctrl.p, sizeof(h), hipMemcpyDeviceToHost, st));
  MX_HIP(hipStreamSynchronize(st));
  if (h[3]) P->failed = MX_EPIVOT;
  else if (h[2]) P->failed = MX_ESTALL;
  precond_refuse_failed(P);
  return MX_OK;
}

void precond_refuse_failed(const mx_precond *P) {
  if (P->failed == MX_EPIVOT) fail(MX_EPIVOT, "zero or non-finite pivot in a local factorisation");
  if (P->failed == MX_ESTALL)
    fail(MX_ESTALL, "a device-side wait in the block sweeps expired; the preconditioner is unusable");
}

void precond_setup(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *mh, const mx_partition *ph,
                   const mx_precond_opts *opts, mx_precond *P, hipStream_t st) {
  PrecondPlan plan;
  precond_plan(ctx, A, mh, ph, opts, P, plan);
  precond_materialize(P, plan, st);
}

void set_sweep_grid(mx_precond *P, int cus) {
  const int grid = P->sweep_grid > 0 ? P->sweep_grid : cus;
  P->trsv_grid = std::max(1, std::min(P->n_items / 2, grid));
}

void precond_plan(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *mh, const mx_partition *ph,
                  const mx_precond_opts *opts, mx_precond *P, PrecondPlan &plan) {
  const Mesh &m = mh->m;
  const Partition &part = ph->p;
  if (opts->kind < MX_AS || opts->kind > MX_ORAS) fail(MX_EINVAL, "unknown preconditioner kind");
  if (A->order != 1 && A->order != 2) fail(MX_EINVAL, "unknown element order");
  const Order2 *o2 = A->order == 2 ? &mh->order2() : nullptr;
  const int64_t ndof = o2 ? o2->N : m.ne;
  if (A->h.n != ndof) fail(MX_EINVAL, "matrix and mesh disagree");
  if (opts->precision != MX_C128 && opts->precision != MX_C64) fail(MX_EINVAL, "unknown precision");
  const double t0 = now_s();
  P->kind = opts->kind;
  P->prec = opts->precision;
  P->k = A->k;
  P->xi_prec = opts->kind == MX_ORAS ? opts->xi_prec : A->xi;
  P->bc = A->bc;
  P->E = ndof;
  P->order = A->order;
  P->device = ctx ? ctx->device : -1;
  int s0 = opts->sub_begin, s1 = opts->sub_end;
  if (s0 == 0 && s1 == 0) s1 = part.nsub;
  if (s0 < 0 || s1 > part.nsub || s0 >= s1) fail(MX_EINVAL, "subdomain share out of range");
  if (opts->pool_limit < 0) fail(MX_EINVAL, "pool_limit must be >= 0");
  P->pool_limit = opts->pool_limit;
  if (opts->factor_schedule < 0 || opts->factor_schedule > MX_FACTOR_LOOKAHEAD)
    fail(MX_EINVAL, "unknown factor_schedule");
  if (opts->factor_width < 0 || opts->factor_width > kMaxWidth)
    fail(MX_EINVAL, "factor_width must be 0 .. 4");
  P->schedule = opts->factor_schedule;
  P->width = opts->factor_width > 0 ? opts->factor_width
                                    : P->prec == MX_C128 ? kDefaultWidthC128 : kDefaultWidthC64;
  P->sub_begin = s0;
  P->nsub = s1 - s0;
  P->share = s0 != 0 || s1 != part.nsub;
  const int N = P->nsub;
  // subdomain j of this preconditioner is subdomain s0 + j of the partition
  // local DOF sets and owners: the partition's edge sets, or those of the order-2 space
  std::vector<std::vector<int32_t>> sets2;
  std::vector<int32_t> owner2;
  if (o2) order2_sets(m, *o2, part, opts->kind, sets2, owner2);
  const auto &all_sets = o2 ? sets2 : part.set(opts->kind);
  const std::vector<int32_t> &owner = o2 ? owner2 : part.owner;
  const uint8_t *boundary = o2 ? o2->dof_boundary.data() : m.edge_on_boundary.data();
  std::vector<std::vector<int32_t>> sets_share(all_sets.begin() + s0, all_sets.begin() + s1);
  const auto &sets = sets_share;
  // local matrices and their orderings
  std::vector<LocalCSR> loc(N);
  P->sky.assign(N, Skyline());
  KuhnElements ke;
  kuhn_elements(m.lx / m.nx, m.ly / m.ny, m.lz / m.nz, ke);
  parallel_items(N, [&](auto next) {
    std::vector<int32_t> g2l(ndof, -1), tstamp;
    if (opts->kind == MX_ORAS) tstamp.assign(m.nt, -1);
    for (int64_t l; (l = next()) >= 0;) {
      if (opts->kind == MX_ORAS && o2)
        local_impedance2(m, *o2, A->k, opts->xi_prec, A->bc, part.tets[s0 + l], sets[l], loc[l], g2l, tstamp);
      else if (opts->kind == MX_ORAS)
        local_impedance(m, ke, A->k, opts->xi_prec, A->bc, part.tets[s0 + l], sets[l], loc[l], g2l, tstamp);
      else
        local_minor(boundary, A->h, A->bc, sets[l], loc[l], g2l);
      build_skyline(loc[l], P->sky[l]);
    }
  });
  // layout
  P->sub_nb.resize(N);
  P->sub_brow_base.resize(N);
  P->sub_tile_base.resize(N);
  P->sub_vec_base.resize(N + 1);
  int64_t tiles = 0, blocks = 0, vec = 0;
  P->max_nb = 0;
  for (int l = 0; l < N; ++l) {
    const Skyline &s = P->sky[l];
    P->sub_nb[l] = (int32_t)s.nb;
    P->sub_brow_base[l] = (int32_t)blocks;
    P->sub_tile_base[l] = tiles;
    P->sub_vec_base[l] = vec;
    tiles += s.tiles;
    blocks += s.nb;
    vec += s.nb * kTile;
    P->max_nb = std::max<int>(P->max_nb, (int)s.nb);
  }
  P->sub_vec_base[N] = vec;
  if (blocks > INT32_MAX) fail(MX_EINVAL, "too many block rows");
  P->tiles_total = tiles;
  P->blocks_total = blocks;
  P->vec_total = vec;
  std::vector<int64_t> &brow_off = plan.brow_off;
  std::vector<int32_t> &bfirst = plan.bfirst, &blast = plan.blast;
  brow_off.assign(blocks, 0);
  bfirst.assign(blocks, 0);
  blast.assign(blocks, 0);
  for (int l = 0; l < N; ++l) {
    const Skyline &s = P->sky[l];
    for (int64_t I = 0; I < s.nb; ++I) {
      brow_off[P->sub_brow_base[l] + I] = s.brow_off[I];
      bfirst[P->sub_brow_base[l] + I] = s.bfirst[I];
      blast[P->sub_brow_base[l] + I] = s.blast[I];
    }
  }
  // trimmed tiles read by the sweeps: row i of block row I is kept in tile (I, J) iff
  // first_i < 64 (J + 1) (padding rows have first_i = i); kept rows are packed tile after tile
  std::vector<int64_t> &rmeta = plan.rmeta, &cmeta = plan.cmeta, &cptr = plan.cptr;
  rmeta.assign(2 * tiles, 0);
  parallel_items(N, [&](auto next) {
    for (int64_t l; (l = next()) >= 0;) {
      const Skyline &s = P->sky[l];
      for (int64_t I = 0; I < s.nb; ++I) {
        const int64_t f = s.bfirst[I], t0 = P->sub_tile_base[l] + s.brow_off[I];
        std::vector<uint64_t> bits(I - f + 1, 0);
        for (int r = 0; r < kTile; ++r) {
          const int64_t i = I * kTile + r, fi = i < s.n ? s.first[i] : i;
          bits[std::max(f, fi / kTile) - f] |= 1ull << r;
        }
        uint64_t m = 0;
        for (int64_t J = f; J <= I; ++J) {
          m |= bits[J - f];
          rmeta[2 * (t0 + J - f) + 1] = (int64_t)m;
        }
      }
    }
  });
  int64_t packed = 0;
  for (int64_t t = 0; t < tiles; ++t) {
    rmeta[2 * t] = packed;
    packed += (int64_t)__builtin_popcountll((uint64_t)rmeta[2 * t + 1]) * kTile;
  }
  P->pack_entries = packed;
  cptr.assign(blocks, 0);
  cmeta.assign(2 * tiles, 0);
  {
    // a subdomain's block columns cover exactly its tiles, so its column-ordered entries start
    // where its tiles start
    std::atomic<int> bad(0);
    parallel_items(N, [&](auto next) {
      for (int64_t l; (l = next()) >= 0;) {
        const Skyline &s = P->sky[l];
        const int64_t bb = P->sub_brow_base[l], tb = P->sub_tile_base[l];
        int64_t c = tb;
        for (int64_t B = 0; B < s.nb; ++B) {
          cptr[bb + B] = c;
          for (int64_t I = B; I <= s.blast[B]; ++I, ++c) {
            const int64_t t = tb + s.brow_off[I] + (B - s.bfirst[I]);
            cmeta[2 * c] = rmeta[2 * t];
            cmeta[2 * c + 1] = rmeta[2 * t + 1];
          }
        }
        if (c != tb + s.tiles) bad = 1;
      }
    });
    if (bad) fail(MX_EINVAL, "internal: block columns do not cover the stored tiles");
  }
  // scatter list: lower-triangle entries of each permuted local matrix + unit diagonal padding
  std::vector<int64_t> cnt(N + 1, 0);
  parallel_items(N, [&](auto next) {
    for (int64_t l; (l = next()) >= 0;) {
      const LocalCSR &a = loc[l];
      const Skyline &s = P->sky[l];
      int64_t c = 0;
      for (int64_t r = 0; r < a.n; ++r)
        for (int64_t q = a.rowptr[r]; q < a.rowptr[r + 1]; ++q) c += s.iperm[a.col[q]] <= s.iperm[r];
      cnt[l + 1] = c + (s.nb * kTile - s.n);
    }
  });
  for (int l = 0; l < N; ++l) cnt[l + 1] += cnt[l];
  plan.scat = cnt;
  std::vector<int64_t> &off = plan.off;
  std::vector<double> &val = plan.val;
  off.assign(cnt[N], 0);
  val.assign(2 * cnt[N], 0.0);
  parallel_items(N, [&](auto next) {
    for (int64_t l; (l = next()) >= 0;) {
      const LocalCSR &a = loc[l];
      const Skyline &s = P->sky[l];
      int64_t w = cnt[l];
      const int64_t tb = P->sub_tile_base[l];
      auto pos = [&](int64_t i, int64_t j) {
        int64_t I = i / kTile, J = j / kTile;
        return (tb + s.brow_off[I] + (J - s.bfirst[I])) * (int64_t)kTileElems + (i % kTile) * kTile +
               (j % kTile);
      };
      for (int64_t r = 0; r < a.n; ++r)
        for (int64_t q = a.rowptr[r]; q < a.rowptr[r + 1]; ++q) {
          int64_t i = s.iperm[r], j = s.iperm[a.col[q]];
          if (j > i) continue;
          off[w] = pos(i, j);
          val[2 * w] = a.val[2 * q];
          val[2 * w + 1] = a.val[2 * q + 1];
          ++w;
        }
      for (int64_t i = s.n; i < s.nb * kTile; ++i) {
        off[w] = pos(i, i);
        val[2 * w] = 1.0;
        val[2 * w + 1] = 0.0;
        ++w;
      }
    }
  });
  // restriction / prolongation maps
  std::vector<int32_t> &glob = plan.glob;
  glob.assign(vec, -1);
  parallel_items(N, [&](auto next) {
    for (int64_t l; (l = next()) >= 0;) {
      const Skyline &s = P->sky[l];
      for (int64_t i = 0; i < s.n; ++i) glob[P->sub_vec_base[l] + i] = sets[l][s.perm[i]];
    }
  });
  std::vector<int64_t> &src = plan.src, &sum_ptr = plan.sum_ptr, &sum_idx = plan.sum_idx;
  if (opts->kind == MX_AS) {
    sum_ptr.assign(ndof + 1, 0);
    for (int l = 0; l < N; ++l)
      for (int32_t g : sets[l]) sum_ptr[g + 1]++;
    for (int64_t e = 0; e < ndof; ++e) sum_ptr[e + 1] += sum_ptr[e];
    sum_idx.resize(sum_ptr[ndof]);
    std::vector<int64_t> fill(sum_ptr.begin(), sum_ptr.end() - 1);
    for (int l = 0; l < N; ++l) {
      const Skyline &s = P->sky[l];
      for (int64_t r = 0; r < (int64_t)sets[l].size(); ++r)
        sum_idx[fill[sets[l][r]]++] = P->sub_vec_base[l] + s.iperm[r];
    }
  } else {
    src.assign(ndof, -1);
    std::atomic<int> bad(0);
    parallel_for(ndof, [&](int64_t a0, int64_t a1) {
      for (int64_t e = a0; e < a1; ++e) {
        int o = owner[e] - s0;
        if (o < 0 || o >= N) continue;  // owned outside the resident share
        const auto &st = sets[o];
        auto it = std::lower_bound(st.begin(), st.end(), (int32_t)e);
        if (it == st.end() || *it != e) {
          bad = 1;
          continue;
        }
        src[e] = P->sub_vec_base[o] + P->sky[o].iperm[it - st.begin()];
      }
    });
    if (bad) fail(MX_EINVAL, "internal: owner does not hold its DOF");
  }
  // factor step tables
  P->panel_pref.assign((int64_t)P->max_nb * (N + 1), 0);
  P->update_pref.assign((int64_t)P->max_nb * (N + 1), 0);
  for (int K = 0; K < P->max_nb; ++K) {
    int64_t ap = 0, au = 0;
    for (int l = 0; l < N; ++l) {
      P->panel_pref[(int64_t)K * (N + 1) + l] = (int32_t)ap;
      P->update_pref[(int64_t)K * (N + 1) + l] = (int32_t)au;
      if (K < P->sub_nb[l]) {
        int64_t mK = P->sky[l].blast[K] - K;
        ap += mK;                 // panel tiles = block column K+1 tiles of the trailing update
        au += mK * (mK - 1) / 2;  // the remaining trailing tiles
      }
    }
    if (au > INT32_MAX) fail(MX_EINVAL, "factor step too large");
    P->panel_pref[(int64_t)K * (N + 1) + N] = (int32_t)ap;
    P->update_pref[(int64_t)K * (N + 1) + N] = (int32_t)au;
  }
  // look-ahead groups of W block columns (group G = 0, W, 2W, ...; rows up to b = blast of the
  // group's last column, blast being nondecreasing): column Kc of a group from the group's
  // columns before it; the next group's W columns; the remaining tiles G+2W <= J <= I <= b
  {
    const int W = P->width;
    const size_t sz = (size_t)P->max_nb * (N + 1);
    P->intra_pref.assign(sz, 0);
    P->next_pref.assign(sz, 0);
    P->rest_pref.assign(sz, 0);
    for (int K = 0; K < P->max_nb; ++K) {
      int64_t ai = 0, an = 0, ar = 0;
      const bool start = K % W == 0;
      for (int l = 0; l < N; ++l) {
        const int64_t row = (int64_t)K * (N + 1) + l;
        P->intra_pref[row] = (int32_t)ai;
        P->next_pref[row] = (int32_t)an;
        P->rest_pref[row] = (int32_t)ar;
        const int nbl = P->sub_nb[l];
        if (K >= nbl) continue;
        const auto &bl = P->sky[l].blast;
        if (!start) ai += std::max<int64_t>(0, bl[K - 1] - K + 1);
        if (start) {
          const int64_t b = bl[std::min(K + W, nbl) - 1];
          for (int64_t J = K + W; J < K + 2 * W; ++J) an += std::max<int64_t>(0, b - J + 1);
          const int64_t m = std::max<int64_t>(0, b - (K + 2 * W) + 1);
          ar += m * (m + 1) / 2;
        }
      }
      if (ar > INT32_MAX || an > INT32_MAX) fail(MX_EINVAL, "factor step too large");
      P->intra_pref[(int64_t)K * (N + 1) + N] = (int32_t)ai;
      P->next_pref[(int64_t)K * (N + 1) + N] = (int32_t)an;
      P->rest_pref[(int64_t)K * (N + 1) + N] = (int32_t)ar;
    }
  }
  // sweep schedule: forward rows by relative progress, then backward rows likewise
  struct Item {
    double key;
    int32_t l, b;
  };
  std::vector<Item> fw, bw;
  for (int l = 0; l < N; ++l) {
    const int64_t nb = P->sub_nb[l];
    for (int64_t I = 0; I < nb; ++I) {
      fw.push_back({(I + 0.5) / nb, l, (int32_t)I});
      bw.push_back({(I + 0.5) / nb, l, (int32_t)(nb - 1 - I)});
    }
  }
  auto by_key = [](const Item &a, const Item &b) { return a.key != b.key ? a.key < b.key : a.l < b.l; };
  std::sort(fw.begin(), fw.end(), by_key);
  std::sort(bw.begin(), bw.end(), by_key);
  std::vector<int32_t> &sched_sub = plan.sched_sub, &sched_blk = plan.sched_blk;
  for (const auto *lst : {&fw, &bw})
    for (const auto &it : *lst) {
      sched_sub.push_back(it.l);
      sched_blk.push_back(it.b);
    }
  P->n_items = (int)sched_sub.size();
  // persistent sweeps: one workgroup per CU (a second co-resident workgroup streaming tiles delays
  // the dependency chain of the first one more than it adds bandwidth, measured); without a
  // context the grid is chosen when the preconditioner is materialised
  P->sweep_grid = opts->sweep_grid;
  if (ctx) set_sweep_grid(P, ctx->cus);
  const double t1 = now_s();
  P->info.t_host_setup = t1 - t0;
  const size_t esz = P->prec == MX_C128 ? 16 : 8;
  // peak: the tile pool and the packed factor coexist while packing
  plan.device_bytes = (size_t)tiles * kTileElems * esz + (size_t)packed * esz + 3 * (size_t)vec * esz +
                      2 * (size_t)blocks * 4 + 24 * (size_t)blocks + 32 * (size_t)tiles + 4 * (size_t)vec +
                      8 * (size_t)std::max(src.size(), sum_idx.size() + sum_ptr.size()) +
                      8 * (size_t)sched_sub.size() + 20 * P->panel_pref.size() +
                      24 * off.size() + (1 << 20);
}

// Everything the device half reads from the plan except the local matrices' entries.
static void upload_metadata(mx_precond *P, PrecondPlan &plan) {
  P->d_sub_nb.upload(P->sub_nb);
  P->d_sub_brow_base.upload(P->sub_brow_base);
  P->d_sub_tile_base.upload(P->sub_tile_base);
  P->d_sub_vec_base.upload(P->sub_vec_base);
  P->d_brow_off.upload(plan.brow_off);
  P->d_bfirst.upload(plan.bfirst);
  P->d_blast.upload(plan.blast);
  P->d_glob.upload(plan.glob);
  if (P->kind == MX_AS) {
    P->d_sum_ptr.upload(plan.sum_ptr);
    P->d_sum_idx.upload(plan.sum_idx);
  } else {
    P->d_src.upload(plan.src);
  }
  P->d_panel_pref.upload(P->panel_pref);
  P->d_update_pref.upload(P->update_pref);
  P->d_intra_pref.upload(P->intra_pref);
  P->d_next_pref.upload(P->next_pref);
  P->d_rest_pref.upload(P->rest_pref);
  P->d_sched_sub.upload(plan.sched_sub);
  P->d_sched_blk.upload(plan.sched_blk);
  P->d_rmeta.upload(plan.rmeta);
  P->d_cmeta.upload(plan.cmeta);
  P->d_cptr.upload(plan.cptr);
}

size_t precond_one_group_bytes(const mx_precond *P, const PrecondPlan &plan) {
  const size_t esz = P->prec == MX_C128 ? 16 : 8;
  return (size_t)P->tiles_total * kTileElems * esz + (size_t)(plan.scat.back() - plan.scat.front()) * 24;
}

void precond_release_device(mx_precond *P) {
  for (DevBuf *b : {&P->d_sub_nb, &P->d_sub_brow_base, &P->d_sub_tile_base, &P->d_sub_vec_base,
                    &P->d_brow_off, &P->d_bfirst, &P->d_blast, &P->pool, &P->d_off_all, &P->d_val_all,
                    &P->pack, &P->d_rmeta, &P->d_cmeta, &P->d_cptr, &P->d_r, &P->d_y, &P->d_z,
                    &P->d_glob, &P->d_src, &P->d_sum_ptr, &P->d_sum_idx, &P->d_ctrl, &P->d_sched_sub,
                    &P->d_sched_blk, &P->d_panel_pref, &P->d_update_pref, &P->d_intra_pref,
                    &P->d_next_pref, &P->d_rest_pref})
    b->release();
  P->staged = false;
}

// Optional middle step: the host-to-device copies of the device half, on a private stream that
// does not wait for other streams (so another host thread can run it while the device works).
// Buffers are allocated unscoped: they outlive that stream.
void precond_stage(mx_precond *P, PrecondPlan &plan) {
  hipStream_t own;
  MX_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
  const hipStream_t prev = t_alloc_stream;
  const int prev_scoped = t_alloc_scoped;
  t_alloc_stream = own;
  t_alloc_scoped = 0;
  auto restore = [&]() {
    t_alloc_stream = prev;
    t_alloc_scoped = prev_scoped;
    (void)hipStreamSynchronize(own);
    (void)hipStreamDestroy(own);
  };
  try {
    upload_metadata(P, plan);
    P->d_off_all.upload(plan.off);
    P->d_val_all.upload(plan.val);
  } catch (...) {
    restore();
    throw;
  }
  restore();
  P->staged = true;
}

void precond_materialize(mx_precond *P, PrecondPlan &plan, hipStream_t st) {
  const double t1 = now_s();
  const int N = P->nsub;
  const int64_t vec = P->vec_total, tiles = P->tiles_total;
  AllocScope scope(st);
  // device buffers
  const size_t esz = P->prec == MX_C128 ? 16 : 8;
  if (!P->staged) upload_metadata(P, plan);
  P->d_r.alloc(vec * esz);
  P->d_y.alloc(vec * esz);
  P->d_z.alloc(vec * esz);
  P->d_ctrl.alloc(64);
  MX_HIP(hipMemsetAsync(P->d_ctrl.p, 0, 64, st));
  MX_HIP(hipMemsetAsync(P->d_y.p, 0, vec * esz, st));
  MX_HIP(hipMemsetAsync(P->d_z.p, 0, vec * esz, st));
  // Trimmed tiles (what the sweeps read) first; then the full tiles of as many consecutive
  // subdomains at a time as fit (all of them unless memory or pool_limit says otherwise), each
  // group scattered, factored and trimmed in turn.
  P->pack.alloc((size_t)P->pack_entries * esz);
  if (tiles > INT32_MAX) fail(MX_EINVAL, "too many tiles");
  auto tile_end = [&](int l) { return l < N ? P->sub_tile_base[l] : tiles; };
  auto group_bytes = [&](int l) {
    return (size_t)(tile_end(l + 1) - P->sub_tile_base[l]) * kTileElems * esz +
           (size_t)(plan.scat[l + 1] - plan.scat[l]) * 24;
  };
  size_t cap = (size_t)P->pool_limit;
  if (cap == 0) {
    size_t free_b = 0, total_b = 0;
    MX_HIP(hipStreamSynchronize(st));
    MX_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t avail = free_b + big_cached(P->device);
    const size_t margin = (size_t)2 << 30;
    cap = avail > margin ? avail - margin : 0;
  }
  std::vector<int> groups = {0};
  {
    size_t acc = 0;
    for (int l = 0; l < N; ++l) {
      const size_t b = group_bytes(l);
      if (b > cap) fail(MX_ENOMEM, "one subdomain's factor tiles exceed the memory available");
      if (acc + b > cap && l > groups.back()) {
        groups.push_back(l);
        acc = 0;
      }
      acc += b;
    }
    groups.push_back(N);
  }
  int64_t max_group_tiles = 0;
  for (size_t g = 0; g + 1 < groups.size(); ++g)
    max_group_tiles = std::max(max_group_tiles, tile_end(groups[g + 1]) - P->sub_tile_base[groups[g]]);
  const size_t pool_bytes = (size_t)max_group_tiles * kTileElems * esz;
  P->pool.alloc(pool_bytes);
  P->n_groups = (int)groups.size() - 1;
  double t_upload = now_s() - t1, t_factor = 0, t_pack = 0;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    const int l0 = groups[g], l1 = groups[g + 1];
    const int64_t T0 = P->sub_tile_base[l0], T1 = tile_end(l1);
    double ta = now_s();
    k_zero<<<4096, 256, 0, st>>>((int64_t)((T1 - T0) * kTileElems * esz / 16), P->pool.as<uint4>());
    {
      const int64_t e0 = plan.scat[l0], ne = plan.scat[l1] - e0;
      DevBuf d_off, d_val;
      const int64_t *off = P->staged ? P->d_off_all.as<int64_t>() + e0 : nullptr;
      const cx<double> *val = P->staged ? P->d_val_all.as<cx<double>>() + e0 : nullptr;
      if (!P->staged) {
        d_off.alloc((size_t)ne * 8);
        d_val.alloc((size_t)ne * 16);
        if (ne > 0) {
          MX_HIP(hipMemcpyAsync(d_off.p, plan.off.data() + e0, (size_t)ne * 8, hipMemcpyHostToDevice, st));
          MX_HIP(hipMemcpyAsync(d_val.p, plan.val.data() + 2 * e0, (size_t)ne * 16, hipMemcpyHostToDevice, st));
        }
        off = d_off.as<int64_t>();
        val = d_val.as<cx<double>>();
      }
      if (ne > 0) {
        const int64_t shift = T0 * kTileElems;
        if (P->prec == MX_C128)
          k_scatter<double><<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(ne, off, val, shift,
                                                                          P->pool.as<cx<double>>());
        else
          k_scatter<float><<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(ne, off, val, shift,
                                                                         P->pool.as<cx<float>>());
      }
      MX_HIP(hipGetLastError());
      MX_HIP(hipStreamSynchronize(st));
    }
    double tb = now_s();
    SubView v = view_of(P);
    v.tile_shift = T0;
    if (P->prec == MX_C128) factor_group<double>(P, st, l0, l1, v, P->pool.as<cx<double>>());
    else factor_group<float>(P, st, l0, l1, v, P->pool.as<cx<float>>());
    MX_HIP(hipStreamSynchronize(st));
    double tc = now_s();
    if (T1 > T0) {
      if (P->prec == MX_C128)
        k_pack<double><<<(unsigned)(T1 - T0), 256, 0, st>>>(T1 - T0, P->d_rmeta.as<TileMeta>() + T0,
                                                         P->pool.as<cx<double>>(), P->pack.as<cx<double>>());
      else
        k_pack<float><<<(unsigned)(T1 - T0), 256, 0, st>>>(T1 - T0, P->d_rmeta.as<TileMeta>() + T0,
                                                        P->pool.as<cx<float>>(), P->pack.as<cx<float>>());
      MX_HIP(hipGetLastError());
    }
    MX_HIP(hipStreamSynchronize(st));
    double td = now_s();
    t_upload += tb - ta;
    t_factor += tc - tb;
    t_pack += td - tc;
  }
  precond_check(P, st);
  P->pool.release();
  MX_HIP(hipStreamSynchronize(st));
  P->d_off_all.release();
  P->d_val_all.release();
  // The plan's host arrays stay: a caller may materialise the same plan again after releasing
  // the device half (the server does, when a later allocation of the request fails).  Callers
  // drop the plan when they are done with it.
  // info
  mx_precond_info &in = P->info;
  in.n_sub = N;
  in.tile = kTile;
  in.n_local_total = 0;
  in.max_local = 0;
  in.env_entries = 0;
  in.env_flops = 0;
  in.tile_flops = 0;
  for (int l = 0; l < N; ++l) {
    const Skyline &s = P->sky[l];
    in.n_local_total += s.n;
    in.max_local = std::max<int64_t>(in.max_local, s.n);
    in.env_entries += s.env;
    in.env_flops += s.env_flops;
    in.tile_flops += s.tile_flops;
  }
  in.max_blocks = P->max_nb;
  in.tiles = tiles;
  in.factor_bytes = (int64_t)pool_bytes;
  in.pack_bytes = (int64_t)(P->pack_entries * (int64_t)esz);
  // algorithmic bytes per application: the envelope factor read twice, the local vectors
  // (restricted input written and read, forward result written and read twice, backward result
  // written and read), the global input gathered and output written, the 4-byte gather maps
  const int64_t nloc = in.n_local_total;
  in.apply_bytes = (int64_t)(2 * in.env_entries * esz + 6 * nloc * esz + 2 * P->E * 16 + 4 * nloc +
                             8 * P->E);
  // one block-sweep launch: the envelope read once; forward: r read, y written, y read once
  // (backward: y read, z written, z read once)
  in.sweep_bytes = (int64_t)(in.env_entries * esz + 3 * nloc * esz);
  in.t_upload = t_upload;
  in.t_factor = t_factor;
  in.t_pack = t_pack;
  in.factor_groups = P->n_groups;
}

}  // namespace mx
